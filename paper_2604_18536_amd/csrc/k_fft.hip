// Spectral pressure solve of Sec. 2.6.1 on gfx950: p = DFT^-1 L^-1 DFT r with
// the exact discrete transfer function, as a real-to-complex FFT along x
// followed by complex FFTs along y (and z), all hand-written.
//
// Each workgroup moves a batch of whole lines into LDS, runs a Stockham
// autosort FFT of mixed radix (8, 7, 5, 4, 3, 2) on them there (every
// butterfly's inputs are read into registers, a barrier, then its outputs are
// written, so one LDS buffer suffices), and writes the lines back.
//   x pass   : rows of n_x reals, packed as n_x/2 complex values; the
//              divergence of the stage velocity is formed on the fly while
//              loading, so r is never stored.
//   y/z pass : lines of a strided axis; a workgroup takes `lines` adjacent kx
//              so each global access is a contiguous run of `lines` values.
//   last axis: forward FFT, multiply by 1/(L(k) #cells), inverse FFT in the
//              same launch (the spectrum of that axis never leaves LDS).
// The spectral arithmetic runs in the precision of the complex type C: cd
// (float64, every mode but one) or cf (float32, the all-float32 comparison
// mode), with twiddles and eigenvalues tabulated in that precision.
#include "k_common.hpp"

namespace ins {

#define INS_INLINE __attribute__((always_inline))

// LDS layout of a batch of `nl` lines of length N: element j of line l lives at
// lds[j * ls + l] with the line stride ls = nl + pad. The plan pads (pad = 1,
// an odd stride, so neighbouring elements of one line fall in different banks)
// whenever the padded batch still fits the LDS budget.

// cos(2 pi j / R), sin(2 pi j / R), correctly rounded.
__device__ __forceinline__ constexpr double kcos(int R, int j) {
    return R == 3 ? (j == 0 ? 1.0 : -0.5)
         : R == 5 ? (j == 0 ? 1.0 : (j == 1 || j == 4) ? 0.30901699437494745 : -0.8090169943749475)
         : /*7*/ (j == 0 ? 1.0 : (j == 1 || j == 6) ? 0.6234898018587335
                            : (j == 2 || j == 5) ? -0.2225209339563144 : -0.9009688679024191);
}
__device__ __forceinline__ constexpr double ksin(int R, int j) {
    return R == 3 ? (j == 0 ? 0.0 : j == 1 ? 0.8660254037844386 : -0.8660254037844386)
         : R == 5 ? (j == 0 ? 0.0 : j == 1 ? 0.9510565162951535 : j == 2 ? 0.5877852522924731
                   : j == 3 ? -0.5877852522924731 : -0.9510565162951535)
         : (j == 0 ? 0.0 : j == 1 ? 0.7818314824680298 : j == 2 ? 0.9749279121818236
            : j == 3 ? 0.4338837391175581 : j == 4 ? -0.4338837391175581
            : j == 5 ? -0.9749279121818236 : -0.7818314824680298);
}

// i * z * sgn
template <int SIGN, class C>
__device__ __forceinline__ C rot(C z) {
    return SIGN < 0 ? C{z.y, -z.x} : C{-z.y, z.x};
}

// Small DFTs X[m] = sum_q x[q] exp(SIGN 2 pi i q m / R), in place.
template <int SIGN, class C>
__device__ __forceinline__ void dft2(C* v) {
    const C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <int SIGN, class C>
__device__ __forceinline__ void dft4(C& x0, C& x1, C& x2, C& x3) {
    const C s02 = cadd(x0, x2), d02 = csub(x0, x2);
    const C s13 = cadd(x1, x3), d13 = rot<SIGN>(csub(x1, x3));
    x0 = cadd(s02, s13);
    x2 = csub(s02, s13);
    x1 = cadd(d02, d13);
    x3 = csub(d02, d13);
}

template <int SIGN, class C>
__device__ __forceinline__ void dft8(C* v) {
    using F = real_of<C>;
    C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<SIGN>(e0, e1, e2, e3);
    dft4<SIGN>(o0, o1, o2, o3);
    constexpr F r = F(0.7071067811865476);
    // w^1 = (1 + SIGN i)/sqrt2, w^2 = SIGN i, w^3 = (-1 + SIGN i)/sqrt2
    const C t1 = {r * (o1.x - SIGN * o1.y), r * (o1.y + SIGN * o1.x)};
    const C t2 = rot<SIGN>(o2);
    const C t3 = {r * (-o3.x - SIGN * o3.y), r * (-o3.y + SIGN * o3.x)};
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, t1);
    v[5] = csub(e1, t1);
    v[2] = cadd(e2, t2);
    v[6] = csub(e2, t2);
    v[3] = cadd(e3, t3);
    v[7] = csub(e3, t3);
}

// Odd R: pair x[q] with x[R-q]; X[m] = A_m + SIGN i B_m, X[R-m] = A_m - SIGN i B_m with
// A_m = x0 + sum_q (x_q + x_{R-q}) cos(2 pi q m / R), B_m = sum_q (x_q - x_{R-q}) sin(2 pi q m / R).
template <int R, int SIGN, class C>
__device__ __forceinline__ void dft_odd(C* v) {
    using F = real_of<C>;
    constexpr int H = (R - 1) / 2;
    C s[H], d[H];
#pragma unroll
    for (int q = 1; q <= H; ++q) {
        s[q - 1] = cadd(v[q], v[R - q]);
        d[q - 1] = csub(v[q], v[R - q]);
    }
    const C x0 = v[0];
    C sum = x0;
#pragma unroll
    for (int q = 0; q < H; ++q) sum = cadd(sum, s[q]);
    v[0] = sum;
#pragma unroll
    for (int m = 1; m <= H; ++m) {
        C A = x0, B = {F(0), F(0)};
#pragma unroll
        for (int q = 1; q <= H; ++q) {
            const int j = (q * m) % R;
            A.x += s[q - 1].x * F(kcos(R, j));
            A.y += s[q - 1].y * F(kcos(R, j));
            B.x += d[q - 1].x * F(ksin(R, j));
            B.y += d[q - 1].y * F(ksin(R, j));
        }
        const C iB = rot<SIGN>(B);
        v[m] = cadd(A, iB);
        v[R - m] = csub(A, iB);
    }
}

template <int R, int SIGN, class C>
__device__ __forceinline__ void dft(C* v) {
    if constexpr (R == 2) dft2<SIGN>(v);
    else if constexpr (R == 4) dft4<SIGN>(v[0], v[1], v[2], v[3]);
    else if constexpr (R == 8) dft8<SIGN>(v);
    else dft_odd<R, SIGN>(v);
}

// q = n / d and r = n % d for 0 <= n < 2^21 and d >= 1, given rd ~ 1/d in float
// to within 2 ulp: the float quotient is then within one unit of the true one,
// and one correction each way makes it exact.
__device__ __forceinline__ int fdivmod(int n, int d, float rd, int& r) {
    int q = static_cast<int>(static_cast<float>(n) * rd);
    r = n - q * d;
    if (r < 0) {
        --q;
        r += d;
    }
    if (r >= d) {
        ++q;
        r -= d;
    }
    return q;
}

// The twiddles of every stage are powers of W_N = exp(-2 pi i / N): stage
// (p, R) multiplies element q of butterfly k by W_N^(q k N / (p R)). Each
// strided-pass workgroup copies the roots W_N^j into LDS once (j < N/2 for
// even N, using W_N^(j + N/2) = -W_N^j; all N for odd N), so no stage issues
// a global load for them. The host tabulates the roots in the precision of C from an exact
// integer angle reduction.
template <class C>
struct Roots {
    const C* t;  // LDS (or the global table, with half = N)
    int half;    // number of stored roots
    __device__ __forceinline__ C operator()(int j) const {
        const C w = t[j < half ? j : j - half];
        return j < half ? w : C{-w.x, -w.y};
    }
    // the twiddles W_N^(q k sN), q = 1 .. R-1, of butterfly k
    struct Cursor {
        const C* t;
        int half, j, ks;
        __device__ __forceinline__ C next() {
            j += ks;
            const C w = t[j < half ? j : j - half];
            return j < half ? w : C{-w.x, -w.y};
        }
    };
    __device__ __forceinline__ Cursor at(int, int k, int, int sN) const { return Cursor{t, half, 0, k * sN}; }
};

// Per-stage twiddle tables in global memory (the x passes, whose element-fast
// stages would read LDS roots with bank conflicts): stage s keeps
// exp(-2 pi i q k / (p R)) at tw[off[s] + k (R - 1) + q - 1].
template <class C>
struct TabTw {
    const C* tw;
    const int* off;
    struct Cursor {
        const C* p;
        __device__ __forceinline__ C next() { return *++p; }
    };
    __device__ __forceinline__ Cursor at(int s, int k, int R, int) const {
        return Cursor{tw + off[s] + k * (R - 1) - 1};
    }
};

// Number of roots a plan of length n keeps in LDS.
__host__ __device__ __forceinline__ int roots_count(int n) { return (n & 1) ? n : n / 2; }

// How the butterflies t = 0 .. S*nl-1 of a stage map to (line l, index i):
// line-fast keeps neighbouring threads on neighbouring lines (contiguous in LDS
// and, for a strided axis, in memory); element-fast keeps them on neighbouring
// elements of one line (contiguous in memory along x).
enum : int { kLineFast = 0, kElemFast = 1 };

template <int MAP>
__device__ __forceinline__ void slot_of(int t, int lnl, int S, float rS, int& l, int& i) {
    if constexpr (MAP == kLineFast) {
        l = t & ((1 << lnl) - 1);
        i = t >> lnl;
    } else {
        l = fdivmod(t, S, rS, i);
    }
}

// One Stockham stage of radix R over the nl lines of length N, p = product of
// the earlier radices. Butterfly (l, i) takes elements i + q S (S = N / R) of
// line l, multiplies element q by exp(SIGN 2 pi i q k / (p R)) with k = i mod p,
// applies DFT_R and produces elements (i - k) R + k + q p. A thread runs
// butterflies t = threadIdx.x + b NTH (NTH threads per workgroup), b < VM / R, in registers.
//   IN  0: inputs from load(l, e) (global memory);  1: from LDS.
//   OUT 0: outputs to LDS, then a barrier;
//       1: outputs handed to sink(l, e, z) (last stage: element i + q S);
//       2: pivot of a forward solve along this axis: every output z of the
//          last forward stage is replaced by divf(l, e, z), and the first stage
//          of the inverse (the same radix, p = 1, so the same butterflies) is
//          applied at once; its outputs i R + q go to LDS when the inverse has
//          more stages (`more`), else to sink.
// The LDS reads of an IN 1 stage that writes LDS are followed by a barrier.
template <int R, int SIGN, int VM, int NTH, int IN, int OUT, int MAP, class C, class TW, class Load, class Sink,
          class Div>
__device__ __forceinline__ void fft_stage(C* __restrict__ lds, int lnl, int ls, int N, int p, int s, const TW& tw,
                                          const Load& load, const Sink& sink, const Div& divf, bool more) {
    constexpr int BMAX = VM / R > 0 ? VM / R : 1;
    const int S = N / R;
    const int sN = S / p;  // exp(2 pi i q k / (p R)) = W_N^(q k sN)
    const int nb = S << lnl;
    const float rS = __builtin_amdgcn_rcpf(static_cast<float>(S));
    const float rp = __builtin_amdgcn_rcpf(static_cast<float>(p));
    C w[BMAX * R];
#pragma unroll
    for (int b = 0; b < BMAX; ++b) {
        const int t = threadIdx.x + b * NTH;
        if (t < nb) {
            int l, i;
            slot_of<MAP>(t, lnl, S, rS, l, i);
#pragma unroll
            for (int q = 0; q < R; ++q) {
                if constexpr (IN == 0) w[b * R + q] = load(l, i + q * S);
                else w[b * R + q] = lds[(i + q * S) * ls + l];
            }
        }
    }
    if constexpr (IN == 1 && OUT != 1) __syncthreads();
#pragma unroll
    for (int b = 0; b < BMAX; ++b) {
        const int t = threadIdx.x + b * NTH;
        if (t < nb) {
            int l, i;
            slot_of<MAP>(t, lnl, S, rS, l, i);
            int k;
            fdivmod(i, p, rp, k);
            C* x = w + b * R;
            if (k != 0) {
                auto cur = tw.at(s, k, R, sN);
#pragma unroll
                for (int q = 1; q < R; ++q) {
                    const C w = cur.next();
                    x[q] = SIGN < 0 ? cmul(x[q], w) : cmulc(x[q], w);
                }
            }
            dft<R, SIGN>(x);
            if constexpr (OUT == 0) {
                const int base = (i - k) * R + k;
#pragma unroll
                for (int q = 0; q < R; ++q) lds[(base + q * p) * ls + l] = x[q];
            } else if constexpr (OUT == 1) {
#pragma unroll
                for (int q = 0; q < R; ++q) sink(l, i + q * S, x[q]);
            } else {
#pragma unroll
                for (int q = 0; q < R; ++q) x[q] = divf(l, i + q * S, x[q]);
                dft<R, -SIGN>(x);
                if (more) {
#pragma unroll
                    for (int q = 0; q < R; ++q) lds[(i * R + q) * ls + l] = x[q];
                } else {
#pragma unroll
                    for (int q = 0; q < R; ++q) sink(l, i * R + q, x[q]);
                }
            }
        }
    }
    if constexpr (OUT == 0 || OUT == 2) {
        if (OUT == 0 || more) __syncthreads();
    }
}

template <int SIGN, int VM, int NTH, int IN, int OUT, int MAP, class C, class TW, class Load, class Sink, class Div>
__device__ __forceinline__ void fft_stage_r(int R, C* lds, int lnl, int ls, int N, int p, int s, const TW& tw,
                                            const Load& load, const Sink& sink, const Div& divf, bool more) {
    switch (R) {
        case 8: fft_stage<8, SIGN, VM, NTH, IN, OUT, MAP>(lds, lnl, ls, N, p, s, tw, load, sink, divf, more); break;
        case 7: fft_stage<7, SIGN, VM, NTH, IN, OUT, MAP>(lds, lnl, ls, N, p, s, tw, load, sink, divf, more); break;
        case 5: fft_stage<5, SIGN, VM, NTH, IN, OUT, MAP>(lds, lnl, ls, N, p, s, tw, load, sink, divf, more); break;
        case 4: fft_stage<4, SIGN, VM, NTH, IN, OUT, MAP>(lds, lnl, ls, N, p, s, tw, load, sink, divf, more); break;
        case 3: fft_stage<3, SIGN, VM, NTH, IN, OUT, MAP>(lds, lnl, ls, N, p, s, tw, load, sink, divf, more); break;
        default: fft_stage<2, SIGN, VM, NTH, IN, OUT, MAP>(lds, lnl, ls, N, p, s, tw, load, sink, divf, more); break;
    }
}

struct NoOp {
    template <class C>
    __device__ C operator()(int, int, C z) const { return z; }
};

// The plan's twiddle table in the precision of C.
__device__ __forceinline__ const cd* plan_tw(const FftPlan& P, cd) { return P.tw; }
__device__ __forceinline__ const cf* plan_tw(const FftPlan& P, cf) { return P.twf; }

// The solve's eigenvalue tables and 1 / #cells in the precision of C.
__device__ __forceinline__ const double* const* solve_lam(const SolveTab& st, cd) { return st.lam; }
__device__ __forceinline__ const float* const* solve_lam(const SolveTab& st, cf) { return st.lamf; }
__device__ __forceinline__ double solve_inv_ncell(const SolveTab& st, cd) { return st.inv_ncell; }
__device__ __forceinline__ float solve_inv_ncell(const SolveTab& st, cf) { return st.inv_ncellf; }

// Every stage of plan P on nl = 2^lnl lines (LDS line stride ls); LDS must be
// free on entry. The first stage reads through `load` with mapping MAP0 (IN0 0)
// or from LDS (IN0 1); stages in between go LDS to LDS, line-fast; the last
// stage, with mapping MAPL (a single stage uses MAP0), writes per OUTL: 0 to
// LDS (element e of line l at lds[e ls + l], synchronised), 1 to sink, 2 as the
// pivot of a solve whose inverse plan is Q (then call fft_inverse_rest).
// The first and last stages are peeled off the loop so that the address
// arithmetic of the memory-facing stages is not kept live across the others.
template <int SIGN, int VM, int NTH, int IN0, int OUTL, int MAP0, int MAPL, class C, class TW, class Load, class Sink,
          class Div>
__device__ __forceinline__ void fft_run(C* lds, int lnl, int ls, const FftPlan& P, const TW& tw, const Load& load,
                                        const Sink& sink, const Div& divf, const FftPlan* Q) {
    const int ns = P.nst;
    const bool more = OUTL == 2 && Q->nst > 1;
    if (ns == 1) {
        fft_stage_r<SIGN, VM, NTH, IN0, OUTL, MAP0>(P.rad[0], lds, lnl, ls, P.n, 1, 0, tw, load, sink, divf, more);
        return;
    }
    fft_stage_r<SIGN, VM, NTH, IN0, 0, MAP0>(P.rad[0], lds, lnl, ls, P.n, 1, 0, tw, load, sink, divf, false);
    int p = P.rad[0];
    for (int st = 1; st < ns - 1; ++st) {
        fft_stage_r<SIGN, VM, NTH, 1, 0, kLineFast>(P.rad[st], lds, lnl, ls, P.n, p, st, tw, load, sink, divf, false);
        p *= P.rad[st];
    }
    fft_stage_r<SIGN, VM, NTH, 1, OUTL, MAPL>(P.rad[ns - 1], lds, lnl, ls, P.n, p, ns - 1, tw, load, sink, divf, more);
}

// The stages of inverse plan Q after a pivot consumed its first one (nothing
// when Q has a single stage): LDS to LDS, the last one to sink (mapping MAPL).
template <int SIGN, int VM, int NTH, int MAPL, class C, class TW, class Sink>
__device__ __forceinline__ void fft_inverse_rest(C* lds, int lnl, int ls, const FftPlan& Q, const TW& tw,
                                                 const Sink& sink) {
    const int ns = Q.nst;
    if (ns == 1) return;
    const NoOp nop;
    int p = Q.rad[0];
    for (int st = 1; st < ns - 1; ++st) {
        fft_stage_r<SIGN, VM, NTH, 1, 0, kLineFast>(Q.rad[st], lds, lnl, ls, Q.n, p, st, tw, nop, sink, nop, false);
        p *= Q.rad[st];
    }
    fft_stage_r<SIGN, VM, NTH, 1, 1, MAPL>(Q.rad[ns - 1], lds, lnl, ls, Q.n, p, ns - 1, tw, nop, sink, nop, false);
}

// Plan P's per-stage twiddle tables in global memory.
template <class C>
__device__ __forceinline__ TabTw<C> plan_tab(const FftPlan& P) {
    return TabTw<C>{plan_tw(P, C{}), P.tw_off};
}

// Copy plan P's roots into LDS at `dst` (synchronised by the caller's next barrier).
template <int NTH, class C>
__device__ __forceinline__ Roots<C> load_roots(C* dst, const FftPlan& P) {
    const C* src = plan_tw(P, C{}) + P.rt_off;
    const int ne = roots_count(P.n);
    for (int j = threadIdx.x; j < ne; j += NTH) dst[j] = src[j];
    return Roots<C>{dst, ne};
}

// Copy the nl lines into LDS element-major (lds[e ls + l]) with element-fast
// threads, so the global reads run along the rows and the LDS writes (odd
// stride ls) are conflict-free; then synchronise. (Along x a first stage that
// read memory directly would write its butterfly outputs i R + q from
// neighbouring threads R elements apart: bank conflicts.)
template <int NTH, class C, class Load>
__device__ __forceinline__ void stage_rows(C* __restrict__ lds, int lnl, int ls, int N, const Load& load) {
    const int nl = 1 << lnl;
    const float rN = __builtin_amdgcn_rcpf(static_cast<float>(N));
    for (int t = threadIdx.x; t < nl * N; t += NTH) {
        int e;
        const int l = fdivmod(t, N, rN, e);
        lds[e * ls + l] = load(l, e);
    }
    __syncthreads();
}

// One spectrum value loaded / stored non-temporally (the strided passes over a
// spectrum much larger than the MALL, where no pass can find the previous
// pass's output in it anyway: their short strided runs then stream better).
template <class C>
__device__ __forceinline__ C ld_stream_c(const C* p) {
    return C{__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y)};
}
template <class C>
__device__ __forceinline__ void st_stream_c(C* p, C z) {
    __builtin_nontemporal_store(z.x, &p->x);
    __builtin_nontemporal_store(z.y, &p->y);
}

// Two consecutive values of a row (x even), as one load.
template <class F>
__device__ __forceinline__ void ld_pair(const double* p, F& a, F& b) {
    const double2 t = *reinterpret_cast<const double2*>(p);
    a = F(t.x);
    b = F(t.y);
}
template <class F>
__device__ __forceinline__ void ld_pair(const float* p, F& a, F& b) {
    const float2 t = *reinterpret_cast<const float2*>(p);
    a = t.x;
    b = t.y;
}

// Row staging of the periodic divergence (the x pass's SRC 0): the offsets of
// the rows a batch row reads (u_x; u_y at y and y-1; u_z at z and z-1) are
// formed once per row in LDS, then each thread issues the loads of kXBatch
// values back to back (clamped, branch-free addresses) before it uses any, so
// it waits for memory once per kXBatch values instead of twice per value
// (x forward pass: 0.143 -> 0.125 ms at 256^3, 5.5 -> 4.9 ms at 840^3 with 256
// instead of 1024 threads per workgroup). Writes r[2m] + i r[2m+1] of
// row l to lds[m ls + l] (rows past nrows: 0) and synchronises; at most 16
// rows (the plan's batch limit). Same arithmetic as the per-value load.
constexpr int kXBatch = 4;
struct DivRows {
    int64_t ux, uy, vy, uz, vz;
};
template <typename T, int DIM, int NTH, class C>
__device__ __forceinline__ void stage_div_rows(const Grid& g, const T* __restrict__ vel, C* __restrict__ lds, int lnl,
                                               int ls, int M, int row0, int nrows) {
    using F = real_of<C>;
    __shared__ DivRows rows[16];
    const int nl = 1 << lnl;
    if (static_cast<int>(threadIdx.x) < nl) {
        const int row = min(row0 + static_cast<int>(threadIdx.x), nrows - 1);
        const int yy = row % g.ny, zb = row / g.ny, zz = zb % g.nz, b = zb / g.nz;
        const int64_t base = int64_t(b) * DIM * g.ncell;
        const int ym = yy == 0 ? g.ny - 1 : yy - 1;
        const int zm = zz == 0 ? g.nz - 1 : zz - 1;
        const int64_t r = int64_t(zz * g.ny + yy) * g.nx;
        DivRows d;
        d.ux = base + r;
        d.uy = base + g.ncell + r;
        d.vy = base + g.ncell + int64_t(zz * g.ny + ym) * g.nx;
        d.uz = DIM == 3 ? base + 2 * g.ncell + r : 0;
        d.vz = DIM == 3 ? base + 2 * g.ncell + int64_t(zm * g.ny + yy) * g.nx : 0;
        rows[threadIdx.x] = d;
    }
    __syncthreads();
    const int total = nl * M;
    const float rM = __builtin_amdgcn_rcpf(static_cast<float>(M));
    const F ihx = F(g.ih[0]), ihy = F(g.ih[1]), ihz = F(g.ih[2]);
    for (int t0 = 0; t0 < total; t0 += kXBatch * NTH) {
        F ux0[kXBatch], ux1[kXBatch], uxm[kXBatch], uy0[kXBatch], uy1[kXBatch], vy0[kXBatch], vy1[kXBatch];
        F uz0[kXBatch], uz1[kXBatch], vz0[kXBatch], vz1[kXBatch];
#pragma unroll
        for (int j = 0; j < kXBatch; ++j) {
            const int t = min(t0 + j * NTH + static_cast<int>(threadIdx.x), total - 1);
            int m;
            const int l = fdivmod(t, M, rM, m);
            const DivRows d = rows[l];
            const int x0 = 2 * m, xm = x0 == 0 ? g.nx - 1 : x0 - 1;
            ld_pair(vel + d.ux + x0, ux0[j], ux1[j]);
            uxm[j] = vel[d.ux + xm];
            ld_pair(vel + d.uy + x0, uy0[j], uy1[j]);
            ld_pair(vel + d.vy + x0, vy0[j], vy1[j]);
            if constexpr (DIM == 3) {
                ld_pair(vel + d.uz + x0, uz0[j], uz1[j]);
                ld_pair(vel + d.vz + x0, vz0[j], vz1[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < kXBatch; ++j) {
            const int t = t0 + j * NTH + static_cast<int>(threadIdx.x);
            if (t < total) {
                int m;
                const int l = fdivmod(t, M, rM, m);
                F r0 = (ux0[j] - uxm[j]) * ihx;
                F r1 = (ux1[j] - ux0[j]) * ihx;
                r0 += (uy0[j] - vy0[j]) * ihy;
                r1 += (uy1[j] - vy1[j]) * ihy;
                if constexpr (DIM == 3) {
                    r0 += (uz0[j] - vz0[j]) * ihz;
                    r1 += (uz1[j] - vz1[j]) * ihz;
                }
                lds[m * ls + l] = row0 + l < nrows ? C{r0, r1} : C{F(0), F(0)};
            }
        }
    }
    __syncthreads();
}

// ----------------------------------------------------------------------------
// x pass, forward: real rows (n_x = 2M) -> half spectrum X[0..M].
// Packing: z[m] = x[2m] + i x[2m+1]; Z = FFT_M(z);
// X[k] = (Z[k] + conj Z[M-k]) / 2 + W^k (Z[k] - conj Z[M-k]) / (2i), W = exp(-2 pi i / n_x).
// ----------------------------------------------------------------------------
// SRC 0: rows are the divergence of the velocity field `vel`;
// SRC 1: rows of the float64 scalar field r; SRC 2: rows of component `comp` of vel;
// SRC 3: the channel divergence D u (both wall faces of u^y read as 0, row
// widths from Grid::ym); SRC 4: the channel's D Omega_u^{-1} u (u^y / d_j,
// tangential components / w_j), the right-hand side inside the transposed
// projection.
// The rows are staged in LDS first (see stage_rows); the untangling needs Z[k]
// and Z[M-k] together, so the last stage writes to LDS as well.
template <typename T, int DIM, int SRC, int VM, int NTH, class C = cd>
__global__ __launch_bounds__(NTH) void k_fft_x_fwd(Grid g, const T* __restrict__ vel,
                                                        const real_of<C>* __restrict__ r, C* __restrict__ spec,
                                                        FftPlan P, const C* __restrict__ post, int lnl, int comp) {
    using F = real_of<C>;
    extern __shared__ __align__(16) unsigned char fft_smem[];
    C* lds = reinterpret_cast<C*>(fft_smem);
    const int nl = 1 << lnl;
    const int ls = nl + P.pad;
    const int M = P.n;
    const int nrows = g.batch * g.nz * g.ny;
    const int row0 = xcd_logical(blockIdx.x, gridDim.x) * nl;
    // (y, z, batch) of the first row; row0 + l follows by carrying (l < nl <= 16)
    const int yy0 = row0 % g.ny, zb0 = row0 / g.ny, zz0 = zb0 % g.nz, b0 = zb0 / g.nz;
    auto load = [&](int l, int m) INS_INLINE -> C {
        const int row = row0 + l;
        if (row >= nrows) return C{F(0), F(0)};
        if constexpr (SRC == 1) {
            return reinterpret_cast<const C*>(r + int64_t(row) * g.nx)[m];
        } else {
            int yy = yy0 + l, zz = zz0, b = b0;
            while (yy >= g.ny) {
                yy -= g.ny;
                if (++zz == g.nz) {
                    zz = 0;
                    ++b;
                }
            }
            const int rowoff = (zz * g.ny + yy) * g.nx;
            const int x0 = 2 * m;
            if constexpr (SRC == 2) {
                F a0, a1;
                ld_pair(vel + (int64_t(b) * DIM + comp) * g.ncell + rowoff + x0, a0, a1);
                return C{a0, a1};
            } else if constexpr (SRC >= 3) {
                const T* wb = vel + int64_t(b) * DIM * g.ncell;
                const int S = g.ny + 2;
                const double sp = SRC == 4 ? g.ym[3 * S + yy] : 1.0;  // w_j
                const int xm = x0 == 0 ? g.nx - 1 : x0 - 1;
                double ux0, ux1;
                ld_pair(wb + rowoff + x0, ux0, ux1);
                const double uxm = wb[rowoff + xm];
                double r0 = (ux0 - uxm) * g.ih[0];
                double r1 = (ux1 - ux0) * g.ih[0];
                if constexpr (DIM == 3) {
                    const int zm = zz == 0 ? g.nz - 1 : zz - 1;
                    const T* wz = wb + 2 * g.ncell;
                    double uz0, uz1, vz0, vz1;
                    ld_pair(wz + rowoff + x0, uz0, uz1);
                    ld_pair(wz + (zm * g.ny + yy) * g.nx + x0, vz0, vz1);
                    r0 += (uz0 - vz0) * g.ih[2];
                    r1 += (uz1 - vz1) * g.ih[2];
                }
                if constexpr (SRC == 4) {
                    r0 /= sp;
                    r1 /= sp;
                }
                const T* wy = wb + g.ncell;
                double uy0 = 0.0, uy1 = 0.0, vy0 = 0.0, vy1 = 0.0;
                if (yy < g.ny - 1) ld_pair(wy + rowoff + x0, uy0, uy1);
                if (yy > 0) ld_pair(wy + rowoff - g.nx + x0, vy0, vy1);
                if constexpr (SRC == 4) {
                    const double iu = g.ym[S + yy + 1], id = g.ym[S + yy];  // 1 / d_j, 1 / d_{j-1}
                    uy0 *= iu;
                    uy1 *= iu;
                    vy0 *= id;
                    vy1 *= id;
                }
                const double iw = g.ym[yy];
                r0 += (uy0 - vy0) * iw;
                r1 += (uy1 - vy1) * iw;
                return C{F(r0), F(r1)};
            } else {
                const T* wb = vel + int64_t(b) * DIM * g.ncell;
                const int xm = x0 == 0 ? g.nx - 1 : x0 - 1;
                F ux0, ux1;
                ld_pair(wb + rowoff + x0, ux0, ux1);
                const F uxm = wb[rowoff + xm];
                F r0 = (ux0 - uxm) * F(g.ih[0]);
                F r1 = (ux1 - ux0) * F(g.ih[0]);
                const int ym = yy == 0 ? g.ny - 1 : yy - 1;
                const T* wy = wb + g.ncell;
                F uy0, uy1, vy0, vy1;
                ld_pair(wy + rowoff + x0, uy0, uy1);
                ld_pair(wy + (zz * g.ny + ym) * g.nx + x0, vy0, vy1);
                r0 += (uy0 - vy0) * F(g.ih[1]);
                r1 += (uy1 - vy1) * F(g.ih[1]);
                if constexpr (DIM == 3) {
                    const int zm = zz == 0 ? g.nz - 1 : zz - 1;
                    const T* wz = wb + 2 * g.ncell;
                    F uz0, uz1, vz0, vz1;
                    ld_pair(wz + rowoff + x0, uz0, uz1);
                    ld_pair(wz + (zm * g.ny + yy) * g.nx + x0, vz0, vz1);
                    r0 += (uz0 - vz0) * F(g.ih[2]);
                    r1 += (uz1 - vz1) * F(g.ih[2]);
                }
                return C{r0, r1};
            }
        }
    };
    const NoOp nop;
    const TabTw<C> rt = plan_tab<C>(P);
    if constexpr (SRC == 0)
        stage_div_rows<T, DIM, NTH>(g, vel, lds, lnl, ls, M, row0, nrows);
    else
        stage_rows<NTH>(lds, lnl, ls, M, load);
    fft_run<-1, VM, NTH, 1, 0, kLineFast, kLineFast>(lds, lnl, ls, P, rt, load, nop, nop, nullptr);
    const int M1 = M + 1;
    const float rM1 = __builtin_amdgcn_rcpf(static_cast<float>(M1));
    for (int t = threadIdx.x; t < nl * M1; t += NTH) {
        int k;
        const int l = fdivmod(t, M1, rM1, k);
        const int row = row0 + l;
        if (row >= nrows) continue;
        const C zk = lds[(k == M ? 0 : k) * ls + l];
        const C zc = cconj(lds[(k == 0 ? 0 : M - k) * ls + l]);
        const C e = cscale(cadd(zk, zc), F(0.5));
        const C dd = csub(zk, zc);
        const C o = {F(0.5) * dd.y, F(-0.5) * dd.x};
        spec[int64_t(row) * g.sx + k] = cadd(e, cmul(post[k], o));
    }
}

// Row staging of the inverse x pass, batched like stage_div_rows: the three
// loads of kXBatch values (X[k], X[M-k], W^k) go out back to back, then the
// tangled values Z[k] are formed and written to lds[k ls + l] (rows past
// nrows: 0); synchronises. Same arithmetic as the per-value load.
template <int NTH, class C>
__device__ __forceinline__ void stage_tangled_rows(const Grid& g, const C* __restrict__ spec, const C* __restrict__ post,
                                                   C* __restrict__ lds, int lnl, int ls, int M, int row0, int nrows) {
    const int total = (1 << lnl) * M;
    const float rM = __builtin_amdgcn_rcpf(static_cast<float>(M));
    for (int t0 = 0; t0 < total; t0 += kXBatch * NTH) {
        C xk[kXBatch], xm[kXBatch], wk[kXBatch];
#pragma unroll
        for (int j = 0; j < kXBatch; ++j) {
            const int t = min(t0 + j * NTH + static_cast<int>(threadIdx.x), total - 1);
            int k;
            const int l = fdivmod(t, M, rM, k);
            const C* sr = spec + int64_t(min(row0 + l, nrows - 1)) * g.sx;
            xk[j] = sr[k];
            xm[j] = sr[M - k];
            wk[j] = post[k];
        }
#pragma unroll
        for (int j = 0; j < kXBatch; ++j) {
            const int t = t0 + j * NTH + static_cast<int>(threadIdx.x);
            if (t < total) {
                int k;
                const int l = fdivmod(t, M, rM, k);
                const C xc = cconj(xm[j]);
                const C e = cadd(xk[j], xc);
                const C o = cmulc(csub(xk[j], xc), wk[j]);
                lds[k * ls + l] = row0 + l < nrows ? C{e.x - o.y, e.y + o.x} : C{real_of<C>(0), real_of<C>(0)};
            }
        }
    }
    __syncthreads();
}

// x pass, inverse: half spectrum -> real rows, scaled by n_x (unnormalised).
// Z[k] = (X[k] + conj X[M-k]) + i (X[k] - conj X[M-k]) conj(W^k), z = IFFT_M(Z),
// x[2m] = Re z[m], x[2m+1] = Im z[m]. The tangled rows are staged in LDS; the
// last stage writes the real rows directly (element-fast).
template <int VM, int NTH, class C = cd>
__global__ __launch_bounds__(NTH) void k_fft_x_inv(Grid g, const C* __restrict__ spec, real_of<C>* __restrict__ p,
                                                        FftPlan P, const C* __restrict__ post, int lnl) {
    extern __shared__ __align__(16) unsigned char fft_smem[];
    C* lds = reinterpret_cast<C*>(fft_smem);
    const int nl = 1 << lnl;
    const int ls = nl + P.pad;
    const int M = P.n;
    const int nrows = g.batch * g.nz * g.ny;
    const int row0 = xcd_logical(blockIdx.x, gridDim.x) * nl;
    auto sink = [&](int l, int m, C z) INS_INLINE {
        const int row = row0 + l;
        if (row < nrows) reinterpret_cast<C*>(p + int64_t(row) * g.nx)[m] = z;
    };
    const NoOp nop;
    const TabTw<C> rt = plan_tab<C>(P);
    stage_tangled_rows<NTH>(g, spec, post, lds, lnl, ls, M, row0, nrows);
    fft_run<1, VM, NTH, 1, 1, kLineFast, kElemFast>(lds, lnl, ls, P, rt, nop, sink, nop, nullptr);
}

// Strided complex pass along y (axis 1) or z (axis 2) of the half spectrum
// [batch][n_z][n_y][sx] (columns 0 .. n_x/2 in use). MODE 0 forward, 1 inverse, 2 forward + divide +
// inverse. Columns kx < n_x/2 go in chunks of nl adjacent kx per batch (each
// access a contiguous run of nl values); the Nyquist column kx = n_x/2 is taken
// by extra batches, nl lines of it (adjacent values of the other non-x index)
// each, so no batch transforms a chunk that is mostly padding. Either way line
// l of a batch starts at lb0 + l*lstep, has wavenumbers (kx0 + l*kxstep,
// fk0 + l*fkstep) and exists for l < nvalid.
struct LineBatch {
    int64_t lb0, lstep;
    int kx0, kxstep, fk0, fkstep, nvalid;
};

__device__ __forceinline__ LineBatch line_batch(const Grid& g, int axis, int lnl, int w) {
    const int M = g.nx / 2;
    const int nchunk = (M + (1 << lnl) - 1) >> lnl;
    const int nfix = axis == 1 ? g.nz : g.ny;  // the other non-x index
    const int nouter = g.batch * nfix;
    const int64_t plane = int64_t(g.nz) * g.ny * g.sx;                          // one batch entry
    const int64_t fstride = axis == 1 ? int64_t(g.sx) * g.ny : int64_t(g.sx);  // along the other index
    LineBatch B;
    if (w < nchunk * nouter) {
        const int outer = w / nchunk;
        const int b = outer / nfix, f = outer - b * nfix;
        B.kx0 = (w - outer * nchunk) << lnl;
        B.kxstep = 1;
        B.fk0 = f;
        B.fkstep = 0;
        B.lb0 = b * plane + f * fstride + B.kx0;
        B.lstep = 1;
        B.nvalid = M - B.kx0;
    } else {
        const int nfc = (nfix + (1 << lnl) - 1) >> lnl;
        const int j = w - nchunk * nouter;
        const int b = j / nfc;
        const int f0 = (j - b * nfc) << lnl;
        B.kx0 = M;
        B.kxstep = 0;
        B.fk0 = f0;
        B.fkstep = 1;
        B.lb0 = b * plane + f0 * fstride + M;
        B.lstep = fstride;
        B.nvalid = nfix - f0;
    }
    return B;
}

// Number of batches of a strided pass.
__host__ __device__ __forceinline__ int strided_batches(const Grid& g, int axis, int lnl) {
    const int nchunk = (g.nx / 2 + (1 << lnl) - 1) >> lnl;
    const int nfix = axis == 1 ? g.nz : g.ny;
    return nchunk * g.batch * nfix + g.batch * ((nfix + (1 << lnl) - 1) >> lnl);
}

// 1 / a to working precision: the hardware estimate refined by Newton's
// iteration r <- r + r (1 - a r) (each step squares the relative error).
__device__ __forceinline__ double recip(double a) {
    double r = __builtin_amdgcn_rcp(a);
    r = fma(r, fma(-a, r, 1.0), r);
    r = fma(r, fma(-a, r, 1.0), r);
    return fma(r, fma(-a, r, 1.0), r);
}
__device__ __forceinline__ float recip(float a) {
    const float r = __builtin_amdgcn_rcpf(a);
    return fmaf(r, fmaf(-a, r, 1.0f), r);
}

// The eigenvalue sum of the directions other than the line's, for this
// thread's line of batch B (line-fast mapping: a thread's butterflies all lie
// on line threadIdx.x mod nl), and whether those wavenumbers are all zero.
template <class F>
struct LineLam {
    F other;
    bool zero;
};
template <class C>
__device__ __forceinline__ LineLam<real_of<C>> line_lam(const SolveTab& st, const LineBatch& B, int axis, int lnl) {
    const auto* const* lt = solve_lam(st, C{});
    const int l = min(static_cast<int>(threadIdx.x) & ((1 << lnl) - 1), B.nvalid - 1);
    const int kx = B.kx0 + l * B.kxstep, fk = B.fk0 + l * B.fkstep;
    if (axis == 2) return {lt[0][kx] + lt[1][fk], kx == 0 && fk == 0};
    return {lt[0][kx], kx == 0};
}

// One batch of a strided pass per workgroup (NT: non-temporal spectrum access).
template <int MODE, int VM, int NTH, bool NT, class C>
__device__ __forceinline__ void strided_batch(const Grid& g, C* __restrict__ spec, const FftPlan& P, const FftPlan& Q,
                                              int axis, int lnl, const SolveTab& st, int w, C* lds,
                                              const Roots<C>& rt, const real_of<C>* lam_line) {
    using F = real_of<C>;
    const int ls = (1 << lnl) + P.pad;
    const int64_t stride = axis == 1 ? int64_t(g.sx) : int64_t(g.sx) * g.ny;  // along the line
    const LineBatch B = line_batch(g, axis, lnl, w);
    auto load = [&](int l, int e) INS_INLINE -> C {
        if (l >= B.nvalid) return C{F(0), F(0)};
        const C* q = spec + B.lb0 + l * B.lstep + e * stride;
        if constexpr (NT) return ld_stream_c(q);
        else return *q;
    };
    auto store = [&](int l, int e, C z) INS_INLINE {
        if (l >= B.nvalid) return;
        C* q = spec + B.lb0 + l * B.lstep + e * stride;
        if constexpr (NT) st_stream_c(q, z);
        else *q = z;
    };
    const NoOp nop;
    if constexpr (MODE == 1) {
        fft_run<1, VM, NTH, 0, 1, kLineFast, kLineFast>(lds, lnl, ls, P, rt, load, store, nop, nullptr);
    } else if constexpr (MODE == 0) {
        fft_run<-1, VM, NTH, 0, 1, kLineFast, kLineFast>(lds, lnl, ls, P, rt, load, store, nop, nullptr);
    } else {
        // divide by L(k) * #cells; L(0) := 1.
        const LineLam<F> lam = line_lam<C>(st, B, axis, lnl);
        const F inv_ncell = solve_inv_ncell(st, C{});
        auto divide = [&](int l, int e, C z) INS_INLINE -> C {
            if (l >= B.nvalid) return z;
            const F sc = (lam.zero && e == 0) ? inv_ncell : -inv_ncell * recip(lam.other + lam_line[e]);
            return cscale(z, sc);
        };
        fft_run<-1, VM, NTH, 0, 2, kLineFast, kLineFast>(lds, lnl, ls, P, rt, load, store, divide, &Q);
        fft_inverse_rest<1, VM, NTH, kLineFast>(lds, lnl, ls, Q, rt, store);
    }
}

// First and last stages touch memory directly; in MODE 2 the forward run leaves
// its outputs in registers, they are divided there, and the inverse runs the
// stages in reverse radix order (plan Q, whose first radix is P's last) from
// those same registers. LDS: the line batch, then the roots, then (MODE 2) the
// eigenvalues of the line axis.
template <int MODE, int VM, int NTH, bool NT, class C = cd>
__global__ __launch_bounds__(NTH) void k_fft_strided(Grid g, C* __restrict__ spec, FftPlan P, FftPlan Q, int axis,
                                                          int lnl, SolveTab st) {
    using F = real_of<C>;
    extern __shared__ __align__(16) unsigned char fft_smem[];
    C* lds = reinterpret_cast<C*>(fft_smem);
    const int ls = (1 << lnl) + P.pad;
    const Roots<C> rt = load_roots<NTH>(lds + ls * P.n, P);
    F* lam_line = nullptr;
    if constexpr (MODE == 2) {
        lam_line = reinterpret_cast<F*>(lds + ls * P.n + roots_count(P.n));
        const F* src = solve_lam(st, C{})[axis];
        for (int j = threadIdx.x; j < P.n; j += NTH) lam_line[j] = src[j];
    }
    __syncthreads();  // roots and eigenvalues in LDS before any stage
    strided_batch<MODE, VM, NTH, NT>(g, spec, P, Q, axis, lnl, st, xcd_logical(blockIdx.x, gridDim.x), lds, rt,
                                     lam_line);
}

// ----------------------------------------------------------------------------
// Launchers
// ----------------------------------------------------------------------------
namespace {

template <typename T, class C>
hipError_t fft_x_fwd(const Grid& g, const T* vel, const real_of<C>* r, C* spec, const FftPlan& px, const C* post,
                     int lnl, hipStream_t s, int comp) {
    const int nl = 1 << lnl;
    const int nrows = g.batch * g.nz * g.ny;
    const int nblk = (nrows + nl - 1) / nl;
    const size_t shm = size_t(nl + px.pad) * px.n * sizeof(C);
#define INS_XF(D, SRC, VM, NTH)                                                                                \
    hipLaunchKernelGGL((k_fft_x_fwd<T, D, SRC, VM, NTH, C>), dim3(nblk), dim3(NTH), shm, s, g, vel, r, spec, px, post, \
                       lnl, comp)
#define INS_XF_VM(D, SRC)                                    \
    do {                                                     \
        if (px.nth == 512) INS_XF(D, SRC, 10, 512);          \
        else if (px.vm == 8) INS_XF(D, SRC, 8, 256);         \
        else INS_XF(D, SRC, 16, 256);                        \
    } while (0)
    if (vel && comp < 0) {
        if (g.dim == 3) INS_XF_VM(3, 0); else INS_XF_VM(2, 0);
    } else if (vel) {
        if (g.dim == 3) INS_XF_VM(3, 2); else INS_XF_VM(2, 2);
    } else {
        INS_XF_VM(3, 1);
    }
#undef INS_XF_VM
#undef INS_XF
    return hipGetLastError();
}

template <class C>
hipError_t fft_x_inv(const Grid& g, const C* spec, real_of<C>* p, const FftPlan& px, const C* post, int lnl,
                     hipStream_t s) {
    const int nl = 1 << lnl;
    const int nrows = g.batch * g.nz * g.ny;
    const int nblk = (nrows + nl - 1) / nl;
    const size_t shm = size_t(nl + px.pad) * px.n * sizeof(C);
    if (px.nth == 512)
        hipLaunchKernelGGL((k_fft_x_inv<10, 512, C>), dim3(nblk), dim3(512), shm, s, g, spec, p, px, post, lnl);
    else if (px.vm == 8)
        hipLaunchKernelGGL((k_fft_x_inv<8, 256, C>), dim3(nblk), dim3(256), shm, s, g, spec, p, px, post, lnl);
    else
        hipLaunchKernelGGL((k_fft_x_inv<16, 256, C>), dim3(nblk), dim3(256), shm, s, g, spec, p, px, post, lnl);
    return hipGetLastError();
}

template <class C>
hipError_t fft_strided(const Grid& g, C* spec, const FftPlan& pl, const FftPlan& rev, int axis, int mode, int lnl,
                       const SolveTab& st, hipStream_t s) {
    const int nl = 1 << lnl;
    const int nwork = strided_batches(g, axis, lnl);
    const size_t shm = (size_t(nl + pl.pad) * pl.n + roots_count(pl.n)) * sizeof(C) +
                       (mode == 2 ? size_t(pl.n) * sizeof(real_of<C>) : 0);
    // non-temporal access once the spectrum is well beyond the 256 MB MALL and the
    // batches give 128-byte runs (512^3: y passes 7-10% faster; with the 64-byte
    // runs of 840 lines it changed nothing)
    const bool nt = nl >= 8 && size_t(g.batch) * g.nz * g.ny * g.sx * sizeof(C) > (size_t(512) << 20);
#define INS_ST2(MODE, VM, NTH, NT)                                                                                   \
    hipLaunchKernelGGL((k_fft_strided<MODE, VM, NTH, NT, C>), dim3(nwork), dim3(NTH), shm, s, g, spec, pl, rev, axis, \
                       lnl, st)
#define INS_ST(MODE, VM, NTH)                                            \
    do {                                                                 \
        if (nt) INS_ST2(MODE, VM, NTH, true);                            \
        else INS_ST2(MODE, VM, NTH, false);                              \
    } while (0)
#define INS_ST_VM(MODE)                                                  \
    do {                                                                 \
        if (pl.nth == 512) INS_ST(MODE, 8, 512);                         \
        else if (pl.vm == 8) INS_ST(MODE, 8, 256);                       \
        else INS_ST(MODE, 16, 256);                                      \
    } while (0)
    if (mode == 0)
        INS_ST_VM(0);
    else if (mode == 1)
        INS_ST_VM(1);
    else
        INS_ST_VM(2);
#undef INS_ST_VM
#undef INS_ST
#undef INS_ST2
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_fft_x_fwd(const Grid& g, const T* vel, const double* r, cd* spec, const FftPlan& px, const cd* post,
                            int lnl, hipStream_t s, int comp) {
    return fft_x_fwd<T, cd>(g, vel, r, spec, px, post, lnl, s, comp);
}

hipError_t launch_fft_x_inv(const Grid& g, const cd* spec, double* p, const FftPlan& px, const cd* post, int lnl,
                            hipStream_t s) {
    return fft_x_inv<cd>(g, spec, p, px, post, lnl, s);
}

hipError_t launch_fft_strided(const Grid& g, cd* spec, const FftPlan& pl, const FftPlan& rev, int axis, int mode,
                              int lnl, const SolveTab& st, hipStream_t s) {
    return fft_strided<cd>(g, spec, pl, rev, axis, mode, lnl, st, s);
}

hipError_t launch_fft_x_fwd_f32(const Grid& g, const float* vel, const float* r, cf* spec, const FftPlan& px,
                                const cf* post, int lnl, hipStream_t s) {
    return fft_x_fwd<float, cf>(g, vel, r, spec, px, post, lnl, s, -1);
}

hipError_t launch_fft_x_inv_f32(const Grid& g, const cf* spec, float* p, const FftPlan& px, const cf* post, int lnl,
                                hipStream_t s) {
    return fft_x_inv<cf>(g, spec, p, px, post, lnl, s);
}

hipError_t launch_fft_strided_f32(const Grid& g, cf* spec, const FftPlan& pl, const FftPlan& rev, int axis, int mode,
                                  int lnl, const SolveTab& st, hipStream_t s) {
    return fft_strided<cf>(g, spec, pl, rev, axis, mode, lnl, st, s);
}

template <typename T>
hipError_t launch_fft_x_fwd_wall(const Grid& g, const T* vel, bool scaled, cd* spec, const FftPlan& px, const cd* post,
                                 int lnl, hipStream_t s) {
    const int nl = 1 << lnl;
    const int nrows = g.batch * g.nz * g.ny;
    const int nblk = (nrows + nl - 1) / nl;
    const size_t shm = size_t(nl + px.pad) * px.n * sizeof(cd);
#define INS_XF(D, SRC, VM, NTH)                                                                                \
    hipLaunchKernelGGL((k_fft_x_fwd<T, D, SRC, VM, NTH>), dim3(nblk), dim3(NTH), shm, s, g, vel, nullptr, spec, px, \
                       post, lnl, 0)
#define INS_XF_VM(D, SRC)                                    \
    do {                                                     \
        if (px.nth == 512) INS_XF(D, SRC, 10, 512);          \
        else if (px.vm == 8) INS_XF(D, SRC, 8, 256);         \
        else INS_XF(D, SRC, 16, 256);                        \
    } while (0)
    if (g.dim == 3) {
        if (scaled) INS_XF_VM(3, 4); else INS_XF_VM(3, 3);
    } else {
        if (scaled) INS_XF_VM(2, 4); else INS_XF_VM(2, 3);
    }
#undef INS_XF_VM
#undef INS_XF
    return hipGetLastError();
}

template hipError_t launch_fft_x_fwd_wall<double>(const Grid&, const double*, bool, cd*, const FftPlan&, const cd*,
                                                  int, hipStream_t);
template hipError_t launch_fft_x_fwd_wall<float>(const Grid&, const float*, bool, cd*, const FftPlan&, const cd*, int,
                                                 hipStream_t);
template hipError_t launch_fft_x_fwd<double>(const Grid&, const double*, const double*, cd*, const FftPlan&, const cd*,
                                             int, hipStream_t, int);
template hipError_t launch_fft_x_fwd<float>(const Grid&, const float*, const double*, cd*, const FftPlan&, const cd*,
                                            int, hipStream_t, int);

}  // namespace ins
