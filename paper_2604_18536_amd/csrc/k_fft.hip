// Spectral pressure solve of Sec. 2.5.1 on gfx950: p = DFT^-1 L^-1 DFT r with
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
// All spectral arithmetic is float64.
#include "k_common.hpp"

namespace ins {

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
template <int SIGN>
__device__ __forceinline__ cd rot(cd z) {
    return SIGN < 0 ? cd{z.y, -z.x} : cd{-z.y, z.x};
}

// Small DFTs X[m] = sum_q x[q] exp(SIGN 2 pi i q m / R), in place.
template <int SIGN>
__device__ __forceinline__ void dft2(cd* v) {
    const cd a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <int SIGN>
__device__ __forceinline__ void dft4(cd& x0, cd& x1, cd& x2, cd& x3) {
    const cd s02 = cadd(x0, x2), d02 = csub(x0, x2);
    const cd s13 = cadd(x1, x3), d13 = rot<SIGN>(csub(x1, x3));
    x0 = cadd(s02, s13);
    x2 = csub(s02, s13);
    x1 = cadd(d02, d13);
    x3 = csub(d02, d13);
}

template <int SIGN>
__device__ __forceinline__ void dft8(cd* v) {
    cd e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cd o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<SIGN>(e0, e1, e2, e3);
    dft4<SIGN>(o0, o1, o2, o3);
    constexpr double r = 0.7071067811865476;
    // w^1 = (1 + SIGN i)/sqrt2, w^2 = SIGN i, w^3 = (-1 + SIGN i)/sqrt2
    const cd t1 = {r * (o1.x - SIGN * o1.y), r * (o1.y + SIGN * o1.x)};
    const cd t2 = rot<SIGN>(o2);
    const cd t3 = {r * (-o3.x - SIGN * o3.y), r * (-o3.y + SIGN * o3.x)};
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
template <int R, int SIGN>
__device__ __forceinline__ void dft_odd(cd* v) {
    constexpr int H = (R - 1) / 2;
    cd s[H], d[H];
#pragma unroll
    for (int q = 1; q <= H; ++q) {
        s[q - 1] = cadd(v[q], v[R - q]);
        d[q - 1] = csub(v[q], v[R - q]);
    }
    const cd x0 = v[0];
    cd sum = x0;
#pragma unroll
    for (int q = 0; q < H; ++q) sum = cadd(sum, s[q]);
    v[0] = sum;
#pragma unroll
    for (int m = 1; m <= H; ++m) {
        cd A = x0, B = {0.0, 0.0};
#pragma unroll
        for (int q = 1; q <= H; ++q) {
            const int j = (q * m) % R;
            A.x += s[q - 1].x * kcos(R, j);
            A.y += s[q - 1].y * kcos(R, j);
            B.x += d[q - 1].x * ksin(R, j);
            B.y += d[q - 1].y * ksin(R, j);
        }
        const cd iB = rot<SIGN>(B);
        v[m] = cadd(A, iB);
        v[R - m] = csub(A, iB);
    }
}

template <int R, int SIGN>
__device__ __forceinline__ void dft(cd* v) {
    if constexpr (R == 2) dft2<SIGN>(v);
    else if constexpr (R == 4) dft4<SIGN>(v[0], v[1], v[2], v[3]);
    else if constexpr (R == 8) dft8<SIGN>(v);
    else dft_odd<R, SIGN>(v);
}

// One Stockham stage over `nl` lines of length N stored element-major in LDS
// (element j of line l at lds[j*nl + l]). Butterfly i of a line reads
// elements i + q N/R, multiplies by exp(SIGN 2 pi i q k / (p R)) with k = i mod p,
// applies DFT_R and writes elements (i - k) R + k + q p.
template <int R, int SIGN, int VM>
__device__ __forceinline__ void fft_stage(cd* __restrict__ lds, int lnl, int ls, int N, int p, const cd* __restrict__ tw) {
    constexpr int BMAX = VM / R > 0 ? VM / R : 1;
    const int nl = 1 << lnl;
    const int s = N / R;
    const int nb = s << lnl;
    cd v[BMAX][R];
#pragma unroll
    for (int b = 0; b < BMAX; ++b) {
        const int t = threadIdx.x + b * kBlock;
        if (t < nb) {
            const int l = t & (nl - 1), i = t >> lnl;
#pragma unroll
            for (int q = 0; q < R; ++q) v[b][q] = lds[(i + q * s) * ls + l];
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BMAX; ++b) {
        const int t = threadIdx.x + b * kBlock;
        if (t < nb) {
            const int l = t & (nl - 1), i = t >> lnl;
            const int k = i % p;
            if (k != 0) {
                const cd* twk = tw + k * (R - 1) - 1;
#pragma unroll
                for (int q = 1; q < R; ++q) v[b][q] = SIGN < 0 ? cmul(v[b][q], twk[q]) : cmulc(v[b][q], twk[q]);
            }
            dft<R, SIGN>(v[b]);
            const int base = (i - k) * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) lds[(base + q * p) * ls + l] = v[b][q];
        }
    }
    __syncthreads();
}

// Full FFT of the lines in LDS; the caller has synchronised after filling LDS.
template <int SIGN, int VM>
__device__ void fft_lines(cd* lds, int lnl, const FftPlan& P) {
    const int ls = (1 << lnl) + P.pad;
    int p = 1;
    for (int st = 0; st < P.nst; ++st) {
        const int R = P.rad[st];
        const cd* tw = P.tw + P.tw_off[st];
        switch (R) {
            case 8: fft_stage<8, SIGN, VM>(lds, lnl, ls, P.n, p, tw); break;
            case 7: fft_stage<7, SIGN, VM>(lds, lnl, ls, P.n, p, tw); break;
            case 5: fft_stage<5, SIGN, VM>(lds, lnl, ls, P.n, p, tw); break;
            case 4: fft_stage<4, SIGN, VM>(lds, lnl, ls, P.n, p, tw); break;
            case 3: fft_stage<3, SIGN, VM>(lds, lnl, ls, P.n, p, tw); break;
            default: fft_stage<2, SIGN, VM>(lds, lnl, ls, P.n, p, tw); break;
        }
        p *= R;
    }
}

// ----------------------------------------------------------------------------
// x pass, forward: real rows (n_x = 2M) -> half spectrum X[0..M].
// Packing: z[m] = x[2m] + i x[2m+1]; Z = FFT_M(z);
// X[k] = (Z[k] + conj Z[M-k]) / 2 + W^k (Z[k] - conj Z[M-k]) / (2i), W = exp(-2 pi i / n_x).
// ----------------------------------------------------------------------------
// SRC 0: rows are the divergence of the velocity field `vel`;
// SRC 1: rows of the float64 scalar field r; SRC 2: rows of component `comp` of vel.
template <typename T, int DIM, int SRC, int VM>
__global__ __launch_bounds__(kBlock) void k_fft_x_fwd(Grid g, const T* __restrict__ vel, const double* __restrict__ r,
                                                        cd* __restrict__ spec, FftPlan P, const cd* __restrict__ post,
                                                        int lnl, int comp) {
    extern __shared__ cd lds[];
    const int nl = 1 << lnl;
    const int M = P.n;
    const int nrows = g.batch * g.nz * g.ny;
    const int row0 = xcd_logical(blockIdx.x, gridDim.x) * nl;
    for (int t = threadIdx.x; t < nl * M; t += kBlock) {
        const int l = t / M, m = t - l * M;
        const int row = row0 + l;
        cd val = {0.0, 0.0};
        if (row < nrows) {
            if constexpr (SRC == 0) {
                const int yy = row % g.ny;
                const int zb = row / g.ny;
                const int zz = zb % g.nz;
                const int b = zb / g.nz;
                const T* wb = vel + int64_t(b) * DIM * g.ncell;
                const int rowoff = (zz * g.ny + yy) * g.nx;
                const int x0 = 2 * m;
                const int xm = x0 == 0 ? g.nx - 1 : x0 - 1;
                const T* wx = wb + rowoff;
                const double ux_m = wx[xm], ux_0 = wx[x0], ux_1 = wx[x0 + 1];
                double r0 = (ux_0 - ux_m) * g.ih[0];
                double r1 = (ux_1 - ux_0) * g.ih[0];
                const int ym = yy == 0 ? g.ny - 1 : yy - 1;
                const T* wy = wb + g.ncell;
                const int rowy = (zz * g.ny + ym) * g.nx;
                r0 += (double(wy[rowoff + x0]) - double(wy[rowy + x0])) * g.ih[1];
                r1 += (double(wy[rowoff + x0 + 1]) - double(wy[rowy + x0 + 1])) * g.ih[1];
                if constexpr (DIM == 3) {
                    const int zm = zz == 0 ? g.nz - 1 : zz - 1;
                    const T* wz = wb + 2 * g.ncell;
                    const int rowz = (zm * g.ny + yy) * g.nx;
                    r0 += (double(wz[rowoff + x0]) - double(wz[rowz + x0])) * g.ih[2];
                    r1 += (double(wz[rowoff + x0 + 1]) - double(wz[rowz + x0 + 1])) * g.ih[2];
                }
                val = {r0, r1};
            } else if constexpr (SRC == 1) {
                val = reinterpret_cast<const cd*>(r + int64_t(row) * g.nx)[m];
            } else {
                const int yy = row % g.ny;
                const int zb = row / g.ny;
                const int zz = zb % g.nz;
                const int b = zb / g.nz;
                const T* src = vel + (int64_t(b) * DIM + comp) * g.ncell + int64_t(zz * g.ny + yy) * g.nx;
                val = {double(src[2 * m]), double(src[2 * m + 1])};
            }
        }
        lds[m * (nl + P.pad) + l] = val;
    }
    __syncthreads();
    fft_lines<-1, VM>(lds, lnl, P);
    const int M1 = M + 1;
    for (int t = threadIdx.x; t < nl * M1; t += kBlock) {
        const int l = t / M1, k = t - l * M1;
        const int row = row0 + l;
        if (row >= nrows) continue;
        const cd zk = lds[(k == M ? 0 : k) * (nl + P.pad) + l];
        const cd zc = cconj(lds[(k == 0 ? 0 : M - k) * (nl + P.pad) + l]);
        const cd e = cscale(cadd(zk, zc), 0.5);
        const cd dd = csub(zk, zc);
        const cd o = {0.5 * dd.y, -0.5 * dd.x};
        spec[int64_t(row) * M1 + k] = cadd(e, cmul(post[k], o));
    }
}

// x pass, inverse: half spectrum -> real rows, scaled by n_x (unnormalised).
// Z[k] = (X[k] + conj X[M-k]) + i (X[k] - conj X[M-k]) conj(W^k), z = IFFT_M(Z),
// x[2m] = Re z[m], x[2m+1] = Im z[m].
template <int VM>
__global__ __launch_bounds__(kBlock) void k_fft_x_inv(Grid g, const cd* __restrict__ spec, double* __restrict__ p,
                                                        FftPlan P, const cd* __restrict__ post, int lnl) {
    extern __shared__ cd lds[];
    const int nl = 1 << lnl;
    const int M = P.n, M1 = M + 1;
    const int nrows = g.batch * g.nz * g.ny;
    const int row0 = xcd_logical(blockIdx.x, gridDim.x) * nl;
    for (int t = threadIdx.x; t < nl * M; t += kBlock) {
        const int l = t / M, k = t - l * M;
        const int row = row0 + l;
        cd z = {0.0, 0.0};
        if (row < nrows) {
            const cd* sr = spec + int64_t(row) * M1;
            const cd xk = sr[k];
            const cd xc = cconj(sr[M - k]);
            const cd e = cadd(xk, xc);
            const cd o = cmulc(csub(xk, xc), post[k]);
            z = {e.x - o.y, e.y + o.x};
        }
        lds[k * (nl + P.pad) + l] = z;
    }
    __syncthreads();
    fft_lines<1, VM>(lds, lnl, P);
    for (int t = threadIdx.x; t < nl * M; t += kBlock) {
        const int l = t / M, m = t - l * M;
        const int row = row0 + l;
        if (row >= nrows) continue;
        reinterpret_cast<cd*>(p + int64_t(row) * g.nx)[m] = lds[m * (nl + P.pad) + l];
    }
}

// Strided complex pass along y (axis 1) or z (axis 2) of the half spectrum
// [batch][n_z][n_y][n_x/2+1]. MODE 0 forward, 1 inverse, 2 forward + divide + inverse.
template <int MODE, int VM>
__global__ __launch_bounds__(kBlock) void k_fft_strided(Grid g, cd* __restrict__ spec, FftPlan P, int axis, int lnl,
                                                          SolveTab st) {
    extern __shared__ cd lds[];
    const int nl = 1 << lnl;
    const int nxh = g.nx / 2 + 1;
    const int nchunk = (nxh + nl - 1) >> lnl;
    const int wg = xcd_logical(blockIdx.x, gridDim.x);
    const int chunk = wg % nchunk;
    const int outer = wg / nchunk;
    const int N = P.n;
    int64_t base;
    int64_t stride;
    int fixed_k = 0;  // the other (non-line, non-x) wavenumber of this line
    if (axis == 1) {
        stride = nxh;
        base = int64_t(outer) * g.ny * nxh;  // outer = (b, z)
        fixed_k = outer % g.nz;
    } else {
        stride = int64_t(nxh) * g.ny;
        const int yy = outer % g.ny, b = outer / g.ny;
        base = int64_t(b) * g.nz * g.ny * nxh + int64_t(yy) * nxh;
        fixed_k = yy;
    }
    const int kx0 = chunk << lnl;
    base += kx0;
    const int ntot = N << lnl;
    const int ls = nl + P.pad;
    for (int t = threadIdx.x; t < ntot; t += kBlock) {
        const int c = t & (nl - 1), j = t >> lnl;
        lds[j * ls + c] = (kx0 + c < nxh) ? spec[base + j * stride + c] : cd{0.0, 0.0};
    }
    __syncthreads();
    if constexpr (MODE == 1) {
        fft_lines<1, VM>(lds, lnl, P);
    } else {
        fft_lines<-1, VM>(lds, lnl, P);
    }
    if constexpr (MODE == 2) {
        // divide by L(k) * #cells; L(0) := 1.
        for (int t = threadIdx.x; t < ntot; t += kBlock) {
            const int c = t & (nl - 1), j = t >> lnl;
            const int kx = kx0 + c;
            if (kx >= nxh) continue;
            double lam, kzero;
            if (axis == 2) {
                lam = st.lam[0][kx] + st.lam[1][fixed_k] + st.lam[2][j];
                kzero = (kx == 0 && fixed_k == 0 && j == 0);
            } else {
                lam = st.lam[0][kx] + st.lam[1][j];
                kzero = (kx == 0 && j == 0);
            }
            const double sc = kzero ? st.inv_ncell : -st.inv_ncell / lam;
            lds[j * ls + c] = cscale(lds[j * ls + c], sc);
        }
        __syncthreads();
        fft_lines<1, VM>(lds, lnl, P);
    }
    for (int t = threadIdx.x; t < ntot; t += kBlock) {
        const int c = t & (nl - 1), j = t >> lnl;
        if (kx0 + c < nxh) spec[base + j * stride + c] = lds[j * ls + c];
    }
}

// ----------------------------------------------------------------------------
// Launchers
// ----------------------------------------------------------------------------
template <typename T>
hipError_t launch_fft_x_fwd(const Grid& g, const T* vel, const double* r, cd* spec, const FftPlan& px, const cd* post,
                            int lnl, hipStream_t s, int comp) {
    const int nl = 1 << lnl;
    const int nrows = g.batch * g.nz * g.ny;
    const int nblk = (nrows + nl - 1) / nl;
    const size_t shm = size_t(nl + px.pad) * px.n * sizeof(cd);
#define INS_XF(D, SRC, VM) \
    hipLaunchKernelGGL((k_fft_x_fwd<T, D, SRC, VM>), dim3(nblk), dim3(kBlock), shm, s, g, vel, r, spec, px, post, lnl, comp)
#define INS_XF_VM(D, SRC) \
    do { if (px.vm == 8) INS_XF(D, SRC, 8); else INS_XF(D, SRC, 16); } while (0)
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

hipError_t launch_fft_x_inv(const Grid& g, const cd* spec, double* p, const FftPlan& px, const cd* post, int lnl,
                            hipStream_t s) {
    const int nl = 1 << lnl;
    const int nrows = g.batch * g.nz * g.ny;
    const int nblk = (nrows + nl - 1) / nl;
    const size_t shm = size_t(nl + px.pad) * px.n * sizeof(cd);
    if (px.vm == 8)
        hipLaunchKernelGGL(k_fft_x_inv<8>, dim3(nblk), dim3(kBlock), shm, s, g, spec, p, px, post, lnl);
    else
        hipLaunchKernelGGL(k_fft_x_inv<16>, dim3(nblk), dim3(kBlock), shm, s, g, spec, p, px, post, lnl);
    return hipGetLastError();
}

hipError_t launch_fft_strided(const Grid& g, cd* spec, const FftPlan& pl, int axis, int mode, int lnl,
                              const SolveTab& st, hipStream_t s) {
    const int nl = 1 << lnl;
    const int nxh = g.nx / 2 + 1;
    const int nchunk = (nxh + nl - 1) / nl;
    const int nouter = axis == 1 ? g.batch * g.nz : g.batch * g.ny;
    const int nblk = nchunk * nouter;
    const size_t shm = size_t(nl + pl.pad) * pl.n * sizeof(cd);
#define INS_ST(MODE, VM) \
    hipLaunchKernelGGL((k_fft_strided<MODE, VM>), dim3(nblk), dim3(kBlock), shm, s, g, spec, pl, axis, lnl, st)
#define INS_ST_VM(MODE) \
    do { if (pl.vm == 8) INS_ST(MODE, 8); else INS_ST(MODE, 16); } while (0)
    if (mode == 0)
        INS_ST_VM(0);
    else if (mode == 1)
        INS_ST_VM(1);
    else
        INS_ST_VM(2);
#undef INS_ST_VM
#undef INS_ST
    return hipGetLastError();
}

template hipError_t launch_fft_x_fwd<double>(const Grid&, const double*, const double*, cd*, const FftPlan&, const cd*,
                                             int, hipStream_t, int);
template hipError_t launch_fft_x_fwd<float>(const Grid&, const float*, const double*, cd*, const FftPlan&, const cd*,
                                            int, hipStream_t, int);

}  // namespace ins
