// Learned closure m_theta(u) (Sec. 4 of the paper: a neural closure embedded in
// the solver and trained through it) as hand-written bfloat16 MFMA kernels for
// gfx950: a 3D CNN 3 -> 32 -> 32 -> 3 channels, 3x3x3 kernels, circular
// padding, exact GELU, FP32 accumulation.
//
// Activations are channels-last bfloat16 ([cell][C], C = 8 for the packed
// 3-channel input, 32 for hidden layers). A convolution is an implicit GEMM
// D[cell][n] = sum_k A[cell][k] B[k][n] with k = (tap, channel), executed as
// v_mfma_f32_16x16x32_bf16 tiles (lane l holds A[m = l%16][k = 8(l/16)+j],
// B[k = 8(l/16)+j][n = l%16], D[m = 4(l/16)+i][n = l%16]). A K tile of 32 is
// one tap x 32 channels (C = 32) or four taps x 8 channels (C = 8); every lane
// fetches its 8 bfloat16 operands with one 16-byte load. Weights are packed per
// K tile ([kt][n][32]) and staged once per workgroup in LDS. The input
// gradient (dgrad) is the same kernel with flipped taps and transposed
// weights; the weight gradient (wgrad) reduces over cells with operands
// transposed through LDS and per-workgroup partial sums.
#include <hip/hip_bf16.h>

#include "k_common.hpp"

namespace ins {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int kTaps = 27;

__device__ __forceinline__ u16 bf16_bits(float v) {
    const __bf16 b = __bf16(v);  // round to nearest even
    return __builtin_bit_cast(u16, b);
}
__device__ __forceinline__ float bf16_val(u16 bits) { return float(__builtin_bit_cast(__bf16, bits)); }

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// A run of cells inside one x-row (n_x is a multiple of 32, so a 16-cell tile or
// a 32-cell strip never straddles rows): its row coordinates, in 32-bit
// arithmetic (the closure requires fewer than 2^31 cells in the batch).
struct RowPos {
    int x0, y, z, b;
};

__device__ __forceinline__ RowPos row_of(const Grid& g, int first_cell) {
    RowPos r;
    const int row = first_cell / g.nx;
    r.x0 = first_cell - row * g.nx;
    r.y = row % g.ny;
    const int zb = row / g.ny;
    r.z = zb % g.nz;
    r.b = zb / g.nz;
    return r;
}

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// First cell of the row shifted by (dy, dz) with periodic wrap.
__device__ __forceinline__ int row_start(const Grid& g, const RowPos& r, int dy, int dz) {
    return ((r.b * g.nz + wrapi(r.z + dz, g.nz)) * g.ny + wrapi(r.y + dy, g.ny)) * g.nx;
}

// K tile kt, lane group gq: which tap and which first channel the lane's 8 operands hold.
template <int CIN>
__device__ __forceinline__ void ktile_tap(int kt, int gq, int& tap, int& c0) {
    if constexpr (CIN == 32) {
        tap = kt;
        c0 = 8 * gq;
    } else {
        tap = 4 * kt + gq;
        c0 = 0;
    }
}

enum { EPI_HIDDEN = 0, EPI_OUT = 1, EPI_DGRAD_HIDDEN = 2, EPI_DGRAD_INPUT = 3 };

// Implicit-GEMM 3x3x3 convolution over all cells of the batch.
//   in   : [cells][CIN] bfloat16
//   wpk  : [NKT][NT*16][32] bfloat16 packed weights (zero where k or n is padding)
//   EPI_HIDDEN      : z = acc + bias -> zout [cells][32] fp32, a = bf16(gelu(z)) -> aout [cells][32]
//   EPI_OUT         : m[b][n][cell] = acc + bias (n < nout), field type T (planar velocity layout)
//   EPI_DGRAD_HIDDEN: zbar = acc * gelu'(zin[cell][n]) -> aout [cells][32] bf16
//   EPI_DGRAD_INPUT : ubar[b][n][cell] += acc (n < nout), field type T
template <typename T, int CIN, int NT, int EPI>
__global__ __launch_bounds__(kBlock) void k_conv(Grid g, int64_t ncells, const u16* __restrict__ in,
                                                   const u16* __restrict__ wpk, const float* __restrict__ bias,
                                                   const float* __restrict__ zin, float* __restrict__ zout,
                                                   u16* __restrict__ aout, T* __restrict__ fout, int nout) {
    constexpr int NKT = (kTaps * CIN + 31) / 32;
    constexpr int MT = 2;                       // M tiles (16 cells each) per wave
    constexpr int SEG = 4 * MT * 16;            // cells per workgroup iteration
    extern __shared__ __attribute__((aligned(16))) u16 wl[];  // NKT * NT*16 * 32
    const int tid = threadIdx.x;
    {
        const int n16 = NKT * NT * 16 * 32 / 8;  // 16-byte chunks
        const uint4* src = reinterpret_cast<const uint4*>(wpk);
        uint4* dst = reinterpret_cast<uint4*>(wl);
        for (int i = tid; i < n16; i += kBlock) dst[i] = src[i];
    }
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int lm = lane & 15, gq = lane >> 4;
    const int64_t nseg = (ncells + SEG - 1) / SEG;
    for (int64_t seg = blockIdx.x; seg < nseg; seg += gridDim.x) {
        const int64_t base = seg * SEG + int64_t(wave) * MT * 16;
        f32x4 acc[MT][NT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
        RowPos rp[MT];
        int xs[MT][3];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            int c = int(base) + mt * 16;
            c = c < ncells ? c : int(ncells) - 16;  // a tail tile reads valid cells; its results are not stored
            rp[mt] = row_of(g, c);
            const int x = rp[mt].x0 + lm;
            xs[mt][0] = wrapi(x - 1, g.nx);
            xs[mt][1] = x;
            xs[mt][2] = wrapi(x + 1, g.nx);
        }
#pragma unroll 3
        for (int kt = 0; kt < NKT; ++kt) {
            int tap, c0;
            ktile_tap<CIN>(kt, gq, tap, c0);
            const bool tap_ok = tap < kTaps;
            const int t = tap_ok ? tap : 0;
            const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dxi = t % 3;
            bf16x8 bv[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                bv[nt] = *reinterpret_cast<const bf16x8*>(wl + ((kt * NT * 16 + nt * 16 + lm) * 32 + 8 * gq));
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                bf16x8 av;
                if (tap_ok) {
                    const int nc = row_start(g, rp[mt], dy, dz) + xs[mt][dxi];
                    av = *reinterpret_cast<const bf16x8*>(in + int64_t(nc) * CIN + c0);
                } else {
#pragma unroll
                    for (int j = 0; j < 8; ++j) av[j] = __bf16(0.0f);
                }
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[nt], acc[mt][nt], 0, 0, 0);
            }
        }
        // epilogue: lane holds D[m = 4 gq + i][n = nt*16 + lm]
        const int64_t vol = int64_t(g.nx) * g.ny * g.nz;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t c = base + mt * 16 + 4 * gq + i;
                if (c >= ncells) continue;
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const int n = nt * 16 + lm;
                    const float v = acc[mt][nt][i];
                    if constexpr (EPI == EPI_HIDDEN) {
                        const float z = v + bias[n];
                        zout[c * 32 + n] = z;
                        aout[c * 32 + n] = bf16_bits(gelu_f(z));
                    } else if constexpr (EPI == EPI_DGRAD_HIDDEN) {
                        aout[c * 32 + n] = bf16_bits(v * gelu_grad_f(zin[c * 32 + n]));
                    } else {
                        if (n < nout) {
                            const int64_t b = c / vol, r = c - b * vol;
                            T* dst = fout + (b * 3 + n) * vol + r;
                            if constexpr (EPI == EPI_OUT)
                                *dst = T(v + bias[n]);
                            else
                                *dst = T(double(*dst) + double(v));
                        }
                    }
                }
            }
        }
    }
}

// Planar velocity (T) -> channels-last bfloat16 [cell][8] (channels 3..7 zero).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pack_input(int64_t ncells, int64_t vol, const T* __restrict__ u,
                                                         u16* __restrict__ x0) {
    const int64_t c = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (c >= ncells) return;
    const int64_t b = c / vol, r = c - b * vol;
    u16 v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a] = bf16_bits(float(u[(b * 3 + a) * vol + r]));
    uint4 out;
    out.x = v[0] | (unsigned(v[1]) << 16);
    out.y = v[2] | (unsigned(v[3]) << 16);
    out.z = v[4] | (unsigned(v[5]) << 16);
    out.w = v[6] | (unsigned(v[7]) << 16);
    reinterpret_cast<uint4*>(x0)[c] = out;
}

// FP32 parameters -> packed bfloat16 forward and dgrad weights.
// Forward layer (cin, cout): wf[kt][n][32], K tile kt covering (tap, channel) as in ktile_tap<CINP>.
// Dgrad of the layer: a convolution from cout channels to cin channels with
// W'[n = i][k = (t', o)] = W[o][i][26 - t'].
__global__ void k_pack_weights(const float* __restrict__ w, int cin, int cout, int cinp, int ntf, u16* __restrict__ wf,
                               int coutp, int ntd, u16* __restrict__ wd) {
    const int nktf = (kTaps * cinp + 31) / 32;
    const int nktd = (kTaps * coutp + 31) / 32;
    const int totf = nktf * ntf * 16 * 32;
    const int totd = nktd * ntd * 16 * 32;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < totf) {
        const int kk = i & 31, n = (i >> 5) % (ntf * 16), kt = i / (32 * ntf * 16);
        const int gq = kk >> 3, j = kk & 7;
        int tap, c;
        if (cinp == 32) {
            tap = kt;
            c = 8 * gq + j;
        } else {
            tap = 4 * kt + gq;
            c = j;
        }
        float v = 0.f;
        if (tap < kTaps && c < cin && n < cout) v = w[(n * cin + c) * kTaps + tap];
        wf[i] = bf16_bits(v);
    } else if (i < totf + totd) {
        const int e = i - totf;
        const int kk = e & 31, n = (e >> 5) % (ntd * 16), kt = e / (32 * ntd * 16);
        const int gq = kk >> 3, j = kk & 7;
        int tap, o;
        if (coutp == 32) {
            tap = kt;
            o = 8 * gq + j;
        } else {
            tap = 4 * kt + gq;
            o = j;
        }
        float v = 0.f;
        if (tap < kTaps && o < cout && n < cin) v = w[(o * cin + n) * kTaps + (kTaps - 1 - tap)];
        wd[e] = bf16_bits(v);
    }
}

// Weight gradient of one layer: W'[n][tap][c] = sum_p g[p][n] x[p + off(tap)][c],
// bias' [n] = sum_p g[p][n]. The reduction over cells runs over strips of 32
// cells along x (n_x must be a multiple of 32): with q = p + dx the strip is
// aligned in q, and the operands are transposed into LDS as
//   gt[dx][n][q] = g[q - dx][n] (three shifted copies), xt[row][c][q] = x[q, row][c]
// for the 9 (dy, dz) rows. Wave w accumulates the rows r = w, w+4, w+8.
// Each workgroup writes its partial sums; k_wgrad_reduce adds them in order.
template <int CIN, int COUTP>
__global__ __launch_bounds__(kBlock) void k_wgrad(Grid g, int64_t ncells, const u16* __restrict__ gin,
                                                    const u16* __restrict__ xin, float* __restrict__ partial) {
    constexpr int MT = COUTP == 32 ? 2 : 1;  // tiles of output channels n
    constexpr int NT = CIN == 32 ? 2 : 1;    // tiles of input channels c
    constexpr int GC = COUTP;                // channels stored per cell in gin
    __shared__ __attribute__((aligned(16))) u16 gt[3][MT * 16][32];
    __shared__ __attribute__((aligned(16))) u16 xt[9][NT * 16][32];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int lm = lane & 15, gq = lane >> 4;
    constexpr int NR = 3;  // rows per wave (the ninth row belongs to wave 0)
    f32x4 acc[NR][3][MT][NT];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[r][d][mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bacc = 0.f;  // bias partial for channel tid (tid < COUTP)
    // padding rows (output channels >= COUTP, input channels >= CIN) stay zero
    if constexpr (MT * 16 > COUTP) {
        constexpr int PN = MT * 16 - COUTP;
        for (int e = tid; e < 3 * PN * 32; e += kBlock) gt[e / (PN * 32)][COUTP + (e / 32) % PN][e % 32] = 0;
    }
    if constexpr (NT * 16 > CIN) {
        constexpr int PC = NT * 16 - CIN;
        for (int e = tid; e < 9 * PC * 32; e += kBlock) xt[e / (PC * 32)][CIN + (e / 32) % PC][e % 32] = 0;
    }
    const int64_t nstrip = ncells / 32;
    for (int64_t s = blockIdx.x; s < nstrip; s += gridDim.x) {
        const int q0 = int(s) * 32;
        const RowPos rp = row_of(g, q0);
        __syncthreads();
        // gt[d][n][q] = g[q - dx][n], dx = d - 1: 8 channels per 16-byte load
        constexpr int G8 = COUTP / 8;
        const int rs0 = row_start(g, rp, 0, 0);
        for (int e = tid; e < 3 * 32 * G8; e += kBlock) {
            const int j8 = e % G8, q = (e / G8) % 32, d = e / (32 * G8);
            const int p = rs0 + wrapi(rp.x0 + q - (d - 1), g.nx);
            const uint4 v = *reinterpret_cast<const uint4*>(gin + int64_t(p) * GC + 8 * j8);
            const unsigned w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int i = 0; i < 8; ++i) gt[d][8 * j8 + i][q] = u16((w4[i >> 1] >> ((i & 1) * 16)) & 0xffffu);
        }
        // xt[row][c][q] = x[q + (0, dy, dz)][c]
        constexpr int C8 = CIN / 8;
        for (int e = tid; e < 9 * 32 * C8; e += kBlock) {
            const int c8 = e % C8, q = (e / C8) % 32, row = e / (32 * C8);
            const int p = row_start(g, rp, row % 3 - 1, row / 3 - 1) + rp.x0 + q;
            const uint4 v = *reinterpret_cast<const uint4*>(xin + int64_t(p) * CIN + 8 * c8);
            const unsigned w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int i = 0; i < 8; ++i) xt[row][8 * c8 + i][q] = u16((w4[i >> 1] >> ((i & 1) * 16)) & 0xffffu);
        }
        __syncthreads();
        if (tid < COUTP) {
            for (int q = 0; q < 32; ++q) bacc += bf16_val(gt[1][tid][q]);
        }
        bf16x8 av[3][MT];
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) av[d][mt] = *reinterpret_cast<const bf16x8*>(&gt[d][mt * 16 + lm][8 * gq]);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int row = wave + 4 * r;
            if (row >= 9) continue;
            bf16x8 bv[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) bv[nt] = *reinterpret_cast<const bf16x8*>(&xt[row][nt * 16 + lm][8 * gq]);
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        acc[r][d][mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[d][mt], bv[nt], acc[r][d][mt][nt], 0, 0, 0);
        }
    }
    // partial layout per workgroup: [n (COUTP)][tap][c (CIN)] then bias [COUTP]
    float* out = partial + int64_t(blockIdx.x) * (COUTP * kTaps * CIN + COUTP);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int row = wave + 4 * r;
        if (row >= 9) continue;
        const int dy = row % 3, dz = row / 3;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int tap = dz * 9 + dy * 3 + d;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int n = mt * 16 + 4 * gq + i, c = nt * 16 + lm;
                        if (n < COUTP && c < CIN) out[(n * kTaps + tap) * CIN + c] = acc[r][d][mt][nt][i];
                    }
        }
    }
    if (tid < COUTP) out[COUTP * kTaps * CIN + tid] = bacc;
}

// theta_bar += sum over workgroups of the partials, in workgroup order (deterministic).
// Partial layout [n < coutp][tap][c < cinp] then bias [coutp]; only the real
// channels (n < cout, c < cin) map to W[o = n][i = c][tap] and b[o].
__global__ void k_wgrad_reduce(const float* __restrict__ partial, int nwg, int cinp, int coutp, int cin, int cout,
                               float* __restrict__ wbar, float* __restrict__ bbar) {
    const int per = coutp * kTaps * cinp + coutp;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= per) return;
    double s = 0.0;
    for (int w = 0; w < nwg; ++w) s += partial[int64_t(w) * per + e];
    if (e < coutp * kTaps * cinp) {
        const int c = e % cinp, tap = (e / cinp) % kTaps, n = e / (cinp * kTaps);
        if (n < cout && c < cin) wbar[(n * cin + c) * kTaps + tap] += float(s);
    } else {
        const int n = e - coutp * kTaps * cinp;
        if (n < cout) bbar[n] += float(s);
    }
}

// ----------------------------------------------------------------------------
// Launchers
// ----------------------------------------------------------------------------
int conv_grid(int64_t ncells) {
    const int64_t nseg = (ncells + 127) / 128;
    return int(nseg < 2048 ? nseg : 2048);
}

template <typename T>
hipError_t launch_closure_pack_input(const Grid& g, const T* u, u16* x0, hipStream_t s) {
    const int64_t vol = int64_t(g.nx) * g.ny * g.nz, n = vol * g.batch;
    hipLaunchKernelGGL(k_pack_input<T>, dim3(int((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, n, vol, u, x0);
    return hipGetLastError();
}

hipError_t launch_closure_pack_weights(const float* w, int cin, int cout, int cinp, int ntf, u16* wf, int coutp, int ntd,
                                       u16* wd, hipStream_t s) {
    const int tot = ((kTaps * cinp + 31) / 32) * ntf * 512 + ((kTaps * coutp + 31) / 32) * ntd * 512;
    hipLaunchKernelGGL(k_pack_weights, dim3((tot + 255) / 256), dim3(256), 0, s, w, cin, cout, cinp, ntf, wf, coutp, ntd, wd);
    return hipGetLastError();
}

// layer: 0 = 8 -> 32 hidden, 1 = 32 -> 32 hidden, 2 = 32 -> 3 output;
// dgrad: 10 = 8 -> 32 (cotangent of m into the last hidden layer), 11 = 32 -> 32,
// 12 = 32 -> 3 input gradient.
template <typename T>
hipError_t launch_closure_conv(const Grid& g, int which, const u16* in, const u16* wpk, const float* bias,
                               const float* zin, float* zout, u16* aout, T* fout, hipStream_t s) {
    const int64_t n = int64_t(g.nx) * g.ny * g.nz * g.batch;
    const int grid = conv_grid(n);
    auto shm = [](int cin, int nt) { return size_t((kTaps * cin + 31) / 32) * nt * 16 * 32 * 2; };
    switch (which) {
        case 0:
            hipLaunchKernelGGL((k_conv<T, 8, 2, EPI_HIDDEN>), dim3(grid), dim3(kBlock), shm(8, 2), s, g, n, in, wpk, bias,
                               zin, zout, aout, fout, 32);
            break;
        case 1:
            hipLaunchKernelGGL((k_conv<T, 32, 2, EPI_HIDDEN>), dim3(grid), dim3(kBlock), shm(32, 2), s, g, n, in, wpk,
                               bias, zin, zout, aout, fout, 32);
            break;
        case 2:
            hipLaunchKernelGGL((k_conv<T, 32, 1, EPI_OUT>), dim3(grid), dim3(kBlock), shm(32, 1), s, g, n, in, wpk, bias,
                               zin, zout, aout, fout, 3);
            break;
        case 10:
            hipLaunchKernelGGL((k_conv<T, 8, 2, EPI_DGRAD_HIDDEN>), dim3(grid), dim3(kBlock), shm(8, 2), s, g, n, in, wpk,
                               bias, zin, zout, aout, fout, 32);
            break;
        case 11:
            hipLaunchKernelGGL((k_conv<T, 32, 2, EPI_DGRAD_HIDDEN>), dim3(grid), dim3(kBlock), shm(32, 2), s, g, n, in,
                               wpk, bias, zin, zout, aout, fout, 32);
            break;
        default:
            hipLaunchKernelGGL((k_conv<T, 32, 1, EPI_DGRAD_INPUT>), dim3(grid), dim3(kBlock), shm(32, 1), s, g, n, in,
                               wpk, bias, zin, zout, aout, fout, 3);
            break;
    }
    return hipGetLastError();
}

int wgrad_grid(int64_t ncells) {
    const int64_t nstrip = ncells / 32;
    return int(nstrip < 512 ? nstrip : 512);
}

// which: 0 = layer 1 (g: 32 ch, x: 8 packed ch of which 3 real), 1 = layer 2 (32, 32),
// 2 = layer 3 (g: 8 packed ch of which 3 real, x: 32 ch). wbar/bbar point at the
// layer's weights and bias inside the flat parameter gradient.
hipError_t launch_closure_wgrad(const Grid& g, int which, const u16* gin, const u16* xin, float* partial, float* wbar,
                                float* bbar, hipStream_t s) {
    const int64_t n = int64_t(g.nx) * g.ny * g.nz * g.batch;
    const int grid = wgrad_grid(n);
    int cinp, coutp, cin, cout;
    if (which == 0) {
        hipLaunchKernelGGL((k_wgrad<8, 32>), dim3(grid), dim3(kBlock), 0, s, g, n, gin, xin, partial);
        cinp = 8, coutp = 32, cin = 3, cout = 32;
    } else if (which == 1) {
        hipLaunchKernelGGL((k_wgrad<32, 32>), dim3(grid), dim3(kBlock), 0, s, g, n, gin, xin, partial);
        cinp = 32, coutp = 32, cin = 32, cout = 32;
    } else {
        hipLaunchKernelGGL((k_wgrad<32, 8>), dim3(grid), dim3(kBlock), 0, s, g, n, gin, xin, partial);
        cinp = 32, coutp = 8, cin = 32, cout = 3;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int per = coutp * kTaps * cinp + coutp;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((per + 255) / 256), dim3(256), 0, s, partial, grid, cinp, coutp, cin, cout,
                       wbar, bbar);
    return hipGetLastError();
}

// Partial-sum floats needed by launch_closure_wgrad for a grid of n cells.
size_t closure_wgrad_partial_floats(int64_t ncells) {
    return size_t(wgrad_grid(ncells)) * (32 * kTaps * 32 + 32);
}

template hipError_t launch_closure_pack_input<double>(const Grid&, const double*, u16*, hipStream_t);
template hipError_t launch_closure_pack_input<float>(const Grid&, const float*, u16*, hipStream_t);
template hipError_t launch_closure_conv<double>(const Grid&, int, const u16*, const u16*, const float*, const float*,
                                                float*, u16*, double*, hipStream_t);
template hipError_t launch_closure_conv<float>(const Grid&, int, const u16*, const u16*, const float*, const float*,
                                               float*, u16*, float*, hipStream_t);

}  // namespace ins
