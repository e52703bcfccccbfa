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
// fetches its 8 bfloat16 operands with one 16-byte load. A workgroup stages
// its input block (with the periodic halo) in LDS once and reads all 27 taps'
// A operands from there; weights are packed per K tile ([kt][n][32]) and read
// from global memory, where they stay cache-resident. The input gradient
// (dgrad) is the same kernel with flipped taps and transposed weights; the
// weight gradient (wgrad) reduces over cells with operands transposed through
// LDS and per-workgroup partial sums.
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

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
__device__ __forceinline__ int pmod_i(int v, int n) {
    const int r = v % n;
    return r < 0 ? r + n : r;
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
//   EPI_HIDDEN      : z = acc + bias -> zout [cells][32] fp32 (unless null), a = bf16(gelu(z)) -> aout [cells][32]
//   EPI_OUT         : m[b][n][cell] = acc + bias (n < nout), field type T (planar velocity layout)
//   EPI_DGRAD_HIDDEN: zbar = acc * gelu'(zin[cell][n]) -> aout [cells][32] bf16
//   EPI_DGRAD_INPUT : ubar[b][n][cell] += acc (n < nout), field type T
// The input block is staged in LDS. A workgroup owns a
// 32 x 4 x BZ block of output cells (x, y, z); it copies the 34 x 6 x (BZ + 2)
// input block (periodic halo included) into LDS once, so the 27 taps read their
// A operands from LDS instead of re-fetching them from memory. B operands
// (packed weights) come from global memory (every wave of every workgroup reads
// the same few KB per tap; they stay cache-resident). Wave w computes the
// output row y = w of every z plane of the block (M tiles mt: plane mt / 2,
// x half mt % 2). With 32 input channels the K loop runs over the nine (ty, tx)
// tap columns and, inside, over the BZ + 2 halo planes: each A operand fetched
// from LDS serves every output plane it is a tap of (tz = hz - z), and each
// weight operand fetched for a tap column serves 2 BZ M tiles. Hidden
// layer outputs are staged through LDS so that every global store is a full
// 16-byte chunk of one cell. In LDS the input block is split by 8-channel
// chunk, xs[chunk][cell][8]: the 16 lanes of an operand fetch read 16
// consecutive 16-byte cells (no bank conflicts, every access 16-byte aligned).
constexpr int kCbX = 32, kCbY = 4, kCbZ = 2, kCbCells = kCbX * kCbY * kCbZ;
constexpr int kChX = kCbX + 2, kChY = kCbY + 2, kChZ = kCbZ + 2, kChCells = kChX * kChY * kChZ;

// Block row (y + 4 z) of M tile mt of wave w: row y = w of plane mt / 2.
__device__ __forceinline__ int conv_row(int wave, int mt) { return (mt >> 1) * kCbY + wave; }

// The convolution kernel's output block is 32 x 4 x BZ cells: BZ = 4 for the
// 32-channel inputs (every weight operand a wave fetches then feeds 8 MFMAs
// instead of 4), BZ = 2 for the 8-channel ones. Its epilogue stages 256 cells
// (two planes) at a time.
template <int BZ>
constexpr int conv_halo_cells() { return kChX * kChY * (BZ + 2); }

// keep_z false: a forward-only hidden layer stages only its bfloat16 output
// (the smaller footprint lets more workgroups share a CU).
template <int CIN, int BZ>
constexpr size_t conv_t_lds_bytes(bool keep_z = true) {
    const size_t halo = size_t(conv_halo_cells<BZ>()) * CIN * 2;
    const size_t epi = size_t(kCbCells) * 32 * (keep_z ? 4 + 2 : 2);  // float32 z (or zin) + bfloat16 out
    return halo > epi ? halo : epi;
}

template <typename T, int CIN, int NT, int EPI, int BZ>
__global__ __launch_bounds__(kBlock) void k_conv_t(Grid g, const u16* __restrict__ in, const u16* __restrict__ wpk,
                                                     const float* __restrict__ bias, const float* __restrict__ zin,
                                                     float* __restrict__ zout, u16* __restrict__ aout,
                                                     T* __restrict__ fout, int nout) {
    constexpr int NKT = (kTaps * CIN + 31) / 32;
    constexpr int MT = 2 * BZ;  // M tiles per wave: BZ planes x 2 halves of x
    constexpr int HZ = BZ + 2, HCELLS = conv_halo_cells<BZ>();
    constexpr int CH = CIN / 8;  // 16-byte chunks per cell
    extern __shared__ __attribute__((aligned(16))) u16 xs[];
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int nbx = nx / kCbX, nby = (ny + kCbY - 1) / kCbY, nbz = (nz + BZ - 1) / BZ;
    int L = xcd_logical(blockIdx.x, gridDim.x);
    const int bx = L % nbx;
    L /= nbx;
    const int by = L % nby;
    L /= nby;
    const int bz = L % nbz;
    const int b = L / nbz;
    const int x0 = bx * kCbX, y0 = by * kCbY, z0 = bz * BZ;
    const int tid = threadIdx.x;
    const int64_t bcell = int64_t(b) * nz * ny * nx;
    // 1. input block with periodic halo -> LDS
    for (int cell = tid; cell < HCELLS; cell += kBlock) {
        const int hx = cell % kChX, hy = (cell / kChX) % kChY, hz = cell / (kChX * kChY);
        const int gx = wrapi(x0 - 1 + hx, nx);
        const int gy = pmod_i(y0 - 1 + hy, ny), gz = pmod_i(z0 - 1 + hz, nz);
        const int64_t gc = bcell + (int64_t(gz) * ny + gy) * nx + gx;
        uint4 v[CH];
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) v[ch] = *reinterpret_cast<const uint4*>(in + gc * CIN + ch * 8);
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) *reinterpret_cast<uint4*>(xs + (ch * HCELLS + cell) * 8) = v[ch];
    }
    __syncthreads();
    // 2. implicit GEMM from LDS
    const int lane = tid & 63, wave = tid >> 6;
    const int lm = lane & 15, gq = lane >> 4;
    f32x4 acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    int hbase[MT];  // halo cell of (tap offset 0, 0, 0) for this lane's row of each M tile
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int r = conv_row(wave, mt);
        const int yy = r % kCbY, zz = r / kCbY;
        hbase[mt] = (zz * kChY + yy) * kChX + (mt & 1) * 16 + lm;
    }
    if constexpr (CIN == 32) {
        const u16* xq = xs + (gq * HCELLS) * 8;  // this lane's 8-channel chunk
        // the weight operands of tap column tyx (tz = 0, 1, 2), fetched one column ahead
        bf16x8 bn[3][NT];
        auto fetch_w = [&](int tyx) {
#pragma unroll
            for (int tz = 0; tz < 3; ++tz)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    bn[tz][nt] = *reinterpret_cast<const bf16x8*>(
                        wpk + (((tz * 9 + tyx) * NT * 16 + nt * 16 + lm) * 32 + 8 * gq));
        };
        fetch_w(0);
#pragma unroll
        for (int tyx = 0; tyx < 9; ++tyx) {
            const int ty = tyx / 3, tx = tyx % 3;
            bf16x8 bv[3][NT];
#pragma unroll
            for (int tz = 0; tz < 3; ++tz)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) bv[tz][nt] = bn[tz][nt];
            if (tyx < 8) fetch_w(tyx + 1);
            __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of this column's work
#pragma unroll
            for (int hz = 0; hz < HZ; ++hz) {
#pragma unroll
                for (int xh = 0; xh < 2; ++xh) {
                    // halo cell of source plane hz for output row (y = wave) and x half xh
                    const int cell = (hz * kChY + wave + ty) * kChX + xh * 16 + lm + tx;
                    const bf16x8 av = *reinterpret_cast<const bf16x8*>(xq + cell * 8);
#pragma unroll
                    for (int zz = 0; zz < BZ; ++zz) {
                        const int tz = hz - zz;
                        if (tz < 0 || tz > 2) continue;
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt)
                            acc[zz * 2 + xh][nt] =
                                __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[tz][nt], acc[zz * 2 + xh][nt], 0, 0, 0);
                    }
                }
            }
        }
    } else {
    // the weight operands of K tile kt, fetched one tile ahead
    bf16x8 bn[NT];
    auto fetch_w = [&](int kt) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            bn[nt] = *reinterpret_cast<const bf16x8*>(wpk + ((kt * NT * 16 + nt * 16 + lm) * 32 + 8 * gq));
    };
    fetch_w(0);
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt) {
        int tap, c0;
        ktile_tap<CIN>(kt, gq, tap, c0);
        const bool tap_ok = tap < kTaps;
        const int t = tap_ok ? tap : 0;
        const int toff = ((t / 9) * kChY + (t / 3) % 3) * kChX + t % 3;
        bf16x8 bv[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) bv[nt] = bn[nt];
        if (kt + 1 < NKT) fetch_w(kt + 1);
        __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of this tile's work
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            bf16x8 av;
            if (tap_ok) {
                av = *reinterpret_cast<const bf16x8*>(xs + ((c0 >> 3) * HCELLS + hbase[mt] + toff) * 8);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) av[j] = __bf16(0.0f);
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[nt], acc[mt][nt], 0, 0, 0);
        }
    }
    }
    // 3. epilogue: lane holds D[m = 4 gq + i][n = nt*16 + lm] of M tile mt, i.e. block
    // cell q = r * 32 + (mt & 1) * 16 + 4 gq + i with r = conv_row(wave, mt)
    auto block_cell = [&](int q, int64_t& c) -> bool {
        const int r = q >> 5, xx = q & 31;
        const int yy = y0 + r % kCbY, zz = z0 + r / kCbY;
        c = bcell + (int64_t(zz) * ny + yy) * nx + x0 + xx;
        return yy < ny && zz < nz;
    };
    if constexpr (EPI == EPI_HIDDEN || EPI == EPI_DGRAD_HIDDEN) {
        // per half of the block (planes 2h, 2h + 1: 256 cells, q = 256 h + local cell):
        // [256][32] float32 z (not kept by a forward-only EPI_HIDDEN call: zout null),
        // then [256][32] bfloat16
        const bool keep_z = EPI == EPI_DGRAD_HIDDEN || zout != nullptr;
        float* zt = reinterpret_cast<float*>(xs);
        u16* at = keep_z ? reinterpret_cast<u16*>(xs + kCbCells * 32 * 2) : xs;
#pragma unroll
        for (int h = 0; h < BZ / 2; ++h) {
            const int qh = h * kCbCells;
            __syncthreads();  // every wave is done reading the input block / the previous half
            if constexpr (EPI == EPI_DGRAD_HIDDEN) {
                for (int e = tid; e < kCbCells * 8; e += kBlock) {  // zin block, 16-byte chunks
                    const int q = e >> 3, ch = e & 7;
                    int64_t c;
                    float4 v = {0.f, 0.f, 0.f, 0.f};
                    if (block_cell(qh + q, c)) v = *reinterpret_cast<const float4*>(zin + c * 32 + ch * 4);
                    *reinterpret_cast<float4*>(zt + q * 32 + ch * 4) = v;
                }
                __syncthreads();
            }
#pragma unroll
            for (int mt = 4 * h; mt < 4 * h + 4; ++mt) {
                const int qb = conv_row(wave, mt) * 32 + (mt & 1) * 16 + 4 * gq - qh;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int q = qb + i;
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        const int n = nt * 16 + lm;
                        const float v = acc[mt][nt][i];
                        if constexpr (EPI == EPI_HIDDEN) {
                            const float z = v + bias[n];
                            if (keep_z) zt[q * 32 + n] = z;
                            at[q * 32 + n] = bf16_bits(gelu_f(z));
                        } else {
                            at[q * 32 + n] = bf16_bits(v * gelu_grad_f(zt[q * 32 + n]));
                        }
                    }
                }
            }
            __syncthreads();
            for (int e = tid; e < kCbCells * 4; e += kBlock) {  // bfloat16 out: 4 chunks per cell
                const int q = e >> 2, ch = e & 3;
                int64_t c;
                if (block_cell(qh + q, c))
                    *reinterpret_cast<uint4*>(aout + c * 32 + ch * 8) =
                        *reinterpret_cast<const uint4*>(at + q * 32 + ch * 8);
            }
            if (EPI == EPI_HIDDEN && zout) {
                for (int e = tid; e < kCbCells * 8; e += kBlock) {  // float32 z: 8 chunks per cell
                    const int q = e >> 3, ch = e & 7;
                    int64_t c;
                    if (block_cell(qh + q, c))
                        *reinterpret_cast<float4*>(zout + c * 32 + ch * 4) =
                            *reinterpret_cast<const float4*>(zt + q * 32 + ch * 4);
                }
            }
        }
    } else {
        const int64_t vol = int64_t(nx) * ny * nz;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int qb = conv_row(wave, mt) * 32 + (mt & 1) * 16 + 4 * gq;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int64_t c;
                if (!block_cell(qb + i, c)) continue;
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const int n = nt * 16 + lm;
                    if (n < nout) {
                        const int64_t r = c - int64_t(b) * vol;
                        T* dst = fout + (int64_t(b) * 3 + n) * vol + r;
                        const float v = acc[mt][nt][i];
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

// Weight gradient on the same 32 x 4 x 2 cell blocks as k_conv_t:
// W'[n][tap][c] = sum_p g[p][n] x[p + off(tap)][c], bias'[n] = sum_p g[p][n].
// A workgroup stages, transposed to channel-major in LDS, the cotangent g of
// its block (gT[n][p]) and the input x of the block's halo (xT[c][z][y][x]);
// the K dimension of each MFMA is 32 cells of one block row. Wave w owns the
// taps w, w + 4, ...; for each block row it loads its A operands (g) once and
// reuses them for all its taps. A tap's B operand starts dx cells into the
// halo row, i.e. 0, 2 or 4 bytes past a 16-byte boundary: two aligned reads
// and a byte-align select it. Cells outside the grid (partial blocks in y or
// z) stage g = 0. Workgroups loop over a contiguous range of blocks and write
// per-workgroup partial sums (reduced in order by k_wgrad_reduce).
constexpr int kStage = 4;                 // staging items whose loads a thread issues together
constexpr int kGtStride = kCbCells + 8;  // gT row: 256 cells + pad (conflict-free A reads)
constexpr int kXtRow = 40;               // xT halo row: 34 cells padded to 40
constexpr int kXtStride = kChZ * kChY * kXtRow + 8;

template <int CIN, int COUTP>
__global__ __launch_bounds__(kBlock) void k_wgrad_t(Grid g, const u16* __restrict__ gin, const u16* __restrict__ xin,
                                                      float* __restrict__ partial) {
    constexpr int MT = COUTP == 32 ? 2 : 1;  // tiles of output channels n
    constexpr int NT = CIN == 32 ? 2 : 1;    // tiles of input channels c
    constexpr int NTAP = 7;                  // taps per wave (27 over 4 waves)
    extern __shared__ __attribute__((aligned(16))) u16 ws[];
    u16* gT = ws;                                // [MT*16][kGtStride]
    u16* xT = ws + MT * 16 * kGtStride;          // [NT*16][kXtStride]
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int lm = lane & 15, gq = lane >> 4;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    // padding channels stay zero
    if constexpr (MT * 16 > COUTP)
        for (int e = tid; e < (MT * 16 - COUTP) * kGtStride; e += kBlock) gT[COUTP * kGtStride + e] = 0;
    if constexpr (NT * 16 > CIN)
        for (int e = tid; e < (NT * 16 - CIN) * kXtStride; e += kBlock) xT[CIN * kXtStride + e] = 0;
    f32x4 acc[NTAP][MT][NT];
#pragma unroll
    for (int j = 0; j < NTAP; ++j)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[j][mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bacc = 0.f;
    const int nbx = nx / kCbX, nby = (ny + kCbY - 1) / kCbY, nbz = (nz + kCbZ - 1) / kCbZ;
    const int nblocks = nbx * nby * nbz * g.batch;
    // each workgroup takes a contiguous range of blocks, z fastest: consecutive
    // blocks share two of their four halo planes, which are still in cache
    const int per = (nblocks + gridDim.x - 1) / gridDim.x;
    const int blk0 = blockIdx.x * per, blk1 = min(nblocks, blk0 + per);
    for (int blk = blk0; blk < blk1; ++blk) {
        int L = blk;
        const int bz = L % nbz;
        L /= nbz;
        const int bx = L % nbx;
        L /= nbx;
        const int by = L % nby;
        const int b = L / nby;
        const int x0 = bx * kCbX, y0 = by * kCbY, z0 = bz * kCbZ;
        const int64_t bcell = int64_t(b) * nz * ny * nx;
        __syncthreads();  // the previous block's operands are no longer read
        // g of the block, cell pairs along x: gT[n][q], q = row * 32 + x; the loads of
        // kStage items are issued before any is unpacked into LDS
        constexpr int G8 = COUTP / 8;
        constexpr int NG = (kCbCells / 2) * G8;
        for (int e0 = 0; e0 < NG; e0 += kStage * kBlock) {
            uint4 v0[kStage], v1[kStage];
#pragma unroll
            for (int k = 0; k < kStage; ++k) {
                const int e = e0 + k * kBlock + tid;
                const int ch = e % G8, pr = e / G8;
                const int q = 2 * pr, r = q >> 5, xx = q & 31;
                const int yy = y0 + r % kCbY, zz = z0 + r / kCbY;
                v0[k] = uint4{0u, 0u, 0u, 0u};
                v1[k] = uint4{0u, 0u, 0u, 0u};
                if (e < NG && yy < ny && zz < nz) {
                    const int64_t c = bcell + (int64_t(zz) * ny + yy) * nx + x0 + xx;
                    v0[k] = *reinterpret_cast<const uint4*>(gin + c * COUTP + ch * 8);
                    v1[k] = *reinterpret_cast<const uint4*>(gin + (c + 1) * COUTP + ch * 8);
                }
            }
#pragma unroll
            for (int k = 0; k < kStage; ++k) {
                const int e = e0 + k * kBlock + tid;
                if (e >= NG) continue;
                const int ch = e % G8, q = 2 * (e / G8);
                const unsigned a[4] = {v0[k].x, v0[k].y, v0[k].z, v0[k].w};
                const unsigned bb[4] = {v1[k].x, v1[k].y, v1[k].z, v1[k].w};
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const unsigned lo = (a[i >> 1] >> ((i & 1) * 16)) & 0xffffu;
                    const unsigned hi = (bb[i >> 1] >> ((i & 1) * 16)) & 0xffffu;
                    *reinterpret_cast<unsigned*>(gT + (ch * 8 + i) * kGtStride + q) = lo | (hi << 16);
                }
            }
        }
        // x of the halo block, cell pairs along x: xT[c][(hz * 6 + hy) * 40 + hx]
        constexpr int C8 = CIN / 8;
        constexpr int NPAIR = kChZ * kChY * (kChX / 2);
        constexpr int NX = NPAIR * C8;
        for (int e0 = 0; e0 < NX; e0 += kStage * kBlock) {
            uint4 v0[kStage], v1[kStage];
#pragma unroll
            for (int k = 0; k < kStage; ++k) {
                const int e = min(e0 + k * kBlock + tid, NX - 1);
                const int ch = e % C8, pr = e / C8;
                const int hx = 2 * (pr % (kChX / 2)), hrow = pr / (kChX / 2);
                const int hy = hrow % kChY, hz = hrow / kChY;
                const int gy = pmod_i(y0 - 1 + hy, ny), gz = pmod_i(z0 - 1 + hz, nz);
                const int64_t rowc = bcell + (int64_t(gz) * ny + gy) * nx;
                const int gx0 = wrapi(x0 - 1 + hx, nx), gx1 = wrapi(x0 + hx, nx);
                v0[k] = *reinterpret_cast<const uint4*>(xin + (rowc + gx0) * CIN + ch * 8);
                v1[k] = *reinterpret_cast<const uint4*>(xin + (rowc + gx1) * CIN + ch * 8);
            }
#pragma unroll
            for (int k = 0; k < kStage; ++k) {
                const int e = e0 + k * kBlock + tid;
                if (e >= NX) continue;
                const int ch = e % C8, pr = e / C8;
                const int hx = 2 * (pr % (kChX / 2)), hrow = pr / (kChX / 2);
                const unsigned a[4] = {v0[k].x, v0[k].y, v0[k].z, v0[k].w};
                const unsigned bb[4] = {v1[k].x, v1[k].y, v1[k].z, v1[k].w};
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const unsigned lo = (a[i >> 1] >> ((i & 1) * 16)) & 0xffffu;
                    const unsigned hi = (bb[i >> 1] >> ((i & 1) * 16)) & 0xffffu;
                    *reinterpret_cast<unsigned*>(xT + (ch * 8 + i) * kXtStride + hrow * kXtRow + hx) = lo | (hi << 16);
                }
            }
        }
        __syncthreads();
        // bias: thread (n = tid mod 32, part = tid / 32) sums cells part*32 .. +31 of channel n
        if ((tid & 31) < COUTP) {
            const u16* row = gT + (tid & 31) * kGtStride + (tid >> 5) * 32;
#pragma unroll
            for (int q = 0; q < 32; q += 8) {
                const uint4 v = *reinterpret_cast<const uint4*>(row + q);
                const unsigned w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int i = 0; i < 8; ++i) bacc += bf16_val(u16((w4[i >> 1] >> ((i & 1) * 16)) & 0xffffu));
            }
        }
#pragma unroll 1
        for (int r = 0; r < kCbY * kCbZ; ++r) {
            const int yy = r % kCbY, zz = r / kCbY;
            bf16x8 av[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                av[mt] = *reinterpret_cast<const bf16x8*>(gT + (mt * 16 + lm) * kGtStride + r * 32 + 8 * gq);
#pragma unroll
            for (int j = 0; j < NTAP; ++j) {
                const int tap = wave + 4 * j;
                if (tap >= kTaps) continue;
                const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
                const int off = ((zz + dz) * kChY + (yy + dy)) * kXtRow + 8 * gq;
                const unsigned bs = 2u * unsigned(dx & 1);  // byte shift within a dword
                const bool wsh = dx == 2;                    // whole-dword shift
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const u16* rowp = xT + (nt * 16 + lm) * kXtStride + off;
                    const uint4 c0 = *reinterpret_cast<const uint4*>(rowp);
                    const uint4 c1 = *reinterpret_cast<const uint4*>(rowp + 8);
                    const unsigned d[5] = {wsh ? c0.y : c0.x, wsh ? c0.z : c0.y, wsh ? c0.w : c0.z,
                                           wsh ? c1.x : c0.w, wsh ? c1.y : c1.x};
                    unsigned o[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) o[i] = __builtin_amdgcn_alignbyte(d[i + 1], d[i], bs);
                    const bf16x8 bv = __builtin_bit_cast(bf16x8, (uint4{o[0], o[1], o[2], o[3]}));
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
                        acc[j][mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[mt], bv, acc[j][mt][nt], 0, 0, 0);
                }
            }
        }
    }
    // partial layout per workgroup: [n (COUTP)][tap][c (CIN)] then bias [COUTP]
    float* out = partial + int64_t(blockIdx.x) * (COUTP * kTaps * CIN + COUTP);
#pragma unroll
    for (int j = 0; j < NTAP; ++j) {
        const int tap = wave + 4 * j;
        if (tap >= kTaps) continue;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int n = mt * 16 + 4 * gq + i, c = nt * 16 + lm;
                    if (n < COUTP && c < CIN) out[(n * kTaps + tap) * CIN + c] = acc[j][mt][nt][i];
                }
    }
    // the eight partial bias sums of each channel, added in part order
    __syncthreads();
    float* red = reinterpret_cast<float*>(ws);
    red[tid] = bacc;
    __syncthreads();
    if (tid < COUTP) {
        float sum = 0.f;
#pragma unroll
        for (int part = 0; part < kBlock / 32; ++part) sum += red[part * 32 + tid];
        out[COUTP * kTaps * CIN + tid] = sum;
    }
}

template <int CIN, int COUTP>
constexpr size_t wgrad_t_lds_bytes() {
    return (size_t((COUTP == 32 ? 2 : 1) * 16) * kGtStride + size_t((CIN == 32 ? 2 : 1) * 16) * kXtStride) * 2;
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
#define INS_CONV(CIN, NT, EPI, NOUT)                                                                                \
    do {                                                                                                            \
        constexpr int BZ = CIN == 32 && EPI == EPI_HIDDEN ? 4 : 2;                                                  \
        const int grid = (g.nx / kCbX) * ((g.ny + kCbY - 1) / kCbY) * ((g.nz + BZ - 1) / BZ) * g.batch;            \
        const size_t shm = conv_t_lds_bytes<CIN, BZ>(EPI != EPI_HIDDEN || zout != nullptr);                         \
        hipLaunchKernelGGL((k_conv_t<T, CIN, NT, EPI, BZ>), dim3(grid), dim3(kBlock), shm, s, g, in, wpk, bias, zin, \
                           zout, aout, fout, NOUT);                                                                 \
    } while (0)
    switch (which) {
        case 0: INS_CONV(8, 2, EPI_HIDDEN, 32); break;
        case 1: INS_CONV(32, 2, EPI_HIDDEN, 32); break;
        case 2: INS_CONV(32, 1, EPI_OUT, 3); break;
        case 10: INS_CONV(8, 2, EPI_DGRAD_HIDDEN, 32); break;
        case 11: INS_CONV(32, 2, EPI_DGRAD_HIDDEN, 32); break;
        default: INS_CONV(32, 1, EPI_DGRAD_INPUT, 3); break;
    }
#undef INS_CONV
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
    constexpr size_t shm0 = wgrad_t_lds_bytes<8, 32>(), shm1 = wgrad_t_lds_bytes<32, 32>(),
                     shm2 = wgrad_t_lds_bytes<32, 8>();
    if (which == 0) {
        hipLaunchKernelGGL((k_wgrad_t<8, 32>), dim3(grid), dim3(kBlock), shm0, s, g, gin, xin, partial);
        cinp = 8, coutp = 32, cin = 3, cout = 32;
    } else if (which == 1) {
        hipLaunchKernelGGL((k_wgrad_t<32, 32>), dim3(grid), dim3(kBlock), shm1, s, g, gin, xin, partial);
        cinp = 32, coutp = 32, cin = 32, cout = 32;
    } else {
        hipLaunchKernelGGL((k_wgrad_t<32, 8>), dim3(grid), dim3(kBlock), shm2, s, g, gin, xin, partial);
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
