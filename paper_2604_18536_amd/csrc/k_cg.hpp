// Conjugate-gradient building blocks shared by the channel and the
// stretched-grid solvers: work split, fixed-order partial sums, stop test.
#pragma once

#include "k_common.hpp"

namespace ins {

// ----------------------------------------------------------------------------
// Conjugate gradients
//
// Work split: the tiles of each field (64 x 4 cells) are dealt in contiguous
// runs to cg_blocks(g) workgroups per field (the 3D apply kernel uses 64 x 8
// tile columns and z-chunks instead, the same count); the workgroup with
// logical id b * nblk + blk serves field b. Every partial sum goes to a buffer
// of nblk doubles per field; a kernel that needs the total reduces that
// field's nblk partials in every workgroup, in one fixed order, so all
// workgroups agree bitwise. No atomics, fences or inter-workgroup waits: each
// kernel only reads sums its predecessors finished writing.
// ----------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over a workgroup of NT threads, returned to every thread (fixed order).
template <int NT = kBlock>
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += sh[i];
    __syncthreads();
    return s;
}

__host__ __device__ inline int cg_tiles_of(const Grid& g) {
    return ((g.nx + kTileX - 1) / kTileX) * ((g.ny + kTileY - 1) / kTileY) * g.nz;
}

// 3D apply kernel: 64 x kCgTy tile columns, each split into z-chunks.
constexpr int kCgTy = 8;
constexpr int kCgThreads3 = kTileX * kCgTy;

__host__ __device__ inline int cg_cols3(const Grid& g) {
    return ((g.nx + kTileX - 1) / kTileX) * ((g.ny + kCgTy - 1) / kCgTy);
}

__host__ __device__ inline int cg_zchunks(const Grid& g) {
    int n = kCgMaxBlocks / cg_cols3(g);
    if (n < 1) n = 1;
    return n < g.nz ? n : g.nz;
}

// Workgroups per field, the same for every CG kernel (their partial sums are
// reduced by the next kernel): tile columns x z-chunks in 3D, tiles (at most
// kCgMaxBlocks) in 2D. Never more than the 64 x 4 tiles of a field.
__host__ __device__ inline int cg_blocks_of(const Grid& g) {
    if (g.dim == 3) return cg_cols3(g) * cg_zchunks(g);
    const int t = cg_tiles_of(g);
    return t < kCgMaxBlocks ? t : kCgMaxBlocks;
}

struct CgSplit {
    int b, blk, nblk;  // field, workgroup within the field, workgroups per field
    int t0, t1;        // tiles [t0, t1) of the field
    __device__ int64_t slot() const { return int64_t(b) * nblk + blk; }
};

__device__ __forceinline__ CgSplit cg_split(const Grid& g) {
    const int tiles = cg_tiles_of(g);
    CgSplit c;
    c.nblk = cg_blocks_of(g);
    const int id = xcd_logical(blockIdx.x, gridDim.x);
    c.b = id / c.nblk;
    c.blk = id - c.b * c.nblk;
    c.t0 = int(int64_t(tiles) * c.blk / c.nblk);
    c.t1 = int(int64_t(tiles) * (c.blk + 1) / c.nblk);
    return c;
}

// This thread's cell of tile t; false outside the grid. Tiles are numbered
// with z fastest, so a workgroup's run of tiles walks a tile column along z.
__device__ __forceinline__ bool cg_cell(const Grid& g, int t, int& x, int& y, int& z) {
    const int ntx = (g.nx + kTileX - 1) / kTileX;
    z = t % g.nz;
    t /= g.nz;
    const int tx = t % ntx;
    const int ty = t / ntx;
    x = tx * kTileX + (threadIdx.x & (kTileX - 1));
    y = ty * kTileY + (threadIdx.x / kTileX);
    return x < g.nx && y < g.ny;
}

__device__ __forceinline__ int64_t cg_index(const Grid& g, int b, int x, int y, int z) {
    return int64_t(b) * g.ncell + (int64_t(z) * g.ny + y) * g.nx + x;
}

// Total of field b's partials, in every thread of an NT-thread workgroup.
template <int NT = kBlock>
__device__ __forceinline__ double field_total(const double* part, const CgSplit& c, double* sh) {
    double s = 0.0;
    for (int i = threadIdx.x; i < c.nblk; i += NT) s += part[int64_t(c.b) * c.nblk + i];
    return block_sum<NT>(s, sh);
}

// Stop test of iteration k (the oracle's loop condition, negated).
__device__ __forceinline__ bool cg_stopped(double rrk, double rr0, int k, double rtol2, int maxiter) {
    return !(rr0 > 0.0) || rrk <= rtol2 * rr0 || k >= maxiter;
}

// Search direction p = r + beta p_old at a cell (p = r when FIRST).
template <bool FIRST>
__device__ __forceinline__ double cg_dir(const double* rb, const double* pb, int64_t j, double beta) {
    if constexpr (FIRST) {
        return rb[j];
    } else {
        return rb[j] + beta * pb[j];
    }
}

// Step length of iteration k - 1 if its solution update is still pending
// (iteration k - 1 was performed: not stopped, p.q > 0), else 0. The update
// x += alpha_{k-1} p_{k-1} is folded into iteration k's apply kernel (which
// reads p_{k-1} anyway) or, once stopped, into the first stopped one.
__device__ __forceinline__ double cg_pending(double rrm, double pqm, double rr0, int k, double rtol2, int maxiter) {
    if (k == 0 || cg_stopped(rrm, rr0, k - 1, rtol2, maxiter) || !(pqm > 0.0)) return 0.0;
    return rrm / pqm;
}
}  // namespace ins
