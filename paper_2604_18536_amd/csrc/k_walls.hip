// Kernels of the channel grid: no-slip walls at both ends of y, x and z
// periodic (Sec. 2.1, boundary conditions through ghost volumes), and the
// matrix-free conjugate-gradient pressure solve (Sec. 2.5.1, iterative solver).
//
// Wall rules, applied where a stencil reads a neighbour:
//  * u^y on the face right of the last cell row (row N_y - 1) is the upper
//    wall and the face left of row 0 the lower one: both read as 0, and every
//    output writes 0 on the stored wall face;
//  * a tangential component one row beyond a wall is the ghost value minus
//    the first interior value (zero interpolant on the wall);
//  * the pressure gradient exists on interior y-faces only, so D G is the
//    Neumann Laplacian.
// The forward and pullback stencils are the periodic ones of k_common.hpp
// (rhs_cell, rhs_vjp_cell) fed through sources that apply these rules: with
// them the diffusion stays symmetric and every convective wall flux vanishes
// identically, so the gather-form pullback needs no extra terms.
//
// CG (fp64 throughout): A = -D G on each field of the batch, b = mean(r) - r,
// x_0 = 0. One iteration is two fused kernels:
//   k_cg_apply:  p = r + beta p_old (formed at the stencil points), q = A p,
//                partial sums of p.q
//   k_cg_update: alpha = rr / p.q; x += alpha p, r -= alpha q, partial sums of r.r
// Every scalar (rr, beta, alpha, the stop test) is recomputed from partial
// sums in every workgroup, so iterations run back to back without the host
// and results are bitwise reproducible. A stopped field skips the work of
// later iterations.
#include "k_common.hpp"

namespace ins {

// Per-thread flags of the rows y - 1 .. y + 2 seen from cell row y.
struct WallRows {
    int ghost[4];  // 1: the row lies beyond a wall and mirrors the first/last row
    int unk[4];    // 1: the y-face of that row is an unknown (0 <= row <= N_y - 2)
};

// Neighbour offsets with rows beyond the walls mirrored onto the first/last row.
template <int DIM>
__device__ __forceinline__ Nb make_wall_nb(const Grid& g, int x, int y, int z, WallRows& rows) {
    Nb nb;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        nb.xo[k] = wrap(x + k - 1, g.nx);
        const int r = y + k - 1;
        const int m = r < 0 ? 0 : (r >= g.ny ? g.ny - 1 : r);
        nb.yo[k] = m * g.nx;
        nb.zo[k] = (DIM == 3) ? wrap(z + k - 1, g.nz) * g.nx * g.ny : 0;
        rows.ghost[k] = (r < 0 || r >= g.ny) ? 1 : 0;
        rows.unk[k] = (r >= 0 && r <= g.ny - 2) ? 1 : 0;
    }
    return nb;
}

// Velocity (PROJ: w - G p, formed in float64) at a neighbour, wall rules applied.
template <typename T, bool PROJ>
struct WallVel {
    const T* __restrict__ w;
    const double* __restrict__ p;
    int ncell;
    double ih0, ih1, ih2;
    WallRows rows;
    __device__ __forceinline__ T operator()(int c, const Nb& nb, int dx, int dy, int dz) const {
        const int k = dy + 1;
        const int j = nb.at(dx, dy, dz);
        if (c == 1) {
            if (!rows.unk[k]) return T(0);
            if constexpr (!PROJ) {
                return w[ncell + j];
            } else {
                return T(double(w[ncell + j]) - (p[nb.at(dx, dy + 1, dz)] - p[j]) * ih1);
            }
        }
        T v;
        if constexpr (!PROJ) {
            v = w[c * ncell + j];
        } else {
            const int jp = nb.at(dx + (c == 0), dy, dz + (c == 2));
            v = T(double(w[c * ncell + j]) - (p[jp] - p[j]) * (c == 0 ? ih0 : ih2));
        }
        return rows.ghost[k] ? -v : v;
    }
};

// Stage cotangent Fbar = cb ybar + (HAS_W ? cw (un - G q) : 0) with the same rules
// (it is read through the transposed stencils, which are the same stencils).
template <typename T, bool HAS_W>
struct WallFbar {
    const T* __restrict__ ybar;
    const T* __restrict__ un;
    const double* __restrict__ q;
    T cb, cw;
    int ncell;
    double ih0, ih1, ih2;
    WallRows rows;
    __device__ __forceinline__ T operator()(int c, const Nb& nb, int dx, int dy, int dz) const {
        const int k = dy + 1;
        if (c == 1 && !rows.unk[k]) return T(0);
        const int j = nb.at(dx, dy, dz);
        T v = cb * ybar[c * ncell + j];
        if constexpr (HAS_W) {
            const int jp = nb.at(dx + (c == 0), dy + (c == 1), dz + (c == 2));
            const double ih = c == 0 ? ih0 : (c == 1 ? ih1 : ih2);
            v += cw * T(double(un[c * ncell + j]) - (q[jp] - q[j]) * ih);
        }
        return (c != 1 && rows.ghost[k]) ? -v : v;
    }
};

// ----------------------------------------------------------------------------
// Forward stencils
// ----------------------------------------------------------------------------

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_wall_rhs(Grid g, const T* __restrict__ u, T* __restrict__ f) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    WallRows rows;
    const Nb nb = make_wall_nb<DIM>(g, t.x, t.y, t.z, rows);
    const int64_t boff = int64_t(t.b) * DIM * g.ncell;
    WallVel<T, false> U{u + boff, nullptr, int(g.ncell), g.ih[0], g.ih[1], g.ih[2], rows};
    T F[DIM];
    rhs_cell<T, DIM>(g, U, nb, F);
    const int c0 = nb.at(0, 0, 0);
    const bool wall = t.y == g.ny - 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) f[boff + a * g.ncell + c0] = (a == 1 && wall) ? T(0) : F[a];
}

// Runge-Kutta stage (same contract as k_stage): u_i = (PROJ ? w - G p : w),
// F = F(u_i); (if y) y = (yinit ? u0 : y) + cy F; (if wout) wout = u0 + cw F.
template <typename T, int DIM, bool PROJ>
__global__ __launch_bounds__(kBlock) void k_wall_stage(Grid g, const T* __restrict__ w, const double* __restrict__ p,
                                                        const T* __restrict__ u0, T* __restrict__ y, int yinit, T cy,
                                                        T* __restrict__ wout, T cw) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    WallRows rows;
    const Nb nb = make_wall_nb<DIM>(g, t.x, t.y, t.z, rows);
    const int64_t boff = int64_t(t.b) * DIM * g.ncell;
    WallVel<T, PROJ> U{w + boff, PROJ ? p + int64_t(t.b) * g.ncell : nullptr, int(g.ncell), g.ih[0], g.ih[1], g.ih[2],
                       rows};
    T F[DIM];
    rhs_cell<T, DIM>(g, U, nb, F);
    const int c0 = nb.at(0, 0, 0);
    const bool wall = t.y == g.ny - 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int64_t k = boff + a * g.ncell + c0;
        if (a == 1 && wall) {
            if (y) y[k] = T(0);
            if (wout) wout[k] = T(0);
            continue;
        }
        const T base = (wout || yinit) ? u0[k] : T(0);
        if (y) y[k] = (yinit ? base : y[k]) + cy * F[a];
        if (wout) wout[k] = base + cw * F[a];
    }
}

// u_out = w - G p (float64 arithmetic); 0 on the wall face. u_out may alias w.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_wall_project(Grid g, const T* w, const double* __restrict__ p, T* u_out) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const double* pb = p + int64_t(t.b) * g.ncell;
    const int64_t boff = int64_t(t.b) * DIM * g.ncell;
    const int c0 = nb.at(0, 0, 0);
    const double pc = pb[c0];
    const bool wall = t.y == g.ny - 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int64_t k = boff + a * g.ncell + c0;
        if (a == 1 && wall) {
            u_out[k] = T(0);
            continue;
        }
        const int cp = nb.at(a == 0, a == 1, a == 2);
        u_out[k] = T(double(w[k]) - (pb[cp] - pc) * g.ih[a]);
    }
}

// G p on the interior faces, 0 on the wall face.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_wall_gradient(Grid g, const double* __restrict__ p, T* __restrict__ out) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const double* pb = p + int64_t(t.b) * g.ncell;
    T* ob = out + int64_t(t.b) * DIM * g.ncell;
    const int c0 = nb.at(0, 0, 0);
    const double pc = pb[c0];
    const bool wall = t.y == g.ny - 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int cp = nb.at(a == 0, a == 1, a == 2);
        ob[a * g.ncell + c0] = (a == 1 && wall) ? T(0) : T((pb[cp] - pc) * g.ih[a]);
    }
}

// D u at one cell with both wall faces of u^y read as 0.
template <typename T, int DIM>
__device__ __forceinline__ double wall_div_cell(const Grid& g, const T* ub, const Nb& nb, int y) {
    const int c0 = nb.at(0, 0, 0);
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double up = double(ub[a * g.ncell + c0]);
        double dn = double(ub[a * g.ncell + nb.at(-(a == 0), -(a == 1), -(a == 2))]);
        if (a == 1) {
            if (y == g.ny - 1) up = 0.0;
            if (y == 0) dn = 0.0;
        }
        acc += (up - dn) * g.ih[a];
    }
    return acc;
}

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_wall_divergence(Grid g, const T* __restrict__ u, double* __restrict__ r) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    r[int64_t(t.b) * g.ncell + nb.at(0, 0, 0)] = wall_div_cell<T, DIM>(g, u + int64_t(t.b) * DIM * g.ncell, nb, t.y);
}

// ----------------------------------------------------------------------------
// Pullbacks
// ----------------------------------------------------------------------------

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_wall_rhs_vjp(Grid g, const T* __restrict__ u, const T* __restrict__ fbar,
                                                          T* __restrict__ ubar) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    WallRows rows;
    const Nb nb = make_wall_nb<DIM>(g, t.x, t.y, t.z, rows);
    const int64_t boff = int64_t(t.b) * DIM * g.ncell;
    const int nc = int(g.ncell);
    WallVel<T, false> U{u + boff, nullptr, nc, g.ih[0], g.ih[1], g.ih[2], rows};
    WallFbar<T, false> F{fbar + boff, nullptr, nullptr, T(1), T(0), nc, g.ih[0], g.ih[1], g.ih[2], rows};
    T out[DIM];
    rhs_vjp_cell<T, DIM>(g, U, F, nb, out);
    const int c0 = nb.at(0, 0, 0);
    const bool wall = t.y == g.ny - 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) ubar[boff + a * g.ncell + c0] = (a == 1 && wall) ? T(0) : out[a];
}

// Reverse stage (same contract as k_stage_vjp, without the closure output).
template <typename T, int DIM, bool PROJ_U, bool HAS_W>
__global__ __launch_bounds__(kBlock) void k_wall_stage_vjp(Grid g, const T* __restrict__ w, const double* __restrict__ p,
                                                            const T* __restrict__ ybar, const T* __restrict__ un,
                                                            const double* __restrict__ q, T cb, T cw,
                                                            T* __restrict__ u0bar, int mode, T* __restrict__ ubar_out) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    WallRows rows;
    const Nb nb = make_wall_nb<DIM>(g, t.x, t.y, t.z, rows);
    const int64_t boff = int64_t(t.b) * DIM * g.ncell;
    const int64_t soff = int64_t(t.b) * g.ncell;
    const int nc = int(g.ncell);
    WallVel<T, PROJ_U> U{w + boff, PROJ_U ? p + soff : nullptr, nc, g.ih[0], g.ih[1], g.ih[2], rows};
    WallFbar<T, HAS_W> F{ybar + boff, HAS_W ? un + boff : nullptr, HAS_W ? q + soff : nullptr, cb, cw, nc,
                         g.ih[0], g.ih[1], g.ih[2], rows};
    T out[DIM];
    rhs_vjp_cell<T, DIM>(g, U, F, nb, out);
    const int c0 = nb.at(0, 0, 0);
    const bool wall = t.y == g.ny - 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int64_t k = boff + a * g.ncell + c0;
        if (a == 1 && wall) {
            if (u0bar) u0bar[k] = T(0);
            if (ubar_out) ubar_out[k] = T(0);
            continue;
        }
        T acc = (mode == 0 || mode == 3) ? ybar[k] : u0bar[k];
        if constexpr (HAS_W) {
            const int cp = nb.at(a == 0, a == 1, a == 2);
            acc += T(double(un[k]) - (q[soff + cp] - q[soff + c0]) * g.ih[a]);
        }
        if (mode >= 2) acc += out[a];
        if (u0bar) u0bar[k] = acc;
        if (ubar_out) ubar_out[k] = out[a];
    }
}

// ubar^a[J] = (rbar[J] - rbar[J + e_a]) / h_a; 0 on the wall face.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_wall_div_vjp(Grid g, const double* __restrict__ rbar, T* __restrict__ ubar) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const double* rb = rbar + int64_t(t.b) * g.ncell;
    T* ob = ubar + int64_t(t.b) * DIM * g.ncell;
    const int c0 = nb.at(0, 0, 0);
    const double rc = rb[c0];
    const bool wall = t.y == g.ny - 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int cp = nb.at(a == 0, a == 1, a == 2);
        ob[a * g.ncell + c0] = (a == 1 && wall) ? T(0) : T((rc - rb[cp]) * g.ih[a]);
    }
}

// pbar[I] = sum_a (gbar^a[I - e_a] - gbar^a[I]) / h_a over the interior faces.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_wall_grad_vjp(Grid g, const T* __restrict__ gbar, double* __restrict__ pbar) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    pbar[int64_t(t.b) * g.ncell + nb.at(0, 0, 0)] =
        -wall_div_cell<T, DIM>(g, gbar + int64_t(t.b) * DIM * g.ncell, nb, t.y);
}

// ----------------------------------------------------------------------------
// Conjugate gradients
//
// Work split: the tiles of each field (64 x 4 cells, ordered as in tile_of)
// are dealt in contiguous runs to cg_blocks(g) workgroups per field; the
// workgroup with logical id b * nblk + blk serves field b. Every partial sum
// goes to a buffer of nblk doubles per field; a kernel that needs the total
// reduces that field's nblk partials in every workgroup, in one fixed order,
// so all workgroups agree bitwise. No atomics, fences or inter-workgroup
// waits: each kernel only reads sums its predecessors finished writing.
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

// r = D vel (vel != null, wall rules) or a copy of rin; partial sums of r.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_cg_div(Grid g, const T* __restrict__ vel, const double* __restrict__ rin,
                                                    double* __restrict__ r, double* __restrict__ msum) {
    __shared__ double sh[kBlock / 64];
    const CgSplit c = cg_split(g);
    double acc = 0.0;
    for (int t = c.t0; t < c.t1; ++t) {
        int x, y, z;
        if (!cg_cell(g, t, x, y, z)) continue;
        const Nb nb = make_nb<DIM>(g, x, y, z);
        const int64_t k = cg_index(g, c.b, x, y, z);
        const double v = vel ? wall_div_cell<T, DIM>(g, vel + int64_t(c.b) * DIM * g.ncell, nb, y) : rin[k];
        r[k] = v;
        acc += v;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) msum[c.slot()] = s;
}

// r = mean(r) - r, x = 0; partial sums of r.r (rr_0).
__global__ __launch_bounds__(kBlock) void k_cg_init(Grid g, double* __restrict__ r, double* __restrict__ x,
                                                     const double* __restrict__ msum, double* __restrict__ rb0,
                                                     CgScal* st) {
    __shared__ double sh[kBlock / 64];
    const CgSplit c = cg_split(g);
    const double mean = field_total(msum, c, sh) / double(g.ncell);
    double acc = 0.0;
    for (int t = c.t0; t < c.t1; ++t) {
        int cx, cy, cz;
        if (!cg_cell(g, t, cx, cy, cz)) continue;
        const int64_t k = cg_index(g, c.b, cx, cy, cz);
        const double v = mean - r[k];
        r[k] = v;
        x[k] = 0.0;
        acc += v * v;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        rb0[c.slot()] = s;
        if (c.blk == 0) {
            st[c.b].mean = mean;
            st[c.b].it = 0;
            st[c.b].done = 0;
        }
    }
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

// q = A p at one cell from p at the cell (pc), at z -/+ 1 (pm, pp; unused in
// 2D) and at the x/y neighbours read from r, p_old. Wall rule: no y-face
// beyond the first/last row.
template <bool FIRST, int DIM>
__device__ __forceinline__ double cg_ap(const Grid& g, const double* rb, const double* pb, double beta, int64_t c0,
                                        int x, int y, double pc, double pm, double pp) {
    const int xm = x == 0 ? g.nx - 1 : x - 1;
    const int xp = x == g.nx - 1 ? 0 : x + 1;
    const int64_t row = c0 - x;
    double ap = (2.0 * pc - cg_dir<FIRST>(rb, pb, row + xm, beta) - cg_dir<FIRST>(rb, pb, row + xp, beta)) * g.ih2[0];
    double sy = 0.0;
    if (y > 0) sy += pc - cg_dir<FIRST>(rb, pb, c0 - g.nx, beta);
    if (y < g.ny - 1) sy += pc - cg_dir<FIRST>(rb, pb, c0 + g.nx, beta);
    ap += sy * g.ih2[1];
    if constexpr (DIM == 3) ap += (2.0 * pc - pm - pp) * g.ih2[2];
    return ap;
}

// Iteration k. rr_k from rbk, rr_{k-1} from rbm (k > 0). Unless stopped:
// p = r + beta p_old with beta = rr_k / rr_{k-1} (p = r at k = 0), formed at
// every stencil point; q = A p = -D G p; partial sums of p.q. Workgroup 0 of
// each field publishes the stop flag (and rr_0 at k = 0). In 3D each thread
// walks its (x, y) along z keeping p at z - 1, z, z + 1 in registers.
template <bool FIRST, int DIM>
__device__ __forceinline__ double cg_apply_run(const Grid& g, const CgSplit& c, const double* rb, const double* pb,
                                               double* pout, double* q, double beta) {
    double acc = 0.0;
    const int64_t plane = int64_t(g.nx) * g.ny;
    double pm = 0.0, pc = 0.0, pp = 0.0;
    bool fresh = true;
    for (int t = c.t0; t < c.t1; ++t) {
        int x, y, z;
        const bool in = cg_cell(g, t, x, y, z);
        if (!in) continue;
        const int64_t c0 = (int64_t(z) * g.ny + y) * g.nx + x;
        if constexpr (DIM == 3) {
            if (fresh || z == 0) {
                const int zm = z == 0 ? g.nz - 1 : z - 1;
                pm = cg_dir<FIRST>(rb, pb, c0 + (zm - z) * plane, beta);
                pc = cg_dir<FIRST>(rb, pb, c0, beta);
            } else {
                pm = pc;
                pc = pp;
            }
            const int zp = z == g.nz - 1 ? 0 : z + 1;
            pp = cg_dir<FIRST>(rb, pb, c0 + (zp - z) * plane, beta);
            fresh = false;
        } else {
            pc = cg_dir<FIRST>(rb, pb, c0, beta);
        }
        const double ap = cg_ap<FIRST, DIM>(g, rb, pb, beta, c0, x, y, pc, pm, pp);
        pout[c0] = pc;
        q[c0] = ap;
        acc += pc * ap;
    }
    return acc;
}

// 2D: each workgroup takes a run of 64 x 4 tiles.
__global__ __launch_bounds__(kBlock) void k_cg_apply2(Grid g, const double* __restrict__ r,
                                                       const double* __restrict__ pin, double* __restrict__ pout,
                                                       double* __restrict__ q, const double* __restrict__ rbk,
                                                       const double* __restrict__ rbm, double* __restrict__ pqs,
                                                       CgScal* st, int k, double rtol2, int maxiter) {
    __shared__ double sh[kBlock / 64];
    const CgSplit c = cg_split(g);
    const double rrk = field_total(rbk, c, sh);
    const double rr0 = k == 0 ? rrk : st[c.b].rr0;
    const bool stop = cg_stopped(rrk, rr0, k, rtol2, maxiter);
    if (c.blk == 0 && threadIdx.x == 0) {
        if (k == 0) st[c.b].rr0 = rrk;
        st[c.b].done = stop ? 1 : 0;
    }
    if (stop) return;
    const int64_t soff = int64_t(c.b) * g.ncell;
    double acc;
    if (k == 0) {
        acc = cg_apply_run<true, 2>(g, c, r + soff, pin + soff, pout + soff, q + soff, 0.0);
    } else {
        const double beta = rrk / field_total(rbm, c, sh);
        acc = cg_apply_run<false, 2>(g, c, r + soff, pin + soff, pout + soff, q + soff, beta);
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) pqs[c.slot()] = s;
}

// 3D: a workgroup of 64 x 8 threads walks one tile column through its
// z-chunk. p at z - 1, z, z + 1 stays in registers; the x/y neighbours come
// from a two-plane LDS ring holding each plane of the tile with a one-cell
// x/y halo (filled by the first 144 threads). Lanes past n_x load the
// periodic image so the last column's +x neighbour is in place; rows past
// n_y and halo rows beyond a wall are never read (no y-face there).
template <bool FIRST>
__device__ __forceinline__ double cg_apply3_run(const Grid& g, const CgSplit& c, const double* __restrict__ r,
                                                const double* __restrict__ pin, double* __restrict__ pout,
                                                double* __restrict__ q, double beta,
                                                double (*pl)[kCgTy + 2][kTileX + 2]) {
    const int cols = cg_cols3(g);
    const int ntx = (g.nx + kTileX - 1) / kTileX;
    const int nzc = cg_zchunks(g);
    const int col = c.blk % cols, zc = c.blk / cols;
    const int z0 = int(int64_t(g.nz) * zc / nzc), z1 = int(int64_t(g.nz) * (zc + 1) / nzc);
    const int x0 = (col % ntx) * kTileX, y0 = (col / ntx) * kCgTy;
    const int lx = threadIdx.x & (kTileX - 1), ly = threadIdx.x / kTileX;
    const int xw = (x0 + lx) % g.nx;
    const int y = y0 + ly;
    const bool yin = y < g.ny;
    const bool valid = yin && x0 + lx < g.nx;
    const int64_t plane = int64_t(g.nx) * g.ny;
    // halo cell of this thread (threads < 144)
    int hx = 0, hy = 0, hrow = 0, hcol = 0;
    bool hal = false;
    const bool hthr = threadIdx.x < 2 * kCgTy + 2 * kTileX;
    if (threadIdx.x < 2 * kCgTy) {
        const int row = threadIdx.x >> 1, side = threadIdx.x & 1;
        hy = y0 + row;
        hrow = row + 1;
        hcol = side ? kTileX + 1 : 0;
        hx = side ? (x0 + kTileX) % g.nx : (x0 + g.nx - 1) % g.nx;
        hal = hy < g.ny;
    } else if (hthr) {
        const int i = threadIdx.x - 2 * kCgTy;
        const int side = i / kTileX, cx = i % kTileX;
        hy = side ? y0 + kCgTy : y0 - 1;
        hrow = side ? kCgTy + 1 : 0;
        hcol = cx + 1;
        hx = (x0 + cx) % g.nx;
        hal = hy >= 0 && hy < g.ny;
    }
    const int64_t own = int64_t(y) * g.nx + xw;
    const int64_t hal_off = int64_t(hy) * g.nx + hx;
    const int zm0 = z0 == 0 ? g.nz - 1 : z0 - 1;
    double pm = yin ? cg_dir<FIRST>(r, pin, int64_t(zm0) * plane + own, beta) : 0.0;
    double pc = yin ? cg_dir<FIRST>(r, pin, int64_t(z0) * plane + own, beta) : 0.0;
    pl[0][ly + 1][lx + 1] = pc;
    if (hthr) pl[0][hrow][hcol] = hal ? cg_dir<FIRST>(r, pin, int64_t(z0) * plane + hal_off, beta) : 0.0;
    __syncthreads();
    int cur = 0;
    double acc = 0.0;
    for (int z = z0; z < z1; ++z) {
        const int zp = z == g.nz - 1 ? 0 : z + 1;
        const double pp = yin ? cg_dir<FIRST>(r, pin, int64_t(zp) * plane + own, beta) : 0.0;
        const double hv = (hthr && hal) ? cg_dir<FIRST>(r, pin, int64_t(zp) * plane + hal_off, beta) : 0.0;
        if (valid) {
            double ap = (2.0 * pc - pl[cur][ly + 1][lx] - pl[cur][ly + 1][lx + 2]) * g.ih2[0];
            double sy = 0.0;
            if (y > 0) sy += pc - pl[cur][ly][lx + 1];
            if (y < g.ny - 1) sy += pc - pl[cur][ly + 2][lx + 1];
            ap += sy * g.ih2[1] + (2.0 * pc - pm - pp) * g.ih2[2];
            const int64_t c0 = int64_t(z) * plane + int64_t(y) * g.nx + x0 + lx;
            pout[c0] = pc;
            q[c0] = ap;
            acc += pc * ap;
        }
        const int nxt = cur ^ 1;
        pl[nxt][ly + 1][lx + 1] = pp;
        if (hthr) pl[nxt][hrow][hcol] = hv;
        __syncthreads();
        cur = nxt;
        pm = pc;
        pc = pp;
    }
    return acc;
}

__global__ __launch_bounds__(kCgThreads3) void k_cg_apply3(Grid g, const double* __restrict__ r,
                                                            const double* __restrict__ pin, double* __restrict__ pout,
                                                            double* __restrict__ q, const double* __restrict__ rbk,
                                                            const double* __restrict__ rbm, double* __restrict__ pqs,
                                                            CgScal* st, int k, double rtol2, int maxiter) {
    __shared__ double sh[kCgThreads3 / 64];
    __shared__ double pl[2][kCgTy + 2][kTileX + 2];
    CgSplit c;
    c.nblk = cg_blocks_of(g);
    const int id = xcd_logical(blockIdx.x, gridDim.x);
    c.b = id / c.nblk;
    c.blk = id - c.b * c.nblk;
    c.t0 = c.t1 = 0;
    const double rrk = field_total<kCgThreads3>(rbk, c, sh);
    const double rr0 = k == 0 ? rrk : st[c.b].rr0;
    const bool stop = cg_stopped(rrk, rr0, k, rtol2, maxiter);
    if (c.blk == 0 && threadIdx.x == 0) {
        if (k == 0) st[c.b].rr0 = rrk;
        st[c.b].done = stop ? 1 : 0;
    }
    if (stop) return;
    const int64_t soff = int64_t(c.b) * g.ncell;
    double acc;
    if (k == 0) {
        acc = cg_apply3_run<true>(g, c, r + soff, pin + soff, pout + soff, q + soff, 0.0, pl);
    } else {
        const double beta = rrk / field_total<kCgThreads3>(rbm, c, sh);
        acc = cg_apply3_run<false>(g, c, r + soff, pin + soff, pout + soff, q + soff, beta, pl);
    }
    const double s = block_sum<kCgThreads3>(acc, sh);
    if (threadIdx.x == 0) pqs[c.slot()] = s;
}

// Iteration k, unless stopped: alpha = rr_k / p.q, x += alpha p, r -= alpha q,
// partial sums of r.r (rr_{k+1}) into rbn; a stopped field copies its rr_k
// partials forward instead, so the newest buffer always holds the final sum.
// Pointwise: the workgroups of a field sweep it together (grid stride), two
// cells per thread and access when the field size is even.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_cg_update(Grid g, double* __restrict__ x, const double* __restrict__ p,
                                                       double* __restrict__ r, const double* __restrict__ q,
                                                       const double* __restrict__ rbk, const double* __restrict__ pqs,
                                                       double* __restrict__ rbn, CgScal* st, int k, double rtol2,
                                                       int maxiter) {
    __shared__ double sh[kBlock / 64];
    const CgSplit c = cg_split(g);
    const double rrk = field_total(rbk, c, sh);
    if (cg_stopped(rrk, st[c.b].rr0, k, rtol2, maxiter)) {
        if (threadIdx.x == 0) rbn[c.slot()] = rbk[c.slot()];
        return;
    }
    const double pq = field_total(pqs, c, sh);
    const double alpha = pq > 0.0 ? rrk / pq : 0.0;
    const int64_t base = int64_t(c.b) * g.ncell;
    double acc = 0.0;
    if ((g.ncell & 1) == 0) {
        const int64_t npair = g.ncell / 2;
        double2* x2 = reinterpret_cast<double2*>(x + base);
        const double2* p2 = reinterpret_cast<const double2*>(p + base);
        double2* r2 = reinterpret_cast<double2*>(r + base);
        const double2* q2 = reinterpret_cast<const double2*>(q + base);
        const int64_t stride = int64_t(c.nblk) * kBlock;
        for (int64_t i = int64_t(c.blk) * kBlock + threadIdx.x; i < npair; i += stride) {
            const double2 pv = p2[i], qv = q2[i];
            double2 xv = x2[i], rv = r2[i];
            xv.x += alpha * pv.x;
            xv.y += alpha * pv.y;
            rv.x -= alpha * qv.x;
            rv.y -= alpha * qv.y;
            x2[i] = xv;
            r2[i] = rv;
            acc += rv.x * rv.x + rv.y * rv.y;
        }
    } else {
        const int64_t stride = int64_t(c.nblk) * kBlock;
        for (int64_t j = int64_t(c.blk) * kBlock + threadIdx.x; j < g.ncell; j += stride) {
            const int64_t i = base + j;
            x[i] += alpha * p[i];
            const double v = r[i] - alpha * q[i];
            r[i] = v;
            acc += v * v;
        }
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        rbn[c.slot()] = s;
        if (c.blk == 0) st[c.b].it = k + 1;
    }
}

// Final residual of a solve from the newest rr partials: rr, relres.
__global__ __launch_bounds__(kBlock) void k_cg_finish(Grid g, const double* __restrict__ rb, CgScal* st) {
    __shared__ double sh[kBlock / 64];
    CgSplit c;
    c.nblk = cg_blocks_of(g);
    c.b = blockIdx.x;
    const double rr = field_total(rb, c, sh);
    if (threadIdx.x == 0) {
        const double rr0 = st[c.b].rr0;
        st[c.b].rr = rr;
        st[c.b].relres = rr0 > 0.0 ? sqrt(rr / rr0) : 0.0;
    }
}

// ----------------------------------------------------------------------------
// Launchers
// ----------------------------------------------------------------------------
#define INS_WALL_DIM(g, KER, ...)                                                             \
    do {                                                                                      \
        const int nblk = stencil_blocks(g);                                                   \
        if ((g).dim == 3)                                                                     \
            hipLaunchKernelGGL((KER<T, 3>), dim3(nblk), dim3(kBlock), 0, s, __VA_ARGS__);     \
        else                                                                                  \
            hipLaunchKernelGGL((KER<T, 2>), dim3(nblk), dim3(kBlock), 0, s, __VA_ARGS__);     \
    } while (0)

template <typename T>
hipError_t launch_wall_rhs(const Grid& g, const T* u, T* f, hipStream_t s) {
    INS_WALL_DIM(g, k_wall_rhs, g, u, f);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_wall_divergence(const Grid& g, const T* u, double* r, hipStream_t s) {
    INS_WALL_DIM(g, k_wall_divergence, g, u, r);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_wall_gradient(const Grid& g, const double* p, T* out, hipStream_t s) {
    INS_WALL_DIM(g, k_wall_gradient, g, p, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_wall_project(const Grid& g, const T* w, const double* p, T* u_out, hipStream_t s) {
    INS_WALL_DIM(g, k_wall_project, g, w, p, u_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_wall_rhs_vjp(const Grid& g, const T* u, const T* fbar, T* ubar, hipStream_t s) {
    INS_WALL_DIM(g, k_wall_rhs_vjp, g, u, fbar, ubar);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_wall_div_vjp(const Grid& g, const double* rbar, T* ubar, hipStream_t s) {
    INS_WALL_DIM(g, k_wall_div_vjp, g, rbar, ubar);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_wall_grad_vjp(const Grid& g, const T* gbar, double* pbar, hipStream_t s) {
    INS_WALL_DIM(g, k_wall_grad_vjp, g, gbar, pbar);
    return hipGetLastError();
}

template <typename T, int DIM>
static void wall_stage_dim(const Grid& g, const T* w, const double* p, bool proj, const T* u0, T* y, int yi, T cy,
                           T* wout, T cw, hipStream_t s) {
    const int nblk = stencil_blocks(g);
    if (proj)
        hipLaunchKernelGGL((k_wall_stage<T, DIM, true>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, u0, y, yi, cy, wout, cw);
    else
        hipLaunchKernelGGL((k_wall_stage<T, DIM, false>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, u0, y, yi, cy, wout,
                           cw);
}

template <typename T>
hipError_t launch_wall_stage(const Grid& g, const T* w, const double* p, bool proj, const T* u0, T* y, bool yinit,
                             double cy, T* wout, double cw, hipStream_t s) {
    if (g.dim == 3)
        wall_stage_dim<T, 3>(g, w, p, proj, u0, y, yinit ? 1 : 0, T(cy), wout, T(cw), s);
    else
        wall_stage_dim<T, 2>(g, w, p, proj, u0, y, yinit ? 1 : 0, T(cy), wout, T(cw), s);
    return hipGetLastError();
}

template <typename T, int DIM>
static void wall_stage_vjp_dim(const Grid& g, const T* w, const double* p, bool proj_u, const T* ybar, const T* un,
                               const double* q, bool has_w, T cb, T cw, T* u0bar, int mode, T* ubar_out, hipStream_t s) {
    const int nblk = stencil_blocks(g);
    if (proj_u && has_w)
        hipLaunchKernelGGL((k_wall_stage_vjp<T, DIM, true, true>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, ybar, un, q,
                           cb, cw, u0bar, mode, ubar_out);
    else if (proj_u)
        hipLaunchKernelGGL((k_wall_stage_vjp<T, DIM, true, false>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, ybar, un, q,
                           cb, cw, u0bar, mode, ubar_out);
    else if (has_w)
        hipLaunchKernelGGL((k_wall_stage_vjp<T, DIM, false, true>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, ybar, un, q,
                           cb, cw, u0bar, mode, ubar_out);
    else
        hipLaunchKernelGGL((k_wall_stage_vjp<T, DIM, false, false>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, ybar, un,
                           q, cb, cw, u0bar, mode, ubar_out);
}

template <typename T>
hipError_t launch_wall_stage_vjp(const Grid& g, const T* w, const double* p, bool proj_u, const T* ybar, const T* un,
                                 const double* q, bool has_w, double cb, double cw, T* u0bar, int mode, T* ubar_out,
                                 hipStream_t s) {
    if (g.dim == 3)
        wall_stage_vjp_dim<T, 3>(g, w, p, proj_u, ybar, un, q, has_w, T(cb), T(cw), u0bar, mode, ubar_out, s);
    else
        wall_stage_vjp_dim<T, 2>(g, w, p, proj_u, ybar, un, q, has_w, T(cb), T(cw), u0bar, mode, ubar_out, s);
    return hipGetLastError();
}

int cg_blocks(const Grid& g) { return cg_blocks_of(g); }

template <typename T>
hipError_t launch_cg_div(const Grid& g, const T* vel, const double* rin, double* r, double* msum, hipStream_t s) {
    const int nblk = cg_blocks_of(g) * g.batch;
    if (g.dim == 3)
        hipLaunchKernelGGL((k_cg_div<T, 3>), dim3(nblk), dim3(kBlock), 0, s, g, vel, rin, r, msum);
    else
        hipLaunchKernelGGL((k_cg_div<T, 2>), dim3(nblk), dim3(kBlock), 0, s, g, vel, rin, r, msum);
    return hipGetLastError();
}

hipError_t launch_cg_init(const Grid& g, double* r, double* x, const double* msum, double* rb0, CgScal* st,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_cg_init, dim3(cg_blocks_of(g) * g.batch), dim3(kBlock), 0, s, g, r, x, msum, rb0, st);
    return hipGetLastError();
}

hipError_t launch_cg_apply(const Grid& g, const double* r, const double* pin, double* pout, double* q,
                           const double* rbk, const double* rbm, double* pqs, CgScal* st, int k, double rtol2,
                           int maxiter, hipStream_t s) {
    const int nblk = cg_blocks_of(g) * g.batch;
    if (g.dim == 3)
        hipLaunchKernelGGL(k_cg_apply3, dim3(nblk), dim3(kCgThreads3), 0, s, g, r, pin, pout, q, rbk, rbm, pqs, st, k,
                           rtol2, maxiter);
    else
        hipLaunchKernelGGL(k_cg_apply2, dim3(nblk), dim3(kBlock), 0, s, g, r, pin, pout, q, rbk, rbm, pqs, st, k,
                           rtol2, maxiter);
    return hipGetLastError();
}

hipError_t launch_cg_update(const Grid& g, double* x, const double* p, double* r, const double* q, const double* rbk,
                            const double* pqs, double* rbn, CgScal* st, int k, double rtol2, int maxiter,
                            hipStream_t s) {
    const int nblk = cg_blocks_of(g) * g.batch;
    if (g.dim == 3)
        hipLaunchKernelGGL((k_cg_update<3>), dim3(nblk), dim3(kBlock), 0, s, g, x, p, r, q, rbk, pqs, rbn, st, k,
                           rtol2, maxiter);
    else
        hipLaunchKernelGGL((k_cg_update<2>), dim3(nblk), dim3(kBlock), 0, s, g, x, p, r, q, rbk, pqs, rbn, st, k,
                           rtol2, maxiter);
    return hipGetLastError();
}

hipError_t launch_cg_finish(const Grid& g, const double* rb, CgScal* st, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_finish, dim3(g.batch), dim3(kBlock), 0, s, g, rb, st);
    return hipGetLastError();
}

#define INS_WALL_INSTANTIATE(T)                                                                                         \
    template hipError_t launch_wall_rhs<T>(const Grid&, const T*, T*, hipStream_t);                                     \
    template hipError_t launch_wall_divergence<T>(const Grid&, const T*, double*, hipStream_t);                         \
    template hipError_t launch_wall_gradient<T>(const Grid&, const double*, T*, hipStream_t);                           \
    template hipError_t launch_wall_project<T>(const Grid&, const T*, const double*, T*, hipStream_t);                  \
    template hipError_t launch_wall_rhs_vjp<T>(const Grid&, const T*, const T*, T*, hipStream_t);                       \
    template hipError_t launch_wall_div_vjp<T>(const Grid&, const double*, T*, hipStream_t);                            \
    template hipError_t launch_wall_grad_vjp<T>(const Grid&, const T*, double*, hipStream_t);                           \
    template hipError_t launch_wall_stage<T>(const Grid&, const T*, const double*, bool, const T*, T*, bool, double,    \
                                             T*, double, hipStream_t);                                                  \
    template hipError_t launch_wall_stage_vjp<T>(const Grid&, const T*, const double*, bool, const T*, const T*,        \
                                                 const double*, bool, double, double, T*, int, T*, hipStream_t);        \
    template hipError_t launch_cg_div<T>(const Grid&, const T*, const double*, double*, double*, hipStream_t);

INS_WALL_INSTANTIATE(double)
INS_WALL_INSTANTIATE(float)

}  // namespace ins
