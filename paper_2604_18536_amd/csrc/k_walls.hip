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
//                partial sums of p.q        -> alpha = rr / p.q
//   k_cg_update: x += alpha p, r -= alpha q, partial sums of r.r
//                                           -> beta, rr, convergence flag
// Each reduction is finished by the workgroup that completes last (fixed
// summation order, so results are bitwise reproducible); the scalars live in
// device memory, so iterations run back to back without the host. A field
// whose flag is set skips the work of later iterations.
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
// ----------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the workgroup, returned to every thread (fixed order).
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) s += sh[i];
    __syncthreads();
    return s;
}

// Stores this workgroup's partial sum; true in every thread of the workgroup
// that arrives last, after which all partials are visible to it.
__device__ __forceinline__ bool publish(double part, double* partials, int slot, unsigned int* counter, int nblocks) {
    __shared__ int last;
    if (threadIdx.x == 0) {
        partials[slot] = part;
        __threadfence();
        last = atomicAdd(counter, 1u) == unsigned(nblocks - 1) ? 1 : 0;
    }
    __syncthreads();
    const bool am = last != 0;
    if (am) __threadfence();
    return am;
}

// Sum of the partials of batch entry b (blocks b*per .. (b+1)*per - 1), every thread.
__device__ __forceinline__ double batch_total(const double* partials, int b, int per, double* sh) {
    double s = 0.0;
    for (int i = threadIdx.x; i < per; i += kBlock) s += partials[int64_t(b) * per + i];
    return block_sum(s, sh);
}

__device__ __forceinline__ int logical_block() { return xcd_logical(blockIdx.x, gridDim.x); }

__device__ __forceinline__ int blocks_per_field(const Grid& g) {
    return ((g.nx + kTileX - 1) / kTileX) * ((g.ny + kTileY - 1) / kTileY) * g.nz;
}

// r = D vel (vel != null, wall rules) or a copy of rin; mean of r per field.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_cg_div(Grid g, const T* __restrict__ vel, const double* __restrict__ rin,
                                                    double* __restrict__ r, double* partials, unsigned int* counter,
                                                    CgScal* st) {
    __shared__ double sh[kBlock / 64];
    const TileIdx t = tile_of(g);
    double v = 0.0;
    if (t.valid) {
        const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
        const int64_t k = int64_t(t.b) * g.ncell + nb.at(0, 0, 0);
        v = vel ? wall_div_cell<T, DIM>(g, vel + int64_t(t.b) * DIM * g.ncell, nb, t.y) : rin[k];
        r[k] = v;
    }
    const double part = block_sum(v, sh);
    if (!publish(part, partials, logical_block(), counter, gridDim.x)) return;
    const int per = blocks_per_field(g);
    for (int b = 0; b < g.batch; ++b) {
        const double s = batch_total(partials, b, per, sh);
        if (threadIdx.x == 0) st[b].mean = s / double(g.ncell);
    }
    if (threadIdx.x == 0) *counter = 0u;
}

// r = mean - r (the right-hand side of A x = b), x = 0, p_old = 0; rr0 = r.r.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_cg_init(Grid g, double* __restrict__ r, double* __restrict__ x,
                                                     double* __restrict__ p0, double* partials, unsigned int* counter,
                                                     CgScal* st, int maxiter) {
    __shared__ double sh[kBlock / 64];
    const TileIdx t = tile_of(g);
    double v2 = 0.0;
    if (t.valid) {
        const int64_t k = int64_t(t.b) * g.ncell + int64_t(t.z) * g.nx * g.ny + int64_t(t.y) * g.nx + t.x;
        const double v = st[t.b].mean - r[k];
        r[k] = v;
        x[k] = 0.0;
        p0[k] = 0.0;
        v2 = v * v;
    }
    const double part = block_sum(v2, sh);
    if (!publish(part, partials, logical_block(), counter, gridDim.x)) return;
    const int per = blocks_per_field(g);
    for (int b = 0; b < g.batch; ++b) {
        const double s = batch_total(partials, b, per, sh);
        if (threadIdx.x == 0) {
            st[b].rr = s;
            st[b].rr0 = s;
            st[b].beta = 0.0;
            st[b].it = 0;
            st[b].relres = s > 0.0 ? 1.0 : 0.0;
            st[b].done = (s > 0.0 && maxiter > 0) ? 0 : 1;
        }
    }
    if (threadIdx.x == 0) *counter = 0u;
}

// p = r + beta p_old, q = A p = -D G p, partial p.q; alpha = rr / p.q.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_cg_apply(Grid g, const double* __restrict__ r, const double* __restrict__ pin,
                                                      double* __restrict__ pout, double* __restrict__ q, double* partials,
                                                      unsigned int* counter, CgScal* st) {
    __shared__ double sh[kBlock / 64];
    const TileIdx t = tile_of(g);
    double pq = 0.0;
    if (t.valid && !st[t.b].done) {
        const double beta = st[t.b].beta;
        const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
        const int64_t soff = int64_t(t.b) * g.ncell;
        const double* rb = r + soff;
        const double* pb = pin + soff;
        const int c0 = nb.at(0, 0, 0);
        const double pc = rb[c0] + beta * pb[c0];
        double ap = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const bool up = a != 1 || t.y < g.ny - 1;
            const bool dn = a != 1 || t.y > 0;
            double s = 0.0;
            if (up) {
                const int j = nb.at(a == 0, a == 1, a == 2);
                s += pc - (rb[j] + beta * pb[j]);
            }
            if (dn) {
                const int j = nb.at(-(a == 0), -(a == 1), -(a == 2));
                s += pc - (rb[j] + beta * pb[j]);
            }
            ap += s * g.ih2[a];
        }
        pout[soff + c0] = pc;
        q[soff + c0] = ap;
        pq = pc * ap;
    }
    const double part = block_sum(pq, sh);
    if (!publish(part, partials, logical_block(), counter, gridDim.x)) return;
    const int per = blocks_per_field(g);
    for (int b = 0; b < g.batch; ++b) {
        const double s = batch_total(partials, b, per, sh);
        if (threadIdx.x == 0 && !st[b].done) {
            st[b].pq = s;
            if (s > 0.0) {
                st[b].alpha = st[b].rr / s;
            } else {
                st[b].alpha = 0.0;
                st[b].done = 1;
            }
        }
    }
    if (threadIdx.x == 0) *counter = 0u;
}

// x += alpha p, r -= alpha q, partial r.r; beta, rr, iteration count, flag.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_cg_update(Grid g, double* __restrict__ x, const double* __restrict__ p,
                                                       double* __restrict__ r, const double* __restrict__ q,
                                                       double* partials, unsigned int* counter, CgScal* st, double rtol2,
                                                       int maxiter) {
    __shared__ double sh[kBlock / 64];
    const TileIdx t = tile_of(g);
    double rr = 0.0;
    if (t.valid && !st[t.b].done) {
        const double alpha = st[t.b].alpha;
        const int64_t k = int64_t(t.b) * g.ncell + int64_t(t.z) * g.nx * g.ny + int64_t(t.y) * g.nx + t.x;
        x[k] += alpha * p[k];
        const double v = r[k] - alpha * q[k];
        r[k] = v;
        rr = v * v;
    }
    const double part = block_sum(rr, sh);
    if (!publish(part, partials, logical_block(), counter, gridDim.x)) return;
    const int per = blocks_per_field(g);
    for (int b = 0; b < g.batch; ++b) {
        const double s = batch_total(partials, b, per, sh);
        if (threadIdx.x == 0 && !st[b].done) {
            const int it = st[b].it + 1;
            st[b].it = it;
            st[b].beta = s / st[b].rr;
            st[b].rr = s;
            st[b].relres = sqrt(s / st[b].rr0);
            if (s <= rtol2 * st[b].rr0 || it >= maxiter) st[b].done = 1;
        }
    }
    if (threadIdx.x == 0) *counter = 0u;
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

template <typename T>
hipError_t launch_cg_div(const Grid& g, const T* vel, const double* rin, double* r, double* partials,
                         unsigned int* counter, CgScal* st, hipStream_t s) {
    INS_WALL_DIM(g, k_cg_div, g, vel, rin, r, partials, counter, st);
    return hipGetLastError();
}

#define INS_CG_DIM(g, KER, ...)                                                               \
    do {                                                                                      \
        const int nblk = stencil_blocks(g);                                                   \
        if ((g).dim == 3)                                                                     \
            hipLaunchKernelGGL((KER<3>), dim3(nblk), dim3(kBlock), 0, s, __VA_ARGS__);        \
        else                                                                                  \
            hipLaunchKernelGGL((KER<2>), dim3(nblk), dim3(kBlock), 0, s, __VA_ARGS__);        \
    } while (0)

hipError_t launch_cg_init(const Grid& g, double* r, double* x, double* p0, double* partials, unsigned int* counter,
                          CgScal* st, int maxiter, hipStream_t s) {
    INS_CG_DIM(g, k_cg_init, g, r, x, p0, partials, counter, st, maxiter);
    return hipGetLastError();
}

hipError_t launch_cg_apply(const Grid& g, const double* r, const double* pin, double* pout, double* q, double* partials,
                           unsigned int* counter, CgScal* st, hipStream_t s) {
    INS_CG_DIM(g, k_cg_apply, g, r, pin, pout, q, partials, counter, st);
    return hipGetLastError();
}

hipError_t launch_cg_update(const Grid& g, double* x, const double* p, double* r, const double* q, double* partials,
                            unsigned int* counter, CgScal* st, double rtol2, int maxiter, hipStream_t s) {
    INS_CG_DIM(g, k_cg_update, g, x, p, r, q, partials, counter, st, rtol2, maxiter);
    return hipGetLastError();
}

int stencil_block_count(const Grid& g) { return stencil_blocks(g); }

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
    template hipError_t launch_cg_div<T>(const Grid&, const T*, const double*, double*, double*, unsigned int*, CgScal*, \
                                         hipStream_t);

INS_WALL_INSTANTIATE(double)
INS_WALL_INSTANTIATE(float)

}  // namespace ins
