// Reverse-mode stencils of the right-hand side (Sec. 3.4 pullback rule,
// App. B): ubar = J_C(u)^T fbar + nu Lap(fbar), alone and fused into the
// reverse RK4 stage.
//
// The convection pullback is written in gather form, so each thread owns its
// output and no atomics are needed (results are bitwise deterministic). From
// the forward flux F^{ab}[K] = a^{ab}[K] b^{ab}[K] with
// a^{ab} = (u^a[K] + u^a[K+e_b])/2, b^{ab} = (u^b[K] + u^b[K+e_a])/2, the
// cotangent of component g at J collects
//   ubar^g[J] = 1/2 sum_b ( H^{gb}[J] + H^{gb}[J - e_b] ),
//   H^{gb}[K] = (u^b[K] + u^b[K+e_g])/2 * ( (fbar^g[K+e_b] - fbar^g[K]) / h_b
//                                         + (fbar^b[K+e_g] - fbar^b[K]) / h_g ),
// i.e. the a-factor and b-factor cotangents of the two fluxes that contain
// u^g[J]. (The printed eight-term pullback of App. B places the primal factor
// of four of its terms one cell off; this form is derived from the forward
// kernel instead.)
#include "k_common.hpp"

namespace ins {

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_rhs_vjp(Grid g, const T* __restrict__ u, const T* __restrict__ fbar,
                                                      T* __restrict__ ubar) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const int64_t boff = int64_t(t.b) * DIM * g.ncell;
    VelSrc<T, false> U{u + boff, nullptr, int(g.ncell), g.ih[0], g.ih[1], g.ih[2]};
    VelSrc<T, false> F{fbar + boff, nullptr, int(g.ncell), g.ih[0], g.ih[1], g.ih[2]};
    T out[DIM];
    rhs_vjp_cell<T, DIM>(g, U, F, nb, out);
    const int c0 = nb.at(0, 0, 0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) ubar[boff + a * g.ncell + c0] = out[a];
}

// Cotangent of the stage right-hand side F_i, formed on the fly:
// Fbar_i = cb * ybar + cw * (ubar_next - G q_next), where ubar_next - G q_next is
// the projected cotangent of the next stage's unprojected input.
template <typename T, bool HAS_W>
struct FbarSrc {
    const T* __restrict__ ybar;
    const T* __restrict__ un;
    const double* __restrict__ q;
    T cb, cw;
    int ncell;
    double ih0, ih1, ih2;
    __device__ __forceinline__ T operator()(int c, const Nb& nb, int dx, int dy, int dz) const {
        const int j = nb.at(dx, dy, dz);
        T v = cb * ybar[c * ncell + j];
        if constexpr (HAS_W) {
            const int jp = nb.at(dx + (c == 0), dy + (c == 1), dz + (c == 2));
            const double ih = c == 0 ? ih0 : (c == 1 ? ih1 : ih2);
            v += cw * T(double(un[c * ncell + j]) - (q[jp] - q[j]) * ih);
        }
        return v;
    }
};

// Reverse RK4 stage i on 2D grids (3D: k_stage_vjp_zm); see launch_stage_vjp.
template <typename T, int DIM, bool PROJ_U, bool HAS_W>
__global__ __launch_bounds__(kBlock) void k_stage_vjp(Grid g, const T* __restrict__ w, const double* __restrict__ p,
                                                        const T* __restrict__ ybar, const T* __restrict__ un,
                                                        const double* __restrict__ q, T cb, T cw, T* __restrict__ u0bar,
                                                        int u0bar_mode, T* __restrict__ ubar_out, T* __restrict__ fbar_out) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const int64_t boff = int64_t(t.b) * DIM * g.ncell;
    const int64_t soff = int64_t(t.b) * g.ncell;
    const int nc = int(g.ncell);
    VelSrc<T, PROJ_U> U{w + boff, PROJ_U ? p + soff : nullptr, nc, g.ih[0], g.ih[1], g.ih[2]};
    FbarSrc<T, HAS_W> F{ybar + boff, HAS_W ? un + boff : nullptr, HAS_W ? q + soff : nullptr, cb, cw, nc,
                        g.ih[0], g.ih[1], g.ih[2]};
    T out[DIM];
    rhs_vjp_cell<T, DIM>(g, U, F, nb, out);
    const int c0 = nb.at(0, 0, 0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int64_t k = boff + a * g.ncell + c0;
        T acc;
        if (u0bar_mode == 0 || u0bar_mode == 3) {
            acc = ybar[k];  // start from ybar (first reverse stage, or a last stage whose accumulator is ybar)
        } else {
            acc = u0bar[k];
        }
        if constexpr (HAS_W) {
            const int cp = nb.at(a == 0, a == 1, a == 2);
            acc += T(double(un[k]) - (q[soff + cp] - q[soff + c0]) * g.ih[a]);
        }
        if (u0bar_mode >= 2) acc += out[a];
        if (u0bar) u0bar[k] = acc;
        if (ubar_out) ubar_out[k] = out[a];
        if (fbar_out) fbar_out[k] = F(a, nb, 0, 0, 0);
    }
}

template <typename T>
hipError_t launch_rhs_vjp(const Grid& g, const T* u, const T* fbar, T* ubar, hipStream_t s) {
    const int nblk = stencil_blocks(g);
    if (g.dim == 3)
        hipLaunchKernelGGL((k_rhs_vjp<T, 3>), dim3(nblk), dim3(kBlock), 0, s, g, u, fbar, ubar);
    else
        hipLaunchKernelGGL((k_rhs_vjp<T, 2>), dim3(nblk), dim3(kBlock), 0, s, g, u, fbar, ubar);
    return hipGetLastError();
}

template <typename T, int DIM>
static void stage_vjp_dim(const Grid& g, int nblk, const T* w, const double* p, bool proj_u, const T* ybar, const T* un,
                          const double* q, bool has_w, T cb, T cw, T* u0bar, int mode, T* ubar_out, hipStream_t s,
                          T* fbar_out) {
    if (proj_u && has_w)
        hipLaunchKernelGGL((k_stage_vjp<T, DIM, true, true>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, ybar, un, q, cb, cw,
                           u0bar, mode, ubar_out, fbar_out);
    else if (proj_u)
        hipLaunchKernelGGL((k_stage_vjp<T, DIM, true, false>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, ybar, un, q, cb,
                           cw, u0bar, mode, ubar_out, fbar_out);
    else if (has_w)
        hipLaunchKernelGGL((k_stage_vjp<T, DIM, false, true>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, ybar, un, q, cb,
                           cw, u0bar, mode, ubar_out, fbar_out);
    else
        hipLaunchKernelGGL((k_stage_vjp<T, DIM, false, false>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, ybar, un, q, cb,
                           cw, u0bar, mode, ubar_out, fbar_out);
}

// Reverse stage i: with u_i = (proj_u ? w - G p : w) and
// Fbar_i = cb ybar + (has_w ? cw (un - G q) : 0),
//   out = J_F(u_i)^T Fbar_i;
//   u0bar = (mode 0 or 3 ? ybar : u0bar) + (has_w ? un - G q : 0) + (mode 2 or 3 ? out : 0);
//   ubar_out (if not null) = out; u0bar null (modes 0 and 3 only) skips that output.
template <typename T>
hipError_t launch_stage_vjp(const Grid& g, const T* w, const double* p, bool proj_u, const T* ybar, const T* un,
                            const double* q, bool has_w, double cb, double cw, T* u0bar, int mode, T* ubar_out,
                            hipStream_t s, T* fbar_out) {
    if (g.dim == 3)
        return launch_stage_vjp_zm<T>(g, w, p, proj_u, ybar, un, q, has_w, cb, cw, u0bar, mode, ubar_out, s, fbar_out);
    stage_vjp_dim<T, 2>(g, stencil_blocks(g), w, p, proj_u, ybar, un, q, has_w, T(cb), T(cw), u0bar, mode, ubar_out, s,
                        fbar_out);
    return hipGetLastError();
}

template hipError_t launch_rhs_vjp<double>(const Grid&, const double*, const double*, double*, hipStream_t);
template hipError_t launch_rhs_vjp<float>(const Grid&, const float*, const float*, float*, hipStream_t);
template hipError_t launch_stage_vjp<double>(const Grid&, const double*, const double*, bool, const double*,
                                             const double*, const double*, bool, double, double, double*, int, double*,
                                             hipStream_t, double*);
template hipError_t launch_stage_vjp<float>(const Grid&, const float*, const double*, bool, const float*, const float*,
                                            const double*, bool, double, double, float*, int, float*, hipStream_t,
                                            float*);

}  // namespace ins
