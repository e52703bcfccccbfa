// Forward stencil kernels of the staggered periodic grid (App. B of the paper):
// divergence, pressure gradient, diffusion + skew-symmetric convection, the
// projection u - G p, and the fused RK4 stage.
//
// Memory-bound work (about 3 flop per byte in float64): one thread per cell,
// all components of a cell in one thread so each neighbour load is shared by
// the three component stencils, tiles of 64 x 4 cells ordered per XCD so halo
// rows are reused from the L2 of the XCD that loaded them.
#include "k_common.hpp"

namespace ins {

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_rhs(Grid g, const T* __restrict__ u, T* __restrict__ f,
                                                  const T* __restrict__ mc) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const int64_t boff = int64_t(t.b) * DIM * g.ncell;
    VelSrc<T, false> U{u + boff, nullptr, int(g.ncell), g.ih[0], g.ih[1], g.ih[2]};
    T F[DIM];
    rhs_cell<T, DIM>(g, U, nb, F);
    const int c0 = nb.at(0, 0, 0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) f[boff + a * g.ncell + c0] = mc ? F[a] + mc[boff + a * g.ncell + c0] : F[a];
}

// RK4 stage on 2D grids (3D grids use the z-march of k_stage3d.hip):
// u_i = (PROJ ? w - G p : w), F = F(u_i) (+ mc, the closure term at u_i, if given),
// (if y) y = (yinit ? u0 : y) + cy F, and (if wout) wout = u0 + cw F.
template <typename T, int DIM, bool PROJ, typename P = double>
__global__ __launch_bounds__(kBlock) void k_stage(Grid g, const T* __restrict__ w, const P* __restrict__ p,
                                                   const T* __restrict__ u0, T* __restrict__ y, int yinit, T cy,
                                                   T* __restrict__ wout, T cw, const T* __restrict__ mc) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const int64_t boff = int64_t(t.b) * DIM * g.ncell;
    VelSrc<T, PROJ, P> U{w + boff, PROJ ? p + int64_t(t.b) * g.ncell : nullptr, int(g.ncell), g.ih[0], g.ih[1], g.ih[2]};
    T F[DIM];
    rhs_cell<T, DIM>(g, U, nb, F);
    const int c0 = nb.at(0, 0, 0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int64_t k = boff + a * g.ncell + c0;
        if (mc) F[a] += mc[k];
        const T base = (wout || yinit) ? u0[k] : T(0);
        if (y) y[k] = (yinit ? base : y[k]) + cy * F[a];
        if (wout) wout[k] = base + cw * F[a];
    }
}

// r = D u (in P: float64, float32 only in the all-float32 mode), eq. div-kernel.
template <typename T, int DIM, typename P = double>
__global__ __launch_bounds__(kBlock) void k_divergence(Grid g, const T* __restrict__ u, P* __restrict__ r) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const T* ub = u + int64_t(t.b) * DIM * g.ncell;
    const int c0 = nb.at(0, 0, 0);
    P acc = P(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int cm = nb.at(-(a == 0), -(a == 1), -(a == 2));
        acc += (P(ub[a * g.ncell + c0]) - P(ub[a * g.ncell + cm])) * P(g.ih[a]);
    }
    r[int64_t(t.b) * g.ncell + c0] = acc;
}

// g = G p, eq. presgrad-kernel.
template <typename T, int DIM, typename P = double>
__global__ __launch_bounds__(kBlock) void k_gradient(Grid g, const P* __restrict__ p, T* __restrict__ out) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const P* pb = p + int64_t(t.b) * g.ncell;
    T* ob = out + int64_t(t.b) * DIM * g.ncell;
    const int c0 = nb.at(0, 0, 0);
    const P pc = pb[c0];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int cp = nb.at(a == 0, a == 1, a == 2);
        ob[a * g.ncell + c0] = T((pb[cp] - pc) * P(g.ih[a]));
    }
}

// u_out = w - G p, in P (float64 except in the all-float32 mode); u_out may
// alias w (pointwise in w).
template <typename T, int DIM, typename P = double>
__global__ __launch_bounds__(kBlock) void k_apply_projection(Grid g, const T* w, const P* __restrict__ p, T* u_out) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const P* pb = p + int64_t(t.b) * g.ncell;
    const int64_t boff = int64_t(t.b) * DIM * g.ncell;
    const int c0 = nb.at(0, 0, 0);
    const P pc = pb[c0];
    if constexpr (sizeof(T) == 4) {
        // float32 velocity: every load before the first store (u_out may alias
        // w, so a store otherwise holds the next component's loads behind it:
        // three dependent memory round trips per thread); 256^3 0.129 ->
        // 0.120 ms, 512^3 0.94 -> 0.86 ms. For float64 this ordering was 3-5%
        // slower at 256^3 (2% faster at 512^3); float64 keeps the component
        // order and streams w and u non-temporally instead (read and written
        // once: 256^3 0.179 -> 0.159 ms, 512^3 1.425 -> 1.305 ms).
        P wv[DIM], pn[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            wv[a] = P(w[boff + a * g.ncell + c0]);
            pn[a] = pb[nb.at(a == 0, a == 1, a == 2)];
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a) u_out[boff + a * g.ncell + c0] = T(wv[a] - (pn[a] - pc) * P(g.ih[a]));
    } else {
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int cp = nb.at(a == 0, a == 1, a == 2);
            const int64_t k = boff + a * g.ncell + c0;
            __builtin_nontemporal_store(T(P(__builtin_nontemporal_load(w + k)) - (pb[cp] - pc) * P(g.ih[a])), u_out + k);
        }
    }
}

// ubar = D^T rbar: ubar_a[J] = (rbar[J] - rbar[J + e_a]) / h_a.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_div_vjp(Grid g, const double* __restrict__ rbar, T* __restrict__ ubar) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const double* rb = rbar + int64_t(t.b) * g.ncell;
    T* ob = ubar + int64_t(t.b) * DIM * g.ncell;
    const int c0 = nb.at(0, 0, 0);
    const double rc = rb[c0];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int cp = nb.at(a == 0, a == 1, a == 2);
        ob[a * g.ncell + c0] = T((rc - rb[cp]) * g.ih[a]);
    }
}

// pbar = G^T gbar: pbar[I] = sum_a (gbar_a[I - e_a] - gbar_a[I]) / h_a.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_grad_vjp(Grid g, const T* __restrict__ gbar, double* __restrict__ pbar) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const T* gb = gbar + int64_t(t.b) * DIM * g.ncell;
    const int c0 = nb.at(0, 0, 0);
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int cm = nb.at(-(a == 0), -(a == 1), -(a == 2));
        acc += (double(gb[a * g.ncell + cm]) - double(gb[a * g.ncell + c0])) * g.ih[a];
    }
    pbar[int64_t(t.b) * g.ncell + c0] = acc;
}

// ----------------------------------------------------------------------------
// Launchers
// ----------------------------------------------------------------------------
#define INS_DISPATCH_DIM(g, KER, ...)                                                          \
    do {                                                                                       \
        const int nblk = stencil_blocks(g);                                                    \
        if ((g).dim == 3)                                                                      \
            hipLaunchKernelGGL((KER<T, 3>), dim3(nblk), dim3(kBlock), 0, s, __VA_ARGS__);      \
        else                                                                                   \
            hipLaunchKernelGGL((KER<T, 2>), dim3(nblk), dim3(kBlock), 0, s, __VA_ARGS__);      \
    } while (0)

template <typename T>
hipError_t launch_rhs(const Grid& g, const T* u, T* f, hipStream_t s, const T* mc) {
    INS_DISPATCH_DIM(g, k_rhs, g, u, f, mc);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_divergence(const Grid& g, const T* u, double* r, hipStream_t s) {
    INS_DISPATCH_DIM(g, k_divergence, g, u, r);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gradient(const Grid& g, const double* p, T* out, hipStream_t s) {
    INS_DISPATCH_DIM(g, k_gradient, g, p, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_apply_projection(const Grid& g, const T* w, const double* p, T* u_out, hipStream_t s) {
    INS_DISPATCH_DIM(g, k_apply_projection, g, w, p, u_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_div_vjp(const Grid& g, const double* rbar, T* ubar, hipStream_t s) {
    INS_DISPATCH_DIM(g, k_div_vjp, g, rbar, ubar);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_grad_vjp(const Grid& g, const T* gbar, double* pbar, hipStream_t s) {
    INS_DISPATCH_DIM(g, k_grad_vjp, g, gbar, pbar);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_stage(const Grid& g, const T* w, const double* p, bool proj, const T* u0, T* y, bool yinit, double cy,
                        T* wout, double cw, hipStream_t s, const T* mc) {
    if (g.dim == 3) return launch_stage_zm<T>(g, w, p, proj, u0, y, yinit, cy, wout, cw, s, mc);
    const int nblk = stencil_blocks(g);
    const int yi = yinit ? 1 : 0;
    if (proj)
        hipLaunchKernelGGL((k_stage<T, 2, true>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, u0, y, yi, T(cy), wout, T(cw),
                           mc);
    else
        hipLaunchKernelGGL((k_stage<T, 2, false>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, u0, y, yi, T(cy), wout, T(cw),
                           mc);
    return hipGetLastError();
}

// All-float32 comparison mode: float32 pressure-point fields and arithmetic.
hipError_t launch_divergence_f32(const Grid& g, const float* u, float* r, hipStream_t s) {
    const int nblk = stencil_blocks(g);
    if (g.dim == 3)
        hipLaunchKernelGGL((k_divergence<float, 3, float>), dim3(nblk), dim3(kBlock), 0, s, g, u, r);
    else
        hipLaunchKernelGGL((k_divergence<float, 2, float>), dim3(nblk), dim3(kBlock), 0, s, g, u, r);
    return hipGetLastError();
}

hipError_t launch_gradient_f32(const Grid& g, const float* p, float* out, hipStream_t s) {
    const int nblk = stencil_blocks(g);
    if (g.dim == 3)
        hipLaunchKernelGGL((k_gradient<float, 3, float>), dim3(nblk), dim3(kBlock), 0, s, g, p, out);
    else
        hipLaunchKernelGGL((k_gradient<float, 2, float>), dim3(nblk), dim3(kBlock), 0, s, g, p, out);
    return hipGetLastError();
}

hipError_t launch_apply_projection_f32(const Grid& g, const float* w, const float* p, float* u_out, hipStream_t s) {
    const int nblk = stencil_blocks(g);
    if (g.dim == 3)
        hipLaunchKernelGGL((k_apply_projection<float, 3, float>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, u_out);
    else
        hipLaunchKernelGGL((k_apply_projection<float, 2, float>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, u_out);
    return hipGetLastError();
}

hipError_t launch_stage_f32(const Grid& g, const float* w, const float* p, bool proj, const float* u0, float* y,
                            bool yinit, double cy, float* wout, double cw, hipStream_t s) {
    if (g.dim == 3) return launch_stage_zm_f32(g, w, p, proj, u0, y, yinit, cy, wout, cw, s);
    const int nblk = stencil_blocks(g);
    const int yi = yinit ? 1 : 0;
    const float* mc = nullptr;
    if (proj)
        hipLaunchKernelGGL((k_stage<float, 2, true, float>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, u0, y, yi,
                           float(cy), wout, float(cw), mc);
    else
        hipLaunchKernelGGL((k_stage<float, 2, false, float>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, u0, y, yi,
                           float(cy), wout, float(cw), mc);
    return hipGetLastError();
}

#define INS_INSTANTIATE(T)                                                                                          \
    template hipError_t launch_rhs<T>(const Grid&, const T*, T*, hipStream_t, const T*);                            \
    template hipError_t launch_divergence<T>(const Grid&, const T*, double*, hipStream_t);                          \
    template hipError_t launch_gradient<T>(const Grid&, const double*, T*, hipStream_t);                            \
    template hipError_t launch_apply_projection<T>(const Grid&, const T*, const double*, T*, hipStream_t);          \
    template hipError_t launch_div_vjp<T>(const Grid&, const double*, T*, hipStream_t);                             \
    template hipError_t launch_grad_vjp<T>(const Grid&, const T*, double*, hipStream_t);                            \
    template hipError_t launch_stage<T>(const Grid&, const T*, const double*, bool, const T*, T*, bool, double, T*, \
                                        double, hipStream_t, const T*);

INS_INSTANTIATE(double)
INS_INSTANTIATE(float)

}  // namespace ins
