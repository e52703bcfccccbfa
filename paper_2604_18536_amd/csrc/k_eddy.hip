// Smagorinsky eddy-viscosity closure (appendix on eddy-viscosity models:
// general framework, eq. smagorinsky) on the uniform periodic staggered grid,
// and its pullback. Every kernel is a gather stencil (one thread per cell, no
// atomics); arithmetic in float64, fields in the context type.
//
// Locations: D_a = delta_a u^a at the pressure point I; G_ab = delta_b u^a on
// the (a, b) edge J + e_a/2 + e_b/2; the velocity gradient at I takes G_ab as
// the mean of the four edges around I; nu_t = (C_s Delta)^2 sqrt(2 S:S) at I;
// nu_t on an edge is the mean of its four pressure points. The term added to
// the a-momentum right-hand side on the a-face I is
//   M^a = (T_aa[I + e_a] - T_aa[I]) / h_a + sum_{b != a} (T_ab[I] - T_ab[I - e_b]) / h_b,
//   T_aa = 2 nu_t D_a (pressure points), T_ab = 2 nu_e (G_ab + G_ba) / 2 (edges),
// i.e. +sum_b delta_b (2 nu_t S_ab): the appendix's sub-grid stress with the
// sign that makes it dissipate energy.
#include "k_common.hpp"

namespace ins {

namespace {

// Velocity component c at the neighbour (dx, dy, dz) (each in -1..1).
template <typename T>
struct Vel {
    const T* __restrict__ u;
    int ncell;
    const Nb& nb;
    __device__ __forceinline__ double operator()(int c, int dx, int dy, int dz) const {
        return double(u[c * ncell + nb.at(dx, dy, dz)]);
    }
};

template <int DIM>
__device__ __forceinline__ void unit(int a, int& x, int& y, int& z) {
    x = a == 0;
    y = a == 1;
    z = (DIM == 3) && a == 2;
}

// delta_a u^a at the pressure point shifted by o.
template <typename V>
__device__ __forceinline__ double diag_at(const V& U, const Grid& g, int a, int ox, int oy, int oz) {
    const int ax = a == 0, ay = a == 1, az = a == 2;
    return (U(a, ox, oy, oz) - U(a, ox - ax, oy - ay, oz - az)) * g.ih[a];
}

// S_ab = (G_ab + G_ba) / 2 on the (a, b) edge J = I + o.
template <typename V>
__device__ __forceinline__ double edge_strain(const V& U, const Grid& g, int a, int b, int ox, int oy, int oz) {
    const int ax = a == 0, ay = a == 1, az = a == 2;
    const int bx = b == 0, by = b == 1, bz = b == 2;
    const double gab = (U(a, ox + bx, oy + by, oz + bz) - U(a, ox, oy, oz)) * g.ih[b];
    const double gba = (U(b, ox + ax, oy + ay, oz + az) - U(b, ox, oy, oz)) * g.ih[a];
    return 0.5 * (gab + gba);
}

// Symmetric strain S at the pressure point I + o (S[a][b], a, b < DIM) and sqrt(2 S:S).
template <int DIM, typename V>
__device__ __forceinline__ double centre_strain(const V& U, const Grid& g, int ox, int oy, int oz, double S[3][3]) {
    double ss = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        S[a][a] = diag_at(U, g, a, ox, oy, oz);
        ss += S[a][a] * S[a][a];
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
#pragma unroll
        for (int b = a + 1; b < DIM; ++b) {
            // A_ab at I: mean over the 4 edges = (u^a[I+e_b] - u^a[I-e_b] + u^a[I-e_a+e_b] - u^a[I-e_a-e_b]) / (4 h_b)
            const int ax = a == 0, ay = a == 1, az = a == 2;
            const int bx = b == 0, by = b == 1, bz = b == 2;
            const double aab = 0.25 * g.ih[b] *
                               (U(a, ox + bx, oy + by, oz + bz) - U(a, ox - bx, oy - by, oz - bz) +
                                U(a, ox - ax + bx, oy - ay + by, oz - az + bz) - U(a, ox - ax - bx, oy - ay - by, oz - az - bz));
            const double aba = 0.25 * g.ih[a] *
                               (U(b, ox + ax, oy + ay, oz + az) - U(b, ox - ax, oy - ay, oz - az) +
                                U(b, ox - bx + ax, oy - by + ay, oz - bz + az) - U(b, ox - bx - ax, oy - by - ay, oz - bz - az));
            const double s = 0.5 * (aab + aba);
            S[a][b] = S[b][a] = s;
            ss += 2.0 * s * s;
        }
    }
    return sqrt(2.0 * ss);
}

}  // namespace

// nu[b][I] = c2 sqrt(2 S:S).
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_eddy_nu(Grid g, const T* __restrict__ u, T* __restrict__ nu, double c2) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const Vel<T> U{u + int64_t(t.b) * DIM * g.ncell, int(g.ncell), nb};
    double S[3][3];
    const double root = centre_strain<DIM>(U, g, 0, 0, 0, S);
    nu[int64_t(t.b) * g.ncell + nb.at(0, 0, 0)] = T(c2 * root);
}

// m = M(u) (overwritten).
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_eddy_term(Grid g, const T* __restrict__ u, const T* __restrict__ nu,
                                                        T* __restrict__ m) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const int64_t boff = int64_t(t.b) * DIM * g.ncell;
    const Vel<T> U{u + boff, int(g.ncell), nb};
    const T* nub = nu + int64_t(t.b) * g.ncell;
    auto N = [&](int dx, int dy, int dz) { return double(nub[nb.at(dx, dy, dz)]); };
    const int c0 = nb.at(0, 0, 0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        int ax, ay, az;
        unit<DIM>(a, ax, ay, az);
        double acc = (2.0 * N(ax, ay, az) * diag_at(U, g, a, ax, ay, az) - 2.0 * N(0, 0, 0) * diag_at(U, g, a, 0, 0, 0)) *
                     g.ih[a];
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            if (b == a) continue;
            int bx, by, bz;
            unit<DIM>(b, bx, by, bz);
            // edges J = I and J = I - e_b
            const double nu0 = 0.25 * (N(0, 0, 0) + N(ax, ay, az) + N(bx, by, bz) + N(ax + bx, ay + by, az + bz));
            const double nu1 = 0.25 * (N(-bx, -by, -bz) + N(ax - bx, ay - by, az - bz) + N(0, 0, 0) + N(ax, ay, az));
            const double t0 = 2.0 * nu0 * edge_strain(U, g, a, b, 0, 0, 0);
            const double t1 = 2.0 * nu1 * edge_strain(U, g, a, b, -bx, -by, -bz);
            acc += (t0 - t1) * g.ih[b];
        }
        m[boff + a * g.ncell + c0] = T(acc);
    }
}

// Pullback, first pass (pressure points): with tbar_aa = (mbar^a[I - e_a] - mbar^a[I]) / h_a
// and, on each (a, b) edge J, tbar_ab = (mbar^a[J] - mbar^a[J + e_b]) / h_b,
//   nubar[I] = sum_a 2 tbar_aa D_a + sum_{a<b} 1/4 sum_{4 edges J around I} 2 S_ab[J] (tbar_ab + tbar_ba)[J],
//   g = c2 nubar / sqrt(2 S:S) (0 where S = 0), P_ab[I] = 2 g S_ab[I] (symmetric, a <= b),
// the cotangent of the centre velocity gradient. P is stored as DIM (DIM + 1) / 2
// planar fields per batch entry, ordered (0,0), (1,1), [(2,2),] (0,1), [(0,2), (1,2)].
template <int DIM>
__device__ __forceinline__ int pidx(int a, int b) {
    if (a == b) return a;
    if (a > b) {
        const int t = a;
        a = b;
        b = t;
    }
    return DIM == 2 ? 2 : (a == 0 ? (b == 1 ? 3 : 4) : 5);
}

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_eddy_vjp_centre(Grid g, const T* __restrict__ u, const T* __restrict__ mbar,
                                                              T* __restrict__ P, double c2) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    constexpr int NP = DIM * (DIM + 1) / 2;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const int64_t boff = int64_t(t.b) * DIM * g.ncell;
    const Vel<T> U{u + boff, int(g.ncell), nb};
    const Vel<T> MB{mbar + boff, int(g.ncell), nb};
    double S[3][3];
    const double root = centre_strain<DIM>(U, g, 0, 0, 0, S);
    double nubar = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        int ax, ay, az;
        unit<DIM>(a, ax, ay, az);
        const double tbar = (MB(a, -ax, -ay, -az) - MB(a, 0, 0, 0)) * g.ih[a];
        nubar += 2.0 * tbar * S[a][a];
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
#pragma unroll
        for (int b = a + 1; b < DIM; ++b) {
            int ax, ay, az, bx, by, bz;
            unit<DIM>(a, ax, ay, az);
            unit<DIM>(b, bx, by, bz);
            double e = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {  // edges J = I - (k & 1) e_a - (k >> 1) e_b
                const int ox = -(k & 1) * ax - (k >> 1) * bx;
                const int oy = -(k & 1) * ay - (k >> 1) * by;
                const int oz = -(k & 1) * az - (k >> 1) * bz;
                const double tab = (MB(a, ox, oy, oz) - MB(a, ox + bx, oy + by, oz + bz)) * g.ih[b];
                const double tba = (MB(b, ox, oy, oz) - MB(b, ox + ax, oy + ay, oz + az)) * g.ih[a];
                e += edge_strain(U, g, a, b, ox, oy, oz) * (tab + tba);
            }
            nubar += 0.5 * e;  // 1/4 * 2
        }
    }
    const double gg = root > 0.0 ? c2 * nubar / root : 0.0;
    const int c0 = nb.at(0, 0, 0);
    T* pb = P + int64_t(t.b) * NP * g.ncell;
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = a; b < DIM; ++b) pb[pidx<DIM>(a, b) * g.ncell + c0] = T(2.0 * gg * S[a][b]);
}

// Pullback, second pass (faces): ubar^a[I] += (Dbar_a[I] - Dbar_a[I + e_a]) / h_a
//   + sum_{b != a} (Gbar_ab[I - e_b] - Gbar_ab[I]) / h_b, with
//   Dbar_a[K] = 2 tbar_aa[K] nu[K] + P_aa[K],
//   Gbar_ab[J] = nu_e[J] (tbar_ab + tbar_ba)[J] + 1/4 sum_{4 pressure points around J} P_ab.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_eddy_vjp_face(Grid g, const T* __restrict__ nu, const T* __restrict__ mbar,
                                                            const T* __restrict__ P, T* __restrict__ ubar) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    constexpr int NP = DIM * (DIM + 1) / 2;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const int64_t boff = int64_t(t.b) * DIM * g.ncell;
    const Vel<T> MB{mbar + boff, int(g.ncell), nb};
    const T* nub = nu + int64_t(t.b) * g.ncell;
    const T* pb = P + int64_t(t.b) * NP * g.ncell;
    auto N = [&](int dx, int dy, int dz) { return double(nub[nb.at(dx, dy, dz)]); };
    auto PP = [&](int k, int dx, int dy, int dz) { return double(pb[k * g.ncell + nb.at(dx, dy, dz)]); };
    const int c0 = nb.at(0, 0, 0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        int ax, ay, az;
        unit<DIM>(a, ax, ay, az);
        auto dbar = [&](int ox, int oy, int oz) {
            const double tbar = (MB(a, ox - ax, oy - ay, oz - az) - MB(a, ox, oy, oz)) * g.ih[a];
            return 2.0 * tbar * N(ox, oy, oz) + PP(a, ox, oy, oz);
        };
        double acc = (dbar(0, 0, 0) - dbar(ax, ay, az)) * g.ih[a];
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            if (b == a) continue;
            int bx, by, bz;
            unit<DIM>(b, bx, by, bz);
            const int k = pidx<DIM>(a, b);
            auto gbar = [&](int ox, int oy, int oz) {  // on the (a, b) edge J = I + o
                const double nue = 0.25 * (N(ox, oy, oz) + N(ox + ax, oy + ay, oz + az) + N(ox + bx, oy + by, oz + bz) +
                                           N(ox + ax + bx, oy + ay + by, oz + az + bz));
                const double tab = (MB(a, ox, oy, oz) - MB(a, ox + bx, oy + by, oz + bz)) * g.ih[b];
                const double tba = (MB(b, ox, oy, oz) - MB(b, ox + ax, oy + ay, oz + az)) * g.ih[a];
                const double pav = 0.25 * (PP(k, ox, oy, oz) + PP(k, ox + ax, oy + ay, oz + az) +
                                           PP(k, ox + bx, oy + by, oz + bz) + PP(k, ox + ax + bx, oy + ay + by, oz + az + bz));
                return nue * (tab + tba) + pav;
            };
            acc += (gbar(-bx, -by, -bz) - gbar(0, 0, 0)) * g.ih[b];
        }
        T* dst = ubar + boff + a * g.ncell + c0;
        *dst = T(double(*dst) + acc);
    }
}

#define INS_EDDY_DISPATCH(g, KER, ...)                                                     \
    do {                                                                                   \
        const int nblk = stencil_blocks(g);                                                \
        if ((g).dim == 3)                                                                  \
            hipLaunchKernelGGL((KER<T, 3>), dim3(nblk), dim3(kBlock), 0, s, __VA_ARGS__);  \
        else                                                                               \
            hipLaunchKernelGGL((KER<T, 2>), dim3(nblk), dim3(kBlock), 0, s, __VA_ARGS__);  \
    } while (0)

template <typename T>
hipError_t launch_eddy_forward(const Grid& g, const T* u, T* nu, T* m, double c2, hipStream_t s) {
    INS_EDDY_DISPATCH(g, k_eddy_nu, g, u, nu, c2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    INS_EDDY_DISPATCH(g, k_eddy_term, g, u, nu, m);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_eddy_backward(const Grid& g, const T* u, const T* nu, const T* mbar, T* P, T* ubar, double c2,
                                hipStream_t s) {
    INS_EDDY_DISPATCH(g, k_eddy_vjp_centre, g, u, mbar, P, c2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    INS_EDDY_DISPATCH(g, k_eddy_vjp_face, g, nu, mbar, P, ubar);
    return hipGetLastError();
}

#undef INS_EDDY_DISPATCH

template hipError_t launch_eddy_forward<double>(const Grid&, const double*, double*, double*, double, hipStream_t);
template hipError_t launch_eddy_forward<float>(const Grid&, const float*, float*, float*, double, hipStream_t);
template hipError_t launch_eddy_backward<double>(const Grid&, const double*, const double*, const double*, double*,
                                                 double*, double, hipStream_t);
template hipError_t launch_eddy_backward<float>(const Grid&, const float*, const float*, const float*, float*, float*,
                                                double, hipStream_t);

}  // namespace ins
