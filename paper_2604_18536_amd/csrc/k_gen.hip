// Kernels of the stretched grid: non-uniform widths along any direction
// (Sec. 2.5 non-uniform grids, e.g. the tanh grid of eq. tanh-grid; App. B
// kernels with the widths |Delta^a_i|), x and z periodic, y periodic or
// bounded by no-slip walls (the channel's ghost rules: u^y on a wall face
// reads 0 and every output writes 0 on the stored upper-wall face, a
// tangential component beyond a wall is minus the first interior value), and
// the conjugate-gradient pressure solve on it (Sec. 2.6.1 iterative solver).
//
// Metrics per direction a (Grid::gm[a], filled by the runtime; code index i,
// cell i spans [f_i, f_{i+1}]): w_i = f_{i+1} - f_i, d_i = (w_i + w_{i+1}) / 2
// the velocity-volume width around face i (the face on the right of cell i),
// theta_i = w_i / (w_i + w_{i+1}) the mass-flux weight of cell i at face i;
// periodic images wrap, beyond a wall the first/last row is mirrored
// (d_{-1} = w_0, d_{N-1} = w_{N-1}, theta = 1/2 there). Stored for
// i = -1 .. N so that every stencil reads them without branches.
//
// Operators: divergence r[I] = sum_a (u^a[I] - u^a[I - e_a]) / w^a; gradient
// (G p)^a[I] = (p[I + e_a] - p[I]) / d^a; diffusion of eq. diff-kernel (outer
// width of the velocity volume, inner widths between the neighbouring points);
// convection F^{ab} = A^{ab} B^{ab} with the transported component averaged
// along b with weights 1/2 and the transporting one interpolated along a as
// the mass-flux average theta^a (1/2 when b = a), which keeps the discrete
// convection energy-conserving on a grid stretched in every direction. The
// pullbacks gather, for each output, every flux factor it enters with its
// interpolation weight. Volumes: Omega_p = prod_a w^a, Omega_u^a = d^a
// prod_{b != a} w^b; CG runs on the symmetric A = -Omega_p D G.
//
// One thread per cell (64 x 4 tiles): these grids are solved by CG, whose
// iterations dominate the step.
#include "k_cg.hpp"
#include "k_common.hpp"

namespace ins {

namespace {

// Metric arrays of one direction, indexed by the coordinate i in -1 .. N.
struct Axis {
    const double* m;
    int S;
    __device__ __forceinline__ Axis(const Grid& g, int a)
        : m(g.gm[a]), S((a == 0 ? g.nx : (a == 1 ? g.ny : g.nz)) + 2) {}
    __device__ __forceinline__ double iw(int i) const { return m[i + 1]; }
    __device__ __forceinline__ double id(int i) const { return m[S + i + 1]; }
    __device__ __forceinline__ double th(int i) const { return m[2 * S + i + 1]; }
    __device__ __forceinline__ double w(int i) const { return m[3 * S + i + 1]; }
    __device__ __forceinline__ double d(int i) const { return m[4 * S + i + 1]; }
};

// Metrics of the cell at (x, y, z) and its neighbours along each direction,
// loaded once per thread: k = 0, 1, 2 for the coordinates c - 1, c, c + 1.
template <int DIM>
struct CellM {
    double iw[3][3], id[3][3], th[3][2];
    __device__ __forceinline__ CellM(const Grid& g, int x, int y, int z) {
        const int c[3] = {x, y, z};
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const Axis A(g, a);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                iw[a][k] = A.iw(c[a] + k - 1);
                id[a][k] = A.id(c[a] + k - 1);
            }
            th[a][0] = A.th(c[a] - 1);
            th[a][1] = A.th(c[a]);
        }
    }
};

// Neighbour offsets: x and z wrap; y wraps (periodic) or mirrors the first /
// last row beyond a wall, with the wall flags of each row y - 1 .. y + 2.
template <int DIM>
__device__ __forceinline__ Nb make_gen_nb(const Grid& g, int x, int y, int z, int ghost[4], int unk[4]) {
    Nb nb;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        nb.xo[k] = wrap(x + k - 1, g.nx);
        const int r = y + k - 1;
        if (g.ywalls) {
            const int m = r < 0 ? 0 : (r >= g.ny ? g.ny - 1 : r);
            nb.yo[k] = m * g.nx;
            ghost[k] = (r < 0 || r >= g.ny) ? 1 : 0;
            unk[k] = (r >= 0 && r <= g.ny - 2) ? 1 : 0;
        } else {
            nb.yo[k] = wrap(r, g.ny) * g.nx;
            ghost[k] = 0;
            unk[k] = 1;
        }
        nb.zo[k] = (DIM == 3) ? wrap(z + k - 1, g.nz) * g.nx * g.ny : 0;
    }
    return nb;
}

// Velocity at a neighbour (PROJ: the stage velocity w - G p, formed in
// float64 with the neighbour face's 1 / d), wall rules applied.
template <typename T, bool PROJ>
struct GenVel {
    const T* __restrict__ w;
    const double* __restrict__ p;
    int ncell;
    int ghost[4], unk[4];
    Axis ax, ay, az;
    int x, y, z;
    __device__ __forceinline__ T operator()(int c, const Nb& nb, int dx, int dy, int dz) const {
        const int k = dy + 1;
        if (c == 1 && !unk[k]) return T(0);
        const int j = nb.at(dx, dy, dz);
        T v;
        if constexpr (!PROJ) {
            v = w[c * ncell + j];
        } else {
            const int jp = nb.at(dx + (c == 0), dy + (c == 1), dz + (c == 2));
            const double idc = c == 0 ? ax.id(x + dx) : (c == 1 ? ay.id(y + dy) : az.id(z + dz));
            v = T(double(w[c * ncell + j]) - (p[jp] - p[j]) * idc);
        }
        return (c != 1 && ghost[k]) ? -v : v;
    }
};

// Stage cotangent Fbar = cb ybar + (HAS_W ? cw (un - Omega_u G q) : 0) at a
// neighbour, wall rules applied; un - Omega_u G q completes the transposed
// projection Omega_u P Omega_u^{-1} of the next stage's cotangent (q solved
// from D Omega_u^{-1} un): Omega_u^c G^c q = (prod_{b != c} w^b) (q[J + e_c] - q[J]).
template <typename T, bool HAS_W, int DIM>
struct GenFbar {
    const T* __restrict__ ybar;
    const T* __restrict__ un;
    const double* __restrict__ q;
    T cb, cw;
    int ncell;
    int ghost[4], unk[4];
    Axis ax, ay, az;
    int x, y, z;
    __device__ __forceinline__ T operator()(int c, const Nb& nb, int dx, int dy, int dz) const {
        const int k = dy + 1;
        if (c == 1 && !unk[k]) return T(0);
        const int j = nb.at(dx, dy, dz);
        T v = cb * ybar[c * ncell + j];
        if constexpr (HAS_W) {
            const int jp = nb.at(dx + (c == 0), dy + (c == 1), dz + (c == 2));
            const double wx = ax.w(x + dx), wy = ay.w(y + dy), wz = DIM == 3 ? az.w(z + dz) : 1.0;
            const double cross = c == 0 ? wy * wz : (c == 1 ? wx * wz : wx * wy);
            v += cw * T(double(un[c * ncell + j]) - cross * (q[jp] - q[j]));
        }
        return (c != 1 && ghost[k]) ? -v : v;
    }
};

// F^a at the current cell: diffusion (eq. diff-kernel), convection with the
// weights above, and the constant body force.
template <typename T, int DIM, class Src>
__device__ __forceinline__ void gen_rhs_cell(const Grid& g, const Src& U, const Nb& nb, const CellM<DIM>& M, T F[DIM]) {
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int ax = a == 0, ay = a == 1, az = a == 2;
        const T uc = U(a, nb, 0, 0, 0);
        const T tha = T(M.th[a][1]);
        T diff = T(0), conv = T(0);
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            const int bx = b == 0, by = b == 1, bz = b == 2;
            const T up = U(a, nb, bx, by, bz);
            const T um = U(a, nb, -bx, -by, -bz);
            T s;
            if (b == a) {
                diff += ((up - uc) * T(M.iw[a][2]) - (uc - um) * T(M.iw[a][1])) * T(M.id[a][1]);
                s = T(M.id[a][1]);
            } else {
                diff += ((up - uc) * T(M.id[b][1]) - (uc - um) * T(M.id[b][0])) * T(M.iw[b][1]);
                s = T(M.iw[b][1]);
            }
            T vr, vl;
            if (b != a) {
                vr = tha * U(b, nb, 0, 0, 0) + (T(1) - tha) * U(b, nb, ax, ay, az);
                vl = tha * U(b, nb, -bx, -by, -bz) + (T(1) - tha) * U(b, nb, ax - bx, ay - by, az - bz);
            } else {
                vr = T(0.5) * (U(b, nb, 0, 0, 0) + U(b, nb, ax, ay, az));
                vl = T(0.5) * (U(b, nb, -bx, -by, -bz) + U(b, nb, ax - bx, ay - by, az - bz));
            }
            const T fr = T(0.5) * (uc + up) * vr;
            const T fl = T(0.5) * (um + uc) * vl;
            conv -= (fr - fl) * s;
        }
        F[a] = conv + T(g.nu) * diff + T(g.force[a]);
    }
}

// 1 / W^{ab} (W = d^a along a, w^b across) at the point k - 1 along b of the
// a-velocity volume's stencil (k = 0, 1, 2 for offsets -1, 0, +1 along b).
template <typename T, int DIM>
__device__ __forceinline__ T gen_s(const CellM<DIM>& M, int a, int b, int k) {
    return b == a ? T(M.id[a][k]) : T(M.iw[b][k]);
}

// Pullback of the right-hand side at one cell, gather form: the diffusion
// transpose plus, for each flux F^{ab}[K] = A^{ab}[K] B^{ab}[K] containing
// u^g[J], its other factor times Fbar^{ab}[K] = -fbar^a[K] s(K) + fbar^a[K +
// e_b] s(K + e_b), with the interpolation weight of u^g[J] in its own factor.
template <typename T, int DIM, class USrc, class FSrc>
__device__ __forceinline__ void gen_rhs_vjp_cell(const Grid& g, const USrc& U, const FSrc& Fb, const Nb& nb,
                                                 const CellM<DIM>& M, T out[DIM]) {
#pragma unroll
    for (int gm = 0; gm < DIM; ++gm) {
        const int gx = gm == 0, gy = gm == 1, gz = gm == 2;
        const T fc = Fb(gm, nb, 0, 0, 0);
        const T thg = T(M.th[gm][1]);
        T diff = T(0), acc = T(0);
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            const int bx = b == 0, by = b == 1, bz = b == 2;
            const T fp = Fb(gm, nb, bx, by, bz);
            const T fm = Fb(gm, nb, -bx, -by, -bz);
            if (b == gm) {
                diff += fm * T(M.id[b][0] * M.iw[b][1]) - fc * T(M.id[b][1] * (M.iw[b][2] + M.iw[b][1])) +
                        fp * T(M.id[b][2] * M.iw[b][2]);
            } else {
                diff += fm * T(M.iw[b][0] * M.id[b][0]) - fc * T(M.iw[b][1] * (M.id[b][1] + M.id[b][0])) +
                        fp * T(M.iw[b][2] * M.id[b][1]);
            }
            // u^gm transported in F^{gm b} at K = J and K = J - e_b (weights 1/2)
            const T F0 = -fc * gen_s<T, DIM>(M, gm, b, 1) + fp * gen_s<T, DIM>(M, gm, b, 2);
            const T F1 = -fm * gen_s<T, DIM>(M, gm, b, 0) + fc * gen_s<T, DIM>(M, gm, b, 1);
            T B0, B1;
            if (b != gm) {
                B0 = thg * U(b, nb, 0, 0, 0) + (T(1) - thg) * U(b, nb, gx, gy, gz);
                B1 = thg * U(b, nb, -bx, -by, -bz) + (T(1) - thg) * U(b, nb, gx - bx, gy - by, gz - bz);
            } else {
                B0 = T(0.5) * (U(b, nb, 0, 0, 0) + U(b, nb, gx, gy, gz));
                B1 = T(0.5) * (U(b, nb, -bx, -by, -bz) + U(b, nb, gx - bx, gy - by, gz - bz));
            }
            acc += T(0.5) * (F0 * B0 + F1 * B1);
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int ax = a == 0, ay = a == 1, az = a == 2;
            // u^gm transporting in F^{a gm} at K = J and K = J - e_a
            const T sJ = a == gm ? T(M.id[a][1]) : T(M.iw[gm][1]);       // s^{a gm} at J
            const T sJg = a == gm ? T(M.id[a][2]) : T(M.iw[gm][2]);      // at J + e_gm
            const T sJa = a == gm ? T(M.id[a][0]) : T(M.iw[gm][1]);      // at J - e_a
            const T sJag = a == gm ? T(M.id[a][1]) : T(M.iw[gm][2]);     // at J - e_a + e_gm
            const T F0 = -Fb(a, nb, 0, 0, 0) * sJ + Fb(a, nb, gx, gy, gz) * sJg;
            const T A0 = T(0.5) * (U(a, nb, 0, 0, 0) + U(a, nb, gx, gy, gz));
            const T F1 = -Fb(a, nb, -ax, -ay, -az) * sJa + Fb(a, nb, gx - ax, gy - ay, gz - az) * sJag;
            const T A1 = T(0.5) * (U(a, nb, -ax, -ay, -az) + U(a, nb, gx - ax, gy - ay, gz - az));
            T w0 = T(0.5), w1 = T(0.5);
            if (a != gm) {
                w0 = T(M.th[a][1]);
                w1 = T(1) - T(M.th[a][0]);
            }
            acc += w0 * F0 * A0 + w1 * F1 * A1;
        }
        out[gm] = acc + T(g.nu) * diff;
    }
}

template <typename T, bool PROJ>
__device__ __forceinline__ GenVel<T, PROJ> gen_vel(const Grid& g, const T* w, const double* p, const int ghost[4],
                                                   const int unk[4], int x, int y, int z) {
    GenVel<T, PROJ> U{w, p, int(g.ncell), {}, {}, Axis(g, 0), Axis(g, 1), Axis(g, g.dim == 3 ? 2 : 0), x, y, z};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        U.ghost[k] = ghost[k];
        U.unk[k] = unk[k];
    }
    return U;
}

template <typename T, bool HAS_W, int DIM>
__device__ __forceinline__ GenFbar<T, HAS_W, DIM> gen_fbar(const Grid& g, const T* ybar, const T* un, const double* q,
                                                           T cb, T cw, const int ghost[4], const int unk[4], int x,
                                                           int y, int z) {
    GenFbar<T, HAS_W, DIM> F{ybar, un, q, cb, cw, int(g.ncell), {}, {}, Axis(g, 0), Axis(g, 1),
                             Axis(g, DIM == 3 ? 2 : 0), x, y, z};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        F.ghost[k] = ghost[k];
        F.unk[k] = unk[k];
    }
    return F;
}

__device__ __forceinline__ bool upper_wall(const Grid& g, int y) { return g.ywalls && y == g.ny - 1; }

// ----------------------------------------------------------------------------
// Forward stencils
// ----------------------------------------------------------------------------

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_gen_rhs(Grid g, const T* __restrict__ u, T* __restrict__ f) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    int ghost[4], unk[4];
    const Nb nb = make_gen_nb<DIM>(g, t.x, t.y, t.z, ghost, unk);
    const int64_t boff = int64_t(t.b) * DIM * g.ncell;
    const auto U = gen_vel<T, false>(g, u + boff, nullptr, ghost, unk, t.x, t.y, t.z);
    T F[DIM];
    gen_rhs_cell<T, DIM>(g, U, nb, CellM<DIM>(g, t.x, t.y, t.z), F);
    const int c0 = nb.at(0, 0, 0);
    const bool wall = upper_wall(g, t.y);
#pragma unroll
    for (int a = 0; a < DIM; ++a) f[boff + a * g.ncell + c0] = (a == 1 && wall) ? T(0) : F[a];
}

// Runge-Kutta stage (the contract of the periodic and channel stages):
// u_i = (PROJ ? w - G p : w), F = F(u_i); (if y) y = (yinit ? u0 : y) + cy F;
// (if wout) wout = u0 + cw F.
template <typename T, int DIM, bool PROJ>
__global__ __launch_bounds__(kBlock) void k_gen_stage(Grid g, const T* __restrict__ w, const double* __restrict__ p,
                                                       const T* __restrict__ u0, T* __restrict__ y, int yinit, T cy,
                                                       T* __restrict__ wout, T cw) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    int ghost[4], unk[4];
    const Nb nb = make_gen_nb<DIM>(g, t.x, t.y, t.z, ghost, unk);
    const int64_t boff = int64_t(t.b) * DIM * g.ncell;
    const auto U = gen_vel<T, PROJ>(g, w + boff, PROJ ? p + int64_t(t.b) * g.ncell : nullptr, ghost, unk, t.x, t.y, t.z);
    T F[DIM];
    gen_rhs_cell<T, DIM>(g, U, nb, CellM<DIM>(g, t.x, t.y, t.z), F);
    const int c0 = nb.at(0, 0, 0);
    const bool wall = upper_wall(g, t.y);
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

// u_out = w - G p (ADJ: w - Omega_u G p, the transposed projection's
// correction); float64 arithmetic; 0 on the upper-wall face; u_out may alias w.
template <typename T, int DIM, bool ADJ>
__global__ __launch_bounds__(kBlock) void k_gen_project(Grid g, const T* w, const double* __restrict__ p, T* u_out) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const double* pb = p + int64_t(t.b) * g.ncell;
    const int64_t boff = int64_t(t.b) * DIM * g.ncell;
    const int c0 = nb.at(0, 0, 0);
    const double pc = pb[c0];
    const bool wall = upper_wall(g, t.y);
    const int c[3] = {t.x, t.y, t.z};
    double wv[3] = {1.0, 1.0, 1.0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) wv[a] = Axis(g, a).w(c[a]);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int64_t k = boff + a * g.ncell + c0;
        if (a == 1 && wall) {
            u_out[k] = T(0);
            continue;
        }
        const double dp = pb[nb.at(a == 0, a == 1, a == 2)] - pc;
        double gp;
        if constexpr (ADJ) {
            gp = dp * (a == 0 ? wv[1] * wv[2] : (a == 1 ? wv[0] * wv[2] : wv[0] * wv[1]));
        } else {
            gp = dp * Axis(g, a).id(c[a]);
        }
        u_out[k] = T(double(w[k]) - gp);
    }
}

// G p on the faces (0 on the upper-wall face).
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_gen_gradient(Grid g, const double* __restrict__ p, T* __restrict__ out) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const double* pb = p + int64_t(t.b) * g.ncell;
    T* ob = out + int64_t(t.b) * DIM * g.ncell;
    const int c0 = nb.at(0, 0, 0);
    const double pc = pb[c0];
    const bool wall = upper_wall(g, t.y);
    const int c[3] = {t.x, t.y, t.z};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double dp = pb[nb.at(a == 0, a == 1, a == 2)] - pc;
        ob[a * g.ncell + c0] = (a == 1 && wall) ? T(0) : T(dp * Axis(g, a).id(c[a]));
    }
}

// D u at one cell with the wall faces of u^y read as 0; SCALED reads
// Omega_u^{-1} u instead of u.
template <typename T, int DIM, bool SCALED>
__device__ __forceinline__ double gen_div_cell(const Grid& g, const T* ub, const Nb& nb, int x, int y, int z) {
    const int c[3] = {x, y, z};
    const int c0 = nb.at(0, 0, 0);
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const Axis A(g, a);
        double up = double(ub[a * g.ncell + c0]);
        double dn = double(ub[a * g.ncell + nb.at(-(a == 0), -(a == 1), -(a == 2))]);
        if (a == 1 && g.ywalls) {
            if (y == g.ny - 1) up = 0.0;
            if (y == 0) dn = 0.0;
        }
        if constexpr (SCALED) {
            // Omega_u^a at the two faces: d^a of the face times the cross widths of this cell
            double cross = 1.0;
#pragma unroll
            for (int b = 0; b < DIM; ++b)
                if (b != a) cross *= Axis(g, b).w(c[b]);
            up /= A.d(c[a]) * cross;
            dn /= A.d(c[a] - 1) * cross;
        }
        acc += (up - dn) * A.iw(c[a]);
    }
    return acc;
}

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_gen_divergence(Grid g, const T* __restrict__ u, double* __restrict__ r) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    r[int64_t(t.b) * g.ncell + nb.at(0, 0, 0)] =
        gen_div_cell<T, DIM, false>(g, u + int64_t(t.b) * DIM * g.ncell, nb, t.x, t.y, t.z);
}

// ----------------------------------------------------------------------------
// Pullbacks
// ----------------------------------------------------------------------------

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_gen_rhs_vjp(Grid g, const T* __restrict__ u, const T* __restrict__ fbar,
                                                         T* __restrict__ ubar) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    int ghost[4], unk[4];
    const Nb nb = make_gen_nb<DIM>(g, t.x, t.y, t.z, ghost, unk);
    const int64_t boff = int64_t(t.b) * DIM * g.ncell;
    const auto U = gen_vel<T, false>(g, u + boff, nullptr, ghost, unk, t.x, t.y, t.z);
    const auto F = gen_fbar<T, false, DIM>(g, fbar + boff, nullptr, nullptr, T(1), T(0), ghost, unk, t.x, t.y, t.z);
    T out[DIM];
    gen_rhs_vjp_cell<T, DIM>(g, U, F, nb, CellM<DIM>(g, t.x, t.y, t.z), out);
    const int c0 = nb.at(0, 0, 0);
    const bool wall = upper_wall(g, t.y);
#pragma unroll
    for (int a = 0; a < DIM; ++a) ubar[boff + a * g.ncell + c0] = (a == 1 && wall) ? T(0) : out[a];
}

// Reverse stage (the contract of the periodic and channel reverse stages,
// without a closure): the right-hand-side cotangent is Fbar = cb ybar +
// (HAS_W ? cw (un - Omega_u G q) : 0); out = J_F(u_i)^T Fbar at the stage
// velocity u_i = (PROJ_U ? w - G p : w); the running sum u0bar becomes
// (mode 0, 3: ybar; else u0bar) + (HAS_W ? un - Omega_u G q : 0) + (mode >= 2 ? out : 0).
template <typename T, int DIM, bool PROJ_U, bool HAS_W>
__global__ __launch_bounds__(kBlock) void k_gen_stage_vjp(Grid g, const T* __restrict__ w, const double* __restrict__ p,
                                                           const T* __restrict__ ybar, const T* __restrict__ un,
                                                           const double* __restrict__ q, T cb, T cw,
                                                           T* __restrict__ u0bar, int mode, T* __restrict__ ubar_out) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    int ghost[4], unk[4];
    const Nb nb = make_gen_nb<DIM>(g, t.x, t.y, t.z, ghost, unk);
    const int64_t boff = int64_t(t.b) * DIM * g.ncell;
    const int64_t soff = int64_t(t.b) * g.ncell;
    const auto U = gen_vel<T, PROJ_U>(g, w + boff, PROJ_U ? p + soff : nullptr, ghost, unk, t.x, t.y, t.z);
    const auto F = gen_fbar<T, HAS_W, DIM>(g, ybar + boff, HAS_W ? un + boff : nullptr, HAS_W ? q + soff : nullptr, cb,
                                           cw, ghost, unk, t.x, t.y, t.z);
    T out[DIM];
    gen_rhs_vjp_cell<T, DIM>(g, U, F, nb, CellM<DIM>(g, t.x, t.y, t.z), out);
    const int c0 = nb.at(0, 0, 0);
    const bool wall = upper_wall(g, t.y);
    const int c[3] = {t.x, t.y, t.z};
    double wv[3] = {1.0, 1.0, 1.0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) wv[a] = Axis(g, a).w(c[a]);
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
            const double dq = q[soff + nb.at(a == 0, a == 1, a == 2)] - q[soff + c0];
            const double cross = a == 0 ? wv[1] * wv[2] : (a == 1 ? wv[0] * wv[2] : wv[0] * wv[1]);
            acc += T(double(un[k]) - cross * dq);
        }
        if (mode >= 2) acc += out[a];
        if (u0bar) u0bar[k] = acc;
        if (ubar_out) ubar_out[k] = out[a];
    }
}

// D^T: ubar^a[J] = rbar[J] / w^a_{J_a} - rbar[J + e_a] / w^a_{J_a + 1}; 0 on the upper-wall face.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_gen_div_vjp(Grid g, const double* __restrict__ rbar, T* __restrict__ ubar) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const double* rb = rbar + int64_t(t.b) * g.ncell;
    T* ob = ubar + int64_t(t.b) * DIM * g.ncell;
    const int c0 = nb.at(0, 0, 0);
    const double rc = rb[c0];
    const bool wall = upper_wall(g, t.y);
    const int c[3] = {t.x, t.y, t.z};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const Axis A(g, a);
        const double rp = rb[nb.at(a == 0, a == 1, a == 2)];
        ob[a * g.ncell + c0] = (a == 1 && wall) ? T(0) : T(rc * A.iw(c[a]) - rp * A.iw(c[a] + 1));
    }
}

// G^T: pbar[I] = sum_a (gbar^a[I - e_a] / d^a_{I_a - 1} - gbar^a[I] / d^a_{I_a}) over the faces that exist.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_gen_grad_vjp(Grid g, const T* __restrict__ gbar, double* __restrict__ pbar) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const T* gb = gbar + int64_t(t.b) * DIM * g.ncell;
    const int c0 = nb.at(0, 0, 0);
    const int c[3] = {t.x, t.y, t.z};
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const Axis A(g, a);
        const double gc = double(gb[a * g.ncell + c0]);
        const double gm = double(gb[a * g.ncell + nb.at(-(a == 0), -(a == 1), -(a == 2))]);
        const bool lo_ok = !(a == 1 && g.ywalls && t.y == 0);
        const bool hi_ok = !(a == 1 && g.ywalls && t.y == g.ny - 1);
        if (lo_ok) acc += gm * A.id(c[a] - 1);
        if (hi_ok) acc -= gc * A.id(c[a]);
    }
    pbar[int64_t(t.b) * g.ncell + c0] = acc;
}

// ----------------------------------------------------------------------------
// Conjugate gradients on A = -Omega_p D G (same work split, partial sums and
// scalar protocol as the channel's kernels; one thread per cell in 2D and 3D)
// ----------------------------------------------------------------------------

__device__ __forceinline__ double cell_volume(const Grid& g, int x, int y, int z) {
    double v = Axis(g, 0).w(x) * Axis(g, 1).w(y);
    if (g.dim == 3) v *= Axis(g, 2).w(z);
    return v;
}

// q = A p at one cell (p formed as r + beta p_old at every point it reads).
template <bool FIRST>
__device__ __forceinline__ double gen_ap(const Grid& g, const double* rb, const double* pb, double beta, int x, int y,
                                         int z, double pc) {
    const Axis X(g, 0), Yx(g, 1);
    const double wx = X.w(x), wy = Yx.w(y);
    double wz = 1.0;
    if (g.dim == 3) wz = Axis(g, 2).w(z);
    const int64_t plane = int64_t(g.nx) * g.ny;
    const int64_t c0 = int64_t(z) * plane + int64_t(y) * g.nx + x;
    const int64_t row = c0 - x;
    const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
    double ap = wy * wz *
                ((pc - cg_dir<FIRST>(rb, pb, row + xp, beta)) * X.id(x) +
                 (pc - cg_dir<FIRST>(rb, pb, row + xm, beta)) * X.id(x - 1));
    const int64_t cy0 = c0 - int64_t(y) * g.nx;
    if (!g.ywalls || y < g.ny - 1) {
        const int yp = y == g.ny - 1 ? 0 : y + 1;
        ap += wx * wz * (pc - cg_dir<FIRST>(rb, pb, cy0 + int64_t(yp) * g.nx, beta)) * Yx.id(y);
    }
    if (!g.ywalls || y > 0) {
        const int ym = y == 0 ? g.ny - 1 : y - 1;
        ap += wx * wz * (pc - cg_dir<FIRST>(rb, pb, cy0 + int64_t(ym) * g.nx, beta)) * Yx.id(y - 1);
    }
    if (g.dim == 3) {
        const Axis Z(g, 2);
        const int64_t cz0 = c0 - int64_t(z) * plane;
        const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
        ap += wx * wy *
              ((pc - cg_dir<FIRST>(rb, pb, cz0 + int64_t(zp) * plane, beta)) * Z.id(z) +
               (pc - cg_dir<FIRST>(rb, pb, cz0 + int64_t(zm) * plane, beta)) * Z.id(z - 1));
    }
    return ap;
}

// Right-hand side. mode 0: r = D vel; 1: r = D Omega_u^{-1} vel; 2, 3: r = rin.
// Partial sums of Omega_p r (modes 0-2) or of r (mode 3).
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_gen_cg_div(Grid g, const T* __restrict__ vel, const double* __restrict__ rin,
                                                        double* __restrict__ r, double* __restrict__ msum, int mode) {
    __shared__ double sh[kBlock / 64];
    const CgSplit c = cg_split(g);
    double acc = 0.0;
    for (int t = c.t0; t < c.t1; ++t) {
        int x, y, z;
        if (!cg_cell(g, t, x, y, z)) continue;
        const Nb nb = make_nb<DIM>(g, x, y, z);
        const int64_t k = cg_index(g, c.b, x, y, z);
        double v;
        if (mode == 0)
            v = gen_div_cell<T, DIM, false>(g, vel + int64_t(c.b) * DIM * g.ncell, nb, x, y, z);
        else if (mode == 1)
            v = gen_div_cell<T, DIM, true>(g, vel + int64_t(c.b) * DIM * g.ncell, nb, x, y, z);
        else
            v = rin[k];
        r[k] = v;
        acc += mode == 3 ? v : cell_volume(g, x, y, z) * v;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) msum[c.slot()] = s;
}

// b = Omega_p (mean_w - r) (modes 0-2) or mean - r (mode 3), stored in r;
// x = 0; partial sums of b.b.
__global__ __launch_bounds__(kBlock) void k_gen_cg_init(Grid g, double* __restrict__ r, double* __restrict__ x,
                                                         const double* __restrict__ msum, double* __restrict__ rb0,
                                                         CgScal* st, int mode, double wsum) {
    __shared__ double sh[kBlock / 64];
    const CgSplit c = cg_split(g);
    const double mean = field_total(msum, c, sh) / (mode == 3 ? double(g.ncell) : wsum);
    double acc = 0.0;
    for (int t = c.t0; t < c.t1; ++t) {
        int cx, cy, cz;
        if (!cg_cell(g, t, cx, cy, cz)) continue;
        const int64_t k = cg_index(g, c.b, cx, cy, cz);
        const double v = mode == 3 ? mean - r[k] : cell_volume(g, cx, cy, cz) * (mean - r[k]);
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

template <bool FIRST>
__device__ __forceinline__ double gen_apply_run(const Grid& g, const CgSplit& c, const double* rb, const double* pb,
                                                double* pout, double* x, double beta, double am) {
    double acc = 0.0;
    for (int t = c.t0; t < c.t1; ++t) {
        int cx, cy, cz;
        if (!cg_cell(g, t, cx, cy, cz)) continue;
        const int64_t c0 = (int64_t(cz) * g.ny + cy) * g.nx + cx;
        const double pc = cg_dir<FIRST>(rb, pb, c0, beta);
        if (!FIRST && am != 0.0) x[c0] += am * pb[c0];
        const double ap = gen_ap<FIRST>(g, rb, pb, beta, cx, cy, cz, pc);
        pout[c0] = pc;
        acc += pc * ap;
    }
    return acc;
}

// Iteration k (the protocol of the channel's apply kernel): stop test from
// rr_k; the pending x += alpha_{k-1} p_{k-1}; unless stopped p = r + beta
// p_old at every stencil point, stored, and partial sums of p.(A p).
__global__ __launch_bounds__(kBlock) void k_gen_cg_apply(Grid g, const double* __restrict__ r,
                                                          const double* __restrict__ pin, double* __restrict__ pout,
                                                          double* __restrict__ x, const double* __restrict__ rbk,
                                                          const double* __restrict__ rbm,
                                                          const double* __restrict__ pqm, double* __restrict__ pqs,
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
    double rrm = 0.0, am = 0.0;
    if (k > 0) {
        rrm = field_total(rbm, c, sh);
        am = cg_pending(rrm, field_total(pqm, c, sh), rr0, k, rtol2, maxiter);
    }
    const int64_t soff = int64_t(c.b) * g.ncell;
    if (stop) {
        if (am != 0.0) {
            for (int t = c.t0; t < c.t1; ++t) {
                int cx, cy, cz;
                if (!cg_cell(g, t, cx, cy, cz)) continue;
                const int64_t i = cg_index(g, c.b, cx, cy, cz);
                x[i] += am * pin[i];
            }
        }
        return;
    }
    double acc;
    if (k == 0)
        acc = gen_apply_run<true>(g, c, r + soff, pin + soff, pout + soff, x + soff, 0.0, 0.0);
    else
        acc = gen_apply_run<false>(g, c, r + soff, pin + soff, pout + soff, x + soff, rrk / rrm, am);
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) pqs[c.slot()] = s;
}

// Iteration k, unless stopped: alpha = rr_k / p.q, r -= alpha A p (A p
// recomputed from the stored p with the apply kernel's arithmetic), partial
// sums of r.r; a stopped field copies its partials forward, a breakdown
// (p.q <= 0) writes 0.
__global__ __launch_bounds__(kBlock) void k_gen_cg_update(Grid g, double* __restrict__ r, const double* __restrict__ p,
                                                           const double* __restrict__ rbk,
                                                           const double* __restrict__ pqs, double* __restrict__ rbn,
                                                           CgScal* st, int k, double rtol2, int maxiter) {
    __shared__ double sh[kBlock / 64];
    const CgSplit c = cg_split(g);
    const double rrk = field_total(rbk, c, sh);
    if (cg_stopped(rrk, st[c.b].rr0, k, rtol2, maxiter)) {
        if (threadIdx.x == 0) rbn[c.slot()] = rbk[c.slot()];
        return;
    }
    const double pq = field_total(pqs, c, sh);
    if (!(pq > 0.0)) {
        if (threadIdx.x == 0) rbn[c.slot()] = 0.0;
        return;
    }
    const double alpha = rrk / pq;
    const int64_t soff = int64_t(c.b) * g.ncell;
    const double* pf = p + soff;
    double* rf = r + soff;
    double acc = 0.0;
    for (int t = c.t0; t < c.t1; ++t) {
        int cx, cy, cz;
        if (!cg_cell(g, t, cx, cy, cz)) continue;
        const int64_t c0 = (int64_t(cz) * g.ny + cy) * g.nx + cx;
        const double ap = gen_ap<true>(g, pf, nullptr, 0.0, cx, cy, cz, pf[c0]);
        const double v = rf[c0] - alpha * ap;
        rf[c0] = v;
        acc += v * v;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        rbn[c.slot()] = s;
        if (c.blk == 0) st[c.b].it = k + 1;
    }
}

// Partial sums of Omega_p t, then t = Omega_p (t - mean_w(t)) in place (the
// output side of the solve's pullback).
__global__ __launch_bounds__(kBlock) void k_gen_cg_wsum(Grid g, const double* __restrict__ t, double* __restrict__ msum) {
    __shared__ double sh[kBlock / 64];
    const CgSplit c = cg_split(g);
    double acc = 0.0;
    for (int tt = c.t0; tt < c.t1; ++tt) {
        int x, y, z;
        if (!cg_cell(g, tt, x, y, z)) continue;
        acc += cell_volume(g, x, y, z) * t[cg_index(g, c.b, x, y, z)];
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) msum[c.slot()] = s;
}

__global__ __launch_bounds__(kBlock) void k_gen_cg_post(Grid g, double* __restrict__ t, const double* __restrict__ msum,
                                                         double wsum) {
    __shared__ double sh[kBlock / 64];
    const CgSplit c = cg_split(g);
    const double mean = field_total(msum, c, sh) / wsum;
    for (int tt = c.t0; tt < c.t1; ++tt) {
        int x, y, z;
        if (!cg_cell(g, tt, x, y, z)) continue;
        const int64_t k = cg_index(g, c.b, x, y, z);
        t[k] = cell_volume(g, x, y, z) * (t[k] - mean);
    }
}

}  // namespace

// ----------------------------------------------------------------------------
// Launchers
// ----------------------------------------------------------------------------
#define INS_GEN_DIM(g, KER, ...)                                                              \
    do {                                                                                      \
        const int nblk = stencil_blocks(g);                                                   \
        if ((g).dim == 3)                                                                     \
            hipLaunchKernelGGL((KER<T, 3>), dim3(nblk), dim3(kBlock), 0, s, __VA_ARGS__);     \
        else                                                                                  \
            hipLaunchKernelGGL((KER<T, 2>), dim3(nblk), dim3(kBlock), 0, s, __VA_ARGS__);     \
    } while (0)

template <typename T>
hipError_t launch_gen_rhs(const Grid& g, const T* u, T* f, hipStream_t s) {
    INS_GEN_DIM(g, k_gen_rhs, g, u, f);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gen_divergence(const Grid& g, const T* u, double* r, hipStream_t s) {
    INS_GEN_DIM(g, k_gen_divergence, g, u, r);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gen_gradient(const Grid& g, const double* p, T* out, hipStream_t s) {
    INS_GEN_DIM(g, k_gen_gradient, g, p, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gen_rhs_vjp(const Grid& g, const T* u, const T* fbar, T* ubar, hipStream_t s) {
    INS_GEN_DIM(g, k_gen_rhs_vjp, g, u, fbar, ubar);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gen_div_vjp(const Grid& g, const double* rbar, T* ubar, hipStream_t s) {
    INS_GEN_DIM(g, k_gen_div_vjp, g, rbar, ubar);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gen_grad_vjp(const Grid& g, const T* gbar, double* pbar, hipStream_t s) {
    INS_GEN_DIM(g, k_gen_grad_vjp, g, gbar, pbar);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gen_project(const Grid& g, const T* w, const double* p, T* u_out, bool adj, hipStream_t s) {
    const int nblk = stencil_blocks(g);
    if (g.dim == 3) {
        if (adj)
            hipLaunchKernelGGL((k_gen_project<T, 3, true>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, u_out);
        else
            hipLaunchKernelGGL((k_gen_project<T, 3, false>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, u_out);
    } else {
        if (adj)
            hipLaunchKernelGGL((k_gen_project<T, 2, true>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, u_out);
        else
            hipLaunchKernelGGL((k_gen_project<T, 2, false>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, u_out);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gen_stage(const Grid& g, const T* w, const double* p, bool proj, const T* u0, T* y, bool yinit,
                            double cy, T* wout, double cw, hipStream_t s) {
    const int nblk = stencil_blocks(g);
    const int yi = yinit ? 1 : 0;
#define INS_GEN_STAGE(D, P)                                                                                       \
    hipLaunchKernelGGL((k_gen_stage<T, D, P>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, u0, y, yi, T(cy), wout, \
                       T(cw))
    if (g.dim == 3) {
        if (proj)
            INS_GEN_STAGE(3, true);
        else
            INS_GEN_STAGE(3, false);
    } else {
        if (proj)
            INS_GEN_STAGE(2, true);
        else
            INS_GEN_STAGE(2, false);
    }
#undef INS_GEN_STAGE
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gen_stage_vjp(const Grid& g, const T* w, const double* p, bool proj_u, const T* ybar, const T* un,
                                const double* q, bool has_w, double cb, double cw, T* u0bar, int mode, T* out,
                                hipStream_t s) {
    const int nblk = stencil_blocks(g);
#define INS_GEN_SVJP(D, PU, HW)                                                                                  \
    hipLaunchKernelGGL((k_gen_stage_vjp<T, D, PU, HW>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, ybar, un, q,  \
                       T(cb), T(cw), u0bar, mode, out)
#define INS_GEN_SVJP_D(D)              \
    do {                               \
        if (proj_u) {                  \
            if (has_w)                 \
                INS_GEN_SVJP(D, true, true);  \
            else                       \
                INS_GEN_SVJP(D, true, false); \
        } else {                       \
            if (has_w)                 \
                INS_GEN_SVJP(D, false, true); \
            else                       \
                INS_GEN_SVJP(D, false, false); \
        }                              \
    } while (0)
    if (g.dim == 3)
        INS_GEN_SVJP_D(3);
    else
        INS_GEN_SVJP_D(2);
#undef INS_GEN_SVJP_D
#undef INS_GEN_SVJP
    return hipGetLastError();
}

#define INS_GEN_INST(T)                                                                                             \
    template hipError_t launch_gen_rhs<T>(const Grid&, const T*, T*, hipStream_t);                                  \
    template hipError_t launch_gen_divergence<T>(const Grid&, const T*, double*, hipStream_t);                      \
    template hipError_t launch_gen_gradient<T>(const Grid&, const double*, T*, hipStream_t);                        \
    template hipError_t launch_gen_rhs_vjp<T>(const Grid&, const T*, const T*, T*, hipStream_t);                    \
    template hipError_t launch_gen_div_vjp<T>(const Grid&, const double*, T*, hipStream_t);                         \
    template hipError_t launch_gen_grad_vjp<T>(const Grid&, const T*, double*, hipStream_t);                        \
    template hipError_t launch_gen_project<T>(const Grid&, const T*, const double*, T*, bool, hipStream_t);         \
    template hipError_t launch_gen_stage<T>(const Grid&, const T*, const double*, bool, const T*, T*, bool, double, \
                                            T*, double, hipStream_t);                                               \
    template hipError_t launch_gen_stage_vjp<T>(const Grid&, const T*, const double*, bool, const T*, const T*,     \
                                                const double*, bool, double, double, T*, int, T*, hipStream_t);
INS_GEN_INST(double)
INS_GEN_INST(float)
#undef INS_GEN_INST

template <typename T>
hipError_t launch_gen_cg_div(const Grid& g, const T* vel, const double* rin, double* r, double* msum, int mode,
                             hipStream_t s) {
    const int nblk = cg_blocks_of(g) * g.batch;
    if (g.dim == 3)
        hipLaunchKernelGGL((k_gen_cg_div<T, 3>), dim3(nblk), dim3(kBlock), 0, s, g, vel, rin, r, msum, mode);
    else
        hipLaunchKernelGGL((k_gen_cg_div<T, 2>), dim3(nblk), dim3(kBlock), 0, s, g, vel, rin, r, msum, mode);
    return hipGetLastError();
}
template hipError_t launch_gen_cg_div<double>(const Grid&, const double*, const double*, double*, double*, int,
                                              hipStream_t);
template hipError_t launch_gen_cg_div<float>(const Grid&, const float*, const double*, double*, double*, int,
                                             hipStream_t);

hipError_t launch_gen_cg_init(const Grid& g, double* r, double* x, const double* msum, double* rb0, CgScal* st,
                              int mode, double wsum, hipStream_t s) {
    hipLaunchKernelGGL(k_gen_cg_init, dim3(cg_blocks_of(g) * g.batch), dim3(kBlock), 0, s, g, r, x, msum, rb0, st,
                       mode, wsum);
    return hipGetLastError();
}

hipError_t launch_gen_cg_apply(const Grid& g, const double* r, const double* pin, double* pout, double* x,
                               const double* rbk, const double* rbm, const double* pqm, double* pqs, CgScal* st, int k,
                               double rtol2, int maxiter, hipStream_t s) {
    hipLaunchKernelGGL(k_gen_cg_apply, dim3(cg_blocks_of(g) * g.batch), dim3(kBlock), 0, s, g, r, pin, pout, x, rbk,
                       rbm, pqm, pqs, st, k, rtol2, maxiter);
    return hipGetLastError();
}

hipError_t launch_gen_cg_update(const Grid& g, double* r, const double* p, const double* rbk, const double* pqs,
                                double* rbn, CgScal* st, int k, double rtol2, int maxiter, hipStream_t s) {
    hipLaunchKernelGGL(k_gen_cg_update, dim3(cg_blocks_of(g) * g.batch), dim3(kBlock), 0, s, g, r, p, rbk, pqs, rbn,
                       st, k, rtol2, maxiter);
    return hipGetLastError();
}

hipError_t launch_gen_cg_weighted_center(const Grid& g, double* t, double* msum, double wsum, hipStream_t s) {
    const int nblk = cg_blocks_of(g) * g.batch;
    hipLaunchKernelGGL(k_gen_cg_wsum, dim3(nblk), dim3(kBlock), 0, s, g, t, msum);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gen_cg_post, dim3(nblk), dim3(kBlock), 0, s, g, t, msum, wsum);
    return hipGetLastError();
}

}  // namespace ins
