// Kernels of the channel grid: no-slip walls at both ends of y, x and z
// periodic and uniform, y uniform or stretched (Sec. 2.4 boundary conditions
// through ghost volumes and non-uniform grids; App. B kernels with
// non-uniform widths), and the matrix-free conjugate-gradient pressure solve
// (Sec. 2.6.1, iterative solver).
//
// Wall rules, applied where a stencil reads a neighbour:
//  * u^y on the face on top of the last cell row (row N_y - 1) is the upper
//    wall and the face below row 0 the lower one: both read as 0, and every
//    output writes 0 on the stored wall face;
//  * a tangential component one row beyond a wall is minus the first
//    interior value (zero interpolant on the wall; the ghost row mirrors the
//    first/last row, widths included);
//  * the pressure gradient exists on interior y-faces only, so D G is the
//    Neumann Laplacian.
// y metrics (Grid::ym, filled by the runtime): w_j the width of row j, d_j the
// distance of the centres around y-face j (d_{-1} = w_0, d_{N_y-1} = w_{N_y-1}),
// theta_j = w_j / (w_j + w_{j+1}). Convection: the transported component is
// averaged with weights 1/2, the transporting one interpolated as the
// mass-flux average of the pressure-volume faces it spans (theta on a
// stretched y, 1/2 otherwise), which keeps convection energy-conserving.
// The pullback stencils are written in gather form from the same flux
// definitions; the sources below apply the wall rules to both the primal
// field and the cotangent, which is exact because every convective wall flux
// vanishes identically and the mirrored ghost makes the diffusion transpose
// the printed one.
//
// CG (fp64 throughout) on the symmetric A = -Omega_p D G (the pressure-volume
// scaling, a factor w_j per row, makes it symmetric), from x_0 = 0. One
// iteration is two fused kernels:
//   k_cg_apply:  x += alpha_old p_old (the previous iteration's update, folded
//                in here since p_old is read anyway), p = r + beta p_old
//                (formed at the stencil points), partial sums of p.(A p)
//   k_cg_update: alpha = rr / p.(A p); r -= alpha A p with A p recomputed from
//                the stored p, partial sums of r.r
// (8 field sweeps per iteration: apply reads r, p_old, x and writes p, x;
// update reads r, p and writes r; A p is never stored.)
// Every scalar (rr, beta, alpha, the stop test) is recomputed in every
// workgroup from partial sums, so iterations run back to back without the
// host and results are bitwise reproducible. A stopped field skips the work
// of later iterations.
#include "k_cg.hpp"
#include "k_common.hpp"

namespace ins {

// Per-row y metrics, indices clamped to the ghost conventions above.
struct YMetric {
    const double* m;
    int ny, S;
    __device__ __forceinline__ explicit YMetric(const Grid& g) : m(g.ym), ny(g.ny), S(g.ny + 2) {}
    __device__ __forceinline__ int rc(int r) const { return r < 0 ? 0 : (r > ny - 1 ? ny - 1 : r); }
    __device__ __forceinline__ int rf(int r) const { return r < -1 ? -1 : (r > ny - 1 ? ny - 1 : r); }
    __device__ __forceinline__ double iw(int r) const { return m[rc(r)]; }
    __device__ __forceinline__ double id(int r) const { return m[S + rf(r) + 1]; }
    __device__ __forceinline__ double th(int r) const { return (r >= 0 && r < ny) ? m[2 * S + r] : 0.5; }
    __device__ __forceinline__ double w(int r) const { return m[3 * S + rc(r)]; }
    __device__ __forceinline__ double d(int r) const { return m[4 * S + rf(r) + 1]; }
};

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
    double ih0, ih2;
    WallRows rows;
    YMetric M;
    int y;
    __device__ __forceinline__ T operator()(int c, const Nb& nb, int dx, int dy, int dz) const {
        const int k = dy + 1;
        const int j = nb.at(dx, dy, dz);
        if (c == 1) {
            if (!rows.unk[k]) return T(0);
            if constexpr (!PROJ) {
                return w[ncell + j];
            } else {
                return T(double(w[ncell + j]) - (p[nb.at(dx, dy + 1, dz)] - p[j]) * M.id(y + dy));
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

// Stage cotangent Fbar = cb ybar + (HAS_W ? cw (un - Omega_u G q) : 0) with the
// same rules; un - Omega_u G q is the transposed projection P^T = Omega_u P
// Omega_u^{-1} of the next stage's cotangent (q solved from D Omega_u^{-1} un).
template <typename T, bool HAS_W>
struct WallFbar {
    const T* __restrict__ ybar;
    const T* __restrict__ un;
    const double* __restrict__ q;
    T cb, cw;
    int ncell;
    double ih0, ih2;
    WallRows rows;
    YMetric M;
    int y;
    __device__ __forceinline__ T operator()(int c, const Nb& nb, int dx, int dy, int dz) const {
        const int k = dy + 1;
        if (c == 1 && !rows.unk[k]) return T(0);
        const int j = nb.at(dx, dy, dz);
        T v = cb * ybar[c * ncell + j];
        if constexpr (HAS_W) {
            const int jp = nb.at(dx + (c == 0), dy + (c == 1), dz + (c == 2));
            const double og = c == 1 ? (q[jp] - q[j]) : M.w(y + dy) * (q[jp] - q[j]) * (c == 0 ? ih0 : ih2);
            v += cw * T(double(un[c * ncell + j]) - og);
        }
        return (c != 1 && rows.ghost[k]) ? -v : v;
    }
};

// y metrics of the rows y-1, y, y+1 that the stencils of a cell of row y read
// (clamped as YMetric), loaded once per thread.
struct RowM {
    double iw[3], id[3], th, thm;
    __device__ __forceinline__ RowM(const Grid& g, int y) {
        const YMetric M(g);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            iw[k] = M.iw(y + k - 1);
            id[k] = M.id(y + k - 1);
        }
        th = M.th(y);
        thm = M.th(y - 1);
    }
};

// F^a at the current cell (row y, metrics R): diffusion (eq. diff-kernel),
// convection (eq. conv-kernel with the weights described above) and the constant
// body force on the channel grid. The pullback below has no force term: a
// constant has no Jacobian.
template <typename T, int DIM, class Src>
__device__ __forceinline__ void rhs_cell_wall(const Grid& g, const Src& U, const Nb& nb, const RowM& R, T F[DIM]) {
    const T iwj = T(R.iw[1]), iwp = T(R.iw[2]), idj = T(R.id[1]), idm = T(R.id[0]), th = T(R.th);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int ax = a == 0, ay = a == 1, az = a == 2;
        const T uc = U(a, nb, 0, 0, 0);
        T diff = T(0), conv = T(0);
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            const int bx = b == 0, by = b == 1, bz = b == 2;
            const T up = U(a, nb, bx, by, bz);
            const T um = U(a, nb, -bx, -by, -bz);
            if (b != 1)
                diff += ((up - uc) - (uc - um)) * T(g.ih2[b]);
            else if (a != 1)
                diff += ((up - uc) * idj - (uc - um) * idm) * iwj;
            else
                diff += ((up - uc) * iwp - (uc - um) * iwj) * idj;
            T vr, vl;
            if (a == 1 && b != 1) {
                vr = th * U(b, nb, 0, 0, 0) + (T(1) - th) * U(b, nb, 0, 1, 0);
                vl = th * U(b, nb, -bx, 0, -bz) + (T(1) - th) * U(b, nb, -bx, 1, -bz);
            } else {
                vr = T(0.5) * (U(b, nb, 0, 0, 0) + U(b, nb, ax, ay, az));
                vl = T(0.5) * (U(b, nb, -bx, -by, -bz) + U(b, nb, ax - bx, ay - by, az - bz));
            }
            const T fr = T(0.5) * (uc + up) * vr;
            const T fl = T(0.5) * (um + uc) * vl;
            const T s = b != 1 ? T(g.ih[b]) : (a == 1 ? idj : iwj);
            conv -= (fr - fl) * s;
        }
        F[a] = conv + T(g.nu) * diff + T(g.force[a]);
    }
}

// 1 / |Delta^b| of the a-velocity volume whose point lies on row y + dr (dr in -1..1).
template <typename T>
__device__ __forceinline__ T conv_s(const Grid& g, const RowM& R, int a, int b, int dr) {
    return b != 1 ? T(g.ih[b]) : T(a == 1 ? R.id[dr + 1] : R.iw[dr + 1]);
}

// Pullback of the right-hand side at one cell (row y), gather form: the
// diffusion transpose (eq. diff-pullback) plus, for each flux
// F^{ab}[K] = A^{ab}[K] B^{ab}[K] containing u^g[J], its other factor times
// Fbar^{ab}[K] = -fbar^a[K] s(K) + fbar^a[K + e_b] s(K + e_b), with the
// interpolation weight of u^g[J] in its own factor.
template <typename T, int DIM, class USrc, class FSrc>
__device__ __forceinline__ void rhs_vjp_cell_wall(const Grid& g, const USrc& U, const FSrc& Fb, const Nb& nb,
                                                  const RowM& R, T out[DIM]) {
    const T thy = T(R.th), thm = T(R.thm);
#pragma unroll
    for (int gm = 0; gm < DIM; ++gm) {
        const int gx = gm == 0, gy = gm == 1, gz = gm == 2;
        const T fc = Fb(gm, nb, 0, 0, 0);
        T diff = T(0), acc = T(0);
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            const int bx = b == 0, by = b == 1, bz = b == 2;
            const T fp = Fb(gm, nb, bx, by, bz);
            const T fm = Fb(gm, nb, -bx, -by, -bz);
            if (b != 1) {
                diff += (fp - T(2) * fc + fm) * T(g.ih2[b]);
            } else if (gm != 1) {
                diff += fm * T(R.iw[0] * R.id[0]) - fc * T(R.iw[1] * (R.id[1] + R.id[0])) + fp * T(R.iw[2] * R.id[1]);
            } else {
                diff += fm * T(R.id[0] * R.iw[1]) - fc * T(R.id[1] * (R.iw[2] + R.iw[1])) + fp * T(R.id[2] * R.iw[2]);
            }
            // u^gm transported in F^{gm b} at K = J and K = J - e_b (weights 1/2)
            const T s0 = conv_s<T>(g, R, gm, b, 0);
            const T F0 = -fc * s0 + fp * conv_s<T>(g, R, gm, b, by);
            const T F1 = -fm * conv_s<T>(g, R, gm, b, -by) + fc * s0;
            T B0, B1;
            if (gm == 1 && b != 1) {
                B0 = thy * U(b, nb, 0, 0, 0) + (T(1) - thy) * U(b, nb, 0, 1, 0);
                B1 = thy * U(b, nb, -bx, 0, -bz) + (T(1) - thy) * U(b, nb, -bx, 1, -bz);
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
            const T F0 = -Fb(a, nb, 0, 0, 0) * conv_s<T>(g, R, a, gm, 0) +
                         Fb(a, nb, gx, gy, gz) * conv_s<T>(g, R, a, gm, gy);
            const T A0 = T(0.5) * (U(a, nb, 0, 0, 0) + U(a, nb, gx, gy, gz));
            const T F1 = -Fb(a, nb, -ax, -ay, -az) * conv_s<T>(g, R, a, gm, -ay) +
                         Fb(a, nb, gx - ax, gy - ay, gz - az) * conv_s<T>(g, R, a, gm, gy - ay);
            const T A1 = T(0.5) * (U(a, nb, -ax, -ay, -az) + U(a, nb, gx - ax, gy - ay, gz - az));
            T w0 = T(0.5), w1 = T(0.5);
            if (a == 1 && gm != 1) {
                w0 = thy;
                w1 = T(1) - thm;
            }
            acc += w0 * F0 * A0 + w1 * F1 * A1;
        }
        out[gm] = acc + T(g.nu) * diff;
    }
}

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
    WallVel<T, false> U{u + boff, nullptr, int(g.ncell), g.ih[0], g.ih[2], rows, YMetric(g), t.y};
    T F[DIM];
    rhs_cell_wall<T, DIM>(g, U, nb, RowM(g, t.y), F);
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
    WallVel<T, PROJ> U{w + boff, PROJ ? p + int64_t(t.b) * g.ncell : nullptr, int(g.ncell), g.ih[0], g.ih[2],
                       rows, YMetric(g), t.y};
    T F[DIM];
    rhs_cell_wall<T, DIM>(g, U, nb, RowM(g, t.y), F);
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

// 3D stage as a 2.5D z-march (same contract and arithmetic as k_wall_stage):
// a workgroup owns a TX x TY tile of an x-y plane and a chunk of z planes; each
// plane's stage velocity (w - G p with the wall rules: u^y 0 off the interior
// faces, tangential ghosts beyond a wall minus the mirrored row) is formed once
// on the tile plus a one-cell halo into a 4-plane LDS ring, and the stencil of
// plane z reads planes z-1, z, z+1 from there.
template <typename T, int TX, int TY>
struct WallLds {
    static constexpr int HX = TX + 2, HP = HX * (TY + 2);
    const T* zm;
    const T* z0;
    const T* zp;
    int centre;
    __device__ __forceinline__ T operator()(int c, const Nb&, int dx, int dy, int dz) const {
        const T* b = dz < 0 ? zm : (dz > 0 ? zp : z0);
        return b[c * HP + centre + dy * HX + dx];
    }
};

// Every global load of the plane loop is issued unconditionally (halo slots
// past the halo load a valid position and are not parked; a ghost row's
// interior-face loads read the clamped row and are zeroed when parked; the
// last iteration fetches its own last plane again; pointwise cells and planes
// are clamped; the pointwise streams are fixed per instance: PT bit 0 u0,
// bit 1 y), and the halo values are combined only when a plane is parked: the
// compiler's wait counts are then exact, so a plane's compute does not wait
// for the next plane's loads (with a load behind a condition it waited for
// every load in flight; 256^3 channel step 3.36 -> 3.23 ms, float32 3.00 ->
// 2.54 ms). The float32 instance is no longer held to 64 registers (8 waves
// per SIMD): with its loads in flight it spilled 80-96 bytes there and ran
// at the old speed; uncapped it takes 84-88 registers (5 waves).
template <typename T, bool PROJ, int TX, int TY, int PT>
__global__ __launch_bounds__(TX * TY) void k_wall_stage_zm(Grid g, const T* __restrict__ w,
                                                             const double* __restrict__ p, const T* __restrict__ u0,
                                                             T* __restrict__ y, int yinit, T cy, T* __restrict__ wout,
                                                             T cw, int zc) {
    constexpr int NT = TX * TY, HX = TX + 2, HP = HX * (TY + 2);
    constexpr int NS = (HP + NT - 1) / NT;
    __shared__ T ring[4][3][HP];
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY, nzc = (nz + zc - 1) / zc;
    int L = xcd_logical(blockIdx.x, gridDim.x);
    const int tx = L % ntx;
    L /= ntx;
    const int ty = L % nty;
    L /= nty;
    const int zci = L % nzc;
    const int b = L / nzc;
    const int x0 = tx * TX, y0 = ty * TY, z0 = zci * zc;
    const int z1 = min(z0 + zc, nz);
    const int64_t boff = int64_t(b) * 3 * g.ncell;
    const T* wb = w + boff;
    const double* pb = PROJ ? p + int64_t(b) * g.ncell : nullptr;
    const int nc = int(g.ncell);
    const int plane = nx * ny;
    const YMetric M(g);

    // halo positions of this thread: row offset of the (mirrored) row, x and
    // x + 1 (periodic), ghost / interior-face flags, 1 / d of the y-face
    int hq[NS], hrow[NS], hx[NS], hxp[NS];
    bool hghost[NS], hunk[NS];
    double hid[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int q = threadIdx.x + s * NT;
        hq[s] = q;
        const int qq = q < HP ? q : 0;
        const int gx = ((x0 - 1 + qq % HX) % nx + nx) % nx;  // the tile may be wider than n_x
        const int r = y0 - 1 + qq / HX;
        const int m = r < 0 ? 0 : (r > ny - 1 ? ny - 1 : r);
        hrow[s] = m * nx;
        hx[s] = gx;
        hxp[s] = gx + 1 == nx ? 0 : gx + 1;
        hghost[s] = r < 0 || r > ny - 1;
        hunk[s] = r >= 0 && r <= ny - 2;
        hid[s] = hunk[s] ? M.id(r) : 0.0;
    }
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int cxg = x0 + lx, cyg = y0 + ly;
    const bool valid = cxg < nx && cyg < ny;
    const bool wallrow = cyg == ny - 1;
    const int centre = (ly + 1) * HX + (lx + 1);
    const RowM rowm(g, valid ? cyg : 0);

    constexpr bool LB = (PT & 1) != 0, LY = (PT & 2) != 0;
    const int cxy = min(cyg, ny - 1) * nx + min(cxg, nx - 1);  // own cell, clamped for the loads
    // raw halo loads: w and (PROJ) p at the cell, its +x neighbour, the row
    // above (the cell itself when the row has no interior y-face) and +z
    T pw_[NS][3];
    double pp_[NS][4];
    auto fetch = [&](int zz) {
        const int zoff = zz * plane;
        const int zpo = (zz + 1 == nz ? 0 : zz + 1) * plane;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int j = zoff + hrow[s] + hx[s];
            pw_[s][0] = wb[j];
            pw_[s][1] = wb[nc + j];
            pw_[s][2] = wb[2 * nc + j];
            if constexpr (PROJ) {
                pp_[s][0] = pb[j];
                pp_[s][1] = pb[zoff + hrow[s] + hxp[s]];
                pp_[s][2] = pb[hunk[s] ? j + nx : j];
                pp_[s][3] = pb[zpo + hrow[s] + hx[s]];
            }
        }
    };
    auto park = [&](int k) {
        T* slot = &ring[k & 3][0][0];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (hq[s] < HP) {
                T v0 = pw_[s][0], v1 = pw_[s][1], v2 = pw_[s][2];
                if constexpr (PROJ) {
                    const double pc = pp_[s][0];
                    v0 = T(double(pw_[s][0]) - (pp_[s][1] - pc) * g.ih[0]);
                    v1 = T(double(pw_[s][1]) - (pp_[s][2] - pc) * hid[s]);
                    v2 = T(double(pw_[s][2]) - (pp_[s][3] - pc) * g.ih[2]);
                }
                slot[hq[s]] = hghost[s] ? -v0 : v0;
                slot[HP + hq[s]] = hunk[s] ? v1 : T(0);
                slot[2 * HP + hq[s]] = hghost[s] ? -v2 : v2;
            }
        }
    };
    // pointwise streams of the plane computed next: issued after the current
    // plane's stores, used at the next plane's stores
    T pbase[3] = {T(0), T(0), T(0)}, pyv[3] = {T(0), T(0), T(0)};
    auto fetch_point = [&](int z) {
        const int c0 = z * plane + cxy;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int64_t kk = boff + int64_t(a) * nc + c0;
            if constexpr (LB) pbase[a] = __builtin_nontemporal_load(u0 + kk);
            if constexpr (LY) pyv[a] = __builtin_nontemporal_load(y + kk);
        }
    };

    const int nk = (z1 - z0) + 2;
    fetch(wrap(z0 - 1, nz));
    park(0);
    fetch(z0);
    park(1);
    fetch(z0 + 1 == nz ? 0 : z0 + 1);
    park(2);
    fetch_point(z0);
    __syncthreads();
    for (int k = 2; k < nk; ++k) {
        const int z = z0 + k - 2;
        const int zn = z0 - 1 + min(k + 1, nk - 1);
        fetch(zn >= nz ? zn - nz : zn);
        WallLds<T, TX, TY> U{&ring[(k - 2) & 3][0][0], &ring[(k - 1) & 3][0][0], &ring[k & 3][0][0], centre};
        T F[3];
        rhs_cell_wall<T, 3>(g, U, Nb{}, rowm, F);
        if (valid) {
            const int c0 = z * plane + cyg * nx + cxg;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int64_t kk = boff + int64_t(a) * nc + c0;
                const bool zero = a == 1 && wallrow;
                const T base = LB ? pbase[a] : T(0);
                const T yv = LY ? pyv[a] : base;
                if (y) __builtin_nontemporal_store(zero ? T(0) : yv + cy * F[a], y + kk);
                if (wout) __builtin_nontemporal_store(zero ? T(0) : base + cw * F[a], wout + kk);
            }
        }
        fetch_point(min(z + 1, z1 - 1));
        if (k + 1 < nk) park(k + 1);
        __syncthreads();
    }
}

// u_out = w - G p (ADJ: w - Omega_u G p, the transposed projection's
// correction); float64 arithmetic; 0 on the wall face; u_out may alias w.
template <typename T, int DIM, bool ADJ>
__global__ __launch_bounds__(kBlock) void k_wall_project(Grid g, const T* w, const double* __restrict__ p, T* u_out) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const YMetric M(g);
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
        const double dp = pb[nb.at(a == 0, a == 1, a == 2)] - pc;
        double gp;
        if (a == 1)
            gp = ADJ ? dp : dp * M.id(t.y);
        else
            gp = dp * g.ih[a] * (ADJ ? M.w(t.y) : 1.0);
        u_out[k] = T(double(w[k]) - gp);
    }
}

// G p on the interior faces, 0 on the wall face.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_wall_gradient(Grid g, const double* __restrict__ p, T* __restrict__ out) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const YMetric M(g);
    const double* pb = p + int64_t(t.b) * g.ncell;
    T* ob = out + int64_t(t.b) * DIM * g.ncell;
    const int c0 = nb.at(0, 0, 0);
    const double pc = pb[c0];
    const bool wall = t.y == g.ny - 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double dp = pb[nb.at(a == 0, a == 1, a == 2)] - pc;
        ob[a * g.ncell + c0] = (a == 1 && wall) ? T(0) : T(dp * (a == 1 ? M.id(t.y) : g.ih[a]));
    }
}

// D u at one cell (row y) with both wall faces of u^y read as 0; SCALED reads
// Omega_u^{-1} u (u^y / d_j, tangential / w_j) instead of u.
template <typename T, int DIM, bool SCALED>
__device__ __forceinline__ double wall_div_cell(const Grid& g, const T* ub, const Nb& nb, int y) {
    const YMetric M(g);
    const int c0 = nb.at(0, 0, 0);
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double up = double(ub[a * g.ncell + c0]);
        double dn = double(ub[a * g.ncell + nb.at(-(a == 0), -(a == 1), -(a == 2))]);
        if (a == 1) {
            if (y == g.ny - 1) up = 0.0;
            if (y == 0) dn = 0.0;
            if constexpr (SCALED) {
                up /= M.d(y);
                dn /= M.d(y - 1);
            }
            acc += (up - dn) * M.iw(y);
        } else {
            acc += (up - dn) * g.ih[a] * (SCALED ? 1.0 / M.w(y) : 1.0);
        }
    }
    return acc;
}

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_wall_divergence(Grid g, const T* __restrict__ u, double* __restrict__ r) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    r[int64_t(t.b) * g.ncell + nb.at(0, 0, 0)] =
        wall_div_cell<T, DIM, false>(g, u + int64_t(t.b) * DIM * g.ncell, nb, t.y);
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
    const YMetric M(g);
    WallVel<T, false> U{u + boff, nullptr, nc, g.ih[0], g.ih[2], rows, M, t.y};
    WallFbar<T, false> F{fbar + boff, nullptr, nullptr, T(1), T(0), nc, g.ih[0], g.ih[2], rows, M, t.y};
    T out[DIM];
    rhs_vjp_cell_wall<T, DIM>(g, U, F, nb, RowM(g, t.y), out);
    const int c0 = nb.at(0, 0, 0);
    const bool wall = t.y == g.ny - 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) ubar[boff + a * g.ncell + c0] = (a == 1 && wall) ? T(0) : out[a];
}

// Reverse stage (same contract as k_stage_vjp, without the closure output;
// the projected cotangent of the next stage is un - Omega_u G q).
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
    const YMetric M(g);
    WallVel<T, PROJ_U> U{w + boff, PROJ_U ? p + soff : nullptr, nc, g.ih[0], g.ih[2], rows, M, t.y};
    WallFbar<T, HAS_W> F{ybar + boff, HAS_W ? un + boff : nullptr, HAS_W ? q + soff : nullptr, cb, cw, nc,
                         g.ih[0], g.ih[2], rows, M, t.y};
    T out[DIM];
    rhs_vjp_cell_wall<T, DIM>(g, U, F, nb, RowM(g, t.y), out);
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
            const double dq = q[soff + nb.at(a == 0, a == 1, a == 2)] - q[soff + c0];
            const double og = a == 1 ? dq : M.w(t.y) * dq * g.ih[a];
            acc += T(double(un[k]) - og);
        }
        if (mode >= 2) acc += out[a];
        if (u0bar) u0bar[k] = acc;
        if (ubar_out) ubar_out[k] = out[a];
    }
}

// 3D reverse stage as a z-march (same contract and arithmetic as
// k_wall_stage_vjp): two 3-slot LDS rings hold, per plane, the stage velocity
// (WallVel's values) and the right-hand-side cotangent (WallFbar's values) on
// a 32 x 8 tile plus halo; plane z's pullback stencil reads planes z-1, z, z+1.
constexpr int kWvTX = 32, kWvTY = 8;

template <typename T, bool PROJ_U, bool HAS_W>
__global__ __launch_bounds__(kBlock) void k_wall_stage_vjp_zm(Grid g, const T* __restrict__ w,
                                                                const double* __restrict__ p,
                                                                const T* __restrict__ ybar, const T* __restrict__ un,
                                                                const double* __restrict__ q, T cb, T cw,
                                                                T* __restrict__ u0bar, int mode,
                                                                T* __restrict__ ubar_out, int zc) {
    constexpr int TX = kWvTX, TY = kWvTY, HX = TX + 2, HP = HX * (TY + 2);
    constexpr int NS = (HP + kBlock - 1) / kBlock;
    __shared__ T ru[3][3][HP];
    __shared__ T rf[3][3][HP];
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY, nzc = (nz + zc - 1) / zc;
    int L = xcd_logical(blockIdx.x, gridDim.x);
    const int tx = L % ntx;
    L /= ntx;
    const int ty = L % nty;
    L /= nty;
    const int zci = L % nzc;
    const int b = L / nzc;
    const int x0 = tx * TX, y0 = ty * TY, z0 = zci * zc;
    const int z1 = min(z0 + zc, nz);
    const int64_t boff = int64_t(b) * 3 * g.ncell;
    const int64_t soff = int64_t(b) * g.ncell;
    const T* wb = w + boff;
    const double* pb = PROJ_U ? p + soff : nullptr;
    const T* yb = ybar + boff;
    const T* ub = HAS_W ? un + boff : nullptr;
    const double* qb = HAS_W ? q + soff : nullptr;
    const int nc = int(g.ncell);
    const int plane = nx * ny;
    const YMetric M(g);

    int hq[NS], hrow[NS], hx[NS], hxp[NS];
    bool hghost[NS], hunk[NS];
    double hid[NS], hw[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int qi = threadIdx.x + s * kBlock;
        hq[s] = qi;
        const int qq = qi < HP ? qi : 0;
        const int gx = ((x0 - 1 + qq % HX) % nx + nx) % nx;
        const int r = y0 - 1 + qq / HX;
        const int m = r < 0 ? 0 : (r > ny - 1 ? ny - 1 : r);
        hrow[s] = m * nx;
        hx[s] = gx;
        hxp[s] = gx + 1 == nx ? 0 : gx + 1;
        hghost[s] = r < 0 || r > ny - 1;
        hunk[s] = r >= 0 && r <= ny - 2;
        hid[s] = hunk[s] ? M.id(r) : 0.0;
        hw[s] = M.w(m);
    }
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int cxg = x0 + lx, cyg = y0 + ly;
    const bool valid = cxg < nx && cyg < ny;
    const bool wallrow = cyg == ny - 1;
    const int centre = (ly + 1) * HX + (lx + 1);
    const RowM rowm(g, valid ? cyg : 0);
    const double wrow = M.w(valid ? cyg : 0);

    // Raw halo loads (w, ybar and, with PROJ_U / HAS_W, p and un, q at the
    // cell and at its +x, +y (the cell itself when the row has no interior
    // y-face) and +z neighbours), combined into WallVel's and WallFbar's values
    // when the plane is parked. Every load of the plane loop is issued
    // unconditionally (slots past the halo load a valid position; the last
    // iteration fetches its own last plane again; pointwise cells, rows and
    // planes clamped), so the compiler's wait counts are exact and a plane's
    // compute does not wait for the next plane's loads. The instance already
    // runs 2 waves per SIMD, which the raw registers keep.
    const int cxy = min(cyg, ny - 1) * nx + min(cxg, nx - 1);
    T rw[NS][3], ry[NS][3], ru_[NS][3];
    double rp[NS][4], rq[NS][4];
    auto fetch = [&](int zz) {
        const int zoff = zz * plane;
        const int zpo = (zz + 1 == nz ? 0 : zz + 1) * plane;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int j = zoff + hrow[s] + hx[s];
            const int jp[3] = {zoff + hrow[s] + hxp[s], hunk[s] ? j + nx : j, zpo + hrow[s] + hx[s]};
            if constexpr (PROJ_U) rp[s][0] = pb[j];
            if constexpr (HAS_W) rq[s][0] = qb[j];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                rw[s][c] = wb[c * nc + j];
                ry[s][c] = yb[c * nc + j];
                if constexpr (PROJ_U) rp[s][c + 1] = pb[jp[c]];
                if constexpr (HAS_W) {
                    ru_[s][c] = ub[c * nc + j];
                    rq[s][c + 1] = qb[jp[c]];
                }
            }
        }
    };
    auto park = [&](int k) {
        T* su = &ru[k % 3][0][0];
        T* sf = &rf[k % 3][0][0];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (hq[s] < HP) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double gs = c == 1 ? hid[s] : g.ih[c];
                    T uv = rw[s][c];
                    if constexpr (PROJ_U) uv = T(double(rw[s][c]) - (rp[s][c + 1] - rp[s][0]) * gs);
                    T fv = cb * ry[s][c];
                    if constexpr (HAS_W) {
                        const double dq = rq[s][c + 1] - rq[s][0];
                        const double og = c == 1 ? dq : hw[s] * dq * g.ih[c];
                        fv += cw * T(double(ru_[s][c]) - og);
                    }
                    const bool neg = c != 1 && hghost[s];
                    const bool zero = c == 1 && !hunk[s];
                    su[c * HP + hq[s]] = zero ? T(0) : (neg ? -uv : uv);
                    sf[c * HP + hq[s]] = zero ? T(0) : (neg ? -fv : fv);
                }
            }
        }
    };
    // pointwise inputs of the plane computed next, issued after the current
    // plane's stores: the accumulated cotangent (ybar or u0bar) and, with
    // HAS_W, un and q at the cell and at its +x, +y (the cell itself on the
    // wall row, whose u^y outputs are 0) and +z neighbours
    const T* accb = (mode == 0 || mode == 3) ? yb : u0bar + boff;
    T nacc[3] = {T(0), T(0), T(0)}, nun[3] = {T(0), T(0), T(0)};
    double nq[3] = {0.0, 0.0, 0.0}, nqc = 0.0;
    auto fetch_point = [&](int z) {
        const int c0 = z * plane + cxy;
        const int cx = min(cxg, nx - 1), cy = min(cyg, ny - 1);
        const int jpc[3] = {z * plane + cy * nx + (cx + 1 == nx ? 0 : cx + 1), cy == ny - 1 ? c0 : c0 + nx,
                            (z + 1 == nz ? 0 : z + 1) * plane + cxy};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            nacc[a] = accb[int64_t(a) * nc + c0];
            if constexpr (HAS_W) {
                nun[a] = ub[int64_t(a) * nc + c0];
                nq[a] = qb[jpc[a]];
            }
        }
        if constexpr (HAS_W) nqc = qb[c0];
    };

    const int nk = (z1 - z0) + 2;
    fetch(z0 == 0 ? nz - 1 : z0 - 1);
    park(0);
    fetch(z0);
    park(1);
    fetch(z0 + 1 == nz ? 0 : z0 + 1);
    park(2);
    fetch_point(z0);
    __syncthreads();
    for (int k = 2; k < nk; ++k) {
        const int z = z0 + k - 2;
        const int zn = z0 - 1 + min(k + 1, nk - 1);
        fetch(zn >= nz ? zn - nz : zn);
        WallLds<T, TX, TY> U{&ru[(k - 2) % 3][0][0], &ru[(k - 1) % 3][0][0], &ru[k % 3][0][0], centre};
        WallLds<T, TX, TY> F{&rf[(k - 2) % 3][0][0], &rf[(k - 1) % 3][0][0], &rf[k % 3][0][0], centre};
        T out[3];
        rhs_vjp_cell_wall<T, 3>(g, U, F, Nb{}, rowm, out);
        if (valid) {
            const int c0 = z * plane + cyg * nx + cxg;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int64_t kk = boff + int64_t(a) * nc + c0;
                if (a == 1 && wallrow) {
                    if (u0bar) u0bar[kk] = T(0);
                    if (ubar_out) ubar_out[kk] = T(0);
                    continue;
                }
                T acc = nacc[a];
                if constexpr (HAS_W) {
                    const double dq = nq[a] - nqc;
                    const double og = a == 1 ? dq : wrow * dq * g.ih[a];
                    acc += T(double(nun[a]) - og);
                }
                if (mode >= 2) acc += out[a];
                if (u0bar) __builtin_nontemporal_store(acc, u0bar + kk);
                if (ubar_out) __builtin_nontemporal_store(out[a], ubar_out + kk);
            }
        }
        fetch_point(min(z + 1, z1 - 1));
        // slot (k+1) % 3 is the one just read as plane z-1: wait for every reader
        __syncthreads();
        if (k + 1 < nk) park(k + 1);
        __syncthreads();
    }
}

// D^T: ubar^a[J] = rbar[J] / |Delta^a_J| - rbar[J + e_a] / |Delta^a_{J+e_a}| (cell widths); 0 on the wall face.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_wall_div_vjp(Grid g, const double* __restrict__ rbar, T* __restrict__ ubar) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const YMetric M(g);
    const double* rb = rbar + int64_t(t.b) * g.ncell;
    T* ob = ubar + int64_t(t.b) * DIM * g.ncell;
    const int c0 = nb.at(0, 0, 0);
    const double rc = rb[c0];
    const bool wall = t.y == g.ny - 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double rp = rb[nb.at(a == 0, a == 1, a == 2)];
        double v;
        if (a == 1)
            v = wall ? 0.0 : rc * M.iw(t.y) - rp * M.iw(t.y + 1);
        else
            v = (rc - rp) * g.ih[a];
        ob[a * g.ncell + c0] = T(v);
    }
}

// G^T: pbar[I] = sum_a (gbar^a[I - e_a] s[I - e_a] - gbar^a[I] s[I]) over interior faces.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_wall_grad_vjp(Grid g, const T* __restrict__ gbar, double* __restrict__ pbar) {
    const TileIdx t = tile_of(g);
    if (!t.valid) return;
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const YMetric M(g);
    const T* gb = gbar + int64_t(t.b) * DIM * g.ncell;
    const int c0 = nb.at(0, 0, 0);
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double gc = double(gb[a * g.ncell + c0]);
        const double gm = double(gb[a * g.ncell + nb.at(-(a == 0), -(a == 1), -(a == 2))]);
        if (a == 1) {
            if (t.y > 0) acc += gm * M.id(t.y - 1);
            if (t.y < g.ny - 1) acc -= gc * M.id(t.y);
        } else {
            acc += (gm - gc) * g.ih[a];
        }
    }
    pbar[int64_t(t.b) * g.ncell + c0] = acc;
}

// Right-hand side of the solve. mode 0: r = D vel; 1: r = D Omega_u^{-1} vel
// (transposed projection); 2, 3: r = rin. Partial sums of w_j r (modes 0-2,
// for the volume-weighted mean) or of r (mode 3).
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_cg_div(Grid g, const T* __restrict__ vel, const double* __restrict__ rin,
                                                    double* __restrict__ r, double* __restrict__ msum, int mode) {
    __shared__ double sh[kBlock / 64];
    const CgSplit c = cg_split(g);
    const YMetric M(g);
    double acc = 0.0;
    for (int t = c.t0; t < c.t1; ++t) {
        int x, y, z;
        if (!cg_cell(g, t, x, y, z)) continue;
        const Nb nb = make_nb<DIM>(g, x, y, z);
        const int64_t k = cg_index(g, c.b, x, y, z);
        double v;
        if (mode == 0)
            v = wall_div_cell<T, DIM, false>(g, vel + int64_t(c.b) * DIM * g.ncell, nb, y);
        else if (mode == 1)
            v = wall_div_cell<T, DIM, true>(g, vel + int64_t(c.b) * DIM * g.ncell, nb, y);
        else
            v = rin[k];
        r[k] = v;
        acc += mode == 3 ? v : M.w(y) * v;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) msum[c.slot()] = s;
}

// b = w_j (mean_w - r) (modes 0-2; mean_w the volume-weighted mean, wsum the
// field's sum of w_j) or b = mean - r (mode 3), stored in r; x = 0; partial
// sums of b.b (rr_0).
__global__ __launch_bounds__(kBlock) void k_cg_init(Grid g, double* __restrict__ r, double* __restrict__ x,
                                                     const double* __restrict__ msum, double* __restrict__ rb0,
                                                     CgScal* st, int mode, double wsum) {
    __shared__ double sh[kBlock / 64];
    const CgSplit c = cg_split(g);
    const YMetric M(g);
    const double mean = field_total(msum, c, sh) / (mode == 3 ? double(g.ncell) : wsum);
    double acc = 0.0;
    for (int t = c.t0; t < c.t1; ++t) {
        int cx, cy, cz;
        if (!cg_cell(g, t, cx, cy, cz)) continue;
        const int64_t k = cg_index(g, c.b, cx, cy, cz);
        const double v = mode == 3 ? mean - r[k] : M.w(cy) * (mean - r[k]);
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

// 2D: q = A p at one cell of row y (no faces beyond the walls).
template <bool FIRST>
__device__ __forceinline__ double cg_ap2(const Grid& g, const YMetric& M, const double* rb, const double* pb,
                                         double beta, int64_t c0, int x, int y, double pc) {
    const int xm = x == 0 ? g.nx - 1 : x - 1;
    const int xp = x == g.nx - 1 ? 0 : x + 1;
    const int64_t row = c0 - x;
    double ap = (2.0 * pc - cg_dir<FIRST>(rb, pb, row + xm, beta) - cg_dir<FIRST>(rb, pb, row + xp, beta)) *
                g.ih2[0] * M.w(y);
    if (y > 0) ap += (pc - cg_dir<FIRST>(rb, pb, c0 - g.nx, beta)) * M.id(y - 1);
    if (y < g.ny - 1) ap += (pc - cg_dir<FIRST>(rb, pb, c0 + g.nx, beta)) * M.id(y);
    return ap;
}

template <bool FIRST>
__device__ __forceinline__ double cg_apply2_run(const Grid& g, const CgSplit& c, const double* rb, const double* pb,
                                                double* pout, double* x, double beta, double am) {
    const YMetric M(g);
    double acc = 0.0;
    for (int t = c.t0; t < c.t1; ++t) {
        int cx, y, z;
        if (!cg_cell(g, t, cx, y, z)) continue;
        const int64_t c0 = int64_t(y) * g.nx + cx;
        const double pc = cg_dir<FIRST>(rb, pb, c0, beta);
        if (!FIRST && am != 0.0) x[c0] += am * pb[c0];
        const double ap = cg_ap2<FIRST>(g, M, rb, pb, beta, c0, cx, y, pc);
        pout[c0] = pc;
        acc += pc * ap;
    }
    return acc;
}


// Iteration k. rr_k from rbk; for k > 0, rr_{k-1} from rbm and p_{k-1}.q_{k-1}
// from pqm. First x += alpha_{k-1} p_{k-1} if pending; then, unless stopped:
// p = r + beta p_old with beta = rr_k / rr_{k-1} (p = r at k = 0), formed at
// every stencil point and stored; q = A p enters only the partial sums of p.q
// (pqs). Workgroup 0 of each field publishes the stop flag (and rr_0 at
// k = 0). 2D: runs of 64 x 4 tiles.
__global__ __launch_bounds__(kBlock) void k_cg_apply2(Grid g, const double* __restrict__ r,
                                                       const double* __restrict__ pin, double* __restrict__ pout,
                                                       double* __restrict__ x, const double* __restrict__ rbk,
                                                       const double* __restrict__ rbm, const double* __restrict__ pqm,
                                                       double* __restrict__ pqs, CgScal* st, int k, double rtol2,
                                                       int maxiter) {
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
        acc = cg_apply2_run<true>(g, c, r + soff, pin + soff, pout + soff, x + soff, 0.0, 0.0);
    else
        acc = cg_apply2_run<false>(g, c, r + soff, pin + soff, pout + soff, x + soff, rrk / rrm, am);
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) pqs[c.slot()] = s;
}

// 2D update: r -= alpha A p with A p recomputed from the stored p.
__device__ __forceinline__ double cg_update2_run(const Grid& g, const CgSplit& c, const double* p, double* r,
                                                 double alpha) {
    const YMetric M(g);
    double acc = 0.0;
    for (int t = c.t0; t < c.t1; ++t) {
        int cx, y, z;
        if (!cg_cell(g, t, cx, y, z)) continue;
        const int64_t c0 = int64_t(y) * g.nx + cx;
        const double pc = p[c0];
        const double ap = cg_ap2<true>(g, M, p, nullptr, 0.0, c0, cx, y, pc);
        const double v = r[c0] - alpha * ap;
        r[c0] = v;
        acc += v * v;
    }
    return acc;
}

// One 3D CG workgroup: a 64 x 8 tile column of its field, a z-chunk, the
// thread's cell, its halo cell (threads < 144: x halo then y halo) and the
// row-scaled coefficients of -Omega_p D G (w_y / h^2 in x and z, 1 / d
// across the y-faces; no face beyond a wall). Lanes past n_x address the
// periodic image, so the last column's +x neighbour is in place.
struct CgTile3 {
    int x0, y0, z0, z1, lx, ly, y;
    bool yin, valid, hthr, hal;
    int hrow, hcol;
    int64_t plane, own, hal_off;
    double cx, cz, cyp, cym;
    __device__ __forceinline__ CgTile3(const Grid& g, const CgSplit& c) {
        const YMetric M(g);
        const int cols = cg_cols3(g);
        const int ntx = (g.nx + kTileX - 1) / kTileX;
        const int nzc = cg_zchunks(g);
        const int col = c.blk % cols, zc = c.blk / cols;
        z0 = int(int64_t(g.nz) * zc / nzc);
        z1 = int(int64_t(g.nz) * (zc + 1) / nzc);
        x0 = (col % ntx) * kTileX;
        y0 = (col / ntx) * kCgTy;
        lx = threadIdx.x & (kTileX - 1);
        ly = threadIdx.x / kTileX;
        const int xw = (x0 + lx) % g.nx;
        y = y0 + ly;
        yin = y < g.ny;
        valid = yin && x0 + lx < g.nx;
        plane = int64_t(g.nx) * g.ny;
        const double wy = yin ? M.w(y) : 0.0;
        cx = wy * g.ih2[0];
        cz = wy * g.ih2[2];
        cyp = (yin && y < g.ny - 1) ? M.id(y) : 0.0;
        cym = (yin && y > 0) ? M.id(y - 1) : 0.0;
        int hx = 0, hy = 0;
        hrow = hcol = 0;
        hal = false;
        hthr = threadIdx.x < 2 * kCgTy + 2 * kTileX;
        if (threadIdx.x < 2 * kCgTy) {
            const int row = threadIdx.x >> 1, side = threadIdx.x & 1;
            hy = y0 + row;
            hrow = row + 1;
            hcol = side ? kTileX + 1 : 0;
            hx = side ? (x0 + kTileX) % g.nx : (x0 + g.nx - 1) % g.nx;
            hal = hy < g.ny;
        } else if (hthr) {
            const int i = threadIdx.x - 2 * kCgTy;
            const int side = i / kTileX, cxl = i % kTileX;
            hy = side ? y0 + kCgTy : y0 - 1;
            hrow = side ? kCgTy + 1 : 0;
            hcol = cxl + 1;
            hx = (x0 + cxl) % g.nx;
            hal = hy >= 0 && hy < g.ny;
        }
        own = int64_t(y) * g.nx + xw;
        hal_off = int64_t(hy) * g.nx + hx;
    }
    // A p at plane z of the centre, from the LDS plane and the z neighbours.
    __device__ __forceinline__ double ap(const double (*P)[kTileX + 2], double pm, double pc, double pp) const {
        double a = (2.0 * pc - P[ly + 1][lx] - P[ly + 1][lx + 2]) * cx;
        a += (pc - P[ly][lx + 1]) * cym + (pc - P[ly + 2][lx + 1]) * cyp;
        return a + (2.0 * pc - pm - pp) * cz;
    }
    __device__ __forceinline__ int64_t cell(const Grid& g, int z) const {
        return int64_t(z) * plane + int64_t(y) * g.nx + x0 + lx;
    }
};

// 3D apply: each thread walks its (x, y) along the z-chunk with p at z - 1,
// z, z + 1 in registers and the x/y neighbours in a two-plane LDS ring; p_old
// at the centre rides along for the pending solution update.
template <bool FIRST>
__device__ __forceinline__ double cg_apply3_run(const Grid& g, const CgSplit& c, const double* __restrict__ r,
                                                const double* __restrict__ pin, double* __restrict__ pout,
                                                double* __restrict__ x, double beta, double am,
                                                double (*pl)[kCgTy + 2][kTileX + 2]) {
    const CgTile3 t(g, c);
    const int zm0 = t.z0 == 0 ? g.nz - 1 : t.z0 - 1;
    double pm = t.yin ? cg_dir<FIRST>(r, pin, int64_t(zm0) * t.plane + t.own, beta) : 0.0;
    double oc = 0.0, pc = 0.0;
    if (t.yin) {
        const int64_t j = int64_t(t.z0) * t.plane + t.own;
        oc = FIRST ? 0.0 : pin[j];
        pc = FIRST ? r[j] : r[j] + beta * oc;
    }
    pl[0][t.ly + 1][t.lx + 1] = pc;
    if (t.hthr) pl[0][t.hrow][t.hcol] = t.hal ? cg_dir<FIRST>(r, pin, int64_t(t.z0) * t.plane + t.hal_off, beta) : 0.0;
    __syncthreads();
    int cur = 0;
    double acc = 0.0;
    for (int z = t.z0; z < t.z1; ++z) {
        const int zp = z == g.nz - 1 ? 0 : z + 1;
        double op = 0.0, pp = 0.0;
        if (t.yin) {
            const int64_t j = int64_t(zp) * t.plane + t.own;
            op = FIRST ? 0.0 : pin[j];
            pp = FIRST ? r[j] : r[j] + beta * op;
        }
        const double hv = (t.hthr && t.hal) ? cg_dir<FIRST>(r, pin, int64_t(zp) * t.plane + t.hal_off, beta) : 0.0;
        if (t.valid) {
            const double ap = t.ap(pl[cur], pm, pc, pp);
            const int64_t c0 = t.cell(g, z);
            if (!FIRST && am != 0.0) x[c0] += am * oc;
            pout[c0] = pc;
            acc += pc * ap;
        }
        const int nxt = cur ^ 1;
        pl[nxt][t.ly + 1][t.lx + 1] = pp;
        if (t.hthr) pl[nxt][t.hrow][t.hcol] = hv;
        __syncthreads();
        cur = nxt;
        pm = pc;
        pc = pp;
        oc = op;
    }
    return acc;
}

// 3D update: the same walk over the stored p; r -= alpha A p at the centre.
__device__ __forceinline__ double cg_update3_run(const Grid& g, const CgSplit& c, const double* __restrict__ p,
                                                 double* __restrict__ r, double alpha,
                                                 double (*pl)[kCgTy + 2][kTileX + 2]) {
    const CgTile3 t(g, c);
    const int zm0 = t.z0 == 0 ? g.nz - 1 : t.z0 - 1;
    double pm = t.yin ? p[int64_t(zm0) * t.plane + t.own] : 0.0;
    double pc = t.yin ? p[int64_t(t.z0) * t.plane + t.own] : 0.0;
    pl[0][t.ly + 1][t.lx + 1] = pc;
    if (t.hthr) pl[0][t.hrow][t.hcol] = t.hal ? p[int64_t(t.z0) * t.plane + t.hal_off] : 0.0;
    __syncthreads();
    int cur = 0;
    double acc = 0.0;
    for (int z = t.z0; z < t.z1; ++z) {
        const int zp = z == g.nz - 1 ? 0 : z + 1;
        const double pp = t.yin ? p[int64_t(zp) * t.plane + t.own] : 0.0;
        const double hv = (t.hthr && t.hal) ? p[int64_t(zp) * t.plane + t.hal_off] : 0.0;
        if (t.valid) {
            const double ap = t.ap(pl[cur], pm, pc, pp);
            const int64_t c0 = t.cell(g, z);
            const double v = r[c0] - alpha * ap;
            r[c0] = v;
            acc += v * v;
        }
        const int nxt = cur ^ 1;
        pl[nxt][t.ly + 1][t.lx + 1] = pp;
        if (t.hthr) pl[nxt][t.hrow][t.hcol] = hv;
        __syncthreads();
        cur = nxt;
        pm = pc;
        pc = pp;
    }
    return acc;
}

__device__ __forceinline__ CgSplit cg_split3(const Grid& g) {
    CgSplit c;
    c.nblk = cg_blocks_of(g);
    const int id = xcd_logical(blockIdx.x, gridDim.x);
    c.b = id / c.nblk;
    c.blk = id - c.b * c.nblk;
    c.t0 = c.t1 = 0;
    return c;
}

__global__ __launch_bounds__(kCgThreads3) void k_cg_apply3(Grid g, const double* __restrict__ r,
                                                            const double* __restrict__ pin, double* __restrict__ pout,
                                                            double* __restrict__ x, const double* __restrict__ rbk,
                                                            const double* __restrict__ rbm,
                                                            const double* __restrict__ pqm, double* __restrict__ pqs,
                                                            CgScal* st, int k, double rtol2, int maxiter) {
    __shared__ double sh[kCgThreads3 / 64];
    __shared__ double pl[2][kCgTy + 2][kTileX + 2];
    const CgSplit c = cg_split3(g);
    const double rrk = field_total<kCgThreads3>(rbk, c, sh);
    const double rr0 = k == 0 ? rrk : st[c.b].rr0;
    const bool stop = cg_stopped(rrk, rr0, k, rtol2, maxiter);
    if (c.blk == 0 && threadIdx.x == 0) {
        if (k == 0) st[c.b].rr0 = rrk;
        st[c.b].done = stop ? 1 : 0;
    }
    double rrm = 0.0, am = 0.0;
    if (k > 0) {
        rrm = field_total<kCgThreads3>(rbm, c, sh);
        am = cg_pending(rrm, field_total<kCgThreads3>(pqm, c, sh), rr0, k, rtol2, maxiter);
    }
    const int64_t soff = int64_t(c.b) * g.ncell;
    if (stop) {
        if (am != 0.0) {
            const CgTile3 t(g, c);
            if (t.valid)
                for (int z = t.z0; z < t.z1; ++z) {
                    const int64_t i = soff + t.cell(g, z);
                    x[i] += am * pin[i];
                }
        }
        return;
    }
    double acc;
    if (k == 0)
        acc = cg_apply3_run<true>(g, c, r + soff, pin + soff, pout + soff, x + soff, 0.0, 0.0, pl);
    else
        acc = cg_apply3_run<false>(g, c, r + soff, pin + soff, pout + soff, x + soff, rrk / rrm, am, pl);
    const double s = block_sum<kCgThreads3>(acc, sh);
    if (threadIdx.x == 0) pqs[c.slot()] = s;
}

// Iteration k, unless stopped: alpha = rr_k / p.q, r -= alpha A p with A p
// recomputed from the stored p (same stencil, same arithmetic as the apply
// kernel), partial sums of r.r (rr_{k+1}) into rbn; the matching x update is
// pending until the next apply kernel. A stopped field copies its rr_k
// partials forward instead, so the newest buffer always holds the final sum;
// a search direction with p.q <= 0 (no component outside the constants) ends
// the solve without an update (partials written as 0).
template <int NT, int DIM>
__global__ __launch_bounds__(NT) void k_cg_update(Grid g, double* __restrict__ r, const double* __restrict__ p,
                                                  const double* __restrict__ rbk, const double* __restrict__ pqs,
                                                  double* __restrict__ rbn, CgScal* st, int k, double rtol2,
                                                  int maxiter) {
    __shared__ double sh[NT / 64];
    const CgSplit c = DIM == 3 ? cg_split3(g) : cg_split(g);
    const double rrk = field_total<NT>(rbk, c, sh);
    if (cg_stopped(rrk, st[c.b].rr0, k, rtol2, maxiter)) {
        if (threadIdx.x == 0) rbn[c.slot()] = rbk[c.slot()];
        return;
    }
    const double pq = field_total<NT>(pqs, c, sh);
    if (!(pq > 0.0)) {
        if (threadIdx.x == 0) rbn[c.slot()] = 0.0;
        return;
    }
    const double alpha = rrk / pq;
    const int64_t soff = int64_t(c.b) * g.ncell;
    double acc;
    if constexpr (DIM == 3) {
        __shared__ double pl[2][kCgTy + 2][kTileX + 2];
        acc = cg_update3_run(g, c, p + soff, r + soff, alpha, pl);
    } else {
        acc = cg_update2_run(g, c, p + soff, r + soff, alpha);
    }
    const double s = block_sum<NT>(acc, sh);
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

// Partial sums of w_j t (volume-weighted mean of a solution).
__global__ __launch_bounds__(kBlock) void k_cg_wsum(Grid g, const double* __restrict__ t, double* __restrict__ msum) {
    __shared__ double sh[kBlock / 64];
    const CgSplit c = cg_split(g);
    const YMetric M(g);
    double acc = 0.0;
    for (int tt = c.t0; tt < c.t1; ++tt) {
        int x, y, z;
        if (!cg_cell(g, tt, x, y, z)) continue;
        acc += M.w(y) * t[cg_index(g, c.b, x, y, z)];
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) msum[c.slot()] = s;
}

// t = w_j (t - mean_w(t)), in place (the output side of the solve's pullback).
__global__ __launch_bounds__(kBlock) void k_cg_post(Grid g, double* __restrict__ t, const double* __restrict__ msum,
                                                     double wsum) {
    __shared__ double sh[kBlock / 64];
    const CgSplit c = cg_split(g);
    const YMetric M(g);
    const double mean = field_total(msum, c, sh) / wsum;
    for (int tt = c.t0; tt < c.t1; ++tt) {
        int x, y, z;
        if (!cg_cell(g, tt, x, y, z)) continue;
        const int64_t k = cg_index(g, c.b, x, y, z);
        t[k] = M.w(y) * (t[k] - mean);
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
hipError_t launch_wall_project(const Grid& g, const T* w, const double* p, T* u_out, bool adj, hipStream_t s) {
    const int nblk = stencil_blocks(g);
    if (g.dim == 3) {
        if (adj)
            hipLaunchKernelGGL((k_wall_project<T, 3, true>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, u_out);
        else
            hipLaunchKernelGGL((k_wall_project<T, 3, false>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, u_out);
    } else {
        if (adj)
            hipLaunchKernelGGL((k_wall_project<T, 2, true>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, u_out);
        else
            hipLaunchKernelGGL((k_wall_project<T, 2, false>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, u_out);
    }
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
    if (g.dim == 3) {
        constexpr int TX = 64, TY = 8;
        const int zc = zm_chunk_stage(g, sizeof(T) == 8);
        const int nblk = ((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY) * ((g.nz + zc - 1) / zc) * g.batch;
        const int yi = yinit ? 1 : 0;
        // pointwise streams: u0 when it seeds the stage register or the
        // accumulator, y when the accumulator is read
        const int pt = ((wout || yinit) ? 1 : 0) | ((y && !yinit) ? 2 : 0);
#define INS_WSZM(PR, PTI)                                                                                            \
    hipLaunchKernelGGL((k_wall_stage_zm<T, PR, TX, TY, PTI>), dim3(nblk), dim3(TX * TY), 0, s, g, w, p, u0, y, yi, T(cy), \
                       wout, T(cw), zc)
        if (proj && pt == 3)
            INS_WSZM(true, 3);
        else if (proj && pt == 2)
            INS_WSZM(true, 2);
        else if (proj)
            INS_WSZM(true, 1);
        else if (pt == 3)
            INS_WSZM(false, 3);
        else
            INS_WSZM(false, 1);
#undef INS_WSZM
    } else
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
    if (g.dim == 3) {
        const int zc = zm_chunk(g, kWvTX, kWvTY, 2048, 32);
        const int nblk =
            ((g.nx + kWvTX - 1) / kWvTX) * ((g.ny + kWvTY - 1) / kWvTY) * ((g.nz + zc - 1) / zc) * g.batch;
        const T tb = T(cb), tw = T(cw);
#define INS_WVJP_ZM(PU, HW)                                                                                       \
    hipLaunchKernelGGL((k_wall_stage_vjp_zm<T, PU, HW>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, ybar, un, q, tb, \
                       tw, u0bar, mode, ubar_out, zc)
        if (proj_u && has_w)
            INS_WVJP_ZM(true, true);
        else if (proj_u)
            INS_WVJP_ZM(true, false);
        else if (has_w)
            INS_WVJP_ZM(false, true);
        else
            INS_WVJP_ZM(false, false);
#undef INS_WVJP_ZM
    } else
        wall_stage_vjp_dim<T, 2>(g, w, p, proj_u, ybar, un, q, has_w, T(cb), T(cw), u0bar, mode, ubar_out, s);
    return hipGetLastError();
}

int cg_blocks(const Grid& g) { return cg_blocks_of(g); }

template <typename T>
hipError_t launch_cg_div(const Grid& g, const T* vel, const double* rin, double* r, double* msum, int mode,
                         hipStream_t s) {
    if (g.gm[0]) return launch_gen_cg_div<T>(g, vel, rin, r, msum, mode, s);
    const int nblk = cg_blocks_of(g) * g.batch;
    if (g.dim == 3)
        hipLaunchKernelGGL((k_cg_div<T, 3>), dim3(nblk), dim3(kBlock), 0, s, g, vel, rin, r, msum, mode);
    else
        hipLaunchKernelGGL((k_cg_div<T, 2>), dim3(nblk), dim3(kBlock), 0, s, g, vel, rin, r, msum, mode);
    return hipGetLastError();
}

hipError_t launch_cg_init(const Grid& g, double* r, double* x, const double* msum, double* rb0, CgScal* st, int mode,
                          double wsum, hipStream_t s) {
    if (g.gm[0]) return launch_gen_cg_init(g, r, x, msum, rb0, st, mode, wsum, s);
    hipLaunchKernelGGL(k_cg_init, dim3(cg_blocks_of(g) * g.batch), dim3(kBlock), 0, s, g, r, x, msum, rb0, st, mode,
                       wsum);
    return hipGetLastError();
}

hipError_t launch_cg_apply(const Grid& g, const double* r, const double* pin, double* pout, double* x,
                           const double* rbk, const double* rbm, const double* pqm, double* pqs, CgScal* st, int k,
                           double rtol2, int maxiter, hipStream_t s) {
    if (g.gm[0]) return launch_gen_cg_apply(g, r, pin, pout, x, rbk, rbm, pqm, pqs, st, k, rtol2, maxiter, s);
    const int nblk = cg_blocks_of(g) * g.batch;
    if (g.dim == 3)
        hipLaunchKernelGGL(k_cg_apply3, dim3(nblk), dim3(kCgThreads3), 0, s, g, r, pin, pout, x, rbk, rbm, pqm, pqs, st,
                           k, rtol2, maxiter);
    else
        hipLaunchKernelGGL(k_cg_apply2, dim3(nblk), dim3(kBlock), 0, s, g, r, pin, pout, x, rbk, rbm, pqm, pqs, st, k,
                           rtol2, maxiter);
    return hipGetLastError();
}

hipError_t launch_cg_update(const Grid& g, double* r, const double* p, const double* rbk, const double* pqs,
                            double* rbn, CgScal* st, int k, double rtol2, int maxiter, hipStream_t s) {
    if (g.gm[0]) return launch_gen_cg_update(g, r, p, rbk, pqs, rbn, st, k, rtol2, maxiter, s);
    const int nblk = cg_blocks_of(g) * g.batch;
    if (g.dim == 3)
        hipLaunchKernelGGL((k_cg_update<kCgThreads3, 3>), dim3(nblk), dim3(kCgThreads3), 0, s, g, r, p, rbk, pqs, rbn,
                           st, k, rtol2, maxiter);
    else
        hipLaunchKernelGGL((k_cg_update<kBlock, 2>), dim3(nblk), dim3(kBlock), 0, s, g, r, p, rbk, pqs, rbn, st, k,
                           rtol2, maxiter);
    return hipGetLastError();
}

hipError_t launch_cg_finish(const Grid& g, const double* rb, CgScal* st, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_finish, dim3(g.batch), dim3(kBlock), 0, s, g, rb, st);
    return hipGetLastError();
}

hipError_t launch_cg_weighted_center(const Grid& g, double* t, double* msum, double wsum, hipStream_t s) {
    if (g.gm[0]) return launch_gen_cg_weighted_center(g, t, msum, wsum, s);
    const int nblk = cg_blocks_of(g) * g.batch;
    hipLaunchKernelGGL(k_cg_wsum, dim3(nblk), dim3(kBlock), 0, s, g, t, msum);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cg_post, dim3(nblk), dim3(kBlock), 0, s, g, t, msum, wsum);
    return hipGetLastError();
}

#define INS_WALL_INSTANTIATE(T)                                                                                      \
    template hipError_t launch_wall_rhs<T>(const Grid&, const T*, T*, hipStream_t);                                  \
    template hipError_t launch_wall_divergence<T>(const Grid&, const T*, double*, hipStream_t);                      \
    template hipError_t launch_wall_gradient<T>(const Grid&, const double*, T*, hipStream_t);                        \
    template hipError_t launch_wall_project<T>(const Grid&, const T*, const double*, T*, bool, hipStream_t);          \
    template hipError_t launch_wall_rhs_vjp<T>(const Grid&, const T*, const T*, T*, hipStream_t);                    \
    template hipError_t launch_wall_div_vjp<T>(const Grid&, const double*, T*, hipStream_t);                         \
    template hipError_t launch_wall_grad_vjp<T>(const Grid&, const T*, double*, hipStream_t);                        \
    template hipError_t launch_wall_stage<T>(const Grid&, const T*, const double*, bool, const T*, T*, bool, double, \
                                             T*, double, hipStream_t);                                               \
    template hipError_t launch_wall_stage_vjp<T>(const Grid&, const T*, const double*, bool, const T*, const T*,     \
                                                 const double*, bool, double, double, T*, int, T*, hipStream_t);     \
    template hipError_t launch_cg_div<T>(const Grid&, const T*, const double*, double*, double*, int, hipStream_t);

INS_WALL_INSTANTIATE(double)
INS_WALL_INSTANTIATE(float)

}  // namespace ins
