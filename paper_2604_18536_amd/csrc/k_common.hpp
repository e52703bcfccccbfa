// Device helpers shared by the gfx950 kernels: periodic neighbour offsets,
// XCD-aware workgroup order, complex arithmetic.
#pragma once

#include "ins_internal.hpp"

namespace ins {

constexpr int kBlock = 256;   // threads per workgroup (4 wave64)
constexpr int kTileX = 64;    // stencil tile: one wave64 per x-row
constexpr int kTileY = 4;

// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with a private L2. Map the hardware order to a logical order in which every
// XCD receives one contiguous range of tiles, so that tiles sharing halos
// share an L2. The map is a bijection of [0, n) whatever the dispatch order.
__device__ __forceinline__ int xcd_logical(int hw, int n) {
    const int q = n >> 3, r = n & 7;
    const int x = hw & 7, pos = hw >> 3;
    return x * q + (x < r ? x : r) + pos;
}

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Offsets of the periodic neighbours of a cell: coordinate c-1, c, c+1, c+2 per
// direction, already multiplied by the direction's stride.
struct Nb {
    int xo[4], yo[4], zo[4];
    __device__ __forceinline__ int at(int dx, int dy, int dz) const { return xo[dx + 1] + yo[dy + 1] + zo[dz + 1]; }
};

template <int DIM>
__device__ __forceinline__ Nb make_nb(const Grid& g, int x, int y, int z) {
    Nb nb;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        nb.xo[k] = wrap(x + k - 1, g.nx);
        nb.yo[k] = wrap(y + k - 1, g.ny) * g.nx;
        nb.zo[k] = (DIM == 3) ? wrap(z + k - 1, g.nz) * g.nx * g.ny : 0;
    }
    return nb;
}

__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ cd cmulc(cd a, cd b) { return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }  // a*conj(b)
__device__ __forceinline__ cd cscale(cd a, double s) { return {a.x * s, a.y * s}; }
__device__ __forceinline__ cd cconj(cd a) { return {a.x, -a.y}; }
__device__ __forceinline__ cf cadd(cf a, cf b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cf csub(cf a, cf b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cf cmul(cf a, cf b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ cf cmulc(cf a, cf b) { return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }  // a*conj(b)
__device__ __forceinline__ cf cscale(cf a, float s) { return {a.x * s, a.y * s}; }
__device__ __forceinline__ cf cconj(cf a) { return {a.x, -a.y}; }

// Tile decomposition of a stencil launch: (x-tile, y-tile, z, batch).
struct TileIdx {
    int x, y, z, b;
    bool valid;
};

// Tile number t (no XCD reordering) of a stencil launch.
__device__ __forceinline__ TileIdx tile_at(const Grid& g, int t) {
    const int ntx = (g.nx + kTileX - 1) / kTileX;
    const int nty = (g.ny + kTileY - 1) / kTileY;
    TileIdx r;
    const int tx = t % ntx;
    t /= ntx;
    const int ty = t % nty;
    t /= nty;
    r.z = t % g.nz;
    r.b = t / g.nz;
    r.x = tx * kTileX + (threadIdx.x & (kTileX - 1));
    r.y = ty * kTileY + (threadIdx.x / kTileX);
    r.valid = r.x < g.nx && r.y < g.ny;
    return r;
}

__device__ __forceinline__ TileIdx tile_of(const Grid& g) {
    const int ntx = (g.nx + kTileX - 1) / kTileX;
    const int nty = (g.ny + kTileY - 1) / kTileY;
    int t = xcd_logical(blockIdx.x, gridDim.x);
    TileIdx r;
    const int tx = t % ntx;
    t /= ntx;
    const int ty = t % nty;
    t /= nty;
    r.z = t % g.nz;
    r.b = t / g.nz;
    r.x = tx * kTileX + (threadIdx.x & (kTileX - 1));
    r.y = ty * kTileY + (threadIdx.x / kTileX);
    r.valid = r.x < g.nx && r.y < g.ny;
    return r;
}

// Velocity value at a neighbour of the current cell. With PROJ the stored
// field is the unprojected stage value w and the velocity is w - G p, formed
// in float64 (the projection of the previous RK stage, Sec. 2.6.2, fused into
// this stencil so the projected field is never written out).
// P: the pressure type and the precision of w - G p (float64 except in the
// all-float32 comparison mode).
template <typename T, bool PROJ, typename P = double>
struct VelSrc {
    const T* __restrict__ w;
    const P* __restrict__ p;
    int ncell;
    double ih0, ih1, ih2;
    __device__ __forceinline__ T operator()(int c, const Nb& nb, int dx, int dy, int dz) const {
        const int j = nb.at(dx, dy, dz);
        if constexpr (!PROJ) {
            return w[c * ncell + j];
        } else {
            const int jp = nb.at(dx + (c == 0), dy + (c == 1), dz + (c == 2));
            const P ih = P(c == 0 ? ih0 : (c == 1 ? ih1 : ih2));
            return T(P(w[c * ncell + j]) - (p[jp] - p[j]) * ih);
        }
    }
};

// F^a at the current cell: diffusion (eq. diff-kernel) + convection
// (eq. conv-kernel with weights 1/2). The flux through the b-face of the
// a-velocity volume is F^{ab}[K] = (u^a[K] + u^a[K+e_b]) (u^b[K] + u^b[K+e_a]) / 4,
// formed at K = I and K = I - e_b and consumed at once (lazy components, Sec. 3.3).
template <typename T, int DIM, class Src>
__device__ __forceinline__ void rhs_cell(const Grid& g, const Src& U, const Nb& nb, T F[DIM]) {
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
            diff += ((up - uc) - (uc - um)) * T(g.ih2[b]);
            const T vr = U(b, nb, 0, 0, 0) + U(b, nb, ax, ay, az);
            const T vl = U(b, nb, -bx, -by, -bz) + U(b, nb, ax - bx, ay - by, az - bz);
            const T fr = (uc + up) * vr * T(0.25);
            const T fl = (um + uc) * vl * T(0.25);
            conv -= (fr - fl) * T(g.ih[b]);
        }
        F[a] = conv + T(g.nu) * diff;
    }
}

// Pullback of the right-hand side at one cell (gather form; see k_vjp.hip).
template <typename T, int DIM, class USrc, class FSrc>
__device__ __forceinline__ void rhs_vjp_cell(const Grid& g, const USrc& U, const FSrc& Fb, const Nb& nb, T out[DIM]) {
#pragma unroll
    for (int gm = 0; gm < DIM; ++gm) {
        const int gx = gm == 0, gy = gm == 1, gz = gm == 2;
        const T ihg = T(g.ih[gm]);
        const T fc = Fb(gm, nb, 0, 0, 0);
        T diff = T(0), acc = T(0);
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            const int bx = b == 0, by = b == 1, bz = b == 2;
            const T ihb = T(g.ih[b]);
            const T fp = Fb(gm, nb, bx, by, bz);
            const T fm = Fb(gm, nb, -bx, -by, -bz);
            diff += ((fp - fc) - (fc - fm)) * T(g.ih2[b]);
            const T m0 = U(b, nb, 0, 0, 0) + U(b, nb, gx, gy, gz);
            const T g0 = (fp - fc) * ihb + (Fb(b, nb, gx, gy, gz) - Fb(b, nb, 0, 0, 0)) * ihg;
            const T m1 = U(b, nb, -bx, -by, -bz) + U(b, nb, gx - bx, gy - by, gz - bz);
            const T g1 = (fc - fm) * ihb + (Fb(b, nb, gx - bx, gy - by, gz - bz) - Fb(b, nb, -bx, -by, -bz)) * ihg;
            acc += m0 * g0 + m1 * g1;
        }
        out[gm] = T(0.25) * acc + T(g.nu) * diff;
    }
}

inline int stencil_blocks(const Grid& g) {
    const int ntx = (g.nx + kTileX - 1) / kTileX;
    const int nty = (g.ny + kTileY - 1) / kTileY;
    return ntx * nty * g.nz * g.batch;
}

}  // namespace ins
