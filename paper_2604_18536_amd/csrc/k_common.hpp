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

// Tile decomposition of a stencil launch: (x-tile, y-tile, z, batch).
struct TileIdx {
    int x, y, z, b;
    bool valid;
};

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
// in float64 (the projection of the previous RK stage, Sec. 2.5.2, fused into
// this stencil so the projected field is never written out).
template <typename T, bool PROJ>
struct VelSrc {
    const T* __restrict__ w;
    const double* __restrict__ p;
    int ncell;
    double ih0, ih1, ih2;
    __device__ __forceinline__ T operator()(int c, const Nb& nb, int dx, int dy, int dz) const {
        const int j = nb.at(dx, dy, dz);
        if constexpr (!PROJ) {
            return w[c * ncell + j];
        } else {
            const int jp = nb.at(dx + (c == 0), dy + (c == 1), dz + (c == 2));
            const double ih = c == 0 ? ih0 : (c == 1 ? ih1 : ih2);
            return T(double(w[c * ncell + j]) - (p[jp] - p[j]) * ih);
        }
    }
};

inline int stencil_blocks(const Grid& g) {
    const int ntx = (g.nx + kTileX - 1) / kTileX;
    const int nty = (g.ny + kTileY - 1) / kTileY;
    return ntx * nty * g.nz * g.batch;
}

}  // namespace ins
