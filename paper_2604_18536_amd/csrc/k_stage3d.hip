// Fused RK4 stage for 3D grids as a 2.5D z-march (the forward counterpart of
// k_stage in k_stencil.hip; same arithmetic, different data movement).
//
// A workgroup owns a 64 x 8 tile of an x-y plane (the reverse stage: 32 x 8)
// and a chunk of consecutive z planes. For every plane it forms the stage
// velocity u = w - G p (float64 projection, Sec. 2.6.2) on the tile plus a
// one-cell halo exactly once and
// keeps it in a 4-plane LDS ring; the right-hand side of plane z then reads
// planes z-1, z, z+1 from LDS only. Each plane of w and p is therefore fetched
// once per tile (plus the x-y halo, which neighbouring tiles of the same XCD
// share through L2) instead of three times. With four ring slots the plane
// being filled is never one being read, so one barrier per plane suffices.
#include "k_common.hpp"

namespace ins {

constexpr int kZmTX = 32, kZmTY = 8;  // reverse-stage tile
constexpr int kZmHX = kZmTX + 2, kZmHY = kZmTY + 2, kZmHP = kZmHX * kZmHY;  // 340 halo-plane cells

template <typename T, int HX = kZmHX, int HP = kZmHP>
struct LdsSrc {
    const T* zm;  // ring slot of plane z-1
    const T* z0;  // plane z
    const T* zp;  // plane z+1
    int centre;   // index of the cell in the halo plane
    __device__ __forceinline__ T operator()(int c, const Nb&, int dx, int dy, int dz) const {
        const T* b = dz < 0 ? zm : (dz > 0 ? zp : z0);
        return b[c * HP + centre + dy * HX + dx];
    }
};

__device__ __forceinline__ int pmod(int v, int n) {
    const int r = v % n;
    return r < 0 ? r + n : r;
}

// Streams touched exactly once per step (u0, y, the new stage register) bypass
// the caches' normal allocation.
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
    return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void st_stream(T v, T* p) {
    __builtin_nontemporal_store(v, p);
}

// P: type of the pressure and of the projection arithmetic w - G p (float64;
// float32 only in the all-float32 comparison mode).
// PT: the pointwise streams the stage reads at its own cells, fixed per
// instance (bit 0: base = u0, the stage register's origin and, with yinit, the
// accumulator's; bit 1: the accumulator y, or with YW the earlier stage input
// wprev). y and wout are written when non-null; yinit starts y at u0.
// YW: the accumulator is formed from unprojected stage inputs as
// y = u0 + ry (wprev - u0) + rw (w - u0): RK4's third stage forms
// u0 + dt/6 F1 + dt/3 F2 from W2 = u0 + dt/2 F1 (wprev) and W3 = u0 + dt/2 F2
// (w), so the first two stages need not store y nor this stage read it. wprev
// may be the buffer wout writes: each cell's wprev is read one plane before
// that cell's output is written (hence no restrict).
//
// Every global load in the plane loop is issued unconditionally (halo slots
// past the halo load a valid position and are not parked; the last iteration
// fetches its own last plane again, an L2 hit; the pointwise cells and planes
// are clamped), so the compiler counts the loads in flight exactly and waits
// only for the ones a step needs. With a load behind a condition it must
// assume the shortest path and waits for every load in flight: the next
// plane's halo loads were then waited for before the current plane's compute.
template <typename T, bool PROJ, int TX, int TY, typename P = double, bool YW = false, int PT = 1>
__global__ __launch_bounds__(TX * TY) void k_stage_zm(Grid g, const T* __restrict__ w, const P* __restrict__ p,
                                                        const T* __restrict__ u0, T* __restrict__ y, int yinit, T cy,
                                                        T* wout, T cw, int zc, const T* __restrict__ mc,
                                                        const T* wprev, T ry, T rw) {
    constexpr int NT = TX * TY, HX = TX + 2, HP = HX * (TY + 2);
    constexpr int NS = (HP + NT - 1) / NT;  // halo-plane cells per thread
    constexpr bool LB = (PT & 1) != 0, LY = (PT & 2) != 0;
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
    const P* pb = PROJ ? p + int64_t(b) * g.ncell : nullptr;
    const int nc = int(g.ncell);
    const int plane = nx * ny;

    // halo-plane positions loaded by this thread (slots past the halo load the
    // first position and are not parked)
    int hq[NS], hxy[NS], hxp[NS], hyp[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int q = threadIdx.x + s * NT;
        hq[s] = q;
        const int qq = q < HP ? q : 0;
        const int gx = pmod(x0 - 1 + qq % HX, nx);
        const int gy = pmod(y0 - 1 + qq / HX, ny);
        hxy[s] = gy * nx + gx;
        hxp[s] = gy * nx + (gx + 1 == nx ? 0 : gx + 1);
        hyp[s] = (gy + 1 == ny ? 0 : gy + 1) * nx + gx;
    }
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int cxg = x0 + lx, cyg = y0 + ly;
    const bool valid = cxg < nx && cyg < ny;
    const int cxy = min(cyg, ny - 1) * nx + min(cxg, nx - 1);  // own cell, clamped for the loads
    const int centre = (ly + 1) * HX + (lx + 1);
    const int nk = (z1 - z0) + 2;  // ring planes z0-1 .. z1

    if constexpr (!PROJ && sizeof(T) == 8) {
        // The unprojected stage (its stage velocity is u0 itself, w == u0) in
        // float64: two planes ahead. The loads of ring plane k+2 are issued in
        // iteration k and parked at the end of iteration k+1, so each has two
        // planes' compute to land (the LDS ring already holds the kernel to two
        // workgroups per CU, so the extra registers cost no occupancy). The two
        // planes in flight alternate between two register sets (static indices:
        // the loop is unrolled by two). u0 at a thread's own cell is the centre
        // of the ring plane it computes, so no pointwise stream is loaded.
        T rwA[NS][3], rwB[NS][3];
        auto fetch_raw = [&](int zz, T (&rw_)[NS][3]) {
            const int zoff = zz * plane;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int j = zoff + hxy[s];
                rw_[s][0] = wb[j];
                rw_[s][1] = wb[nc + j];
                rw_[s][2] = wb[2 * nc + j];
            }
        };
        auto park_raw = [&](int k, const T (&rw_)[NS][3]) {
            T* slot = &ring[k & 3][0][0];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (hq[s] < HP) {
                    slot[hq[s]] = rw_[s][0];
                    slot[HP + hq[s]] = rw_[s][1];
                    slot[2 * HP + hq[s]] = rw_[s][2];
                }
            }
        };
        // iteration k: issue ring plane k+2 into iw (the last plane again near
        // the end), compute plane z0+k-2, park ring plane k+1 from pw
        auto iter = [&](int k, T (&iw)[NS][3], const T (&pw)[NS][3]) {
            const int z = z0 + k - 2;
            fetch_raw(pmod(z0 - 1 + min(k + 2, nk - 1), nz), iw);
            const T* zc0 = &ring[(k - 1) & 3][0][0];
            LdsSrc<T, HX, HP> U{&ring[(k - 2) & 3][0][0], zc0, &ring[k & 3][0][0], centre};
            T F[3];
            rhs_cell<T, 3>(g, U, Nb{}, F);
            if (valid) {
                const int c0 = z * plane + cyg * nx + cxg;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int64_t kk = boff + int64_t(a) * nc + c0;
                    const T b0 = zc0[a * HP + centre];
                    if (mc) F[a] += mc[kk];
                    if (y) st_stream((yinit ? b0 : ld_stream(y + kk)) + cy * F[a], y + kk);
                    if (wout) st_stream(b0 + cw * F[a], wout + kk);
                }
            }
            if (k + 1 < nk) park_raw(k + 1, pw);
            __syncthreads();
        };
        fetch_raw(pmod(z0 - 1, nz), rwA);
        park_raw(0, rwA);
        fetch_raw(pmod(z0, nz), rwA);
        park_raw(1, rwA);
        fetch_raw(pmod(z0 + 1, nz), rwA);
        fetch_raw(pmod(z0 - 1 + min(3, nk - 1), nz), rwB);
        park_raw(2, rwA);
        __syncthreads();
        int k = 2;
        for (; k + 1 < nk; k += 2) {
            iter(k, rwA, rwB);
            iter(k + 1, rwB, rwA);
        }
        if (k < nk) iter(k, rwA, rwB);
        return;
    }

    // raw loads of the halo plane at this thread's positions (w, and with PROJ
    // p at the cell and at its +x, +y, +z neighbours); the projection
    // u = w - G p is formed when the plane is parked, so that the loads stay in
    // flight through the plane computed meanwhile
    T pw_[NS][3];
    P pp_[NS][4];
    // YW in float64: the unprojected w at this thread's own cell of the ring
    // planes k-1 (wcA), k (wcB) and k+1 (wcN, in flight), loaded with the
    // plane's halo (whose requests cover the same lines; a later re-read went
    // back to memory). In float32 the registers would cost a wave per SIMD, so
    // that instance reads it as a third pointwise stream.
    constexpr bool WREG = YW && sizeof(T) == 8;
    T wcA[3] = {T(0), T(0), T(0)}, wcB[3] = {T(0), T(0), T(0)}, wcN[3] = {T(0), T(0), T(0)};
    auto fetch = [&](int zz) {
        const int zoff = zz * plane;
        const int zpo = (zz + 1 == nz ? 0 : zz + 1) * plane;
        if constexpr (WREG) {
#pragma unroll
            for (int a = 0; a < 3; ++a) wcN[a] = wb[int64_t(a) * nc + zoff + cxy];
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int j = zoff + hxy[s];
            pw_[s][0] = wb[j];
            pw_[s][1] = wb[nc + j];
            pw_[s][2] = wb[2 * nc + j];
            if constexpr (PROJ) {
                pp_[s][0] = pb[j];
                pp_[s][1] = pb[zoff + hxp[s]];
                pp_[s][2] = pb[zoff + hyp[s]];
                pp_[s][3] = pb[zpo + hxy[s]];
            }
        }
    };
    auto park = [&](int k) {
        T* slot = &ring[k & 3][0][0];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (hq[s] < HP) {
                if constexpr (PROJ) {
                    const P pc = pp_[s][0];
                    slot[hq[s]] = T(P(pw_[s][0]) - (pp_[s][1] - pc) * P(g.ih[0]));
                    slot[HP + hq[s]] = T(P(pw_[s][1]) - (pp_[s][2] - pc) * P(g.ih[1]));
                    slot[2 * HP + hq[s]] = T(P(pw_[s][2]) - (pp_[s][3] - pc) * P(g.ih[2]));
                } else {
                    slot[hq[s]] = pw_[s][0];
                    slot[HP + hq[s]] = pw_[s][1];
                    slot[2 * HP + hq[s]] = pw_[s][2];
                }
            }
        }
    };
    // Pointwise streams of the plane computed next: issued after the current
    // plane's stores, used at the next plane's stores (raw values, combined
    // only there).
    constexpr bool WPT = YW && !WREG;
    T pbase[3] = {T(0), T(0), T(0)}, pyv[3] = {T(0), T(0), T(0)}, pwc[3] = {T(0), T(0), T(0)};
    const T* ysrc = YW ? wprev : y;
    auto fetch_point = [&](int z) {
        const int c0 = z * plane + cxy;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int64_t kk = boff + int64_t(a) * nc + c0;
            if constexpr (LB) pbase[a] = ld_stream(u0 + kk);
            if constexpr (LY) pyv[a] = ld_stream(ysrc + kk);
            if constexpr (WPT) pwc[a] = wb[int64_t(a) * nc + c0];
        }
    };

    // Pipeline: iteration k issues ring plane k+1, computes plane z0+k-2 from
    // ring slots k-2, k-1, k, stores it, issues the next plane's pointwise
    // streams and parks plane k+1 in slot k+1, which no thread reads in
    // iteration k.
    fetch(pmod(z0 - 1, nz));
    park(0);
    fetch(pmod(z0, nz));
    park(1);
    if constexpr (WREG) {
#pragma unroll
        for (int a = 0; a < 3; ++a) wcA[a] = wcN[a];
    }
    fetch(pmod(z0 + 1, nz));
    park(2);
    if constexpr (WREG) {
#pragma unroll
        for (int a = 0; a < 3; ++a) wcB[a] = wcN[a];
    }
    fetch_point(z0);
    __syncthreads();
    for (int k = 2; k < nk; ++k) {
        const int z = z0 + k - 2;
        fetch(pmod(z0 - 1 + min(k + 1, nk - 1), nz));
        LdsSrc<T, HX, HP> U{&ring[(k - 2) & 3][0][0], &ring[(k - 1) & 3][0][0], &ring[k & 3][0][0], centre};
        T F[3];
        rhs_cell<T, 3>(g, U, Nb{}, F);
        if (valid) {
            const int c0 = z * plane + cyg * nx + cxg;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int64_t kk = boff + int64_t(a) * nc + c0;
                const T base = LB ? pbase[a] : T(0);
                T yv;
                if constexpr (YW) yv = base + ry * (pyv[a] - base) + rw * ((WREG ? wcA[a] : pwc[a]) - base);
                else if constexpr (LY) yv = pyv[a];
                else yv = base;
                if (mc) F[a] += mc[kk];
                if (y) st_stream(yv + cy * F[a], y + kk);
                if (wout) st_stream(base + cw * F[a], wout + kk);
            }
        }
        fetch_point(min(z + 1, z1 - 1));
        if (k + 1 < nk) park(k + 1);
        if constexpr (WREG) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                wcA[a] = wcB[a];
                wcB[a] = wcN[a];
            }
        }
        __syncthreads();
    }
}

// z planes per workgroup: long enough that the two extra halo planes are a
// small overhead, short enough to give the chip at least `want` workgroups
// (at most zmax planes, halved while there are fewer).
int zm_chunk(const Grid& g, int tx, int ty, int want, int zmax) {
    const int ntiles = ((g.nx + tx - 1) / tx) * ((g.ny + ty - 1) / ty) * g.batch;
    int zc = zmax;
    while (zc > 4 && int64_t(ntiles) * ((g.nz + zc - 1) / zc) < want) zc /= 2;
    return zc;
}

// Reverse stage (32 x 8 tiles of 256 threads): 2048 workgroups, at most 32 planes.
int zm_chunk(const Grid& g) { return zm_chunk(g, kZmTX, kZmTY, 2048, 32); }

// Forward stage (64 x 8 tiles of 512 threads): one full wave of resident
// workgroups, two per CU in float64 (128 VGPRs, 63 KB of LDS ring), four in
// float32, up to 64 planes. Measured at 256^3: float64 64 planes (512
// workgroups) 1.5% faster per step than 32; float32 32 planes (1024) 14%
// faster than 64.
int zm_chunk_stage(const Grid& g, bool fp64) { return zm_chunk(g, 64, 8, fp64 ? 512 : 1024, 64); }

template <typename T, int TX, int TY, typename P = double>
void launch_stage_zm_tile(const Grid& g, const T* w, const P* p, bool proj, const T* u0, T* y, int yinit,
                          double cy, T* wout, double cw, hipStream_t s, const T* mc, const T* wprev = nullptr,
                          double ry = 0.0, double rw = 0.0) {
    const int zc = zm_chunk_stage(g, sizeof(T) == 8);
    const int nblk = ((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY) * ((g.nz + zc - 1) / zc) * g.batch;
    // pointwise streams: u0 when it seeds the stage register or the accumulator,
    // y when the accumulator is read
    const int pt = ((wout || yinit) ? 1 : 0) | ((y && !yinit) ? 2 : 0);
#define INS_SZM(PR, YWI, PTI, YI, RY, RW)                                                                          \
    hipLaunchKernelGGL((k_stage_zm<T, PR, TX, TY, P, YWI, PTI>), dim3(nblk), dim3(TX * TY), 0, s, g, w, p, u0, y, YI, \
                       T(cy), wout, T(cw), zc, mc, wprev, T(RY), T(RW))
    if (wprev)
        INS_SZM(true, true, 3, 0, ry, rw);
    else if (!proj && pt == 3)
        INS_SZM(false, false, 3, yinit, 0.0, 0.0);
    else if (!proj)
        INS_SZM(false, false, 1, yinit, 0.0, 0.0);
    else if (pt == 3)
        INS_SZM(true, false, 3, yinit, 0.0, 0.0);
    else if (pt == 2)
        INS_SZM(true, false, 2, yinit, 0.0, 0.0);
    else
        INS_SZM(true, false, 1, yinit, 0.0, 0.0);
#undef INS_SZM
}

// The forward stage runs 64 x 8 tiles of 512 threads: the 512-byte row runs
// stream better than 32-wide ones (measured at 256^3: +1% FP64, +3% FP32 mode
// over 32 x 8; 64 x 4 and 128 x 4 were no better), and the 66 x 10 halo adds
// 29% re-reads instead of 33%.
template <typename T>
hipError_t launch_stage_zm(const Grid& g, const T* w, const double* p, bool proj, const T* u0, T* y, bool yinit,
                           double cy, T* wout, double cw, hipStream_t s, const T* mc) {
    if (!proj && w != u0) return hipErrorInvalidValue;  // the unprojected stage takes its centre u0 from w
    launch_stage_zm_tile<T, 64, 8>(g, w, p, proj, u0, y, yinit ? 1 : 0, cy, wout, cw, s, mc);
    return hipGetLastError();
}

// The projected stage whose accumulator is formed from stage inputs:
// y = u0 + ry (wprev - u0) + rw (w - u0) + cy F, wout = u0 + cw F (F at
// u = w - G p); wprev may be wout's buffer.
template <typename T>
hipError_t launch_stage_zm_yw(const Grid& g, const T* w, const double* p, const T* u0, const T* wprev, double ry,
                              double rw, T* y, double cy, T* wout, double cw, hipStream_t s, const T* mc) {
    launch_stage_zm_tile<T, 64, 8>(g, w, p, true, u0, y, 0, cy, wout, cw, s, mc, wprev, ry, rw);
    return hipGetLastError();
}
template hipError_t launch_stage_zm_yw<double>(const Grid&, const double*, const double*, const double*, const double*,
                                               double, double, double*, double, double*, double, hipStream_t,
                                               const double*);
template hipError_t launch_stage_zm_yw<float>(const Grid&, const float*, const double*, const float*, const float*,
                                              double, double, float*, double, float*, double, hipStream_t,
                                              const float*);

template hipError_t launch_stage_zm<double>(const Grid&, const double*, const double*, bool, const double*, double*, bool,
                                            double, double*, double, hipStream_t, const double*);
template hipError_t launch_stage_zm<float>(const Grid&, const float*, const double*, bool, const float*, float*, bool,
                                           double, float*, double, hipStream_t, const float*);

// All-float32 comparison mode: float32 pressure and projection arithmetic.
hipError_t launch_stage_zm_f32(const Grid& g, const float* w, const float* p, bool proj, const float* u0, float* y,
                               bool yinit, double cy, float* wout, double cw, hipStream_t s) {
    launch_stage_zm_tile<float, 64, 8, float>(g, w, p, proj, u0, y, yinit ? 1 : 0, cy, wout, cw, s, nullptr);
    return hipGetLastError();
}

}  // namespace ins

namespace ins {

// Reverse RK4 stage for 3D grids as a z-march (counterpart of k_stage_vjp in
// k_vjp.hip, same arithmetic). Two LDS rings hold, per plane, the stage
// velocity u_i = w - G p and the right-hand-side cotangent
// Fbar_i = cb ybar + cw (un - G q) on the tile plus halo; four slots each and
// the same load/compute pipeline as k_stage_zm.
template <typename T, bool PROJ_U, bool HAS_W>
__global__ __launch_bounds__(kBlock) void k_stage_vjp_zm(Grid g, const T* __restrict__ w, const double* __restrict__ p,
                                                           const T* __restrict__ ybar, const T* __restrict__ un,
                                                           const double* __restrict__ q, T cb, T cw,
                                                           T* __restrict__ u0bar, int mode, T* __restrict__ ubar_out,
                                                           int zc, T* __restrict__ fbar_out) {
    __shared__ T ru[3][3][kZmHP];
    __shared__ T rf[3][3][kZmHP];
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int ntx = (nx + kZmTX - 1) / kZmTX, nty = (ny + kZmTY - 1) / kZmTY, nzc = (nz + zc - 1) / zc;
    int L = xcd_logical(blockIdx.x, gridDim.x);
    const int tx = L % ntx;
    L /= ntx;
    const int ty = L % nty;
    L /= nty;
    const int zci = L % nzc;
    const int b = L / nzc;
    const int x0 = tx * kZmTX, y0 = ty * kZmTY, z0 = zci * zc;
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

    int hq[2], hxy[2], hxp[2], hyp[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int qi = threadIdx.x + s * kBlock;
        hq[s] = qi;
        const int qq = qi < kZmHP ? qi : 0;
        const int gx = pmod(x0 - 1 + qq % kZmHX, nx);
        const int gy = pmod(y0 - 1 + qq / kZmHX, ny);
        hxy[s] = gy * nx + gx;
        hxp[s] = gy * nx + (gx + 1 == nx ? 0 : gx + 1);
        hyp[s] = (gy + 1 == ny ? 0 : gy + 1) * nx + gx;
    }
    const int lx = threadIdx.x % kZmTX, ly = threadIdx.x / kZmTX;
    const int cxg = x0 + lx, cyg = y0 + ly;
    const bool valid = cxg < nx && cyg < ny;
    const int centre = (ly + 1) * kZmHX + (lx + 1);

    if constexpr (!(PROJ_U && HAS_W && sizeof(T) == 8)) {
        // Raw halo loads (w, ybar and, with PROJ_U / HAS_W, p and un, q at the
        // cell and at its +x, +y, +z neighbours), combined into u_i and Fbar_i
        // only when the plane is parked, and every load of the plane loop
        // issued unconditionally (slots past the halo load a valid position;
        // the last iteration fetches its own last plane again; pointwise cells
        // and planes clamped), so the compiler's wait counts are exact and a
        // plane's compute does not wait for the next plane's loads (256^3:
        // the last RK stage's pullback 0.604 -> 0.499 ms, the first's 0.609 ->
        // 0.590 ms). With HAS_W the cell's un - G q is recovered from its parked
        // Fbar = cb ybar + cw (un - G q), so the pointwise inputs are the
        // accumulated cotangent and ybar (6 values instead of 10). The float64
        // instance with a projection and a second cotangent keeps the schedule
        // below: its raw halo needs 184 registers (2 waves per SIMD instead of
        // 3; 0.778 vs 0.771 ms, and 0.977 ms capped at 168 with a spill).
        const int cxy = min(cyg, ny - 1) * nx + min(cxg, nx - 1);
        T hw[2][3], hy[2][3], hu[2][3];
        double hp[2][4], hqv[2][4];
        auto fetch_raw = [&](int zz) {
            const int zoff = zz * plane;
            const int zpo = (zz + 1 == nz ? 0 : zz + 1) * plane;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int j = zoff + hxy[s];
                const int jp[3] = {zoff + hxp[s], zoff + hyp[s], zpo + hxy[s]};
                if constexpr (PROJ_U) hp[s][0] = pb[j];
                if constexpr (HAS_W) hqv[s][0] = qb[j];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    hw[s][c] = wb[c * nc + j];
                    hy[s][c] = yb[c * nc + j];
                    if constexpr (PROJ_U) hp[s][c + 1] = pb[jp[c]];
                    if constexpr (HAS_W) {
                        hu[s][c] = ub[c * nc + j];
                        hqv[s][c + 1] = qb[jp[c]];
                    }
                }
            }
        };
        auto park_raw = [&](int k) {
            T* su = &ru[k % 3][0][0];
            T* sf = &rf[k % 3][0][0];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                if (hq[s] < kZmHP) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        T uv = hw[s][c];
                        if constexpr (PROJ_U) uv = T(double(hw[s][c]) - (hp[s][c + 1] - hp[s][0]) * g.ih[c]);
                        T fv = cb * hy[s][c];
                        if constexpr (HAS_W) fv += cw * T(double(hu[s][c]) - (hqv[s][c + 1] - hqv[s][0]) * g.ih[c]);
                        su[c * kZmHP + hq[s]] = uv;
                        sf[c * kZmHP + hq[s]] = fv;
                    }
                }
            }
        };
        // the accumulated cotangent (ybar or u0bar) of the plane computed next,
        // issued after the current plane's stores
        const T* accb = (mode == 0 || mode == 3) ? yb : u0bar + boff;
        T nacc[3] = {T(0), T(0), T(0)}, nyb[3] = {T(0), T(0), T(0)};
        auto fetch_acc = [&](int z) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                nacc[a] = accb[int64_t(a) * nc + z * plane + cxy];
                if constexpr (HAS_W) nyb[a] = yb[int64_t(a) * nc + z * plane + cxy];
            }
        };
        // un - G q at the cell, recovered from the parked Fbar = cb ybar + cw (un - G q)
        const T rcw = HAS_W ? T(1) / cw : T(0);
        const int nk = (z1 - z0) + 2;
        fetch_raw(pmod(z0 - 1, nz));
        park_raw(0);
        fetch_raw(pmod(z0, nz));
        park_raw(1);
        fetch_raw(pmod(z0 + 1, nz));
        park_raw(2);
        fetch_acc(z0);
        __syncthreads();
        for (int k = 2; k < nk; ++k) {
            const int z = z0 + k - 2;
            fetch_raw(pmod(z0 - 1 + min(k + 1, nk - 1), nz));
            LdsSrc<T> U{&ru[(k - 2) % 3][0][0], &ru[(k - 1) % 3][0][0], &ru[k % 3][0][0], centre};
            LdsSrc<T> F{&rf[(k - 2) % 3][0][0], &rf[(k - 1) % 3][0][0], &rf[k % 3][0][0], centre};
            T out[3];
            rhs_vjp_cell<T, 3>(g, U, F, Nb{}, out);
            if (valid) {
                const int c0 = z * plane + cyg * nx + cxg;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int64_t kk = boff + int64_t(a) * nc + c0;
                    T acc = nacc[a];
                    if constexpr (HAS_W) acc += (rf[(k - 1) % 3][a][centre] - cb * nyb[a]) * rcw;
                    if (u0bar) st_stream(mode >= 2 ? acc + out[a] : acc, u0bar + kk);
                    if (ubar_out) st_stream(out[a], ubar_out + kk);
                    if (fbar_out) fbar_out[kk] = rf[(k - 1) % 3][a][centre];
                }
            }
            fetch_acc(min(z + 1, z1 - 1));
            // slot (k+1) % 3 is the one just read as plane z-1: wait for every reader
            __syncthreads();
            if (k + 1 < nk) park_raw(k + 1);
            __syncthreads();
        }
        return;
    }

    T pu[2][3], pf[2][3];
    auto fetch = [&](int zz) {
        const int zoff = zz * plane;
        const int zpo = (zz + 1 == nz ? 0 : zz + 1) * plane;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (hq[s] < kZmHP) {
                const int j = zoff + hxy[s];
                const int jp[3] = {zoff + hxp[s], zoff + hyp[s], zpo + hxy[s]};
                double pc = 0.0, qc = 0.0;
                if constexpr (PROJ_U) pc = pb[j];
                if constexpr (HAS_W) qc = qb[j];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if constexpr (PROJ_U)
                        pu[s][c] = T(double(wb[c * nc + j]) - (pb[jp[c]] - pc) * g.ih[c]);
                    else
                        pu[s][c] = wb[c * nc + j];
                    T fv = cb * yb[c * nc + j];
                    if constexpr (HAS_W) fv += cw * T(double(ub[c * nc + j]) - (qb[jp[c]] - qc) * g.ih[c]);
                    pf[s][c] = fv;
                }
            }
        }
    };
    auto park = [&](int k) {
        T* su = &ru[k % 3][0][0];
        T* sf = &rf[k % 3][0][0];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (hq[s] < kZmHP) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    su[c * kZmHP + hq[s]] = pu[s][c];
                    sf[c * kZmHP + hq[s]] = pf[s][c];
                }
            }
        }
    };

    // pointwise inputs of the plane computed next, loaded one plane ahead and
    // combined only when used (so the loads stay in flight through a plane):
    // the accumulated cotangent (ybar or u0bar) and, with HAS_W, un and q at the
    // cell and q at its +x, +y, +z neighbours
    T nacc[3] = {T(0), T(0), T(0)}, nun[3] = {T(0), T(0), T(0)};
    double nq[3] = {0.0, 0.0, 0.0}, nqc = 0.0;
    auto fetch_point = [&](int z) {
        if (!valid) return;
        const int cyx = cyg * nx + cxg;
        const int c0 = z * plane + cyx;
        const int jpc[3] = {z * plane + cyg * nx + (cxg + 1 == nx ? 0 : cxg + 1),
                            z * plane + (cyg + 1 == ny ? 0 : cyg + 1) * nx + cxg,
                            (z + 1 == nz ? 0 : z + 1) * plane + cyx};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int64_t kk = boff + int64_t(a) * nc + c0;
            nacc[a] = (mode == 0 || mode == 3) ? yb[int64_t(a) * nc + c0] : ld_stream(u0bar + kk);
            if constexpr (HAS_W) {
                nun[a] = ub[int64_t(a) * nc + c0];
                nq[a] = qb[jpc[a]];
            }
        }
        if constexpr (HAS_W) nqc = qb[c0];
    };

    const int nk = (z1 - z0) + 2;
    fetch(pmod(z0 - 1, nz));
    park(0);
    fetch(pmod(z0, nz));
    park(1);
    fetch(pmod(z0 + 1, nz));
    park(2);
    fetch_point(z0);
    __syncthreads();
    for (int k = 2; k < nk; ++k) {
        const int z = z0 + k - 2;
        const bool more = k + 1 < nk;
        if (more) fetch(pmod(z0 - 1 + k + 1, nz));
        T acc[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            acc[a] = nacc[a];
            if constexpr (HAS_W) acc[a] += T(double(nun[a]) - (nq[a] - nqc) * g.ih[a]);
        }
        if (more) fetch_point(z + 1);
        if (valid) {
            const int c0 = z * plane + cyg * nx + cxg;
            LdsSrc<T> U{&ru[(k - 2) % 3][0][0], &ru[(k - 1) % 3][0][0], &ru[k % 3][0][0], centre};
            LdsSrc<T> F{&rf[(k - 2) % 3][0][0], &rf[(k - 1) % 3][0][0], &rf[k % 3][0][0], centre};
            T out[3];
            rhs_vjp_cell<T, 3>(g, U, F, Nb{}, out);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int64_t kk = boff + int64_t(a) * nc + c0;
                if (u0bar) st_stream(mode >= 2 ? acc[a] + out[a] : acc[a], u0bar + kk);
                if (ubar_out) st_stream(out[a], ubar_out + kk);
                if (fbar_out) fbar_out[kk] = rf[(k - 1) % 3][a][centre];
            }
        }
        // slot (k+1) % 3 is the one just read as plane z-1: wait for every reader
        __syncthreads();
        if (more) park(k + 1);
        __syncthreads();
    }
}

template <typename T>
hipError_t launch_stage_vjp_zm(const Grid& g, const T* w, const double* p, bool proj_u, const T* ybar, const T* un,
                               const double* q, bool has_w, double cb, double cw, T* u0bar, int mode, T* ubar_out,
                               hipStream_t s, T* fbar_out) {
    if (has_w && cw == 0.0) return hipErrorInvalidValue;  // un - G q is recovered through 1 / cw
    const int zc = zm_chunk(g);
    const int nblk = ((g.nx + kZmTX - 1) / kZmTX) * ((g.ny + kZmTY - 1) / kZmTY) * ((g.nz + zc - 1) / zc) * g.batch;
    const T tb = T(cb), tw = T(cw);
#define INS_VJP_ZM(PU, HW)                                                                                           \
    hipLaunchKernelGGL((k_stage_vjp_zm<T, PU, HW>), dim3(nblk), dim3(kBlock), 0, s, g, w, p, ybar, un, q, tb, tw, u0bar, \
                       mode, ubar_out, zc, fbar_out)
    if (proj_u && has_w)
        INS_VJP_ZM(true, true);
    else if (proj_u)
        INS_VJP_ZM(true, false);
    else if (has_w)
        INS_VJP_ZM(false, true);
    else
        INS_VJP_ZM(false, false);
#undef INS_VJP_ZM
    return hipGetLastError();
}

template hipError_t launch_stage_vjp_zm<double>(const Grid&, const double*, const double*, bool, const double*,
                                                const double*, const double*, bool, double, double, double*, int,
                                                double*, hipStream_t, double*);
template hipError_t launch_stage_vjp_zm<float>(const Grid&, const float*, const double*, bool, const float*,
                                               const float*, const double*, bool, double, double, float*, int, float*,
                                               hipStream_t, float*);

}  // namespace ins
