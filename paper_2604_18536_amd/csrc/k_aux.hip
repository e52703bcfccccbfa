// Diagnostics and bandwidth calibration: field statistics (kinetic energy,
// max |u|, max |D u|, finiteness) and a plain streaming copy.
#include "k_common.hpp"

namespace ins {

int stats_blocks(const Grid& g) { return stencil_blocks(g); }

// Statistics of one cell of tile t accumulated into s2 (sum u^2), mu
// (max |u|), md (max |D u|) and nf (count of non-finite entries).
template <typename T, int DIM>
__device__ __forceinline__ void stats_cell(const Grid& g, const T* __restrict__ u, const TileIdx& t, double& s2,
                                           double& mu, double& md, double& nf) {
    const Nb nb = make_nb<DIM>(g, t.x, t.y, t.z);
    const T* ub = u + int64_t(t.b) * DIM * g.ncell;
    const int c0 = nb.at(0, 0, 0);
    double dv = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double v = ub[a * g.ncell + c0];
        const double vm = ub[a * g.ncell + nb.at(-(a == 0), -(a == 1), -(a == 2))];
        s2 += v * v;
        mu = fmax(mu, fabs(v));
        nf += isfinite(v) ? 0.0 : 1.0;
        const int ca = a == 0 ? t.x : (a == 1 ? t.y : t.z);
        // stretched grid: 1 / w of this cell per direction; channel: 1 / w_j along y
        dv += (v - vm) * (g.gm[a] ? g.gm[a][ca + 1] : ((a == 1 && g.ym) ? g.ym[t.y] : g.ih[a]));
    }
    md = fmax(md, fabs(dv));
}

// Workgroup reduction of the four statistics (sums and maxima, fixed order);
// thread i < 4 writes statistic i to out[i].
__device__ __forceinline__ void stats_block_store(double s2, double mu, double md, double nf, double* out) {
    __shared__ double sh[4][kBlock];
    const int i = threadIdx.x;
    sh[0][i] = s2;
    sh[1][i] = mu;
    sh[2][i] = md;
    sh[3][i] = nf;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (i < w) {
            sh[0][i] += sh[0][i + w];
            sh[1][i] = fmax(sh[1][i], sh[1][i + w]);
            sh[2][i] = fmax(sh[2][i], sh[2][i + w]);
            sh[3][i] += sh[3][i + w];
        }
        __syncthreads();
    }
    if (i < 4) out[i] = sh[i][0];
}

// Per-workgroup partials: [4*blk + 0] = sum u^2, +1 = max|u|, +2 = max|Du|,
// +3 = count of non-finite entries. Reduced on the host.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_stats(Grid g, const T* __restrict__ u, double* __restrict__ part) {
    const TileIdx t = tile_of(g);
    double s2 = 0.0, mu = 0.0, md = 0.0, nf = 0.0;
    if (t.valid) stats_cell<T, DIM>(g, u, t, s2, mu, md, nf);
    stats_block_store(s2, mu, md, nf, part + 4 * int64_t(blockIdx.x));
}

// The same partials from a capped number of workgroups (the allocation-free
// entry point's fixed scratch): workgroup k walks tiles k, k + gridDim.x, ...
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_stats_capped(Grid g, const T* __restrict__ u, double* __restrict__ part,
                                                          int ntiles) {
    double s2 = 0.0, mu = 0.0, md = 0.0, nf = 0.0;
    for (int k = blockIdx.x; k < ntiles; k += gridDim.x) {
        const TileIdx t = tile_at(g, k);
        if (t.valid) stats_cell<T, DIM>(g, u, t, s2, mu, md, nf);
    }
    stats_block_store(s2, mu, md, nf, part + 4 * int64_t(blockIdx.x));
}

// One workgroup: the nblk partials reduced in a fixed order into out[0..3]
// (kinetic energy = s2 * ke_scale, max |u|, max |D u|, 1 if all finite).
__global__ __launch_bounds__(kBlock) void k_stats_final(const double* __restrict__ part, int nblk, double ke_scale,
                                                         double* __restrict__ out) {
    double s2 = 0.0, mu = 0.0, md = 0.0, nf = 0.0;
    for (int k = threadIdx.x; k < nblk; k += kBlock) {
        s2 += part[4 * k];
        mu = fmax(mu, part[4 * k + 1]);
        md = fmax(md, part[4 * k + 2]);
        nf += part[4 * k + 3];
    }
    __shared__ double res[4];
    stats_block_store(s2, mu, md, nf, res);
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = ke_scale * res[0];
        out[1] = res[1];
        out[2] = res[2];
        out[3] = res[3] == 0.0 ? 1.0 : 0.0;
    }
}

template <typename T>
hipError_t launch_stats(const Grid& g, const T* u, double* partial, int nblocks, hipStream_t s) {
    if (g.dim == 3)
        hipLaunchKernelGGL((k_stats<T, 3>), dim3(nblocks), dim3(kBlock), 0, s, g, u, partial);
    else
        hipLaunchKernelGGL((k_stats<T, 2>), dim3(nblocks), dim3(kBlock), 0, s, g, u, partial);
    return hipGetLastError();
}

template hipError_t launch_stats<double>(const Grid&, const double*, double*, int, hipStream_t);
template hipError_t launch_stats<float>(const Grid&, const float*, double*, int, hipStream_t);

int stats_capped_blocks(const Grid& g) {
    const int n = stencil_blocks(g);
    return n < kStatsCapBlocks ? n : kStatsCapBlocks;
}

template <typename T>
hipError_t launch_stats_capped(const Grid& g, const T* u, double* partial, double* out, hipStream_t s) {
    const int ntiles = stencil_blocks(g);
    const int nblk = stats_capped_blocks(g);
    if (g.dim == 3)
        hipLaunchKernelGGL((k_stats_capped<T, 3>), dim3(nblk), dim3(kBlock), 0, s, g, u, partial, ntiles);
    else
        hipLaunchKernelGGL((k_stats_capped<T, 2>), dim3(nblk), dim3(kBlock), 0, s, g, u, partial, ntiles);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const double ke_scale = 0.5 / (double(g.ncell) * g.batch);
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(kBlock), 0, s, partial, nblk, ke_scale, out);
    return hipGetLastError();
}

template hipError_t launch_stats_capped<double>(const Grid&, const double*, double*, double*, hipStream_t);
template hipError_t launch_stats_capped<float>(const Grid&, const float*, double*, double*, hipStream_t);

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// One 16-byte element per thread, non-temporal: the fastest copy shape measured
// on MI355X (about 6.2 TB/s read + write).
__global__ __launch_bounds__(kBlock) void k_stream_copy(const v4u* __restrict__ src, v4u* __restrict__ dst, int64_t n16) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_stream_copy(const void* src, void* dst, size_t nbytes, hipStream_t s) {
    const int64_t n16 = int64_t(nbytes / 16);
    const int64_t chunk = int64_t(1) << 30;  // elements per launch keeps the grid size in range
    for (int64_t off = 0; off < n16; off += chunk) {
        const int64_t n = n16 - off < chunk ? n16 - off : chunk;
        const int nblk = int((n + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_stream_copy, dim3(nblk), dim3(kBlock), 0, s, reinterpret_cast<const v4u*>(src) + off,
                           reinterpret_cast<v4u*>(dst) + off, n);
    }
    return hipGetLastError();
}

}  // namespace ins

namespace ins {

// Face filter (DNS -> LES): coarse cell I covers fine cells f*I .. f*I+f-1; its
// a-face is the right a-face of fine cell f*I+f-1 along a, and the f^(d-1)
// fine a-faces covering it are averaged. A discretely solenoidal field stays
// discretely solenoidal (the coarse divergence is the volume mean of the fine one).
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_face_filter(Grid g, int f, const T* __restrict__ u, T* __restrict__ uc) {
    const int cx = g.nx / f, cy = g.ny / f, cz = DIM == 3 ? g.nz / f : 1;
    const int64_t nco = int64_t(cx) * cy * cz;
    const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (t >= nco * DIM * g.batch) return;
    const int64_t cell = t % nco;
    const int a = int((t / nco) % DIM);
    const int b = int(t / (nco * DIM));
    const int ix = int(cell % cx), iy = int((cell / cx) % cy), iz = int(cell / (int64_t(cx) * cy));
    const int base[3] = {ix * f, iy * f, iz * f};
    const int n2 = DIM == 3 ? f : 1;
    const T* ua = u + (int64_t(b) * DIM + a) * g.ncell;
    double acc = 0.0;
    for (int j2 = 0; j2 < n2; ++j2) {
        for (int j1 = 0; j1 < f; ++j1) {
            // the two directions other than a run over f fine faces; a is fixed at f*I+f-1
            int c[3] = {base[0], base[1], base[2]};
            c[a] += f - 1;
            const int o1 = a == 0 ? 1 : 0;
            const int o2 = a == 2 ? 1 : 2;
            c[o1] += j1;
            if (DIM == 3) c[o2] += j2;
            acc += double(ua[(int64_t(c[2]) * g.ny + c[1]) * g.nx + c[0]]);
        }
    }
    const double inv = 1.0 / double(f * n2);
    uc[(int64_t(b) * DIM + a) * nco + cell] = T(acc * inv);
}

template <typename T>
hipError_t launch_face_filter(const Grid& fine, int f, const T* u, T* uc, hipStream_t s) {
    const int64_t nco = int64_t(fine.nx / f) * (fine.ny / f) * (fine.dim == 3 ? fine.nz / f : 1);
    const int64_t nthr = nco * fine.dim * fine.batch;
    const int nblk = int((nthr + kBlock - 1) / kBlock);
    if (fine.dim == 3)
        hipLaunchKernelGGL((k_face_filter<T, 3>), dim3(nblk), dim3(kBlock), 0, s, fine, f, u, uc);
    else
        hipLaunchKernelGGL((k_face_filter<T, 2>), dim3(nblk), dim3(kBlock), 0, s, fine, f, u, uc);
    return hipGetLastError();
}

template hipError_t launch_face_filter<double>(const Grid&, int, const double*, double*, hipStream_t);
template hipError_t launch_face_filter<float>(const Grid&, int, const float*, float*, hipStream_t);

// Shell binning of one half spectrum [batch][nz][ny][sx] (columns 0 .. nx/2 in
// use): every stored kx in (0, nx/2) stands for the pair kx, -kx and counts twice.
__global__ __launch_bounds__(kBlock) void k_spectrum_bins(Grid g, const cd* __restrict__ spec, double* __restrict__ bins,
                                                            int nbins) {
    const int nxh = g.nx / 2 + 1;
    const int64_t per = int64_t(nxh) * g.ny * g.nz;
    const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (t >= per * g.batch) return;
    const int b = int(t / per);
    const int64_t r = t % per;
    const int kx = int(r % nxh);
    const int ky0 = int((r / nxh) % g.ny);
    const int kz0 = int(r / (int64_t(nxh) * g.ny));
    const int ky = ky0 <= g.ny / 2 ? ky0 : ky0 - g.ny;
    const int kz = kz0 <= g.nz / 2 ? kz0 : kz0 - g.nz;
    const double kk = sqrt(double(kx) * kx + double(ky) * ky + double(kz) * kz);
    const int shell = int(floor(kk + 0.5));
    if (shell >= nbins) return;
    const cd v = spec[(int64_t(b) * g.nz * g.ny + int64_t(kz0) * g.ny + ky0) * g.sx + kx];
    const double w = (kx == 0 || 2 * kx == g.nx) ? 1.0 : 2.0;
    const double n = double(g.ncell);
    atomicAdd(&bins[int64_t(b) * nbins + shell], 0.5 * w * (v.x * v.x + v.y * v.y) / (n * n));
}

__global__ void k_fill_zero(double* __restrict__ p, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

hipError_t launch_fill_zero(double* p, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_zero, dim3(int((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, p, int64_t(n));
    return hipGetLastError();
}

__global__ void k_fill_zero_f(float* __restrict__ p, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

hipError_t launch_fill_zero_f(float* p, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_zero_f, dim3(int((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, p, int64_t(n));
    return hipGetLastError();
}

hipError_t launch_spectrum_bins(const Grid& g, const cd* spec, double* bins, int nbins, hipStream_t s) {
    const int64_t n = int64_t(g.nx / 2 + 1) * g.ny * g.nz * g.batch;
    hipLaunchKernelGGL(k_spectrum_bins, dim3(int((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, g, spec, bins, nbins);
    return hipGetLastError();
}

}  // namespace ins
