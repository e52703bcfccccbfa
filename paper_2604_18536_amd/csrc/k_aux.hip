// Diagnostics and bandwidth calibration: field statistics (kinetic energy,
// max |u|, max |D u|, finiteness) and a plain streaming copy.
#include "k_common.hpp"

namespace ins {

int stats_blocks(const Grid& g) { return stencil_blocks(g); }

// Per-workgroup partials: [4*blk + 0] = sum u^2, +1 = max|u|, +2 = max|Du|,
// +3 = count of non-finite entries. Reduced on the host.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_stats(Grid g, const T* __restrict__ u, double* __restrict__ part) {
    __shared__ double sh[4][kBlock];
    const TileIdx t = tile_of(g);
    double s2 = 0.0, mu = 0.0, md = 0.0, nf = 0.0;
    if (t.valid) {
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
            dv += (v - vm) * g.ih[a];
        }
        md = fabs(dv);
    }
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
    if (i < 4) part[4 * blockIdx.x + i] = sh[i][0];
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

__global__ __launch_bounds__(kBlock) void k_stream_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                          int64_t n16) {
    const int64_t stride = int64_t(gridDim.x) * kBlock;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

hipError_t launch_stream_copy(const void* src, void* dst, size_t nbytes, hipStream_t s) {
    const int64_t n16 = int64_t(nbytes / 16);
    int64_t nblk = (n16 + kBlock - 1) / kBlock;
    if (nblk > 65536) nblk = 65536;
    if (nblk < 1) nblk = 1;
    hipLaunchKernelGGL(k_stream_copy, dim3(int(nblk)), dim3(kBlock), 0, s, reinterpret_cast<const uint4*>(src),
                       reinterpret_cast<uint4*>(dst), n16);
    return hipGetLastError();
}

}  // namespace ins
