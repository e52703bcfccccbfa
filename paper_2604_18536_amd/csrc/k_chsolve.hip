// Direct pressure solve of the channel grid (x and z periodic and uniform, y
// bounded by walls, uniform or stretched).
//
// Fourier modes in x and z diagonalise the periodic parts of D G (Sec. 2.6.1
// transfer function, 4 sin^2(pi k / n) / h^2 per direction), so after forward
// FFTs along x and z every wavenumber pair (k_x, k_z) leaves one tridiagonal
// system along y: the Neumann second difference across the stretched widths,
// shifted by the periodic eigenvalue. The paper solves its uniform channel with
// FFTs in the periodic directions and a type-II cosine transform along y
// (Sec. 6, DNS on a uniform grid); that transform diagonalises exactly this
// uniform Neumann operator, so the tridiagonal solve yields the same discrete
// pressure there and, unchanged, on a stretched y, where the paper falls back
// to its sparse direct or iterative solver.
//
// Row j of the system for the mode with periodic eigenvalue lam >= 0, scaled by
// the row width w_j so that it is symmetric:
//   a_j p_{j-1} + b_j p_j + c_j p_{j+1} = w_j r_j,
//   a_j = 1/d_{j-1} (0 at j = 0), c_j = 1/d_j (0 at j = n_y - 1),
//   b_j = -(a_j + c_j) - lam w_j.
// Every mode but (0, 0) is strictly diagonally dominant. The (0, 0) mode is
// the singular Neumann problem: its right-hand side loses its volume-weighted
// mean (the augmented system of the direct solver sets L p = r - mean_w r),
// row 0 is replaced by p_0 = 0, and the unweighted mean is removed afterwards
// (zero-mean pressure). Only this mode carries means: every other mode sums
// to zero over x and z.
//
// Parallel scheme (partition method): a line of n_y rows is split over P
// threads, each holding a segment of m >= 2 consecutive rows in registers. A
// thread eliminates inside its segment until each row depends only on the
// segment's first and last unknowns; those 2P unknowns of the line form a
// tridiagonal system, reduced in LDS by cyclic reduction (every equation
// eliminates its neighbours at distance 1, 2, 4, ...). Each thread then
// recovers its interior rows from the two boundary values. Global memory is
// read and written once; the lines of a workgroup are adjacent k_x, so every
// row access is a contiguous run.
#include "k_common.hpp"

namespace ins {

namespace {

// Sum over the P segments of line l of per-thread values, in a fixed order so
// that every thread of the line gets the same bits. Called by all threads.
template <int P, int L>
__device__ __forceinline__ cd line_sum(cd v, cd* red, int s, int l) {
    red[s * L + l] = v;
    __syncthreads();
    cd t = {0.0, 0.0};
#pragma unroll 4
    for (int q = 0; q < P; ++q) t = cadd(t, red[q * L + l]);
    __syncthreads();
    return t;
}

}  // namespace

// One workgroup of NT threads: L = NT / P lines (adjacent k_x at one k_z of one
// field), P threads per line (thread = s L + l: segment s of line l), at most MR
// rows per segment. ADJ: the transpose of the solve (see launch_channel_ysolve).
template <int MR, int P, int NT, bool ADJ>
__global__ __launch_bounds__(NT) void k_channel_ysolve(Grid g, cd* __restrict__ spec, const double* __restrict__ lamx,
                                                       const double* __restrict__ lamz, double wysum, double scale) {
    constexpr int L = NT / P;
    __shared__ double ra[2 * P * L], rc[2 * P * L];
    __shared__ cd rd[2 * P * L];
    __shared__ cd red[P * L];
    const int nxh = g.nx / 2 + 1;
    const int ny = g.ny, S = g.ny + 2;
    const double* ym = g.ym;
    const int nchunk = (nxh + L - 1) / L;
    const int wg = xcd_logical(blockIdx.x, gridDim.x);
    const int outer = wg / nchunk;  // field * n_z + k_z
    const int kx0 = (wg - outer * nchunk) * L;
    const int kz = outer % g.nz;
    const int l = threadIdx.x % L, s = threadIdx.x / L;
    const int kx = kx0 + l;
    const bool valid = kx < nxh;
    const bool wg_zero = kx0 == 0 && kz == 0;  // uniform over the workgroup
    const bool zero = wg_zero && l == 0;       // the (0, 0) mode's line
    const int j0 = s * ny / P;
    const int m = (s + 1) * ny / P - j0;  // >= 2
    const double lam = valid ? lamx[kx] + lamz[kz] : 1.0;
    cd* line = spec + int64_t(outer) * ny * g.sx + (valid ? kx : 0);

    cd D[MR];
    double A[MR], C[MR];
#pragma unroll
    for (int i = 0; i < MR; ++i) D[i] = (valid && i < m) ? line[int64_t(j0 + i) * g.sx] : cd{0.0, 0.0};

    // right-hand side in the symmetric form, w_j r_j
    if (ADJ && wg_zero) {
        // transpose: subtract the unweighted mean of the (0, 0) line first
        cd t = {0.0, 0.0};
#pragma unroll
        for (int i = 0; i < MR; ++i)
            if (i < m) t = cadd(t, D[i]);
        t = line_sum<P, L>(t, red, s, l);
        if (zero) {
            const cd mu = cscale(t, 1.0 / ny);
#pragma unroll
            for (int i = 0; i < MR; ++i) D[i] = csub(D[i], mu);
        }
    }
    if (ADJ) {
#pragma unroll
        for (int i = 0; i < MR; ++i)
            if (i < m) D[i] = cscale(D[i], ym[j0 + i]);  // / w_j
    }
    if (wg_zero) {
        cd t = {0.0, 0.0};
#pragma unroll
        for (int i = 0; i < MR; ++i)
            if (i < m) t = cadd(t, cscale(D[i], ym[3 * S + j0 + i]));
        t = line_sum<P, L>(t, red, s, l);
        if (zero) {
            const cd mw = cscale(t, 1.0 / wysum);
#pragma unroll
            for (int i = 0; i < MR; ++i) D[i] = csub(D[i], mw);
        }
    }

    // elimination inside the segment: row i becomes
    //   A_i x_first + x_i + C_i x_{i+1} = D_i   (row 0: A_0 multiplies x_{-1})
#pragma unroll
    for (int i = 0; i < MR; ++i) {
        if (i < m) {
            const int j = j0 + i;
            const double w = ym[3 * S + j];
            double a = j > 0 ? ym[S + j] : 0.0;
            double c = j < ny - 1 ? ym[S + j + 1] : 0.0;
            double b = -(a + c) - lam * w;
            cd rhs = cscale(D[i], w);
            if (zero && j == 0) {
                a = 0.0;
                c = 0.0;
                b = 1.0;
                rhs = cd{0.0, 0.0};
            }
            if (i < 2) {
                const double r = 1.0 / b;
                A[i] = a * r;
                C[i] = c * r;
                D[i] = cscale(rhs, r);
            } else {
                const double r = 1.0 / (b - a * C[i - 1]);
                A[i] = -a * A[i - 1] * r;
                C[i] = c * r;
                D[i] = cscale(csub(rhs, cscale(D[i - 1], a)), r);
            }
        }
    }
    // back substitution towards row 1: x_i = D_i - A_i x_first - C_i x_last
    // (row m - 2 is already of that form; row m - 1 is x_last itself)
#pragma unroll
    for (int i = MR - 3; i >= 1; --i) {
        if (i <= m - 3) {
            D[i] = csub(D[i], cscale(D[i + 1], C[i]));
            A[i] = A[i] - C[i] * A[i + 1];
            C[i] = -C[i] * C[i + 1];
        }
    }
    // the two equations of the reduced system: first row (index 2s) and last row (2s + 1)
    double ea[2], ec[2];
    cd ed[2];
    if (m == 2) {
        ea[0] = A[0];
        ec[0] = C[0];
        ed[0] = D[0];
    } else {
        const double inv = 1.0 / (1.0 - C[0] * A[1]);
        ea[0] = A[0] * inv;
        ec[0] = -C[0] * C[1] * inv;
        ed[0] = cscale(csub(D[0], cscale(D[1], C[0])), inv);
    }
#pragma unroll
    for (int i = 1; i < MR; ++i) {
        if (i == m - 1) {
            ea[1] = A[i];
            ec[1] = C[i];
            ed[1] = D[i];
        }
    }

    // cyclic reduction of the 2P equations of each line in LDS
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int k = (2 * s + e) * L + l;
        ra[k] = ea[e];
        rc[k] = ec[e];
        rd[k] = ed[e];
    }
    __syncthreads();
#pragma unroll
    for (int dl = 1; dl < 2 * P; dl *= 2) {
        double na[2], nc[2];
        cd nd[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int q = 2 * s + e;
            double alo = 0.0, clo = 0.0, ahi = 0.0, chi = 0.0;
            cd dlo = {0.0, 0.0}, dhi = {0.0, 0.0};
            if (q - dl >= 0) {
                const int k = (q - dl) * L + l;
                alo = ra[k];
                clo = rc[k];
                dlo = rd[k];
            }
            if (q + dl < 2 * P) {
                const int k = (q + dl) * L + l;
                ahi = ra[k];
                chi = rc[k];
                dhi = rd[k];
            }
            const double inv = 1.0 / (1.0 - ea[e] * clo - ec[e] * ahi);
            na[e] = -ea[e] * alo * inv;
            nc[e] = -ec[e] * chi * inv;
            nd[e] = cscale(csub(csub(ed[e], cscale(dlo, ea[e])), cscale(dhi, ec[e])), inv);
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            ea[e] = na[e];
            ec[e] = nc[e];
            ed[e] = nd[e];
            const int k = (2 * s + e) * L + l;
            ra[k] = na[e];
            rc[k] = nc[e];
            rd[k] = nd[e];
        }
        __syncthreads();
    }
    const cd xf = ed[0], xl = ed[1];
    cd X[MR];
#pragma unroll
    for (int i = 0; i < MR; ++i) {
        if (i == 0)
            X[i] = xf;
        else if (i == m - 1)
            X[i] = xl;
        else
            X[i] = csub(csub(D[i], cscale(xf, A[i])), cscale(xl, C[i]));
    }

    // (0, 0) line: zero unweighted mean
    if (wg_zero) {
        cd t = {0.0, 0.0};
#pragma unroll
        for (int i = 0; i < MR; ++i)
            if (i < m) t = cadd(t, X[i]);
        t = line_sum<P, L>(t, red, s, l);
        if (zero) {
            const cd mu = cscale(t, 1.0 / ny);
#pragma unroll
            for (int i = 0; i < MR; ++i) X[i] = csub(X[i], mu);
        }
    }
    if (ADJ) {
        // transpose: subtract the weighted mean of the (0, 0) line, then scale by w_j
        if (wg_zero) {
            cd t = {0.0, 0.0};
#pragma unroll
            for (int i = 0; i < MR; ++i)
                if (i < m) t = cadd(t, cscale(X[i], ym[3 * S + j0 + i]));
            t = line_sum<P, L>(t, red, s, l);
            if (zero) {
                const cd mw = cscale(t, 1.0 / wysum);
#pragma unroll
                for (int i = 0; i < MR; ++i) X[i] = csub(X[i], mw);
            }
        }
#pragma unroll
        for (int i = 0; i < MR; ++i)
            if (i < m) X[i] = cscale(X[i], ym[3 * S + j0 + i]);
    }
    if (valid) {
#pragma unroll
        for (int i = 0; i < MR; ++i)
            if (i < m) line[int64_t(j0 + i) * g.sx] = cscale(X[i], scale);
    }
}

// Segment shape for n_y rows: MR rows at most per thread, P a power of two
// with every segment holding at least 2 rows.
int channel_ysolve_segments(int ny, int& mr) {
    mr = ny <= 1024 ? 16 : 32;
    const int need = (ny + mr - 1) / mr;
    int p = 1;
    while (p < need) p *= 2;
    return p;
}

hipError_t launch_channel_ysolve(const Grid& g, cd* spec, const double* lamx, const double* lamz, double wysum,
                                 double scale, bool adj, hipStream_t s) {
    int mr = 0;
    const int p = channel_ysolve_segments(g.ny, mr);
    // 512 threads when a line takes 32 or 64 segments of at most 16 rows, so a
    // workgroup still holds 16 or 8 adjacent k_x (row accesses of 256 or 128
    // contiguous bytes); 32-row segments keep 256 threads (register budget)
    const int nt = (p >= 32 && mr == 16) ? 512 : 256;
    const int lpw = nt / p;
    const int nxh = g.nx / 2 + 1;
    const int nblk = ((nxh + lpw - 1) / lpw) * g.nz * g.batch;
#define INS_YS(MR, P, NT)                                                                                        \
    do {                                                                                                         \
        if (adj)                                                                                                 \
            hipLaunchKernelGGL((k_channel_ysolve<MR, P, NT, true>), dim3(nblk), dim3(NT), 0, s, g, spec, lamx,  \
                               lamz, wysum, scale);                                                              \
        else                                                                                                     \
            hipLaunchKernelGGL((k_channel_ysolve<MR, P, NT, false>), dim3(nblk), dim3(NT), 0, s, g, spec, lamx, \
                               lamz, wysum, scale);                                                              \
    } while (0)
    if (mr == 16) {
        switch (p) {
            case 1: INS_YS(16, 1, 256); break;
            case 2: INS_YS(16, 2, 256); break;
            case 4: INS_YS(16, 4, 256); break;
            case 8: INS_YS(16, 8, 256); break;
            case 16: INS_YS(16, 16, 256); break;
            case 32: INS_YS(16, 32, 512); break;
            default: INS_YS(16, 64, 512); break;
        }
    } else {
        INS_YS(32, 64, 256);
    }
#undef INS_YS
    return hipGetLastError();
}

}  // namespace ins
