// Internal declarations shared by the runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace ins {

// Complex float64 value of the spectral path.
struct cd {
    double x, y;
};
// Complex float32 value (the all-float32 comparison mode's spectrum).
struct cf {
    float x, y;
};
template <class C>
struct RealOf;
template <>
struct RealOf<cd> {
    using type = double;
};
template <>
struct RealOf<cf> {
    using type = float;
};
template <class C>
using real_of = typename RealOf<C>::type;

// Grid description handed to every kernel by value.
struct Grid {
    int dim;            // 2 or 3
    int nx, ny, nz;     // nz == 1 in 2D
    int batch;
    int64_t ncell;      // nx * ny * nz
    double ih[3];       // 1 / h_a
    double ih2[3];      // 1 / h_a^2
    double nu;
    // channel grid only (null otherwise): y metrics, 5 arrays of stride n_y + 2:
    // [0..n_y) 1 / w_j; [S..S+n_y] 1 / d_j for j = -1 .. n_y - 1; [2S..) theta_j;
    // [3S..) w_j; [4S..4S+n_y] d_j for j = -1 .. n_y - 1. w_j is the width of
    // row j, d_j the distance of the centres around y-face j (mirrored ghosts:
    // d_{-1} = w_0, d_{n_y-1} = w_{n_y-1}), theta_j = w_j / (w_j + w_{j+1}).
    const double* ym;
    // channel grid only: constant body force per component (the forcing term of F), 0 by default
    double force[3];
    // stretched grid (null unless a direction other than the channel's y is
    // stretched): per direction a, 5 arrays of stride n_a + 2 indexed by i + 1
    // for i = -1 .. n_a: 1 / w_i, 1 / d_i, theta_i, w_i, d_i, periodic
    // images (or the mirrored rows beyond a wall) already applied; see k_gen.hip
    const double* gm[3];
    int ywalls;  // stretched grid: 1 when y is bounded by no-slip walls, 0 when periodic
    // row stride of the half spectrum [batch][nz][ny][sx]: n_x/2 + 1 rounded up to a
    // multiple of 8, so every row, and every 8-column chunk of the strided passes,
    // starts on a 128-byte boundary (columns beyond n_x/2 are never touched)
    int sx;
};

// One 1D FFT length: Stockham stages with their radices and twiddle tables.
constexpr int kMaxStages = 12;
struct FftPlan {
    int n;                   // transform length
    int nst;                 // number of stages
    int rad[kMaxStages];     // radix of stage s (applied in order)
    int tw_off[kMaxStages];  // offset in tw of stage s's twiddles: p*(R-1) entries
    int rt_off;              // offset in tw of the roots W_n^j = exp(-2 pi i j / n), j < n
    const cd* tw;            // device twiddle and root tables (float64, forward sign)
    int vm;                  // complex values a thread holds per stage (8 or 16)
    int pad;                 // LDS line-stride padding (0 or 1)
    int nth;                 // threads per workgroup: 256; with vm 8 also 512 (strided passes)
    const cf* twf;           // the same tables rounded to float32 (all-float32 mode; null otherwise)
};

// Which FFT pass shape a launch uses.
struct FftPassCfg {
    int lines;   // lines per workgroup (power of two)
};

// Spectral solve data: 4 sin^2(pi k / n) / h^2 per direction and 1/(#cells).
struct SolveTab {
    const double* lam[3];
    double inv_ncell;
    const float* lamf[3];  // float32 copies (all-float32 mode; null otherwise)
    float inv_ncellf;
};

// Field-type tags for the stencil kernels.
enum class Prec { F64 = 0, F32 = 1 };

// ----------------------------------------------------------------------------
// Launchers (defined in the kernel translation units). All return hipError_t
// from hipGetLastError after the launch.
// ----------------------------------------------------------------------------
// f = F(u) (+ mc when mc != nullptr: the closure term).
template <typename T>
hipError_t launch_rhs(const Grid& g, const T* u, T* f, hipStream_t s, const T* mc = nullptr);
template <typename T>
hipError_t launch_divergence(const Grid& g, const T* u, double* r, hipStream_t s);
template <typename T>
hipError_t launch_gradient(const Grid& g, const double* p, T* gout, hipStream_t s);
template <typename T>
hipError_t launch_div_vjp(const Grid& g, const double* rbar, T* ubar, hipStream_t s);
template <typename T>
hipError_t launch_grad_vjp(const Grid& g, const T* gbar, double* pbar, hipStream_t s);
// u_out = w - G p (float64 arithmetic), u_out may equal w.
template <typename T>
hipError_t launch_apply_projection(const Grid& g, const T* w, const double* p, T* u_out, hipStream_t s);

// RK4 stage: u_i = proj ? w - G p : w; F = rhs(u_i) (+ mc, the closure term at u_i);
//   if y: y = (yinit ? u0 : y) + cy F;  if wout: wout = u0 + cw F.
template <typename T>
hipError_t launch_stage(const Grid& g, const T* w, const double* p, bool proj, const T* u0, T* y, bool yinit, double cy,
                        T* wout, double cw, hipStream_t s, const T* mc = nullptr);

// z planes per workgroup of a z-marching 3D stencil on tx x ty tiles: at most
// zmax, halved while the launch would have fewer than `want` workgroups.
int zm_chunk(const Grid& g, int tx, int ty, int want, int zmax);
// the same for the forward stage kernels (64 x 8 tiles), by field precision
int zm_chunk_stage(const Grid& g, bool fp64);
// 3D variant of launch_stage: 2.5D z-march with an LDS ring of projected planes.
template <typename T>
hipError_t launch_stage_zm(const Grid& g, const T* w, const double* p, bool proj, const T* u0, T* y, bool yinit,
                           double cy, T* wout, double cw, hipStream_t s, const T* mc);
// The projected 3D stage with its accumulator formed from stage inputs instead
// of read: y = u0 + ry (wprev - u0) + rw (w - u0) + cy F, wout = u0 + cw F;
// wprev may be wout's buffer.
template <typename T>
hipError_t launch_stage_zm_yw(const Grid& g, const T* w, const double* p, const T* u0, const T* wprev, double ry,
                              double rw, T* y, double cy, T* wout, double cw, hipStream_t s, const T* mc);

// Spectral Poisson solve pieces.
// Forward x pass: real rows -> half spectrum. vel != nullptr and comp < 0:
// rows are the divergence of vel computed on the fly; vel != nullptr and
// comp >= 0: rows of velocity component comp; else rows come from r.
template <typename T>
hipError_t launch_fft_x_fwd(const Grid& g, const T* vel, const double* r, cd* spec, const FftPlan& px, const cd* post_tw,
                            int lines, hipStream_t s, int comp = -1);
hipError_t launch_fft_x_inv(const Grid& g, const cd* spec, double* p, const FftPlan& px, const cd* post_tw, int lines,
                            hipStream_t s);
// Strided C2C pass over the half spectrum. mode 0: forward, 1: inverse,
// 2: forward + spectral divide + inverse, the inverse running plan `rev` (the
// same length with the radices in reverse order; unused by modes 0 and 1).
// axis 1 = y, 2 = z.
hipError_t launch_fft_strided(const Grid& g, cd* spec, const FftPlan& pl, const FftPlan& rev, int axis, int mode,
                              int lines, const SolveTab& st, hipStream_t s);

// All-float32 comparison mode (float32 velocity and pressure-point fields,
// every operation in float32): divergence, gradient, projection and RK stage
// (no closure term; 3D stages as the z-march).
hipError_t launch_divergence_f32(const Grid& g, const float* u, float* r, hipStream_t s);
hipError_t launch_gradient_f32(const Grid& g, const float* p, float* out, hipStream_t s);
hipError_t launch_apply_projection_f32(const Grid& g, const float* w, const float* p, float* u_out, hipStream_t s);
hipError_t launch_stage_f32(const Grid& g, const float* w, const float* p, bool proj, const float* u0, float* y,
                            bool yinit, double cy, float* wout, double cw, hipStream_t s);
hipError_t launch_stage_zm_f32(const Grid& g, const float* w, const float* p, bool proj, const float* u0, float* y,
                               bool yinit, double cy, float* wout, double cw, hipStream_t s);

// All-float32 comparison mode: the same passes on a float32 half spectrum
// [batch][n_z][n_y][sx] of cf, float32 twiddles (FftPlan::twf), eigenvalues
// (SolveTab::lamf) and pressure-point fields. The forward x pass takes the
// divergence of vel (vel != null) or the rows of r.
hipError_t launch_fft_x_fwd_f32(const Grid& g, const float* vel, const float* r, cf* spec, const FftPlan& px,
                                const cf* post, int lnl, hipStream_t s);
hipError_t launch_fft_x_inv_f32(const Grid& g, const cf* spec, float* p, const FftPlan& px, const cf* post, int lnl,
                                hipStream_t s);
hipError_t launch_fft_strided_f32(const Grid& g, cf* spec, const FftPlan& pl, const FftPlan& rev, int axis, int mode,
                                  int lnl, const SolveTab& st, hipStream_t s);

// Channel grid, direct pressure solve (x, z FFTs + one tridiagonal system
// along y per wavenumber pair). Forward x pass whose rows are the channel
// divergence D vel (scaled: D Omega_u^{-1} vel).
template <typename T>
hipError_t launch_fft_x_fwd_wall(const Grid& g, const T* vel, bool scaled, cd* spec, const FftPlan& px, const cd* post_tw,
                                 int lines, hipStream_t s);
// Tridiagonal solves along y of the half spectrum [batch][n_z][n_y][n_x/2+1]
// (in place), each mode's solution multiplied by `scale`; lamx, lamz the
// periodic eigenvalues 4 sin^2(pi k / n) / h^2, wysum = sum_j w_j. adj: the
// transpose of the solve map.
hipError_t launch_channel_ysolve(const Grid& g, cd* spec, const double* lamx, const double* lamz, double wysum,
                                 double scale, bool adj, hipStream_t s);
// Segments per line (return) and rows per segment bound (mr) of that solve.
int channel_ysolve_segments(int ny, int& mr);
constexpr int kChannelDirectMaxNy = 2048;

// Reverse-pass kernels.
template <typename T>
hipError_t launch_rhs_vjp(const Grid& g, const T* u, const T* fbar, T* ubar, hipStream_t s);
// Reverse Runge-Kutta stage: u_i = (proj_u ? w - G p : w),
// Fbar_i = cb ybar + (has_w ? cw (un - G q) : 0), out = J_F(u_i)^T Fbar_i,
// u0bar = (mode 0 or 3 ? ybar : u0bar) + (has_w ? un - G q : 0) + (mode 2 or 3 ? out : 0),
// ubar_out (if not null) = out, fbar_out (if not null) = Fbar_i; a null u0bar
// (modes 0 and 3, which do not read it) skips that output.
template <typename T>
hipError_t launch_stage_vjp(const Grid& g, const T* w, const double* p, bool proj_u, const T* ybar, const T* un,
                            const double* q, bool has_w, double cb, double cw, T* u0bar, int mode, T* ubar_out,
                            hipStream_t s, T* fbar_out = nullptr);

template <typename T>
hipError_t launch_stage_vjp_zm(const Grid& g, const T* w, const double* p, bool proj_u, const T* ybar, const T* un,
                               const double* q, bool has_w, double cb, double cw, T* u0bar, int mode, T* ubar_out,
                               hipStream_t s, T* fbar_out);

// Smagorinsky closure (k_eddy.hip). forward: nu = c2 sqrt(2 S:S) at pressure
// points, m = sum_b delta_b (2 nu S_ab) on the faces (overwritten). backward:
// ubar += (dm/du)^T mbar at the u of the forward whose nu is passed; P is
// scratch of DIM (DIM + 1) / 2 pressure-point fields per batch entry.
template <typename T>
hipError_t launch_eddy_forward(const Grid& g, const T* u, T* nu, T* m, double c2, hipStream_t s);
template <typename T>
hipError_t launch_eddy_backward(const Grid& g, const T* u, const T* nu, const T* mbar, T* P, T* ubar, double c2,
                                hipStream_t s);

// LES data helpers.
// Coarse staggered field: mean of the f^(d-1) fine a-faces on each coarse a-face.
template <typename T>
hipError_t launch_face_filter(const Grid& fine, int f, const T* u, T* uc, hipStream_t s);
// Accumulate 1/2 |X|^2 / N^2 of one half spectrum into integer-|k| shells (atomic adds).
hipError_t launch_spectrum_bins(const Grid& g, const cd* spec, double* bins, int nbins, hipStream_t s);
// p[0..n) = 0 with a kernel (kept out of hipMemsetAsync so callers may capture it).
hipError_t launch_fill_zero(double* p, size_t n, hipStream_t s);
hipError_t launch_fill_zero_f(float* p, size_t n, hipStream_t s);

// Learned closure (bfloat16 MFMA convolutions). Activations are channels-last
// bfloat16 stored as 16-bit words.
template <typename T>
hipError_t launch_closure_pack_input(const Grid& g, const T* u, unsigned short* x0, hipStream_t s);
hipError_t launch_closure_pack_weights(const float* w, int cin, int cout, int cinp, int ntf, unsigned short* wf,
                                       int coutp, int ntd, unsigned short* wd, hipStream_t s);
// which: 0, 1 hidden layers, 2 output layer; 10, 11 dgrad into hidden layers; 12 dgrad to the input.
template <typename T>
hipError_t launch_closure_conv(const Grid& g, int which, const unsigned short* in, const unsigned short* wpk,
                               const float* bias, const float* zin, float* zout, unsigned short* aout, T* fout,
                               hipStream_t s);
hipError_t launch_closure_wgrad(const Grid& g, int which, const unsigned short* gin, const unsigned short* xin,
                                float* partial, float* wbar, float* bbar, hipStream_t s);
size_t closure_wgrad_partial_floats(int64_t ncells);

// Channel grid (k_walls.hip): no-slip walls at both y ends, x and z periodic.
// Same contracts as the periodic launchers above; the wall face of u^y is
// written as 0 by every velocity output.
template <typename T>
hipError_t launch_wall_rhs(const Grid& g, const T* u, T* f, hipStream_t s);
template <typename T>
hipError_t launch_wall_divergence(const Grid& g, const T* u, double* r, hipStream_t s);
template <typename T>
hipError_t launch_wall_gradient(const Grid& g, const double* p, T* out, hipStream_t s);
// adj: u_out = w - Omega_u G p (the correction of the transposed projection).
template <typename T>
hipError_t launch_wall_project(const Grid& g, const T* w, const double* p, T* u_out, bool adj, hipStream_t s);
template <typename T>
hipError_t launch_wall_rhs_vjp(const Grid& g, const T* u, const T* fbar, T* ubar, hipStream_t s);
template <typename T>
hipError_t launch_wall_div_vjp(const Grid& g, const double* rbar, T* ubar, hipStream_t s);
template <typename T>
hipError_t launch_wall_grad_vjp(const Grid& g, const T* gbar, double* pbar, hipStream_t s);
template <typename T>
hipError_t launch_wall_stage(const Grid& g, const T* w, const double* p, bool proj, const T* u0, T* y, bool yinit,
                             double cy, T* wout, double cw, hipStream_t s);
template <typename T>
hipError_t launch_wall_stage_vjp(const Grid& g, const T* w, const double* p, bool proj_u, const T* ybar, const T* un,
                                 const double* q, bool has_w, double cb, double cw, T* u0bar, int mode, T* ubar_out,
                                 hipStream_t s);

// Scalars of one field's conjugate-gradient solve that the host reads: rr_0,
// the final rr and relres = sqrt(rr / rr_0), iterations done, stop flag (set
// by each iteration's first kernel), mean of the right-hand side.
struct CgScal {
    double rr, rr0, relres, mean;
    int it, done;
};
// Work split of the CG kernels: workgroups per field (<= kCgMaxBlocks); every
// partial-sum buffer holds cg_blocks(g) * batch doubles.
constexpr int kCgMaxBlocks = 1024;
int cg_blocks(const Grid& g);
// mode 0: r = D vel; 1: r = D Omega_u^{-1} vel; 2, 3: r = rin. Partial sums of
// w_j r (modes 0-2) or r (mode 3) into msum.
template <typename T>
hipError_t launch_cg_div(const Grid& g, const T* vel, const double* rin, double* r, double* msum, int mode,
                         hipStream_t s);
// r = w_j (mean_w - r) (modes 0-2; wsum = sum of w_j over a field) or mean - r
// (mode 3); x = 0; partial sums of r.r into rb0; resets st.it / st.done.
hipError_t launch_cg_init(const Grid& g, double* r, double* x, const double* msum, double* rb0, CgScal* st, int mode,
                          double wsum, hipStream_t s);
// Iteration k: stop test from rr_k (partials rbk); x += alpha_{k-1} p_{k-1}
// if iteration k - 1 was performed (rr_{k-1} partials rbm, p.q partials pqm,
// p_{k-1} = pin); unless stopped, pout = r + beta pin (beta = rr_k / rr_{k-1})
// and partial sums of pout.(A pout) into pqs, A = -Omega_p D G.
hipError_t launch_cg_apply(const Grid& g, const double* r, const double* pin, double* pout, double* x,
                           const double* rbk, const double* rbm, const double* pqm, double* pqs, CgScal* st, int k,
                           double rtol2, int maxiter, hipStream_t s);
// Iteration k: r -= alpha A p (alpha = rr_k / p.q, A p recomputed from p), partial sums of r.r into rbn.
hipError_t launch_cg_update(const Grid& g, double* r, const double* p, const double* rbk, const double* pqs,
                            double* rbn, CgScal* st, int k, double rtol2, int maxiter, hipStream_t s);
// st.rr / st.relres from the newest rr partials.
hipError_t launch_cg_finish(const Grid& g, const double* rb, CgScal* st, hipStream_t s);
// t = w_j (t - mean_w(t)) in place (msum: partial-sum scratch).
hipError_t launch_cg_weighted_center(const Grid& g, double* t, double* msum, double wsum, hipStream_t s);

// Stretched grid (Grid::gm set; k_gen.hip): the same contracts as the channel's
// launchers above, every width taken from the per-direction metrics, y
// periodic or walled (Grid::ywalls). The launch_cg_* launchers above hand
// over to the launch_gen_cg_* ones when Grid::gm is set.
template <typename T>
hipError_t launch_gen_rhs(const Grid& g, const T* u, T* f, hipStream_t s);
template <typename T>
hipError_t launch_gen_divergence(const Grid& g, const T* u, double* r, hipStream_t s);
template <typename T>
hipError_t launch_gen_gradient(const Grid& g, const double* p, T* out, hipStream_t s);
template <typename T>
hipError_t launch_gen_rhs_vjp(const Grid& g, const T* u, const T* fbar, T* ubar, hipStream_t s);
template <typename T>
hipError_t launch_gen_div_vjp(const Grid& g, const double* rbar, T* ubar, hipStream_t s);
template <typename T>
hipError_t launch_gen_grad_vjp(const Grid& g, const T* gbar, double* pbar, hipStream_t s);
template <typename T>
hipError_t launch_gen_project(const Grid& g, const T* w, const double* p, T* u_out, bool adj, hipStream_t s);
template <typename T>
hipError_t launch_gen_stage(const Grid& g, const T* w, const double* p, bool proj, const T* u0, T* y, bool yinit,
                            double cy, T* wout, double cw, hipStream_t s);
template <typename T>
hipError_t launch_gen_stage_vjp(const Grid& g, const T* w, const double* p, bool proj_u, const T* ybar, const T* un,
                                const double* q, bool has_w, double cb, double cw, T* u0bar, int mode, T* out,
                                hipStream_t s);
template <typename T>
hipError_t launch_gen_cg_div(const Grid& g, const T* vel, const double* rin, double* r, double* msum, int mode,
                             hipStream_t s);
hipError_t launch_gen_cg_init(const Grid& g, double* r, double* x, const double* msum, double* rb0, CgScal* st,
                              int mode, double wsum, hipStream_t s);
hipError_t launch_gen_cg_apply(const Grid& g, const double* r, const double* pin, double* pout, double* x,
                               const double* rbk, const double* rbm, const double* pqm, double* pqs, CgScal* st, int k,
                               double rtol2, int maxiter, hipStream_t s);
hipError_t launch_gen_cg_update(const Grid& g, double* r, const double* p, const double* rbk, const double* pqs,
                                double* rbn, CgScal* st, int k, double rtol2, int maxiter, hipStream_t s);
hipError_t launch_gen_cg_weighted_center(const Grid& g, double* t, double* msum, double wsum, hipStream_t s);


// Utilities.
template <typename T>
hipError_t launch_stats(const Grid& g, const T* u, double* partial, int nblocks, hipStream_t s);
hipError_t launch_stream_copy(const void* src, void* dst, size_t nbytes, hipStream_t s);

// Number of workgroups used by launch_stats (partials buffer holds 4 per block).
int stats_blocks(const Grid& g);
// Statistics from at most kStatsCapBlocks workgroups into a caller-provided
// partials buffer of 4 * stats_capped_blocks(g) doubles, then reduced on the
// device into out[4] (kinetic energy, max |u|, max |D u|, all-finite flag).
constexpr int kStatsCapBlocks = 2048;
int stats_capped_blocks(const Grid& g);
template <typename T>
hipError_t launch_stats_capped(const Grid& g, const T* u, double* partial, double* out, hipStream_t s);

}  // namespace ins
