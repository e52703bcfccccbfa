/*
 * ins.h - C ABI of the MI355X (gfx950) staggered-grid incompressible
 * Navier-Stokes hot path: matrix-free operators, spectral pressure solve,
 * projection, classical RK4 and Wray's low-storage RK3 steps, and the
 * pullback (vector-Jacobian product) of each, plus the learned convolutional
 * closure, the Smagorinsky eddy-viscosity closure and LES data helpers.
 *
 * Method: Agdestein & Sanderse, "A differentiable software suite for
 * accelerated simulation of turbulent flows" (arXiv 2604.18536):
 *   Sec. 2.1   staggered Harlow-Welch grid, code-index convention (Sec. 3.1)
 *   Sec. 2.2   discrete operators; App. B explicit kernels and pullbacks
 *   Sec. 2.4   boundary conditions (no-slip walls through ghost volumes)
 *   Sec. 2.6.1 pressure Poisson equation, spectral (DFT) and iterative (CG) solvers
 *   Sec. 2.6.2 explicit Runge-Kutta with a projection at every stage
 *   Sec. 3.3   memory: array reuse, low-storage stepping, lazy fluxes
 *   Sec. 3.4   pullback rule and hand-written adjoint kernels
 *   Sec. 4     neural closure inside the solver, a-posteriori training
 *   App.       eddy-viscosity models (general framework, Smagorinsky)
 *
 * ----------------------------------------------------------------------------
 * Conventions shared by every entry point
 * ----------------------------------------------------------------------------
 * Grid. Dim 2 or 3, cell counts n[0] (x), n[1] (y), n[2] (z; ignored in
 * 2D), box [lo, hi] per direction, and `batch` independent fields processed
 * by every call. Periodic in every direction (INS_BC_PERIODIC), or a channel
 * (INS_BC_WALLS_Y): no-slip walls at y = lo[1] and y = hi[1], x and z
 * periodic; see the channel section below. Uniform unless faces are given
 * (ins_set_y_faces, ins_set_faces).
 *
 * Layout. All field arguments are device pointers to dense arrays, x fastest:
 *   velocity-point field (u, f, ubar, ...):  [batch][dim][n_z][n_y][n_x]
 *   pressure-point field (r, p, ...):        [batch][n_z][n_y][n_x]
 * (2D: drop n_z.) Component a of a velocity field at index I is the
 * a-velocity on the face to the right of cell I in direction a (Sec. 2.1 /
 * Sec. 3.1). There are no ghost cells: neighbours wrap periodically.
 *
 * Precision (ins_dtype).
 *   INS_FP64: every field and all arithmetic in float64.
 *   INS_FP32: velocity-point fields are float32 and the stencils and RK
 *             stage arithmetic run in float32; the divergence, the Poisson
 *             solve and the projection u - G p are computed in float64 and
 *             pressure-point fields (r, p) are float64. (The paper supports a
 *             choice of format but no mixed strategy, Sec. 8.2; this mode is
 *             the mixed strategy its outlook proposes.)
 *   INS_FP32_ALL: for comparison only: every field (pressure-point fields
 *             too) and all arithmetic in float32, the FFT solve included
 *             (float32 spectrum, twiddles and eigenvalues), so the mixed mode
 *             can be measured against a path that keeps nothing in float64.
 *             Periodic grid, forward calls only: ins_rhs, ins_divergence,
 *             ins_gradient, ins_poisson_solve (and its pullback, the same
 *             solve), ins_project (and its pullback), the steps, ins_stats,
 *             ins_face_filter; every other call returns INS_ERR_UNSUPPORTED.
 *
 * Ownership. The caller owns every field buffer; buffers must be 256-byte
 * aligned (torch allocations are) and lie on the context's device. The
 * context owns its FFT plans, twiddle tables, spectrum, pressure and RK
 * stage registers. Forward workspace is allocated in ins_create; the
 * reverse-pass stage storage on the first *_vjp call that needs it; the
 * closure workspace in ins_closure_set / ins_eddy_set. ins_workspace_bytes
 * reports the total.
 *
 * Streams. Every call enqueues its kernels on the context's stream
 * (default: the null stream) and returns without a host synchronisation,
 * except where a host scalar is returned (ins_stats, ins_profile_*, ins_cg_info),
 * in ins_set_y_faces, and in the channel's CG pressure solves, which read their
 * convergence flags every check_every iterations (ins_cg_set; 0 turns it off).
 *
 * Aliasing. Outputs must not alias inputs, except where an entry point says
 * so. Outputs are overwritten, never accumulated into.
 *
 * Errors. Every entry point returns an ins_status and never throws or
 * aborts. INS_ERR_INVALID: null pointer, bad size or parameter.
 * INS_ERR_UNSUPPORTED: a grid the context cannot take (see ins_create), or a
 * feature the grid lacks (closures and LES helpers on the channel and on
 * stretched grids, CG settings on the uniform periodic grid).
 * INS_ERR_OOM: device allocation failed. INS_ERR_HIP: a HIP call or kernel
 * launch failed. ins_last_error() returns a thread-local message for the
 * last non-OK status of the calling thread. Faults inside a kernel surface
 * asynchronously at the caller's next synchronisation.
 *
 * Threading. A context is not thread-safe; use one context per stream.
 */
#ifndef INS_H_
#define INS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ins_ctx_s* ins_ctx;

typedef enum {
    INS_OK = 0,
    INS_ERR_INVALID = -1,
    INS_ERR_UNSUPPORTED = -2,
    INS_ERR_OOM = -3,
    INS_ERR_HIP = -4
} ins_status;

typedef enum { INS_FP64 = 0, INS_FP32 = 1, INS_FP32_ALL = 2 } ins_dtype;

/* INS_BC_PERIODIC: periodic in every direction; pressure by FFT.
 * INS_BC_WALLS_Y:  channel: no-slip walls at both y ends (Sec. 2.4 Dirichlet
 *   condition u = 0 imposed through ghost volumes), x and z periodic;
 *   pressure by a direct solve (FFTs along x and z, a tridiagonal solve along
 *   y per mode) or by matrix-free conjugate gradients (Sec. 2.6.1 iterative
 *   solver); see ins_set_pressure_solver.
 *   The layout is unchanged: u^y[..][n_y - 1][..] is the upper-wall face, a
 *   boundary value, not an unknown. Every operator reads it (and the lower-wall
 *   face) as 0 and every velocity output, forward or pullback, writes 0 there.
 *   A tangential component one cell beyond a wall reads as minus the first
 *   interior value (zero linear interpolant on the wall). The gradient lives
 *   on interior faces only, so D G is the Neumann Laplacian; the pressure solve
 *   returns the zero-mean solution of D G p = r - mean(r). */
typedef enum { INS_BC_PERIODIC = 0, INS_BC_WALLS_Y = 1 } ins_bc;

typedef struct {
    int32_t dim;     /* 2 or 3 */
    int64_t n[3];    /* cells per direction x, y, z (n[2] ignored in 2D) */
    double lo[3];    /* box lower corner */
    double hi[3];    /* box upper corner; h_a = (hi[a]-lo[a]) / n[a] */
    int64_t batch;   /* number of independent fields per call, >= 1 */
} ins_grid;

/* ---------------------------------------------------------------------------
 * Context
 * ------------------------------------------------------------------------- */

/* Create a context on the current HIP device.
 * Requirements (else INS_ERR_UNSUPPORTED): every n in [2, 4096]; for
 * INS_BC_PERIODIC also n_x even and >= 4 and n_x/2, n_y, n_z products of the
 * primes 2, 3, 5, 7 (the real-to-complex FFT along x works on n_x/2 complex
 * points; the spectral solver of Sec. 2.6.1 needs a uniform periodic grid).
 * nu >= 0 is the kinematic viscosity of the diffusion term. Allocates the
 * forward workspace: stage registers (3 velocity fields), pressure, the half
 * spectrum (periodic grid, and the channel when its direct solver applies) and
 * three CG pressure-point fields (channel). */
ins_status ins_create(const ins_grid* grid, ins_bc bc, double nu, ins_dtype dtype, ins_ctx* out);
ins_status ins_destroy(ins_ctx ctx);
/* stream: a hipStream_t (NULL = null stream). */
ins_status ins_set_stream(ins_ctx ctx, void* stream);
/* Device bytes currently held by the context. */
ins_status ins_workspace_bytes(ins_ctx ctx, size_t* bytes);
const char* ins_last_error(void);

/* ---------------------------------------------------------------------------
 * Channel grid (INS_BC_WALLS_Y): pressure solvers
 *
 * Both solvers return the same discrete solution, the zero-mean p with
 * D G p = r - mean_w(r) (the augmented system of the direct solver of
 * Sec. 2.6.1), up to rounding (direct) or up to the CG stopping rule.
 *
 * INS_PRESSURE_FFT (the default when it applies: n_x even, n_x/2 and n_z
 * products of 2, 3, 5, 7, n_y <= 2048): FFTs along the periodic x and z leave
 * one tridiagonal system along y per wavenumber pair (the Neumann second
 * difference across the y widths, shifted by the periodic eigenvalue
 * 4 sin^2(pi k / n) / h^2 of Sec. 2.6.1), solved exactly; the (0, 0) mode is
 * the singular Neumann problem, solved with its weighted mean removed and its
 * solution centred. On a uniform y this is the paper's channel solver (FFTs
 * and a type-II cosine transform, Sec. 6, which diagonalises the same
 * operator); it also holds on a stretched y. No host synchronisation; the
 * spectrum is the only workspace.
 *
 * INS_PRESSURE_CG: every pressure solve (ins_poisson_solve, ins_project, the
 * steps and their pullbacks) runs CG on A = -D G, the Laplace operator applied as the
 * divergence of the gradient without assembling it (Sec. 2.6.1 iterative
 * solver), from p = 0, for A p = mean(r) - r, independently per batch field.
 * A field stops once ||res|| <= rtol ||res_0|| (res the recursively updated
 * residual) or after maxiter iterations. Iterations run back to back on the
 * stream; every check_every iterations the call reads the convergence flags
 * to the host once (a stream synchronisation), and stops launching when all
 * fields are done. check_every = 0 never synchronises and always launches
 * maxiter iterations (done fields skip the work), which keeps a captured
 * graph free of host reads. On a uniform channel the pressure solve is
 * self-adjoint and its pullback is the same solve (see ins_set_y_faces for a
 * stretched y). A search direction with no component outside the constants
 * (p . A p <= 0, e.g. a constant right-hand side) ends the solve without an
 * update (relres then reads 0). Closures, the face filter and the energy spectrum need
 * the periodic grid (INS_ERR_UNSUPPORTED).
 * ------------------------------------------------------------------------- */

/* Stretched y (Sec. 2.5 non-uniform grids, e.g. the tanh grid of eq. tanh-grid):
 * faces is a host array of the n_y + 1 y-face coordinates, strictly increasing
 * (the walls are faces[0] and faces[n_y]); x and z stay uniform. Replaces the
 * uniform spacing of the box for every later call. The operators follow App. B
 * with the non-uniform widths: cell widths w_j, centre distances d_j across the
 * y-faces (mirrored ghost rows beyond the walls); in the convection the
 * transported component is averaged with weights 1/2 and the transporting one
 * interpolated as the mass-flux average w_j / (w_j + w_{j+1}) (the weights that
 * keep the discrete convection energy-conserving). The CG runs on the symmetric
 * -Omega_p D G (pressure volumes Omega_p); the pressure solve returns the
 * zero-mean p with D G p = r - mean_w(r), mean_w the volume-weighted mean. The
 * projection is no longer its own transpose: ins_project_vjp applies
 * Omega_u P Omega_u^{-1} (velocity volumes Omega_u) and ins_poisson_solve_vjp the
 * transpose of the solve; the step pullbacks use both. Synchronises the stream.
 * INS_ERR_UNSUPPORTED on a periodic context; INS_ERR_INVALID for non-increasing
 * or non-finite coordinates. */
ins_status ins_set_y_faces(ins_ctx ctx, const double* faces);

/* Stretched grid in any direction (Sec. 2.5 non-uniform grids: the cosine,
 * tanh (eq. tanh-grid) and geometric stretchings, or any increasing faces):
 * faces is a host array of the n_axis + 1 face coordinates of direction axis
 * (0 = x, 1 = y, 2 = z), strictly increasing; cell i spans [faces[i],
 * faces[i + 1]]. Along a periodic direction the faces close the period (cell
 * n - 1 neighbours cell 0; the period is faces[n] - faces[0]), so the
 * convergence study of Sec. 7 (Taylor-Green on a tanh grid) runs on the
 * periodic context. On a channel, axis 1 is ins_set_y_faces; axes 0 and 2
 * stretch the periodic directions. Directions not given keep the box's
 * uniform spacing. Operators (App. B with the widths of each direction): cell
 * widths w_i in the divergence, centre distances d_i = (w_i + w_{i+1}) / 2 in
 * the gradient, eq. diff-kernel with outer and inner widths, and in the
 * convection F^{ab} = A^{ab} B^{ab} the transported component averaged with
 * weights 1/2 and the transporting one interpolated as the mass-flux average
 * w_i / (w_i + w_{i+1}) of direction a (eq. interp-weights read so that
 * convection conserves energy on a grid stretched in every direction).
 * Volumes Omega_p = prod_a w^a, Omega_u^a = d^a prod_{b != a} w^b.
 * The first call that stretches a periodic direction switches the context to
 * the stretched-grid kernels for good (one thread per cell) and to the CG
 * pressure solve (ins_cg_set applies; allocates its workspace on a periodic
 * context): the solve returns the zero-mean p with D G p = r - mean_w(r) by CG
 * on the symmetric -Omega_p D G, the pullbacks use the transposed projection
 * Omega_u P Omega_u^{-1} and the transposed solve, exactly as on a stretched
 * channel. Closures, the face filter and the energy spectrum need the uniform
 * periodic grid (INS_ERR_UNSUPPORTED, also when a closure is set at this
 * call). Synchronises the stream. INS_ERR_INVALID for a bad axis, a null
 * pointer, or non-increasing or non-finite coordinates. */
ins_status ins_set_faces(ins_ctx ctx, int axis, const double* faces);

/* Constant body force (the forcing term that F(u) collects, App. A momentum
 * equation; the channel of Sec. 6 is driven by f = (1, 0, 0)): force is a host
 * array of dim values, added to F on the velocity unknowns by ins_rhs and every
 * step from the next call on (default 0). A constant has no Jacobian, so the
 * pullbacks change only through the forward stages they linearise about. A
 * wall-normal component is balanced by the pressure. The value is captured by
 * the kernels launched after the call (no synchronisation; work already queued
 * keeps the old force). INS_ERR_UNSUPPORTED on a periodic context;
 * INS_ERR_INVALID for a null or non-finite force. */
ins_status ins_set_body_force(ins_ctx ctx, const double* force);

/* Defaults: rtol 1e-10, maxiter 20000, check_every 16 (the channel, and any
 * grid stretched by ins_set_faces). INS_ERR_UNSUPPORTED on a uniform periodic
 * context (solved by FFT); INS_ERR_INVALID for rtol < 0, maxiter < 1 or
 * check_every < 0. */
ins_status ins_cg_set(ins_ctx ctx, double rtol, int maxiter, int check_every);
/* Iterations and final relative residual ||res|| / ||res_0|| of the last
 * CG solve (maxima over the batch; 0 and 0 before the first). Synchronises
 * the context's stream. INS_ERR_UNSUPPORTED on a uniform periodic context. */
ins_status ins_cg_info(ins_ctx ctx, int* iterations, double* relres);

typedef enum { INS_PRESSURE_AUTO = 0, INS_PRESSURE_FFT = 1, INS_PRESSURE_CG = 2 } ins_pressure;

/* Choose the pressure solver (an ins_pressure value) for every later call.
 * INS_PRESSURE_AUTO: FFT where it applies, else CG (the default). Periodic
 * grid: only FFT (INS_PRESSURE_CG gives INS_ERR_UNSUPPORTED). Channel:
 * INS_PRESSURE_FFT gives INS_ERR_UNSUPPORTED when the sizes above rule it out.
 * INS_ERR_INVALID for any other value. Host-side only: no synchronisation, and
 * both solvers' workspace is allocated at ins_create, so switching allocates
 * nothing. */
ins_status ins_set_pressure_solver(ins_ctx ctx, int solver);
/* The solver in use: INS_PRESSURE_FFT or INS_PRESSURE_CG. */
ins_status ins_get_pressure_solver(ins_ctx ctx, int* solver);

/* ---------------------------------------------------------------------------
 * Forward operators (Sec. 2.2 discrete operators; App. B kernels)
 * ------------------------------------------------------------------------- */

/* f = C(u) + nu * Lap(u) (+ m_theta(u) when a closure is set; + the body
 * force on a channel, see ins_set_body_force): the
 * convection of eq. conv-kernel (uniform weights 1/2, skew-symmetric form)
 * and the diffusion of eq. diff-kernel. u, f: velocity fields. */
ins_status ins_rhs(ins_ctx ctx, const void* u, void* f);

/* r = D u, eq. div-kernel: r[I] = sum_a (u_a[I] - u_a[I - e_a]) / h_a.
 * r is a pressure-point field: float64 (float32 in INS_FP32_ALL, the type of
 * every pressure-point argument declared void* below). */
ins_status ins_divergence(ins_ctx ctx, const void* u, void* r);

/* g = G p, eq. presgrad-kernel: g_a[I] = (p[I + e_a] - p[I]) / h_a.
 * p pressure-point field; g velocity field in the context dtype. */
ins_status ins_gradient(ins_ctx ctx, const void* p, void* g);

/* Solve D G p = r by the spectral solver of Sec. 2.6.1: p = DFT^-1 L^-1 DFT r
 * with the exact discrete transfer function
 * L(k) = -sum_a 4 sin^2(pi k_a / n_a) / h_a^2 and L(0) := 1 (so the mean of
 * p equals the mean of r). r, p: pressure-point fields; r may equal p. */
ins_status ins_poisson_solve(ins_ctx ctx, const void* r, void* p);

/* u_out = P u = u - G p with p = (D G)^-1 D u (the projection applied at every
 * RK stage, Sec. 2.6.2). The divergence, Poisson solve and u - G p run in
 * float64 (float32 in INS_FP32_ALL). p_out (a pressure-point field, may be
 * NULL) receives p. u == u_out is allowed. */
ins_status ins_project(ins_ctx ctx, const void* u, void* u_out, void* p_out);

/* One classical RK4 step with the velocity projected after every stage
 * (Sec. 2.6.2): u_{i+1} = P(u0 + dt a_{i+1} F(u_i)), a = (1/2, 1/2, 1);
 * u1 = P(u0 + dt (F1 + 2F2 + 2F3 + F4) / 6), F = ins_rhs. u0 is used as
 * given (callers pass a solenoidal field). Low-storage schedule: stage
 * register, accumulator and one pressure solve per stage, with the
 * projection of each stage fused into the next stage's stencil.
 * u0 == u1 is allowed (in-place step). dt > 0. */
ins_status ins_step_rk4(ins_ctx ctx, const void* u0, void* u1, double dt);

/* ---------------------------------------------------------------------------
 * Pullbacks (Sec. 3.4 eq. pullback; App. B)
 * ------------------------------------------------------------------------- */

/* ubar = J_F(u)^T fbar: the convection pullback derived from the forward
 * kernel (gather form, no atomics) plus the diffusion pullback (the
 * diffusion itself on a uniform grid). With a closure set, also adds the
 * closure's input gradient and accumulates its parameter gradient (see
 * ins_closure_grad). */
ins_status ins_rhs_vjp(ins_ctx ctx, const void* u, const void* fbar, void* ubar);

/* ubar = D^T rbar = -G rbar: ubar_a[J] = (rbar[J] - rbar[J + e_a]) / h_a.
 * rbar float64 pressure-point field. */
ins_status ins_divergence_vjp(ins_ctx ctx, const double* rbar, void* ubar);

/* pbar = G^T gbar = -D gbar. gbar velocity field, pbar float64. */
ins_status ins_gradient_vjp(ins_ctx ctx, const void* gbar, double* pbar);

/* rbar = L^-T pbar = L^-1 pbar: the Poisson solve is self-adjoint (Sec. 2.6.1).
 * pbar, rbar: pressure-point fields. */
ins_status ins_poisson_solve_vjp(ins_ctx ctx, const void* pbar, void* rbar);

/* ubar = P^T ubar_out = P ubar_out (P is symmetric on the uniform periodic
 * grid). ubar == ubar_out is allowed. */
ins_status ins_project_vjp(ins_ctx ctx, const void* ubar_out, void* ubar);

/* u0bar = (d u1 / d u0)^T u1bar for u1 = ins_step_rk4(u0, dt): recomputes the
 * stage states from u0, then runs the stages backwards (pullbacks of the
 * projection and of the right-hand side). Allocates the reverse-pass stage
 * storage on first use. u0bar must not alias u0 or u1bar. */
ins_status ins_step_rk4_vjp(ins_ctx ctx, const void* u0, const void* u1bar, void* u0bar, double dt);

/* One step of Wray's low-storage three-stage, third-order Runge-Kutta
 * scheme (Sec. 2.6.2 lists it among the explicit integrators; Sec. 3.3 cites
 * it as the low-storage method), velocity projected after every stage like
 * ins_step_rk4. The paper gives no coefficients; these are Wray's:
 *   u_1 = P(u0 + dt g1 F(u0)),  u_2 = P(u_1 + dt (g2 F(u_1) + z1 F(u0))),
 *   u1 = P(u_2 + dt (g3 F(u_2) + z2 F(u_1))),
 *   g = (8/15, 5/12, 3/4), z = (-17/60, -5/12)
 * (Butcher form: c = (0, 8/15, 2/3), b = (1/4, 0, 3/4)). Three stage kernels
 * and three pressure solves per step instead of four of each. Same buffers,
 * aliasing (u0 == u1 allowed), closure coupling and errors as ins_step_rk4. */
ins_status ins_step_wray3(ins_ctx ctx, const void* u0, void* u1, double dt);

/* u0bar = (d u1 / d u0)^T u1bar for u1 = ins_step_wray3(u0, dt): recomputes
 * the two inner stage states, then runs the stages backwards. Same storage,
 * aliasing rules, closure-gradient accumulation and errors as
 * ins_step_rk4_vjp. */
ins_status ins_step_wray3_vjp(ins_ctx ctx, const void* u0, const void* u1bar, void* u0bar, double dt);

/* ---------------------------------------------------------------------------
 * Steps that keep their stage inputs for the pullback. Reverse-mode training
 * stores the forward states of every sub-step for the backward pass (Sec. 4);
 * ins_step_*_vjp instead recompute them from u0 (less memory, one more
 * forward per step). These variants let the caller hold the stage inputs:
 * the unprojected stage sums W_i and their pressures P_i (u_i = W_i - G P_i),
 * i.e. ins_scheme_stage_count(scheme) velocity fields and as many float64
 * pressure-point fields, contiguous:
 *   stages  [count][batch][dim][n_z][n_y][n_x]  (context type),
 *   pstages [count][batch][n_z][n_y][n_x]        (float64).
 * ins_step_save does the same work as the plain step, writing the stage
 * registers to these buffers; ins_step_vjp_saved skips the recomputation and
 * must get the stages of the same (u0, dt), with the same closure setting.
 * ------------------------------------------------------------------------- */
typedef enum { INS_RK4 = 0, INS_WRAY3 = 1 } ins_scheme;

/* Stage inputs a scheme keeps: 3 for RK4, 2 for Wray3; -1 for an unknown scheme. */
int ins_scheme_stage_count(int scheme);

/* u1 = step(u0, dt) (scheme per ins_scheme; u0 == u1 allowed), keeping the
 * stage inputs in stages / pstages (overwritten). */
ins_status ins_step_save(ins_ctx ctx, int scheme, const void* u0, void* u1, double dt, void* stages,
                         double* pstages);

/* u0bar = (d u1 / d u0)^T u1bar from the stage inputs of ins_step_save (read
 * only). u0bar must not alias u0, u1bar or stages. */
ins_status ins_step_vjp_saved(ins_ctx ctx, int scheme, const void* u0, const void* stages, const double* pstages,
                              const void* u1bar, void* u0bar, double dt);

/* ---------------------------------------------------------------------------
 * Learned closure (Sec. 4: a neural closure inside the solver, trained
 * a-posteriori through it). The paper does not fix an architecture; this one
 * is a 3D CNN 3 -> 32 -> 32 -> 3 channels, 3x3x3 kernels with circular
 * padding, biases, exact-erf GELU between layers, no output activation. The
 * three staggered velocity components are its input channels on the cell grid
 * and output channel a is added to the a-velocity right-hand side, so the
 * step integrates du/dt = P(F(u) + m_theta(u)). Convolutions run on bfloat16
 * matrix cores with float32 accumulation: u, the weights and every GELU output
 * are rounded to bfloat16 (nearest even); in the backward pass the cotangent
 * entering each convolution is rounded to bfloat16. 3D only; n_x must be a
 * multiple of 32.
 *
 * Parameters: 32,899 float32 values on the device, per layer in order
 * W[out][in][kz][ky][kx] then b[out]; tap (kz, ky, kx) multiplies
 * u[I + (kx-1, ky-1, kz-1)] (cross-correlation).
 * ------------------------------------------------------------------------- */

/* Set (params != NULL: copied, packed to bfloat16 for the kernels) or clear
 * (params == NULL) the closure. While set, ins_rhs, ins_step_rk4, ins_rhs_vjp
 * and ins_step_rk4_vjp include it, and the *_vjp calls accumulate the
 * parameter gradient. Allocates the closure workspace (about 330 bytes per
 * cell of the batch) on first use. */
ins_status ins_closure_set(ins_ctx ctx, const float* params);

/* Copy the accumulated parameter gradient (float32, 32,899 values, device) to
 * params_bar and reset the accumulator to zero. */
ins_status ins_closure_grad(ins_ctx ctx, float* params_bar);

/* m = m_theta(u) alone (velocity layout, context dtype). */
ins_status ins_cnn_forward(ins_ctx ctx, const void* u, void* m);

/* ubar = (d m_theta / d u)^T mbar (overwritten) and params_bar =
 * (d m_theta / d theta)^T mbar (overwritten; the accumulator of
 * ins_closure_grad is left at zero). */
ins_status ins_cnn_backward(ins_ctx ctx, const void* u, const void* mbar, void* ubar, float* params_bar);

/* Diagnostic copy of one of the closure's internal tensors as the last
 * ins_cnn_backward left them (for layer-by-layer parity checks); out is a
 * device buffer of the stated size, cells of the batch in velocity-field order
 * and channels fastest (channels-last):
 *   0: bfloat16 input x0 [cells][8] (channels 3..7 zero)
 *   1: float32 pre-activation z1 [cells][32]      2: bfloat16 GELU(z1) [cells][32]
 *   3: float32 pre-activation z2 [cells][32]      4: bfloat16 GELU(z2) [cells][32]
 *   5: bfloat16 cotangent of m [cells][8]
 *   6: bfloat16 cotangent of z2 [cells][32]       7: bfloat16 cotangent of z1 [cells][32]
 *   8: m itself (velocity layout, context dtype).
 * INS_ERR_INVALID for another `which` or when no learned closure is set. */
ins_status ins_cnn_saved(ins_ctx ctx, int which, void* out);

/* ---------------------------------------------------------------------------
 * Smagorinsky eddy-viscosity closure (appendix on eddy-viscosity models:
 * general framework and eq. smagorinsky), the classical LES baseline.
 * On the staggered grid: D_a = delta_a u^a at pressure points, G_ab =
 * delta_b u^a on the (a, b) edges; the velocity gradient at a pressure point
 * averages G_ab over its four (a, b) edges; nu_t = (C_s Delta)^2 sqrt(2 S:S)
 * at pressure points and, on an edge, the mean of its four pressure points.
 * The right-hand side gains M^a = sum_b delta_b (2 nu_t S_ab) on the a-faces
 * (the appendix's sub-grid stress with the sign that dissipates energy), so
 * steps integrate du/dt = P(F(u) + M(u)). 2D and 3D. One closure at a time:
 * setting this one replaces a learned closure and vice versa.
 * ------------------------------------------------------------------------- */

/* Set (cs > 0) or clear (cs == 0, if this closure is the one set) the
 * Smagorinsky closure with constant cs (the paper proposes 0.17) and filter
 * width delta (delta <= 0: the geometric mean of the spacings). While set,
 * ins_rhs, the steps and their pullbacks include it (it has no learnable
 * parameters). Allocates its workspace (1 + d(d+1)/2 pressure-point fields
 * of the context type, plus three velocity fields) on first use.
 * INS_ERR_INVALID for cs < 0 or non-finite arguments. */
ins_status ins_eddy_set(ins_ctx ctx, double cs, double delta);

/* m = M(u) alone (velocity layout, context type). INS_ERR_INVALID when the
 * Smagorinsky closure is not set. */
ins_status ins_eddy_forward(ins_ctx ctx, const void* u, void* m);

/* ubar = (dM/du)^T mbar (overwritten). Where S = 0 the square root has no
 * derivative and its pullback is taken as 0. ubar must not alias u or mbar. */
ins_status ins_eddy_backward(ins_ctx ctx, const void* u, const void* mbar, void* ubar);

/* ---------------------------------------------------------------------------
 * LES data helpers (filtered DNS and its spectrum). The paper names the
 * pipeline DNS -> filter -> LES (Sec. 4) but not the filter or the spectrum
 * binning; the readings are stated with each call.
 * ------------------------------------------------------------------------- */

/* Face filter from the context's (fine) grid to a grid coarser by `factor` in
 * every direction: coarse cell I covers fine cells factor*I .. factor*I +
 * factor - 1, and its a-velocity is the mean of the factor^(dim-1) fine
 * a-velocities on its right a-face. Maps solenoidal to solenoidal (the coarse
 * divergence is the volume mean of the fine one). u: fine velocity field;
 * u_coarse: [batch][dim][n_z/f][n_y/f][n_x/f], context dtype. Every n must be
 * divisible by factor (else INS_ERR_INVALID). */
ins_status ins_face_filter(ins_ctx ctx, const void* u, int factor, void* u_coarse);

/* Kinetic-energy spectrum E(k) = 1/2 sum over the shell k - 1/2 <= |k| < k + 1/2
 * of sum_a |uhat_a(k)|^2 / N^2 (integer wavenumber index k, N cells, uhat the
 * unnormalised DFT), k = 0 .. nbins-1, per field of the batch. e: device
 * float64 array [batch][nbins], overwritten; shells beyond nbins are dropped
 * (nbins = floor(sqrt(dim) * n_max / 2 + 1/2) + 1 keeps every mode, so the sum
 * of e equals the mean kinetic energy). Uses the context's spectrum buffer;
 * shell sums are accumulated with atomic adds (order-dependent rounding). */
ins_status ins_energy_spectrum(ins_ctx ctx, const void* u, double* e, int nbins);

/* ---------------------------------------------------------------------------
 * Utilities (diagnostics, benchmarking)
 * ------------------------------------------------------------------------- */

/* Host-returned statistics of a velocity field, summed over the batch:
 * out[0] = kinetic energy (1/2) mean_I sum_a u_a^2 (mean over batch),
 * out[1] = max |u_a[I]|, out[2] = max |(D u)[I]|, out[3] = 1 if every entry
 * is finite else 0. Synchronises the stream. */
ins_status ins_stats(ins_ctx ctx, const void* u, double out[4]);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the statistics of
 * ins_stats, written to out, a DEVICE array of 4 doubles (same order and
 * meaning; the kinetic-energy sum is reduced in another order, so it may
 * differ from ins_stats in the last bits), with no host synchronisation.
 * Allocates nothing and creates no events: its partial sums live in a fixed
 * 64 KiB device scratch array that the library holds on every device it runs
 * on until the process ends (at most 2048 workgroups of 4 doubles; larger
 * fields are walked by the same workgroups). Every call on a device shares
 * that device's scratch and leaves its partials there: calls that overlap on
 * one device (different streams or threads, any contexts) race and must be
 * serialised by the caller. INS_ERR_INVALID for a null u or out. */
ins_status ins_stats_noalloc(ins_ctx ctx, const void* u, double* out);

/* Plain device copy of nbytes (multiple of 16) from src to dst with the
 * library's streaming-copy kernel; used to calibrate bandwidth counters. */
ins_status ins_stream_copy(ins_ctx ctx, const void* src, void* dst, size_t nbytes);

/* Kernel timing: when enabled, every kernel launch of this context is
 * bracketed by HIP events on the context stream. ins_profile_read
 * synchronises, then reports for entry i < count: the kernel name, the
 * number of launches and their summed duration in milliseconds, and clears
 * nothing; ins_profile_reset clears the records. */
ins_status ins_profile_enable(ins_ctx ctx, int enable);
ins_status ins_profile_reset(ins_ctx ctx);
ins_status ins_profile_count(ins_ctx ctx, int* count);
ins_status ins_profile_read(ins_ctx ctx, int i, char* name, size_t name_len, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* INS_H_ */
