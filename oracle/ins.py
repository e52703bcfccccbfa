"""Float64 numpy oracle of the discrete operators, pressure solve, RK4 and Wray3 steps and their adjoints.

TEST INFRASTRUCTURE ONLY (see the package docstring). Not used by the product path.

Notation follows the paper (Sec. 2 and App. A/B). A velocity field ``u`` has
shape ``(d, N_z, N_y, N_x)`` (3D) or ``(d, N_y, N_x)`` (2D); ``u[a][I]`` is the
a-velocity on the face to the right of cell ``I`` in direction ``a`` (the
code-index convention of Sec. 3.1). A pressure-point field has shape
``(N_z, N_y, N_x)``. The grid is uniform and periodic, so every width
``|Delta^a_i|`` equals ``h[a]``, the interpolation weights A^{ab+-} of App. B
are all 1/2, and periodic extension replaces the ghost volumes of Sec. 2.1:
``f[I + e_a]`` is ``np.roll(f, -1)`` along the array axis of direction ``a``.
"""
from __future__ import annotations

import numpy as np

_HALF = 0.5


def _axis(a, d):
    return d - 1 - a


def _next(f, a, d):
    """f[I + e_a] with periodic extension."""
    return np.roll(f, -1, axis=_axis(a, d))


def _prev(f, a, d):
    """f[I - e_a] with periodic extension."""
    return np.roll(f, 1, axis=_axis(a, d))


def spacing_of(n, lo=None, hi=None):
    d = len(n)
    lo = [0.0] * d if lo is None else lo
    hi = [2 * np.pi] * d if hi is None else hi
    return tuple((hi[a] - lo[a]) / n[a] for a in range(d))


def kinetic_energy(u):
    """(1/2) mean over cells of sum_a u_a^2 (uniform grid)."""
    return 0.5 * float(np.mean(np.sum(np.asarray(u) ** 2, axis=0)))


# ----------------------------------------------------------------------------
# Forward operators (App. B: eq. div-kernel, presgrad-kernel, diff-kernel,
# conv-kernel; Sec. 2.2 discrete derivative)
# ----------------------------------------------------------------------------

def divergence(u, h):
    """phi_I = sum_a (u^a_{I+h_a} - u^a_{I-h_a}) / |Delta^a|   (App. B, divergence kernel).

    In code indices the face to the right of cell I is ``u[a][I]`` and the one to
    its left is ``u[a][I - e_a]``.
    """
    d = u.shape[0]
    r = np.zeros(u.shape[1:], dtype=np.float64)
    for a in range(d):
        r += (u[a] - _prev(u[a], a, d)) / h[a]
    return r


def gradient(p, h):
    """phi^a_I = (p_{I+h_a} - p_{I-h_a}) / |Delta^a|   (App. B, pressure-gradient kernel).

    At the a-face right of cell I this is (p[I + e_a] - p[I]) / h_a.
    """
    d = p.ndim
    return np.stack([(_next(p, a, d) - p) / h[a] for a in range(d)])


def diffusion(u, h, nu):
    """phi^a_I = nu sum_b ((u_{I+2h_b} - u_I)/|D| - (u_I - u_{I-2h_b})/|D|) / |D|   (App. B, diffusion kernel)."""
    d = u.shape[0]
    out = np.zeros_like(u, dtype=np.float64)
    for a in range(d):
        ua = u[a]
        for b in range(d):
            right = (_next(ua, b, d) - ua) / h[b]
            left = (ua - _prev(ua, b, d)) / h[b]
            out[a] += (right - left) / h[b]
    return nu * out


def convection(u, h):
    """Skew-symmetric (energy-conserving) convection of App. B, eq. conv-kernel, uniform weights 1/2.

    phi^a_I = -sum_b [ (A u^a_I + A u^a_{I+2h_b}) (A u^b_I + A u^b_{I+2h_a})
                      - (A u^a_{I-2h_b} + A u^a_I) (A u^b_{I-2h_b} + A u^b_{I-2h_b+2h_a}) ] / |Delta^b|

    read with code indices, so the two products are the flux
    F^{ab}[I] = a^{ab}[I] b^{ab}[I], a^{ab}[I] = (u^a[I] + u^a[I+e_b])/2,
    b^{ab}[I] = (u^b[I] + u^b[I+e_a])/2, at the right and left b-faces of the
    a-velocity volume. Each flux component is built and consumed one at a time
    (the lazy tensor components of Sec. 3.3).
    """
    d = u.shape[0]
    out = np.zeros_like(u, dtype=np.float64)
    for a in range(d):
        for b in range(d):
            a_ab = _HALF * u[a] + _HALF * _next(u[a], b, d)
            b_ab = _HALF * u[b] + _HALF * _next(u[b], a, d)
            flux = a_ab * b_ab
            out[a] -= (flux - _prev(flux, b, d)) / h[b]
    return out


def rhs(u, h, nu):
    """F(u) = convection + diffusion (momentum equation of App. A, zero body force)."""
    return convection(u, h) + diffusion(u, h, nu)


# ----------------------------------------------------------------------------
# Pressure Poisson solve and projection (Sec. 2.6.1, spectral solver)
# ----------------------------------------------------------------------------

def laplace_eigenvalues(n, h):
    """Transfer function of L = D G on the DFT modes: -sum_a 4 sin^2(pi k_a / N_a) / h_a^2.

    Array of the full complex-DFT shape (N_z, N_y, N_x). The zero mode is set to
    one, as the spectral solver of Sec. 2.6.1 prescribes.
    """
    d = len(n)
    lam = np.zeros(tuple(reversed(n)), dtype=np.float64)
    for a in range(d):
        k = np.arange(n[a], dtype=np.float64)
        s = np.sin(np.pi * k / n[a])
        shape = [1] * d
        shape[_axis(a, d)] = n[a]
        lam = lam - (4.0 * s * s / (h[a] * h[a])).reshape(shape)
    lam[(0,) * d] = 1.0
    return lam


def poisson_solve(r, h):
    """p = DFT^{-1} Lhat^{-1} DFT r with Lhat(0) := 1 (Sec. 2.6.1, spectral solver).

    Solves D G p = r (the sign makes p the physical pressure); the zero mode of
    p equals that of r.
    """
    n = tuple(reversed(r.shape))
    lam = laplace_eigenvalues(n, h)
    return np.real(np.fft.ifftn(np.fft.fftn(r) / lam))


def project(u, h):
    """P u = u - G L^{-1} D u: the pressure projection applied at every RK stage (Sec. 2.6.2)."""
    p = poisson_solve(divergence(u, h), h)
    return u - gradient(p, h), p


# ----------------------------------------------------------------------------
# Classical RK4 with projection after every stage (Sec. 2.6.2)
# ----------------------------------------------------------------------------

RK4_A = (0.5, 0.5, 1.0)
RK4_B = (1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0)


def _proj_fn(h, project_fn):
    return project_fn if project_fn is not None else (lambda v: project(v, h)[0])


def rk4_stages(u0, h, nu, dt, rhs_fn=None, project_fn=None):
    """Stage velocities u_1..u_4 and stage right-hand sides F_1..F_4 of one step.

    u_1 = u0 and u_{i+1} = P(u0 + dt a_{i+1} F(u_i)); returns (us, Fs).
    rhs_fn(u) replaces F when given (e.g. F plus a closure term), project_fn(u)
    replaces P (e.g. the projection of a wall-bounded grid).
    """
    F = rhs_fn if rhs_fn is not None else (lambda v: rhs(v, h, nu))
    P = _proj_fn(h, project_fn)
    us = [np.array(u0, dtype=np.float64)]
    fs = []
    for i in range(4):
        fs.append(F(us[i]))
        if i < 3:
            us.append(P(u0 + dt * RK4_A[i] * fs[i]))
    return us, fs


def step_rk4(u0, h, nu, dt, rhs_fn=None, project_fn=None):
    """One classical RK4 step with the velocity projected at every stage.

    u_{n+1} = P(u0 + dt (F_1 + 2 F_2 + 2 F_3 + F_4) / 6).
    """
    _, fs = rk4_stages(u0, h, nu, dt, rhs_fn, project_fn)
    y = u0 + dt * (fs[0] + 2.0 * fs[1] + 2.0 * fs[2] + fs[3]) / 6.0
    return _proj_fn(h, project_fn)(y)


# ----------------------------------------------------------------------------
# Wray's low-storage three-stage Runge-Kutta scheme (one of the explicit
# integrators named in Sec. 2.6.2 and the low-storage method of Sec. 3.3),
# velocity projected after every stage as for RK4. The paper cites the scheme
# without its coefficients; they are Wray's two-register ones:
#   u_1 = P(u_0 + dt g1 F(u_0))
#   u_2 = P(u_1 + dt (g2 F(u_1) + z1 F(u_0)))
#   u_3 = P(u_2 + dt (g3 F(u_2) + z2 F(u_1)))
# with g = (8/15, 5/12, 3/4), z = (-17/60, -5/12); u_3 is the new state.
# ----------------------------------------------------------------------------

WRAY3_G = (8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0)
WRAY3_Z = (-17.0 / 60.0, -5.0 / 12.0)


def wray3_stages(u0, h, nu, dt, rhs_fn=None, project_fn=None):
    """Stage velocities (u_0, u_1, u_2) and right-hand sides F(u_0), F(u_1), F(u_2)."""
    F = rhs_fn if rhs_fn is not None else (lambda v: rhs(v, h, nu))
    P = _proj_fn(h, project_fn)
    us = [np.array(u0, dtype=np.float64)]
    fs = [F(us[0])]
    us.append(P(us[0] + dt * WRAY3_G[0] * fs[0]))
    fs.append(F(us[1]))
    us.append(P(us[1] + dt * (WRAY3_G[1] * fs[1] + WRAY3_Z[0] * fs[0])))
    fs.append(F(us[2]))
    return us, fs


def step_wray3(u0, h, nu, dt, rhs_fn=None, project_fn=None):
    """One step of Wray's scheme: u_3 = P(u_2 + dt (g3 F(u_2) + z2 F(u_1)))."""
    us, fs = wray3_stages(u0, h, nu, dt, rhs_fn, project_fn)
    return _proj_fn(h, project_fn)(us[2] + dt * (WRAY3_G[2] * fs[2] + WRAY3_Z[1] * fs[1]))


# ----------------------------------------------------------------------------
# Pullbacks (Sec. 3.4 general pullback rule, App. B adjoint kernels)
# ----------------------------------------------------------------------------

def divergence_vjp(rbar, h):
    """ubar^a_I = rbar_{I-h_a}/|D| - rbar_{I+h_a}/|D|  (App. B): ubar[a][J] = (rbar[J] - rbar[J+e_a]) / h_a."""
    d = rbar.ndim
    return np.stack([(rbar - _next(rbar, a, d)) / h[a] for a in range(d)])


def gradient_vjp(gbar, h):
    """pbar_I = sum_a (gbar^a_{I-h_a} - gbar^a_{I+h_a}) / |D|  (App. B): sum_a (gbar[a][I-e_a] - gbar[a][I]) / h_a."""
    d = gbar.shape[0]
    out = np.zeros(gbar.shape[1:], dtype=np.float64)
    for a in range(d):
        out += (_prev(gbar[a], a, d) - gbar[a]) / h[a]
    return out


def diffusion_vjp(fbar, h, nu):
    """The diffusion pullback of App. B; on a uniform grid it is the diffusion operator itself."""
    return diffusion(fbar, h, nu)


def convection_vjp(u, fbar, h):
    """Pullback of the convection kernel, derived from the forward kernel (Sec. 3.4 rule).

    The forward kernel is phi^a = -sum_b delta^-_b F^{ab} with
    F^{ab} = a^{ab} b^{ab}; its transpose step by step is
      Fbar^{ab}[I] = (fbar^a[I+e_b] - fbar^a[I]) / h_b,
      abar = Fbar b^{ab},  bbar = Fbar a^{ab},
      ubar^a[J] += (abar[J] + abar[J-e_b]) / 2,
      ubar^b[J] += (bbar[J] + bbar[J-e_a]) / 2.
    (The printed eight-term pullback in App. B evaluates the primal factor of
    its last four terms at a shifted face and fails the dot-product test; the
    forward kernel is taken as authoritative.)
    """
    d = u.shape[0]
    ubar = np.zeros_like(u, dtype=np.float64)
    for a in range(d):
        for b in range(d):
            a_ab = _HALF * u[a] + _HALF * _next(u[a], b, d)
            b_ab = _HALF * u[b] + _HALF * _next(u[b], a, d)
            fl_bar = (_next(fbar[a], b, d) - fbar[a]) / h[b]
            abar = fl_bar * b_ab
            bbar = fl_bar * a_ab
            ubar[a] += _HALF * abar + _HALF * _prev(abar, b, d)
            ubar[b] += _HALF * bbar + _HALF * _prev(bbar, a, d)
    return ubar


def rhs_vjp(u, fbar, h, nu):
    """J_F(u)^T fbar = convection pullback + diffusion pullback."""
    return convection_vjp(u, fbar, h) + diffusion_vjp(fbar, h, nu)


def poisson_solve_vjp(pbar, h):
    """The Poisson solve is self-adjoint, so its pullback is a Poisson solve (Sec. 2.6.1)."""
    return poisson_solve(pbar, h)


def project_vjp(ubar_out, h):
    """P^T = I - D^T L^{-T} G^T = I - G L^{-1} D = P on the uniform periodic grid."""
    return project(ubar_out, h)[0]


def step_rk4_vjp(u0, u1bar, h, nu, dt, rhs_fn=None, rhs_vjp_fn=None, project_fn=None, project_vjp_fn=None):
    """Reverse pass of ``step_rk4``: the stage loop run backwards with the pullbacks above.

    Stage states are recomputed from u0 first (the forward states must exist
    before back-propagation, Sec. 3.4). rhs_vjp_fn(u, fbar) replaces the
    right-hand-side pullback when given (it may accumulate parameter gradients);
    project_fn / project_vjp_fn replace P and its pullback.
    """
    us, _ = rk4_stages(u0, h, nu, dt, rhs_fn, project_fn)
    G = rhs_vjp_fn if rhs_vjp_fn is not None else (lambda v, fb: rhs_vjp(v, fb, h, nu))
    PT = project_vjp_fn if project_vjp_fn is not None else (lambda v: project_vjp(v, h))
    ybar = PT(u1bar)
    u0bar = ybar.copy()
    fbar = [dt * RK4_B[i] * ybar for i in range(4)]
    for i in range(3, -1, -1):
        ubar_i = G(us[i], fbar[i])
        if i == 0:
            u0bar += ubar_i
        else:
            wbar = PT(ubar_i)
            u0bar += wbar
            fbar[i - 1] = fbar[i - 1] + dt * RK4_A[i - 1] * wbar
    return u0bar


def step_wray3_vjp(u0, u1bar, h, nu, dt, rhs_fn=None, rhs_vjp_fn=None, project_fn=None, project_vjp_fn=None):
    """Reverse pass of ``step_wray3``, transposing its two-register recurrence.

    With w_k the unprojected stage sums (u_k = P w_k) and wbar_k = P^T ubar(u_k):
      wbar_3 = P u3bar;  u2bar = wbar_3 + J(u_2)^T (dt g3 wbar_3);  F1bar = dt z2 wbar_3
      wbar_2 = P u2bar;  u1bar = wbar_2 + J(u_1)^T (dt g2 wbar_2 + F1bar);  F0bar = dt z1 wbar_2
      wbar_1 = P u1bar;  u0bar = wbar_1 + J(u_0)^T (dt g1 wbar_1 + F0bar).
    """
    us, _ = wray3_stages(u0, h, nu, dt, rhs_fn, project_fn)
    G = rhs_vjp_fn if rhs_vjp_fn is not None else (lambda v, fb: rhs_vjp(v, fb, h, nu))
    PT = project_vjp_fn if project_vjp_fn is not None else (lambda v: project_vjp(v, h))
    wbar = PT(u1bar)
    ubar = wbar + G(us[2], dt * WRAY3_G[2] * wbar)
    f1bar = dt * WRAY3_Z[1] * wbar
    wbar = PT(ubar)
    ubar = wbar + G(us[1], dt * WRAY3_G[1] * wbar + f1bar)
    f0bar = dt * WRAY3_Z[0] * wbar
    wbar = PT(ubar)
    return wbar + G(us[0], dt * WRAY3_G[0] * wbar + f0bar)


# ----------------------------------------------------------------------------
# Unrolled trajectory loss and its gradient (back-propagation relation, Sec. 3.4)
# ----------------------------------------------------------------------------

def rollout_loss(u0, refs, h, nu, dt):
    """L(u0) = (1/S) sum_{s=1..S} mean((u_s - refs[s-1])^2), u_s = step_rk4^s(u0)."""
    S = len(refs)
    u = np.array(u0, dtype=np.float64)
    total = 0.0
    for s in range(S):
        u = step_rk4(u, h, nu, dt)
        total += float(np.mean((u - refs[s]) ** 2)) / S
    return total


def rollout_loss_grad(u0, refs, h, nu, dt):
    """dL/du0: store the states, then run x_bar_n = pullback_n(x_bar_{n+1}) from the last step back."""
    S = len(refs)
    states = [np.array(u0, dtype=np.float64)]
    for s in range(S):
        states.append(step_rk4(states[-1], h, nu, dt))
    m = states[0].size
    ubar = np.zeros_like(states[0])
    for s in range(S, 0, -1):
        ubar = ubar + 2.0 * (states[s] - refs[s - 1]) / (m * S)
        ubar = step_rk4_vjp(states[s - 1], ubar, h, nu, dt)
    return ubar
