"""Float64 oracle of the staggered operators, pressure solves, time steps and
pullbacks on a channel: no-slip walls at both ends of the y direction, x (and
z) periodic.

TEST INFRASTRUCTURE ONLY (see the package docstring). Not used by the product path.

Boundary treatment (Sec. 2.1, boundary conditions: Dirichlet velocity imposed
through ghost volumes adjacent to the domain; the paper gives no ghost
formula, the reading taken here is stated in full):

* cells I_y = 0 .. N_y - 1 span [lo_y + I_y h_y, lo_y + (I_y + 1) h_y]; the
  walls sit at lo_y and hi_y;
* the normal velocity u^y lives on the y-faces; the face right of cell
  N_y - 1 is the upper wall and the face left of cell 0 (index -1) the lower
  one. Both hold the prescribed value 0: they are boundary values, not
  unknowns. Storage keeps the periodic layout, so u^y[..., N_y - 1, ...] is
  that wall face; every operator reads it as 0 and writes 0 there;
* the tangential components (x, z) sit at cell centres in y. Their ghost
  values one cell beyond a wall are chosen so the linear interpolant between
  ghost and first interior centre vanishes on the wall:
  u^a[-1] = -u^a[0], u^a[N_y] = -u^a[N_y - 1];
* pressure lives at the N_y centres; the gradient is formed on the interior
  y-faces only (none on the walls), so L = D G is the Neumann Laplacian;
  its null space is the constants.

With these rules D^T = -G on the unknowns, the diffusion operator is symmetric
and negative definite, and every convective flux through a wall vanishes
identically (one of its two factors is the zero wall velocity, the other the
zero wall interpolant), so convection stays energy-conserving for solenoidal
fields.

Arrays keep the periodic layout: velocity (d, [N_z,] N_y, N_x), pressure
([N_z,] N_y, N_x). Internally a component is extended to N_y + 2 rows
(padded row k holds index I_y = k - 1) by ``_pad``; pullbacks fold the padded
cotangent back with ``_fold``, the transpose of ``_pad``.

Pressure solves (Sec. 2.5.1): ``poisson_solve`` is the direct solver, the
augmented system [L e; e^T 0] [p; lam] = [r; 0] solved with a sparse LU
factorisation (so p has zero mean and L p = r - mean(r)); ``cg_solve`` is the
iterative solver, conjugate gradients with the Laplace operator applied as the
divergence of the gradient, never assembled.
"""
from __future__ import annotations

import numpy as np

from . import ins

Y = 1  # wall-normal direction


def _yaxis(d):
    """Array axis of the y direction in a component or pressure array."""
    return d - 2


def _rows(f, start, count, d):
    sl = [slice(None)] * f.ndim
    sl[_yaxis(d)] = slice(start, start + count)
    return f[tuple(sl)]


def _roll_periodic(f, shift, d):
    """f[I + shift] along the periodic directions (shift[a] for a != y)."""
    for a in range(d):
        if a != Y and shift[a]:
            f = np.roll(f, -shift[a], axis=d - 1 - a)
    return f


def _unit(a, d, s=1):
    e = [0] * d
    e[a] = s
    return e


def dof_mask(n):
    """1 on the velocity unknowns, 0 on the upper-wall face of u^y."""
    d = len(n)
    m = np.ones((d,) + tuple(reversed(n)))
    sl = [Y] + [slice(None)] * d
    sl[1 + _yaxis(d)] = n[Y] - 1
    m[tuple(sl)] = 0.0
    return m


def _pad(u, a):
    """Component a of u extended by one ghost row below and above the walls."""
    d = u.shape[0]
    ny = u.shape[1 + _yaxis(d)]
    c = u[a]
    if a == Y:
        inner = _rows(c, 0, ny - 1, d)  # faces 0 .. N_y - 2 (unknowns)
        z = np.zeros_like(_rows(c, 0, 1, d))
        return np.concatenate([z, inner, z, z], axis=_yaxis(d))  # rows -1, 0..N_y-2, N_y-1 (wall), N_y
    lo = -_rows(c, 0, 1, d)
    hi = -_rows(c, ny - 1, 1, d)
    return np.concatenate([lo, c, hi], axis=_yaxis(d))


def _fold(pbar, a, d, ny):
    """Transpose of _pad: cotangent of the padded rows -> cotangent of component a."""
    inner = _rows(pbar, 1, ny, d).copy()
    if a == Y:
        sl = [slice(None)] * inner.ndim
        sl[_yaxis(d)] = ny - 1
        inner[tuple(sl)] = 0.0  # the wall face is a constant, not an unknown
        return inner
    sl0 = [slice(None)] * inner.ndim
    sl0[_yaxis(d)] = slice(0, 1)
    inner[tuple(sl0)] -= _rows(pbar, 0, 1, d)
    sl1 = [slice(None)] * inner.ndim
    sl1[_yaxis(d)] = slice(ny - 1, ny)
    inner[tuple(sl1)] -= _rows(pbar, ny + 1, 1, d)
    return inner


def _at(P, shift, d, ny, extra=0):
    """Padded component P at I + shift for I_y = -extra .. N_y - 1."""
    return _rows(_roll_periodic(P, shift, d), 1 - extra + shift[Y], ny + extra, d)


def _at_T(X, shift, d, ny, shape, extra=0):
    """Transpose of _at: scatter X (rows I_y = -extra .. N_y - 1) into a zero padded array."""
    out = np.zeros(shape)
    sl = [slice(None)] * len(shape)
    sl[_yaxis(d)] = slice(1 - extra + shift[Y], 1 - extra + shift[Y] + ny + extra)
    out[tuple(sl)] += X
    neg = [-s if a != Y else 0 for a, s in enumerate(shift)]
    return _roll_periodic(out, neg, d)


# ----------------------------------------------------------------------------
# Forward operators (App. B kernels with the wall rules above)
# ----------------------------------------------------------------------------

def divergence(u, h):
    """r[I] = sum_a (u^a[I] - u^a[I - e_a]) / h_a, wall faces read as 0."""
    d = u.shape[0]
    ny = u.shape[1 + _yaxis(d)]
    r = np.zeros(u.shape[1:])
    for a in range(d):
        P = _pad(u, a)
        r += (_at(P, [0] * d, d, ny) - _at(P, _unit(a, d, -1), d, ny)) / h[a]
    return r


def gradient(p, h):
    """(G p)^a[I] = (p[I + e_a] - p[I]) / h_a on the interior faces; 0 on the upper wall face of u^y."""
    g = ins.gradient(p, h)
    return g * dof_mask(tuple(reversed(p.shape)))


def diffusion(u, h, nu):
    """nu sum_b (u^a[I + e_b] - 2 u^a[I] + u^a[I - e_b]) / h_b^2 with ghost values; 0 on the wall face."""
    d = u.shape[0]
    ny = u.shape[1 + _yaxis(d)]
    out = np.zeros(u.shape)
    for a in range(d):
        P = _pad(u, a)
        c = _at(P, [0] * d, d, ny)
        for b in range(d):
            out[a] += (_at(P, _unit(b, d), d, ny) - 2.0 * c + _at(P, _unit(b, d, -1), d, ny)) / h[b] ** 2
    return nu * out * dof_mask(tuple(reversed(u.shape[1:])))


def _fluxes(u, a, b, d, ny):
    """a- and b-factors of F^{ab}[I] for I_y = -1 .. N_y - 1 (N_y + 1 rows)."""
    Pa, Pb = _pad(u, a), _pad(u, b)
    z = [0] * d
    fa = 0.5 * (_at(Pa, z, d, ny, 1) + _at(Pa, _unit(b, d), d, ny, 1))
    fb = 0.5 * (_at(Pb, z, d, ny, 1) + _at(Pb, _unit(a, d), d, ny, 1))
    return fa, fb


def _flux_at(F, shift_b, d, ny):
    """F (rows I_y = -1 .. N_y - 1) at I - e_b for I_y = 0 .. N_y - 1; shift_b = e_b."""
    if shift_b[Y]:
        return _rows(F, 0, ny, d)
    return _roll_periodic(_rows(F, 1, ny, d), [-s for s in shift_b], d)


def convection(u, h):
    """phi^a[I] = -sum_b (F^{ab}[I] - F^{ab}[I - e_b]) / h_b (App. B convection kernel, weights 1/2)."""
    d = u.shape[0]
    ny = u.shape[1 + _yaxis(d)]
    out = np.zeros(u.shape)
    for a in range(d):
        for b in range(d):
            fa, fb = _fluxes(u, a, b, d, ny)
            F = fa * fb
            out[a] -= (_rows(F, 1, ny, d) - _flux_at(F, _unit(b, d), d, ny)) / h[b]
    return out * dof_mask(tuple(reversed(u.shape[1:])))


def rhs(u, h, nu):
    return convection(u, h) + diffusion(u, h, nu)


def laplacian(p, h):
    """L p = D G p (Neumann at the walls)."""
    return divergence(gradient(p, h), h)


# ----------------------------------------------------------------------------
# Pressure solves (Sec. 2.5.1)
# ----------------------------------------------------------------------------

def laplace_matrix(n, h):
    """Sparse matrix of L = D G on the flattened pressure array, written from the stencil:
    -2/h_a^2 on the diagonal and 1/h_a^2 to both periodic neighbours per periodic direction;
    in y, 1/h_y^2 to each existing neighbour and -1/h_y^2 on the diagonal per existing neighbour."""
    import scipy.sparse as sp

    d = len(n)
    shape = tuple(reversed(n))
    idx = np.arange(int(np.prod(shape))).reshape(shape)
    rows, cols, vals = [], [], []
    for a in range(d):
        ax = d - 1 - a
        w = 1.0 / h[a] ** 2
        for s in (1, -1):
            nb = np.roll(idx, -s, axis=ax)
            valid = np.ones(shape, dtype=bool)
            if a == Y:
                coord = np.arange(n[a]).reshape([-1 if k == ax else 1 for k in range(d)])
                valid = np.broadcast_to((coord + s >= 0) & (coord + s <= n[a] - 1), shape)
            rows += [idx[valid], idx[valid]]
            cols += [nb[valid], idx[valid]]
            vals += [np.full(int(valid.sum()), w), np.full(int(valid.sum()), -w)]
    m = idx.size
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(m, m))


def poisson_solve(r, h):
    """Direct solver of Sec. 2.5.1: [L e; e^T 0][p; lam] = [r; 0] (sparse LU)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    n = tuple(reversed(r.shape))
    L = laplace_matrix(n, h)
    m = L.shape[0]
    e = sp.csr_matrix(np.ones((m, 1)))
    A = sp.bmat([[L, e], [e.T, None]], format="csc")
    sol = spla.spsolve(A, np.concatenate([r.ravel(), [0.0]]))
    return sol[:m].reshape(r.shape)


def cg_solve(r, h, rtol=1e-12, maxiter=10000):
    """Iterative solver of Sec. 2.5.1: conjugate gradients on A = -D G (positive
    semi-definite) for A p = -(r - mean r), from p = 0, with A applied matrix-free.

    Stops once ||res|| <= rtol ||res_0|| or after maxiter iterations; returns
    (p, iterations, ||res|| / ||res_0||) with res the recursively updated residual.
    """
    b = -(r - np.mean(r))
    x = np.zeros_like(b)
    res = b.copy()
    d = res.copy()
    rr = float(np.sum(res * res))
    rr0 = rr
    it = 0
    if rr0 == 0.0:
        return x, 0, 0.0
    while it < maxiter and rr > rtol * rtol * rr0:
        q = -laplacian(d, h)
        alpha = rr / float(np.sum(d * q))
        x = x + alpha * d
        res = res - alpha * q
        rr_new = float(np.sum(res * res))
        d = res + (rr_new / rr) * d
        rr = rr_new
        it += 1
    return x, it, float(np.sqrt(rr / rr0))


def project(u, h, solve=None):
    """P u = u - G L^{-1} D u on the unknowns (the projection of Sec. 2.5.2)."""
    solve = solve or poisson_solve
    p = solve(divergence(u, h), h)
    return (u - gradient(p, h)) * dof_mask(tuple(reversed(u.shape[1:]))), p


# ----------------------------------------------------------------------------
# Pullbacks (Sec. 3.4 rule), each the transpose of the forward formula
# ----------------------------------------------------------------------------

def divergence_vjp(rbar, h):
    """ubar^a[J] = (rbar[J] - rbar[J + e_a]) / h_a on the unknowns (0 on the wall face)."""
    d = rbar.ndim
    ny = rbar.shape[_yaxis(d)]
    out = np.zeros((d,) + rbar.shape)
    for a in range(d):
        # r[I] reads the padded component at I and I - e_a; scatter back and fold
        shape = list(rbar.shape)
        shape[_yaxis(d)] = ny + 2
        Pbar = _at_T(rbar / h[a], [0] * d, d, ny, shape) - _at_T(rbar / h[a], _unit(a, d, -1), d, ny, shape)
        out[a] = _fold(Pbar, a, d, ny)
    return out


def gradient_vjp(gbar, h):
    """pbar[I] = sum_a (gbar^a[I - e_a] - gbar^a[I]) / h_a over the interior faces only."""
    return ins.gradient_vjp(gbar * dof_mask(tuple(reversed(gbar.shape[1:]))), h)


def diffusion_vjp(fbar, h, nu):
    """Transpose of ``diffusion``: scatter the stencil onto the padded rows, then fold the ghosts."""
    d = fbar.shape[0]
    ny = fbar.shape[1 + _yaxis(d)]
    fb = fbar * dof_mask(tuple(reversed(fbar.shape[1:])))
    shape = list(fbar.shape[1:])
    shape[_yaxis(d)] = ny + 2
    out = np.zeros(fbar.shape)
    for a in range(d):
        Pbar = np.zeros(shape)
        for b in range(d):
            w = nu * fb[a] / h[b] ** 2
            Pbar += _at_T(w, _unit(b, d), d, ny, shape) - 2.0 * _at_T(w, [0] * d, d, ny, shape)
            Pbar += _at_T(w, _unit(b, d, -1), d, ny, shape)
        out[a] = _fold(Pbar, a, d, ny)
    return out


def convection_vjp(u, fbar, h):
    """Transpose of ``convection`` at u: Fbar from the divergence of the fluxes,
    abar = Fbar * (b-factor), bbar = Fbar * (a-factor), each averaged back onto
    the padded rows it was read from, then folded."""
    d = u.shape[0]
    ny = u.shape[1 + _yaxis(d)]
    fb = fbar * dof_mask(tuple(reversed(u.shape[1:])))
    shape = list(u.shape[1:])
    shape[_yaxis(d)] = ny + 2
    Pbar = [np.zeros(shape) for _ in range(d)]
    z = [0] * d
    for a in range(d):
        for b in range(d):
            fa, fbf = _fluxes(u, a, b, d, ny)
            # phi^a[I] -= (F[I] - F[I - e_b]) / h_b, I_y = 0..N_y-1; F rows I_y = -1..N_y-1
            Fbar = np.zeros(fa.shape)
            g = fb[a] / h[b]
            sl = [slice(None)] * Fbar.ndim
            sl[_yaxis(d)] = slice(1, ny + 1)
            Fbar[tuple(sl)] -= g
            if b == Y:
                sl[_yaxis(d)] = slice(0, ny)
                Fbar[tuple(sl)] += g
            else:
                sl[_yaxis(d)] = slice(1, ny + 1)
                Fbar[tuple(sl)] += _roll_periodic(g, _unit(b, d), d)
            abar = 0.5 * Fbar * fbf
            bbar = 0.5 * Fbar * fa
            Pbar[a] += _at_T(abar, z, d, ny, shape, 1) + _at_T(abar, _unit(b, d), d, ny, shape, 1)
            Pbar[b] += _at_T(bbar, z, d, ny, shape, 1) + _at_T(bbar, _unit(a, d), d, ny, shape, 1)
    return np.stack([_fold(Pbar[a], a, d, ny) for a in range(d)])


def rhs_vjp(u, fbar, h, nu):
    return convection_vjp(u, fbar, h) + diffusion_vjp(fbar, h, nu)


def project_vjp(ubar_out, h):
    """P^T = I - D^T L^{-T} G^T = I - G L^{-1} D = P on the unknowns (D^T = -G, L symmetric)."""
    return project(ubar_out, h)[0]


# ----------------------------------------------------------------------------
# Time steps: the periodic schedules of the oracle with the channel's
# right-hand side and projection.
# ----------------------------------------------------------------------------

def _fns(h, nu):
    return dict(rhs_fn=lambda v: rhs(v, h, nu), project_fn=lambda v: project(v, h)[0])


def step_rk4(u0, h, nu, dt):
    return ins.step_rk4(u0, h, nu, dt, **_fns(h, nu))


def step_wray3(u0, h, nu, dt):
    return ins.step_wray3(u0, h, nu, dt, **_fns(h, nu))


def step_rk4_vjp(u0, u1bar, h, nu, dt):
    return ins.step_rk4_vjp(u0, u1bar, h, nu, dt, rhs_vjp_fn=lambda v, fb: rhs_vjp(v, fb, h, nu),
                            project_vjp_fn=lambda v: project_vjp(v, h), **_fns(h, nu))


def step_wray3_vjp(u0, u1bar, h, nu, dt):
    return ins.step_wray3_vjp(u0, u1bar, h, nu, dt, rhs_vjp_fn=lambda v, fb: rhs_vjp(v, fb, h, nu),
                              project_vjp_fn=lambda v: project_vjp(v, h), **_fns(h, nu))
