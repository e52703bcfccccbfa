"""Float64 oracle of the staggered operators, pressure solves, time steps and
pullbacks on a channel: no-slip walls at both ends of the y direction, x (and
z) periodic and uniform; the y direction uniform or stretched.

TEST INFRASTRUCTURE ONLY (see the package docstring). Not used by the product path.

Grid. ``h = (h_x, h_y[, h_z])``; ``h_y`` is either a spacing (uniform) or the
array of the N_y + 1 y-face coordinates y_0 < ... < y_{N_y} (the walls are
y_0 and y_{N_y}; Sec. 2.5 volumes Delta^y_i and App. B widths |Delta^y_i|).
In code indices: w_j = y_{j+1} - y_j is the width of cell row j (a pressure
volume, half-integer paper index j + 1/2), c_j its centre, and
d_j = c_{j+1} - c_j the width of the velocity volume around y-face j (the face
on top of row j, integer paper index j + 1). Beyond a wall a ghost row mirrors
the first/last row, so d_{-1} = w_0 and d_{N_y - 1} = w_{N_y - 1}.

Boundary treatment (Sec. 2.4, boundary conditions: Dirichlet velocity imposed
through ghost volumes adjacent to the domain; the paper gives no ghost
formula, the reading taken here is stated in full):

* the normal velocity u^y lives on the y-faces; the face on top of the last
  row (index N_y - 1) is the upper wall and the face below row 0 (index -1)
  the lower one. Both hold the prescribed value 0: they are boundary values,
  not unknowns. Storage keeps the periodic layout, so u^y[..., N_y - 1, ...]
  is that wall face; every operator reads it as 0 and writes 0 there;
* the tangential components (x, z) sit at cell centres in y. Their ghost
  values one row beyond a wall are minus the first interior value, so the
  linear interpolant vanishes on the wall (which lies midway between the
  ghost centre and the first centre);
* pressure lives at the N_y centres; the gradient is formed on the interior
  y-faces only (none on the walls), so L = D G is the Neumann Laplacian; its
  null space is the constants.

Operators (App. B, with the widths above; x, z spacings uniform):
  divergence  r[I] = sum_a (u^a[I] - u^a[I - e_a]) / |Delta^a|, cell widths;
  gradient    (G p)^a[I] = (p[I + e_a] - p[I]) / |Delta^a|, velocity-volume widths;
  diffusion   App. B eq. diff-kernel: outer width of the velocity volume,
              inner widths between the neighbouring points;
  convection  phi^a[I] = -sum_b (F^{ab}[I] - F^{ab}[I - e_b]) / |Delta^b| with
              F^{ab} = a^{ab} b^{ab}: the transported component u^a averaged
              along b with weights 1/2, the transporting component u^b
              interpolated along a as the mass-flux average of the two
              pressure-volume faces it spans (weights w_j / (w_j + w_{j+1}) on a
              stretched y, 1/2 otherwise); on a uniform grid every weight is 1/2.
              The 1/2 average of the transported component makes the flux form
              skew; the mass-flux average makes each velocity volume's discrete
              divergence of the transporting velocity a combination of the two
              pressure volumes' divergences, so convection conserves energy
              for solenoidal fields on a stretched grid too.

With these rules D and G are dual in the volume-weighted inner products
(sum Omega_p (D u) p = -sum Omega_u u (G p)), diffusion is symmetric in the
velocity-volume inner product, every convective flux through a wall vanishes
identically, and sum Omega_u u . C(u) = 0 for solenoidal u.

Arrays keep the periodic layout: velocity (d, [N_z,] N_y, N_x), pressure
([N_z,] N_y, N_x). Internally a component is extended to N_y + 2 rows
(padded row k holds index I_y = k - 1) by ``_pad``; pullbacks fold the padded
cotangent back with ``_fold``, the transpose of ``_pad``.

Pressure solves (Sec. 2.6.1): ``poisson_solve`` is the direct solver, the
augmented system [L e; e^T 0] [p; lam] = [r; 0] solved with a sparse LU
factorisation (p has zero mean and L p = r - lam, lam the volume-weighted mean
of r); ``cg_solve`` is the iterative solver: conjugate gradients on the
symmetric A = -Omega_p D G (the volume scaling makes it symmetric) applied as a
chain of scaling, divergence and gradient, never assembled.
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


# ----------------------------------------------------------------------------
# y metrics
# ----------------------------------------------------------------------------

def y_faces(h, ny):
    """The N_y + 1 y-face coordinates (from 0 for a uniform spacing)."""
    hy = h[Y]
    if np.ndim(hy) == 0:
        return np.arange(ny + 1) * float(hy)
    yf = np.asarray(hy, dtype=np.float64)
    assert yf.shape == (ny + 1,) and np.all(np.diff(yf) > 0)
    return yf


def _metrics(h, ny):
    """w_j (cell widths), d_j for j = -1 .. N_y - 1 (entry j + 1), theta_j (j = 0 .. N_y - 1).
    A scalar h_y gives exactly constant widths and weights 1/2."""
    if np.ndim(h[Y]) == 0:
        hy = float(h[Y])
        return np.full(ny, hy), np.full(ny + 1, hy), np.full(ny, 0.5)
    yf = y_faces(h, ny)
    w = np.diff(yf)
    c = 0.5 * (yf[:-1] + yf[1:])
    d = np.empty(ny + 1)
    d[0] = w[0]
    d[1:ny] = np.diff(c)
    d[ny] = w[-1]
    theta = np.full(ny, 0.5)
    theta[: ny - 1] = w[:-1] / (w[:-1] + w[1:])
    return w, d, theta


def _rowvec(v, d, shape_rows):
    """Broadcast a per-row vector along the y axis of a d-dimensional component array."""
    sh = [1] * d
    sh[_yaxis(d)] = shape_rows
    return np.asarray(v).reshape(sh)


def cell_widths(h, ny):
    return _metrics(h, ny)[0]


def volumes_u(h, n):
    """Velocity-volume sizes Omega^a_I (velocity layout), y-faces with d_j (wall face: d of the wall)."""
    d = len(n)
    ny = n[Y]
    w, dd, _ = _metrics(h, ny)
    out = np.ones((d,) + tuple(reversed(n)))
    for a in range(d):
        ext = 1.0
        for b in range(d):
            if b != Y:
                ext *= float(h[b])
        if a == Y:
            out[a] *= ext * _rowvec(dd[1:], d, ny)
        else:
            out[a] *= ext * _rowvec(w, d, ny)
    return out


def volumes_p(h, n):
    """Pressure-volume sizes Omega_I."""
    d = len(n)
    ny = n[Y]
    w = cell_widths(h, ny)
    ext = 1.0
    for b in range(d):
        if b != Y:
            ext *= float(h[b])
    return ext * np.broadcast_to(_rowvec(w, d, ny), tuple(reversed(n))).copy()


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


def _inv_width_div(h, a, d, ny):
    """1 / |Delta^a| of the pressure volume (per row for a = y)."""
    if a == Y:
        return _rowvec(1.0 / cell_widths(h, ny), d, ny)
    return 1.0 / float(h[a])


def _inv_width_grad(h, a, d, ny):
    """1 / |Delta^a| of the a-velocity volume (per row for a = y; d_j, rows 0..N_y-1)."""
    if a == Y:
        dd = _metrics(h, ny)[1]
        return _rowvec(1.0 / dd[1:], d, ny)
    return 1.0 / float(h[a])


# ----------------------------------------------------------------------------
# Forward operators (App. B kernels with the wall rules above)
# ----------------------------------------------------------------------------

def divergence(u, h):
    """r[I] = sum_a (u^a[I] - u^a[I - e_a]) / |Delta^a|, wall faces read as 0."""
    d = u.shape[0]
    ny = u.shape[1 + _yaxis(d)]
    r = np.zeros(u.shape[1:])
    for a in range(d):
        P = _pad(u, a)
        r += (_at(P, [0] * d, d, ny) - _at(P, _unit(a, d, -1), d, ny)) * _inv_width_div(h, a, d, ny)
    return r


def gradient(p, h):
    """(G p)^a[I] = (p[I + e_a] - p[I]) / |Delta^a| on the interior faces; 0 on the upper wall face of u^y."""
    d = p.ndim
    ny = p.shape[_yaxis(d)]
    g = np.stack([(ins._next(p, a, d) - p) * _inv_width_grad(h, a, d, ny) for a in range(d)])
    return g * dof_mask(tuple(reversed(p.shape)))


def _diff_coeffs(h, a, b, d, ny):
    """(outer, inner right, inner left) inverse widths of eq. diff-kernel for component a along b."""
    if b != Y:
        ih = 1.0 / float(h[b])
        return ih, ih, ih
    w, dd, _ = _metrics(h, ny)
    if a == Y:  # u^y at face j: outer d_j, inner w_{j+1} (above), w_j (below)
        wn = np.append(w[1:], w[-1])
        return (_rowvec(1.0 / dd[1:], d, ny), _rowvec(1.0 / wn, d, ny), _rowvec(1.0 / w, d, ny))
    # tangential at row j: outer w_j, inner d_j (above), d_{j-1} (below)
    return (_rowvec(1.0 / w, d, ny), _rowvec(1.0 / dd[1:], d, ny), _rowvec(1.0 / dd[:-1], d, ny))


def diffusion(u, h, nu):
    """App. B eq. diff-kernel with ghost values; 0 on the wall face."""
    d = u.shape[0]
    ny = u.shape[1 + _yaxis(d)]
    out = np.zeros(u.shape)
    for a in range(d):
        P = _pad(u, a)
        c = _at(P, [0] * d, d, ny)
        for b in range(d):
            o, ir, il = _diff_coeffs(h, a, b, d, ny)
            out[a] += o * ((_at(P, _unit(b, d), d, ny) - c) * ir - (c - _at(P, _unit(b, d, -1), d, ny)) * il)
    return nu * out * dof_mask(tuple(reversed(u.shape[1:])))


def _theta_rows(h, d, ny, extra):
    """Mass-flux weight of row j in the y-face j|j+1, for rows -extra .. N_y - 1 (1/2 outside)."""
    th = _metrics(h, ny)[2]
    if extra:
        th = np.concatenate([[0.5], th])
    return _rowvec(th, d, ny + extra)


def _fluxes(u, h, a, b, d, ny):
    """a- and b-factors of F^{ab}[K] for K_y = -1 .. N_y - 1 (N_y + 1 rows)."""
    Pa, Pb = _pad(u, a), _pad(u, b)
    z = [0] * d
    fa = 0.5 * (_at(Pa, z, d, ny, 1) + _at(Pa, _unit(b, d), d, ny, 1))
    if a == Y and b != Y:
        th = _theta_rows(h, d, ny, 1)
        fb = th * _at(Pb, z, d, ny, 1) + (1.0 - th) * _at(Pb, _unit(a, d), d, ny, 1)
    else:
        fb = 0.5 * (_at(Pb, z, d, ny, 1) + _at(Pb, _unit(a, d), d, ny, 1))
    return fa, fb


def _conv_inv_width(h, a, b, d, ny):
    """1 / |Delta^b| of the a-velocity volume (rows 0..N_y-1)."""
    if b != Y:
        return 1.0 / float(h[b])
    w, dd, _ = _metrics(h, ny)
    return _rowvec(1.0 / (dd[1:] if a == Y else w), d, ny)


def _flux_at(F, shift_b, d, ny):
    """F (rows I_y = -1 .. N_y - 1) at I - e_b for I_y = 0 .. N_y - 1; shift_b = e_b."""
    if shift_b[Y]:
        return _rows(F, 0, ny, d)
    return _roll_periodic(_rows(F, 1, ny, d), [-s for s in shift_b], d)


def convection(u, h):
    """phi^a[I] = -sum_b (F^{ab}[I] - F^{ab}[I - e_b]) / |Delta^b| (App. B convection kernel)."""
    d = u.shape[0]
    ny = u.shape[1 + _yaxis(d)]
    out = np.zeros(u.shape)
    for a in range(d):
        for b in range(d):
            fa, fb = _fluxes(u, h, a, b, d, ny)
            F = fa * fb
            out[a] -= (_rows(F, 1, ny, d) - _flux_at(F, _unit(b, d), d, ny)) * _conv_inv_width(h, a, b, d, ny)
    return out * dof_mask(tuple(reversed(u.shape[1:])))


def rhs(u, h, nu, force=None):
    """F(u) = C(u) + nu D(u) + f (App. A momentum equation, the forcing collected in F):
    f a constant vector (the channel's driving body force, Sec. 6), added on the
    velocity unknowns only."""
    out = convection(u, h) + diffusion(u, h, nu)
    if force is not None:
        mask = dof_mask(tuple(reversed(u.shape[1:])))
        for a in range(u.shape[0]):
            out[a] += float(force[a]) * mask[a]
    return out


def laplacian(p, h):
    """L p = D G p (Neumann at the walls)."""
    return divergence(gradient(p, h), h)


# ----------------------------------------------------------------------------
# Pressure solves (Sec. 2.6.1)
# ----------------------------------------------------------------------------

def laplace_matrix(n, h):
    """Sparse matrix of L = D G on the flattened pressure array, written from the stencil:
    per periodic direction -2/h_a^2 on the diagonal and 1/h_a^2 to both neighbours; in y,
    1/(w_j d) to each existing neighbour across a face of width d and minus that on the
    diagonal."""
    import scipy.sparse as sp

    d = len(n)
    ny = n[Y]
    w, dd, _ = _metrics(h, ny)
    shape = tuple(reversed(n))
    idx = np.arange(int(np.prod(shape))).reshape(shape)
    rows, cols, vals = [], [], []
    for a in range(d):
        ax = d - 1 - a
        for s in (1, -1):
            nb = np.roll(idx, -s, axis=ax)
            if a == Y:
                j = np.broadcast_to(_rowvec(np.arange(ny), d, ny), shape)
                valid = (j + s >= 0) & (j + s <= ny - 1)
                face = np.where(s > 0, j, j - 1)  # face index between the two rows
                coef = 1.0 / (w[j] * dd[np.clip(face, -1, ny - 1) + 1])
            else:
                valid = np.ones(shape, dtype=bool)
                coef = np.full(shape, 1.0 / float(h[a]) ** 2)
            rows += [idx[valid], idx[valid]]
            cols += [nb[valid], idx[valid]]
            vals += [coef[valid], -coef[valid]]
    m = idx.size
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(m, m))


def _augmented(n, h):
    import scipy.sparse as sp

    L = laplace_matrix(n, h)
    m = L.shape[0]
    e = sp.csr_matrix(np.ones((m, 1)))
    return sp.bmat([[L, e], [e.T, None]], format="csc"), m


def poisson_solve(r, h):
    """Direct solver of Sec. 2.6.1: [L e; e^T 0][p; lam] = [r; 0] (sparse LU)."""
    import scipy.sparse.linalg as spla

    A, m = _augmented(tuple(reversed(r.shape)), h)
    sol = spla.spsolve(A, np.concatenate([r.ravel(), [0.0]]))
    return sol[:m].reshape(r.shape)


def cg_solve(r, h, rtol=1e-12, maxiter=10000):
    """Iterative solver of Sec. 2.6.1: conjugate gradients on the symmetric positive
    semi-definite A = -Omega_p D G for A p = -Omega_p (r - rbar), rbar the volume-weighted
    mean of r, from p = 0, with A applied matrix-free (scaling, divergence, gradient).

    Stops once ||res|| <= rtol ||res_0|| or after maxiter iterations, or when the
    search direction has no component outside the null space (p . A p <= 0: the
    remaining residual is a constant, which the gradient does not see); returns
    (p, iterations, ||res|| / ||res_0||) with res the recursively updated residual
    (0 after such a breakdown).
    """
    n = tuple(reversed(r.shape))
    om = volumes_p(h, n)
    rbar = float(np.sum(om * r) / np.sum(om))
    b = -om * (r - rbar)
    x = np.zeros_like(b)
    res = b.copy()
    dvec = res.copy()
    rr = float(np.sum(res * res))
    rr0 = rr
    it = 0
    if rr0 == 0.0:
        return x, 0, 0.0
    while it < maxiter and rr > rtol * rtol * rr0:
        q = -om * laplacian(dvec, h)
        pq = float(np.sum(dvec * q))
        if not pq > 0.0:
            rr = 0.0
            break
        alpha = rr / pq
        x = x + alpha * dvec
        res = res - alpha * q
        rr_new = float(np.sum(res * res))
        dvec = res + (rr_new / rr) * dvec
        rr = rr_new
        it += 1
    return x, it, float(np.sqrt(rr / rr0))


def project(u, h, solve=None):
    """P u = u - G L^{-1} D u on the unknowns (the projection of Sec. 2.6.2)."""
    solve = solve or poisson_solve
    p = solve(divergence(u, h), h)
    return (u - gradient(p, h)) * dof_mask(tuple(reversed(u.shape[1:]))), p


# ----------------------------------------------------------------------------
# Pullbacks (Sec. 3.4 rule), each the transpose of the forward formula
# ----------------------------------------------------------------------------

def divergence_vjp(rbar, h):
    """Transpose of ``divergence``: scatter onto the padded rows, fold; 0 on the wall face."""
    d = rbar.ndim
    ny = rbar.shape[_yaxis(d)]
    out = np.zeros((d,) + rbar.shape)
    shape = list(rbar.shape)
    shape[_yaxis(d)] = ny + 2
    for a in range(d):
        g = rbar * _inv_width_div(h, a, d, ny)
        Pbar = _at_T(g, [0] * d, d, ny, shape) - _at_T(g, _unit(a, d, -1), d, ny, shape)
        out[a] = _fold(Pbar, a, d, ny)
    return out


def gradient_vjp(gbar, h):
    """Transpose of ``gradient``: pbar[I] = sum_a (gbar^a[I - e_a] s[I - e_a] - gbar^a[I] s[I])."""
    d = gbar.shape[0]
    ny = gbar.shape[1 + _yaxis(d)]
    gb = gbar * dof_mask(tuple(reversed(gbar.shape[1:])))
    out = np.zeros(gbar.shape[1:])
    for a in range(d):
        t = gb[a] * _inv_width_grad(h, a, d, ny)
        out += ins._prev(t, a, d) - t
    return out


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
            o, ir, il = _diff_coeffs(h, a, b, d, ny)
            g = nu * fb[a] * o
            Pbar += _at_T(g * ir, _unit(b, d), d, ny, shape) - _at_T(g * (ir + il), [0] * d, d, ny, shape)
            Pbar += _at_T(g * il, _unit(b, d, -1), d, ny, shape)
        out[a] = _fold(Pbar, a, d, ny)
    return out


def convection_vjp(u, fbar, h):
    """Transpose of ``convection`` at u: Fbar from the divergence of the fluxes,
    abar = Fbar * (b-factor), bbar = Fbar * (a-factor), each scattered back onto
    the padded rows it was read from with its interpolation weights, then folded."""
    d = u.shape[0]
    ny = u.shape[1 + _yaxis(d)]
    fb = fbar * dof_mask(tuple(reversed(u.shape[1:])))
    shape = list(u.shape[1:])
    shape[_yaxis(d)] = ny + 2
    Pbar = [np.zeros(shape) for _ in range(d)]
    z = [0] * d
    for a in range(d):
        for b in range(d):
            fa, fbf = _fluxes(u, h, a, b, d, ny)
            # phi^a[I] -= (F[I] - F[I - e_b]) s[I], I_y = 0..N_y-1; F rows I_y = -1..N_y-1
            Fbar = np.zeros(fa.shape)
            g = fb[a] * _conv_inv_width(h, a, b, d, ny)
            sl = [slice(None)] * Fbar.ndim
            sl[_yaxis(d)] = slice(1, ny + 1)
            Fbar[tuple(sl)] -= g
            if b == Y:
                sl[_yaxis(d)] = slice(0, ny)
                Fbar[tuple(sl)] += g
            else:
                Fbar[tuple(sl)] += _roll_periodic(g, _unit(b, d), d)
            abar = Fbar * fbf
            bbar = Fbar * fa
            Pbar[a] += _at_T(0.5 * abar, z, d, ny, shape, 1) + _at_T(0.5 * abar, _unit(b, d), d, ny, shape, 1)
            if a == Y and b != Y:
                th = _theta_rows(h, d, ny, 1)
                Pbar[b] += _at_T(th * bbar, z, d, ny, shape, 1) + _at_T((1.0 - th) * bbar, _unit(a, d), d, ny, shape, 1)
            else:
                Pbar[b] += _at_T(0.5 * bbar, z, d, ny, shape, 1) + _at_T(0.5 * bbar, _unit(a, d), d, ny, shape, 1)
    return np.stack([_fold(Pbar[a], a, d, ny) for a in range(d)])


def rhs_vjp(u, fbar, h, nu):
    return convection_vjp(u, fbar, h) + diffusion_vjp(fbar, h, nu)


def poisson_solve_vjp(pbar, h):
    """Transpose of the direct solve: the first block of [L e; e^T 0]^{-T} [pbar; 0]."""
    import scipy.sparse.linalg as spla

    A, m = _augmented(tuple(reversed(pbar.shape)), h)
    sol = spla.spsolve(A.T.tocsc(), np.concatenate([pbar.ravel(), [0.0]]))
    return sol[:m].reshape(pbar.shape)


def project_vjp(ubar_out, h):
    """P^T v = v - D^T L^{-T} G^T v on the unknowns (transposes of the three steps of P)."""
    v = ubar_out * dof_mask(tuple(reversed(ubar_out.shape[1:])))
    return v - divergence_vjp(poisson_solve_vjp(gradient_vjp(v, h), h), h)


# ----------------------------------------------------------------------------
# Time steps: the periodic schedules of the oracle with the channel's
# right-hand side and projection.
# ----------------------------------------------------------------------------

def _fns(h, nu, force=None):
    return dict(rhs_fn=lambda v: rhs(v, h, nu, force), project_fn=lambda v: project(v, h)[0])


def step_rk4(u0, h, nu, dt, force=None):
    return ins.step_rk4(u0, h, nu, dt, **_fns(h, nu, force))


def step_wray3(u0, h, nu, dt, force=None):
    return ins.step_wray3(u0, h, nu, dt, **_fns(h, nu, force))


# A constant force has no Jacobian: it enters the pullbacks only through the
# forward stages they linearise about.
def step_rk4_vjp(u0, u1bar, h, nu, dt, force=None):
    return ins.step_rk4_vjp(u0, u1bar, h, nu, dt, rhs_vjp_fn=lambda v, fb: rhs_vjp(v, fb, h, nu),
                            project_vjp_fn=lambda v: project_vjp(v, h), **_fns(h, nu, force))


def step_wray3_vjp(u0, u1bar, h, nu, dt, force=None):
    return ins.step_wray3_vjp(u0, u1bar, h, nu, dt, rhs_vjp_fn=lambda v, fb: rhs_vjp(v, fb, h, nu),
                              project_vjp_fn=lambda v: project_vjp(v, h), **_fns(h, nu, force))
