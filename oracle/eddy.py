"""Float64 oracle of the Smagorinsky eddy-viscosity closure on the uniform
periodic staggered grid (the appendix on eddy-viscosity models: general
framework and the Smagorinsky model), and its pullback.

TEST INFRASTRUCTURE ONLY (see the package docstring). Not used by the product path.

Discretisation, following the appendix on the staggered grid:
* velocity-gradient components delta_b u^a: the diagonal ones
  D_a[I] = (u^a[I] - u^a[I - e_a]) / h_a sit at the pressure point I; the
  off-diagonal ones G_ab[J] = (u^a[J + e_b] - u^a[J]) / h_b sit at the
  (a, b) edge J + e_a/2 + e_b/2;
* the velocity gradient A at pressure points: A_aa = D_a, A_ab = mean of G_ab
  over the four (a, b) edges around the cell (J = I, I - e_a, I - e_b,
  I - e_a - e_b); S = (A + A^T) / 2;
* eddy viscosity at pressure points nu_t = (C_s Delta)^2 sqrt(2 S_ab S_ab)
  (eq. smagorinsky, C_s = 0.17 proposed);
* strain rate at its own points: S_aa = D_a (pressure points),
  S_ab[J] = (G_ab[J] + G_ba[J]) / 2 (edges); nu_t at an edge is the mean of the
  four pressure points around it;
* tensor T_ab = 2 nu_t S_ab and the closure term on the a-faces
  M^a = sum_b delta_b T_ab: (T_aa[I + e_a] - T_aa[I]) / h_a for b = a and
  (T_ab[I] - T_ab[I - e_b]) / h_b for b != a.

Reading of the sign: the appendix writes the sub-grid stress as
m^a = -sum_b d_b (2 nu_t S_ab); the term that enters the momentum right-hand
side is M = -m = +sum_b d_b (2 nu_t S_ab), the choice for which nu_t >= 0
dissipates kinetic energy (pinned by the energy identity in the tests).
Delta is the filter width; for the uniform grid the geometric mean of the
spacings, (prod_a h_a)^(1/d), unless given.
"""
from __future__ import annotations

import numpy as np

from .ins import _next, _prev

C_SMAGORINSKY = 0.17


def filter_width(h):
    return float(np.prod(h)) ** (1.0 / len(h))


def _diag(u, h):
    d = u.shape[0]
    return [(u[a] - _prev(u[a], a, d)) / h[a] for a in range(d)]


def _edge_grad(u, h):
    """G[a][b] = delta_b u^a at the (a, b) edges (a != b)."""
    d = u.shape[0]
    G = [[None] * d for _ in range(d)]
    for a in range(d):
        for b in range(d):
            if a != b:
                G[a][b] = (_next(u[a], b, d) - u[a]) / h[b]
    return G


def _edges_to_centre(e, a, b, d):
    """Mean over the four (a, b) edges around each pressure point."""
    return 0.25 * (e + _prev(e, a, d) + _prev(e, b, d) + _prev(_prev(e, a, d), b, d))


def _centre_to_edge(c, a, b, d):
    """Mean over the four pressure points around each (a, b) edge."""
    return 0.25 * (c + _next(c, a, d) + _next(c, b, d) + _next(_next(c, a, d), b, d))


def centre_gradient(u, h):
    """Velocity gradient A[a][b] = delta_b u^a interpolated to the pressure points."""
    d = u.shape[0]
    D = _diag(u, h)
    G = _edge_grad(u, h)
    return [[D[a] if a == b else _edges_to_centre(G[a][b], a, b, d) for b in range(d)] for a in range(d)]


def eddy_viscosity(u, h, cs=C_SMAGORINSKY, delta=None):
    """nu_t = (C_s Delta)^2 sqrt(2 S:S) at the pressure points."""
    d = u.shape[0]
    delta = filter_width(h) if delta is None else delta
    A = centre_gradient(u, h)
    ss = np.zeros(u.shape[1:])
    for a in range(d):
        for b in range(d):
            s = 0.5 * (A[a][b] + A[b][a])
            ss = ss + s * s
    return (cs * delta) ** 2 * np.sqrt(2.0 * ss)


def smagorinsky(u, h, cs=C_SMAGORINSKY, delta=None):
    """Closure term M^a = sum_b delta_b (2 nu_t S_ab) on the a-faces."""
    d = u.shape[0]
    nu = eddy_viscosity(u, h, cs, delta)
    D = _diag(u, h)
    G = _edge_grad(u, h)
    M = np.zeros_like(u, dtype=np.float64)
    for a in range(d):
        taa = 2.0 * nu * D[a]
        M[a] += (_next(taa, a, d) - taa) / h[a]
        for b in range(d):
            if b == a:
                continue
            tab = 2.0 * _centre_to_edge(nu, a, b, d) * 0.5 * (G[a][b] + G[b][a])
            M[a] += (tab - _prev(tab, b, d)) / h[b]
    return M


def smagorinsky_vjp(u, mbar, h, cs=C_SMAGORINSKY, delta=None):
    """ubar = (dM/du)^T mbar, transposing every step of ``smagorinsky``.

    Where S = 0 the square root has no derivative; its pullback is taken as 0
    there (the one-sided derivatives of nu_t are then all >= 0 and the choice
    is a subgradient).
    """
    d = u.shape[0]
    delta = filter_width(h) if delta is None else delta
    c2 = (cs * delta) ** 2
    D = _diag(u, h)
    G = _edge_grad(u, h)
    A = centre_gradient(u, h)
    Sc = [[0.5 * (A[a][b] + A[b][a]) for b in range(d)] for a in range(d)]
    ss = sum(Sc[a][b] ** 2 for a in range(d) for b in range(d))
    root = np.sqrt(2.0 * ss)
    nu = c2 * root

    Dbar = [np.zeros_like(D[0]) for _ in range(d)]
    Gbar = [[np.zeros_like(D[0]) if a != b else None for b in range(d)] for a in range(d)]
    nubar = np.zeros_like(nu)
    for a in range(d):
        # M^a += (T_aa[I + e_a] - T_aa[I]) / h_a
        tbar = (_prev(mbar[a], a, d) - mbar[a]) / h[a]
        nubar += 2.0 * tbar * D[a]
        Dbar[a] += 2.0 * tbar * nu
        for b in range(d):
            if b == a:
                continue
            # M^a += (T_ab[J] - T_ab[J - e_b]) / h_b, T_ab = 2 nu_e S_e
            tbar = (mbar[a] - _next(mbar[a], b, d)) / h[b]
            nu_e = _centre_to_edge(nu, a, b, d)
            s_e = 0.5 * (G[a][b] + G[b][a])
            nue_bar = 2.0 * tbar * s_e
            se_bar = 2.0 * tbar * nu_e
            # transpose of the centre -> edge mean
            nubar += 0.25 * (nue_bar + _prev(nue_bar, a, d) + _prev(nue_bar, b, d) + _prev(_prev(nue_bar, a, d), b, d))
            Gbar[a][b] += 0.5 * se_bar
            Gbar[b][a] += 0.5 * se_bar
    # nu = c2 sqrt(2 ss): d nu / d Sc_ab = c2 * 2 Sc_ab / root
    with np.errstate(divide="ignore", invalid="ignore"):
        g = np.where(root > 0, c2 * 2.0 * nubar / root, 0.0)
    for a in range(d):
        for b in range(d):
            scbar = g * Sc[a][b]  # Sc symmetric: Abar_ab = (Scbar_ab + Scbar_ba) / 2 = Scbar_ab
            if a == b:
                Dbar[a] += scbar
            else:
                # transpose of the edge -> centre mean
                Gbar[a][b] += 0.25 * (scbar + _next(scbar, a, d) + _next(scbar, b, d) + _next(_next(scbar, a, d), b, d))
    ubar = np.zeros_like(u, dtype=np.float64)
    for a in range(d):
        ubar[a] += (Dbar[a] - _next(Dbar[a], a, d)) / h[a]
        for b in range(d):
            if b != a:
                ubar[a] += (_prev(Gbar[a][b], b, d) - Gbar[a][b]) / h[b]
    return ubar


def rhs_with_smagorinsky(u, h, nu, cs=C_SMAGORINSKY, delta=None):
    from . import ins

    return ins.rhs(u, h, nu) + smagorinsky(u, h, cs, delta)


def rhs_vjp_with_smagorinsky(u, fbar, h, nu, cs=C_SMAGORINSKY, delta=None):
    from . import ins

    return ins.rhs_vjp(u, fbar, h, nu) + smagorinsky_vjp(u, fbar, h, cs, delta)
