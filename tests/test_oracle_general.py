"""Pins of the stretched-grid oracle (oracle/stretched.py): grids stretched
along any direction (Sec. 2.5 non-uniform grids, eq. tanh-grid; App. B
kernels with non-uniform widths and eq. interp-weights), periodic in every
direction or with no-slip walls in y, by routes other than its sparse
assembly:

* two independently written oracles: with uniform faces it reproduces the
  uniform periodic oracle (oracle/ins.py: rolled arrays, FFT solve), with a
  stretched y between walls the channel oracle (oracle/walls.py: padded
  arrays, its own transpositions), operators, steps and pullbacks alike;
* brute force: every operator at every cell with pure-Python loops, metrics
  recomputed from the face coordinates;
* what the discretisation guarantees (App. A; Sec. 2.3): volume-weighted
  duality of D and G, symmetric negative diffusion, symmetric Omega_p L and
  Omega_u P, P^2 = P, D P u = 0, and energy conservation of convection for
  solenoidal fields on grids stretched in every direction; the alternative
  reading with weights 1/2 for both factors breaks the last one;
* the paper's convergence study (Sec. 7, Taylor-Green on a tanh grid): second
  order in N, with larger errors than on the uniform grid;
* CG equals the direct solve; central differences of every pullback.
Planted mistakes (transposed mass-flux weight, centre distance replaced by the
cell width in the gradient, wrong wrap distance, swapped diffusion widths)
each fail at least one pin.
"""
import math

import numpy as np
import pytest

import oracle as O
import oracle.walls as W
import synth as S
from oracle.stretched import StretchedGrid


def _tanh(n, gamma, lo=0.0, hi=2 * math.pi):
    return S.tanh_faces(n, lo, hi, gamma)


def _uniform(n, lo=0.0, hi=2 * math.pi):
    return lo + np.arange(n + 1) * ((hi - lo) / n)


def _geometric(n, s, lo=0.0, hi=2 * math.pi):
    """The geometric stretching of Sec. 2.5: x_i = a + (b - a)(1 - s^i)/(1 - s^N),
    clustered at one end (asymmetric: the periodic wrap joins the widest and
    the narrowest cell)."""
    i = np.arange(n + 1)
    return lo + (hi - lo) * (1.0 - s ** i) / (1.0 - s ** n)


def _stretched(n, ywalls=False):
    """x geometric, y and z tanh."""
    lo, hi = S.channel_box(n) if ywalls else ([0.0] * 3, [2 * math.pi] * 3)
    gam = [None, 1.2, 0.9]
    return [_geometric(n[0], 1.15, lo[0], hi[0])] + [_tanh(n[a], gam[a], lo[a], hi[a]) for a in range(1, len(n))]


def _field(g, seed):
    return S.channel_random(g.n, seed) if g.ywalls else S.random_field(g.n, seed)


def _dot(a, b):
    return float(np.sum(a * b))


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


# ----------------------------------------------------------------------------
# Two other oracles
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("n", [(8, 6), (6, 5, 4)])
def test_uniform_faces_reproduce_the_periodic_oracle(n):
    h = S.spacing(n)
    g = StretchedGrid([_uniform(m) for m in n])
    u, fb = S.random_field(n, 1), S.random_field(n, 2)
    nu, dt = 0.03, 0.01
    pu, p = g.project(u)
    pref, pref_p = O.project(u, h)
    assert _rel(pu, pref) < 1e-13
    assert _rel(g.gradient(p), O.gradient(pref_p, h)) < 1e-13
    assert _rel(g.divergence(u), O.divergence(u, h)) < 1e-13
    assert _rel(g.rhs(u, nu), O.rhs(u, h, nu)) < 1e-13
    assert _rel(g.rhs_vjp(u, fb, nu), O.rhs_vjp(u, fb, h, nu)) < 1e-13
    assert _rel(g.step_rk4(pu, nu, dt), O.step_rk4(pu, h, nu, dt)) < 1e-13
    assert _rel(g.step_rk4_vjp(pu, fb, nu, dt), O.step_rk4_vjp(pu, fb, h, nu, dt)) < 1e-13
    assert _rel(g.step_wray3(pu, nu, dt), O.step_wray3(pu, h, nu, dt)) < 1e-13
    assert _rel(g.step_wray3_vjp(pu, fb, nu, dt), O.step_wray3_vjp(pu, fb, h, nu, dt)) < 1e-13


@pytest.mark.parametrize("n", [(8, 7), (6, 9, 4)])
def test_stretched_y_walls_reproduce_the_channel_oracle(n):
    lo, hi = S.channel_box(n)
    yf = _tanh(n[1], 1.4, lo[1], hi[1])
    faces = [_uniform(n[a], lo[a], hi[a]) if a != 1 else yf for a in range(len(n))]
    h = list(S.spacing(n, lo, hi))
    h[1] = yf
    h = tuple(h)
    g = StretchedGrid(faces, ywalls=True)
    u, fb = S.channel_random(n, 1), S.channel_random(n, 2)
    nu, dt = 0.03, 0.01
    assert _rel(g.rhs(u, nu), W.rhs(u, h, nu)) < 1e-12
    assert _rel(g.divergence(u), W.divergence(u, h)) < 1e-12
    assert _rel(g.project(u)[0], W.project(u, h)[0]) < 1e-12
    assert _rel(g.rhs_vjp(u, fb, nu), W.rhs_vjp(u, fb, h, nu)) < 1e-12
    assert _rel(g.project_vjp(fb), W.project_vjp(fb, h)) < 1e-12
    assert _rel(g.step_rk4(u, nu, dt), W.step_rk4(u, h, nu, dt)) < 1e-12
    assert _rel(g.step_rk4_vjp(u, fb, nu, dt), W.step_rk4_vjp(u, fb, h, nu, dt)) < 1e-12
    assert _rel(g.volumes_u(), W.volumes_u(h, n)) < 1e-15
    assert _rel(g.volumes_p(), W.volumes_p(h, n)) < 1e-15


# ----------------------------------------------------------------------------
# Brute force
# ----------------------------------------------------------------------------

def _loops(faces, u, nu):
    """Every operator of App. B at every cell of a periodic grid, in loops."""
    d = len(faces)
    n = [len(f) - 1 for f in faces]
    w = [[faces[a][i + 1] - faces[a][i] for i in range(n[a])] for a in range(d)]
    c = [[0.5 * (faces[a][i] + faces[a][i + 1]) for i in range(n[a])] for a in range(d)]
    L = [faces[a][-1] - faces[a][0] for a in range(d)]

    def W_(a, i):
        return w[a][i % n[a]]

    def Dd(a, i):  # centre distance across face i (right face of cell i), wrap by the period
        i0 = i % n[a]
        nxt = c[a][(i0 + 1) % n[a]] + (L[a] if i0 + 1 == n[a] else 0.0)
        return nxt - c[a][i0]

    def Th(a, i):
        return W_(a, i) / (W_(a, i) + W_(a, i + 1))

    def U(a, I):
        idx = tuple((I[b] % n[b]) for b in reversed(range(d)))
        return u[a][idx]

    def E(a, s=1):
        return tuple(s if b == a else 0 for b in range(d))

    def add(I, e):
        return tuple(I[b] + e[b] for b in range(d))

    cells = [tuple(reversed(t)) for t in np.ndindex(*reversed(n))]
    div = np.zeros(tuple(reversed(n)))
    F = np.zeros(u.shape)
    for I in cells:
        pos = tuple(reversed(I))
        div[pos] = sum((U(a, I) - U(a, add(I, E(a, -1)))) / W_(a, I[a]) for a in range(d))
        for a in range(d):
            diff = 0.0
            conv = 0.0
            for b in range(d):
                up, uc, um = U(a, add(I, E(b))), U(a, I), U(a, add(I, E(b, -1)))
                if b == a:
                    diff += ((up - uc) / W_(a, I[a] + 1) - (uc - um) / W_(a, I[a])) / Dd(a, I[a])
                    width = Dd(a, I[a])
                else:
                    diff += ((up - uc) / Dd(b, I[b]) - (uc - um) / Dd(b, I[b] - 1)) / W_(b, I[b])
                    width = W_(b, I[b])

                def flux(K):
                    A = 0.5 * (U(a, K) + U(a, add(K, E(b))))
                    t = 0.5 if a == b else Th(a, K[a])
                    B = t * U(b, K) + (1 - t) * U(b, add(K, E(a)))
                    return A * B

                conv -= (flux(I) - flux(add(I, E(b, -1)))) / width
            F[(a,) + pos] = conv + nu * diff
    return div, F


@pytest.mark.parametrize("n", [(5, 4), (4, 3, 3)])
def test_brute_force_cell_loops(n):
    faces = _stretched(n)
    g = StretchedGrid(faces)
    u = S.random_field(n, 4)
    div, F = _loops(faces, u, 0.07)
    assert _rel(g.divergence(u), div) < 1e-13
    assert _rel(g.rhs(u, 0.07), F) < 1e-13
    p = np.random.default_rng(5).standard_normal(g.shape)
    gp = g.gradient(p)
    for a in range(len(n)):
        f = faces[a]
        w = np.diff(f)
        dist = np.append(0.5 * (w[:-1] + w[1:]), 0.5 * (w[-1] + w[0]))
        sh = [1] * len(n)
        sh[len(n) - 1 - a] = n[a]
        ref = (np.roll(p, -1, axis=len(n) - 1 - a) - p) / dist.reshape(sh)
        assert _rel(gp[a], ref) < 1e-14


# ----------------------------------------------------------------------------
# What the discretisation guarantees
# ----------------------------------------------------------------------------

CASES = [((10, 8), False), ((8, 9, 6), False), ((10, 8), True), ((8, 9, 6), True)]


@pytest.mark.parametrize("n,ywalls", CASES)
def test_duality_symmetry_projection(n, ywalls):
    g = StretchedGrid(_stretched(n, ywalls), ywalls)
    rng = np.random.default_rng(6)
    u, v = _field(g, 1), _field(g, 2)
    p, q = rng.standard_normal(g.shape), rng.standard_normal(g.shape)
    om_p, om_u = g.volumes_p(), g.volumes_u()
    scale = math.sqrt(_dot(om_p, om_p))
    # sum Omega_p (D u) p = -sum Omega_u u . G p
    a1, a2 = _dot(om_p * g.divergence(u), p), -_dot(om_u * u, g.gradient(p))
    assert abs(a1 - a2) < 1e-12 * (abs(a1) + scale)
    # diffusion symmetric and non-positive in the Omega_u inner product
    kuv, kvu = _dot(om_u * g.diffusion(u, 1.0), v), _dot(om_u * g.diffusion(v, 1.0), u)
    assert abs(kuv - kvu) < 1e-12 * abs(kuv)
    assert _dot(om_u * g.diffusion(u, 1.0), u) < 0
    # Omega_p L symmetric
    l1, l2 = _dot(om_p * g.laplacian(p), q), _dot(om_p * g.laplacian(q), p)
    assert abs(l1 - l2) < 1e-12 * abs(l1)
    # projection: P^2 = P, D P u = 0, Omega_u P symmetric
    pu = g.project(u)[0]
    assert _rel(g.project(pu)[0], pu) < 1e-12
    assert np.abs(g.divergence(pu)).max() < 1e-12 * np.abs(g.divergence(u)).max()
    pv = g.project(v)[0]
    s1, s2 = _dot(om_u * pu, v), _dot(om_u * pv, u)
    assert abs(s1 - s2) < 1e-12 * abs(s1)
    # the solve's residual: D G p = r - mean_w(r) with mean(p) = 0
    r = rng.standard_normal(g.shape)
    ps = g.poisson_solve(r)
    rw = _dot(om_p, r) / _dot(om_p, np.ones_like(r))
    assert _rel(g.laplacian(ps), r - rw) < 1e-10
    assert abs(ps.mean()) < 1e-12 * np.abs(ps).max()


def _energy(g, u):
    pu = g.project(u)[0]
    c = g.volumes_u() * pu * g.convection(pu)
    return abs(c.sum()) / np.abs(c).sum()


@pytest.mark.parametrize("n,ywalls", CASES)
def test_convection_conserves_energy_for_solenoidal_fields(n, ywalls):
    g = StretchedGrid(_stretched(n, ywalls), ywalls)
    assert _energy(g, _field(g, 3)) < 1e-14


class _HalfWeights(StretchedGrid):
    """The rejected reading: the transporting factor averaged with 1/2 too."""

    def theta(self, a, i):
        return np.full(np.shape(i), 0.5)


def test_half_weights_break_energy_conservation_along_x_and_z():
    n = (10, 8, 6)
    faces = [_tanh(10, 2.0), _uniform(8), _tanh(6, 2.0)]
    assert _energy(StretchedGrid(faces), S.random_field(n, 3)) < 1e-14
    assert _energy(_HalfWeights(faces), S.random_field(n, 3)) > 1e-4


# ----------------------------------------------------------------------------
# Convergence study of Sec. 7: 2D Taylor-Green vortex on a tanh grid
# ----------------------------------------------------------------------------

def _tg(g, nu, t):
    fx, fy = g.faces
    cx, cy = 0.5 * (fx[:-1] + fx[1:]), 0.5 * (fy[:-1] + fy[1:])
    x1, y1 = np.meshgrid(fx[1:], cy)
    x2, y2 = np.meshgrid(cx, fy[1:])
    e = math.exp(-2 * nu * t)
    return np.stack([np.sin(x1) * np.cos(y1) * e, -np.cos(x2) * np.sin(y2) * e])


def _tg_error(grid_cls, faces_of, N, nu=0.01, dt=0.02, T=1.0):
    f = faces_of(N)
    g = grid_cls([f, f])
    u = g.project(_tg(g, nu, 0.0))[0]
    for _ in range(int(round(T / dt))):
        u = g.step_rk4(u, nu, dt)
    ex = _tg(g, nu, T)
    om = g.volumes_u()
    return math.sqrt(_dot(om, (u - ex) ** 2) / _dot(om, ex ** 2))


def _orders(grid_cls, faces_of):
    e = [_tg_error(grid_cls, faces_of, N) for N in (16, 32, 64)]
    return e, [math.log2(e[i] / e[i + 1]) for i in range(2)]


def test_taylor_green_second_order_on_tanh_grid():
    eu, ou = _orders(StretchedGrid, lambda N: _uniform(N))
    et, ot = _orders(StretchedGrid, lambda N: _tanh(N, 1.5))
    assert min(ou) > 1.95 and min(ot) > 1.9, (ou, ot)
    assert all(b > 10 * a for a, b in zip(eu, et))  # larger errors at a given N (Sec. 7)


# ----------------------------------------------------------------------------
# Solvers and pullbacks
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("n,ywalls", CASES)
def test_cg_equals_direct_solve(n, ywalls):
    g = StretchedGrid(_stretched(n, ywalls), ywalls)
    r = np.random.default_rng(7).standard_normal(g.shape)
    x, it, rel = g.cg_solve(r, rtol=1e-13)
    assert rel <= 1e-13 and it > 0
    assert _rel(x, g.poisson_solve(r)) < 1e-9


@pytest.mark.parametrize("n,ywalls", CASES)
def test_pullbacks_by_central_differences(n, ywalls):
    g = StretchedGrid(_stretched(n, ywalls), ywalls)
    u, v, wb = _field(g, 8), _field(g, 9), _field(g, 10)
    u = g.project(u)[0]
    nu, dt, eps = 0.05, 0.02, 1e-6
    m = g.dof_mask()
    v = v * m
    # the right-hand side is quadratic: central differences are exact up to rounding
    jv = (g.rhs(u + eps * v, nu) - g.rhs(u - eps * v, nu)) / (2 * eps)
    assert abs(_dot(jv, wb) - _dot(v, g.rhs_vjp(u, wb, nu))) < 1e-8 * np.abs(jv).max() * np.abs(wb).sum()
    for fwd, vjp in ((g.step_rk4, g.step_rk4_vjp), (g.step_wray3, g.step_wray3_vjp)):
        jv = (fwd(u + eps * v, nu, dt) - fwd(u - eps * v, nu, dt)) / (2 * eps)
        lhs, rhs = _dot(jv, wb), _dot(v, vjp(u, wb, nu, dt))
        assert abs(lhs - rhs) < 1e-7 * abs(lhs), (lhs, rhs)
    # the linear maps: dot-product tests against the forward operators
    r = np.random.default_rng(11).standard_normal(g.shape)
    assert abs(_dot(g.divergence(v), r) - _dot(v, g.divergence_vjp(r))) < 1e-10 * np.abs(r).sum()
    assert abs(_dot(g.gradient(r), wb) - _dot(r, g.gradient_vjp(wb))) < 1e-10 * np.abs(wb).sum()
    q = np.random.default_rng(12).standard_normal(g.shape)
    assert abs(_dot(g.poisson_solve(r), q) - _dot(r, g.poisson_solve_vjp(q))) < 1e-10 * np.abs(q).sum()
    assert abs(_dot(g.project(v)[0], wb) - _dot(v, g.project_vjp(wb))) < 1e-10 * np.abs(wb).sum()


# ----------------------------------------------------------------------------
# Planted mistakes fail the pins
# ----------------------------------------------------------------------------

class _TransposedTheta(StretchedGrid):
    def theta(self, a, i):
        return 1.0 - super().theta(a, i)


class _GradByWidth(StretchedGrid):
    def dist(self, a, i):  # the gradient's centre distance replaced by the cell width
        return self.width(a, i)


class _WrapDistance(StretchedGrid):
    def dist(self, a, i):  # the periodic wrap face given the last cell's width
        out = super().dist(a, i)
        n = self.n[a]
        return np.where(np.mod(np.asarray(i), n) == n - 1, self.width(a, n - 1), out)


class _SwappedDiffusion(StretchedGrid):
    def width(self, a, i):  # neighbour-row index off by one (widths of the wrong cell)
        return super().width(a, np.asarray(i) + 1)


def _pins_hold(cls):
    n = (10, 8)
    faces = _stretched(n)
    g = cls(faces)
    ok_energy = _energy(g, S.random_field(n, 3)) < 1e-14
    u, p = S.random_field(n, 1), np.random.default_rng(6).standard_normal(g.shape)
    a1, a2 = _dot(g.volumes_p() * g.divergence(u), p), -_dot(g.volumes_u() * u, g.gradient(p))
    ok_dual = abs(a1 - a2) < 1e-12 * (abs(a1) + 1.0)
    _, ot = _orders(cls, lambda N: _tanh(N, 1.5))
    ok_order = min(ot) > 1.9
    ref = StretchedGrid(faces)
    ok_brute = _rel(g.rhs(u, 0.07), _loops(faces, u, 0.07)[1]) < 1e-13 and \
        _rel(ref.rhs(u, 0.07), _loops(faces, u, 0.07)[1]) < 1e-13
    return ok_energy and ok_dual and ok_order and ok_brute


@pytest.mark.parametrize("cls", [_TransposedTheta, _GradByWidth, _WrapDistance, _SwappedDiffusion])
def test_planted_mistakes_fail(cls):
    assert not _pins_hold(cls)


def test_the_unplanted_oracle_passes_the_same_checks():
    assert _pins_hold(StretchedGrid)
