"""Pins of the channel oracle (no-slip walls at both y ends; Sec. 2.1 boundary
conditions through ghost volumes, Sec. 2.6.1 direct and iterative pressure
solvers), by routes other than its own array code:

* brute force: every operator re-evaluated cell by cell with pure-Python loops
  and the ghost rule written as an index function, on tiny grids;
* the matrix of L assembled column by column from D(G(e_k)) equals the
  stencil matrix the direct solver factorises;
* a textbook route for the Neumann-periodic Poisson problem: DCT-II along y,
  DFT along x (and z), division by the eigenvalues;
* CG (the iterative solver) converges to the direct solution;
* closed form: a sine shear between the walls is an exact discrete solution
  (eigenvector of the diffusion, no convection, solenoidal), so one RK4 or
  Wray3 step multiplies it by the stability polynomial;
* duality D^T = -G, symmetry of diffusion and of P, P^2 = P, energy
  conservation of convection for solenoidal fields;
* every pullback by the dot-product test (central differences are exact for
  the quadratic convection) and the step pullbacks by finite differences.
"""
import math

import numpy as np
import pytest

import oracle.walls as W
import synth as S

GRIDS = [(6, 5), (4, 5, 3)]


def _dot(a, b):
    return float(np.sum(a * b))


def _h(n):
    lo, hi = S.channel_box(n)
    return S.spacing(n, lo, hi)


def _mask(n):
    return W.dof_mask(n)


# ---------------------------------------------------------------- brute force
def _U(u, n, a, I):
    """u^a at integer index I = (i, j[, k]) with the wall rules as an index function."""
    d = len(n)
    i, j = I[0] % n[0], I[1]
    k = I[2] % n[2] if d == 3 else None
    ny = n[1]

    def get(jj):
        return u[a][k, jj, i] if d == 3 else u[a][jj, i]

    if a == 1:
        return 0.0 if (j < 0 or j >= ny - 1) else get(j)
    if j == -1:
        return -get(0)
    if j == ny:
        return -get(ny - 1)
    return get(j)


def _cells(n):
    d = len(n)
    if d == 2:
        return [(i, j) for j in range(n[1]) for i in range(n[0])]
    return [(i, j, k) for k in range(n[2]) for j in range(n[1]) for i in range(n[0])]


def _put(arr, n, I, v):
    if len(n) == 3:
        arr[I[2], I[1], I[0]] = v
    else:
        arr[I[1], I[0]] = v


def _e(b, d, s=1):
    e = [0] * d
    e[b] = s
    return e


def _add(I, e):
    return tuple(x + y for x, y in zip(I, e))


def _brute_rhs(u, n, h, nu):
    d = len(n)
    out = np.zeros(u.shape)
    for a in range(d):
        for I in _cells(n):
            if a == 1 and I[1] == n[1] - 1:
                continue  # wall face: no equation
            diff = conv = 0.0
            for b in range(d):
                eb, ea = _e(b, d), _e(a, d)
                diff += (_U(u, n, a, _add(I, eb)) - 2 * _U(u, n, a, I) + _U(u, n, a, _add(I, _e(b, d, -1)))) / h[b] ** 2

                def F(K):
                    return 0.25 * (_U(u, n, a, K) + _U(u, n, a, _add(K, eb))) * (_U(u, n, b, K) + _U(u, n, b, _add(K, ea)))

                conv -= (F(I) - F(_add(I, _e(b, d, -1)))) / h[b]
            _put(out[a], n, I, conv + nu * diff)
    return out


def _brute_div(u, n, h):
    d = len(n)
    r = np.zeros(tuple(reversed(n)))
    for I in _cells(n):
        _put(r, n, I, sum((_U(u, n, a, I) - _U(u, n, a, _add(I, _e(a, d, -1)))) / h[a] for a in range(d)))
    return r


def _brute_grad(p, n, h):
    d = len(n)
    g = np.zeros((d,) + tuple(reversed(n)))

    def P(I):
        J = list(I)
        J[0] %= n[0]
        if d == 3:
            J[2] %= n[2]
        return p[J[2], J[1], J[0]] if d == 3 else p[J[1], J[0]]

    for a in range(d):
        for I in _cells(n):
            if a == 1 and I[1] == n[1] - 1:
                continue
            _put(g[a], n, I, (P(_add(I, _e(a, d))) - P(I)) / h[a])
    return g


@pytest.mark.parametrize("n", GRIDS)
def test_operators_match_cellwise_brute_force(n):
    h = _h(n)
    u = S.channel_random(n, 1)
    p = S.random_scalar(n, 2)
    nu = 0.3
    np.testing.assert_allclose(W.rhs(u, h, nu), _brute_rhs(u, n, h, nu), atol=1e-12)
    np.testing.assert_allclose(W.divergence(u, h), _brute_div(u, n, h), atol=1e-12)
    np.testing.assert_allclose(W.gradient(p, h), _brute_grad(p, n, h), atol=1e-12)


# ------------------------------------------------------------------ Poisson
@pytest.mark.parametrize("n", GRIDS)
def test_laplace_matrix_columns_are_the_operator(n):
    h = _h(n)
    shape = tuple(reversed(n))
    m = int(np.prod(shape))
    L = W.laplace_matrix(n, h).toarray()
    for k in range(m):
        e = np.zeros(m)
        e[k] = 1.0
        np.testing.assert_allclose(L[:, k], W.laplacian(e.reshape(shape), h).ravel(), atol=1e-12)
    assert np.allclose(L, L.T)
    assert np.abs(L.sum(axis=1)).max() < 1e-12  # constants are the null space


def _dct_solve(r, n, h):
    """Neumann in y (DCT-II diagonalises it), periodic DFT in x and z."""
    import scipy.fft as sf

    d = len(n)
    rm = r - r.mean()
    yax = d - 2
    c = sf.dct(rm, type=2, axis=yax, norm="ortho")
    per = [d - 1 - a for a in range(d) if a != 1]
    c = np.fft.fftn(c, axes=per)
    lam = np.zeros(tuple(reversed(n)))
    for a in range(d):
        k = np.arange(n[a])
        s = np.sin(np.pi * k / (2 * n[a])) if a == 1 else np.sin(np.pi * k / n[a])
        sh = [1] * d
        sh[d - 1 - a] = n[a]
        lam = lam - (4 * s * s / h[a] ** 2).reshape(sh)
    lam[(0,) * d] = 1.0
    c = c / lam
    c[(0,) * d] = 0.0
    c = np.real(np.fft.ifftn(c, axes=per))
    return sf.idct(c, type=2, axis=yax, norm="ortho")


@pytest.mark.parametrize("n", [(8, 6), (6, 7, 4), (12, 10, 6)])
def test_direct_solve_matches_dct_route_and_cg(n):
    h = _h(n)
    r = S.random_scalar(n, 3)
    p = W.poisson_solve(r, h)
    assert abs(p.mean()) < 1e-13
    np.testing.assert_allclose(W.laplacian(p, h), r - r.mean(), atol=1e-11 * np.abs(r).max())
    np.testing.assert_allclose(p, _dct_solve(r, n, h), atol=1e-12 * np.abs(p).max())
    x, it, rel = W.cg_solve(r, h, rtol=1e-13)
    assert rel <= 1e-13 and 0 < it < 500
    np.testing.assert_allclose(x - x.mean(), p, atol=1e-10 * np.abs(p).max())


def test_cg_fixed_iterations_and_zero_rhs():
    n = (8, 6)
    h = _h(n)
    r = S.random_scalar(n, 4)
    x1, it1, rel1 = W.cg_solve(r, h, rtol=0.0, maxiter=3)
    assert it1 == 3 and rel1 > 1e-6
    x0, it0, rel0 = W.cg_solve(np.full((6, 8), 2.5), h)  # constant r: consistent part is zero
    assert it0 == 0 and np.abs(x0).max() == 0.0


# --------------------------------------------------------------- invariants
@pytest.mark.parametrize("n", GRIDS)
def test_duality_symmetry_and_definiteness(n):
    h = _h(n)
    u = S.channel_random(n, 5)
    v = S.channel_random(n, 6)
    p = S.random_scalar(n, 7)
    assert abs(_dot(W.divergence(u, h), p) + _dot(u, W.gradient(p, h))) < 1e-12 * np.abs(u).sum()
    du, dv = W.diffusion(u, h, 1.0), W.diffusion(v, h, 1.0)
    assert abs(_dot(du, v) - _dot(u, dv)) < 1e-11 * abs(_dot(du, v))
    assert _dot(u, du) < 0


@pytest.mark.parametrize("n", [(8, 6), (6, 5, 4)])
def test_projection_and_energy(n):
    h = _h(n)
    u = S.channel_random(n, 8)
    v = S.channel_random(n, 9)
    Pu = W.project(u, h)[0]
    assert np.abs(W.divergence(Pu, h)).max() < 1e-11
    np.testing.assert_allclose(W.project(Pu, h)[0], Pu, atol=1e-12)
    Pv = W.project(v, h)[0]
    assert abs(_dot(Pu, v) - _dot(u, Pv)) < 1e-12 * np.abs(u).sum()
    p = S.random_scalar(n, 10)
    assert np.abs(W.project(W.gradient(p, h), h)[0]).max() < 1e-11
    assert np.abs(Pu[1].take([n[1] - 1], axis=len(n) - 2)).max() == 0.0
    # convection conserves energy for solenoidal fields, not for others
    c = W.convection(Pu, h)
    assert abs(_dot(Pu, c)) < 1e-13 * np.abs(Pu * c).sum()
    assert abs(_dot(u, W.convection(u, h))) > 1e-3 * np.abs(u * W.convection(u, h)).sum()


# ------------------------------------------------------------- closed forms
def _r4(z):
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


def _r3(z):
    return 1 + z + z * z / 2 + z ** 3 / 6


@pytest.mark.parametrize("n,comp", [((6, 16), 0), ((4, 12, 5), 0), ((4, 12, 5), 2)])
def test_sine_shear_is_an_exact_discrete_solution(n, comp):
    h = _h(n)
    nu, dt, m = 0.05, 2e-2, 2
    u0 = S.channel_shear(n, m=m, amplitude=1.3, component=comp)
    lam = -4 * math.sin(math.pi * m / (2 * n[1])) ** 2 / h[1] ** 2
    np.testing.assert_allclose(W.diffusion(u0, h, nu), nu * lam * u0, atol=1e-12)
    assert np.abs(W.convection(u0, h)).max() < 1e-13
    assert np.abs(W.divergence(u0, h)).max() < 1e-13
    u = u0
    for _ in range(4):
        u = W.step_rk4(u, h, nu, dt)
    np.testing.assert_allclose(u, _r4(nu * lam * dt) ** 4 * u0, atol=1e-13)
    u = u0
    for _ in range(4):
        u = W.step_wray3(u, h, nu, dt)
    np.testing.assert_allclose(u, _r3(nu * lam * dt) ** 4 * u0, atol=1e-13)


@pytest.mark.parametrize("n", [(8, 6), (6, 5, 4)])
def test_step_keeps_walls_and_dissipates(n):
    h = _h(n)
    u = S.channel_ic(n, 11)
    e0 = float(np.sum(u ** 2))
    u1 = W.step_rk4(u, h, 0.05, 1e-2)
    assert np.abs(W.divergence(u1, h)).max() < 1e-11
    assert np.abs(u1[1].take([n[1] - 1], axis=len(n) - 2)).max() == 0.0
    assert float(np.sum(u1 ** 2)) < e0


# ----------------------------------------------------------------- pullbacks
@pytest.mark.parametrize("n", GRIDS)
def test_linear_pullbacks_dot_product(n):
    h = _h(n)
    u = S.channel_random(n, 12)
    w = S.channel_random(n, 13)
    p = S.random_scalar(n, 14)
    q = S.random_scalar(n, 15)
    assert abs(_dot(W.divergence(u, h), q) - _dot(u, W.divergence_vjp(q, h))) < 1e-12 * np.abs(u).sum() * 10
    assert abs(_dot(W.gradient(p, h), w) - _dot(p, W.gradient_vjp(w, h))) < 1e-12 * np.abs(w).sum() * 10
    assert abs(_dot(W.diffusion(u, h, 0.7), w) - _dot(u, W.diffusion_vjp(w, h, 0.7))) < 1e-10
    Pw = W.project_vjp(w, h)
    assert abs(_dot(W.project(u, h)[0], w) - _dot(u, Pw)) < 1e-11 * np.abs(u).sum()
    # the pullbacks give nothing to the wall face (not an unknown)
    for g in (W.divergence_vjp(q, h), W.diffusion_vjp(w, h, 0.7), Pw):
        assert np.abs(g[1].take([n[1] - 1], axis=len(n) - 2)).max() == 0.0


@pytest.mark.parametrize("n", GRIDS)
def test_convection_and_rhs_pullback(n):
    h = _h(n)
    u = S.channel_random(n, 16)
    fbar = S.channel_random(n, 17)
    g = W.rhs_vjp(u, fbar, h, 0.4)
    for seed in (18, 19):
        v = S.channel_random(n, seed)
        eps = 1e-3  # exact for the quadratic convection and linear diffusion
        fd = _dot(fbar, (W.rhs(u + eps * v, h, 0.4) - W.rhs(u - eps * v, h, 0.4)) / (2 * eps))
        assert abs(fd - _dot(g, v)) < 1e-11 * np.abs(g * v).sum()
    assert np.abs(g[1].take([n[1] - 1], axis=len(n) - 2)).max() == 0.0


@pytest.mark.parametrize("n", [(6, 5), (4, 5, 3)])
@pytest.mark.parametrize("scheme", ["rk4", "wray3"])
def test_step_pullbacks_by_finite_differences(n, scheme):
    h = _h(n)
    nu, dt = 0.05, 2e-2
    step = W.step_rk4 if scheme == "rk4" else W.step_wray3
    vjp = W.step_rk4_vjp if scheme == "rk4" else W.step_wray3_vjp
    u0 = S.channel_ic(n, 20)
    ubar = S.channel_random(n, 21)
    g = vjp(u0, ubar, h, nu, dt)
    for seed in (22, 23):
        v = S.channel_random(n, seed)
        eps = 1e-5
        fd = _dot(ubar, (step(u0 + eps * v, h, nu, dt) - step(u0 - eps * v, h, nu, dt)) / (2 * eps))
        assert abs(fd - _dot(g, v)) < 1e-8 * np.abs(g * v).sum()
