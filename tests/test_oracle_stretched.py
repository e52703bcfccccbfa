"""Pins of the channel oracle on a stretched y grid (Sec. 2.5 non-uniform grids,
eq. tanh-grid; App. B kernels with non-uniform widths), by routes other than
its array code:

* brute force: every operator cell by cell with pure-Python loops, metrics
  recomputed here from the face coordinates;
* the pullbacks App. B prints for the divergence, the pressure gradient and
  the diffusion, transcribed as loops, against the oracle's transposition
  (interior rows, where the printed formulas need no ghost rule);
* volume-weighted duality of D and G, symmetry and negativity of diffusion,
  symmetry of Omega_p L and of Omega_u P, P^2 = P;
* energy conservation of convection for solenoidal fields (and its failure
  with plain linear interpolation of both factors, which is why the reading
  averages the transported component with 1/2 and takes the mass-flux average
  of the transporting one);
* second-order convergence of the diffusion on tanh grids;
* CG equals the direct solve; a uniform face array reproduces the uniform
  oracle; dot-product and finite-difference tests of every pullback.
"""
import math

import numpy as np
import pytest

import oracle.walls as W
import synth as S

GRIDS = [(6, 7), (4, 6, 3)]


def _h(n, gamma=1.4):
    lo, hi = S.channel_box(n)
    h = list(S.spacing(n, lo, hi))
    h[1] = S.tanh_faces(n[1], lo[1], hi[1], gamma)
    return tuple(h)


def _dot(a, b):
    return float(np.sum(a * b))


def _metric(h, n):
    """Independent recomputation: cell widths, centre distances with mirrored ghosts."""
    yf = np.asarray(h[1])
    w = yf[1:] - yf[:-1]
    c = (yf[1:] + yf[:-1]) / 2
    dist = {j: c[j + 1] - c[j] for j in range(n[1] - 1)}
    dist[-1] = w[0]
    dist[n[1] - 1] = w[-1]
    return w, dist


def _U(u, n, a, I):
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
    if len(n) == 2:
        return [(i, j) for j in range(n[1]) for i in range(n[0])]
    return [(i, j, k) for k in range(n[2]) for j in range(n[1]) for i in range(n[0])]


def _put(arr, n, I, v):
    if len(n) == 3:
        arr[I[2], I[1], I[0]] = v
    else:
        arr[I[1], I[0]] = v


def _get(arr, n, I):
    J = list(I)
    J[0] %= n[0]
    if len(n) == 3:
        J[2] %= n[2]
        return arr[J[2], J[1], J[0]]
    return arr[J[1], J[0]]


def _e(b, d, s=1):
    e = [0] * d
    e[b] = s
    return tuple(e)


def _add(I, e):
    return tuple(x + y for x, y in zip(I, e))


def _brute(u, p, n, h, nu):
    """rhs, divergence and gradient cell by cell from the App. B formulas and the reading."""
    d = len(n)
    w, dist = _metric(h, n)
    hx = [float(h[a]) if a != 1 else None for a in range(d)]

    def cellw(a, j):
        return w[j] if a == 1 else hx[a]

    def volw(a, j):  # width along a of the a-velocity volume on row j
        return dist[j] if a == 1 else hx[a]

    F = np.zeros(u.shape)
    r = np.zeros(tuple(reversed(n)))
    g = np.zeros(u.shape)
    for I in _cells(n):
        j = I[1]
        _put(r, n, I, sum((_U(u, n, a, I) - _U(u, n, a, _add(I, _e(a, d, -1)))) / cellw(a, j) for a in range(d)))
        for a in range(d):
            if a == 1 and j == n[1] - 1:
                continue
            _put(g[a], n, I, (_get(p, n, _add(I, _e(a, d))) - _get(p, n, I)) / volw(a, j))
            diff = conv = 0.0
            for b in range(d):
                up, uc, um = _U(u, n, a, _add(I, _e(b, d))), _U(u, n, a, I), _U(u, n, a, _add(I, _e(b, d, -1)))
                if b != 1:
                    diff += (up - 2 * uc + um) / hx[b] ** 2
                elif a != 1:
                    diff += ((up - uc) / dist[j] - (uc - um) / dist[j - 1]) / w[j]
                else:
                    diff += ((up - uc) / w[j + 1] - (uc - um) / w[j]) / dist[j]

                def flux(K):
                    fa = 0.5 * (_U(u, n, a, K) + _U(u, n, a, _add(K, _e(b, d))))
                    if a == 1 and b != 1:
                        jj = K[1]
                        th = w[jj] / (w[jj] + w[jj + 1]) if 0 <= jj < n[1] - 1 else 0.5
                        fb = th * _U(u, n, b, K) + (1 - th) * _U(u, n, b, _add(K, _e(1, d)))
                    else:
                        fb = 0.5 * (_U(u, n, b, K) + _U(u, n, b, _add(K, _e(a, d))))
                    return fa * fb

                s = 1.0 / hx[b] if b != 1 else (1.0 / dist[j] if a == 1 else 1.0 / w[j])
                conv -= (flux(I) - flux(_add(I, _e(b, d, -1)))) * s
            _put(F[a], n, I, conv + nu * diff)
    return F, r, g


@pytest.mark.parametrize("n", GRIDS)
def test_operators_match_cellwise_brute_force(n):
    h = _h(n)
    u = S.channel_random(n, 1)
    p = S.random_scalar(n, 2)
    F, r, g = _brute(u, p, n, h, 0.3)
    np.testing.assert_allclose(W.rhs(u, h, 0.3), F, atol=1e-11)
    np.testing.assert_allclose(W.divergence(u, h), r, atol=1e-11)
    np.testing.assert_allclose(W.gradient(p, h), g, atol=1e-11)


@pytest.mark.parametrize("n", GRIDS)
def test_printed_linear_pullbacks_on_interior_rows(n):
    """App. B eq. div-kernel, presgrad-kernel and diff-pullback, as printed."""
    d = len(n)
    h = _h(n)
    w, dist = _metric(h, n)
    hx = [float(h[a]) if a != 1 else None for a in range(d)]
    rb = S.random_scalar(n, 3)
    gb = S.channel_random(n, 4)
    fb = S.channel_random(n, 5)
    nu = 0.7
    div_t, grad_t, diff_t = W.divergence_vjp(rb, h), W.gradient_vjp(gb, h), W.diffusion_vjp(fb, h, nu)

    def cw(a, j):
        return w[j] if a == 1 else hx[a]

    def vw(a, j):
        return dist[j] if a == 1 else hx[a]

    for I in _cells(n):
        j = I[1]
        if not 1 <= j <= n[1] - 3:
            continue
        for a in range(d):
            # divergence pullback: rbar of the cells left and right of face I over their widths
            ja = j + (a == 1)
            want = _get(rb, n, I) / cw(a, j) - _get(rb, n, _add(I, _e(a, d))) / cw(a, ja)
            assert abs(_get(div_t[a], n, I) - want) < 1e-10 * (1 + abs(want))
            # diffusion pullback, component a, summed over b
            tot = 0.0
            for b in range(d):
                fm, fc, fp = (_get(fb[a], n, _add(I, _e(b, d, -1))), _get(fb[a], n, I),
                              _get(fb[a], n, _add(I, _e(b, d))))
                if b != 1:
                    tot += (fm - 2 * fc + fp) / hx[b] ** 2
                elif a != 1:  # u^a at cell centres in y: |Delta_I| = w_j, |Delta_{I +- 1/2}| = d_j, d_{j-1}
                    tot += (fm / (w[j - 1] * dist[j - 1]) - fc / w[j] * (1 / dist[j] + 1 / dist[j - 1])
                            + fp / (w[j + 1] * dist[j]))
                else:  # u^y on faces: |Delta_I| = d_j, |Delta_{I +- 1/2}| = w_{j+1}, w_j
                    tot += (fm / (dist[j - 1] * w[j]) - fc / dist[j] * (1 / w[j + 1] + 1 / w[j])
                            + fp / (dist[j + 1] * w[j + 1]))
            assert abs(_get(diff_t[a], n, I) - nu * tot) < 1e-10 * (1 + abs(nu * tot))
        # gradient pullback: gbar of the faces left and right of cell I over their volume widths
        want = sum(_get(gb[a], n, _add(I, _e(a, d, -1))) / vw(a, j - (a == 1)) - _get(gb[a], n, I) / vw(a, j)
                   for a in range(d))
        assert abs(_get(grad_t, n, I) - want) < 1e-10 * (1 + abs(want))


@pytest.mark.parametrize("n", GRIDS)
def test_weighted_duality_symmetry_and_projection(n):
    h = _h(n)
    ou, op = W.volumes_u(h, n), W.volumes_p(h, n)
    u = S.channel_random(n, 6)
    v = S.channel_random(n, 7)
    p = S.random_scalar(n, 8)
    assert abs(_dot(op * W.divergence(u, h), p) + _dot(ou * u, W.gradient(p, h))) < 1e-12 * np.abs(u).sum()
    du, dv = W.diffusion(u, h, 1.0), W.diffusion(v, h, 1.0)
    assert abs(_dot(ou * du, v) - _dot(ou * u, dv)) < 1e-11 * abs(_dot(ou * du, v))
    assert _dot(ou * u, du) < 0
    L = W.laplace_matrix(n, h).toarray()
    S_ = op.ravel()[:, None] * L
    np.testing.assert_allclose(S_, S_.T, atol=1e-12 * np.abs(S_).max())
    assert not np.allclose(L, L.T)  # D G alone is not symmetric on a stretched grid
    Pu, Pv = W.project(u, h)[0], W.project(v, h)[0]
    assert abs(_dot(ou * Pu, v) - _dot(ou * u, Pv)) < 1e-11 * np.abs(u).sum()
    np.testing.assert_allclose(W.project(Pu, h)[0], Pu, atol=1e-11)
    assert np.abs(W.divergence(Pu, h)).max() < 1e-10


def _convection_variant(u, h, transported_linear):
    """Alternative readings of the stretched-y weights (not taken): the
    transporting component linearly interpolated between the two cells it
    spans, and the transported one linearly too (transported_linear) or with
    the weights 1/2 (the paper's words for the convection term)."""
    d = u.shape[0]
    ny = u.shape[1 + W._yaxis(d)]
    w, dd, th = W._metrics(h, ny)
    lin = np.concatenate([[0.5], w[1:] / (w[:-1] + w[1:]), [0.5]])  # weight of row j toward face j|j+1
    out = np.zeros(u.shape)
    for a in range(d):
        for b in range(d):
            Pa, Pb = W._pad(u, a), W._pad(u, b)
            z = [0] * d
            t = W._rowvec(lin, d, ny + 1)
            if transported_linear and b == 1 and a != 1:
                fa = t * W._at(Pa, z, d, ny, 1) + (1 - t) * W._at(Pa, W._unit(b, d), d, ny, 1)
            else:
                fa = 0.5 * (W._at(Pa, z, d, ny, 1) + W._at(Pa, W._unit(b, d), d, ny, 1))
            if a == 1 and b != 1:
                fb = t * W._at(Pb, z, d, ny, 1) + (1 - t) * W._at(Pb, W._unit(a, d), d, ny, 1)
            else:
                fb = 0.5 * (W._at(Pb, z, d, ny, 1) + W._at(Pb, W._unit(a, d), d, ny, 1))
            F = fa * fb
            out[a] -= (W._rows(F, 1, ny, d) - W._flux_at(F, W._unit(b, d), d, ny)) * W._conv_inv_width(h, a, b, d, ny)
    return out * W.dof_mask(tuple(reversed(u.shape[1:])))


@pytest.mark.parametrize("n", [(8, 10), (6, 9, 4)])
def test_energy_conservation_and_the_reading(n):
    """The reading taken (transported component 1/2, transporting component the
    mass-flux average) conserves energy to rounding; both linear readings, the
    literal one of the convection paragraph (1/2 transported, linear
    transporting) included, leave a relative residual of order 1e-3."""
    h = _h(n, gamma=2.0)
    ou = W.volumes_u(h, n)
    u = W.project(S.channel_random(n, 9), h)[0]
    c = W.convection(u, h)
    assert abs(_dot(ou * u, c)) < 1e-13 * np.abs(ou * u * c).sum()
    for transported_linear in (True, False):
        cl = _convection_variant(u, h, transported_linear)
        assert abs(_dot(ou * u, cl)) > 1e-4 * np.abs(ou * u * cl).sum(), transported_linear


def test_second_order_diffusion_on_tanh_grids():
    errs = []
    for ny in (16, 32, 64):
        n = (4, ny)
        h = _h(n, gamma=1.5)
        yc = 0.5 * (h[1][1:] + h[1][:-1])
        L = h[1][-1] - h[1][0]
        u = np.zeros((2, ny, 4))
        u[0] = np.sin(math.pi * (yc - h[1][0]) / L)[:, None]
        exact = -(math.pi / L) ** 2 * u[0]
        errs.append(np.abs(W.diffusion(u, h, 1.0)[0] - exact).max())
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


@pytest.mark.parametrize("n", [(8, 6), (6, 7, 4)])
def test_cg_and_direct_solve_and_uniform_limit(n):
    h = _h(n)
    r = S.random_scalar(n, 10)
    p = W.poisson_solve(r, h)
    op = W.volumes_p(h, n)
    rbar = np.sum(op * r) / np.sum(op)
    np.testing.assert_allclose(W.laplacian(p, h), r - rbar, atol=1e-10 * np.abs(r).max())
    assert abs(p.mean()) < 1e-13
    x, it, rel = W.cg_solve(r, h, rtol=1e-13)
    assert rel <= 1e-13 and 0 < it < 500
    np.testing.assert_allclose(x - x.mean(), p, atol=1e-10 * np.abs(p).max())
    # a uniform face array reproduces the uniform-spacing oracle
    lo, hi = S.channel_box(n)
    hu = list(S.spacing(n, lo, hi))
    hf = list(hu)
    hf[1] = np.linspace(lo[1], hi[1], n[1] + 1)
    u = S.channel_ic(n, 11)
    np.testing.assert_allclose(W.rhs(u, tuple(hf), 0.1), W.rhs(u, tuple(hu), 0.1), atol=1e-11)
    np.testing.assert_allclose(W.poisson_solve(r, tuple(hf)), W.poisson_solve(r, tuple(hu)), atol=1e-10)


@pytest.mark.parametrize("n", GRIDS)
def test_pullbacks_dot_product(n):
    h = _h(n)
    u = S.channel_random(n, 12)
    fbar = S.channel_random(n, 13)
    v = S.channel_random(n, 14)
    q = S.random_scalar(n, 15)
    p = S.random_scalar(n, 16)
    assert abs(_dot(W.divergence(v, h), q) - _dot(v, W.divergence_vjp(q, h))) < 1e-11 * np.abs(v).sum()
    assert abs(_dot(W.gradient(p, h), fbar) - _dot(p, W.gradient_vjp(fbar, h))) < 1e-11 * np.abs(fbar).sum()
    assert abs(_dot(W.poisson_solve(q, h), p) - _dot(q, W.poisson_solve_vjp(p, h))) < 1e-10 * np.abs(q).sum()
    assert abs(_dot(W.project(v, h)[0], fbar) - _dot(v, W.project_vjp(fbar, h))) < 1e-10 * np.abs(v).sum()
    g = W.rhs_vjp(u, fbar, h, 0.4)
    eps = 1e-3  # exact for the quadratic convection and linear diffusion
    fd = _dot(fbar, (W.rhs(u + eps * v, h, 0.4) - W.rhs(u - eps * v, h, 0.4)) / (2 * eps))
    assert abs(fd - _dot(g, v)) < 1e-10 * np.abs(g * v).sum()


@pytest.mark.parametrize("scheme", ["rk4", "wray3"])
def test_step_pullbacks_by_finite_differences(scheme):
    n = (4, 6, 3)
    h = _h(n)
    nu, dt = 0.05, 1e-2
    step = W.step_rk4 if scheme == "rk4" else W.step_wray3
    vjp = W.step_rk4_vjp if scheme == "rk4" else W.step_wray3_vjp
    u0 = S.channel_ic(n, 20)
    ubar = S.channel_random(n, 21)
    g = vjp(u0, ubar, h, nu, dt)
    u1 = step(u0, h, nu, dt)
    assert np.abs(W.divergence(u1, h)).max() < 1e-10
    for seed in (22, 23):
        v = S.channel_random(n, seed)
        eps = 1e-5
        fd = _dot(ubar, (step(u0 + eps * v, h, nu, dt) - step(u0 - eps * v, h, nu, dt)) / (2 * eps))
        assert abs(fd - _dot(g, v)) < 1e-8 * np.abs(g * v).sum()


def test_tanh_gamma_gives_the_requested_first_cell():
    for ny, length, w0 in [(256, 2.0, 0.49 / 180), (64, 2.0, 0.01), (9, 1.0, 0.05)]:
        g = S.tanh_gamma(ny, length, w0)
        w = np.diff(S.tanh_faces(ny, 0.0, length, g))
        assert abs(w[0] - w0) < 1e-12 * length and abs(w[-1] - w0) < 1e-12 * length
        assert np.isclose(w.min(), w0, rtol=1e-12, atol=0) and np.isclose(w.sum(), length)
    with pytest.raises(ValueError):
        S.tanh_gamma(16, 2.0, 0.2)
