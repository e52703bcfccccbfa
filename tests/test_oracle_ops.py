"""Pins of the float64 oracle's operators against what the paper and the mathematics fix.

Each test checks the oracle against something other than its own formula:
closed forms of the discrete operators on sampled trigonometric fields,
invariants stated in the paper (D and G negative transposes, Sec. 5.8 test
suite; skew-symmetric convection conserves energy, App. A), a textbook
Laplacian matrix, and brute-force loops of the printed convection kernel.
"""
import math

import numpy as np
import pytest

import oracle as O
import synth as S

GRIDS = [(8, 6), (5, 7), (4, 6, 5), (6, 4, 8)]


def _h(n, lengths=None):
    d = len(n)
    lengths = lengths or [2 * math.pi] * d
    return tuple(lengths[a] / n[a] for a in range(d))


def _dot(a, b):
    return float(np.sum(a * b))


@pytest.mark.parametrize("n", GRIDS)
def test_divergence_of_sine_face_field(n):
    """u = (sin x on x-faces, 0, ...): D u = (sin x_{i+1} - sin x_i)/h = 2 cos(x_{i+1/2}) sin(h/2) / h."""
    d = len(n)
    h = S.spacing(n)
    u = np.zeros((d,) + tuple(reversed(n)))
    x, *_ = S.face_coords(n, 0)
    u[0] = np.sin(x) * np.ones(tuple(reversed(n)))
    xc = (np.arange(n[0]) + 0.5) * h[0]
    expect = 2.0 * np.cos(xc) * math.sin(h[0] / 2) / h[0]
    r = O.divergence(u, h)
    np.testing.assert_allclose(r, np.broadcast_to(expect, r.shape), atol=1e-13)


def test_divergence_of_taylor_green_vanishes():
    for n in [(8, 8), (12, 12), (64, 64)]:
        h = S.spacing(n)
        assert np.abs(O.divergence(S.taylor_green_2d(n), h)).max() < 1e-13
    n = (8, 8, 4)
    assert np.abs(O.divergence(S.taylor_green_3d_extruded(n), S.spacing(n))).max() < 1e-13


@pytest.mark.parametrize("n", [(16, 12), (8, 10, 6)])
def test_divergence_of_turbulence_ic_vanishes(n):
    u = S.turbulence_ic(n, seed=3, k0=2)
    r = O.divergence(u, S.spacing(n))
    scale = np.abs(u).max() / min(S.spacing(n))
    assert np.abs(r).max() < 1e-13 * scale


@pytest.mark.parametrize("n", GRIDS)
def test_gradient_is_negative_transpose_of_divergence(n):
    """<D u, p> = -<u, G p> (Sec. 2.3 duality; Sec. 5.8 physical verification test)."""
    h = _h(n, [1.0, 2.5, 0.7][: len(n)])
    u = S.random_field(n, 11)
    p = S.random_scalar(n, 12)
    lhs = _dot(O.divergence(u, h), p)
    rhs = -_dot(u, O.gradient(p, h))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.abs(u).sum())


def test_gradient_of_cosine():
    """p = cos(x) at centres: (G p)^x = (cos x_{i+3/2} - cos x_{i+1/2})/h = -2 sin(x_{i+1}) sin(h/2)/h."""
    n = (12, 5, 3)
    h = S.spacing(n)
    xc = (np.arange(n[0]) + 0.5) * h[0]
    p = np.broadcast_to(np.cos(xc), tuple(reversed(n))).copy()
    g = O.gradient(p, h)
    xf = (np.arange(n[0]) + 1.0) * h[0]
    np.testing.assert_allclose(g[0], np.broadcast_to(-2 * np.sin(xf) * math.sin(h[0] / 2) / h[0], g[0].shape), atol=1e-13)
    assert np.abs(g[1]).max() < 1e-13 and np.abs(g[2]).max() < 1e-13


@pytest.mark.parametrize("n,k", [((8, 6), (1, 2)), ((10, 8), (3, 1)), ((6, 8, 10), (1, 2, 3)), ((5, 7, 9), (2, 0, 4))])
def test_diffusion_fourier_eigenvalue(n, k):
    """Fourier modes are eigenvectors of the discrete Laplacian: -sum_b 4 sin^2(k_b h_b / 2) / h_b^2."""
    d = len(n)
    lengths = [2 * math.pi * (1 + 0.3 * a) for a in range(d)]
    h = _h(n, lengths)
    nu = 0.37
    u = np.zeros((d,) + tuple(reversed(n)))
    for a in range(d):
        xs = S.face_coords(n, a, hi=lengths)
        phase = sum(2 * math.pi * k[b] / lengths[b] * xs[b] for b in range(d))
        u[a] = np.cos(phase + 0.3 * a) * np.ones(tuple(reversed(n)))
    lam = -sum(4 * math.sin(math.pi * k[b] / n[b]) ** 2 / h[b] ** 2 for b in range(d))
    np.testing.assert_allclose(O.diffusion(u, h, nu), nu * lam * u, atol=1e-12 * abs(lam))


@pytest.mark.parametrize("n", GRIDS)
def test_diffusion_symmetric(n):
    h = _h(n, [1.0, 2.0, 3.0][: len(n)])
    u, v = S.random_field(n, 1), S.random_field(n, 2)
    a = _dot(O.diffusion(u, h, 0.1), v)
    b = _dot(u, O.diffusion(v, h, 0.1))
    assert abs(a - b) < 1e-12 * abs(a)


@pytest.mark.parametrize("nn", [8, 16, 64, 250])
def test_convection_of_taylor_green_is_a_gradient(nn):
    """C(u_TG) = G q with q = cos^2(h/2) (cos 2x + cos 2y) / 4 at the cell centres (derived closed form).

    Hence the projection removes it and the discrete pressure of the TG vortex is q.
    """
    n = (nn, nn)
    h = S.spacing(n)
    u = S.taylor_green_2d(n)
    xc = (np.arange(nn) + 0.5) * h[0]
    q = math.cos(h[0] / 2) ** 2 * (np.cos(2 * xc)[None, :] + np.cos(2 * xc)[:, None]) / 4
    np.testing.assert_allclose(O.convection(u, h), O.gradient(q, h), atol=2e-14 * nn)
    p = O.poisson_solve(O.divergence(O.rhs(u, h, 0.01), h), h)
    np.testing.assert_allclose(p, q, atol=1e-13)


@pytest.mark.parametrize("n", [(8, 10), (6, 8, 4)])
def test_convection_of_shear_wave_vanishes(n):
    u = S.shear_wave(n, m=2, amplitude=1.7)
    assert np.abs(O.convection(u, S.spacing(n))).max() < 1e-13


@pytest.mark.parametrize("n", GRIDS)
def test_convection_energy_identity(n):
    """u.C(u) = -1/4 sum_a sum_I (u^a_I)^2 (Du_I + Du_{I+e_a}) for any u; zero when Du = 0 (App. A skew-symmetry)."""
    d = len(n)
    h = _h(n, [1.0, 1.7, 0.8][:d])
    u = S.random_field(n, 5)
    du = O.divergence(u, h)
    expect = 0.0
    for a in range(d):
        expect += -0.25 * float(np.sum(u[a] ** 2 * (du + np.roll(du, -1, axis=d - 1 - a))))
    got = _dot(u, O.convection(u, h))
    assert abs(got - expect) < 1e-12 * np.sum(np.abs(u) ** 3) / min(h)


@pytest.mark.parametrize("n", [(16, 16), (8, 12, 10)])
def test_convection_conserves_energy_for_solenoidal(n):
    h = S.spacing(n)
    u = S.turbulence_ic(n, seed=7, k0=2)
    c = O.convection(u, h)
    assert abs(_dot(u, c)) < 1e-12 * np.sqrt(_dot(u, u) * _dot(c, c))


def test_convection_quadratic_homogeneity():
    n = (6, 5, 4)
    h = S.spacing(n)
    u = S.random_field(n, 9)
    np.testing.assert_allclose(O.convection(-2.5 * u, h), 6.25 * O.convection(u, h), rtol=1e-13, atol=1e-12)


def _printed_conv_loops(u, h):
    """The App. B convection kernel written as loops with the interpolation weights of
    eq. interp-weights evaluated from the (uniform) volume widths, code indices."""
    d = u.shape[0]
    shape = u.shape[1:]
    n = tuple(reversed(shape))

    def width(b, i):
        return h[b]

    def A_plus(a, b, i):
        dl = 1 if a == b else 0
        return width(b, i - dl + 1) / (width(b, i - dl) + width(b, i - dl + 1))

    def A_minus(a, b, i):
        dl = 1 if a == b else 0
        return width(b, i + dl - 1) / (width(b, i + dl - 1) + width(b, i + dl))

    def at(f, idx):
        return f[tuple((idx[d - 1 - ax]) % n[d - 1 - ax] for ax in range(d))]

    out = np.zeros_like(u)
    for a in range(d):
        for flat in range(int(np.prod(shape))):
            arr_idx = np.unravel_index(flat, shape)
            I = [arr_idx[d - 1 - b] for b in range(d)]  # I[b] = index along direction b
            total = 0.0
            for b in range(d):
                e_b = [1 if c == b else 0 for c in range(d)]
                e_a = [1 if c == a else 0 for c in range(d)]
                dl = 1 if a == b else 0
                ip = [I[c] + e_b[c] for c in range(d)]
                im = [I[c] - e_b[c] for c in range(d)]
                ia = [I[c] + e_a[c] for c in range(d)]
                ima = [I[c] - e_b[c] + e_a[c] for c in range(d)]
                right = (A_plus(a, b, I[b]) * at(u[a], I) + A_minus(a, b, I[b] + 1) * at(u[a], ip)) * (
                    A_plus(b, a, I[a]) * at(u[b], I) + A_minus(b, a, I[a] + 1) * at(u[b], ia))
                left = (A_plus(a, b, I[b] - 1) * at(u[a], im) + A_minus(a, b, I[b]) * at(u[a], I)) * (
                    A_plus(b, a, I[a] - dl) * at(u[b], im) + A_minus(b, a, I[a] - dl + 1) * at(u[b], ima))
                total -= (right - left) / width(b, I[b])
            out[a][arr_idx] = total
    return out


@pytest.mark.parametrize("n", [(4, 5), (3, 4, 5)])
def test_convection_matches_printed_kernel_loops(n):
    h = _h(n, [1.0, 1.3, 0.9][: len(n)])
    u = S.random_field(n, 21)
    np.testing.assert_allclose(O.convection(u, h), _printed_conv_loops(u, h), rtol=1e-13, atol=1e-13)


def _textbook_laplacian(n, h):
    """Dense periodic 5/7-point Laplacian as a Kronecker sum of 1D circulant second differences."""
    import scipy.sparse as sp

    d = len(n)
    mats = []
    for a in range(d):
        m = n[a]
        t = sp.diags([np.ones(m - 1), -2 * np.ones(m), np.ones(m - 1)], [-1, 0, 1], format="lil")
        t[0, m - 1] += 1
        t[m - 1, 0] += 1
        mats.append(t.tocsr() / h[a] ** 2)
    # array axis order is (N_{d-1}, ..., N_0): kron with direction d-1 outermost
    total = None
    for a in range(d):
        parts = [sp.identity(n[b], format="csr") for b in reversed(range(d))]
        parts[d - 1 - a] = mats[a]
        k = parts[0]
        for p in parts[1:]:
            k = sp.kron(k, p, format="csr")
        total = k if total is None else total + k
    return total.toarray()


@pytest.mark.parametrize("n", [(8, 8), (6, 4), (4, 6, 5)])
def test_poisson_matches_dense_augmented_solve(n):
    """Sec. 2.6.1 direct solver: [L e; e^T 0][p; lambda] = [r; 0] vs the spectral solve."""
    d = len(n)
    h = _h(n, [1.0, 2.0, 1.5][:d])
    L = _textbook_laplacian(n, h)
    N = L.shape[0]
    # the oracle's D G equals the textbook Laplacian
    DG = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        DG[:, j] = O.divergence(O.gradient(e.reshape(tuple(reversed(n))), h), h).ravel()
    np.testing.assert_allclose(DG, L, atol=1e-12 * np.abs(L).max())
    r = S.random_scalar(n, 4)
    r -= r.mean()
    aug = np.zeros((N + 1, N + 1))
    aug[:N, :N] = L
    aug[:N, N] = 1.0
    aug[N, :N] = 1.0
    sol = np.linalg.solve(aug, np.concatenate([r.ravel(), [0.0]]))
    p = O.poisson_solve(r, h)
    np.testing.assert_allclose(p.ravel() - p.mean(), sol[:N], atol=1e-12 * np.abs(sol).max())


def test_poisson_zero_mode_kept():
    """Lhat(0) := 1 keeps the mean: mean(p) = mean(r)."""
    n = (6, 8)
    h = S.spacing(n)
    r = S.random_scalar(n, 2) + 3.0
    assert abs(O.poisson_solve(r, h).mean() - r.mean()) < 1e-12


@pytest.mark.parametrize("n", GRIDS)
def test_projection_properties(n):
    h = _h(n, [1.0, 1.4, 2.2][: len(n)])
    u = S.random_field(n, 8)
    pu, _ = O.project(u, h)
    assert np.abs(O.divergence(pu, h)).max() < 1e-11 * np.abs(u).max() / min(h)
    np.testing.assert_allclose(O.project(pu, h)[0], pu, atol=1e-12)
    v = S.random_field(n, 9)
    assert abs(_dot(pu, v) - _dot(u, O.project(v, h)[0])) < 1e-11 * np.abs(u).sum()
    q = S.random_scalar(n, 10)
    assert np.abs(O.project(O.gradient(q, h), h)[0]).max() < 1e-11 * np.abs(q).max() / min(h)


def _rk4_factor(z):
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


def test_taylor_green_2d_rk4_closed_form():
    """Taylor-Green vortex, 64^2, nu = 0.01, dt = 1e-3, 100 steps.

    The stage map keeps the TG shape (convection is a gradient, removed by the
    projection; the Laplacian scales it by lam = -2*4 sin^2(h/2)/h^2), so
    u_n = R(z)^n u_TG with R the RK4 stability polynomial, z = nu lam dt.
    Against the analytic exp(-2 nu t) the difference is the O(h^2) error.
    """
    nn, nu, dt, steps = 64, 0.01, 1e-3, 100
    n = (nn, nn)
    h = S.spacing(n)
    u0 = S.taylor_green_2d(n)
    u = u0.copy()
    for _ in range(steps):
        u = O.step_rk4(u, h, nu, dt)
    lam = -2 * 4 * math.sin(h[0] / 2) ** 2 / h[0] ** 2
    exact_discrete = _rk4_factor(nu * lam * dt) ** steps * u0
    rel = np.linalg.norm(u - exact_discrete) / np.linalg.norm(exact_discrete)
    assert rel < 1e-13
    analytic = math.exp(-2 * nu * steps * dt) * u0
    rel_a = np.linalg.norm(u - analytic) / np.linalg.norm(analytic)
    assert 1e-7 < rel_a < 5e-6


def test_extruded_taylor_green_3d_rk4_closed_form():
    n = (8, 8, 4)
    nu, dt = 0.05, 1e-2
    h = S.spacing(n)
    u0 = S.taylor_green_3d_extruded(n, amplitude=2.0)
    u = u0.copy()
    for _ in range(5):
        u = O.step_rk4(u, h, nu, dt)
    lam = -2 * 4 * math.sin(h[0] / 2) ** 2 / h[0] ** 2
    np.testing.assert_allclose(u, _rk4_factor(nu * lam * dt) ** 5 * u0, atol=1e-13)


def test_shear_wave_rk4_closed_form():
    n = (6, 12, 4)
    nu, dt, m = 0.1, 5e-3, 2
    h = S.spacing(n)
    u0 = S.shear_wave(n, m=m, amplitude=1.5)
    u = u0.copy()
    for _ in range(7):
        u = O.step_rk4(u, h, nu, dt)
    lam = -4 * math.sin(m * h[1] / 2) ** 2 / h[1] ** 2
    np.testing.assert_allclose(u, _rk4_factor(nu * lam * dt) ** 7 * u0, atol=1e-13)


@pytest.mark.parametrize("n", [(16, 16), (8, 6, 10)])
def test_projected_rhs_energy_budget(n):
    """<u, P F(u)> = nu <u, Lap u> for solenoidal u: convection and pressure do no work."""
    h = S.spacing(n)
    nu = 0.02
    u = S.turbulence_ic(n, seed=2, k0=2)
    pf = O.project(O.rhs(u, h, nu), h)[0]
    a = _dot(u, pf)
    b = nu * _dot(u, O.diffusion(u, h, 1.0))
    assert abs(a - b) < 1e-11 * abs(b)


def test_step_preserves_solenoidality_and_decays_energy():
    n = (12, 10, 8)
    h = S.spacing(n)
    u = S.turbulence_ic(n, seed=4, k0=2)
    e0 = O.kinetic_energy(u)
    u1 = O.step_rk4(u, h, 0.01, 1e-2)
    assert np.abs(O.divergence(u1, h)).max() < 1e-12 / min(h)
    assert O.kinetic_energy(u1) < e0
