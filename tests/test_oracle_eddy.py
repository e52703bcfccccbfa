"""Pins of the Smagorinsky eddy-viscosity oracle (appendix on eddy-viscosity
models) and of its pullback, by routes other than its own formulas:
* discrete energy identity: <u, M(u)> = -2 sum_I nu_t sum_a D_a^2
  - 4 sum_{a<b} sum_J nu_e S_ab^2 <= 0 (summation by parts of the assembly);
* closed form for a single shear mode u_x = sin(k y), written in 1D;
* degree-2 homogeneity and equivariance under exchanging the axes;
* central differences of the term against its pullback.
"""
import math

import numpy as np
import pytest

import oracle.eddy as E
import synth as S


def _dot(a, b):
    return float(np.sum(a * b))


def _h(n):
    return tuple([1.0, 1.3, 0.8][a] * 2 * math.pi / n[a] for a in range(len(n)))


@pytest.mark.parametrize("n", [(8, 6), (6, 5, 7)])
def test_energy_identity_and_dissipation(n):
    h = _h(n)
    d = len(n)
    u = S.random_field(n, 3)
    M = E.smagorinsky(u, h)
    nu = E.eddy_viscosity(u, h)
    ax = lambda a: d - 1 - a  # noqa: E731  array axis of direction a
    rhs = 0.0
    for a in range(d):
        Da = (u[a] - np.roll(u[a], 1, axis=ax(a))) / h[a]
        rhs -= 2.0 * np.sum(nu * Da * Da)
    for a in range(d):
        for b in range(a + 1, d):
            gab = (np.roll(u[a], -1, axis=ax(b)) - u[a]) / h[b]
            gba = (np.roll(u[b], -1, axis=ax(a)) - u[b]) / h[a]
            se = 0.5 * (gab + gba)
            nue = 0.25 * (nu + np.roll(nu, -1, axis=ax(a)) + np.roll(nu, -1, axis=ax(b))
                          + np.roll(np.roll(nu, -1, axis=ax(a)), -1, axis=ax(b)))
            rhs -= 4.0 * np.sum(nue * se * se)
    lhs = _dot(u, M)
    assert lhs < 0
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


def test_single_shear_mode_closed_form():
    nx, ny, k = 6, 16, 2
    h = (2 * math.pi / nx, 2 * math.pi / ny)
    cs, delta = 0.17, 0.3
    hy = h[1]
    ys = (np.arange(ny) + 0.5) * hy          # u^x sits at cell centres in y
    ux = np.sin(k * ys)
    G = (np.roll(ux, -1) - ux) / hy          # delta_y u^x on the edge above row j
    Ac = 0.5 * (G + np.roll(G, 1))           # mean of the edges around row j
    nu = (cs * delta) ** 2 * np.abs(Ac)      # sqrt(2 S:S) = |A_xy| for this field
    nue = 0.5 * (nu + np.roll(nu, -1))
    T = 2.0 * nue * 0.5 * G
    Mx = (T - np.roll(T, 1)) / hy
    u = np.zeros((2, ny, nx))
    u[0] = ux[:, None]
    M = E.smagorinsky(u, h, cs, delta)
    np.testing.assert_allclose(M[0], np.broadcast_to(Mx[:, None], (ny, nx)), atol=1e-13)
    np.testing.assert_allclose(M[1], 0.0, atol=1e-13)


def test_homogeneity():
    n = (6, 5, 7)
    h = _h(n)
    u = S.random_field(n, 4)
    M = E.smagorinsky(u, h)
    for lam in (2.5, -0.7):
        np.testing.assert_allclose(E.smagorinsky(lam * u, h), lam * abs(lam) * M, atol=1e-12 * np.abs(M).max())


def test_axis_exchange_equivariance():
    n = (7, 5)
    h = (0.4, 0.9)
    u = S.random_field(n, 5)
    M = E.smagorinsky(u, h, delta=0.5)
    # exchange x and y: component 0 <-> 1, array axes transposed, spacings swapped
    ut = np.stack([u[1].T, u[0].T])
    Mt = E.smagorinsky(ut, (h[1], h[0]), delta=0.5)
    np.testing.assert_allclose(Mt[0], M[1].T, atol=1e-12)
    np.testing.assert_allclose(Mt[1], M[0].T, atol=1e-12)


@pytest.mark.parametrize("n", [(8, 6), (5, 6, 4)])
def test_pullback_central_difference(n):
    h = _h(n)
    u = S.random_field(n, 6)
    mbar = S.random_field(n, 7)
    g = E.smagorinsky_vjp(u, mbar, h)
    for seed in (8, 9, 10):
        v = S.random_field(n, seed)
        eps = 1e-6
        fd = _dot(mbar, (E.smagorinsky(u + eps * v, h) - E.smagorinsky(u - eps * v, h)) / (2 * eps))
        assert abs(fd - _dot(g, v)) < 1e-7 * np.abs(g * v).sum()


def test_zero_and_constant_fields():
    n = (6, 5, 4)
    h = _h(n)
    u = np.zeros((3, 4, 5, 6))
    u[0] = 1.3
    u[2] = -0.4
    assert np.abs(E.smagorinsky(u, h)).max() == 0.0
    assert np.abs(E.smagorinsky_vjp(u, S.random_field(n, 1), h)).max() == 0.0
