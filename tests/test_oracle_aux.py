"""Pins of the oracle's filter and spectrum, and of the seeded input generators."""
import math

import numpy as np
import pytest

import oracle as O
import synth as S


@pytest.mark.parametrize("n", [(16, 8), (8, 12, 16)])
def test_face_filter_commutes_with_divergence(n):
    """D_coarse(Phi u) equals the volume mean of D u over each coarse cell (telescoping sums)."""
    d = len(n)
    f = 4
    u = S.random_field(n, 3)
    h = S.spacing(n)
    nc = tuple(v // f for v in n)
    H = S.spacing(nc)
    lhs = O.divergence(O.face_filter(u, f), H)
    du = O.divergence(u, h)
    shp = []
    for s in du.shape:
        shp += [s // f, f]
    rhs = du.reshape(shp).mean(axis=tuple(range(1, 2 * d, 2)))
    np.testing.assert_allclose(lhs, rhs, atol=1e-12 * np.abs(du).max())


def test_face_filter_of_constant_and_brute_force():
    n = (8, 4, 12)
    u = S.random_field(n, 4)
    c = O.face_filter(u, 4)
    # brute force one entry: coarse x-face (i=1, j=0, k=2) averages fine x-faces i=7, j in 0..3, k in 8..11
    expect = u[0][8:12, 0:4, 7].mean()
    assert abs(c[0][2, 0, 1] - expect) < 1e-15
    expect_z = u[2][4 * 1 + 3, 0:4, 4:8].mean()
    assert abs(c[2][1, 0, 1] - expect_z) < 1e-15


@pytest.mark.parametrize("n", [(16, 16), (8, 10, 12)])
def test_spectrum_parseval(n):
    u = S.random_field(n, 5)
    e = O.energy_spectrum(u)
    assert abs(e.sum() - O.kinetic_energy(u)) < 1e-12 * O.kinetic_energy(u)


def test_spectrum_of_single_mode():
    """u_x = cos(3 y): all energy (1/4 per unit amplitude^2) in shell k = 3."""
    n = (8, 16)
    u = np.zeros((2, 16, 8))
    y = (np.arange(16) + 0.5) * 2 * math.pi / 16
    u[0] = np.cos(3 * y)[:, None]
    e = O.energy_spectrum(u)
    assert abs(e[3] - 0.25) < 1e-14 and abs(e.sum() - 0.25) < 1e-14


@pytest.mark.parametrize("n,k0", [((32, 32), 4), ((24, 24, 24), 4)])
def test_turbulence_ic_properties(n, k0):
    u = S.turbulence_ic(n, seed=0, k0=k0)
    assert abs(O.kinetic_energy(u) - 1.0) < 1e-12
    assert np.abs(O.divergence(u, S.spacing(n))).max() < 1e-12 * np.abs(u).max() * max(n)
    e = O.energy_spectrum(u)
    assert 2 <= int(np.argmax(e)) <= 6
    u2 = S.turbulence_ic(n, seed=0, k0=k0)
    assert np.array_equal(u, u2)
