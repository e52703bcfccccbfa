"""Float64 oracle of the auxiliary LES data steps: face filter and energy spectrum.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper does not define the filter or the spectrum binning (it refers to
spectra only in passing, Sec. 5.7); the readings used here are:
* face filter: the coarse a-velocity is the mean of the ``f**(d-1)`` fine
  a-velocities lying on the coarse a-face (coarse cell I covers fine cells
  f*I .. f*I+f-1; its right a-face is the right face of fine cell f*I+f-1);
* spectrum: E(k) = 1/2 sum over the shell k-1/2 <= |k| < k+1/2 of
  sum_a |uhat_a|^2 / N_cells^2, integer k.
"""
from __future__ import annotations

import numpy as np


def face_filter(u, factor=4):
    """Coarse staggered field from the fine face averages (see module docstring)."""
    d = u.shape[0]
    fine = u.shape[1:]
    if any(s % factor for s in fine):
        raise ValueError("grid not divisible by the filter factor")
    coarse = tuple(s // factor for s in fine)
    out = np.zeros((d,) + coarse, dtype=np.float64)
    for a in range(d):
        ax = d - 1 - a
        v = u[a]
        # select the last fine face inside each coarse cell along a
        idx = np.arange(factor - 1, fine[ax], factor)
        v = np.take(v, idx, axis=ax)
        # average over the f fine faces along every other direction
        for b in range(d):
            if b == a:
                continue
            bx = d - 1 - b
            shp = list(v.shape)
            shp[bx] = shp[bx] // factor
            shp.insert(bx + 1, factor)
            v = v.reshape(shp).mean(axis=bx + 1)
        out[a] = v
    return out


def energy_spectrum(u):
    """Shell-binned kinetic-energy spectrum (k = 0, 1, ..., kmax) of a periodic field."""
    d = u.shape[0]
    shape = u.shape[1:]
    ncell = int(np.prod(shape))
    e = np.zeros(shape, dtype=np.float64)
    for a in range(d):
        uh = np.fft.fftn(u[a])
        e += (uh.real ** 2 + uh.imag ** 2)
    e *= 0.5 / (ncell * ncell)
    kk = np.zeros(shape, dtype=np.float64)
    for ax in range(d):
        k = np.fft.fftfreq(shape[ax], 1.0 / shape[ax])
        s = [1] * d
        s[ax] = shape[ax]
        kk = kk + (k * k).reshape(s)
    kmag = np.sqrt(kk)
    shell = np.floor(kmag + 0.5).astype(np.int64)
    return np.bincount(shell.ravel(), weights=e.ravel())
