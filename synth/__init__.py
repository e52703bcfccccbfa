"""Seeded synthetic inputs for the staggered periodic Navier-Stokes path.

This module is shared by the CPU oracle, the tests and the benchmark. It only
*samples* input fields; it contains none of the method's operators (no
divergence, gradient, diffusion, convection, Poisson solve, projection or time
stepping). Random numbers are drawn here and handed to both sides as plain
arrays.

Layout (same for every consumer): a velocity field on a d-dimensional grid with
cell counts ``n = (N_x, N_y[, N_z])`` is a float64 array of shape
``(d, N_z, N_y, N_x)`` (3D) or ``(d, N_y, N_x)`` (2D); component ``a`` is the
velocity normal to the ``a``-faces and entry ``[a][I]`` sits on the face to the
right of cell centre ``I`` in direction ``a`` (paper Sec. 2.1 and App. A.1:
one pressure and one of each velocity component per volume, velocity to the
right of the centre). Cell ``i`` spans ``[lo + i h, lo + (i+1) h]``.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "turbulence_ic_torch",
    "spacing",
    "face_coords",
    "taylor_green_2d",
    "taylor_green_3d_extruded",
    "shear_wave",
    "random_field",
    "random_scalar",
    "turbulence_ic",
    "energy_spectrum_shape",
    "channel_box",
    "channel_shear",
    "channel_ic",
    "channel_random",
    "tanh_faces",
]

TWO_PI = 2.0 * math.pi


def spacing(n, lo=None, hi=None):
    """Uniform spacings h_a = (hi_a - lo_a) / N_a for a 2pi-periodic box by default."""
    d = len(n)
    lo = [0.0] * d if lo is None else list(lo)
    hi = [TWO_PI] * d if hi is None else list(hi)
    return tuple((hi[a] - lo[a]) / n[a] for a in range(d))


def face_coords(n, alpha, lo=None, hi=None):
    """Coordinates of the alpha-velocity points as broadcastable arrays.

    Returns a list ``[x_0, x_1, ...]`` (x_0 = x-coordinate) of arrays shaped to
    broadcast against ``(N_z, N_y, N_x)``: along ``alpha`` the point is the
    right face ``lo + (i+1) h``, along the other directions the cell centre
    ``lo + (i+1/2) h``.
    """
    d = len(n)
    lo = [0.0] * d if lo is None else list(lo)
    h = spacing(n, lo, hi)
    out = []
    for b in range(d):
        off = 1.0 if b == alpha else 0.5
        c = lo[b] + (np.arange(n[b], dtype=np.float64) + off) * h[b]
        shape = [1] * d
        shape[d - 1 - b] = n[b]
        out.append(c.reshape(shape))
    return out


def taylor_green_2d(n, amplitude=1.0):
    """2D Taylor-Green vortex u = sin(x)cos(y), v = -cos(x)sin(y) on [0,2pi]^2.

    Sampled at the staggered velocity points. ``n`` is an int or (N_x, N_y).
    """
    if np.isscalar(n):
        n = (int(n), int(n))
    nx, ny = n
    u = np.empty((2, ny, nx), dtype=np.float64)
    x, y = face_coords(n, 0)
    u[0] = np.sin(x) * np.cos(y)
    x, y = face_coords(n, 1)
    u[1] = -np.cos(x) * np.sin(y)
    return amplitude * u


def taylor_green_3d_extruded(n, amplitude=1.0):
    """The 2D Taylor-Green field repeated along z, with zero z-velocity."""
    if np.isscalar(n):
        n = (int(n),) * 3
    nx, ny, nz = n
    u = np.zeros((3, nz, ny, nx), dtype=np.float64)
    u2 = taylor_green_2d((nx, ny), amplitude)
    u[0] = u2[0][None]
    u[1] = u2[1][None]
    return u


def shear_wave(n, m=1, amplitude=1.0):
    """u_x = A sin(m y) (a parallel shear flow), other components zero."""
    d = len(n)
    shape = (d,) + tuple(reversed(n))
    u = np.zeros(shape, dtype=np.float64)
    coords = face_coords(n, 0)
    u[0] = amplitude * np.sin(m * coords[1]) * np.ones(tuple(reversed(n)))
    return u


def random_field(n, seed, components=None):
    """Seeded standard-normal vector field of shape (d, *reversed(n))."""
    d = len(n)
    c = d if components is None else components
    rng = np.random.default_rng(seed)
    return rng.standard_normal((c,) + tuple(reversed(n)))


def random_scalar(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(tuple(reversed(n)))


def energy_spectrum_shape(k, k0):
    """Target shape E(k) ~ k^4 exp(-2 (k/k0)^2) of the decaying-turbulence initial field."""
    k = np.asarray(k, dtype=np.float64)
    return k ** 4 * np.exp(-2.0 * (k / k0) ** 2)


def _int_wavenumbers(n):
    d = len(n)
    ks = []
    for b in range(d):
        k = np.fft.fftfreq(n[b], 1.0 / n[b])
        shape = [1] * d
        shape[d - 1 - b] = n[b]
        ks.append(k.reshape(shape))
    return ks


def _filtered_noise(n, rng, amp):
    w = rng.standard_normal(tuple(reversed(n)))
    return np.real(np.fft.ifftn(np.fft.fftn(w) * amp))


def turbulence_ic(n, seed, k0=4.0, energy=1.0):
    """Random solenoidal velocity with E(k) ~ k^4 exp(-2(k/k0)^2), mean KE = ``energy``.

    The field is the staggered-grid curl of a random potential (a stream
    function on cell corners in 2D, a vector potential on cell edges in 3D)
    whose Fourier amplitudes follow sqrt(E(|k|) / S_d(|k|)) / |k| with
    S_2 = 2 pi k and S_3 = 4 pi k^2, applied to seeded white noise. The discrete
    divergence of a discrete curl vanishes identically, so the result is
    solenoidal up to rounding without using the solver's projection. It is
    then scaled so that (1/2) mean_I sum_a u_a[I]^2 = energy.
    """
    n = tuple(int(v) for v in n)
    d = len(n)
    if d not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    rng = np.random.default_rng(seed)
    h = spacing(n)
    ks = _int_wavenumbers(n)
    kk = np.sqrt(sum(k * k for k in ks))
    shell = 2.0 * math.pi * kk if d == 2 else 4.0 * math.pi * kk ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        amp = np.sqrt(energy_spectrum_shape(kk, k0) / shell) / kk
    amp[(0,) * d] = 0.0

    def back(f, b):  # f[I - e_b]
        return np.roll(f, 1, axis=d - 1 - b)

    u = np.empty((d,) + tuple(reversed(n)), dtype=np.float64)
    if d == 2:
        psi = _filtered_noise(n, rng, amp)
        u[0] = (psi - back(psi, 1)) / h[1]
        u[1] = -(psi - back(psi, 0)) / h[0]
    else:
        ax_, ay_, az_ = (_filtered_noise(n, rng, amp) for _ in range(3))
        u[0] = (az_ - back(az_, 1)) / h[1] - (ay_ - back(ay_, 2)) / h[2]
        u[1] = (ax_ - back(ax_, 2)) / h[2] - (az_ - back(az_, 0)) / h[0]
        u[2] = (ay_ - back(ay_, 0)) / h[0] - (ax_ - back(ax_, 1)) / h[1]
    ke = 0.5 * np.mean(np.sum(u * u, axis=0))
    u *= math.sqrt(energy / ke)
    return u


def turbulence_ic_torch(n, seed, k0=4.0, energy=1.0, device="cuda", dtype=None):
    """``turbulence_ic`` built on the GPU with torch (for grids too large for numpy).

    Same construction (staggered curl of a potential with spectral amplitude
    sqrt(E(|k|)/S_d(|k|))/|k|, then scaling to the mean kinetic energy), but the
    white noise comes from torch's seeded generator, so the field differs from
    ``turbulence_ic`` for the same seed. Returns a float64 (or ``dtype``) tensor
    of shape (d, *reversed(n)).
    """
    import torch

    n = tuple(int(v) for v in n)
    d = len(n)
    dtype = torch.float64 if dtype is None else dtype
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    h = spacing(n)
    shape = tuple(reversed(n))
    # wavenumbers on the half spectrum of the last (x) axis
    kk = torch.zeros((), dtype=torch.float64, device=device)
    for b in range(d):
        ax = d - 1 - b
        if b == 0:
            k = torch.fft.rfftfreq(n[0], 1.0 / n[0], dtype=torch.float64, device=device)
        else:
            k = torch.fft.fftfreq(n[b], 1.0 / n[b], dtype=torch.float64, device=device)
        s = [1] * d
        s[ax] = k.numel()
        kk = kk + (k * k).reshape(s)
    kmag = torch.sqrt(kk)
    shell = 2 * math.pi * kmag if d == 2 else 4 * math.pi * kmag ** 2
    e = kmag ** 4 * torch.exp(-2.0 * (kmag / k0) ** 2)
    amp = torch.where(kmag > 0, torch.sqrt(e / torch.where(shell > 0, shell, 1.0)) / torch.where(kmag > 0, kmag, 1.0),
                      torch.zeros_like(kmag))

    def noise_field():
        w = torch.randn(shape, generator=gen, dtype=torch.float64, device=device)
        return torch.fft.irfftn(torch.fft.rfftn(w) * amp, s=shape)

    def back(f, b):
        return torch.roll(f, 1, dims=d - 1 - b)

    u = torch.empty((d,) + shape, dtype=torch.float64, device=device)
    if d == 2:
        psi = noise_field()
        u[0] = (psi - back(psi, 1)) / h[1]
        u[1] = -(psi - back(psi, 0)) / h[0]
    else:
        ax_ = noise_field()
        ay_ = noise_field()
        az_ = noise_field()
        u[0] = (az_ - back(az_, 1)) / h[1] - (ay_ - back(ay_, 2)) / h[2]
        u[1] = (ax_ - back(ax_, 2)) / h[2] - (az_ - back(az_, 0)) / h[0]
        u[2] = (ay_ - back(ay_, 0)) / h[0] - (ax_ - back(ax_, 1)) / h[1]
        del ax_, ay_, az_
    ke = 0.5 * (u * u).sum(0).mean()
    u *= torch.sqrt(energy / ke)
    return u.to(dtype)


# ----------------------------------------------------------------------------
# Channel inputs: no-slip walls at both ends of y (x, z periodic). The normal
# velocity u^y[..., N_y - 1, ...] is the upper-wall face and is always 0.
# ----------------------------------------------------------------------------

def channel_box(n):
    """Box of the channel inputs: x in [0, 2pi], y in [0, 2] (walls), z in [0, pi]."""
    d = len(n)
    lo = [0.0] * d
    hi = [TWO_PI, 2.0, math.pi][:d]
    return lo, hi


def channel_shear(n, m=1, amplitude=1.0, component=0):
    """u^c = A sin(pi m (y - lo_y) / L_y) (c = x or z) sampled at the cell centres in y."""
    lo, hi = channel_box(n)
    d = len(n)
    u = np.zeros((d,) + tuple(reversed(n)))
    y = face_coords(n, component, lo, hi)[1]
    u[component] = amplitude * np.sin(math.pi * m * (y - lo[1]) / (hi[1] - lo[1])) * np.ones(tuple(reversed(n)))
    return u


def _wall_potential(n, rng, modes, lo, hi, yoff):
    """Smooth random potential sampled at y faces j = 0 .. N_y - 1 (y = lo + (j + 1) h_y), exactly
    zero on the upper wall row; other coordinates at the offsets given by yoff (x, z offsets)."""
    d = len(n)
    h = spacing(n, lo, hi)
    shape = tuple(reversed(n))
    grids = []
    for b in range(d):
        off = 1.0 if b == 1 else yoff[b]
        c = lo[b] + (np.arange(n[b]) + off) * h[b]
        sh = [1] * d
        sh[d - 1 - b] = n[b]
        grids.append(c.reshape(sh))
    ly = hi[1] - lo[1]
    psi = np.zeros(shape)
    for _ in range(modes):
        m = int(rng.integers(1, 4))
        kx = int(rng.integers(0, 4))
        kz = int(rng.integers(0, 3)) if d == 3 else 0
        ph = rng.uniform(0, 2 * math.pi)
        amp = rng.normal() / (1.0 + m + kx + kz)
        arg = kx * TWO_PI * grids[0] / (hi[0] - lo[0]) + ph
        if d == 3:
            arg = arg + kz * TWO_PI * grids[2] / (hi[2] - lo[2])
        psi = psi + amp * np.sin(math.pi * m * (grids[1] - lo[1]) / ly) * np.cos(arg)
    psi[(Ellipsis, slice(n[1] - 1, n[1]), slice(None))] = 0.0  # upper wall row, exactly
    return psi


def channel_ic(n, seed, bulk=1.0, noise=0.2, modes=12, box=None):
    """Laminar profile u^x = 1.5 bulk (1 - eta^2), eta = 2 (y - lo_y) / L_y - 1, plus a
    perturbation that is the discrete curl of a random potential vanishing on both walls.

    The curl is taken on the staggered positions (potential on cell edges, j the
    y-face index, the row below the grid being the lower wall where it is 0), so the
    field has zero discrete divergence and zero normal velocity on the walls.
    ``noise`` is the RMS of the perturbation relative to the bulk velocity; ``box`` =
    (lo, hi) replaces the default box of ``channel_box``.
    """
    d = len(n)
    lo, hi = channel_box(n) if box is None else box
    h = spacing(n, lo, hi)
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(n))
    yax = d - 2

    def below(f):  # f at y-face j - 1, zero below the lower wall
        return np.concatenate([np.zeros_like(np.take(f, [0], axis=yax)), np.take(f, range(n[1] - 1), axis=yax)],
                              axis=yax)

    def prev(f, a):  # f at I - e_a along a periodic direction
        return np.roll(f, 1, axis=d - 1 - a)

    up = np.zeros((d,) + shape)
    # psi_z on (x-face, y-face) edges: u^x += d_y psi_z, u^y -= d_x psi_z
    psz = _wall_potential(n, rng, modes, lo, hi, [1.0, 1.0, 0.5])
    up[0] += (psz - below(psz)) / h[1]
    up[1] -= (psz - prev(psz, 0)) / h[0]
    if d == 3:
        # psi_x on (y-face, z-face) edges: u^y += d_z psi_x, u^z -= d_y psi_x
        psx = _wall_potential(n, rng, modes, lo, hi, [0.5, 1.0, 1.0])
        up[1] += (psx - prev(psx, 2)) / h[2]
        up[2] -= (psx - below(psx)) / h[1]
    rms = float(np.sqrt(np.mean(up ** 2)))
    if rms > 0:
        up *= noise * bulk / rms
    y = face_coords(n, 0, lo, hi)[1]
    eta = 2.0 * (y - lo[1]) / (hi[1] - lo[1]) - 1.0
    u = up
    u[0] += 1.5 * bulk * (1.0 - eta ** 2) * np.ones(shape)
    u[(1, Ellipsis, slice(n[1] - 1, n[1]), slice(None))] = 0.0
    return u


def channel_random(n, seed):
    """Seeded standard-normal velocity with the upper-wall face of u^y set to 0."""
    u = random_field(n, seed)
    u[(1, Ellipsis, slice(n[1] - 1, n[1]), slice(None))] = 0.0
    return u


def tanh_gamma(ny, length, first_width):
    """Stretching parameter of ``tanh_faces`` whose first (and last) cell has the given
    width, by bisection (the width decreases monotonically as gamma grows)."""
    def w0(g):
        return 0.5 * length * (1.0 + np.tanh(g * (2.0 / ny - 1.0)) / np.tanh(g))
    if not first_width < length / ny:
        raise ValueError("first_width must be below the uniform width")
    a, b = 1e-6, 1.0
    while w0(b) > first_width:
        b *= 2.0
    for _ in range(200):
        m = 0.5 * (a + b)
        if w0(m) > first_width:
            a = m
        else:
            b = m
    return 0.5 * (a + b)


def tanh_faces(ny, lo, hi, gamma):
    """y-face coordinates of the hyperbolic-tangent grid (Sec. 2.5 non-uniform grids,
    eq. tanh-grid): clustered at both ends, stretching set by gamma > 0."""
    t = np.arange(ny + 1) / ny
    return lo + 0.5 * (hi - lo) * (1.0 + np.tanh(gamma * (2.0 * t - 1.0)) / np.tanh(gamma))
