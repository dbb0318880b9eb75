"""Synthetic streamer-shaped coefficient and source fields (see package doc).

Readings of the workload descriptions that the paper leaves open:

* smoothstep window of the filament along z over [0.2, 0.8]:
  s(z) = S((z - 0.2)/0.05) * S((0.8 - z)/0.05), S(t) = c^2 (3 - 2c), c = clamp(t, 0, 1);
* lognormal noise multiplies the electron density: xi = exp(0.1 * N(0, 1)) per cell;
* the ion density is the noiseless profile shifted by +0.02 in z, times 0.9 and
  the same noise field;
* kappa is fixed after the noise is drawn so that max(a) equals the requested
  contrast exactly.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 1812086060

# Default edge length (cells per side) of each numbered workload.
CONFIG_SIZES = {1: 64, 2: 256, 3: 512, 4: 256, 5: 768}


@dataclass
class Problem:
    """One solve: -div(a grad phi) = f on the unit cube, phi = phi_bot at z=0,
    phi = phi_top at z=1, homogeneous Neumann on the x and y faces."""

    name: str
    shape: tuple  # (nx, ny, nz)
    h: tuple  # (hx, hy, hz)
    a: np.ndarray  # (nz, ny, nx) float64, > 0
    f: np.ndarray  # (nz, ny, nx) float64
    phi_bot: float = 0.0
    phi_top: float = 1.0
    meta: dict = field(default_factory=dict)


def cell_centres(n: int, length: float = 1.0) -> np.ndarray:
    """Centres (i + 1/2) h of n uniform cells on [0, length]."""
    h = length / n
    return (np.arange(n, dtype=np.float64) + 0.5) * h


def smoothstep_window(z: np.ndarray, lo: float = 0.2, hi: float = 0.8,
                      width: float = 0.05) -> np.ndarray:
    def S(t):
        c = np.clip(t, 0.0, 1.0)
        return c * c * (3.0 - 2.0 * c)

    return S((z - lo) / width) * S((hi - z) / width)


def _rng(config_number: int) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + config_number)


def config_gaussian_source(n: int = 64, seed_number: int = 1) -> Problem:
    """Constant coefficient a = 1, Gaussian source at the cube centre plus
    uniform noise in [-1e-3, 1e-3]; phi = 0 / 1 on the plates."""
    rng = _rng(seed_number)
    c = cell_centres(n)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    r2 = (x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2
    f = 100.0 * np.exp(-r2 / (2.0 * 0.05 ** 2))
    f += rng.uniform(-1e-3, 1e-3, size=f.shape)
    a = np.ones((n, n, n), dtype=np.float64)
    return Problem(name=f"gaussian_source_{n}", shape=(n, n, n),
                   h=(1.0 / n,) * 3, a=a, f=f, phi_bot=0.0, phi_top=1.0,
                   meta={"seed": SEED_BASE + seed_number, "a_max": 1.0})


def _filament_profile(n: int, xc: float, yc: float, sigma: float,
                      z_shift: float) -> np.ndarray:
    """exp(-r^2 / (2 sigma^2)) * s(z - z_shift) with r the distance from the
    axis (xc, yc), as a (nz, ny, nx) array."""
    c = cell_centres(n)
    radial = np.exp(-((c[None, :] - xc) ** 2 + (c[:, None] - yc) ** 2)
                    / (2.0 * sigma ** 2))  # (ny, nx)
    s = smoothstep_window(c - z_shift)  # (nz,)
    return s[:, None, None] * radial[None, :, :]


def config_filament(n: int = 256, a_max: float = 1e3, seed_number: int = 2,
                    sigma: float = 0.03) -> Problem:
    """One filament along the z axis through (0.5, 0.5): n_e is the
    Gaussian-in-r, smoothstep-in-z profile times lognormal noise;
    a = 1 + kappa n_e with max(a) = a_max; f = 50 (n_p - n_e)."""
    rng = _rng(seed_number)
    xi = np.exp(0.1 * rng.standard_normal((n, n, n)))
    n_e = _filament_profile(n, 0.5, 0.5, sigma, 0.0) * xi
    n_p = 0.9 * _filament_profile(n, 0.5, 0.5, sigma, 0.02) * xi
    del xi
    kappa = (a_max - 1.0) / n_e.max()
    a = 1.0 + kappa * n_e
    f = 50.0 * (n_p - n_e)
    return Problem(name=f"filament_{n}_amax{a_max:g}", shape=(n, n, n),
                   h=(1.0 / n,) * 3, a=a, f=f, phi_bot=0.0, phi_top=1.0,
                   meta={"seed": SEED_BASE + seed_number, "a_max": a_max,
                         "kappa": kappa})


def config_two_filaments(n: int = 768, a_max: float = 1e4, seed_number: int = 5,
                         step: int = 0, sigma: float = 0.02,
                         x_centres=(0.42, 0.58)) -> Problem:
    """Two filaments along z at x = 0.42 and 0.58 (y = 0.5), each with its own
    lognormal noise.  ``step`` advects both one cell per step in +z: the
    profiles are evaluated at z - step*h and the noise is rolled by ``step``
    cells along z."""
    rng = _rng(seed_number)
    h = 1.0 / n
    n_e = np.zeros((n, n, n), dtype=np.float64)
    n_p = np.zeros((n, n, n), dtype=np.float64)
    for xc in x_centres:
        xi = np.exp(0.1 * rng.standard_normal((n, n, n)))
        if step:
            xi = np.roll(xi, step, axis=0)
        n_e += _filament_profile(n, xc, 0.5, sigma, step * h) * xi
        n_p += 0.9 * _filament_profile(n, xc, 0.5, sigma, step * h + 0.02) * xi
        del xi
    kappa = (a_max - 1.0) / n_e.max()
    a = 1.0 + kappa * n_e
    f = 50.0 * (n_p - n_e)
    return Problem(name=f"two_filaments_{n}_step{step}", shape=(n, n, n),
                   h=(h,) * 3, a=a, f=f, phi_bot=0.0, phi_top=1.0,
                   meta={"seed": SEED_BASE + seed_number, "a_max": a_max,
                         "kappa": kappa, "step": step})


def config_streamer_mesh(nx: int = 256, ny: int = 256, nz: int = 320, a_max: float = 1e4,
                         seed_number: int = 6, sigma: float = 0.03,
                         constant_a: bool = False) -> Problem:
    """The channel of a double-headed streamer on the unit cube meshed with
    nx x ny x nz cells (the meshes of the scalability and solver-comparison
    runs of Sec. 5.3 are 256 x 256 x 320 and its refinements, so h_z < h_x =
    h_y).  One filament along z through (0.5, 0.5), the same profile and
    noise as ``config_filament``, sampled at this mesh's cell centres;
    ``constant_a`` keeps f and sets a = 1 (the constant-coefficient problem of
    the explicit scheme, Table t2)."""
    rng = _rng(seed_number)
    cx, cy, cz = cell_centres(nx), cell_centres(ny), cell_centres(nz)
    radial = np.exp(-((cx[None, :] - 0.5) ** 2 + (cy[:, None] - 0.5) ** 2) / (2.0 * sigma ** 2))
    xi = np.exp(0.1 * rng.standard_normal((nz, ny, nx)))
    n_e = smoothstep_window(cz)[:, None, None] * radial[None, :, :] * xi
    n_p = 0.9 * smoothstep_window(cz - 0.02)[:, None, None] * radial[None, :, :] * xi
    del xi
    f = 50.0 * (n_p - n_e)
    if constant_a:
        a = np.ones((nz, ny, nx), dtype=np.float64)
        kappa = 0.0
        a_max = 1.0
    else:
        kappa = (a_max - 1.0) / n_e.max()
        a = 1.0 + kappa * n_e
    return Problem(name=f"streamer_mesh_{nx}x{ny}x{nz}_amax{a_max:g}", shape=(nx, ny, nz),
                   h=(1.0 / nx, 1.0 / ny, 1.0 / nz), a=a, f=f, phi_bot=0.0, phi_top=1.0,
                   meta={"seed": SEED_BASE + seed_number, "a_max": a_max, "kappa": kappa})


def probe_box_mask(n: int, box=((0.4, 0.6), (0.4, 0.6), (0.45, 0.55))) -> np.ndarray:
    """Boolean (nz, ny, nx) mask of cells whose centre lies in the closed box
    [x0,x1] x [y0,y1] x [z0,z1]."""
    c = cell_centres(n)
    (x0, x1), (y0, y1), (z0, z1) = box
    mx = (c >= x0) & (c <= x1)
    my = (c >= y0) & (c <= y1)
    mz = (c >= z0) & (c <= z1)
    return mz[:, None, None] & my[None, :, None] & mx[None, None, :]


def make_config(number: int, n: int | None = None, step: int = 0) -> Problem:
    """Numbered workload at its default size, or at edge length ``n``.

    1: constant a, Gaussian source (64^3).
    2: one filament, max(a) = 1e3 (256^3).
    3: one filament, max(a) = 1e4 (512^3, the headline size).
    4: as 2; used with the probe-box loss for the gradient.
    5: two filaments, max(a) = 1e4 (768^3), ``step`` = advection step.
    """
    n = CONFIG_SIZES[number] if n is None else n
    if number == 1:
        return config_gaussian_source(n, seed_number=1)
    if number == 2:
        return config_filament(n, a_max=1e3, seed_number=2)
    if number == 3:
        return config_filament(n, a_max=1e4, seed_number=3)
    if number == 4:
        return config_filament(n, a_max=1e3, seed_number=4)
    if number == 5:
        return config_two_filaments(n, a_max=1e4, seed_number=5, step=step)
    raise ValueError(f"unknown workload {number}")
