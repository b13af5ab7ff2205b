"""Seeded synthetic inputs for the lattice-Boltzmann Maxwell solver.

This module only *shapes inputs*: permittivity/permeability maps, initial
fields, current-source footprints and source time series.  It holds none of
the scheme's arithmetic (no equilibria, no moments, no collision), so both the
FP64 CPU oracle and the HIP path can be fed from it without sharing code.

Conventions
-----------
* Cell index ``x + nx*(y + ny*z)``; numpy arrays are shaped ``(nz, ny, nx)``
  (2D: ``(1, ny, nx)``) so that ``arr.ravel()`` follows that index.
* Vector fields are component-major ``(3, n)`` float64.
* Distances are periodic minimum-image distances in cell units.
* A source is ``(comp, cells, weights)`` with a separate amplitude series
  ``amp[k]`` for the k-th step; the current density is
  ``j_comp(cell, t) = weight * amp[t]``.

The workloads mirror the paper's experiments (homogeneous pulse, heterogeneous
high-contrast medium, line / dipole current forcing; Section "Numerical
results") with synthetic, seeded media standing in for the medium of the
paper's Figure 2, which exists only as a picture.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem", "seed_for", "vacuum_speed", "ricker", "gaussian_pulse",
    "smooth_noise", "heterogeneous_2d", "spheres_3d", "layered_3d",
    "line_source", "dipole_source", "crop", "config1", "config2", "config3",
    "config4", "serving_requests", "paper_jz_source", "paper_vortex_ic",
]


def seed_for(config: int) -> int:
    """Seed convention of the workload recipes: 1108*10 + config number."""
    return 1108 * 10 + int(config)


def vacuum_speed(dim: int, w0_vac: float) -> float:
    """Lattice-unit speed of light where eps_r*mu_r = 1.

    Unit convention used to choose source wavelengths: with rest weight
    ``w0_vac`` the per-axis second moment is (1-w0_vac)/D and the Maxwell
    speed squared is that divided by (D-1).
    """
    return math.sqrt((1.0 - w0_vac) / (dim * (dim - 1)))


@dataclass
class Problem:
    """A complete synthetic solve: lattice, medium, initial fields, source."""
    dim: int
    shape: tuple            # (nx, ny, nz) ; nz == 1 in 2D
    eps_r: np.ndarray       # (n,) float64
    mu_r: np.ndarray | None  # (n,) float64 or None for mu == 1
    E0: np.ndarray          # (3, n) float64
    B0: np.ndarray          # (3, n) float64
    src_comp: int = 2
    src_cells: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))
    src_weights: np.ndarray = field(default_factory=lambda: np.zeros(0))
    amp: np.ndarray | None = None   # (nsteps,) float64 or None
    nsteps: int = 0
    w0_vac: float = 1.0 / 3.0
    tau: float = 0.5
    name: str = ""

    @property
    def n(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz


# ----------------------------------------------------------------------------
# time series
# ----------------------------------------------------------------------------

def ricker(nsteps: int, f: float, t0: float | None = None, t_start: int = 0,
           amplitude: float = 1.0) -> np.ndarray:
    """Ricker wavelet (1-2 pi^2 f^2 s^2) exp(-pi^2 f^2 s^2), s = t - t0,
    sampled at integer times t_start .. t_start+nsteps-1 (float64)."""
    if t0 is None:
        t0 = 1.5 / f
    t = np.arange(t_start, t_start + nsteps, dtype=np.float64)
    a = (math.pi * f * (t - t0)) ** 2
    return amplitude * (1.0 - 2.0 * a) * np.exp(-a)


# ----------------------------------------------------------------------------
# geometry helpers
# ----------------------------------------------------------------------------

def _periodic_delta(coord: np.ndarray, centre: float, size: int) -> np.ndarray:
    d = coord - centre
    return d - size * np.round(d / size)


def _grids(shape):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64),
                          np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def gaussian_pulse(shape, centre, sigma: float, amplitude: float = 1.0) -> np.ndarray:
    """exp(-|x-c|^2/(2 sigma^2)) with minimum-image distance, shaped (nz,ny,nx)."""
    nx, ny, nz = shape
    x, y, z = _grids(shape)
    r2 = _periodic_delta(x, centre[0], nx) ** 2 + _periodic_delta(y, centre[1], ny) ** 2
    if nz > 1:
        r2 = r2 + _periodic_delta(z, centre[2], nz) ** 2
    return amplitude * np.exp(-r2 / (2.0 * sigma * sigma))


def smooth_noise(rng: np.random.Generator, shape2or3, sigma: float) -> np.ndarray:
    """iid U[0,1) noise smoothed by a periodic Gaussian of std ``sigma`` cells
    (FFT convolution), min-max rescaled to [0, 1]."""
    u = rng.random(shape2or3)
    k = [np.fft.fftfreq(s) * 2.0 * np.pi for s in shape2or3]
    kk = np.meshgrid(*k, indexing="ij")
    k2 = sum(ki * ki for ki in kk)
    s = np.fft.ifftn(np.fft.fftn(u) * np.exp(-0.5 * sigma * sigma * k2)).real
    s -= s.min()
    mx = s.max()
    return s / mx if mx > 0 else s


# ----------------------------------------------------------------------------
# media
# ----------------------------------------------------------------------------

def heterogeneous_2d(rng, nx: int, ny: int, sigma: float = 16.0,
                     lo: float = 1.0, contrast: float = 3.0) -> np.ndarray:
    """eps_r = lo + contrast * s(x,y), s smoothed noise in [0,1]; (1,ny,nx)."""
    s = smooth_noise(rng, (ny, nx), sigma)
    return (lo + contrast * s)[None, :, :]


def spheres_3d(rng, n: int, count: int = 64, r_lo: float = 8, r_hi: float = 24,
               eps_lo: float = 2.0, eps_hi: float = 9.0) -> np.ndarray:
    """Background 1 with ``count`` sharp spheres (radius U[r_lo,r_hi], centre
    U[0,n)^3, eps U[eps_lo,eps_hi]); later spheres overwrite earlier ones."""
    eps = np.ones((n, n, n))
    radii = rng.uniform(r_lo, r_hi, count)
    centres = rng.uniform(0, n, (count, 3))
    values = rng.uniform(eps_lo, eps_hi, count)
    for r, c, v in zip(radii, centres, values):
        lo = [int(math.floor(ci - r)) for ci in c]
        hi = [int(math.ceil(ci + r)) + 1 for ci in c]
        idx = [np.arange(l, h) for l, h in zip(lo, hi)]
        d = [(ii - ci) for ii, ci in zip(idx, c)]
        dx, dy, dz = np.meshgrid(d[0], d[1], d[2], indexing="ij")
        inside = dx * dx + dy * dy + dz * dz <= r * r
        ix, iy, iz = np.meshgrid(idx[0] % n, idx[1] % n, idx[2] % n, indexing="ij")
        eps[iz[inside], iy[inside], ix[inside]] = v
    return eps


def layered_3d(rng, n: int, layers: int = 20, t_lo: int = 8, t_hi: int = 40,
               eps_lo: float = 1.0, eps_hi: float = 6.0, lateral: float = 0.1,
               sigma: float = 16.0, nxy: int | None = None) -> np.ndarray:
    """Layered eps(z) stack (thickness U{t_lo..t_hi} rescaled to sum to n, the
    last layer absorbing rounding; eps per layer U[eps_lo, eps_hi]) times a
    smooth lateral modulation (1 + lateral*(2 s(x,y) - 1))."""
    nxy = n if nxy is None else nxy
    th = rng.integers(t_lo, t_hi + 1, layers).astype(np.float64)
    th = np.floor(th * n / th.sum()).astype(np.int64)
    th[-1] += n - th.sum()
    vals = rng.uniform(eps_lo, eps_hi, layers)
    ez = np.repeat(vals, th)
    s = smooth_noise(rng, (nxy, nxy), sigma)
    return ez[:, None, None] * (1.0 + lateral * (2.0 * s[None, :, :] - 1.0))


def crop(arr: np.ndarray, lo, size) -> np.ndarray:
    """Periodic crop of a (nz,ny,nx) or (3,nz,ny,nx) array: [lo, lo+size)^d."""
    sl = tuple(slice(l, l + s) for l, s in zip(lo, size))
    if arr.ndim == 4:
        return np.ascontiguousarray(arr[(slice(None),) + sl])
    return np.ascontiguousarray(arr[sl])


# ----------------------------------------------------------------------------
# sources
# ----------------------------------------------------------------------------

def line_source(nx: int, ny: int, x0: int):
    """Unit-weight line of cells x = x0, all y (2D)."""
    cells = np.asarray([x0 + nx * y for y in range(ny)], dtype=np.int64)
    return cells, np.ones(ny)


def dipole_source(shape, centre, sigma: float = 2.0, cutoff: float = 3.0):
    """Gaussian footprint exp(-|x-c|^2/(2 sigma^2)) on the box of half-width
    cutoff*sigma around the (integer) centre; returns (cells, weights)."""
    nx, ny, nz = shape
    h = int(math.ceil(cutoff * sigma))
    cells, weights = [], []
    for dz in range(-h, h + 1):
        for dy in range(-h, h + 1):
            for dx in range(-h, h + 1):
                w = math.exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * sigma * sigma))
                x = (centre[0] + dx) % nx
                y = (centre[1] + dy) % ny
                z = (centre[2] + dz) % nz
                cells.append(x + nx * (y + ny * z))
                weights.append(w)
    order = np.argsort(cells)
    return np.asarray(cells, np.int64)[order], np.asarray(weights)[order]


# ----------------------------------------------------------------------------
# the workload recipes
# ----------------------------------------------------------------------------

def _zeros3(n):
    return np.zeros((3, n))


def config1(nsteps: int = 500, n: int = 128, seed: int | None = None) -> Problem:
    """2D homogeneous periodic box, eps=mu=1, Gaussian E_z pulse (sigma=6,
    amplitude 1, seeded random centre), B=0, no source."""
    rng = np.random.default_rng(seed_for(1) if seed is None else seed)
    centre = rng.uniform(0, n, 2)
    shape = (n, n, 1)
    E = _zeros3(n * n)
    E[2] = gaussian_pulse(shape, (centre[0], centre[1], 0.0), 6.0).ravel()
    return Problem(dim=2, shape=shape, eps_r=np.ones(n * n), mu_r=None, E0=E,
                   B0=_zeros3(n * n), nsteps=nsteps, name=f"2d-homog-{n}")


def config2(nsteps: int = 5000, n: int = 2048, seed: int | None = None,
            w0_vac: float = 1.0 / 3.0) -> Problem:
    """2D heterogeneous medium eps=1+3s (s smoothed noise, sigma 16), mu=1,
    plane-wave line current j_z at x=64 with a Ricker wavelet (wavelength 40
    cells in vacuum), fields start at zero."""
    rng = np.random.default_rng(seed_for(2) if seed is None else seed)
    eps = heterogeneous_2d(rng, n, n).ravel()
    cells, w = line_source(n, n, min(64, n - 1))
    f = vacuum_speed(2, w0_vac) / 40.0
    return Problem(dim=2, shape=(n, n, 1), eps_r=eps, mu_r=None,
                   E0=_zeros3(n * n), B0=_zeros3(n * n), src_comp=2,
                   src_cells=cells, src_weights=w, amp=ricker(nsteps, f),
                   nsteps=nsteps, w0_vac=w0_vac, name=f"2d-hetero-{n}")


def config3(nsteps: int = 2000, n: int = 256, seed: int | None = None,
            crop_lo: int | None = None, crop_n: int | None = None,
            w0_vac: float = 1.0 / 3.0) -> Problem:
    """3D: background eps=1 with 64 sharp spherical inclusions (eps U[2,9]),
    mu=1, Gaussian dipole j_z (sigma 2) at the box centre with a Ricker
    wavelet.  With ``crop_n`` the medium is cropped to [crop_lo, crop_lo +
    crop_n)^3 and run as its own periodic box, dipole at the crop's centre."""
    rng = np.random.default_rng(seed_for(3) if seed is None else seed)
    eps = spheres_3d(rng, n)
    centre = (n // 2, n // 2, n // 2)
    if crop_n is not None:
        lo = (n - crop_n) // 2 if crop_lo is None else crop_lo
        eps = crop(eps, (lo, lo, lo), (crop_n,) * 3)
        centre = tuple(c - lo for c in centre)
        n = crop_n
    shape = (n, n, n)
    cells, w = dipole_source(shape, centre)
    f = vacuum_speed(3, w0_vac) / 40.0
    N = n ** 3
    return Problem(dim=3, shape=shape, eps_r=eps.ravel(), mu_r=None,
                   E0=_zeros3(N), B0=_zeros3(N), src_comp=2, src_cells=cells,
                   src_weights=w, amp=ricker(nsteps, f), nsteps=nsteps,
                   w0_vac=w0_vac, name=f"3d-spheres-{n}")


def config4(nsteps: int = 1000, n: int = 512, seed: int | None = None,
            crop_n: int | None = None, w0_vac: float = 1.0 / 3.0) -> Problem:
    """3D layered eps(z) stack (20 layers, eps U[1,6]) with +-10% smooth
    lateral noise, mu=1, Gaussian dipole at the centre (Ricker).  ``crop_n``
    takes the centred crop as its own periodic box."""
    rng = np.random.default_rng(seed_for(4) if seed is None else seed)
    eps = layered_3d(rng, n)
    centre = (n // 2, n // 2, n // 2)
    if crop_n is not None:
        lo = (n - crop_n) // 2
        eps = crop(eps, (lo, lo, lo), (crop_n,) * 3)
        centre = tuple(c - lo for c in centre)
        n = crop_n
    shape = (n, n, n)
    cells, w = dipole_source(shape, centre)
    f = vacuum_speed(3, w0_vac) / 40.0
    N = n ** 3
    return Problem(dim=3, shape=shape, eps_r=eps.ravel(), mu_r=None,
                   E0=_zeros3(N), B0=_zeros3(N), src_comp=2, src_cells=cells,
                   src_weights=w, amp=ricker(nsteps, f), nsteps=nsteps,
                   w0_vac=w0_vac, name=f"3d-layered-{n}")


def pulse_problem(dim: int, n: int, sigma: float, rng, eps: np.ndarray | None = None,
                  mu: np.ndarray | None = None, nsteps: int = 0,
                  w0_vac: float = 1.0 / 3.0) -> Problem:
    """Source-free problem: one Gaussian E_z pulse at a seeded centre."""
    shape = (n, n, 1) if dim == 2 else (n, n, n)
    N = n ** dim
    centre = rng.uniform(0, n, 3)
    E = _zeros3(N)
    E[2] = gaussian_pulse(shape, centre, sigma).ravel()
    return Problem(dim=dim, shape=shape,
                   eps_r=np.ones(N) if eps is None else eps.ravel(),
                   mu_r=None if mu is None else mu.ravel(), E0=E, B0=_zeros3(N),
                   nsteps=nsteps, w0_vac=w0_vac, name=f"{dim}d-pulse-{n}")


def serving_requests(count: int = 2000, rate: float = 200.0, seed: int | None = None,
                     frac_2d: float = 0.7, steps_lo: int = 200, steps_hi: int = 2000,
                     side2d=(6, 10), side3d=(5, 7), frac_lowp: float = 0.5):
    """Poisson request stream: arrival times and per-request solve recipes.

    Returns a list of dicts {t_arrive, dim, n, nsteps, lowp, seed}; the medium
    of each request is built lazily with ``request_problem``.
    """
    rng = np.random.default_rng(seed_for(5) if seed is None else seed)
    gaps = rng.exponential(1.0 / rate, count)
    t = np.cumsum(gaps)
    out = []
    for k in range(count):
        is2d = rng.random() < frac_2d
        if is2d:
            side = int(round(2 ** rng.uniform(*side2d) / 16.0)) * 16
            side = max(side, 16)
        else:
            side = int(round(2 ** rng.uniform(*side3d) / 8.0)) * 8
            side = max(side, 8)
        out.append(dict(t_arrive=float(t[k]), dim=2 if is2d else 3, n=side,
                        nsteps=int(rng.integers(steps_lo, steps_hi + 1)),
                        lowp=bool(rng.random() < frac_lowp),
                        seed=int(rng.integers(0, 2 ** 31))))
    return out


def request_problem(req: dict, w0_vac: float = 1.0 / 3.0) -> Problem:
    """Materialise one serving request: smooth random eps in [1,4], mu=1,
    one Gaussian E_z pulse (sigma 6, clipped to n/6), no source."""
    rng = np.random.default_rng(req["seed"])
    dim, n = req["dim"], req["n"]
    shp = (n, n) if dim == 2 else (n, n, n)
    s = smooth_noise(rng, shp, min(8.0, n / 8.0))
    eps = 1.0 + 3.0 * s
    return pulse_problem(dim, n, min(6.0, n / 6.0), rng, eps=eps,
                         nsteps=req["nsteps"], w0_vac=w0_vac)


# ----------------------------------------------------------------------------
# the paper's own test problems (Section "Numerical results")
# ----------------------------------------------------------------------------

def paper_jz_source(n: int, x0: float = 0.3, y0: float = 0.4, width: float = 0.03):
    """Homogeneous-medium forcing of the paper: a Gaussian j_z of width 0.03
    centred at (0.3, 0.4) on the unit square, sampled at x_j = j/n.
    Returns (cells, weights) with all n*n cells."""
    xs = np.arange(n) / n
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    w = np.exp(-((X - x0) ** 2 + (Y - y0) ** 2) / (2.0 * width * width))
    return np.arange(n * n, dtype=np.int64), w.ravel()


def paper_vortex_ic(n: int, amp: float = 10.0, xc: float = 0.5, yc: float = 0.35,
                    width: float = 0.04):
    """Heterogeneous-medium initial condition of the paper: a magnetic vortex
    B_x = (y-yc) f, B_y = -(x-xc) f, f = amp exp(-r^2/(2 width^2)) on the
    unit square.  Returns B as (3, n*n) in unit-square field units."""
    xs = np.arange(n) / n
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    f = amp * np.exp(-((X - xc) ** 2 + (Y - yc) ** 2) / (2.0 * width * width))
    B = np.zeros((3, n * n))
    B[0] = ((Y - yc) * f).ravel()
    B[1] = (-(X - xc) * f).ravel()
    return B
