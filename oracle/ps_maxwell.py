"""Pseudo-spectral Maxwell solver (independent physics reference).

TEST INFRASTRUCTURE ONLY.  The paper validates its lattice-BGK scheme against
a pseudo-spectral code (spectral spatial derivatives, Runge-Kutta in time;
Section "Heterogeneous media").  This is an independent numpy
re-implementation of that comparison solver: it integrates the continuum
Maxwell system of the Maxwell section directly,

    dB/dt = -curl E
    dE/dt = (1/eps_abs) (curl (B/mu_r) - j(x, t))

on a periodic box with unit grid spacing, spectral derivatives (Nyquist
mode dropped) and classical RK4 with ``substeps`` RK steps per lattice time
unit.  It shares nothing with the lattice code: no populations, no weights.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft


class PSMaxwell:
    def __init__(self, shape, eps_abs, mu_r=None):
        """shape = (nx, ny, nz) (nz = 1 for 2D); eps_abs, mu_r as (n,) arrays."""
        nx, ny, nz = shape
        self.dim = 2 if nz == 1 else 3
        self.grid = (nz, ny, nx) if self.dim == 3 else (ny, nx)
        self.eps = np.asarray(eps_abs, np.float64).reshape(self.grid)
        self.mu = None if mu_r is None else np.asarray(mu_r, np.float64).reshape(self.grid)
        ks = []
        for ax, m in enumerate(self.grid):
            # last axis uses the real-to-complex half spectrum
            k = 2.0 * np.pi * (np.fft.rfftfreq(m) if ax == len(self.grid) - 1 else np.fft.fftfreq(m))
            if m % 2 == 0:
                k[np.isclose(np.abs(k), np.pi)] = 0.0  # drop the Nyquist derivative
            ks.append(k)
        kk = np.meshgrid(*ks, indexing="ij")
        # derivative operators along x, y, z (array axes are reversed)
        if self.dim == 2:
            self.ik = [1j * kk[1], 1j * kk[0], None]
        else:
            self.ik = [1j * kk[2], 1j * kk[1], 1j * kk[0]]

    def curl(self, F):
        g = self.grid
        # identically-zero components (e.g. the TE half of a 2D TM run) are skipped
        Fk = [sfft.rfftn(F[c], workers=-1) if F[c].any() else None for c in range(3)]
        ik = self.ik

        def d(c, axis):
            return None if (ik[axis] is None or Fk[c] is None) else Fk[c] * ik[axis]

        def comb(a, b):
            if a is None and b is None:
                return np.zeros(g)
            if b is None:
                return sfft.irfftn(a, s=g, workers=-1)
            if a is None:
                return -sfft.irfftn(b, s=g, workers=-1)
            return sfft.irfftn(a - b, s=g, workers=-1)

        return np.stack([comb(d(2, 1), d(1, 2)), comb(d(0, 2), d(2, 0)), comb(d(1, 0), d(0, 1))])

    def rhs(self, E, B, jt):
        H = B if self.mu is None else B / self.mu
        dE = (self.curl(H) - jt) / self.eps
        dB = -self.curl(E)
        return dE, dB

    def run(self, E0, B0, t_end: float, substeps: int = 10, j=None, amp=None):
        """Integrate from t=0 to t_end (lattice time units).

        j: (3, n) current footprint or None; amp: callable amp(t) (continuous
        time) scaling the footprint.  Returns (E, B) as (3, n)."""
        g = self.grid
        E = np.asarray(E0, np.float64).reshape((3,) + g).copy()
        B = np.asarray(B0, np.float64).reshape((3,) + g).copy()
        jf = None if j is None else np.asarray(j, np.float64).reshape((3,) + g)
        nsub = int(round(t_end * substeps))
        dt = t_end / nsub if nsub else 0.0

        def jat(t):
            if jf is None:
                return 0.0
            return jf * (amp(t) if amp is not None else 1.0)

        t = 0.0
        for _ in range(nsub):
            k1 = self.rhs(E, B, jat(t))
            k2 = self.rhs(E + 0.5 * dt * k1[0], B + 0.5 * dt * k1[1], jat(t + 0.5 * dt))
            k3 = self.rhs(E + 0.5 * dt * k2[0], B + 0.5 * dt * k2[1], jat(t + 0.5 * dt))
            k4 = self.rhs(E + dt * k3[0], B + dt * k3[1], jat(t + dt))
            E = E + dt / 6.0 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0])
            B = B + dt / 6.0 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
            t += dt
        return E.reshape(3, -1), B.reshape(3, -1)


def divb_spectral_error(B, shape):
    """Spectral divergence error of eq. error.def with the unit kernel F = 1,
    for a periodic field B on the unit box (physical wavenumbers 2 pi m):

        eps = sum_k |i k . B(k)| / sum_k |B(k)|,   |B(k)| = sqrt(sum_c |B_c(k)|^2)

    (the paper's kernel width is unspecified; F = 1 is the choice every use
    here makes).  B is (>= dim, n); only the in-lattice components enter."""
    nx, ny, nz = shape
    dim = 2 if nz == 1 else 3
    grid = (ny, nx) if dim == 2 else (nz, ny, nx)
    Bk = [np.fft.fftn(np.asarray(B[c]).reshape(grid)) for c in range(dim)]
    ms = [np.fft.fftfreq(m) * m for m in grid]
    mm = np.meshgrid(*ms, indexing="ij")
    # component order x, y, (z) matches reversed array axes
    kv = [2.0 * np.pi * mm[dim - 1 - c] for c in range(dim)]
    div = np.abs(sum(1j * kv[c] * Bk[c] for c in range(dim)))
    mag = np.sqrt(sum(np.abs(Bk[c]) ** 2 for c in range(dim)))
    den = np.sum(mag)
    return float(np.sum(div) / den) if den > 0 else 0.0
