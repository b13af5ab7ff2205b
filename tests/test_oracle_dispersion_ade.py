"""Pins of the oracle's frequency-dispersive permittivity (one Lorentz pole
per cell, auxiliary differential equations for the convolution term of the
source in the Maxwell section).

Physics fixes what the discrete scheme must approach:
* a uniform field (k = 0) in a Lorentz medium oscillates at
  Omega = sqrt(w0^2 + wp^2) about D wp^2/Omega^2 below its start value D
  (Drude, w0 = 0: the plasma oscillation at wp), decaying at gamma/2;
* a standing wave cos(kx) splits into the two polariton branches, the roots
  of w^4 - w^2 (w0^2 + wp^2 + c^2 k^2) + c^2 k^2 w0^2 = 0.
Both are met to second order in the lattice spacing: halving k and the pole
frequencies (a twice finer lattice for the same physical problem) divides
the frequency errors by about four.  A sign or factor slip in the auxiliary
update (a dropped 1/2, an uncentred source, a flipped coupling) breaks the
order, the amplitude or the frequencies themselves.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1108_2651_amd import inputs

C2 = inputs.vacuum_speed(2, 1.0 / 3.0) ** 2


def pencil(y, m):
    """Matrix-pencil estimate of the m complex exponentials in y[t]."""
    n = len(y)
    L = n // 2
    Y = np.array([y[i:i + L + 1] for i in range(n - L)])
    _, _, Vt = np.linalg.svd(Y, full_matrices=False)
    V = Vt[:m].T
    return np.linalg.eigvals(np.linalg.pinv(V[:-1]) @ V[1:])


def series(nx, E0, steps, wp2, w02, gamma, probe=0, dim=2, comp=2):
    o = O.Oracle(dim, (nx, 1, 1))
    o.set_medium(np.ones(nx))
    o.set_dispersion(wp2, w02, gamma)
    o.init_fields(E0, np.zeros((3, nx)))
    out = [o.fields()[0][comp, probe]]
    for _ in range(steps):
        o.step(1)
        out.append(o.fields()[0][comp, probe])
    return np.array(out)


@pytest.mark.parametrize("w02_over", [0.0, 0.6])
def test_uniform_oscillation(w02_over):
    """k = 0: frequency, offset, amplitude and decay against the closed form."""
    errs = []
    for scale in (1.0, 0.5, 0.25):
        Om = 0.2 * scale
        w02 = w02_over * Om ** 2
        wp2 = Om ** 2 - w02
        nx = 4
        E0 = np.zeros((3, nx))
        E0[2] = 1.0
        y = series(nx, E0, int(40 / Om), wp2, w02, 0.0)
        z = pencil(y, 3)                                          # offset (if any) + the oscillation
        z = z[np.abs(z.imag) > 1e-6]                              # the conjugate pair
        assert len(z) == 2
        wd = np.abs(np.angle(z)).max()
        assert np.allclose(np.abs(z), 1.0, atol=1e-9)            # lossless without gamma
        errs.append(abs(wd - Om) / Om)
        r = wp2 / Om ** 2
        # offset D (1 - r) and swing D r, to the same second order
        assert abs((y.max() + y.min()) / 2 - (1 - r)) < 0.1 * Om ** 2 + 2e-3 * scale
        assert abs((y.max() - y.min()) / 2 - r) < 0.1 * Om ** 2 + 2e-3 * scale
    assert errs[0] < 0.01
    assert 3.3 < errs[0] / errs[1] < 4.7 and 3.3 < errs[1] / errs[2] < 4.7, errs


def test_uniform_oscillation_3d_components():
    """k = 0 in 3D: each E component is its own plasma oscillator."""
    Om = 0.1
    nx = 4
    E0 = np.zeros((3, nx))
    E0[:, :] = np.array([1.0, -2.0, 0.5])[:, None]
    for comp in range(3):
        y = series(nx, E0, int(40 / Om), Om ** 2, 0.0, 0.0, dim=3, comp=comp)
        z = pencil(y, 3)
        z = z[np.abs(z.imag) > 1e-6]
        assert len(z) == 2 and np.allclose(np.abs(z), 1.0, atol=1e-9)
        assert abs(np.abs(np.angle(z)).max() - Om) / Om < 0.002
        assert abs(np.abs(y).max() - abs(E0[comp, 0])) < 2e-3 * abs(E0[comp, 0])


def test_uniform_damping_rate():
    Om, gamma = 0.05, 0.004
    nx = 4
    E0 = np.zeros((3, nx))
    E0[2] = 1.0
    y = series(nx, E0, 3000, Om ** 2, 0.0, gamma)
    z = pencil(y, 3)
    osc = z[np.argmax(z.imag)]
    rate = -np.log(np.abs(osc))
    assert abs(rate - gamma / 2) < 0.02 * gamma / 2
    # the polarisation is kept by the oracle and settles with the field
    o = O.Oracle(2, (nx, 1, 1))
    o.set_medium(np.ones(nx))
    o.set_dispersion(Om ** 2, 0.0, gamma)
    o.init_fields(E0, np.zeros((3, nx)))
    o.step(3000)
    P, J = o.polarisation()
    E = o.fields()[0]
    assert abs(E[2, 0] + P[2, 0] - 1.0) < 1e-2            # displacement E + P stays ~ D


@pytest.mark.parametrize("dim,comp", [(2, 2), (3, 1), (3, 2)])
def test_polariton_branches_second_order(dim, comp):
    """Standing transverse wave along x (E_z in 2D; E_y or E_z in 3D)."""
    c2 = inputs.vacuum_speed(dim, 1.0 / 3.0) ** 2
    errs = []
    for scale in (1.0, 0.5, 0.25):
        nx = int(round(64 / scale))
        k = 2 * np.pi * 2 / nx
        w02, wp2 = (0.12 * scale) ** 2, (0.10 * scale) ** 2
        x = np.arange(nx)
        E0 = np.zeros((3, nx))
        E0[comp] = np.cos(k * x)
        y = series(nx, E0, int(60 / (0.1 * scale)), wp2, w02, 0.0, dim=dim, comp=comp)
        z = pencil(y, 6)
        w = np.sort(np.unique(np.round(np.abs(np.angle(z[np.abs(np.abs(z) - 1) < 1e-6])), 12)))
        c2k2 = c2 * k * k
        b = w02 + wp2 + c2k2
        roots = np.sqrt([(b - np.sqrt(b * b - 4 * c2k2 * w02)) / 2, (b + np.sqrt(b * b - 4 * c2k2 * w02)) / 2])
        got = np.array([w[np.argmin(np.abs(w - r))] for r in roots])
        errs.append(np.abs(got - roots) / roots)
    errs = np.array(errs)
    assert errs[0].max() < 0.02
    ratio = errs[:-1] / errs[1:]
    assert np.all((ratio > 3.3) & (ratio < 4.7)), (errs, ratio)


def test_zero_pole_is_the_plain_scheme():
    nx, ny = 24, 10
    rng = np.random.default_rng(4)
    eps = rng.uniform(1, 3, nx * ny)
    E = np.zeros((3, nx * ny))
    E[2] = rng.standard_normal(nx * ny)
    B = np.zeros((3, nx * ny))
    B[:2] = rng.standard_normal((2, nx * ny))
    runs = []
    for disp in (False, True):
        o = O.Oracle(2, (nx, ny, 1))
        o.set_medium(eps)
        if disp:
            o.set_dispersion(0.0, 0.3, 0.1)       # no coupling: wp2 = 0
        o.init_fields(E, B)
        o.step(40)
        runs.append(o.fields())
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
