"""Pins of the pseudo-spectral comparison solver and of the spectral divergence
error (test infrastructure, CPU only).

The paper validates its lattice-BGK scheme against a pseudo-spectral Maxwell
code (Subsection "Heterogeneous media") and measures div B with the spectral
error of eq. error.def.  oracle/ps_maxwell.py re-implements both; the checks
here fix them against closed forms, independently of the lattice code:

* A resolved Fourier mode has an exact spectral derivative, so for a plane
  wave the solver is the linear ODE y' = -i w y of the travelling eigenmode
  (w^2 = |k|^2 / (eps mu)), and N classical RK4 steps of size dt multiply it
  by R(z)^N with the RK4 stability polynomial R(z) = 1 + z + z^2/2 + z^3/6 +
  z^4/24, z = -i w dt.  The result is known to rounding: a wrong curl sign,
  a lost mu or eps, a degraded Runge-Kutta stage or a wrong direction of
  travel all move it by far more than 1e-12.
* Nyquist modes: the solver drops the derivative of the Nyquist wavenumber
  on even grids, so such a field is static.
* A uniform current in a uniform box: dE/dt = -j amp(t)/eps, and RK4 is
  Simpson's rule on that ODE, exact for a cubic amplitude.
* eq. error.def with F = 1: closed forms for single and mixed modes.
"""
import numpy as np
import pytest

from oracle import ps_maxwell as PS


def rk4_factor(z):
    return 1.0 + z + z * z / 2.0 + z ** 3 / 6.0 + z ** 4 / 24.0


def coords(shape):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def plane_wave(shape, m, e, eps, mu):
    """E = e cos(k.x), B = (k x e)/w cos(k.x), k = 2 pi m / (nx, ny, nz)."""
    k = 2.0 * np.pi * np.asarray(m, float) / np.asarray(shape, float)
    w = np.linalg.norm(k) / np.sqrt(eps * mu)
    x, y, z = coords(shape)
    ph = k[0] * x + k[1] * y + k[2] * z
    e = np.asarray(e, float)
    b = np.cross(k, e) / w
    return k, w, ph, e, b


@pytest.mark.parametrize("case", [
    dict(shape=(24, 20, 1), m=(2, 3, 0), e=(0, 0, 1), eps=2.5, mu=1.0),
    dict(shape=(24, 20, 1), m=(-5, 1, 0), e=(0, 0, 1), eps=1.5, mu=1.7),
    dict(shape=(12, 10, 8), m=(1, 2, 1), e=None, eps=2.5, mu=1.3),
    dict(shape=(12, 10, 8), m=(3, 0, -2), e=None, eps=1.0, mu=1.0),
])
@pytest.mark.parametrize("substeps", [4, 10])
def test_ps_plane_wave_is_rk4_of_the_eigenmode(case, substeps):
    shape, m, eps, mu = case["shape"], case["m"], case["eps"], case["mu"]
    k = 2.0 * np.pi * np.asarray(m, float) / np.asarray(shape, float)
    e = case["e"]
    if e is None:                                   # a polarisation normal to k
        e = np.cross(k, (0.3, -0.2, 1.0))
        e = e / np.linalg.norm(e)
    k, w, ph, e, b = plane_wave(shape, m, e, eps, mu)
    n = ph.size
    E0 = np.outer(e, np.cos(ph))
    B0 = np.outer(b, np.cos(ph))
    T = 7.0
    ps = PS.PSMaxwell(shape, np.full(n, eps), None if mu == 1.0 else np.full(n, mu))
    E, B = ps.run(E0, B0, T, substeps=substeps)
    N = int(round(T * substeps))
    R = rk4_factor(-1j * w * (T / N)) ** N
    want = np.real(R * np.exp(1j * ph))
    scale = max(np.abs(e).max(), np.abs(b).max())
    assert np.abs(E - np.outer(e, want)).max() < 1e-12 * scale
    assert np.abs(B - np.outer(b, want)).max() < 1e-12 * scale
    # R^N is the continuum phase exp(-i w T) to RK4 accuracy (global error
    # below N (w dt)^5 / 100): the wave travels along +k, where a curl of the
    # wrong sign would send it the other way
    wdt = w * T / N
    assert abs(R - np.exp(-1j * w * T)) < N * wdt ** 5 / 100
    assert abs(R - np.exp(1j * w * T)) > 10 * abs(R - np.exp(-1j * w * T))


def test_ps_nyquist_modes_are_static():
    shape = (16, 12, 1)
    x, y, _ = coords(shape)
    n = x.size
    E0 = np.zeros((3, n))
    E0[2] = np.cos(np.pi * x) + 0.5 * np.cos(np.pi * y)      # Nyquist along x and along y
    B0 = np.zeros((3, n))
    B0[1] = 0.25 * np.cos(np.pi * x)
    E, B = PS.PSMaxwell(shape, np.full(n, 2.0)).run(E0, B0, 5.0, substeps=4)
    assert np.abs(E - E0).max() < 1e-13 and np.abs(B - B0).max() < 1e-13


def test_ps_uniform_current_follows_simpson():
    shape = (8, 6, 4)
    n = 8 * 6 * 4
    eps = 3.0
    j = np.zeros((3, n))
    j[1] = 0.7
    amp = lambda t: 1.0 + t - 2.0 * t * t + 0.5 * t ** 3
    T = 3.0
    E, B = PS.PSMaxwell(shape, np.full(n, eps)).run(np.zeros((3, n)), np.zeros((3, n)), T, substeps=3,
                                                     j=j, amp=amp)
    integral = T + T ** 2 / 2 - 2 * T ** 3 / 3 + 0.5 * T ** 4 / 4
    want = -0.7 * integral / eps
    assert np.abs(E[1] - want).max() < 1e-13 * abs(want)
    assert np.abs(E[0]).max() == 0.0 and np.abs(E[2]).max() == 0.0
    assert np.abs(B).max() < 1e-14


def _unit_box_field(shape, comps):
    """comps: per component a function of physical coordinates (x, y, z) in [0,1)."""
    nx, ny, nz = shape
    x, y, z = coords(shape)
    X, Y, Z = x / nx, y / ny, z / max(nz, 1)
    return np.stack([f(X, Y, Z) for f in comps])


def test_divb_error_closed_forms():
    s2 = (32, 32, 1)
    c2p = 2.0 * np.pi
    zero = lambda X, Y, Z: np.zeros_like(X)
    # solenoidal: B_x depends on y only, B_y on x only
    B = _unit_box_field(s2, [lambda X, Y, Z: np.sin(c2p * 2 * Y), lambda X, Y, Z: np.cos(c2p * 3 * X), zero])
    assert PS.divb_spectral_error(B, s2) < 1e-14
    # one mode, both components: |k . B| / |B| = 2 pi m |a| / sqrt(a^2 + b^2)
    a, b, m = 0.6, -1.7, 3
    B = _unit_box_field(s2, [lambda X, Y, Z: a * np.cos(c2p * m * X), lambda X, Y, Z: b * np.cos(c2p * m * X), zero])
    want = c2p * m * abs(a) / np.hypot(a, b)
    assert abs(PS.divb_spectral_error(B, s2) - want) < 1e-12 * want
    # two modes of different weight: the sums are of magnitudes, not squares
    m1, m2 = 2, 5
    B = _unit_box_field(s2, [lambda X, Y, Z: np.cos(c2p * m1 * X) + 3 * np.cos(c2p * m2 * X), zero, zero])
    want = c2p * (m1 + 3 * m2) / 4.0
    assert abs(PS.divb_spectral_error(B, s2) - want) < 1e-12 * want
    # 3D, a z-mode of B_z on a non-cubic box (wavenumber in units of the box)
    s3 = (8, 12, 16)
    B = _unit_box_field(s3, [zero, zero, lambda X, Y, Z: np.sin(c2p * 3 * Z)])
    assert abs(PS.divb_spectral_error(B, s3) - c2p * 3) < 1e-12 * c2p * 3
