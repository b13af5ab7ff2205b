"""Heterogeneous mu on the GPU.  A pulse crossing a slab whose permittivity
and permeability rise together (matched impedance, eps = mu) is not
reflected, while a slab of the same light speed from eps alone is: the
mu-gradient source term carries exactly the impedance information.  The same
runs are checked element-wise against the oracle."""
import numpy as np
import pytest

from gpu_util import announce, rel
from oracle import oracle as O
from paper_1108_2651_amd import inputs, lbem

pytestmark = pytest.mark.gpu

NX = 512
# long enough for the pulse (starting 100 cells before the slab) to reach it
# and for a reflection to come back past x = 180; the 3D light speed is
# 1/sqrt(3) of the 2D one (c_M^2 = c_L^2/(D-1))
STEPS = {2: 330, 3: 570}


def slab_problem(dim, matched):
    ny = 4
    nz = 4 if dim == 3 else 1
    x = np.arange(NX)
    ramp = 0.5 * (np.tanh((x - 200) / 4.0) - np.tanh((x - 400) / 4.0))
    eps1 = 1 + ramp if matched else 1 + 3 * ramp
    mu1 = 1 + ramp if matched else None
    n = NX * ny * nz
    cv = inputs.vacuum_speed(dim, 1.0 / 3.0)
    f = np.exp(-(x - 100.0) ** 2 / (2 * 8.0 ** 2))
    E0 = np.zeros((3, n))
    B0 = np.zeros((3, n))
    E0[2] = np.tile(f, ny * nz)
    B0[1] = -np.tile(f, ny * nz) / cv                  # right-moving plane pulse
    eps = np.tile(eps1, ny * nz)
    mu = None if mu1 is None else np.tile(mu1, ny * nz)
    return (NX, ny, nz), eps, mu, E0, B0


def reflected_fraction(E, B, eps_abs, mu, e0):
    dens = eps_abs * (E ** 2).sum(0) + (B ** 2).sum(0) / (1.0 if mu is None else mu)
    x = np.arange(dens.size) % NX
    return dens[x < 180].sum() / e0


@pytest.mark.parametrize("dim", [2, 3])
def test_matched_slab_gpu(dim):
    refl = {}
    for matched in (False, True):
        shape, eps, mu, E0, B0 = slab_problem(dim, matched)
        o = O.Oracle(dim, shape)
        o.set_medium(eps, mu)
        o.init_fields(E0, B0)
        e0 = o.diag()["energy"]
        ea = o.medium()["eps_abs"]
        o.step(STEPS[dim])
        Eo, Bo = o.fields()
        for prec in ("f64", "f32", "f16dev", "f16ghost"):
            s = lbem.Solver(dim, shape, prec, mu_varies=mu is not None)
            s.set_medium(eps, mu)
            s.init_fields(E0, B0)
            s.step(STEPS[dim])
            E, B = s.moments()
            r = reflected_fraction(E, B, ea, mu, e0)
            eE, eB = rel(E, Eo), rel(B, Bo)
            announce(f"{dim}D slab matched={matched} {prec}: reflected {r:.2e}, vs oracle E {eE:.1e} B {eB:.1e}")
            tol = {"f64": 1e-12, "f32": 1e-5}.get(prec, 1e-3)
            assert eE <= tol and eB <= tol, (prec, eE, eB)
            refl[(matched, prec)] = r
            s.close()
    for prec in ("f64", "f32", "f16dev", "f16ghost"):
        assert refl[(False, prec)] > 0.03
        assert refl[(True, prec)] < 1e-4
