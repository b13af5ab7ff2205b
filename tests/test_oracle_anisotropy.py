"""Pins of the oracle's anisotropic media (per-axis weights of the moving
particles, as the lattice section suggests).

* Uniform factors f on the isotropic c_L^2 of permittivity eps are the
  isotropic scheme for permittivity eps/f (the same lattice speed and the
  same eps_abs); factors of one are the isotropic scheme itself.
* Wave speeds: along axis a a standing wave travels at c^2 = s_a in 2D and,
  in 3D, at s_a^2/(s_a + s_b) when polarised along b (s_a = 2 w_a, the
  per-axis second moment) -- the continuum limit of the scheme with the
  K-conserving Bbar -- reached at second order in the lattice spacing.
* The equilibrium is the orthogonal projection onto the conserved moments in
  the 1/w_i inner product, so with uniform anisotropy ratios Q_c is an exact
  invariant even in a heterogeneous medium.
"""
import numpy as np
import pytest

from oracle import oracle as O
from test_oracle_dispersion_ade import pencil


def random_fields(dim, n, rng):
    E = np.zeros((3, n))
    B = np.zeros((3, n))
    if dim == 2:
        E[2] = rng.standard_normal(n)
        B[:2] = rng.standard_normal((2, n))
    else:
        E[:] = rng.standard_normal((3, n))
        B[:] = rng.standard_normal((3, n))
    return E, B


@pytest.mark.parametrize("dim,shape", [(2, (20, 14, 1)), (3, (10, 8, 7))])
def test_uniform_factors_are_the_isotropic_scheme(dim, shape):
    rng = np.random.default_rng(31 + dim)
    n = int(np.prod(shape))
    eps = rng.uniform(1.5, 4.0, n)
    mu = rng.uniform(0.9, 1.2, n)
    E, B = random_fields(dim, n, rng)
    for kappa in (1.0, 0.8):
        a = O.Oracle(dim, shape)
        a.set_medium(eps, mu)
        a.set_anisotropy(np.full((dim, n), kappa))
        a.init_fields(E, B)
        a.step(30)
        b = O.Oracle(dim, shape)
        b.set_medium(eps / kappa, mu)
        b.init_fields(E, B)
        b.step(30)
        for x, y in zip(a.fields(), b.fields()):
            assert np.abs(x - y).max() <= 1e-13 * np.abs(y).max()
        np.testing.assert_allclose(a.diag()["energy"], b.diag()["energy"], rtol=1e-13)


def standing_wave_speed2(dim, nx, axis, pol, fac, steps):
    shape = [1, 1, 1]
    shape[axis] = nx
    n = nx
    k = 2 * np.pi * 2 / nx
    o = O.Oracle(dim, tuple(shape))
    o.set_medium(np.ones(n))
    o.set_anisotropy(np.asarray(fac, np.float64)[:, None] * np.ones((dim, n)))
    E = np.zeros((3, n))
    E[pol] = np.cos(k * np.arange(nx))
    o.init_fields(E, np.zeros((3, n)))
    ys = [o.fields()[0][pol, 0]]
    for _ in range(steps):
        o.step(1)
        ys.append(o.fields()[0][pol, 0])
    z = pencil(np.array(ys), 4)
    z = z[np.abs(np.abs(z) - 1) < 1e-8]
    w = np.abs(np.angle(z)).min()
    return (w / k) ** 2


@pytest.mark.parametrize("dim,axis,pol,fac", [
    (2, 0, 2, (1.4, 0.6)), (2, 1, 2, (1.4, 0.6)),
    (3, 0, 1, (1.3, 0.8, 0.6)), (3, 0, 2, (1.3, 0.8, 0.6)), (3, 2, 0, (1.3, 0.8, 0.6))])
def test_axis_speeds_second_order(dim, axis, pol, fac):
    cl2_iso = (1.0 - 1.0 / 3.0) / dim              # eps = mu = 1
    s = np.array(fac) * cl2_iso                     # per-axis second moments
    if dim == 2:
        want = s[axis]
    else:
        want = s[axis] ** 2 / (s[axis] + s[pol])
    errs = []
    for nx in (32, 64, 128):
        got = standing_wave_speed2(dim, nx, axis, pol, fac, steps=3 * nx)
        errs.append(abs(got - want) / want)
    assert errs[0] < 0.05
    assert 3.3 < errs[0] / errs[1] < 4.7 and 3.3 < errs[1] / errs[2] < 4.7, errs


@pytest.mark.parametrize("dim,shape,fac", [(2, (24, 18, 1), (1.5, 0.5)), (3, (10, 9, 8), (1.4, 0.9, 0.6))])
def test_qc_invariant_with_uniform_ratios(dim, shape, fac):
    rng = np.random.default_rng(7 + dim)
    n = int(np.prod(shape))
    eps = rng.uniform(1.5, 5.0, n)                   # heterogeneous speed, uniform anisotropy ratios
    E, B = random_fields(dim, n, rng)
    o = O.Oracle(dim, shape)
    o.set_medium(eps)
    o.set_anisotropy(np.asarray(fac)[:, None] * np.ones((dim, n)))
    o.init_fields(E, B)
    q0 = o.diag()["qc"]
    for _ in range(4):
        o.step(40)
        assert abs(o.diag()["qc"] / q0 - 1.0) < 1e-13


def test_unstable_factors_rejected():
    o = O.Oracle(2, (8, 8, 1))
    o.set_medium(np.ones(64))
    with pytest.raises(O.OracleError) as e:
        o.set_anisotropy(np.full((2, 64), 1.6))     # sum_a s_a = 2 * 1.6/3 > 1: negative rest weight
    assert e.value.code == -3
    with pytest.raises(O.OracleError):
        o.set_anisotropy(np.full((2, 64), -1.0))
