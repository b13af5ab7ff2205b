"""Anisotropic media (per-axis weights, plain formats) on the GPU through the
C ABI: parity with the oracle on heterogeneous permittivity and anisotropy
with every other term present, the birefringent wave speeds, and the call
rules."""
import numpy as np
import pytest

from gpu_util import announce, random_problem, rel
from oracle import oracle as O
from paper_1108_2651_amd import lbem
from test_gpu_parity import TOL
from test_oracle_dispersion_ade import pencil

pytestmark = pytest.mark.gpu

CASES = [(2, (70, 33, 1), False, []), (2, (48, 40, 1), True, [(1, "pec")]), (3, (19, 13, 11), True, []),
         (3, (16, 12, 10), False, [(0, "pmc")])]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dim,shape,mu,walls", CASES)
def test_anisotropy_matches_oracle(dim, shape, mu, walls, prec):
    steps = 70
    p = random_problem(dim, shape, seed=sum(shape) + 5, mu=mu, nsteps=steps)
    rng = np.random.default_rng(sum(shape))
    eps = rng.uniform(1.5, 5.0, p.n)
    fac = rng.uniform(0.6, 1.4, (dim, p.n))
    s = lbem.Solver(dim, shape, prec, mu_varies=mu, streaming="pull")
    o = O.Oracle(dim, shape)
    for a, k in walls:
        s.set_boundary(a, k)
        o.set_boundary(a, k)
    for x in (s, o):
        x.set_medium(eps, p.mu_r)
        x.set_anisotropy(fac)
        x.init_fields(p.E0, p.B0)
        x.set_source(p.src_comp, p.src_cells, p.src_weights)
    assert s.steps_per_launch == 1
    s.step(steps, p.amp[:steps])
    o.step(steps, p.amp[:steps])
    (Eg, Bg), (Eo, Bo) = s.moments(), o.fields()
    eE, eB = rel(Eg, Eo), rel(Bg, Bo)
    announce(f"anisotropy {dim}D {shape} mu={mu} walls={walls} {prec}: E {eE:.2e} B {eB:.2e}")
    assert eE <= TOL[prec] and eB <= TOL[prec], (eE, eB)
    dg, do = s.energy(), o.diag()
    for k in ("energy", "qc", "divb2", "b2"):
        assert abs(dg[k] - do[k]) <= (1e-11 if prec == "f64" else 2e-5) * abs(do[k]), k
    s.close()


@pytest.mark.parametrize("pol", [1, 2])
def test_birefringent_speeds_on_gpu(pol):
    nx, fac = 128, (1.3, 0.8, 0.6)
    k = 2 * np.pi * 2 / nx
    s = lbem.Solver(3, (nx, 2, 2), "f64", streaming="pull")
    s.set_medium(np.ones(s.n))
    s.set_anisotropy(np.asarray(fac)[:, None] * np.ones((3, s.n)))
    E0 = np.zeros((3, s.n))
    E0[pol] = np.cos(k * (np.arange(s.n) % nx))
    s.init_fields(E0, np.zeros_like(E0))
    ys = [s.moments()[0][pol, 0]]
    for _ in range(3 * nx):
        s.step(1)
        ys.append(s.moments()[0][pol, 0])
    z = pencil(np.array(ys), 4)
    w = np.abs(np.angle(z[np.abs(np.abs(z) - 1) < 1e-8])).min()
    sx, sb = np.array(fac)[[0, pol]] * (2.0 / 3.0) / 3.0
    want = sx * sx / (sx + sb)
    announce(f"wave along x polarised {pol}: c^2 {(w / k) ** 2:.6f} vs {want:.6f}")
    assert abs((w / k) ** 2 - want) / want < 2e-3


def test_anisotropy_call_rules():
    n = 8 * 8 * 8
    for prec in ("f16dev", "f16ghost"):
        d = lbem.Solver(3, (8, 8, 8), prec)
        d.set_medium(np.ones(n))
        with pytest.raises(lbem.LbemError) as e:
            d.set_anisotropy(np.ones((3, n)))      # plain formats only
        assert e.value.code == lbem.LBEM_EINVAL
        d.close()
    s = lbem.Solver(3, (8, 8, 8), "f32", streaming="pull")
    with pytest.raises(lbem.LbemError) as e:
        s.set_anisotropy(np.ones((3, n)))          # before the medium
    assert e.value.code == lbem.LBEM_ESTATE
    s.set_medium(np.full(n, 2.0))
    bad = np.ones((3, n))
    bad[:, 5] = 20.0                               # negative rest weight in one cell
    with pytest.raises(lbem.LbemError) as e:
        s.set_anisotropy(bad)
    assert e.value.code == lbem.LBEM_EUNSTABLE
    # the rejected call changed nothing: the box is still the isotropic one
    rng = np.random.default_rng(2)
    E = rng.standard_normal((3, n))
    B = rng.standard_normal((3, n))
    s.init_fields(E, B)
    s.step(10)
    iso = lbem.Solver(3, (8, 8, 8), "f32", streaming="pull")
    iso.set_medium(np.full(n, 2.0))
    iso.init_fields(E, B)
    iso.step(10)
    assert all(np.array_equal(x, y) for x, y in zip(s.moments(), iso.moments()))
    for x in (s, iso):
        x.close()
