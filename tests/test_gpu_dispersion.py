"""Frequency-dispersive permittivity (one Lorentz pole per cell, auxiliary
differential equations) on the GPU through the C ABI: parity with the oracle
on seeded inputs with every other term present, the polariton frequencies of
a standing wave against the continuum dispersion relation, and exact resume
of the auxiliary fields."""
import numpy as np
import pytest

from gpu_util import announce, random_problem, rel
from oracle import oracle as O
from paper_1108_2651_amd import inputs, lbem
from test_gpu_parity import TOL, energy_norm_error, white_noise_bar
from test_oracle_dispersion_ade import pencil

pytestmark = pytest.mark.gpu


def poles(n, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 0.02, n), rng.uniform(0, 0.03, n), rng.uniform(0, 0.01, n)


CASES = [(2, (70, 33, 1), False, []), (2, (48, 40, 1), True, [(0, "pec")]), (3, (19, 13, 11), True, []),
         (3, (16, 12, 10), False, [(2, "pmc")])]


@pytest.mark.parametrize("prec", ["f64", "f32", "f16dev", "f16ghost"])
@pytest.mark.parametrize("dim,shape,mu,walls", CASES)
def test_dispersion_matches_oracle(dim, shape, mu, walls, prec):
    steps = 80
    p = random_problem(dim, shape, seed=sum(shape) + 3, mu=mu, nsteps=steps)
    wp2, w02, gam = poles(p.n, sum(shape))
    s = lbem.Solver(dim, shape, prec, mu_varies=mu, streaming="pull")
    o = O.Oracle(dim, shape)
    for a, k in walls:
        s.set_boundary(a, k)
        o.set_boundary(a, k)
    s.set_medium(p.eps_r, p.mu_r)
    o.set_medium(p.eps_r, p.mu_r)
    s.set_dispersion(wp2, w02, gam)
    o.set_dispersion(wp2, w02, gam)
    s.init_fields(p.E0, p.B0)
    o.init_fields(p.E0, p.B0)
    s.set_source(p.src_comp, p.src_cells, p.src_weights)
    o.set_source(p.src_comp, p.src_cells, p.src_weights)
    assert s.steps_per_launch == 1
    s.step(steps, p.amp[:steps])
    o.step(steps, p.amp[:steps])
    (Eg, Bg), (Eo, Bo) = s.moments(), o.fields()
    eE, eB = rel(Eg, Eo), rel(Bg, Bo)
    eN = energy_norm_error(Eg, Bg, Eo, Bo, o, p.mu_r)
    announce(f"dispersion {dim}D {shape} mu={mu} walls={walls} {prec}: E {eE:.2e} B {eB:.2e} energy {eN:.2e}")
    if prec in ("f64", "f32"):
        assert eE <= TOL[prec] and eB <= TOL[prec], (eE, eB)
    else:
        tol = white_noise_bar(prec, steps)     # white-noise fields
        assert eE <= tol and eB <= tol, (eE, eB, eN)
    s.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dim", [2, 3])
def test_polariton_frequencies_on_gpu(dim, prec):
    nx, ny = 128, 4
    nz = 4 if dim == 3 else 1
    k = 2 * np.pi * 2 / nx
    w02, wp2 = 0.06 ** 2, 0.05 ** 2
    x = np.tile(np.arange(nx), ny * nz)
    E0 = np.zeros((3, nx * ny * nz))
    E0[2] = np.cos(k * x)
    s = lbem.Solver(dim, (nx, ny, nz), prec, streaming="pull")
    s.set_medium(np.ones(s.n))
    s.set_dispersion(wp2, w02)
    s.init_fields(E0, np.zeros_like(E0))
    ys = [s.moments()[0][2, 0]]
    for _ in range(1200):
        s.step(1)
        ys.append(s.moments()[0][2, 0])
    z = pencil(np.array(ys), 6)
    w = np.abs(np.angle(z[np.abs(np.abs(z) - 1) < 1e-5]))
    c2k2 = inputs.vacuum_speed(dim, 1.0 / 3.0) ** 2 * k * k
    b = w02 + wp2 + c2k2
    roots = np.sqrt([(b - np.sqrt(b * b - 4 * c2k2 * w02)) / 2, (b + np.sqrt(b * b - 4 * c2k2 * w02)) / 2])
    got = np.array([w[np.argmin(np.abs(w - r))] for r in roots])
    announce(f"polaritons {dim}D {prec}: {got} vs continuum {roots}")
    assert np.all(np.abs(got - roots) / roots < 5e-3)


def test_dispersion_checkpoint_and_rules():
    p = random_problem(2, (40, 30, 1), seed=8, nsteps=50)
    wp2, w02, gam = poles(p.n, 8)

    def make():
        s = lbem.Solver(2, p.shape, "f32", streaming="pull")
        s.set_medium(p.eps_r)
        s.set_dispersion(wp2, w02, gam)
        s.set_source(p.src_comp, p.src_cells, p.src_weights)
        return s

    a = make()
    a.init_fields(p.E0, p.B0)
    a.step(50, p.amp[:50])
    ref = a.moments()
    b = make()
    b.init_fields(p.E0, p.B0)
    b.step(21, p.amp[:21])
    blob = b.get_state()
    c = make()
    c.set_state(blob)
    c.step(29, p.amp[21:50])
    got = c.moments()
    assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1])
    # a blob without the auxiliary fields does not fit a dispersive handle
    d = lbem.Solver(2, p.shape, "f32", streaming="pull")
    d.set_medium(p.eps_r)
    with pytest.raises(lbem.LbemError) as e:
        d.set_state(blob)
    assert e.value.code == lbem.LBEM_EINVAL
    with pytest.raises(lbem.LbemError) as e:
        d.set_dispersion(-np.ones(d.n))
    assert e.value.code == lbem.LBEM_EINVAL
    aa = lbem.Solver(2, p.shape, "f32", streaming="aa")
    with pytest.raises(lbem.LbemError) as e:
        aa.set_dispersion(0.01)
    assert e.value.code == lbem.LBEM_EINVAL
    for s in (a, b, c, d, aa):
        s.close()
