"""lbem_energy_noalloc (static device scratch, no allocation) against
lbem_energy (handle scratch): the same kernels in the same order, so the four
FP64 diagnostics agree bit for bit.  Two calls in a row on two handles, the
second lattice smaller than the first (the static array keeps the first
call's contents), then a lattice above the static limit, rejected before any
work is enqueued."""
import numpy as np
import pytest

from gpu_util import announce, gpu_run, random_problem

pytestmark = pytest.mark.gpu


def _same(a, b):
    return all(a[k] == b[k] for k in ("energy", "qc", "divb2", "b2"))


@pytest.mark.parametrize("prec", ["f64", "f32", "f16ghost"])
def test_noalloc_energy_matches_energy(prec):
    from paper_1108_2651_amd import lbem
    big = random_problem(3, (40, 24, 20), seed=201, mu=False, nsteps=9)
    small = random_problem(2, (30, 18, 1), seed=202, mu=False, nsteps=9)
    for p in (big, small, big):
        announce(f"noalloc energy {prec} {p.shape}")
        s = gpu_run(p, 9, prec)
        ref = s.energy()
        got = s.energy_noalloc()
        assert got["status"] == lbem.LBEM_OK
        assert _same(ref, got), (ref, got)
        s.step(4, p.amp[:4])
        assert _same(s.energy(), s.energy_noalloc())
        s.close()


def test_noalloc_energy_rejects_lattices_above_the_limit():
    from paper_1108_2651_amd import lbem
    n = 1680                                   # 1680^2 = 2822400 > LBEM_NOALLOC_MAX_CELLS
    assert n * n > lbem.NOALLOC_MAX_CELLS
    s = lbem.Solver(2, (n, n, 1), "f32")
    s.set_medium(np.full(n * n, 2.0))
    E = np.zeros((3, n * n))
    E[2, :: 97] = 1.0
    s.init_fields(E, np.zeros((3, n * n)))
    r = s.energy_noalloc(check=False)
    assert r["status"] == lbem.LBEM_ETOOBIG
    assert s.energy()["energy"] > 0              # the handle still works
    s.close()
