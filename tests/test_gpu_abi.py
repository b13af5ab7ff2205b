"""Error paths of the C ABI on a GPU (all conditions forced from the host; no
kernel is made to fault)."""
import numpy as np
import pytest

from gpu_util import announce, random_problem
from paper_1108_2651_amd import lbem

pytestmark = pytest.mark.gpu


def test_call_order_and_argument_errors():
    announce("abi errors")
    s = lbem.Solver(2, (16, 8, 1), "f32")
    n = s.n
    with pytest.raises(lbem.LbemError) as e:
        s.step(1)
    assert e.value.code == lbem.LBEM_ESTATE
    with pytest.raises(lbem.LbemError) as e:
        s.init_fields(np.zeros((3, n)), np.zeros((3, n)))
    assert e.value.code == lbem.LBEM_ESTATE
    # eps*mu below 1 - w0_vac: rest weight negative
    with pytest.raises(lbem.LbemError) as e:
        s.set_medium(np.full(n, 0.5))
    assert e.value.code == lbem.LBEM_EUNSTABLE
    with pytest.raises(lbem.LbemError) as e:
        s.set_medium(np.full(n, np.nan))
    assert e.value.code == lbem.LBEM_EUNSTABLE
    # non-uniform mu without mu_varies
    with pytest.raises(lbem.LbemError) as e:
        s.set_medium(np.ones(n), np.linspace(1, 2, n))
    assert e.value.code == lbem.LBEM_EINVAL
    s.set_medium(np.ones(n))
    # 2D is TM only
    E = np.zeros((3, n)); E[0, 3] = 1.0
    with pytest.raises(lbem.LbemError) as e:
        s.init_fields(E, np.zeros((3, n)))
    assert e.value.code == lbem.LBEM_EINVAL
    with pytest.raises(lbem.LbemError) as e:
        s.set_source(0, [1], [1.0])
    assert e.value.code == lbem.LBEM_EINVAL
    with pytest.raises(lbem.LbemError) as e:
        s.set_source(2, [n], [1.0])
    assert e.value.code == lbem.LBEM_EINVAL
    s.init_fields(np.zeros((3, n)), np.zeros((3, n)))
    s.step(3)
    assert s.t == 3
    s.close()


def test_nonfinite_detected_by_energy():
    announce("nonfinite")
    p = random_problem(2, (24, 16, 1), seed=1, nsteps=4)
    s = lbem.Solver(2, p.shape, "f64")
    s.setup(p)
    s.step(2, [1.0, np.inf])
    d = s.energy(check=False)
    assert d["status"] == lbem.LBEM_ENONFINITE
    s.close()


def test_arena_and_streams():
    """Two handles on two torch streams advance independently."""
    import torch
    announce("two streams")
    p = random_problem(3, (12, 10, 8), seed=2, nsteps=20)
    s1 = lbem.Solver(3, p.shape, "f32", stream=torch.cuda.Stream())
    s2 = lbem.Solver(3, p.shape, "f32", stream=torch.cuda.Stream())
    s1.setup(p)
    s2.setup(p)
    s1.step(20, p.amp)
    s2.step(10, p.amp)
    s2.step(10, p.amp[10:])
    a, b = s1.moments(), s2.moments()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
