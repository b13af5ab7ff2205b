"""Error paths and default choices of the C ABI on a GPU (error conditions forced
from the host; no kernel is made to fault)."""
import os

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


@pytest.mark.parametrize("dim,shape", [(2, (1024, 8, 1)), (2, (2048, 4, 1)), (2, (600, 3, 1)),
                                       (3, (600, 4, 3)), (3, (1024, 2, 2)), (3, (1030, 2, 2))])
def test_rows_longer_than_the_row_kernels(dim, shape):
    """Handles whose rows are longer than the whole-row kernels take (512
    cells for the plain one, 1024 for the deviation one) are created, stepped
    and read back in every format: their tilings fall back to the cell-tile
    kernels."""
    from gpu_util import random_problem
    p = random_problem(dim, shape, seed=sum(shape), nsteps=3)
    for prec in ("f64", "f32", "f16", "f16dev", "f16ghost"):
        announce(f"long rows {dim}D {shape} {prec}")
        s = lbem.Solver(dim, shape, prec, streaming="pull")
        s.setup(p)
        s.step(3, p.amp[:3])
        E, B = s.moments()
        assert np.isfinite(E).all() and np.isfinite(B).all()
        s.close()


@pytest.mark.parametrize("shape,spl", [((96, 96, 96), 1), ((112, 112, 112), 2), ((128, 64, 160), 2)])
def test_3d_fp32_size_policy(shape, spl):
    """3D FP32 with automatic streaming runs single AA steps below 1e6 cells
    (Infinity-Cache resident: the fused pair cannot fill the chip) and two
    fused steps per launch from there on; the pair's result equals single
    steps bit for bit."""
    announce(f"fp32 size policy {shape}")
    p = random_problem(3, shape, seed=sum(shape), nsteps=4)
    s = lbem.Solver(3, shape, "f32")
    assert s.steps_per_launch == spl
    s.setup(p)
    s.step(4, p.amp[:4])
    got = s.moments()
    s.close()
    os.environ["LBEM_FUSE3"] = "1"
    try:
        r = lbem.Solver(3, shape, "f32", streaming="pull")
    finally:
        os.environ.pop("LBEM_FUSE3", None)
    assert r.steps_per_launch == 1
    r.setup(p)
    r.step(4, p.amp[:4])
    want = r.moments()
    r.close()
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
