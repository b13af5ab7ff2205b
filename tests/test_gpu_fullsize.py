"""Parity at the full benchmark sizes, in the launch configuration bench.py
times, on sampled outputs.

After k steps a cell's populations depend only on cells within k lattice
steps (one cell per step along the axes).  So the oracle can compute the
fields at a sample cell exactly on a periodic window of half-width k+1 cut
from the full-size medium and source, around that cell: the window's own
periodic wrap lies outside the sample's dependence cone.
"""
import numpy as np
import pytest

from gpu_util import announce, window_problem
from oracle import oracle as O
from paper_1108_2651_amd import inputs, lbem

pytestmark = pytest.mark.gpu


def sampled_parity(p, prec, k, samples, tol, streaming="auto"):
    s = lbem.Solver(p.dim, p.shape, prec, w0_vac=p.w0_vac, streaming=streaming)
    s.setup(p)
    spl = s.steps_per_launch
    s.step(k, p.amp[:k])
    Eg, Bg = s.moments()
    s.close()
    nx, ny, nz = p.shape
    worst = 0.0
    for centre in samples:
        q, ci = window_problem(p, centre, k)
        o = O.Oracle(q.dim, q.shape, q.tau, q.w0_vac)
        o.set_medium(q.eps_r)
        o.init_fields(q.E0, q.B0)
        if len(q.src_cells):
            o.set_source(q.src_comp, q.src_cells, q.src_weights)
        o.step(k, q.amp[:k] if len(q.src_cells) else None)
        Eo, Bo = o.fields()
        c = centre[0] + nx * (centre[1] + (ny * centre[2] if p.dim == 3 else 0))
        scale = max(np.abs(Eo).max(), np.abs(Bo).max(), 1e-30)
        err = max(np.abs(Eg[:, c] - Eo[:, ci]).max(), np.abs(Bg[:, c] - Bo[:, ci]).max()) / scale
        announce(f"  sample {tuple(int(v) for v in centre)}: max abs diff / window field scale = {err:.2e}")
        worst = max(worst, err)
    assert worst <= tol, worst
    return spl


def test_config2_full_grid_1000_steps_fp32():
    """The benchmark workload on its whole 2048^2 grid, in the benchmark's
    launch configuration, against the oracle on the whole grid after 1000
    steps: relative L2 of E and of B <= 1e-5."""
    from gpu_util import oracle_run, rel
    k = 1000
    p = inputs.config2(nsteps=k)
    announce("config2 2048^2 fp32 full grid, 1000 steps (oracle on all host cores)")
    s = lbem.Solver(p.dim, p.shape, "f32", w0_vac=p.w0_vac)
    s.setup(p)
    assert s.steps_per_launch == 4
    s.step(k, p.amp[:k])
    Eg, Bg = s.moments()
    s.close()
    Eo, Bo = oracle_run(p, k).fields()
    eE, eB = rel(Eg, Eo), rel(Bg, Bo)
    announce(f"  rel L2 E={eE:.3e} B={eB:.3e}")
    assert eE <= 1e-5 and eB <= 1e-5, (eE, eB)


def test_config2_recipe_5000_steps_fp32():
    """The whole length of the 2D benchmark run (5000 steps, waves wrapping
    through the periodic box many times) on the same recipe at 512^2, whole
    grid against the oracle.  FP32 rounding errors add up at most linearly in
    the number of steps, so the bar is the 1000-step one scaled by 5: 5e-5."""
    from gpu_util import oracle_run, rel
    k = 5000
    p = inputs.config2(nsteps=k, n=512)
    announce("config2 recipe 512^2 fp32 full grid, 5000 steps (oracle on all host cores)")
    s = lbem.Solver(p.dim, p.shape, "f32", w0_vac=p.w0_vac)
    s.setup(p)
    assert s.steps_per_launch == 4
    s.step(k, p.amp[:k])
    Eg, Bg = s.moments()
    s.close()
    Eo, Bo = oracle_run(p, k).fields()
    eE, eB = rel(Eg, Eo), rel(Bg, Bo)
    announce(f"  rel L2 E={eE:.3e} B={eB:.3e}")
    assert eE <= 5e-5 and eB <= 5e-5, (eE, eB)


def test_config2_full_2048_fp32_fused():
    """The config-2 workload in its launch configuration (2048^2 FP32, four
    time steps per launch on 512-thread tiles), 64 steps, 6 sampled cells
    including the source line and the periodic seams."""
    k = 64
    p = inputs.config2(nsteps=k)
    announce("config2 2048^2 fp32 full size")
    samples = [(64, 1000), (65, 0), (0, 2047), (700, 1234), (2047, 5), (40, 300)]
    sampled_parity(p, "f32", k, samples, 1e-5)


@pytest.mark.parametrize("streaming", ["pull", "aa"])
def test_config3_full_256_fp32(streaming):
    """Default pull streaming runs two fused steps per launch; AA single steps."""
    k = 24
    p = inputs.config3(nsteps=k)
    announce(f"config3 256^3 fp32 {streaming} full size")
    samples = [(128, 128, 128), (130, 125, 131), (0, 0, 255), (200, 17, 90)]
    sampled_parity(p, "f32", k, samples, 1e-5, streaming=streaming)


@pytest.mark.parametrize("prec", ["f16dev", "f16ghost"])
def test_config4_full_512_deviation_storage(prec):
    k = 16
    p = inputs.config4(nsteps=k)
    announce(f"config4 512^3 {prec} full size")
    samples = [(256, 256, 256), (255, 258, 250), (511, 0, 300)]
    sampled_parity(p, prec, k, samples, 1e-3)


def test_config4_full_512_fp32_fused_pair():
    """The FP32 path at 512^3 in the launch configuration bench.py times for
    it: two fused steps per launch (z-marching frames), streaming stores of
    the state, row-major tile order (no XCD remap above 4e7 cells), 32-bit
    local offsets.  16 steps, samples at the dipole, near it, and on the
    periodic seams of all three axes."""
    k = 16
    p = inputs.config4(nsteps=k)
    announce("config4 512^3 fp32 fused pair, full size")
    samples = [(256, 256, 256), (250, 261, 253), (511, 0, 300), (0, 511, 0), (3, 255, 511)]
    assert sampled_parity(p, "f32", k, samples, 1e-5) == 2
