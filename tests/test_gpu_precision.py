"""Precision of every storage format against the FP64 oracle on the 64^3
centred crops of the two 3D benchmark media (sharp spheres with a dipole;
layered medium with a dipole), run as their own periodic boxes, at 1000 and
2000 steps.  Bars, each field's relative L2: FP64 <= 1e-12, FP32 <= 1e-5,
FP16 deviation and ghost formats <= 1e-3.  The BF16 formats miss 1e-3 and are
held to their measured band (non-compliant); the energy-norm error is
reported beside every row."""
import numpy as np
import pytest

from gpu_util import announce, rel
from test_gpu_parity import TOL
from oracle import oracle as O
from paper_1108_2651_amd import inputs, lbem

pytestmark = pytest.mark.gpu

PRECS = ["f64", "f32", "f16dev", "bf16dev", "f16ghost", "bf16ghost"]
BAR = {k: TOL[k] for k in PRECS}
CHECKPOINTS = (1000, 2000)


def energy_error(Eg, Bg, Eo, Bo, ea):
    num = np.sum(ea * ((Eg - Eo) ** 2).sum(0) + ((Bg - Bo) ** 2).sum(0))
    den = np.sum(ea * (Eo ** 2).sum(0) + (Bo ** 2).sum(0))
    return float(np.sqrt(num / den))


@pytest.mark.parametrize("config", ["config3", "config4"])
def test_precision_table_64_crops(config):
    p = getattr(inputs, config)(nsteps=CHECKPOINTS[-1], crop_n=64)
    o = O.Oracle(3, p.shape, p.tau, p.w0_vac)
    o.set_medium(p.eps_r)
    o.init_fields(p.E0, p.B0)
    o.set_source(p.src_comp, p.src_cells, p.src_weights)
    ea = o.medium()["eps_abs"]
    ref, t = {}, 0
    for k in CHECKPOINTS:
        o.step(k - t, p.amp[t:k])
        ref[k] = o.fields()
        t = k
    failures = []
    for prec in PRECS:
        s = lbem.Solver(3, p.shape, prec, w0_vac=p.w0_vac)
        s.setup(p)
        t = 0
        for k in CHECKPOINTS:
            s.step(k - t, p.amp[t:k])
            t = k
            Eg, Bg = s.moments()
            Eo, Bo = ref[k]
            eE, eB, eN = rel(Eg, Eo), rel(Bg, Bo), energy_error(Eg, Bg, Eo, Bo, ea)
            announce(f"{config} 64^3 crop {prec:9s} {k:5d} steps: E {eE:.2e}  B {eB:.2e}  energy {eN:.2e}")
            bar = BAR[prec]
            if not (eE <= bar and eB <= bar):
                failures.append((prec, k, eE, eB, eN))
        s.close()
    assert not failures, failures
