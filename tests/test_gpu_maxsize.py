"""Lattices of 2^30 cells (32768^2 in 2D, 1024^3 in 3D), in the launch
configurations the solver picks at that size (four fused 2D steps per
launch; the z-marching 16-bit kernel in 3D), checked on sampled cells
against the oracle through light-cone windows.  Array offsets here pass 2^32
elements, so this exercises the 64-bit indexing of every kernel involved."""
import numpy as np
import pytest

from gpu_util import announce, window_problem
from oracle import oracle as O
from paper_1108_2651_amd import inputs, lbem

pytestmark = pytest.mark.gpu


def cheap_medium(shape):
    """eps in [1,4]: a smooth deterministic pattern (fast at 10^9 cells)."""
    nx, ny, nz = shape
    x = np.arange(nx, dtype=np.float32)
    out = np.empty(nx * ny * nz)
    row = 0
    for z in range(nz):
        for y in range(0, ny, 256):
            yy = np.arange(y, min(y + 256, ny), dtype=np.float32)[:, None]
            v = 2.5 + 1.5 * np.sin(0.013 * x[None, :] + 0.021 * yy + 0.017 * z)
            out[row:row + v.size] = v.ravel()
            row += v.size
    return out


def pulses(shape, centres, comp):
    """Fields: Gaussian E pulses (sigma 3) at the given centres, B = 0."""
    nx, ny, nz = shape
    n = nx * ny * nz
    E = np.zeros((3, n))
    B = np.zeros((3, n))
    r = 8
    for c in centres:
        for dz in (range(-r, r + 1) if nz > 1 else [0]):
            for dy in range(-r, r + 1):
                xs = (c[0] + np.arange(-r, r + 1)) % nx
                y = (c[1] + dy) % ny
                z = (c[2] + dz) % nz if nz > 1 else 0
                d2 = np.arange(-r, r + 1) ** 2 + dy * dy + dz * dz
                E[comp, xs + nx * (y + ny * z)] += np.exp(-d2 / 18.0)
    return E, B


def sampled(p, prec, k, samples, tol):
    import torch
    torch.cuda.empty_cache()          # arenas of earlier tests, cached by torch
    s = lbem.Solver(p.dim, p.shape, prec, w0_vac=p.w0_vac)
    s.setup(p)
    spl = s.steps_per_launch
    s.step(k)
    Eg, Bg = s.moments()
    s.close()
    del s
    torch.cuda.empty_cache()
    nx, ny, nz = p.shape
    worst = 0.0
    for centre in samples:
        q, ci = window_problem(p, centre, k)
        o = O.Oracle(q.dim, q.shape, q.tau, q.w0_vac)
        o.set_medium(q.eps_r)
        o.init_fields(q.E0, q.B0)
        o.step(k)
        Eo, Bo = o.fields()
        c = centre[0] + nx * (centre[1] + ny * (centre[2] if p.dim == 3 else 0))
        scale = max(np.abs(Eo).max(), np.abs(Bo).max(), 1e-30)
        err = max(np.abs(Eg[:, c] - Eo[:, ci]).max(), np.abs(Bg[:, c] - Bo[:, ci]).max()) / scale
        worst = max(worst, err)
    announce(f"  {prec} {p.shape} steps/launch={spl}: worst sampled error {worst:.2e}")
    assert worst <= tol, worst
    return spl


def test_2d_2pow30_cells_fused():
    shape = (32768, 32768, 1)
    announce("2D 32768^2 (2^30 cells) fp32")
    centres = [(5, 7, 0), (32760, 32765, 0), (16000, 30000, 0), (300, 32767, 0)]
    E, B = pulses(shape, centres, 2)
    p = inputs.Problem(dim=2, shape=shape, eps_r=cheap_medium(shape), mu_r=None, E0=E, B0=B, nsteps=8,
                       name="2d-32768")
    samples = [(5, 7, 0), (32761, 32766, 0), (0, 0, 0), (16002, 29999, 0), (301, 32767, 0)]
    assert sampled(p, "f32", 8, samples, 1e-5) == 4


def test_3d_2pow30_cells_ghost_zmarch():
    shape = (1024, 1024, 1024)
    announce("3D 1024^3 (2^30 cells) f16ghost")
    centres = [(10, 12, 14), (1020, 1021, 1022), (512, 700, 900)]
    E, B = pulses(shape, centres, 1)
    p = inputs.Problem(dim=3, shape=shape, eps_r=cheap_medium(shape), mu_r=None, E0=E, B0=B, nsteps=3,
                       name="3d-1024")
    samples = [(10, 12, 14), (1021, 1020, 1023), (0, 1023, 1023), (513, 701, 899)]
    sampled(p, "f16ghost", 3, samples, 1e-3)
