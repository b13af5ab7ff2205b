"""Shared helpers for the GPU parity tests (oracle vs HIP path on identical
seeded inputs)."""
import os
import sys

import numpy as np

from oracle import oracle as O
from paper_1108_2651_amd import inputs


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def gpu_run(p, nsteps, prec, streaming="auto", tau=None, env=None):
    from paper_1108_2651_amd import lbem
    old = {}
    for k, v in (env or {}).items():
        old[k] = os.environ.get(k)
        os.environ[k] = str(v)
    try:
        s = lbem.Solver(p.dim, p.shape, prec, tau=p.tau if tau is None else tau, w0_vac=p.w0_vac,
                        streaming=streaming, mu_varies=p.mu_r is not None)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    s.setup(p)
    amp = p.amp[:nsteps] if (p.amp is not None and len(p.src_cells)) else None
    s.step(nsteps, amp)
    return s


def oracle_run(p, nsteps, tau=None):
    o = O.Oracle(p.dim, p.shape, p.tau if tau is None else tau, p.w0_vac)
    o.set_medium(p.eps_r, p.mu_r)
    o.init_fields(p.E0, p.B0)
    if len(p.src_cells):
        o.set_source(p.src_comp, p.src_cells, p.src_weights)
    o.step(nsteps, p.amp[:nsteps] if (p.amp is not None and len(p.src_cells)) else None)
    return o


def random_problem(dim, shape, seed, mu=False, src=True, nsteps=64):
    """Heterogeneous medium, random TM (2D) or full (3D) fields, a scattered
    current source with random amplitudes: exercises every term."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    n = nx * ny * nz
    eps = rng.uniform(1.0, 6.0, n)
    mur = rng.uniform(0.8, 1.6, n) if mu else None
    E = np.zeros((3, n))
    B = np.zeros((3, n))
    if dim == 2:
        E[2] = rng.standard_normal(n)
        B[:2] = rng.standard_normal((2, n))
        comp = 2
    else:
        E[:] = rng.standard_normal((3, n))
        B[:] = rng.standard_normal((3, n))
        comp = int(rng.integers(0, 3))
    p = inputs.Problem(dim=dim, shape=shape, eps_r=eps, mu_r=mur, E0=E, B0=B, nsteps=nsteps,
                       name=f"random-{dim}d-{shape}")
    if src:
        k = max(1, n // 7)
        p.src_cells = rng.choice(n, size=k, replace=False).astype(np.int64)
        p.src_weights = rng.standard_normal(k)
        p.src_comp = comp
        p.amp = rng.standard_normal(nsteps)
    return p


def window_problem(p, centre, k):
    """Periodic window of half-width k+1 around `centre` (x, y[, z])."""
    dim = p.dim
    nx, ny, nz = p.shape
    h = k + 1
    w = 2 * h + 1
    ranges = [(np.arange(-h, h + 1) + centre[a]) % p.shape[a] for a in range(dim)]
    if dim == 2:
        Y, X = np.meshgrid(ranges[1], ranges[0], indexing="ij")
        idx = (X + nx * Y).ravel()
        wshape = (w, w, 1)
    else:
        Z, Y, X = np.meshgrid(ranges[2], ranges[1], ranges[0], indexing="ij")
        idx = (X + nx * (Y + ny * Z)).ravel()
        wshape = (w, w, w)
    pos = {int(c): j for j, c in enumerate(idx)}
    cells, wts = [], []
    for c, wt in zip(p.src_cells, p.src_weights):
        j = pos.get(int(c))
        if j is not None:
            cells.append(j)
            wts.append(wt)
    q = inputs.Problem(dim=dim, shape=wshape, eps_r=p.eps_r[idx], mu_r=None, E0=p.E0[:, idx],
                       B0=p.B0[:, idx], src_comp=p.src_comp, src_cells=np.asarray(cells, np.int64),
                       src_weights=np.asarray(wts), amp=p.amp, w0_vac=p.w0_vac)
    centre_index = h + w * (h + (w * h if dim == 3 else 0))
    return q, centre_index
