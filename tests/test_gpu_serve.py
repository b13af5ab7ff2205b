"""Batched stepping and continuous-batching serving on the GPU: every lattice
advanced in a batch (and every request served in a mix) is bit-identical to
the same lattice stepped alone."""
import os

import numpy as np
import pytest

from gpu_util import announce, random_problem
from paper_1108_2651_amd import inputs, lbem, serve

pytestmark = pytest.mark.gpu


def _solo(p, prec, nsteps, streaming="pull"):
    s = lbem.Solver(p.dim, p.shape, prec, streaming=streaming)
    s.setup(p)
    s.step(nsteps)
    out = s.moments()
    s.close()
    return out


@pytest.mark.parametrize("graph,concurrent,group_mib", [("1", "0", "160"), ("0", "0", "160"), ("1", "1", "160"),
                                                       ("0", "1", "160"), ("1", "0", "1"), ("1", "1", "1"),
                                                       ("0", "0", "0")])
def test_batch_matches_standalone_bitwise(graph, concurrent, group_mib):
    """Classes of a tick run one after another on the batch stream (the
    default) or concurrently on their own streams; graphs or direct launches;
    members in groups that fit a state budget (1 MiB: one or two members per
    group; 0: one group)."""
    import torch
    os.environ["LBEM_BATCH_GRAPH"] = graph
    os.environ["LBEM_BATCH_CONCURRENT"] = concurrent
    os.environ["LBEM_BATCH_GROUP_MIB"] = group_mib
    try:
        st = torch.cuda.Stream()
        batch = serve.Batch(16, 7, st)
    finally:
        os.environ.pop("LBEM_BATCH_GRAPH", None)
        os.environ.pop("LBEM_BATCH_CONCURRENT", None)
        os.environ.pop("LBEM_BATCH_GROUP_MIB", None)
    # plain members with pull or in-place AA storage (odd step counts leave AA
    # lattices in the swapped layout between ticks)
    cases = [(2, (96, 40, 1), "f32", "pull"), (2, (33, 17, 1), "f64", "pull"), (2, (130, 64, 1), "f16dev", "pull"),
             (3, (20, 12, 9), "f32", "pull"), (3, (16, 16, 16), "bf16dev", "pull"), (3, (9, 7, 5), "f64", "aa"),
             (3, (24, 20, 12), "f16dev", "pull"), (2, (64, 64, 1), "bf16dev", "pull"), (2, (70, 30, 1), "f32", "aa"),
             (3, (17, 13, 11), "f32", "aa"), (2, (40, 24, 1), "f64", "aa")]
    probs, solvers = [], []
    other = torch.cuda.Stream()
    for k, (dim, shape, prec, streaming) in enumerate(cases):
        p = random_problem(dim, shape, seed=200 + k, src=False)
        # half of the members live on another stream than the batch
        s = lbem.Solver(dim, shape, prec, streaming=streaming, stream=st if k % 2 == 0 else other)
        s.setup(p)
        probs.append(p)
        solvers.append(s)
    plan = [[7, 3, 7, 0, 5, 7, 1, 7, 3, 5, 7], [7, 7, 0, 7, 7, 2, 7, 7, 7, 0, 1],
            [1, 7, 7, 7, 0, 7, 7, 4, 5, 7, 2]]
    total = np.sum(plan, axis=0)
    for ns in plan:
        batch.run(solvers, ns)
    for k, (dim, shape, prec, streaming) in enumerate(cases):
        announce(f"batch vs solo graph={graph} concurrent={concurrent} group={group_mib} {dim}d {shape} {prec} "
                 f"{streaming} steps={total[k]}")
        got = solvers[k].moments()
        assert solvers[k].t == total[k]
        want = _solo(probs[k], prec, int(total[k]), streaming)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    for s in solvers:
        s.close()
    batch.close()


def test_batch_rejects_unsupported_members():
    import torch
    st = torch.cuda.Stream()
    b = serve.Batch(4, 5, st)
    p = random_problem(2, (32, 16, 1), seed=1, src=True, nsteps=4)
    s2 = lbem.Solver(2, p.shape, "f32", streaming="pull", stream=st)
    with pytest.raises(lbem.LbemError) as e:
        b.run([s2], [3])                        # not initialised
    assert e.value.code == lbem.LBEM_ESTATE
    q = random_problem(2, (32, 16, 1), seed=2, src=False)
    s3 = lbem.Solver(2, q.shape, "f32", streaming="pull", stream=st)
    s3.setup(q)
    with pytest.raises(lbem.LbemError):
        b.run([s3, s3], [1, 1])                 # duplicate member
    with pytest.raises(lbem.LbemError):
        b.run([s3], [6])                        # more than steps_per_tick
    s4 = lbem.Solver(2, q.shape, "f32", streaming="pull", stream=st)
    s4.set_boundary(0, "pec")
    s4.setup(q)
    with pytest.raises(lbem.LbemError) as e:
        b.run([s4], [1])                        # walls: single-step kernels only
    assert e.value.code == lbem.LBEM_EINVAL
    s5 = lbem.Solver(2, q.shape, "f32", streaming="pull", stream=st)
    s5.setup(q)
    s5.set_absorber(np.full(q.n, 0.01))
    with pytest.raises(lbem.LbemError) as e:
        b.run([s5], [1])                        # absorbing layer
    assert e.value.code == lbem.LBEM_EINVAL
    b.close()


@pytest.mark.parametrize("graph", ["1", "0"])
def test_batch_with_sources_mu_and_every_format_bitwise(graph):
    """Members with a current source (their amplitudes per step through
    lbem_batch_run_amp), a non-uniform mu, the ghost-coordinate formats and
    plain FP16 storage: each batched member equals the same lattice stepped
    alone with the same amplitudes, bit for bit."""
    import torch
    os.environ["LBEM_BATCH_GRAPH"] = graph
    try:
        st = torch.cuda.Stream()
        batch = serve.Batch(16, 6, st)
    finally:
        os.environ.pop("LBEM_BATCH_GRAPH", None)
    cases = [(2, (64, 40, 1), "f32", "aa", True, False), (2, (48, 33, 1), "f64", "pull", True, True),
             (2, (70, 24, 1), "f16ghost", "pull", True, False), (2, (40, 40, 1), "bf16ghost", "pull", False, True),
             (2, (50, 30, 1), "f16", "aa", True, False), (3, (20, 12, 9), "f16ghost", "pull", True, True),
             (3, (16, 16, 10), "f16dev", "pull", True, False), (3, (18, 11, 7), "f32", "pull", True, True),
             (3, (12, 10, 8), "f16", "pull", True, False), (3, (14, 9, 6), "bf16dev", "pull", False, True)]
    other = torch.cuda.Stream()
    probs, solvers = [], []
    total_steps = 17
    for k, (dim, shape, prec, streaming, src, mu) in enumerate(cases):
        p = random_problem(dim, shape, seed=300 + k, src=src, mu=mu, nsteps=total_steps)
        s = lbem.Solver(dim, shape, prec, streaming=streaming, mu_varies=mu, stream=st if k % 2 else other)
        s.setup(p)
        probs.append(p)
        solvers.append(s)
    plan = [[6, 2, 6, 6, 0, 6, 3, 6, 6, 1], [6, 6, 5, 6, 6, 6, 6, 0, 6, 6], [5, 6, 6, 5, 6, 5, 6, 6, 5, 6]]
    done = np.zeros(len(cases), int)
    for ns in plan:
        amps = [probs[k].amp[done[k]:done[k] + ns[k]] if cases[k][4] else None for k in range(len(cases))]
        batch.run(solvers, ns, amps)
        done += ns
    for k, (dim, shape, prec, streaming, src, mu) in enumerate(cases):
        announce(f"batch with extras graph={graph} {dim}d {shape} {prec} {streaming} src={src} mu={mu} "
                 f"steps={done[k]}")
        got = solvers[k].get_state()
        p = probs[k]
        ref = lbem.Solver(dim, shape, prec, streaming=streaming, mu_varies=mu)
        ref.setup(p)
        ref.step(int(done[k]), p.amp[:done[k]] if src else None)
        want = ref.get_state()
        ref.close()
        assert solvers[k].t == done[k]
        assert np.array_equal(got, want), (prec, streaming, src, mu)
    for s in solvers:
        s.close()
    batch.close()


# Members of the 3D deviation classes for the whole-row batched tiles: (shape,
# format, source, varying mu).  "rows": every class all on the row tiling with
# mu == 1; "rows_mu": all with varying mu; "cells": classes that fall back to
# the per-cell tiles (a row longer than 2 NT cells, mixed mu).
ROW_SETS = {
    "rows": [((32, 32, 12), "f16dev", False, False), ((9, 30, 10), "f16dev", True, False),
             ((33, 7, 5), "f16dev", True, False), ((128, 9, 1), "f16ghost", False, False),
             ((1024, 2, 3), "f16ghost", True, False), ((40, 1, 12), "f16ghost", True, False),
             ((96, 20, 17), "bf16dev", True, False), ((17, 5, 9), "bf16ghost", False, False)],
    "rows_mu": [((24, 10, 9), "f16dev", True, True), ((33, 7, 5), "f16ghost", True, True),
                ((64, 3, 3), "bf16ghost", False, True), ((20, 12, 9), "f16ghost", False, True)],
    "cells": [((1040, 2, 3), "f16dev", True, True), ((32, 8, 8), "f16dev", False, False),
              ((20, 12, 9), "f16ghost", True, True), ((16, 16, 10), "f16ghost", True, False)],
}


@pytest.mark.parametrize("which", list(ROW_SETS))
def test_batched_row_tiles_bitwise(which):
    """3D deviation members on the batch's whole-row tiling (two cells per
    thread, numbered through the tile's rows), with the row kernel forced on
    for every class that qualifies: short, odd and single rows, tiles taller
    than the box, one plane, chunks longer than the box, rows of exactly 1024
    cells (two per thread of a 512-thread block);
    first steps from the natural layout, members that ran solo steps before
    they joined, sources and mu; and classes that fall back to the per-cell
    tiles.  Each member equals its solo run bit for bit."""
    import torch
    st = torch.cuda.Stream()
    os.environ["LBEM_BATCH_ROWS_MIN"] = "0"
    try:
        batch = serve.Batch(16, 6, st)
    finally:
        os.environ.pop("LBEM_BATCH_ROWS_MIN", None)
    cases = ROW_SETS[which]
    pre = [3 if k % 3 == 2 else 0 for k in range(len(cases))]      # solo steps before joining the batch
    plan = [[6, 5, 6, 6, 0, 6, 1, 6][:len(cases)], [6, 6, 6, 3, 6, 6, 6, 0][:len(cases)],
            [2, 6, 0, 6, 6, 4, 6, 6][:len(cases)]]
    total_steps = max(pre) + sum(max(r) for r in plan)
    probs, solvers = [], []
    for k, (shape, prec, src, mu) in enumerate(cases):
        p = random_problem(3, shape, seed=500 + k, src=src, mu=mu, nsteps=total_steps)
        s = lbem.Solver(3, shape, prec, mu_varies=mu, stream=st)
        s.setup(p)
        if pre[k]:
            s.step(pre[k], p.amp[:pre[k]] if src else None)
        probs.append(p)
        solvers.append(s)
    done = np.array(pre)
    for ns in plan:
        amps = [probs[k].amp[done[k]:done[k] + ns[k]] if cases[k][2] else None for k in range(len(cases))]
        batch.run(solvers, ns, amps)
        done += ns
    for k, (shape, prec, src, mu) in enumerate(cases):
        announce(f"batched row tiles [{which}] {shape} {prec} src={src} mu={mu} steps={done[k]}")
        got = solvers[k].get_state()
        p = probs[k]
        ref = lbem.Solver(3, shape, prec, mu_varies=mu)
        ref.setup(p)
        ref.step(int(done[k]), p.amp[:done[k]] if src else None)
        want = ref.get_state()
        ref.close()
        assert solvers[k].t == done[k]
        assert np.array_equal(got, want), (shape, prec, src, mu)
    for s in solvers:
        s.close()
    batch.close()


def test_serving_mix_results_equal_solo_runs():
    reqs = serve.make_requests(count=20, rate=400.0, seed=11, steps_lo=30, steps_hi=160,
                               side2d=(5, 7.5), side3d=(4, 5.5))
    announce("serving mix of 20 requests")
    rep = serve.serve(reqs, budget_bytes=64 << 20, max_slots=8, steps_per_tick=16, workers=3,
                      keep_results=True)
    announce(f"  completed={rep.completed} p50={rep.p50_ms:.1f} ms p99={rep.p99_ms:.1f} ms "
             f"mean resident={rep.mean_resident:.1f}")
    assert rep.completed == len(reqs)
    assert rep.max_resident > 1                 # requests really shared ticks
    ex = serve.GpuExecutor(4, 16, workers=1)
    try:
        for r in reqs:
            p = serve.request_problem_fast(r, ex)
            want = _solo(p, r.prec, r.nsteps)
            got = r.result
            assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), r.rid
    finally:
        ex.close()


def test_batched_members_match_the_oracle():
    """Members of one batch, advanced together over several ticks with
    different step counts per tick, against the FP64 oracle at each format's
    bar: 2D and 3D, FP64 / FP32 (pull and AA) and the FP16 deviation format,
    on smooth heterogeneous media with a Gaussian pulse (the serving
    workload's kind of input)."""
    import torch
    from gpu_util import oracle_run, rel
    st = torch.cuda.Stream()
    batch = serve.Batch(10, 9, st)
    rng = np.random.default_rng(77)
    cases = [(2, 96, "f64", "aa"), (2, 128, "f32", "pull"), (2, 80, "f16dev", "pull"),
             (3, 24, "f32", "aa"), (3, 32, "f16dev", "pull"), (3, 20, "f64", "pull"),
             (2, 72, "f16ghost", "pull"), (3, 28, "f16ghost", "pull")]
    tol = {"f64": 1e-12, "f32": 1e-5, "f16dev": 1e-3, "f16ghost": 1e-3}
    probs, solvers = [], []
    for dim, n, prec, streaming in cases:
        shp = (n, n) if dim == 2 else (n, n, n)
        eps = 1.0 + 3.0 * inputs.smooth_noise(rng, shp, n / 8.0)
        p = inputs.pulse_problem(dim, n, n / 8.0, rng, eps=eps)
        s = lbem.Solver(dim, p.shape, prec, streaming=streaming, stream=st)
        s.setup(p)
        probs.append(p)
        solvers.append(s)
    plan = [[9, 9, 9, 9, 9, 9, 9, 9], [9, 4, 9, 9, 0, 9, 9, 2], [9, 9, 9, 5, 9, 9, 9, 9], [3, 9, 9, 9, 9, 9, 9, 9]]
    total = np.sum(plan, axis=0)
    for ns in plan:
        batch.run(solvers, ns)
    for k, (dim, n, prec, streaming) in enumerate(cases):
        Eg, Bg = solvers[k].moments()
        o = oracle_run(probs[k], int(total[k]))
        Eo, Bo = o.fields()
        eE, eB = rel(Eg, Eo), rel(Bg, Bo)
        announce(f"batched member {dim}d {n} {prec} {streaming} steps={total[k]}: E {eE:.2e} B {eB:.2e}")
        assert eE <= tol[prec] and eB <= tol[prec], (prec, eE, eB)
    for s in solvers:
        s.close()
    batch.close()


@pytest.mark.parametrize("prec", ["f32", "f16ghost"])
def test_batched_forced_member_matches_the_oracle(prec):
    """The paper's forced problem inside a batch: the homogeneous test's
    Gaussian current j_z (Subsection "Homogeneous media"), here with a
    Ricker amplitude per step handed over through lbem_batch_run_amp, in a
    heterogeneous medium with mu = 1 + (eps - 1)/3 (the B x grad ln mu source
    term of the Maxwell section), against the FP64 oracle."""
    import torch
    from gpu_util import oracle_run, rel
    n, K = 96, 8
    rng = np.random.default_rng(5)
    eps = 1.0 + 3.0 * inputs.smooth_noise(rng, (n, n), 10.0)
    cells, w = inputs.paper_jz_source(n)
    steps = 60
    p = inputs.Problem(dim=2, shape=(n, n, 1), eps_r=eps.ravel(), mu_r=1.0 + (eps.ravel() - 1.0) / 3.0,
                       E0=np.zeros((3, n * n)), B0=np.zeros((3, n * n)), src_comp=2, src_cells=cells,
                       src_weights=w, amp=inputs.ricker(steps, 0.02), nsteps=steps)
    st = torch.cuda.Stream()
    batch = serve.Batch(4, K, st)
    s = lbem.Solver(2, p.shape, prec, streaming="pull", mu_varies=True, stream=st)
    s.setup(p)
    done = 0
    while done < steps:
        k = min(K, steps - done)
        batch.run([s], [k], [p.amp[done:done + k]])
        done += k
    Eg, Bg = s.moments()
    Eo, Bo = oracle_run(p, steps).fields()
    eE, eB = rel(Eg, Eo), rel(Bg, Bo)
    announce(f"batched forced member {prec}: E {eE:.2e} B {eB:.2e}")
    tol = 1e-5 if prec == "f32" else 1e-3
    assert eE <= tol and eB <= tol, (eE, eB)
    s.close()
    batch.close()
