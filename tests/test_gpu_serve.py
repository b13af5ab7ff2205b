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


@pytest.mark.parametrize("graph", ["1", "0"])
def test_batch_matches_standalone_bitwise(graph):
    import torch
    os.environ["LBEM_BATCH_GRAPH"] = graph
    try:
        st = torch.cuda.Stream()
        batch = serve.Batch(16, 7, st)
    finally:
        os.environ.pop("LBEM_BATCH_GRAPH", None)
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
        announce(f"batch vs solo graph={graph} {dim}d {shape} {prec} {streaming} steps={total[k]}")
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
    s = lbem.Solver(2, p.shape, "f32", streaming="pull", stream=st)
    s.setup(p)                                  # has a current source
    with pytest.raises(lbem.LbemError) as e:
        b.run([s], [3])
    assert e.value.code == lbem.LBEM_EINVAL
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
    s4 = lbem.Solver(2, q.shape, "f16ghost", streaming="pull", stream=st)
    s4.setup(q)
    with pytest.raises(lbem.LbemError) as e:
        b.run([s4], [1])                        # no batched ghost-coordinate kernels
    assert e.value.code == lbem.LBEM_EINVAL
    s5 = lbem.Solver(2, q.shape, "f16", streaming="aa", stream=st)
    s5.setup(q)
    with pytest.raises(lbem.LbemError) as e:
        b.run([s5], [1])                        # nor plain FP16 ones
    assert e.value.code == lbem.LBEM_EINVAL
    b.close()


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
    batch = serve.Batch(8, 9, st)
    rng = np.random.default_rng(77)
    cases = [(2, 96, "f64", "aa"), (2, 128, "f32", "pull"), (2, 80, "f16dev", "pull"),
             (3, 24, "f32", "aa"), (3, 32, "f16dev", "pull"), (3, 20, "f64", "pull")]
    tol = {"f64": 1e-12, "f32": 1e-5, "f16dev": 1e-3}
    probs, solvers = [], []
    for dim, n, prec, streaming in cases:
        shp = (n, n) if dim == 2 else (n, n, n)
        eps = 1.0 + 3.0 * inputs.smooth_noise(rng, shp, n / 8.0)
        p = inputs.pulse_problem(dim, n, n / 8.0, rng, eps=eps)
        s = lbem.Solver(dim, p.shape, prec, streaming=streaming, stream=st)
        s.setup(p)
        probs.append(p)
        solvers.append(s)
    plan = [[9, 9, 9, 9, 9, 9], [9, 4, 9, 9, 0, 9], [9, 9, 9, 5, 9, 9], [3, 9, 9, 9, 9, 9]]
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
