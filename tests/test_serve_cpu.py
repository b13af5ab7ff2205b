"""Scheduler logic on the CPU with a virtual-time executor (a test double of
the scheduler's executor only; no solver arithmetic runs here)."""
import numpy as np
import pytest

from paper_1108_2651_amd.serve import Request, Scheduler


class _Fut:
    def __init__(self, slot):
        self.slot = slot


class FakeExecutor:
    """Virtual clock: set-up costs `setup_s`, a tick costs its cell-steps / rate."""

    def __init__(self, rate=1e9, setup_s=1e-3, bytes_per_cell=100):
        self.t = 0.0
        self.rate, self.setup_s, self.bpc = rate, setup_s, bytes_per_cell
        self.steps = {}
        self.live = {}
        self.max_live_bytes = 0
        self.max_concurrent = 0
        self.max_tick = 0
        self.admit_order = []
        self.finished = []
        self._next = 0

    def now(self):
        return self.t

    def sleep_until(self, t):
        self.t = max(self.t, t)

    def nbytes(self, r):
        return r.cells * self.bpc

    def admit(self, r):
        self.t += self.setup_s
        slot = self._next
        self._next += 1
        self.live[slot] = (r, r.cells * self.bpc)
        self.steps[slot] = 0
        self.admit_order.append(r.rid)
        self.max_live_bytes = max(self.max_live_bytes, sum(b for _, b in self.live.values()))
        self.max_concurrent = max(self.max_concurrent, len(self.live))
        return _Fut(slot)

    def ready(self, f):
        return True

    def result(self, f):
        return f.slot     # the admitted slot, or (result, completion time) of a read-back

    def wait_any(self, futs):
        pass

    def tick(self, slots, nsteps):
        assert len(set(slots)) == len(slots)
        self.max_tick = max(self.max_tick, len(slots))
        work = 0
        for s, k in zip(slots, nsteps):
            assert 0 < k
            self.steps[s] += k
            work += self.live[s][0].cells * k
        self.t += work / self.rate

    def finish_async(self, slot, want=True):
        r, _ = self.live.pop(slot)
        self.finished.append((r.rid, self.steps[slot], want))
        return _Fut((("result", r.rid) if want else None, self.t))


def mix(count=60, rate=200.0, seed=3):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1 / rate, count))
    out = []
    for k in range(count):
        dim = 2 if rng.random() < 0.7 else 3
        n = int(rng.integers(4, 40)) * (4 if dim == 2 else 1)
        out.append(Request(rid=k, t_arrive=float(t[k]), dim=dim, n=n, nsteps=int(rng.integers(20, 400))))
    return out


def test_every_request_completes_with_its_step_count():
    ex = FakeExecutor()
    reqs = mix()
    rep = Scheduler(ex, budget_bytes=50_000_000, max_slots=16, steps_per_tick=50).run(reqs)
    assert rep.completed == len(reqs)
    got = {rid: steps for rid, steps, want in ex.finished}
    for r in reqs:
        assert got[r.rid] == r.nsteps
        assert r.status == "done" and r.t_done >= r.t_arrive
    assert rep.p99_ms >= rep.p50_ms > 0


def test_budget_and_slots_bound_residency():
    ex = FakeExecutor(rate=2e8)
    reqs = mix(80)
    budget = 3_000_000
    rep = Scheduler(ex, budget_bytes=budget, max_slots=5, steps_per_tick=25).run(reqs)
    assert ex.max_live_bytes <= budget          # memory held, including solves being read back
    assert ex.max_tick <= 5                     # lattices per tick never exceed the slots
    assert rep.max_resident <= 5
    assert rep.completed + rep.rejected == len(reqs)
    # every request that fits the budget alone is served
    assert rep.rejected == sum(r.cells * 100 > budget for r in reqs)


def test_fifo_admission_order():
    ex = FakeExecutor(rate=1e8)
    reqs = mix(50)
    Scheduler(ex, budget_bytes=4_000_000, max_slots=4, steps_per_tick=40).run(reqs)
    order = [rid for rid in ex.admit_order]
    arrival = [r.rid for r in sorted(reqs, key=lambda r: r.t_arrive) if r.cells * 100 <= 4_000_000]
    assert order == arrival


def test_oversized_request_rejected_others_served():
    ex = FakeExecutor()
    reqs = [Request(rid=0, t_arrive=0.0, dim=3, n=200, nsteps=10),
            Request(rid=1, t_arrive=0.001, dim=2, n=32, nsteps=10)]
    rep = Scheduler(ex, budget_bytes=1_000_000, max_slots=4, steps_per_tick=5).run(reqs)
    assert reqs[0].status == "rejected" and reqs[1].status == "done"
    assert rep.completed == 1 and rep.rejected == 1


def test_cancellation_releases_memory():
    ex = FakeExecutor(rate=1e7)
    reqs = [Request(rid=k, t_arrive=0.0, dim=2, n=64, nsteps=400) for k in range(6)]
    sched = Scheduler(ex, budget_bytes=64 * 64 * 100 * 2, max_slots=8, steps_per_tick=50)

    def hook(s, tick):
        if tick == 2:
            s.cancel(0)          # resident
            s.cancel(5)          # still waiting for memory
    rep = sched.run(reqs, on_tick=hook)
    assert reqs[0].status == "cancelled" and reqs[5].status == "cancelled"
    assert rep.cancelled == 2 and rep.completed == 4
    assert all(want is False for rid, steps, want in ex.finished if rid == 0)
    assert not ex.live


def test_requests_joining_mid_flight_overlap():
    """Continuous batching: a request arriving while others run is admitted at
    the next tick boundary and shares ticks with them."""
    ex = FakeExecutor(rate=1e7)
    long = Request(rid=0, t_arrive=0.0, dim=2, n=64, nsteps=1000)
    late = Request(rid=1, t_arrive=0.01, dim=2, n=32, nsteps=100)
    shared = []

    class Spy(FakeExecutor):
        def tick(self, slots, nsteps):
            shared.append(len(slots))
            super().tick(slots, nsteps)
    ex = Spy(rate=1e7)
    Scheduler(ex, budget_bytes=10**9, max_slots=8, steps_per_tick=50).run([long, late])
    assert max(shared) == 2
    assert late.t_done < long.t_done


class _Pending:
    """A worker-thread future that completes at a virtual time."""

    def __init__(self, ex, t_ready, value):
        self.ex, self.t_ready, self.value = ex, t_ready, value

    def done(self):
        return self.ex.t >= self.t_ready


class WorkerExecutor(FakeExecutor):
    """Set-up and read-back take virtual time on worker threads.  A tick may
    only name lattices whose set-up has completed and whose read-back has not
    been issued: the library's handles are not shared between a worker call
    and a batch tick."""

    def __init__(self, setup_s=2e-3, finish_s=1e-3, **kw):
        super().__init__(setup_s=0.0, **kw)
        self.setup_dt, self.finish_dt = setup_s, finish_s
        self.busy = set()        # slots a worker is still setting up or reading back
        self.pending = []

    def admit(self, r):
        f = super().admit(r)
        self.busy.add(f.slot)
        fut = _Pending(self, self.t + self.setup_dt, f.slot)
        self.pending.append(fut)
        return fut

    def ready(self, f):
        if f.done() and getattr(f, "value", None) in self.busy and f in self.pending:
            self.busy.discard(f.value)     # the worker finished the set-up
            self.pending.remove(f)
        return f.done()

    def result(self, f):
        assert f.done()
        self.ready(f)
        return f.value

    def wait_any(self, futs):
        ts = [f.t_ready for f in futs if not f.done()]
        if ts:
            self.t = max(self.t, min(ts))

    def tick(self, slots, nsteps):
        assert not (set(slots) & self.busy), "a tick names a lattice owned by a worker"
        super().tick(slots, nsteps)

    def finish_async(self, slot, want=True):
        assert slot not in self.busy
        f = super().finish_async(slot, want)
        return _Pending(self, self.t + self.finish_dt, f.slot)


def test_ticks_never_touch_lattices_owned_by_workers():
    ex = WorkerExecutor(rate=5e8)
    reqs = mix(120, rate=400.0, seed=9)
    rep = Scheduler(ex, budget_bytes=20_000_000, max_slots=12, steps_per_tick=40).run(reqs)
    assert rep.completed + rep.rejected == len(reqs)
    got = {rid: steps for rid, steps, want in ex.finished}
    for r in reqs:
        if r.status == "done":
            assert got[r.rid] == r.nsteps
