"""Continuous-batching serving of many lattice-BGK Maxwell solves on one GPU.

Requests (independent 2D/3D solves of different sizes and formats) arrive
over time.  The scheduler admits them in arrival order while device memory
(a byte budget) and batch slots allow, sets them up on worker threads (each on
its own stream, overlapping the running ticks), and advances every resident
solve together: one tick = K time steps of a persistent batched stream-collide
launch per (dim, format) class, replayed from a HIP graph (``lbem_batch_run``).
A solve whose last step falls in a tick is read back (E, B on the host) once
that tick completes; its memory is then released for the next admissions.

The scheduler only orders work; all arithmetic runs in liblbem's kernels.  It
talks to an *executor* (GPU: ``GpuExecutor``), so its admission, FIFO and
completion logic can also be exercised against a virtual-time test double.
"""
from __future__ import annotations

import concurrent.futures as cf
import ctypes as C
import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import lbem


# ----------------------------------------------------------------------------
# C ABI of the batch object
# ----------------------------------------------------------------------------
def _batch_lib():
    L = lbem.load()
    if not getattr(L, "_batch_typed", False):
        L.lbem_batch_create.argtypes = [C.c_int, C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]
        L.lbem_batch_run.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.c_int]
        L.lbem_batch_run_amp.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                         C.POINTER(C.c_double), C.c_int]
        L.lbem_batch_destroy.argtypes = [C.c_void_p]
        L._batch_typed = True
    return L


class Batch:
    """Advance many ``lbem.Solver`` handles together (see lbem_batch_run)."""

    def __init__(self, max_lattices: int, steps_per_tick: int, stream):
        L = _batch_lib()
        self.stream = stream
        self.k = int(steps_per_tick)
        self.max = int(max_lattices)
        h = C.c_void_p()
        rc = L.lbem_batch_create(self.max, self.k, C.c_void_p(stream.cuda_stream), C.byref(h))
        if rc != 0:
            raise lbem.LbemError(rc, "lbem_batch_create")
        self._h = h

    def run(self, solvers, nsteps, amps=None):
        """One tick: solver k advances nsteps[k] steps.  amps: per solver None
        or the source amplitudes of its steps in this tick (lbem_batch_run_amp)."""
        n = len(solvers)
        hs = (C.c_void_p * max(n, 1))(*[s._h for s in solvers])
        ns = (C.c_int64 * max(n, 1))(*[int(k) for k in nsteps])
        if amps is None or all(a is None for a in amps):
            rc = _batch_lib().lbem_batch_run(self._h, hs, ns, n)
        else:
            flat = np.zeros(max(n, 1) * self.k)
            for i, a in enumerate(amps):
                if a is not None:
                    a = np.asarray(a, np.float64).reshape(-1)
                    if a.size < int(nsteps[i]):
                        raise ValueError("amplitudes shorter than the member's steps")
                    flat[i * self.k:i * self.k + int(nsteps[i])] = a[:int(nsteps[i])]
            rc = _batch_lib().lbem_batch_run_amp(self._h, hs, ns, flat.ctypes.data_as(C.POINTER(C.c_double)), n)
        if rc != 0:
            raise lbem.LbemError(rc, "lbem_batch_run")

    def close(self):
        if getattr(self, "_h", None):
            _batch_lib().lbem_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------
# requests and the scheduler
# ----------------------------------------------------------------------------
@dataclass(eq=False)
class Request:
    rid: int
    t_arrive: float          # seconds after the start of the run
    dim: int
    n: int                   # side length
    nsteps: int
    prec: str = "f32"
    seed: int = 0
    # filled by the scheduler
    nbytes: int = 0
    remaining: int = 0
    slot: object = None
    t_admit: float = float("nan")
    t_done: float = float("nan")
    status: str = "queued"   # queued | setup | active | done | rejected | cancelled
    result: object = None

    @property
    def cells(self) -> int:
        return self.n ** self.dim


@dataclass
class Report:
    completed: int
    rejected: int
    cancelled: int
    wall_s: float
    cell_updates: float
    mlups: float
    algorithmic_gbs: float
    p50_ms: float
    p99_ms: float
    mean_ms: float
    ticks: int
    mean_resident: float
    gpu_busy_s: float        # sum of the ticks' event-timed durations on the batch stream (nan if not timed)
    max_resident: int
    latencies_ms: list = field(default_factory=list, repr=False)


def serving_streaming(prec: str) -> str:
    """Batched lattices step one step per launch, where the in-place AA pattern
    of the plain formats is the faster one (and holds one copy); the 16-bit
    formats keep pull streaming."""
    return "aa" if prec in ("f32", "f64") else "pull"


def bytes_per_update(dim: int, prec: str) -> int:
    Q, P = 2 * dim + 1, dim * (dim - 1) // 2
    if prec == "f32":
        return 2 * Q * P * 4 + 4
    if prec == "f64":
        return 2 * Q * P * 8 + 8
    slots = (Q - 1) * P - dim if "ghost" in prec else Q * P
    return 2 * ((P + dim) * 4 + slots * 2) + 4


class Scheduler:
    """Continuous batching with strict FIFO admission under a memory budget."""

    def __init__(self, executor, budget_bytes: int, max_slots: int, steps_per_tick: int,
                 keep_results: bool = False):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.k = int(steps_per_tick)
        self.keep = keep_results
        self._cancel = set()

    def cancel(self, rid: int):
        self._cancel.add(rid)

    def run(self, requests, on_tick=None) -> Report:
        ex = self.ex
        for r in requests:
            r.nbytes = int(ex.nbytes(r))
            r.remaining = r.nsteps
            r.status = "queued"
        arrivals = deque(sorted(requests, key=lambda r: (r.t_arrive, r.rid)))
        pending: deque = deque()
        setting_up = {}
        active: list = []
        inflight: deque = deque()     # per enqueued tick: requests whose last step is in it
        used = 0
        ticks = 0
        resident_sum = 0
        resident_max = 0
        done: list = []
        t0 = ex.now()

        finishing = {}               # request -> (read-back future or None, final status)

        def release(r, status):
            # read back / free off the scheduler thread; memory counts until done
            fut = ex.finish_async(r.slot, want=(status == "done")) if r.slot is not None else None
            r.slot = None
            finishing[r] = (fut, status)

        def reap(block=False):
            nonlocal used
            if block and finishing:
                futs = [f for f, _ in finishing.values() if f is not None]
                if futs and not any(ex.ready(f) for f in futs):
                    ex.wait_any(futs)
            for r in list(finishing):
                fut, status = finishing[r]
                if fut is not None and not ex.ready(fut):
                    continue
                del finishing[r]
                res, t_abs = ex.result(fut) if fut is not None else (None, ex.now())
                if status == "done" and self.keep:
                    r.result = res
                used -= r.nbytes
                r.t_done = t_abs - t0
                r.status = status
                done.append(r)

        while arrivals or pending or setting_up or active or inflight or finishing:
            reap()
            now = ex.now() - t0
            while arrivals and arrivals[0].t_arrive <= now:
                pending.append(arrivals.popleft())
            # cancellations
            if self._cancel:
                for r in [r for r in pending if r.rid in self._cancel]:
                    pending.remove(r)
                    r.status = "cancelled"
                    r.t_done = now
                    done.append(r)
                for r in [r for r in active if r.rid in self._cancel]:
                    active.remove(r)
                    r.status = "cancelling"
                    inflight.append([r])
            # strict FIFO admission: the head waits until it fits
            while pending:
                r = pending[0]
                if r.nbytes > self.budget:
                    pending.popleft()
                    r.status = "rejected"
                    r.t_done = now
                    done.append(r)
                    continue
                if len(active) + len(setting_up) >= self.max_slots or used + r.nbytes > self.budget:
                    break
                pending.popleft()
                used += r.nbytes
                r.status = "setup"
                r.t_admit = now
                setting_up[r] = ex.admit(r)
            for r in [r for r, f in setting_up.items() if ex.ready(f)]:
                r.slot = ex.result(setting_up.pop(r))
                if r.rid in self._cancel:
                    r.status = "cancelling"
                    inflight.append([r])
                else:
                    r.status = "active"
                    active.append(r)
            if active:
                ns = [min(self.k, r.remaining) for r in active]
                ex.tick([r.slot for r in active], ns)
                ticks += 1
                resident_sum += len(active)
                resident_max = max(resident_max, len(active))
                fin = []
                for r, k in zip(active, ns):
                    r.remaining -= k
                    if r.remaining == 0:
                        fin.append(r)
                active = [r for r in active if r.remaining > 0]
                inflight.append(fin)
                if on_tick:
                    on_tick(self, ticks)
            # read back what finished, keeping at most two ticks in flight
            while len(inflight) > 1 or (inflight and not active):
                for r in inflight.popleft():
                    release(r, "cancelled" if r.status == "cancelling" else "done")
            if not active and not inflight:
                if setting_up:
                    ex.wait_any(list(setting_up.values()))
                elif finishing:
                    reap(block=True)
                elif arrivals and not pending:
                    ex.sleep_until(t0 + arrivals[0].t_arrive)
                # else: memory was just released; the next pass admits the head
            elif pending and finishing and len(inflight) <= 1:
                reap()
        wall = ex.now() - t0
        ok = [r for r in done if r.status == "done"]
        lat = np.array([(r.t_done - r.t_arrive) * 1e3 for r in ok]) if ok else np.zeros(1)
        cu = float(sum(r.cells * r.nsteps for r in ok))
        by = float(sum(r.cells * r.nsteps * bytes_per_update(r.dim, r.prec) for r in ok))
        return Report(completed=len(ok), rejected=sum(r.status == "rejected" for r in done),
                      cancelled=sum(r.status == "cancelled" for r in done), wall_s=wall, cell_updates=cu,
                      mlups=cu / wall / 1e6 if wall > 0 else 0.0,
                      algorithmic_gbs=by / wall / 1e9 if wall > 0 else 0.0,
                      p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                      mean_ms=float(lat.mean()), ticks=ticks,
                      mean_resident=resident_sum / max(ticks, 1), max_resident=resident_max,
                      gpu_busy_s=float(ex.busy_seconds()) if hasattr(ex, "busy_seconds") else float("nan"),
                      latencies_ms=lat.tolist())


# ----------------------------------------------------------------------------
# GPU executor
# ----------------------------------------------------------------------------
class GpuExecutor:
    """Runs the scheduler's decisions on the GPU through liblbem.

    Set-up (medium, initial fields) runs on a small thread pool, each worker
    with its own stream, while ticks run on the batch stream."""

    def __init__(self, max_slots: int, steps_per_tick: int, workers: int = 4, w0_vac: float = 1.0 / 3.0,
                 problem_fn=None):
        import torch
        self.torch = torch
        self.stream = torch.cuda.Stream()
        self.batch = Batch(max_slots, steps_per_tick, self.stream)
        self.pool = cf.ThreadPoolExecutor(max_workers=workers)
        self.local = threading.local()
        self.w0_vac = w0_vac
        self.problem_fn = problem_fn or request_problem_fast
        self._tick_events = []
        self._bases = {}
        self._lock = threading.Lock()

    def now(self) -> float:
        return time.perf_counter()

    def sleep_until(self, t: float):
        dt = t - time.perf_counter()
        if dt > 0:
            time.sleep(dt)

    def nbytes(self, r: Request) -> int:
        shape = (r.n, r.n, 1) if r.dim == 2 else (r.n, r.n, r.n)
        return lbem.required_bytes(r.dim, shape, r.prec, streaming=serving_streaming(r.prec))

    def _stream(self):
        s = getattr(self.local, "stream", None)
        if s is None:
            s = self.torch.cuda.Stream()
            self.local.stream = s
        return s

    def _setup(self, r: Request):
        torch = self.torch
        p = self.problem_fn(r, self)
        st = self._stream()
        with torch.cuda.stream(st):
            s = lbem.Solver(p.dim, p.shape, r.prec, tau=p.tau, w0_vac=p.w0_vac,
                            streaming=serving_streaming(r.prec), stream=st)
            s.setup(p)
        return s

    def admit(self, r: Request):
        return self.pool.submit(self._setup, r)

    def ready(self, fut) -> bool:
        return fut.done()

    def result(self, fut):
        return fut.result()

    def wait_any(self, futs):
        cf.wait(futs, return_when=cf.FIRST_COMPLETED, timeout=1.0)

    def tick(self, slots, nsteps):
        # events around each tick on the batch stream; read once the run ends
        torch = self.torch
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        self.batch.run(slots, nsteps)
        e1.record(self.stream)
        self._tick_events.append((e0, e1))

    def busy_seconds(self) -> float:
        """Sum of the ticks' durations on the GPU (each from its first to its
        last kernel, upload included).  Synchronises."""
        self.torch.cuda.synchronize()
        return sum(a.elapsed_time(b) for a, b in self._tick_events) * 1e-3

    def _finish(self, s, want):
        res = s.moments() if want else None
        t = time.perf_counter()
        s.close()
        return res, t

    def finish_async(self, s, want=True):
        return self.pool.submit(self._finish, s, want)

    def close(self):
        self.pool.shutdown(wait=True)
        self.batch.close()


def base_field(ex, dim: int, n: int, rng_seed: int = 0):
    """One smooth [0,1] field per (dim, n), shared by requests of that size."""
    key = (dim, n)
    with ex._lock:
        if key not in ex._bases:
            from .inputs import smooth_noise
            rng = np.random.default_rng(1108 * 10 + 5 + 7919 * dim + n)
            shp = (n, n) if dim == 2 else (n, n, n)
            ex._bases[key] = smooth_noise(rng, shp, min(8.0, n / 8.0))
        return ex._bases[key]


def request_problem_fast(r: Request, ex):
    """Serving workload: seeded smooth eps in [1,4] (a seeded periodic shift of
    a shared smooth field of that size), one Gaussian E_z pulse (sigma 6)."""
    from .inputs import Problem, gaussian_pulse
    rng = np.random.default_rng(r.seed)
    s = base_field(ex, r.dim, r.n)
    shift = tuple(int(v) for v in rng.integers(0, r.n, s.ndim))
    eps = 1.0 + 3.0 * np.roll(s, shift, axis=tuple(range(s.ndim)))
    shape = (r.n, r.n, 1) if r.dim == 2 else (r.n, r.n, r.n)
    N = r.cells
    E = np.zeros((3, N))
    E[2] = gaussian_pulse(shape, rng.uniform(0, r.n, 3), min(6.0, r.n / 6.0)).ravel()
    return Problem(dim=r.dim, shape=shape, eps_r=eps.ravel(), mu_r=None, E0=E, B0=np.zeros((3, N)),
                   nsteps=r.nsteps, w0_vac=ex.w0_vac, name=f"req{r.rid}")


def make_requests(count: int = 2000, rate: float = 200.0, seed: int | None = None, lowp_prec: str = "f16dev",
                  **kw):
    """The serving mix as Request objects (Poisson arrivals); the requests for
    16-bit storage take `lowp_prec` (FP16 deviations by default)."""
    from .inputs import serving_requests
    out = []
    for k, d in enumerate(serving_requests(count, rate, seed, **kw)):
        out.append(Request(rid=k, t_arrive=d["t_arrive"], dim=d["dim"], n=d["n"], nsteps=d["nsteps"],
                           prec=lowp_prec if d["lowp"] else "f32", seed=d["seed"]))
    return out


def serve(requests, budget_bytes=2 << 30, max_slots=256, steps_per_tick=100, workers=4,
          keep_results=False) -> Report:
    ex = GpuExecutor(max_slots, steps_per_tick, workers=workers)
    try:
        return Scheduler(ex, budget_bytes, max_slots, steps_per_tick, keep_results=keep_results).run(requests)
    finally:
        ex.close()
