#!/usr/bin/env python3
"""Benchmark of the lattice-BGK Maxwell hot path on one MI355X.

A step is one time step of the whole hot path (gather/stream, moments,
equilibrium, source, BGK collision, store) over the full lattice.  The primary
workload is the large 3D configuration: 512^3 periodic lattice, 20 eps layers
along z with smooth lateral noise, Gaussian dipole current with a Ricker
wavelet, FP16 deviation storage (ghost coordinates, FP32 moments) with FP32
collision.  Its state (7.2 GB per copy pair) is far beyond the 256 MB Infinity
Cache, so the roofline is an HBM one.  Inputs are synthetic and resident in
HBM before timing.

Prints ONE JSON line.  `value` is MLUPS (million lattice-cell updates per
second); `roofline` prices the stream-collide kernel against the 8 TB/s HBM
peak with its algorithmic bytes; `cpu_baseline` is the FP64 CPU oracle on a
bounded sample of the same workload; `variants` holds the other formats and
sizes (3D FP32 vs 16-bit deviation storage, HBM-resident sweep points).

Extra modes used for profiling:
  --only NAME       run one workload (for rocprofv3 runs), no baseline
  --copy-calibration  a plain device copy of known size (counter calibration)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def bytes_per_cell(dim: int, prec: str, mu: bool = False) -> int:
    """Algorithmic HBM bytes per lattice update: every stored value read once
    and written once, plus the c_L^2 medium read (and the D components of
    grad ln mu when mu varies)."""
    Q, P = 2 * dim + 1, dim * (dim - 1) // 2
    tm = 8 if prec == "f64" else 4
    extra = dim * tm if mu else 0
    if prec == "f64":
        return 2 * Q * P * 8 + 8 + extra
    if prec == "f32":
        return 2 * Q * P * 4 + 4 + extra
    if prec == "f16":
        return 2 * Q * P * 2 + 4 + extra
    slots = (Q - 1) * P - dim if "ghost" in prec else Q * P
    return 2 * ((P + dim) * 4 + slots * 2) + 4 + extra


def extra_bytes(p, prec: str) -> int:
    """Algorithmic bytes per cell update of the cell extras: the absorber's
    1 - sigma, the dispersion pole's 3 coefficients read plus its 2P
    auxiliary values read and written, the D anisotropy ratios."""
    tm = 8 if prec == "f64" else 4
    P = p.dim * (p.dim - 1) // 2
    extra = 0
    if getattr(p, "sigma", None) is not None:
        extra += tm
    if getattr(p, "disp", None) is not None:
        extra += 3 * tm + 2 * (2 * P * tm)
    if getattr(p, "aniso", None) is not None:
        extra += p.dim * tm
    return extra


def _code_only(text: str) -> str:
    """C++ source without its comments and blank lines (a comment edit leaves
    the compiled code, and so a counter record, valid)."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def kernel_source_hash() -> str:
    """Hash of the device code, the host code that picks its launch geometry
    (tiling, block order) and the compiler flags, comments left out; the kernel
    instantiation is checked separately, by the kernel name recorded with the
    counters."""
    h = hashlib.sha256()
    for f in ("paper_1108_2651_amd/csrc/kernels.h", "paper_1108_2651_amd/csrc/lattice.h",
              "paper_1108_2651_amd/csrc/lbem.hip"):
        h.update(_code_only(open(os.path.join(ROOT, f), encoding="utf-8").read()).encode())
    h.update(open(os.path.join(ROOT, "paper_1108_2651_amd/build.py"), "rb").read())
    return h.hexdigest()[:16]


_CACHE = {}


def make_problem(name: str, nsteps: int):
    key = (name, nsteps)
    if key not in _CACHE:
        _CACHE.clear()
        _CACHE[key] = _make_problem(name, nsteps)
    return _CACHE[key]


def _make_problem(name: str, nsteps: int):
    from paper_1108_2651_amd import inputs as I
    if name == "c2":
        return I.config2(nsteps=nsteps)
    if name == "c1":
        return I.config1(nsteps=nsteps)
    if name.startswith("2d"):          # "2d8192": the config2 medium tiled (or cropped) periodically
        n = int(name[2:])
        p = I.config2(nsteps=nsteps)
        k = max(1, n // 2048)
        eps = np.tile(p.eps_r.reshape(2048, 2048), (k, k))[:n, :n].ravel()
        cells, w = I.line_source(n, n, 64)
        return I.Problem(dim=2, shape=(n, n, 1), eps_r=eps, mu_r=None, E0=np.zeros((3, n * n)),
                         B0=np.zeros((3, n * n)), src_comp=2, src_cells=cells, src_weights=w,
                         amp=p.amp, nsteps=nsteps, name=f"2d-hetero-{n}")
    if name == "c3":
        return I.config3(nsteps=nsteps)
    if name == "c4":
        return I.config4(nsteps=nsteps)
    if name.startswith("3d"):          # "3d128": spheres recipe at another size
        return I.config3(nsteps=nsteps, n=int(name[2:]))
    if name == "c2walls":              # config2 inside PEC walls with a 32-cell absorbing layer
        import copy
        p = copy.copy(_make_problem("c2", nsteps))
        n = p.shape[0]
        d = np.minimum(np.arange(n), n - 1 - np.arange(n)).astype(float)
        prof = np.where(d < 32, 0.05 * ((32 - d - 0.5) / 32) ** 2, 0.0)
        p.walls = [(0, "pec"), (1, "pec")]
        p.sigma = np.maximum(prof[None, :], prof[:, None]).ravel()
        p.name = p.name + "-walls-absorber"
        return p
    if name == "c3disp":               # config3 with a Lorentz pole inside the spheres
        import copy
        p = copy.copy(_make_problem("c3", nsteps))
        inside = p.eps_r > 1.0
        p.disp = (np.where(inside, 0.01, 0.0), np.where(inside, 0.002, 0.0), np.where(inside, 0.001, 0.0))
        p.name = p.name + "-lorentz"
        return p
    if name == "c3aniso":              # config3 with per-axis factors (1.2, 1.0, 0.8)
        import copy
        p = copy.copy(_make_problem("c3", nsteps))
        p.aniso = np.array([1.2, 1.0, 0.8])[:, None] * np.ones((3, p.n))
        p.name = p.name + "-anisotropic"
        return p
    if name in ("c2mu", "c3mu"):       # the same media with mu_r = 1 + (eps_r - 1)/3 as well
        import copy
        p = copy.copy(_make_problem(name[:2], nsteps))
        p.mu_r = 1.0 + (p.eps_r - 1.0) / 3.0
        p.name = p.name + "-mu"
        return p
    raise ValueError(name)


def run_workload(name: str, prec: str, steps: int, warmup: int, streaming: str = "auto", p=None):
    import torch

    from paper_1108_2651_amd import lbem
    if p is None:
        p = make_problem(name, warmup + steps)
    amp = p.amp
    if amp is None or len(amp) < warmup + steps:
        from paper_1108_2651_amd import inputs as I
        amp = I.ricker(warmup + steps, 1.0 / 80.0)
    s = lbem.Solver(p.dim, p.shape, prec, tau=p.tau, w0_vac=p.w0_vac, streaming=streaming,
                    mu_varies=p.mu_r is not None)
    walls, sigma = getattr(p, "walls", None), getattr(p, "sigma", None)
    disp, aniso = getattr(p, "disp", None), getattr(p, "aniso", None)
    for a, kind in walls or []:
        s.set_boundary(a, kind)
    s.set_medium(p.eps_r, p.mu_r)
    if aniso is not None:
        s.set_anisotropy(aniso)
    if sigma is not None:
        s.set_absorber(sigma)
    if disp is not None:
        s.set_dispersion(*disp)
    s.init_fields(p.E0, p.B0)
    if len(p.src_cells):
        s.set_source(p.src_comp, p.src_cells, p.src_weights)
    spl = s.steps_per_launch
    stream = torch.cuda.current_stream()
    s.step(warmup, amp[:warmup])
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    s.step(steps, amp[warmup:warmup + steps])
    e1.record(stream)
    e1.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    diag = s.energy(check=False)
    n = p.n
    bpc = bytes_per_cell(p.dim, prec, p.mu_r is not None) + extra_bytes(p, prec)
    st = streaming if streaming != "auto" else "pull"
    bpu = bpc / max(spl, 1)        # HBM bytes per cell update when spl steps share one pass
    mlups = n * steps / (ms * 1e-3) / 1e6
    gbs = bpu * n * steps / (ms * 1e-3) / 1e9
    res = dict(workload=p.name, dim=p.dim, shape=list(p.shape), prec=prec, streaming=st,
               steps_per_launch=spl, steps=steps, warmup=warmup, ms_per_step=ms / steps, mlups=mlups,
               bytes_per_cell=bpc, bytes_per_update=bpu, algorithmic_gbs=gbs, hbm_frac=gbs / HBM_PEAK_GBS,
               avg_launch_us=ms * 1e3 / steps, wall_s=wall, finite=diag["status"] == 0,
               arena_gb=s.arena_bytes / 1e9)
    s.close()
    del s
    torch.cuda.empty_cache()
    return res


# the headline: config 4 with FP16 deviation storage in ghost coordinates
PRIMARY_PREC = "f16ghost"
PRIMARY_KERNEL = "k_step_dev3r<__half,ghost,mu=0,nts=1,cx=2,512,ext=0>"
PRIMARY_TRAFFIC = "c4_512_f16ghost"
CPU_SAMPLE_CROP = 128


def cpu_baseline(crop: int, budget_s: float = 15.0) -> dict:
    """The FP64 oracle as it stands, all host cores, on a bounded sample of the
    primary workload: the centred crop^3 box of the config-4 medium with its
    dipole (the full 512^3 lattice would need ~135 GB for the oracle's full
    D x D tensor state), for as many steps as fit the time budget.  MLUPS are
    per cell update, so the sample's rate stands for the full lattice's."""
    from oracle import oracle as O
    from paper_1108_2651_amd import inputs as I
    p = I.config4(nsteps=2000, crop_n=crop)
    cores = O.set_threads(os.cpu_count() or 1)
    o = O.Oracle(p.dim, p.shape, p.tau, p.w0_vac)
    o.set_medium(p.eps_r, p.mu_r)
    o.init_fields(p.E0, p.B0)
    o.set_source(p.src_comp, p.src_cells, p.src_weights)
    t = time.perf_counter()
    o.step(2, p.amp[:2])
    per = (time.perf_counter() - t) / 2
    k = max(1, min(len(p.amp) - 2, int(budget_s / max(per, 1e-9))))
    t = time.perf_counter()
    o.step(k, p.amp[2:2 + k])
    el = time.perf_counter() - t
    return dict(value=p.n * k / el / 1e6, unit="MLUPS", cores=cores, kind="oracle",
                sample=f"config-4 medium and dipole, centred {crop}^3 crop as its own periodic box, FP64 "
                       f"full-tensor oracle, {k} steps ({el:.1f} s) after 2 untimed",
                seconds=el)


def cpu_baseline_table(budget_s: float = 4.0) -> list:
    """The FP64 oracle timed at one thread and at all host cores on the small
    configurations: 2D 128^2 (FP64 pulse), 2D 2048^2 (the primary workload)
    and the 64^3 centred crops of the two 3D media."""
    from oracle import oracle as O
    from paper_1108_2651_amd import inputs as I
    allc = os.cpu_count() or 1
    rows = []
    probs = [("c1 128^2", I.config1(nsteps=400)), ("c2 2048^2", I.config2(nsteps=400)),
             ("c3 64^3 crop", I.config3(nsteps=400, crop_n=64)), ("c4 64^3 crop", I.config4(nsteps=400, crop_n=64))]
    for label, p in probs:
        for threads in (1, allc):
            used = O.set_threads(threads)
            o = O.Oracle(p.dim, p.shape, p.tau, p.w0_vac)
            o.set_medium(p.eps_r, p.mu_r)
            o.init_fields(p.E0, p.B0)
            has_src = len(p.src_cells) > 0
            if has_src:
                o.set_source(p.src_comp, p.src_cells, p.src_weights)
            amp = p.amp if has_src else None
            t = time.perf_counter()
            o.step(1, amp[:1] if has_src else None)
            per = time.perf_counter() - t
            k = max(1, min(390, int(budget_s / max(per, 1e-9))))
            t = time.perf_counter()
            o.step(k, amp[1:1 + k] if has_src else None)
            el = time.perf_counter() - t
            rows.append(dict(workload=label, threads=used, steps=k, seconds=el,
                             mlups=p.n * k / el / 1e6))
            print(f"[bench] oracle {label} threads={used}: {rows[-1]['mlups']:.2f} MLUPS", file=sys.stderr,
                  flush=True)
    O.set_threads(allc)
    return rows


def size_sweep(steps: int = 100, warmup: int = 5) -> list:
    """Roofline sweep across the Infinity-Cache boundary: 3D spheres medium
    from 64^3 to 512^3 in FP32 (pull, fused pair; AA single steps), plain
    FP16 storage (AA single steps) and the two 16-bit deviation formats; 2D
    from 512^2 to 8192^2 in FP32 (fused and AA) and the two deviation formats."""
    rows = []
    plan = [(f"3d{n}", prec, st) for n in (64, 96, 128, 160, 192, 256, 320, 384, 448, 512)
            for prec, st in (("f32", "pull"), ("f32", "aa"), ("f16", "aa"), ("f16dev", "pull"), ("f16ghost", "pull"))]
    plan += [(f"2d{n}", prec, st) for n in (512, 1024, 2048, 4096, 8192)
             for prec, st in (("f32", "pull"), ("f32", "aa"), ("f16dev", "pull"), ("f16ghost", "pull"))]
    for name, prec, st in plan:
        n = int(name[2:])
        k = max(20, min(steps * 8, int(steps * (256 ** 3 if name.startswith("3d") else 2048 ** 2) /
                                           (n ** 3 if name.startswith("3d") else n * n))))
        try:
            r = run_workload(name, prec, k, warmup, st, p=make_problem(name, 1100))
        except Exception as e:  # report, do not hide
            r = dict(workload=name, prec=prec, streaming=st, error=str(e))
        print(json.dumps(r), flush=True)
        rows.append(r)
    return rows


SERVING_CONFIG = ("Poisson arrivals; 70% 2D 64^2-1024^2, 30% 3D 32^3-128^3; smooth eps in [1,4]; "
                  "200-2000 steps; half FP32, half FP16-dev (the *_f16ghost row: FP16 ghost coordinates); "
                  "2 GiB device budget; 100 steps per tick; latency = arrival to E,B on the host")


def serving_run(rate: float, count: int, lowp_prec: str = "f16dev") -> dict:
    """The continuous-batching serving mix at `rate` requests/s (its 16-bit
    requests in `lowp_prec`)."""
    from paper_1108_2651_amd import serve as SV
    reqs = SV.make_requests(count=count, rate=rate, lowp_prec=lowp_prec)
    rep = SV.serve(reqs, budget_bytes=2 << 30, max_slots=256, steps_per_tick=100, workers=10)
    return dict(requests=len(reqs), completed=rep.completed, rejected=rep.rejected,
                p50_ms=rep.p50_ms, p99_ms=rep.p99_ms, mean_ms=rep.mean_ms, wall_s=rep.wall_s,
                mlups=rep.mlups, algorithmic_gbs=rep.algorithmic_gbs, ticks=rep.ticks,
                gpu_busy_s=rep.gpu_busy_s, gpu_busy_frac=rep.gpu_busy_s / rep.wall_s if rep.wall_s > 0 else None,
                mean_resident=rep.mean_resident, max_resident=rep.max_resident,
                offered_mlups=sum(r.cells * r.nsteps for r in reqs) / reqs[-1].t_arrive / 1e6)


def batch_classes(ticks: int = 10, warmup: int = 3, k: int = 50) -> list:
    """Each batched class of the serving mix on its own: 20 resident lattices
    of the mix's sizes (2D 64^2 - 1024^2 or 3D 32^3 - 128^3, four of each
    side), one batch, `ticks` ticks of `k` steps event-timed on the batch
    stream; beside it the same lattices stepped one by one with lbem_step."""
    import torch
    from paper_1108_2651_amd import inputs as I, lbem, serve as SV
    rows = []
    plan = [(2, "f32", "aa"), (2, "f16dev", "pull"), (3, "f32", "aa"), (3, "f16dev", "pull"),
            (3, "f16ghost", "pull")]
    for dim, prec, st in plan:
        sides = (64, 128, 256, 512, 1024) if dim == 2 else (32, 48, 64, 96, 128)
        rng = np.random.default_rng(11)
        stream = torch.cuda.Stream()
        solvers = []
        for n in sides:
            shp = (n, n) if dim == 2 else (n, n, n)
            eps = 1.0 + 3.0 * I.smooth_noise(rng, shp, min(8.0, n / 8.0))
            p = I.pulse_problem(dim, n, min(6.0, n / 6.0), rng, eps=eps)
            for _ in range(4):
                s = lbem.Solver(dim, p.shape, prec, streaming=st, stream=stream)
                s.setup(p)
                solvers.append(s)
        cells = sum(s.n for s in solvers)
        batch = SV.Batch(len(solvers), k, stream)
        for _ in range(warmup):
            batch.run(solvers, [k] * len(solvers))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(ticks):
            batch.run(solvers, [k] * len(solvers))
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        batched = cells * k * ticks / (ms * 1e-3) / 1e6
        # the same lattices one by one (their own kernels, single handles)
        with torch.cuda.stream(stream):
            for s in solvers[::4]:
                s.step(k)
            f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            f0.record(stream)
            for s in solvers:
                s.step(k)
            f1.record(stream)
        f1.synchronize()
        solo = cells * k / (f0.elapsed_time(f1) * 1e-3) / 1e6
        row = dict(dim=dim, prec=prec, streaming=st, lattices=len(solvers), cells=cells, steps_per_tick=k,
                   ms_per_tick=ms / ticks, batched_mlups=batched, solo_mlups=solo,
                   batched_gbs=batched * bytes_per_cell(dim, prec) / 1e3)
        print(json.dumps(row), flush=True)
        rows.append(row)
        batch.close()
        for s in solvers:
            s.close()
    return rows


def load_traffic(name: str, kernel: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current device code with the same kernel instantiation."""
    f = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    if not os.path.exists(f):
        return None
    d = json.load(open(f))
    if d.get("kernel_source_hash") != kernel_source_hash() or d.get("kernel") != kernel:
        return None
    return d.get("bytes_per_launch")


def copy_calibration(gib: float = 1.0, reps: int = 8):
    import torch
    n = int(gib * (1 << 30))
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": n, "reps": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-lowp", default="f16dev", help="format of the mix's 16-bit requests")
    ap.add_argument("--only", default=None, help="workload:prec[:streaming], e.g. c2:f32 or c3:f16dev")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--sweep", action="store_true", help="size sweep (one JSON line per point) instead")
    ap.add_argument("--batch-classes", action="store_true",
                    help="each batched serving class on its own, against the same lattices stepped alone")
    ap.add_argument("--oracle-table", action="store_true",
                    help="time the oracle at 1 thread and all cores on the small configurations instead")
    ap.add_argument("--serve-only", type=float, default=None, metavar="RATE",
                    help="run only the serving mix at RATE requests/s (one JSON line)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU slab decomposition is a design note, not an implemented path.", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    if args.copy_calibration:
        copy_calibration()
        return

    if args.oracle_table:
        print(json.dumps({"cpu_baseline_table": cpu_baseline_table()}), flush=True)
        return

    if args.sweep:
        size_sweep()
        return

    if args.batch_classes:
        batch_classes()
        return

    if args.only:
        parts = args.only.split(":")
        r = run_workload(parts[0], parts[1], args.steps, args.warmup,
                         parts[2] if len(parts) > 2 else "auto")
        print(json.dumps(r), flush=True)
        return

    if args.serve_only is not None:
        print(json.dumps(serving_run(args.serve_only, args.serve_requests, args.serve_lowp)), flush=True)
        return

    print(f"[bench] primary: config4 512^3 {PRIMARY_PREC}", file=sys.stderr, flush=True)
    nprob = max(args.warmup + args.steps, 1100)
    p = make_problem("c4", nprob)
    prim = run_workload("c4", PRIMARY_PREC, args.steps, args.warmup, p=p)

    variants = []
    if not args.no_variants:
        # grouped by workload so each medium is generated once
        plan = [("c4", "f16dev", "pull", 200, 5), ("c4", "bf16ghost", "pull", 200, 5),
                ("c4", "f32", "pull", 200, 6), ("c4", "f32", "aa", 200, 5), ("c4", "f16", "aa", 200, 5),
                ("c3", "f32", "pull", 400, 10), ("c3", "f32", "aa", 400, 10),
                ("c3", "f16dev", "pull", 400, 10), ("c3", "f16ghost", "pull", 400, 10),
                ("c3", "bf16dev", "pull", 400, 10), ("c3", "f16", "aa", 400, 10),
                ("c2", "f32", "pull", 2000, 20), ("c2", "f32", "aa", 2000, 20),
                ("2d8192", "f32", "pull", 200, 10), ("2d8192", "f32", "aa", 200, 10),
                ("2d8192", "f16ghost", "pull", 200, 10),
                ("c2mu", "f32", "pull", 1000, 20), ("c3mu", "f32", "auto", 200, 10),
                ("c3mu", "f16ghost", "pull", 200, 10), ("c2walls", "f32", "pull", 1000, 20),
                ("c3disp", "f32", "pull", 200, 10), ("c3disp", "f16ghost", "pull", 200, 10),
                ("c3aniso", "f32", "pull", 200, 10)]
        for name, prec, st, k, w in plan:
            print(f"[bench] variant {name} {prec} {st}", file=sys.stderr, flush=True)
            try:
                r = run_workload(name, prec, k, w, st, p=make_problem(name, nprob if name == "c4" else 1100))
                if name == "c2":
                    r["note"] = ("2048^2 state (101-185 MB) fits the 256 MB Infinity Cache: not an HBM point; "
                                 "the FP32 pull default runs four steps per launch and is bound by vector-ALU "
                                 "issue (0.69 of the VALU issue slots, profiles/k_step_stream_collide.md)")
                variants.append(r)
            except Exception as e:  # report, do not hide
                variants.append(dict(workload=name, prec=prec, streaming=st, error=str(e)))

    serving = None
    if not args.no_serving:
        serving = {}
        for rate in (200.0, 100.0):
            print(f"[bench] serving mix at {rate:.0f} req/s", file=sys.stderr, flush=True)
            serving[f"{rate:.0f}_req_per_s"] = serving_run(rate, args.serve_requests)
        # the same requests with the 16-bit ones in ghost coordinates
        print("[bench] serving mix at 200 req/s, FP16 ghost", file=sys.stderr, flush=True)
        serving["200_req_per_s_f16ghost"] = serving_run(200.0, args.serve_requests, "f16ghost")
        serving["config"] = SERVING_CONFIG

    cpu = None
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(CPU_SAMPLE_CROP)

    # one launch = one time step of the whole lattice: the kernel reads the
    # stored state (FP32 moments + 15 FP16 ghost codes per cell) and c_L^2 once
    # and writes the new state once, 112 B per cell update
    spl = prim["steps_per_launch"]
    launch_us = prim["avg_launch_us"] * spl
    achieved = prim["bytes_per_cell"] * p.n / (launch_us * 1e-6) / 1e9
    out = {
        "metric": "MLUPS",
        "value": prim["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": prim["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3D large heterogeneous medium: 512^3 periodic lattice, 20 eps layers along z "
                               "(eps in [1,6]) with +-10% smooth lateral noise, Gaussian dipole j_z with a "
                               "Ricker wavelet at the centre; FP16 deviation storage (ghost coordinates, "
                               "FP32 moments) with FP32 collision, pull streaming",
                   "shape": list(p.shape), "format": PRIMARY_PREC, "storage": "fp16 codes + fp32 moments",
                   "arithmetic": "fp32"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": load_traffic(PRIMARY_TRAFFIC, PRIMARY_KERNEL),
                     "kernel": PRIMARY_KERNEL, "steps_per_launch": spl, "avg_launch_us": launch_us,
                     "bytes_per_cell_per_launch": prim["bytes_per_cell"], "cells_per_launch": p.n,
                     "bytes_per_cell_update": prim["bytes_per_cell"] / spl,
                     "note": "algorithmic bytes (section 8(d)): 2 x (6 x 4 B moments + 15 x 2 B codes) + 4 B c_L^2 "
                             "per cell update; event-timed over the timed steps on the launch stream"},
        "cpu_baseline": cpu,
        "hbm_frac": prim["hbm_frac"],
        "finite": prim["finite"],
        "kernel_source_hash": kernel_source_hash(),
        "variants": variants,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
