"""Thin ctypes binding of liblbem (C ABI in include/lbem.h).

Argument marshalling only: every step of the solver runs in the HIP kernels
of liblbem.so.  PyTorch supplies device memory (the handle's arena) and the
stream.  There is no fallback: if the library has not been built, or no GPU
is present, the calls fail loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "liblbem.so")

LBEM_OK, LBEM_EINVAL, LBEM_ENOMEM, LBEM_EUNSTABLE, LBEM_ENONFINITE, LBEM_EDEVICE, LBEM_ESTATE = (
    0, -1, -2, -3, -4, -5, -6)
LBEM_ETOOBIG = -7
NOALLOC_MAX_CELLS = 2781712      # LBEM_NOALLOC_MAX_CELLS of include/lbem.h
PREC = {"f64": 0, "f32": 1, "f16dev": 2, "bf16dev": 3, "f16ghost": 4, "bf16ghost": 5, "f16": 6}
STREAMING = {"auto": 0, "pull": 1, "aa": 2}

# every entry point of include/lbem.h
SYMBOLS = ("lbem_required_bytes", "lbem_create", "lbem_destroy", "lbem_set_medium",
           "lbem_init_fields", "lbem_set_source", "lbem_step", "lbem_moments", "lbem_energy",
           "lbem_time", "lbem_strerror", "lbem_batch_create", "lbem_batch_run", "lbem_batch_destroy",
           "lbem_steps_per_launch", "lbem_state_bytes", "lbem_get_state", "lbem_set_state",
           "lbem_set_boundary", "lbem_set_absorber", "lbem_set_dispersion", "lbem_set_anisotropy",
           "lbem_energy_noalloc", "lbem_batch_run_amp")
BOUNDARY = {"periodic": 0, "pec": 1, "pmc": 2}


class Config(C.Structure):
    _fields_ = [("dim", C.c_int), ("prec", C.c_int), ("nx", C.c_int64), ("ny", C.c_int64),
                ("nz", C.c_int64), ("tau", C.c_double), ("w0_vac", C.c_double),
                ("streaming", C.c_int), ("mu_varies", C.c_int), ("stream", C.c_void_p),
                ("dev_mem", C.c_void_p), ("dev_bytes", C.c_size_t)]


class LbemError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


_lib = None


def load():
    """Load liblbem.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"liblbem.so not found at {LIB_PATH}: build it first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    L = C.CDLL(LIB_PATH)
    vp, dp, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int64
    L.lbem_required_bytes.argtypes = [C.POINTER(Config)]
    L.lbem_required_bytes.restype = C.c_size_t
    L.lbem_create.argtypes = [C.POINTER(Config), C.POINTER(vp)]
    L.lbem_destroy.argtypes = [vp]
    L.lbem_set_medium.argtypes = [vp, vp, vp]
    L.lbem_init_fields.argtypes = [vp, vp, vp]
    L.lbem_set_source.argtypes = [vp, C.c_int, vp, vp, i64]
    L.lbem_step.argtypes = [vp, i64, vp]
    L.lbem_moments.argtypes = [vp, vp, vp, C.c_int]
    L.lbem_energy.argtypes = [vp, dp]
    L.lbem_energy_noalloc.argtypes = [vp, dp]
    L.lbem_time.argtypes = [vp]
    L.lbem_time.restype = i64
    L.lbem_steps_per_launch.argtypes = [vp]
    L.lbem_state_bytes.argtypes = [vp]
    L.lbem_state_bytes.restype = C.c_size_t
    L.lbem_get_state.argtypes = [vp, vp, C.c_size_t, C.c_int]
    L.lbem_set_state.argtypes = [vp, vp, C.c_size_t, C.c_int]
    L.lbem_set_boundary.argtypes = [vp, C.c_int, C.c_int]
    L.lbem_set_absorber.argtypes = [vp, vp]
    L.lbem_set_dispersion.argtypes = [vp, vp, vp, vp]
    L.lbem_set_anisotropy.argtypes = [vp, vp]
    L.lbem_strerror.argtypes = [C.c_int]
    L.lbem_strerror.restype = C.c_char_p
    _lib = L
    return L


def strerror(code: int) -> str:
    try:
        return load().lbem_strerror(int(code)).decode()
    except RuntimeError:
        return f"status {code}"


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def make_config(dim, shape, prec="f32", tau=0.5, w0_vac=1.0 / 3.0, streaming="auto",
                mu_varies=False, stream=None, dev_mem=None, dev_bytes=0) -> Config:
    nx, ny, nz = shape
    return Config(dim=int(dim), prec=PREC[prec] if isinstance(prec, str) else int(prec),
                  nx=int(nx), ny=int(ny), nz=int(nz), tau=float(tau), w0_vac=float(w0_vac),
                  streaming=STREAMING[streaming] if isinstance(streaming, str) else int(streaming),
                  mu_varies=int(bool(mu_varies)), stream=stream, dev_mem=dev_mem,
                  dev_bytes=int(dev_bytes))


def required_bytes(dim, shape, prec="f32", **kw) -> int:
    cfg = make_config(dim, shape, prec, **kw)
    return int(load().lbem_required_bytes(C.byref(cfg)))


class Solver:
    """One lattice-BGK Maxwell solve on the current CUDA/HIP device.

    ``prec`` names the storage format (a key of PREC: "f64", "f32", the 16-bit
    deviation formats "f16dev"/"bf16dev", the ghost-coordinate formats
    "f16ghost"/"bf16ghost", or plain "f16"); ``streaming`` is "auto", "pull" or
    "aa".  The device arena is a torch uint8 tensor; launches go to torch's
    current stream (or ``stream``, a torch.cuda.Stream)."""

    def __init__(self, dim, shape, prec="f32", tau=0.5, w0_vac=1.0 / 3.0, streaming="auto",
                 mu_varies=False, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("liblbem needs a GPU (torch.cuda.is_available() is False)")
        L = load()
        self.dim, self.shape = int(dim), tuple(int(s) for s in shape)
        self.n = self.shape[0] * self.shape[1] * self.shape[2]
        self.prec = prec
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        cfg = make_config(dim, shape, prec, tau, w0_vac, streaming, mu_varies,
                          stream=C.c_void_p(self._stream.cuda_stream))
        nbytes = int(L.lbem_required_bytes(C.byref(cfg)))
        if nbytes == 0:
            raise LbemError(LBEM_EINVAL, "lbem_required_bytes")
        self._arena = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self._arena.data_ptr()
        aligned = (base + 255) & ~255
        cfg.dev_mem = C.c_void_p(aligned)
        cfg.dev_bytes = nbytes
        self.arena_bytes = nbytes
        h = C.c_void_p()
        self._chk(L.lbem_create(C.byref(cfg), C.byref(h)), "lbem_create")
        self._h = h

    def _chk(self, rc, where):
        if rc != LBEM_OK:
            raise LbemError(rc, where)

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            load().lbem_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- problem set-up -------------------------------------------------
    def _setup_call(self, fn, *args, where=""):
        """A set-up call stages host arrays through device buffers of its own;
        if the device is out of memory because torch's caching allocator still
        holds freed arenas, release them once and retry."""
        rc = fn(self._h, *args)
        if rc == LBEM_ENOMEM:
            import torch
            torch.cuda.empty_cache()
            rc = fn(self._h, *args)
        self._chk(rc, where)

    def set_medium(self, eps_r, mu_r=None):
        e = _f64(eps_r, self.n)
        m = None if mu_r is None else _f64(mu_r, self.n)
        self._setup_call(load().lbem_set_medium, _ptr(e), _ptr(m), where="lbem_set_medium")

    def init_fields(self, E, B):
        e = _f64(E, 3 * self.n)
        b = _f64(B, 3 * self.n)
        self._setup_call(load().lbem_init_fields, _ptr(e), _ptr(b), where="lbem_init_fields")

    def set_boundary(self, axis: int, kind: str):
        """Walls on both faces of ``axis``: 'pec', 'pmc' or 'periodic' (before
        set_medium)."""
        self._chk(load().lbem_set_boundary(self._h, int(axis), BOUNDARY[kind]), "lbem_set_boundary")

    def set_absorber(self, sigma=None):
        """Absorbing layer sigma(x) in [0,1) per cell; None removes it."""
        s = None if sigma is None else _f64(sigma, self.n)
        self._chk(load().lbem_set_absorber(self._h, _ptr(s)), "lbem_set_absorber")

    def set_anisotropy(self, factors):
        """Per-axis factors [dim][n] (or [dim], broadcast) on the isotropic c_L^2
        (after set_medium, before init_fields)."""
        f = np.ascontiguousarray(np.broadcast_to(np.asarray(factors, np.float64).reshape(self.dim, -1),
                                                 (self.dim, self.n)))
        self._chk(load().lbem_set_anisotropy(self._h, _ptr(f)), "lbem_set_anisotropy")

    def set_dispersion(self, wp2=None, w02=None, gamma=None):
        """One Lorentz pole per cell (lattice units); scalars broadcast; wp2=None
        removes it."""
        if wp2 is None:
            self._chk(load().lbem_set_dispersion(self._h, None, None, None), "lbem_set_dispersion")
            return
        a = [None if v is None else _f64(np.broadcast_to(np.asarray(v, np.float64), (self.n,)))
             for v in (wp2, w02, gamma)]
        self._chk(load().lbem_set_dispersion(self._h, *[_ptr(v) for v in a]), "lbem_set_dispersion")

    def set_source(self, comp, cells, weights):
        c = np.ascontiguousarray(cells, dtype=np.int64).reshape(-1)
        w = _f64(weights, c.size)
        self._chk(load().lbem_set_source(self._h, int(comp), _ptr(c), _ptr(w), c.size), "lbem_set_source")

    def setup(self, p):
        """Medium, fields and source of an ``inputs.Problem``."""
        self.set_medium(p.eps_r, p.mu_r)
        self.init_fields(p.E0, p.B0)
        if len(p.src_cells):
            self.set_source(p.src_comp, p.src_cells, p.src_weights)
        return self

    # -- time stepping ----------------------------------------------------
    def step(self, nsteps: int, amp=None):
        a = None if amp is None else _f64(amp)
        if a is not None and a.size < nsteps:
            raise ValueError("amp shorter than nsteps")
        self._chk(load().lbem_step(self._h, int(nsteps), _ptr(a)), "lbem_step")

    # -- outputs ------------------------------------------------------------
    def moments(self):
        """(E, B) as numpy (3, n) float64 arrays at the current time."""
        E = np.empty((3, self.n))
        B = np.empty((3, self.n))
        self._chk(load().lbem_moments(self._h, _ptr(E), _ptr(B), 0), "lbem_moments")
        return E, B

    def moments_device(self, E, B):
        """Write E, B into device tensors (float64, 3*n elements each)."""
        self._chk(load().lbem_moments(self._h, C.c_void_p(E.data_ptr()) if E is not None else None,
                                      C.c_void_p(B.data_ptr()) if B is not None else None, 1),
                  "lbem_moments")

    def energy(self, check=True) -> dict:
        out = np.zeros(4)
        rc = load().lbem_energy(self._h, out.ctypes.data_as(C.POINTER(C.c_double)))
        if check:
            self._chk(rc, "lbem_energy")
        return dict(energy=out[0], qc=out[1], divb2=out[2], b2=out[3], status=rc)

    def energy_noalloc(self, check=True) -> dict:
        """lbem_energy_noalloc: the same diagnostics with the library's static
        device scratch (no allocation; lattices up to NOALLOC_MAX_CELLS)."""
        out = np.zeros(4)
        rc = load().lbem_energy_noalloc(self._h, out.ctypes.data_as(C.POINTER(C.c_double)))
        if check:
            self._chk(rc, "lbem_energy_noalloc")
        return dict(energy=out[0], qc=out[1], divb2=out[2], b2=out[3], status=rc)

    # -- checkpoint / resume -------------------------------------------------
    def state_bytes(self) -> int:
        return int(load().lbem_state_bytes(self._h))

    def get_state(self, out=None):
        """The exact state blob: into ``out`` (a uint8 numpy array, or a uint8
        device tensor) if given, else a new numpy array."""
        nb = self.state_bytes()
        if out is None:
            out = np.empty(nb, dtype=np.uint8)
        if isinstance(out, np.ndarray):
            self._chk(load().lbem_get_state(self._h, _ptr(out), out.nbytes, 0), "lbem_get_state")
        else:
            self._chk(load().lbem_get_state(self._h, C.c_void_p(out.data_ptr()), out.numel(), 1),
                      "lbem_get_state")
        return out

    def set_state(self, blob):
        """Restore a blob from ``get_state`` (numpy uint8 array or device tensor)."""
        if isinstance(blob, np.ndarray):
            b = np.ascontiguousarray(blob, dtype=np.uint8)
            self._chk(load().lbem_set_state(self._h, _ptr(b), b.nbytes, 0), "lbem_set_state")
        else:
            self._chk(load().lbem_set_state(self._h, C.c_void_p(blob.data_ptr()), blob.numel(), 1),
                      "lbem_set_state")

    @property
    def t(self) -> int:
        return int(load().lbem_time(self._h))

    @property
    def steps_per_launch(self) -> int:
        return int(load().lbem_steps_per_launch(self._h))
