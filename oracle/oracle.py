"""Python view of the FP64 CPU oracle (``lbem_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  Nothing here is shared with, or called
by, the HIP path.

``Oracle`` runs the paper's lattice-BGK scheme literally (full D x D
antisymmetric tensor per velocity, FP64, eqs. distrib.func, COLLI, STREAM);
``equilibrium`` and ``collide`` expose the single-cell pieces so that the
closed-form identities of the lattice section (relate.1-3, CONSERV) can be
checked directly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    """The oracle library.  LBEM_ORACLE_LIB names another build of the same
    source (the tests that plant mistakes in the oracle load their mutants
    this way); by default the in-tree build, compiled on first use."""
    global _lib
    if _lib is None:
        path = os.environ.get("LBEM_ORACLE_LIB") or _build.LIB
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.c_int, C.c_long, C.c_long, C.c_long, C.c_double, C.c_double]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = C.c_int
        L.orc_set_medium.argtypes = [C.c_void_p, dp, C.c_void_p]
        L.orc_init_fields.argtypes = [C.c_void_p, dp, dp]
        L.orc_set_source.argtypes = [C.c_void_p, C.c_long, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.c_long, C.c_void_p]
        L.orc_fields.argtypes = [C.c_void_p, dp, dp]
        L.orc_diag.argtypes = [C.c_void_p, dp]
        L.orc_time.argtypes = [C.c_void_p]
        L.orc_time.restype = C.c_long
        L.orc_state_size.argtypes = [C.c_void_p]
        L.orc_state_size.restype = C.c_long
        L.orc_get_state.argtypes = [C.c_void_p, dp]
        L.orc_set_state.argtypes = [C.c_void_p, dp]
        L.orc_get_medium.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.orc_equilibrium.argtypes = [C.c_int, C.c_double, dp, dp, dp]
        L.orc_collide.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp, dp]
        L.orc_velocities.argtypes = [C.c_int, np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")]
        L.orc_set_boundary.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.orc_set_absorber.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_set_dispersion.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_set_anisotropy.argtypes = [C.c_void_p, dp]
        L.orc_polarisation.argtypes = [C.c_void_p, dp, dp]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}")
        self.code = code


def _chk(rc):
    if rc != 0:
        raise OracleError(rc)


def set_threads(k: int = 0) -> int:
    """Set the OpenMP thread count (k<=0: keep) and return the count in use."""
    return lib().orc_set_threads(int(k))


def velocities(dim: int) -> np.ndarray:
    out = np.zeros((2 * dim + 1, 3), np.int32)
    _chk(lib().orc_velocities(dim, out))
    return out


def equilibrium(dim: int, w0: float, Lam: np.ndarray, Bbar: np.ndarray) -> np.ndarray:
    """g0_{i,a,b} of eq. distrib.func for one cell, shape (Q, D, D)."""
    Q = 2 * dim + 1
    out = np.zeros((Q, dim, dim))
    _chk(lib().orc_equilibrium(dim, float(w0), np.ascontiguousarray(Lam, np.float64).ravel(),
                               np.ascontiguousarray(Bbar, np.float64).ravel(), out.reshape(-1)))
    return out


def collide(dim: int, w0: float, tau: float, g: np.ndarray, S=None) -> np.ndarray:
    """One cell's post-collision state (eq. COLLI), shape (Q, D, D)."""
    S = np.zeros(3) if S is None else np.asarray(S, np.float64)
    out = np.zeros_like(np.asarray(g, np.float64))
    _chk(lib().orc_collide(dim, float(w0), float(tau), np.ascontiguousarray(g, np.float64).ravel(),
                           np.ascontiguousarray(S), out.reshape(-1)))
    return out


class Oracle:
    """FP64 full-tensor lattice-BGK Maxwell solver on a periodic box."""

    def __init__(self, dim: int, shape, tau: float = 0.5, w0_vac: float = 1.0 / 3.0):
        nx, ny, nz = shape
        self.dim, self.shape, self.n = dim, (nx, ny, nz), nx * ny * nz
        self.Q = 2 * dim + 1
        self._h = lib().orc_create(dim, nx, ny, nz, tau, w0_vac)
        if not self._h:
            raise OracleError(-1)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def set_medium(self, eps_r, mu_r=None):
        eps = np.ascontiguousarray(eps_r, np.float64).ravel()
        if mu_r is None:
            _chk(lib().orc_set_medium(self._h, eps, None))
        else:
            mu = np.ascontiguousarray(mu_r, np.float64).ravel()
            _chk(lib().orc_set_medium(self._h, eps, mu.ctypes.data_as(C.c_void_p)))

    BOUNDARY = {"periodic": 0, "pec": 1, "pmc": 2}

    def set_boundary(self, axis: int, kind: str):
        """Walls on both faces of ``axis`` (before set_medium): 'pec' (the box's
        mirror image, tangential E odd), 'pmc' (the opposite), 'periodic'."""
        _chk(lib().orc_set_boundary(self._h, int(axis), self.BOUNDARY[kind]))

    def set_absorber(self, sigma=None):
        """Absorbing layer: every post-collision population of a cell is
        multiplied by 1 - sigma(x); None removes it."""
        if sigma is None:
            _chk(lib().orc_set_absorber(self._h, None))
        else:
            s = np.ascontiguousarray(sigma, np.float64).ravel()
            _chk(lib().orc_set_absorber(self._h, s.ctypes.data_as(C.c_void_p)))

    def set_anisotropy(self, factors):
        """Per-axis factors a[axis][cell] > 0 on the isotropic c_L^2 of the
        medium (after set_medium; set_medium again restores isotropy)."""
        f = np.ascontiguousarray(np.broadcast_to(np.asarray(factors, np.float64).reshape(self.dim, -1),
                                                 (self.dim, self.n)))
        _chk(lib().orc_set_anisotropy(self._h, f.reshape(-1)))

    def set_dispersion(self, wp2=None, w02=None, gamma=None):
        """One Lorentz pole per cell, chi(w) = wp2/(w02 - w^2 - i gamma w)
        relative to the cell's permittivity (lattice units); wp2=None removes
        it.  Scalars broadcast over the cells."""
        if wp2 is None:
            _chk(lib().orc_set_dispersion(self._h, None, None, None))
            return
        arrs = [np.ascontiguousarray(np.broadcast_to(np.asarray(v, np.float64), (self.n,)))
                for v in (wp2, 0.0 if w02 is None else w02, 0.0 if gamma is None else gamma)]
        self._disp = arrs
        _chk(lib().orc_set_dispersion(self._h, *[a.ctypes.data_as(C.c_void_p) for a in arrs]))

    def polarisation(self):
        P = np.zeros((3, self.n))
        J = np.zeros((3, self.n))
        _chk(lib().orc_polarisation(self._h, P.reshape(-1), J.reshape(-1)))
        return P, J

    def init_fields(self, E, B):
        _chk(lib().orc_init_fields(self._h, np.ascontiguousarray(E, np.float64).reshape(-1),
                                   np.ascontiguousarray(B, np.float64).reshape(-1)))

    def set_source(self, comp: int, cells, weights):
        cells = np.ascontiguousarray(cells, np.int64)
        w = np.ascontiguousarray(weights, np.float64)
        comps = np.full(cells.shape, comp, np.int32)
        _chk(lib().orc_set_source(self._h, len(cells), comps.ctypes.data_as(C.c_void_p),
                                  cells.ctypes.data_as(C.c_void_p), w.ctypes.data_as(C.c_void_p)))

    def step(self, nsteps: int, amp=None):
        if amp is None:
            _chk(lib().orc_step(self._h, int(nsteps), None))
        else:
            a = np.ascontiguousarray(amp, np.float64)
            assert len(a) >= nsteps
            _chk(lib().orc_step(self._h, int(nsteps), a.ctypes.data_as(C.c_void_p)))

    def fields(self):
        E = np.zeros((3, self.n))
        B = np.zeros((3, self.n))
        _chk(lib().orc_fields(self._h, E.reshape(-1), B.reshape(-1)))
        return E, B

    def diag(self) -> dict:
        out = np.zeros(4)
        _chk(lib().orc_diag(self._h, out))
        return dict(energy=out[0], qc=out[1], divb2=out[2], b2=out[3])

    @property
    def t(self) -> int:
        return lib().orc_time(self._h)

    def get_state(self) -> np.ndarray:
        """Populations g[x, i, a, b], shape (n, Q, D, D)."""
        out = np.zeros(lib().orc_state_size(self._h))
        _chk(lib().orc_get_state(self._h, out))
        return out.reshape(self.n, self.Q, self.dim, self.dim)

    def set_state(self, g):
        _chk(lib().orc_set_state(self._h, np.ascontiguousarray(g, np.float64).reshape(-1)))

    def medium(self) -> dict:
        n = self.n
        cl2, w0, ea, dl = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(3 * n)
        _chk(lib().orc_get_medium(self._h, cl2, w0, ea, dl))
        return dict(cl2=cl2, w0=w0, eps_abs=ea, dlnmu=dl.reshape(3, n))


def run_problem(p, nsteps: int | None = None, threads: int = 0):
    """Run an ``inputs.Problem`` on the oracle; returns the Oracle object."""
    if threads:
        set_threads(threads)
    o = Oracle(p.dim, p.shape, p.tau, p.w0_vac)
    o.set_medium(p.eps_r, p.mu_r)
    o.init_fields(p.E0, p.B0)
    if len(p.src_cells):
        o.set_source(p.src_comp, p.src_cells, p.src_weights)
    k = p.nsteps if nsteps is None else nsteps
    o.step(k, p.amp if (p.amp is not None and len(p.src_cells)) else None)
    return o
