"""Linear (Fourier) analysis of the lattice-BGK Maxwell scheme.

TEST INFRASTRUCTURE ONLY.  For a homogeneous medium and no source the scheme
is linear and translation invariant, so one time step maps a Fourier mode
exp(i k.x) of the populations to itself through a (Q*P) x (Q*P) matrix

    M(k) = diag_i(exp(-i k.c_i)) [ (1 - 1/tau) I + (1/tau) P_eq ],

streaming (eq. STREAM) after BGK collision (eq. COLLI).  P_eq maps a state to
the equilibrium (eq. distrib.func) of its own moments (relate.1, relate.2).
This module builds M(k) from those equations in numpy (a second, separate
write-up of the same formulas; it calls nothing from the C oracle) so that
tests can check eigenvalues against the continuum Maxwell dispersion
omega = c_M |k| and against the exact leapfrog relation in 2D.

State ordering: index i*P + p, p over the pairs (a<b) of tensor indices.
"""
from __future__ import annotations

import itertools

import numpy as np


def velocities(dim: int) -> np.ndarray:
    if dim == 2:
        return np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1]])
    return np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1],
                     [-1, 0, 0], [0, -1, 0], [0, 0, -1]])


def pairs(dim: int):
    return [(a, b) for a, b in itertools.combinations(range(dim), 2)]


def _to_tensor(h, dim):
    Q = 2 * dim + 1
    g = np.zeros((Q, dim, dim), dtype=h.dtype)
    for p, (a, b) in enumerate(pairs(dim)):
        g[:, a, b] = h[:, p]
        g[:, b, a] = -h[:, p]
    return g


def _from_tensor(g, dim):
    return np.stack([g[:, a, b] for a, b in pairs(dim)], axis=1)


def equilibrium_projection(h, dim: int, w0: float):
    """Equilibrium of the moments of state h (shape (Q, P))."""
    c = velocities(dim)
    Q = 2 * dim + 1
    cl2 = (1.0 - w0) / dim
    w = np.array([w0] + [(1.0 - w0) / (2 * dim)] * (Q - 1))
    g = _to_tensor(h, dim)
    rho = g.sum(axis=0)                                   # relate.1: Lambda / c^2
    K = np.einsum("ia,iab->b", c, g)                      # contracted relate.2
    Lam = cl2 * rho
    Bbar = K / (dim - 1)
    geq = (w / cl2)[:, None, None] * (Lam[None] + c[:, :, None] * Bbar[None, None, :]
                                      - c[:, None, :] * Bbar[None, :, None])
    return _from_tensor(geq, dim)


def step_matrix(dim: int, k, w0: float, tau: float = 0.5) -> np.ndarray:
    """One-step operator M(k) for wavevector k (cells^-1, length dim)."""
    c = velocities(dim)
    Q, P = 2 * dim + 1, len(pairs(dim))
    N = Q * P
    phase = np.exp(-1j * (c @ np.asarray(k, np.float64)))
    M = np.zeros((N, N), complex)
    om = 1.0 / tau
    for col in range(N):
        e = np.zeros((Q, P))
        e.flat[col] = 1.0
        post = (1.0 - om) * e + om * equilibrium_projection(e, dim, w0)
        M[:, col] = (phase[:, None] * post).ravel()
    return M


def maxwell_speed2(dim: int, w0: float) -> float:
    """c_M^2 = c_L^2/(D-1), c_L^2 = (1-w0)/D."""
    return (1.0 - w0) / dim / (dim - 1)


def physical_frequencies(dim: int, k, w0: float, tau: float = 0.5):
    """Frequencies omega = -arg(lambda) of the propagating physical branches
    (the modes that continue the conserved moments at k=0 and move),
    sorted ascending.  2D: 2 values (+-), 3D: 4 values."""
    lam, vec = np.linalg.eig(step_matrix(dim, k, w0, tau))
    om = -np.angle(lam)
    near = np.abs(lam - 1.0) < 0.5 * np.abs(lam + 1.0)     # continues lambda=1 at k=0
    cand = np.sort(om[near])
    nprop = 2 if dim == 2 else 4
    # drop the (near) static modes: keep the nprop largest |omega|
    order = np.argsort(-np.abs(cand))[:nprop]
    return np.sort(cand[order])


def leapfrog_frequency(k, cl2: float) -> float:
    """Exact dispersion of the 5-point leapfrog wave scheme
    E^{n+1} - 2E^n + E^{n-1} = c^2 Lap_h E^n:
    sin^2(omega/2) = c^2 sum_a sin^2(k_a/2)."""
    s = cl2 * sum(np.sin(0.5 * ka) ** 2 for ka in k)
    return 2.0 * np.arcsin(np.sqrt(s))


def eigenmode(dim: int, k, w0: float, tau: float = 0.5, which: int = -1):
    """(lambda, vector (Q,P)) of a propagating physical branch (which = -1:
    the largest positive frequency)."""
    lam, vec = np.linalg.eig(step_matrix(dim, k, w0, tau))
    om = -np.angle(lam)
    near = np.abs(lam - 1.0) < 0.5 * np.abs(lam + 1.0)
    idx = np.where(near)[0]
    j = idx[np.argsort(om[idx])[which]]
    Q, P = 2 * dim + 1, len(pairs(dim))
    return lam[j], vec[:, j].reshape(Q, P)
