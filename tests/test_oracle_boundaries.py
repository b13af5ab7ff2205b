"""Pins of the oracle's non-periodic faces and absorbing layer.

* Method of images: a box with PEC (or PMC) walls on an axis evolves exactly
  like the periodic box of twice the length holding the box and its mirror
  image (medium mirrored evenly; tangential E odd and normal B odd about a
  PEC wall, the opposite for PMC), restricted to the original half.  This
  fixes the wall rule independently of how the oracle implements it.
* A uniform absorber sigma multiplies the solution of the linear scheme
  (no source) by exactly (1 - sigma)^t.
* A closed box with PEC or PMC walls conserves the positive invariant Q_c
  (walls only permute and sign-flip populations at equal weights).
* A graded absorbing layer takes up a pulse with little reflection.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1108_2651_amd import inputs

AX = {0: 3, 1: 2, 2: 1}     # lattice axis -> array axis of a (3, nz, ny, nx) field


def parity(kind, axis):
    """Image signs of the E and B components about a wall normal to axis."""
    pe = -np.ones(3)
    pe[axis] = 1.0          # PEC: tangential E odd, normal E even
    pb = -pe                # PEC: normal B odd, tangential B even
    if kind == "pmc":
        pe, pb = -pe, -pb
    return pe, pb


def mirror(field, shape, axis, sign=None):
    """Box plus its mirror image along axis (cell k <-> 2N-1-k)."""
    nx, ny, nz = shape
    if field.ndim == 1:
        a = field.reshape(nz, ny, nx)
        return np.concatenate([a, np.flip(a, axis=AX[axis] - 1)], axis=AX[axis] - 1).ravel()
    a = field.reshape(3, nz, ny, nx)
    im = np.flip(a, axis=AX[axis]) * sign[:, None, None, None]
    return np.concatenate([a, im], axis=AX[axis]).reshape(3, -1)


def doubled(shape, axis):
    s = list(shape)
    s[axis] *= 2
    return tuple(s)


def restrict(field, shape, big, axis):
    nx, ny, nz = big
    a = field.reshape(3, nz, ny, nx)
    sl = [slice(None)] * 4
    sl[AX[axis]] = slice(0, shape[axis])
    return a[tuple(sl)].reshape(3, -1)


def random_fields(dim, shape, seed, mu=False):
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    eps = rng.uniform(1.0, 5.0, n)
    mur = rng.uniform(0.8, 1.5, n) if mu else None
    E = np.zeros((3, n))
    B = np.zeros((3, n))
    if dim == 2:
        E[2] = rng.standard_normal(n)
        B[:2] = rng.standard_normal((2, n))
    else:
        E[:] = rng.standard_normal((3, n))
        B[:] = rng.standard_normal((3, n))
    return eps, mur, E, B


def run(dim, shape, eps, mur, E, B, steps, walls=(), sigma=None):
    o = O.Oracle(dim, shape)
    for axis, kind in walls:
        o.set_boundary(axis, kind)
    o.set_medium(eps, mur)
    if sigma is not None:
        o.set_absorber(sigma)
    o.init_fields(E, B)
    o.step(steps)
    return o


@pytest.mark.parametrize("dim,shape,axes,kind,mu", [
    (2, (12, 9, 1), (0,), "pec", False), (2, (12, 9, 1), (1,), "pmc", True),
    (2, (10, 7, 1), (0, 1), "pec", True), (3, (8, 6, 5), (0,), "pec", True),
    (3, (6, 7, 5), (2,), "pmc", False), (3, (6, 5, 4), (1, 2), "pec", False)])
def test_walls_are_mirror_images(dim, shape, axes, kind, mu):
    eps, mur, E, B = random_fields(dim, shape, seed=sum(shape) + len(axes), mu=mu)
    steps = 3 * max(shape)
    walled = run(dim, shape, eps, mur, E, B, steps, walls=[(a, kind) for a in axes])
    Ew, Bw = walled.fields()
    big, e2, m2, E2, B2 = shape, eps, mur, E, B
    for a in axes:
        pe, pb = parity(kind, a)
        e2, m2 = mirror(e2, big, a), (None if m2 is None else mirror(m2, big, a))
        E2, B2 = mirror(E2, big, a, pe), mirror(B2, big, a, pb)
        big = doubled(big, a)
    Ep, Bp = run(dim, big, e2, m2, E2, B2, steps).fields()
    for a in reversed(axes):
        pass
    # restrict the periodic solution to the original box, axis by axis
    cur = big
    for a in axes:
        nxt = list(cur)
        nxt[a] = shape[a]
        Ep = restrict(Ep, tuple(nxt), cur, a)
        Bp = restrict(Bp, tuple(nxt), cur, a)
        cur = tuple(nxt)
    scale = max(np.abs(Ep).max(), np.abs(Bp).max())
    assert np.abs(Ew - Ep).max() <= 1e-13 * scale
    assert np.abs(Bw - Bp).max() <= 1e-13 * scale
    # and the walls matter: the periodic box of the original size differs
    Eq, _ = run(dim, shape, eps, mur, E, B, steps).fields()
    assert np.abs(Eq - Ew).max() > 1e-3 * scale


@pytest.mark.parametrize("dim,shape", [(2, (16, 12, 1)), (3, (8, 7, 6))])
def test_uniform_absorber_is_exact_decay(dim, shape):
    eps, mur, E, B = random_fields(dim, shape, seed=7, mu=True)
    steps, sig = 30, 0.013
    free = run(dim, shape, eps, mur, E, B, steps, walls=[(0, "pec")]).fields()
    damped = run(dim, shape, eps, mur, E, B, steps, walls=[(0, "pec")], sigma=np.full(eps.size, sig)).fields()
    f = (1.0 - sig) ** steps
    for a, b in zip(free, damped):
        assert np.abs(b - f * a).max() <= 1e-13 * np.abs(a).max()


@pytest.mark.parametrize("dim,shape,kind", [(2, (20, 14, 1), "pec"), (2, (20, 14, 1), "pmc"),
                                            (3, (9, 8, 7), "pec"), (3, (9, 8, 7), "pmc")])
def test_closed_box_conserves_qc(dim, shape, kind):
    eps, _, E, B = random_fields(dim, shape, seed=11)
    o = O.Oracle(dim, shape)
    for a in range(dim):
        o.set_boundary(a, kind)
    o.set_medium(eps)
    o.init_fields(E, B)
    q0 = o.diag()["qc"]
    for _ in range(4):
        o.step(50)
        assert abs(o.diag()["qc"] / q0 - 1.0) < 1e-13


def test_graded_layer_absorbs_pulse():
    """A right-moving pulse meets a 60-cell layer with sigma rising
    quadratically to 0.1 in front of a PEC wall; without the layer the wall
    returns the whole pulse."""
    nx, ny = 600, 4
    x = np.tile(np.arange(nx), ny)
    cv = inputs.vacuum_speed(2, 1.0 / 3.0)
    f = np.exp(-(x - 150.0) ** 2 / (2 * 8.0 ** 2))
    E = np.zeros((3, nx * ny))
    B = np.zeros((3, nx * ny))
    E[2] = f
    B[1] = -f / cv
    eps = np.ones(nx * ny)
    x0, L = nx - 60, 60.0
    sigma = np.where(x >= x0, 0.1 * ((x - x0 + 0.5) / L) ** 2, 0.0)
    out = {}
    for name, sg in (("wall", None), ("layer", sigma)):
        o = O.Oracle(2, (nx, ny, 1))
        o.set_boundary(0, "pec")
        o.set_medium(eps)
        if sg is not None:
            o.set_absorber(sg)
        o.init_fields(E, B)
        e0 = o.diag()["energy"]
        o.step(int(2 * (nx - 150) / cv))     # to the wall and most of the way back
        Ef, Bf = o.fields()
        dens = (Ef ** 2).sum(0) * o.medium()["eps_abs"] + (Bf ** 2).sum(0)
        out[name] = (dens[x < x0].sum() / e0, o.diag()["energy"] / e0)
    assert out["wall"][0] > 0.9                # the bare wall reflects everything
    assert out["layer"][0] < 1e-3              # the layer reflects little ...
    assert out["layer"][1] < 2e-3              # ... and keeps almost nothing
