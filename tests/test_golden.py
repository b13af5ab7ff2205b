"""The oracle and the input generators against constants printed in the paper
(tests/golden/paper_constants.json, each entry citing its passage)."""
import json
import os

import numpy as np

from oracle import oracle as O
from paper_1108_2651_amd import inputs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_lattice_velocities_match_paper():
    v = O.velocities(2)[:, :2]
    assert v.tolist() == GOLD["lattice_2d_velocities"]["value"]
    v3 = O.velocities(3)
    # 6+1 lattice: rest particle plus +-unit vectors along each axis
    assert sorted(map(tuple, v3.tolist())) == sorted(
        [(0, 0, 0)] + [tuple(s * np.eye(3, dtype=int)[a]) for a in range(3) for s in (1, -1)])


def test_six_plus_one_light_speed():
    """Per-axis second moment of the 6+1 weights is (1 - w0)/3, which is what
    makes relate.2 hold with the equilibrium's 1/c^2 prefactor."""
    c = O.velocities(3)
    for w0 in (0.0, 0.2, 1 / 3, 0.9):
        w = np.array([w0] + [(1 - w0) / 6] * 6)
        for a in range(3):
            assert abs(np.sum(w * c[:, a] ** 2) - (1 - w0) / 3) < 1e-15
        g0 = O.equilibrium(3, w0, np.zeros((3, 3)), np.array([1.0, 0.0, 0.0]))
        # relate.2 with (a,b,g) = (y,x,y): sum_i c_iy g0_{i,y,x} = B_x
        assert abs(np.einsum("i,i->", c[:, 1].astype(float), g0[:, 1, 0]) - 1.0) < 1e-14


def test_homogeneous_forcing_profile():
    g = GOLD["homogeneous_forcing"]
    n = 100
    cells, w = inputs.paper_jz_source(n, g["x0"], g["y0"], g["width"])
    k = int(np.argmax(w))
    assert (k % n, k // n) == (30, 40)
    assert abs(w[k] - 1.0) < 1e-15
    # one width away along x: exp(-1/2)
    assert abs(w[k + 3] - np.exp(-0.5)) < 1e-12


def test_vortex_initial_condition():
    g = GOLD["vortex_initial_condition"]
    n = 200
    B = inputs.paper_vortex_ic(n, g["amp"], g["xc"], g["yc"], g["width"])
    Bx, By = B[0].reshape(n, n), B[1].reshape(n, n)
    # zero at the centre, rotation sense: B_x > 0 above the centre, B_y < 0 to its right
    i, j = int(g["yc"] * n), int(g["xc"] * n)
    assert Bx[i, j] == 0 and By[i, j] == 0
    assert Bx[i + 4, j] > 0 and By[i, j + 4] < 0
    # B is divergence free in the continuum: the central difference is O(h^2)
    div = (np.roll(Bx, -1, 1) - np.roll(Bx, 1, 1) + np.roll(By, -1, 0) - np.roll(By, 1, 0)) * n / 2
    assert np.abs(div).max() < 1e-2 * np.abs(Bx).max() * n
    assert abs(GOLD["tau"]["value"] - 0.5) == 0
