"""Pins of the FP64 oracle's single-cell algebra against what the paper fixes.

* eq. relate.1-3: closed-form moments of the equilibrium (eq. distrib.func);
* eq. CONSERV: collision leaves the conserved moments (rho_ab and the
  contracted first moment K) unchanged;
* the equilibrium map is an orthogonal projection in the 1/w_i-weighted inner
  product (this fixes Bbar = K/(D-1) and the weights), so that at tau=1/2 the
  collision is the reflection 2 P - I;
* the tensor source T_i = -(w_i/c^2) eps_{gab} S_g has zeroth moment
  -eps S/c^2 (right side of eq. GMOM.1) and no first moment;
* Levi-Civita recovery E_g = -1/2 eps_gab Lambda_ab round-trips;
* built-in antisymmetry g_iab = -g_iba (Introduction) holds bit-for-bit
  after many steps, and a uniform current gives the closed form
  E(n) = -n j/eps_abs with B = 0.
"""
import numpy as np
import pytest

from oracle import oracle as O


def rand_antisym(rng, D):
    A = rng.standard_normal((D, D))
    return A - A.T


def levi3():
    e = np.zeros((3, 3, 3))
    e[0, 1, 2] = e[1, 2, 0] = e[2, 0, 1] = 1
    e[0, 2, 1] = e[2, 1, 0] = e[1, 0, 2] = -1
    return e


def weights(dim, w0):
    return np.array([w0] + [(1 - w0) / (2 * dim)] * (2 * dim))


def proj(dim, w0, g):
    """Equilibrium of the state's own moments (relate.1, contracted relate.2)."""
    c = O.velocities(dim)[:, :dim]
    cl2 = (1 - w0) / dim
    rho = g.sum(0)
    K = np.einsum("ia,iab->b", c, g)
    return O.equilibrium(dim, w0, cl2 * rho, K / (dim - 1))


@pytest.mark.parametrize("dim", [2, 3])
def test_equilibrium_moments_relate(dim):
    rng = np.random.default_rng(100 + dim)
    c = O.velocities(dim)[:, :dim].astype(float)
    d = np.eye(dim)
    for _ in range(25):
        w0 = rng.uniform(0.0, 0.95)
        cl2 = (1 - w0) / dim
        Lam = rand_antisym(rng, dim)
        B = rng.standard_normal(dim)
        g0 = O.equilibrium(dim, w0, Lam, B)
        # relate.1
        np.testing.assert_allclose(g0.sum(0), Lam / cl2, rtol=0, atol=1e-13 / cl2)
        # relate.2: sum_i c_ig g0_iab = d_ga B_b - d_gb B_a
        G3 = np.einsum("ig,iab->abg", c, g0)
        exp3 = np.einsum("ga,b->abg", d, B) - np.einsum("gb,a->abg", d, B)
        np.testing.assert_allclose(G3, exp3, rtol=0, atol=1e-13)
        # relate.3: sum_i c_ig c_ik g0_iab = d_gk Lambda_ab
        G4 = np.einsum("ig,ik,iab->abgk", c, c, g0)
        exp4 = np.einsum("gk,ab->abgk", d, Lam)
        np.testing.assert_allclose(G4, exp4, rtol=0, atol=1e-13)
        # antisymmetric and traceless per velocity
        assert np.array_equal(g0, -np.transpose(g0, (0, 2, 1)))


@pytest.mark.parametrize("dim", [2, 3])
def test_equilibrium_is_orthogonal_projection(dim):
    rng = np.random.default_rng(200 + dim)
    Q = 2 * dim + 1
    for _ in range(20):
        w0 = rng.uniform(0.0, 0.9)
        g = np.stack([rand_antisym(rng, dim) for _ in range(Q)])
        P1 = proj(dim, w0, g)
        # idempotent: the equilibrium reproduces its own moments (CONSERV)
        np.testing.assert_allclose(proj(dim, w0, P1), P1, rtol=0, atol=1e-12)
        # orthogonal in <f,g> = sum_i f_i g_i / w_i
        w = weights(dim, w0)
        ip = np.einsum("iab,iab,i->", g - P1, P1, 1.0 / w)
        assert abs(ip) < 1e-11 * (1 + np.einsum("iab,iab,i->", g, g, 1.0 / w))


@pytest.mark.parametrize("dim", [2, 3])
def test_collision_conserves_and_reflects(dim):
    rng = np.random.default_rng(300 + dim)
    Q = 2 * dim + 1
    c = O.velocities(dim)[:, :dim]
    for _ in range(20):
        w0 = rng.uniform(0.0, 0.9)
        g = np.stack([rand_antisym(rng, dim) for _ in range(Q)])
        gp = O.collide(dim, w0, 0.5, g)
        # CONSERV: rho_ab and K_b unchanged
        np.testing.assert_allclose(gp.sum(0), g.sum(0), rtol=0, atol=1e-12)
        np.testing.assert_allclose(np.einsum("ia,iab->b", c, gp), np.einsum("ia,iab->b", c, g),
                                   rtol=0, atol=1e-12)
        # tau = 1/2: g' = 2 g0 - g
        np.testing.assert_allclose(gp, 2 * proj(dim, w0, g) - g, rtol=0, atol=1e-12)
        # general tau: g' = g - (g - g0)/tau
        tau = rng.uniform(0.55, 2.0)
        gt = O.collide(dim, w0, tau, g)
        np.testing.assert_allclose(gt, g - (g - proj(dim, w0, g)) / tau, rtol=0, atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_source_term_moments(dim):
    rng = np.random.default_rng(400 + dim)
    Q = 2 * dim + 1
    c = O.velocities(dim)[:, :dim]
    eps = levi3()[:, :dim, :dim]
    for _ in range(10):
        w0 = rng.uniform(0.0, 0.9)
        cl2 = (1 - w0) / dim
        g = np.stack([rand_antisym(rng, dim) for _ in range(Q)])
        S = rng.standard_normal(3)
        T = O.collide(dim, w0, 0.5, g, S) - O.collide(dim, w0, 0.5, g)
        # zeroth moment: -eps_gab S_g / c^2 (right side of GMOM.1)
        np.testing.assert_allclose(T.sum(0), -np.einsum("gab,g->ab", eps, S) / cl2,
                                   rtol=1e-12, atol=1e-12)
        # no first moment
        np.testing.assert_allclose(np.einsum("ig,iab->abg", c, T), 0.0, atol=1e-12)
        # shape: proportional to w_i
        w = weights(dim, w0)
        np.testing.assert_allclose(T / w[:, None, None], np.broadcast_to(T[1] / w[1], T.shape),
                                   rtol=1e-12, atol=1e-12)


def test_levi_civita_round_trip():
    rng = np.random.default_rng(5)
    # 3D: uniform random E, B
    o = O.Oracle(3, (2, 2, 2))
    o.set_medium(np.full(8, 1.7))
    E = np.repeat(rng.standard_normal((3, 1)), 8, axis=1)
    B = np.repeat(rng.standard_normal((3, 1)), 8, axis=1)
    o.init_fields(E, B)
    E2, B2 = o.fields()
    np.testing.assert_allclose(E2, E, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(B2, B, rtol=1e-14, atol=1e-15)
    g = o.get_state()[0]
    # Lambda_ab = -eps_gab E_g
    cl2 = o.medium()["cl2"][0]
    np.testing.assert_allclose(cl2 * g.sum(0), -np.einsum("gab,g->ab", levi3(), E[:, 0]),
                               rtol=1e-14, atol=1e-15)
    # 2D TM: E_z, B_x, B_y
    o2 = O.Oracle(2, (3, 3, 1))
    o2.set_medium(np.full(9, 2.5))
    E = np.zeros((3, 9)); E[2] = rng.standard_normal(9)
    B = np.zeros((3, 9)); B[:2] = rng.standard_normal((2, 9))
    o2.init_fields(E, B)
    E2, B2 = o2.fields()
    np.testing.assert_allclose(E2, E, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(B2, B, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("dim,shape", [(2, (12, 10, 1)), (3, (6, 5, 4))])
def test_antisymmetry_bitwise(dim, shape):
    rng = np.random.default_rng(600 + dim)
    n = int(np.prod(shape))
    o = O.Oracle(dim, shape)
    eps = rng.uniform(1.0, 4.0, n)
    mu = rng.uniform(0.8, 1.5, n)
    o.set_medium(eps, mu)
    E = rng.standard_normal((3, n)); B = rng.standard_normal((3, n))
    if dim == 2:
        E[:2] = 0; B[2] = 0
    o.init_fields(E, B)
    o.set_source(2, np.arange(0, n, 3), rng.standard_normal(len(range(0, n, 3))))
    o.step(30, rng.standard_normal(30))
    g = o.get_state()
    assert np.array_equal(g, -np.transpose(g, (0, 1, 3, 2)))
    assert np.all(np.diagonal(g, axis1=2, axis2=3) == 0)


@pytest.mark.parametrize("dim,shape,comp", [(2, (8, 6, 1), 2), (3, (4, 4, 4), 0), (3, (4, 4, 4), 2)])
def test_uniform_current_closed_form(dim, shape, comp):
    n = int(np.prod(shape))
    eps_r = 2.0
    w0_vac = 1.0 / 3.0
    o = O.Oracle(dim, shape, 0.5, w0_vac)
    o.set_medium(np.full(n, eps_r))
    o.init_fields(np.zeros((3, n)), np.zeros((3, n)))
    j = 0.7
    o.set_source(comp, np.arange(n), np.full(n, j))
    eps_abs = eps_r / ((1 - w0_vac) / (dim * (dim - 1)))
    for k in range(1, 21):
        o.step(1, [1.0])
        E, B = o.fields()
        np.testing.assert_allclose(E[comp], -k * j / eps_abs, rtol=1e-13)
        others = [c for c in range(3) if c != comp]
        assert np.abs(E[others]).max() < 1e-14
        assert np.abs(B).max() < 1e-14
    # populations remain at equilibrium
    g = o.get_state()
    w0 = o.medium()["w0"][0]
    np.testing.assert_allclose(g[0], proj(dim, w0, g[0]), rtol=0, atol=1e-13)


@pytest.mark.parametrize("dim,shape,comp", [(2, (6, 5, 1), 2), (3, (4, 3, 4), 1)])
def test_uniform_current_follows_the_amplitude_series(dim, shape, comp):
    # the current of step t enters that step (source time level): after the
    # steps t0..t1-1 of one call, E has moved by -sum(amp[t0:t1]) j / eps_abs
    n = int(np.prod(shape))
    eps_r, w0_vac, j = 3.0, 1.0 / 3.0, 0.4
    o = O.Oracle(dim, shape, 0.5, w0_vac)
    o.set_medium(np.full(n, eps_r))
    o.init_fields(np.zeros((3, n)), np.zeros((3, n)))
    o.set_source(comp, np.arange(n), np.full(n, j))
    eps_abs = eps_r / ((1 - w0_vac) / (dim * (dim - 1)))
    amp = np.random.default_rng(5).standard_normal(20)
    for t0, t1 in ((0, 7), (7, 20)):
        o.step(t1 - t0, amp[t0:t1])
        E, B = o.fields()
        np.testing.assert_allclose(E[comp], -amp[:t1].sum() * j / eps_abs, rtol=1e-12)
        assert np.abs(B).max() < 1e-14


def test_source_entries_add_up():
    # the current density is the sum of the listed contributions: a cell
    # listed twice carries the sum of its weights
    shape = (9, 7, 1)
    n = 63
    rng = np.random.default_rng(12)
    eps = rng.uniform(1.0, 3.0, n)
    amp = rng.standard_normal(12)
    out = []
    for cells, weights in (([3, 3, 40], [0.5, 0.25, 1.0]), ([3, 40], [0.75, 1.0])):
        o = O.Oracle(2, shape)
        o.set_medium(eps)
        o.init_fields(np.zeros((3, n)), np.zeros((3, n)))
        o.set_source(2, np.array(cells), np.array(weights))
        o.step(12, amp)
        out.append(o.fields())
    for a, b in zip(out[0], out[1]):
        assert np.abs(a - b).max() <= 1e-15 * max(np.abs(b).max(), 1e-300)


def test_medium_stability_bounds():
    o = O.Oracle(2, (4, 4, 1), 0.5, 1.0 / 3.0)
    # eps_r * mu_r < 1 - w0_vac gives w0 < 0: rejected
    with pytest.raises(O.OracleError) as e:
        o.set_medium(np.full(16, 0.5))
    assert e.value.code == -3
    with pytest.raises(O.OracleError):
        o.set_medium(np.full(16, -1.0))
    o.set_medium(np.full(16, 2.0 / 3.0 + 1e-12))
    assert O.Oracle(2, (4, 4, 1)).t == 0
