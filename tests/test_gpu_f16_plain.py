"""Plain FP16 storage (FP16 populations, FP32 medium and arithmetic): a
bandwidth comparison point for the deviation formats, not a format that meets
the 16-bit accuracy bar.

* Structure, bit for bit: initialising and then every single step of the FP16
  handle equals the FP32 handle run on the decoded FP16 state, rounded to
  FP16 (round to nearest even) -- with mu, walls, absorber, a dispersion
  pole, the source, pull and AA streaming.  The FP32 path itself is held to
  the oracle elsewhere.
* Against the oracle: each store perturbs every population by at most the
  FP16 unit roundoff u = 2^-11 relative; at tau = 1/2 the collision reflects
  about the equilibrium, so the step is an isometry in the 1/w-weighted norm
  and k steps add at most k*u to the relative error of the state.  The field
  error in the energy norm is held to that bound.
* The reason the deviation formats exist: on a benchmark medium the plain
  FP16 error exceeds the FP16 deviation format's by an order of magnitude.
"""
import numpy as np
import pytest

from gpu_util import announce, random_problem, rel
from oracle import oracle as O
from paper_1108_2651_amd import inputs, lbem
from test_gpu_precision import energy_error

pytestmark = pytest.mark.gpu

HDR = 128
U16 = 2.0 ** -11

CASES = [(2, (70, 33, 1), "pull", False, [], False, False), (2, (64, 48, 1), "aa", True, [], False, False),
         (3, (19, 13, 11), "pull", True, [(1, "pec")], True, False), (3, (16, 12, 10), "aa", False, [], False, False),
         (3, (20, 9, 14), "pull", False, [(0, "pmc"), (2, "pec")], False, False),
         (2, (50, 36, 1), "pull", False, [], False, True), (3, (18, 14, 12), "pull", True, [(2, "pmc")], True, True)]


def populations(s, dtype, m):
    blob = s.get_state()
    return blob, blob[HDR:HDR + m * np.dtype(dtype).itemsize].view(dtype).copy()


def aux_region(blob):
    """Byte range of the dispersion auxiliaries (payload and aux sizes are the
    header's int64 fields at offsets 56 and 64)."""
    pay, aux = (int(v) for v in blob[56:72].view(np.int64))
    return slice(HDR + pay, HDR + pay + aux)


@pytest.mark.parametrize("dim,shape,st,mu,walls,absorber,disp", CASES)
def test_f16_steps_are_rounded_fp32_steps(dim, shape, st, mu, walls, absorber, disp):
    p = random_problem(dim, shape, seed=sum(shape) + 11, mu=mu, nsteps=8)
    Q, P = 2 * dim + 1, dim * (dim - 1) // 2
    m = Q * P * p.n
    h = lbem.Solver(dim, shape, "f16", mu_varies=mu, streaming=st)
    f = lbem.Solver(dim, shape, "f32", mu_varies=mu, streaming=st)
    sigma = np.linspace(0.0, 0.3, p.n) if absorber else None
    for x in (h, f):
        for a, k in walls:
            x.set_boundary(a, k)
        x.set_medium(p.eps_r, p.mu_r)
        if sigma is not None:
            x.set_absorber(sigma)
        if disp:
            x.set_dispersion(np.linspace(0.0, 0.02, p.n), 0.01, 0.05)
        x.init_fields(p.E0, p.B0)
        x.set_source(p.src_comp, p.src_cells, p.src_weights)
    _, a16 = populations(h, np.float16, m)
    _, a32 = populations(f, np.float32, m)
    assert np.array_equal(a16.view(np.uint16), a32.astype(np.float16).view(np.uint16))
    for k in range(6):
        blob, _ = populations(f, np.float32, m)
        blob[HDR:HDR + 4 * m] = a16.astype(np.float32).view(np.uint8)
        if disp:   # the auxiliary P, J follow the FP16 handle's fields too
            b16 = h.get_state()
            blob[aux_region(blob)] = b16[aux_region(b16)]
        f.set_state(blob)
        h.step(1, p.amp[k:k + 1])
        f.step(1, p.amp[k:k + 1])
        _, a16 = populations(h, np.float16, m)
        _, a32 = populations(f, np.float32, m)
        diff = np.count_nonzero(a16.view(np.uint16) != a32.astype(np.float16).view(np.uint16))
        assert diff == 0, (k, diff)
    announce(f"f16 plain {dim}D {shape} {st} mu={mu} walls={walls} disp={disp}: 6 steps bitwise = rounded FP32 steps")
    for x in (h, f):
        x.close()


@pytest.mark.parametrize("dim,shape,st", [(2, (96, 80, 1), "pull"), (3, (24, 20, 18), "aa")])
def test_f16_error_within_rounding_bound(dim, shape, st):
    k = 200
    p = random_problem(dim, shape, seed=sum(shape), src=False, nsteps=k)
    s = lbem.Solver(dim, shape, "f16", streaming=st)
    s.setup(p)
    s.step(k)
    o = O.Oracle(dim, shape)
    o.set_medium(p.eps_r)
    o.init_fields(p.E0, p.B0)
    o.step(k)
    (Eg, Bg), (Eo, Bo) = s.moments(), o.fields()
    eN = energy_error(Eg, Bg, Eo, Bo, o.medium()["eps_abs"])
    announce(f"f16 plain {dim}D {shape} {st} {k} steps: energy-norm error {eN:.2e} "
             f"(bound k*u = {k * U16:.2e}; E {rel(Eg, Eo):.2e} B {rel(Bg, Bo):.2e})")
    assert eN <= k * U16
    s.close()


def test_f16_plain_vs_deviation_storage_on_benchmark_medium():
    k = 1000
    p = inputs.config3(nsteps=k, crop_n=64)
    o = O.Oracle(3, p.shape, p.tau, p.w0_vac)
    o.set_medium(p.eps_r)
    o.init_fields(p.E0, p.B0)
    o.set_source(p.src_comp, p.src_cells, p.src_weights)
    o.step(k, p.amp[:k])
    Eo, Bo = o.fields()
    ea = o.medium()["eps_abs"]
    err = {}
    for prec in ("f16", "f16dev"):
        s = lbem.Solver(3, p.shape, prec, w0_vac=p.w0_vac)
        s.setup(p)
        s.step(k, p.amp[:k])
        Eg, Bg = s.moments()
        err[prec] = energy_error(Eg, Bg, Eo, Bo, ea)
        s.close()
    announce(f"config3 64^3 crop {k} steps energy-norm error: plain f16 {err['f16']:.2e}, "
             f"f16 deviations {err['f16dev']:.2e}")
    assert err["f16dev"] <= 1e-3
    assert err["f16"] >= 10 * err["f16dev"]
