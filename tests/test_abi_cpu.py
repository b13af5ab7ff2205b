"""liblbem loads, exports every entry point declared in include/lbem.h, and its
pure-host calls behave (no GPU needed: no kernel is launched here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1108_2651_amd import lbem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lbem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbem_[a-z_]+)\s*\(", src)))


def test_library_exports_all_declared_symbols():
    L = lbem.load()
    decl = declared_functions()
    assert len(decl) >= 11
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(lbem.SYMBOLS) == decl


def test_strerror_and_required_bytes():
    assert lbem.strerror(0) == "success"
    assert "unstable" not in lbem.strerror(-1)
    assert lbem.strerror(-3).startswith("medium")
    # 2D FP32 pull: 2 copies x 5 pops x 4 B + 4 B medium + 24 B scratch per cell
    n = 256 * 256
    b = lbem.required_bytes(2, (256, 256, 1), "f32")
    assert 2 * 5 * 4 * n + 4 * n + 24 * n <= b <= 2 * 5 * 4 * n + 4 * n + 24 * n + 4 * 256
    # the default is pull (two copies: the fused multi-step kernels need them);
    # the in-place AA pattern keeps one copy of the 21 populations, and is the
    # default for 3D FP64 and for 3D FP32 boxes below 1e6 cells
    b3 = lbem.required_bytes(3, (256, 256, 256), "f32")
    assert b3 == lbem.required_bytes(3, (256, 256, 256), "f32", streaming="pull")
    assert lbem.required_bytes(3, (256, 256, 256), "f32", streaming="aa") < b3
    small = lbem.required_bytes(3, (64, 64, 64), "f32")
    assert small == lbem.required_bytes(3, (64, 64, 64), "f32", streaming="aa")
    # the boundary: 96^3 (0.88e6 cells) still AA, 112^3 (1.4e6) pull for the fused pair
    assert lbem.required_bytes(3, (96, 96, 96), "f32") == lbem.required_bytes(3, (96, 96, 96), "f32", streaming="aa")
    assert lbem.required_bytes(3, (112, 112, 112), "f32") == \
        lbem.required_bytes(3, (112, 112, 112), "f32", streaming="pull")
    assert lbem.required_bytes(3, (256, 256, 256), "f64") == \
        lbem.required_bytes(3, (256, 256, 256), "f64", streaming="aa")
    assert lbem.required_bytes(2, (64, 64, 1), "f64") == lbem.required_bytes(2, (64, 64, 1), "f64", streaming="pull")
    # deviation storage: FP32 moments (P+D) + 16-bit deviations (Q*P), two copies
    bd = lbem.required_bytes(3, (64, 64, 64), "f16dev")
    m = 64 ** 3
    assert bd >= 2 * (6 * 4 + 21 * 2) * m
    # ghost coordinates: 15 of the 21 deviations (3D), 2 of 5 (2D)
    bg = lbem.required_bytes(3, (64, 64, 64), "bf16ghost")
    assert bd - bg == 2 * 6 * 2 * m
    assert (lbem.required_bytes(2, (256, 256, 1), "f16dev") -
            lbem.required_bytes(2, (256, 256, 1), "f16ghost")) == 2 * 3 * 2 * 256 * 256
    # plain FP16 storage: the FP32 layout at half the population bytes (AA: one copy)
    for dim, shape in ((2, (256, 256, 1)), (3, (64, 64, 64))):
        n, QP = int(np.prod(shape)), (5 if dim == 2 else 21)
        for st, copies in (("pull", 2), ("aa", 1)):
            assert (lbem.required_bytes(dim, shape, "f32", streaming=st) -
                    lbem.required_bytes(dim, shape, "f16", streaming=st)) == copies * QP * 2 * n


@pytest.mark.parametrize("kw", [dict(dim=4), dict(dim=2, shape=(8, 8, 2)), dict(prec="f64", tau=0.0),
                                dict(w0_vac=1.0), dict(w0_vac=-0.1), dict(shape=(0, 4, 1)),
                                dict(prec="f16dev", streaming="aa"), dict(prec="f16ghost", streaming="aa"),
                                dict(prec=7), dict(prec=-1), dict(shape=(2048, 2048, 1024), dim=3)])
def test_invalid_configs_rejected_on_host(kw):
    args = dict(dim=2, shape=(8, 8, 1), prec="f32")
    args.update(kw)
    dim, shape, prec = args.pop("dim"), args.pop("shape"), args.pop("prec")
    cfg = lbem.make_config(dim, shape, prec, **args)
    L = lbem.load()
    assert L.lbem_required_bytes(C.byref(cfg)) == 0
    h = C.c_void_p()
    assert L.lbem_create(C.byref(cfg), C.byref(h)) == lbem.LBEM_EINVAL
    assert not h.value


def test_null_handle_calls():
    L = lbem.load()
    assert L.lbem_destroy(None) == 0
    assert L.lbem_time(None) == -1
    assert L.lbem_step(None, 1, None) == lbem.LBEM_EINVAL
    assert L.lbem_moments(None, None, None, 0) == lbem.LBEM_EINVAL
    assert L.lbem_state_bytes(None) == 0
    assert L.lbem_get_state(None, None, 0, 0) == lbem.LBEM_EINVAL
    assert L.lbem_set_state(None, None, 0, 0) == lbem.LBEM_EINVAL
    assert L.lbem_energy_noalloc(None, None) == lbem.LBEM_EINVAL
    assert "static scratch" in lbem.strerror(lbem.LBEM_ETOOBIG)


def test_noalloc_limit_matches_header():
    src = open(os.path.join(ROOT, "include", "lbem.h")).read()
    m = re.search(r"#define LBEM_NOALLOC_MAX_CELLS (\d+)", src)
    assert m and int(m.group(1)) == lbem.NOALLOC_MAX_CELLS
    n = lbem.NOALLOC_MAX_CELLS
    need = lambda k: 3 * k + 4 * (-(-k // 256)) + 4      # doubles: B field, partials, results
    assert need(n) * 8 <= 64 << 20 < need(n + 1) * 8
