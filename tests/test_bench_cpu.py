"""Host-side checks of the benchmark's algorithmic-byte accounting (the
per-unit figures behind every roofline number) and of its contract on a
machine without a GPU."""
import json

import pytest
import subprocess
import sys
import os

import numpy as np

import bench
from paper_1108_2651_amd import inputs, lbem, serve

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bytes_per_cell_counts_every_stored_value_once_each_way():
    # plain: Q*P values read and written + the medium
    assert bench.bytes_per_cell(2, "f32") == 2 * 5 * 4 + 4 == 44
    assert bench.bytes_per_cell(3, "f32") == 2 * 21 * 4 + 4 == 172
    assert bench.bytes_per_cell(2, "f64") == 88 and bench.bytes_per_cell(3, "f64") == 344
    # plain FP16 storage: FP16 populations, FP32 medium
    assert bench.bytes_per_cell(2, "f16") == 2 * 5 * 2 + 4 == 24 and bench.bytes_per_cell(3, "f16") == 88
    # deviation storage: (P + D) FP32 moments + Q*P halves
    assert bench.bytes_per_cell(2, "f16dev") == 2 * (3 * 4 + 5 * 2) + 4 == 48
    assert bench.bytes_per_cell(3, "bf16dev") == 2 * (6 * 4 + 21 * 2) + 4 == 136
    # ghost coordinates: (Q-1)P - D halves
    assert bench.bytes_per_cell(2, "f16ghost") == 2 * (3 * 4 + 2 * 2) + 4 == 36
    assert bench.bytes_per_cell(3, "f16ghost") == 2 * (6 * 4 + 15 * 2) + 4 == 112
    # a varying mu adds the D components of grad ln mu
    assert bench.bytes_per_cell(2, "f32", mu=True) == 52 and bench.bytes_per_cell(3, "f64", mu=True) == 368
    # the serving scheduler charges the same figures
    for dim in (2, 3):
        for prec in ("f32", "f64", "f16dev", "f16ghost"):
            assert serve.bytes_per_update(dim, prec) == bench.bytes_per_cell(dim, prec)


def test_extra_bytes_of_cell_extras():
    p = inputs.config3(nsteps=4, n=16)
    assert bench.extra_bytes(p, "f32") == 0
    p.sigma = np.zeros(p.n)
    assert bench.extra_bytes(p, "f32") == 4
    p.disp = (np.zeros(p.n),) * 3
    assert bench.extra_bytes(p, "f32") == 4 + 12 + 2 * (2 * 3 * 4)       # coefficients + P, J read and written
    p.aniso = np.ones((3, p.n))
    assert bench.extra_bytes(p, "f64") == 8 + 24 + 2 * (2 * 3 * 8) + 3 * 8


def test_multi_gpu_request_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_kernel_hash_and_traffic_record():
    h = bench.kernel_source_hash()
    assert len(h) == 16
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic_c4_512_f16ghost.json")))
    # the record names the headline kernel and carries the calibration it was scaled by
    assert rec["kernel"] == bench.PRIMARY_KERNEL
    assert 1.99 < rec["fetch_scale"] < 2.01 and rec["write_scale"] == 1.0
    assert rec["algorithmic_bytes_per_launch"] == 112 * 512 ** 3
    assert rec["bytes_per_launch"] == pytest.approx(
        rec["fetch_kib_per_dispatch"] * 1024 * rec["fetch_scale"] + rec["write_kib_per_dispatch"] * 1024 *
        rec["write_scale"])
    assert bench.load_traffic("c4_512_f16ghost", "another kernel") is None


def test_symbols_of_the_binding_match_the_header():
    assert "lbem_set_dispersion" in lbem.SYMBOLS and "lbem_get_state" in lbem.SYMBOLS
