"""Host-side logic of bench.py (no GPU): the refusal of several GPUs, the
algorithmic byte model of the PCG kernel classes and the roofline figure
computed from a profile."""
from __future__ import annotations

import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("K", [1, 2, 4, 10])
def test_pcg_bytes_per_outer_iteration(bench, K):
    """K PCG iterations of a Haar slice with the paper's preconditioner: the
    paired form moves K column passes and K - 1 paired launches (16.125 and
    68 B/px); the two-launch form adds K row inverses, the last reading only
    p and d (12 B/px instead of 28)."""
    b = bench.bytes_per_px
    paired = K * b("col", K) + (K - 1) * b("update", K)
    assert paired == pytest.approx(K * 16.125 + (K - 1) * 68.0)
    unpaired = K * b("col", K) + K * b("rowinv", K) + (K - 1) * b("update", K)
    assert unpaired == pytest.approx(K * 16.125 + (K - 1) * 28.0 + 12.0 + (K - 1) * 68.0)
    if K == 4:
        assert paired == pytest.approx(268.5) and unpaired == pytest.approx(364.5)
    # launches across shapes keep only the last row inverse (12 B/px each)
    assert b("rowinv", K, True, True) == 12.0


def test_last_rowinv_only(bench):
    f = bench.last_rowinv_only
    assert f({"rowinv": {"slice_launches": 100}, "col": {"slice_launches": 400}})
    assert not f({"rowinv": {"slice_launches": 400}, "col": {"slice_launches": 400}})
    assert not f({"col": {"slice_launches": 400}})


def test_roofline_of_a_profile(bench, monkeypatch):
    """The dominant PCG class by time; achieved = its algorithmic bytes per
    launch over its average launch time; frac against 8 TB/s; traffic only
    from a record whose source hash matches."""
    monkeypatch.setattr(bench, "traffic_record", lambda: None)
    n, K = 256, 4
    prof = {"col": {"ms": 13.0, "launches": 800, "slice_launches": 51200},
            "update": {"ms": 34.0, "launches": 600, "slice_launches": 38400},
            "r0_rowfwd": {"ms": 7.5, "launches": 200, "slice_launches": 12800}}
    roof, gbs, kms = bench.roofline_of(prof, n, K, 0.070, 500)
    assert roof["kernel"] == "update" and roof["bound"] == "hbm" and roof["traffic"] is None
    per_launch = 68.0 * n * n * 38400 / 600
    assert roof["bytes_per_launch"] == pytest.approx(per_launch)
    assert roof["avg_launch_us"] == pytest.approx(34.0 / 600 * 1e3)
    assert roof["achieved"] == pytest.approx(per_launch / (34.0e-3 / 600) / 1e9)
    assert roof["frac"] == pytest.approx(roof["achieved"] / 8000.0)
    assert kms == {"col": 13.0, "update": 34.0, "r0_rowfwd": 7.5}
    # whole path: every class's bytes over the step; the first residual pass
    # of each of the 500 slices has no x update to fold in (16 B/px less)
    tot = (16.125 * 51200 + 68.0 * 38400 + 36.0 * 12800) * n * n - 16.0 * n * n * 500
    assert gbs == pytest.approx(tot / 0.070 / 1e9)


def test_cpu_baseline_pool():
    """The oracle baseline in a pool of worker processes: every sampled
    slice is solved once, the pool's rate and core count are reported, and
    results handed in as the GPU's (here the oracle's own, in complex64)
    compare to the oracle within single-precision rounding."""
    sys.path.insert(0, ROOT)
    import bench
    import numpy as np
    import synth
    from oracle.firls import Operators, firls
    seeds = [20000, 20001, 20002]
    xs, fes = [], []
    for sd in seeds:
        r = firls(Operators.from_problem(synth.cfg1(sd, n=64)), 4, 4, tau=8e-6)
        xs.append(r.x.astype(np.complex64))
        fes.append((r.F_eps, r.outer_iters))
    cb, per = bench.cpu_baseline(64, 8e-6, 4, 4, seeds, xs, fes, per_worker=2, workers=2)
    assert cb["cores"] == 2 and cb["kind"] == "oracle" and cb["value"] > 0
    assert per["slices"] == 3 and per["same_outer_count"] == 3
    assert sorted(e["seed"] for e in per["per_slice"]) == seeds
    assert per["F_eps_rel_diff_max"] < 1e-6 and per["x_rel_l2_max_same_count"] < 1e-6
