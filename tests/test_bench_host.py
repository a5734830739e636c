"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the method
configuration each option selects, the metric string, and when the committed
counter record may be quoted as the line's `traffic`."""
import json
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _args(**kw):
    base = dict(tail_nnz=None, row_layout=None, second_stage="bgs", decoupling="none", smoother="pgs-scm",
                chunks=None, theta_color=None, amg="rs", coarse_max=None, coarse_solver=None)
    base.update(kw)
    return types.SimpleNamespace(**base)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_default_method_is_rs_with_inverse_coarsest():
    p = bench._params(_args())
    assert (p.amg_kind, p.coarse_solver, p.coarse_max) == (0, 1, 4000)
    assert bench._method_config(_args())["amg"].startswith("RS theta=0.25, V-cycle, coarse<=4000 (explicit inverse)")


def test_lu_coarsest_keeps_fifty_rows():
    p = bench._params(_args(coarse_solver="lu"))
    assert (p.coarse_solver, p.coarse_max) == (0, 50)
    p = bench._params(_args(coarse_solver="lu", coarse_max=200))
    assert p.coarse_max == 200


def test_aggregation_amg_takes_the_papers_coarsest_size():
    p = bench._params(_args(amg="ua"))
    assert (p.amg_kind, p.coarse_max) == (1, 10000)


def test_extra_keywords_win_over_the_defaults():
    p = bench._params(_args(), coarse_solver=0, coarse_max=50, theta_color=0.3)
    assert (p.coarse_solver, p.coarse_max, p.theta_color) == (0, 50, 0.3)


def test_metric_names_the_workload_size():
    want = "CPR-FGMRES time to relres 1e-6 @3.28M DOF, FP32 vs FP64 precond; p50/p99 lat"
    assert bench._metric(3281850) == want
    assert "@12M DOF" in bench._metric(12_000_000)


def test_traffic_record_matches_only_its_configuration():
    if not os.path.exists(bench.TRAFFIC_FILE):
        pytest.skip("no committed counter record")
    with open(bench.TRAFFIC_FILE) as f:
        rec = json.load(f)
    method = {key: rec[key] for key in ("amg", "stage2", "decoupling")}
    assert method == bench._method_config(_args())  # taken with the benchmark's default method
    cls = "pgs_scm_colour_sweep_coarse"
    got = bench._measured_traffic(cls, "spe10", method)
    fresh = rec["classes"][cls]["source_sha256_16"] == bench._source_hash(bench.KERNEL_SOURCES[cls])
    assert (got is not None) == fresh
    if fresh:
        assert got == rec["classes"][cls]["hbm_bytes_per_launch"]
    for key, other in (("amg", method["amg"] + " (other)"), ("stage2", "block ILU(0), level-scheduled solves"),
                       ("decoupling", "quasi-IMPES")):
        assert bench._measured_traffic(cls, "spe10", dict(method, **{key: other})) is None
    assert bench._measured_traffic(cls, "channels", method) is None
