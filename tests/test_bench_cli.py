"""Host-side checks of the benchmark script: it refuses more than one GPU with a message before
touching any device, the committed counter records it reads have the fields it uses and agree
with the workload's sizes (64 pulses x 64x64x16 modes x nt = 16384), and the solver comparison's
cost-to-accuracy interpolation."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def _load(name):
    with open(os.path.join(ROOT, "profiles", name)) as fh:
        return json.load(fh)


def test_traffic_record_fields():
    rec = _load("k_evolve_hbm_traffic_de_generation.json")
    for k in ("evolve_sources_sha256", "bytes_per_call", "algorithmic_bytes_per_call", "fetch_scale", "write_scale",
              "commands"):
        assert k in rec
    assert tuple(rec["evolve_sources"]) == bench.EVOLVE_SOURCES
    # A tables dominate: 64 pulses x 16384 steps x 16 B
    assert rec["algorithmic_bytes_per_call"] >= 64 * 16384 * 16
    assert 1.0 <= rec["bytes_per_call"] / rec["algorithmic_bytes_per_call"] < 1.2


def test_fp64_counter_record_fields():
    rec = _load("k_evolve_fp64_counters_de_generation.json")
    assert rec["mode_steps_per_call"] == 64 * 65536 * 16384
    assert tuple(rec["evolve_sources"]) == bench.EVOLVE_SOURCES
    # 2 x FMA + MUL + ADD, per mode-step, between the cheapest and the costliest series variant
    lo = min(bench.FLOP_PER_MODE_STEP.values())
    assert lo <= rec["flop_per_mode_step"] <= bench.FIXED_FLOP_PER_MODE_STEP
    for c in rec["calls"]:
        v = c["counters"]
        fl = 64 * (2 * v["SQ_INSTS_VALU_FMA_F64"] + v["SQ_INSTS_VALU_MUL_F64"] + v["SQ_INSTS_VALU_ADD_F64"])
        assert abs(fl - c["fp64_flop"]) <= 1e-9 * fl


def test_source_hash_ignores_comments_only():
    text = "int a = 1;  // one\n// a comment line\n\n  b(a);   \n"
    assert bench.code_lines(text) == "int a = 1;\n  b(a);\n"
    assert bench.code_lines(text + "// more\n") == bench.code_lines(text)
    assert bench.code_lines(text.replace("1;", "2;")) != bench.code_lines(text)


def test_cost_to_reach_interpolates_in_log_log():
    # eps = c us^-2 exactly (a second-order method at fixed cost per step): the log-log
    # interpolation between the bracketing rows is then exact
    c = 1e-5
    rows = [{"method": "m2", "us_per_mode": us, "eps": c * us ** -2} for us in (0.02, 0.05, 0.2, 0.5)]
    reach = bench.cost_to_reach(rows, 1e-3)
    assert abs(reach["m2"] - (c / 1e-3) ** 0.5) <= 1e-12
    # first usable row already below the target: its own cost
    assert bench.cost_to_reach(rows, 1.0)["m2"] == 0.02


def test_cost_to_reach_skips_unstable_and_unresolved_rows():
    rows = [{"method": "qke", "us_per_mode": 0.1, "eps": None, "unstable": True},
            {"method": "qke", "us_per_mode": 0.3, "eps": 5e-4},
            {"method": "split2", "us_per_mode": 0.1, "eps": 30.0, "unresolved": True},
            {"method": "split2", "us_per_mode": 0.2, "eps": 0.5},
            {"method": "split2", "us_per_mode": 0.4, "eps": 2e-3},
            {"method": "dirac2", "us_per_mode": 0.1, "eps": 40.0, "unresolved": True},
            {"method": "dirac2", "us_per_mode": 0.2, "eps": 1e-4}]
    reach = bench.cost_to_reach(rows, 1e-3)
    assert reach["qke"] == 0.3 and reach["dirac2"] == 0.2  # nothing to interpolate from
    assert "split2" not in reach  # never at or below the target
