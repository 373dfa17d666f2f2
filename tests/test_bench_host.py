"""Host logic of the benchmark (no GPU): the algorithmic bytes it prices
launches at, the rule that a committed counter record is used only for the
kernel source and launch shape it was taken on, and the refusal of more
than one GPU."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bytes_per_site_of_one_pass_over_the_state():
    # f (9), u (2) and j (2) read once and written once
    assert bench.BYTES_PER_SITE_PASS["fp64"] == 208
    assert bench.BYTES_PER_SITE_PASS["fp32"] == 104
    assert bench.BYTES_PER_SITE_PASS["fp32u64"] == 120
    assert bench.BYTES_PER_SITE_PASS["fp16"] == bench.BYTES_PER_SITE_PASS["bf16"] == 84


def test_general_step_bytes_per_material_site():
    # the state read and written once, and the mask byte
    assert bench.general_bytes_per_site("fp32u64") == 121
    assert bench.general_bytes_per_site("fp64") == 209


def test_counter_record_only_for_its_kernel_and_shape():
    path = os.path.join(ROOT, "profiles", "step_fp32u64_4096_counters.txt")
    with open(path) as fh:
        rec = json.load(fh)
    t = rec["tiling"]
    n = rec["sites"]
    if rec["kernel_hash"] == bench.kernel_source_hash():
        assert bench.traffic_for("fp32u64", n, t["block"], t["n_segs"], t["steps_per_launch"]) == \
            rec["hbm_bytes_per_launch"]
    # another launch shape or plate size: no traffic figure
    assert bench.traffic_for("fp32u64", n, t["block"], t["n_segs"] + 1, t["steps_per_launch"]) is None
    assert bench.traffic_for("fp32u64", n // 4, t["block"], t["n_segs"], t["steps_per_launch"]) is None
    # another storage form's record is for its own launch shape; no record at all
    assert bench.traffic_for("fp64", n, t["block"], t["n_segs"], t["steps_per_launch"]) is None
    assert bench.traffic_for("no-such-form", n, t["block"], t["n_segs"], t["steps_per_launch"]) is None


def test_code_hash_ignores_comments(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2208_13769_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "a.hpp").write_text("int f(int x) { return x + 1; }  // one\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h1 = bench._code_hash(["a.hpp"])
    (csrc / "a.hpp").write_text("// a comment\nint f(int x)  {\n  return x + 1;\n}\n")
    assert bench._code_hash(["a.hpp"]) == h1
    (csrc / "a.hpp").write_text("int f(int x) { return x + 2; }\n")
    assert bench._code_hash(["a.hpp"]) != h1


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr


def test_roofline_counts_updates_per_launch():
    # a two-step launch of 2^24 sites in 536.8 us at 104 B per update (FP32):
    # 104 * 2 * 2^24 B / 536.8 us = 6.50 TB/s, 0.81 of the 8 TB/s peak
    sites = 1 << 24
    r = bench.step_roofline("fp32", sites, 2, 0.5368 / 2, None)
    assert r["updates_per_launch"] == 2 * sites
    assert r["algorithmic_bytes_per_launch"] == 104 * 2 * sites
    assert abs(r["achieved"] - 104 * 2 * sites / 536.8e-6 / 1e9) < 0.1
    assert abs(r["frac"] - 0.8126) < 1e-3
    # the launch's own state traffic is half of that
    assert abs(r["per_launch_state_GBps"] - r["achieved"] / 2) < 0.1
    # one step per launch: one update per site
    r1 = bench.step_roofline("fp16", sites, 1, 0.2, None)
    assert r1["updates_per_launch"] == sites and r1["bytes_per_update"] == 84
