"""Host-side checks of the benchmark script: the kernel-source hash that ties
a committed counter summary to the kernel, the use of that summary, the
weights of the algorithmic work, and the one-GPU rule.  No GPU needed."""

import json
import os
import subprocess
import sys

import bench
import paper_1208_0277_amd as sccg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_code_only_ignores_comments_and_layout():
    a = "int x = 1; // one\n/* block\n comment */ int  y =\n 2;\nconst char* s = \"// kept\";"
    b = "int x = 1;\nint y = 2; const char* s = \"// kept\";"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only("int x = 1;") != bench._code_only("int x = 2;")
    assert "// kept" in bench._code_only(a)


def test_profile_summary_needs_the_same_kernel_source_and_params(monkeypatch):
    stem = bench.PROFILE_STEMS[3]
    path = os.path.join(ROOT, "profiles", stem + ".json")
    with open(path) as f:
        committed = json.load(f)
    params = committed["params"]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: committed["kernel_source_hash"])
    d = bench.profile_summary(3, params)
    assert d is not None and d["bytes_per_launch"] > 0
    assert bench.profile_summary(3, None) is not None  # any parameters (the autotuner's starting point)
    # other tuning parameters than the timed run's: not used
    other = dict(params, queue_chunk=int(params["queue_chunk"]) + 1)
    assert bench.profile_summary(3, other) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.profile_summary(3, params) is None


def test_algorithmic_weights_name_work_counters():
    assert set(bench.ALGO_OPS) <= set(sccg.STAT_KEYS)
    assert all(w > 0 for w in bench.ALGO_OPS.values())
    assert bench.VALU_PEAK_OPS == 256 * 128 * 2.4e9


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
