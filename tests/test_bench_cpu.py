"""The benchmark line's companion parts (the batched and surrogate speed-ups), assembled from
canned child-process lines: the fields the line reports, and a failing child reported in the
line instead of ending the run.  No GPU: the child processes are replaced."""

import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

ENSEMBLE_LINE = {
    "value": 3.5e10, "steps": 200, "ms_per_step": 0.2,
    "config": {"members": 64, "sizes": [128, 256, 512]},
    "roofline": {"kernel": "spec_inv", "frac": 0.48},
    "sequential": {"speedup": 10.0, "bitwise_equal_members": 0, "max_rel_diff": 5e-16},
}
SURROGATE_LINE = {
    "value": 1.3e11, "steps": 1000, "config": {"members": 64, "n": 256},
    "surrogate": {"jumps": 20, "accepted": 20, "rejected": 0, "err_over_change_mean": 0.063,
                  "err_over_change_max": 0.127, "speedup_vs_plain": 3.6},
}


def test_companions_fields(monkeypatch):
    def child(argv, timeout_s):
        assert "--workload" in argv
        return ENSEMBLE_LINE if "ensemble64_fp64" in argv else SURROGATE_LINE
    monkeypatch.setattr(bench, "_child_line", child)
    out = bench.companions()
    b, s = out["batched"], out["surrogate"]
    assert b["speedup_vs_sequential"] == 10.0 and b["members"] == 64 and b["steps"] == 200
    assert b["max_rel_diff"] == 5e-16 and b["dominant_kernel"] == "spec_inv"
    assert s["speedup_vs_plain"] == 3.6 and s["accepted"] == 20 and s["err_over_change_mean"] == 0.063
    assert "error" not in b and "error" not in s


def test_companion_failure_is_reported(monkeypatch):
    def child(argv, timeout_s):
        if "surrogate64_256" in argv:
            raise RuntimeError("exit 134: aborted")
        return ENSEMBLE_LINE
    monkeypatch.setattr(bench, "_child_line", child)
    out = bench.companions()
    assert "error" not in out["batched"]
    assert out["surrogate"]["workload"] == "surrogate64_256"
    assert "exit 134" in out["surrogate"]["error"]


def test_child_line_takes_the_last_json_line(monkeypatch):
    class R:
        returncode = 0
        stdout = "log line\n{\"a\": 1}\nmore\n{\"b\": 2}\n"
        stderr = ""
    monkeypatch.setattr(bench.subprocess, "run", lambda *a, **k: R())
    assert bench._child_line(["--workload", "x"], 5) == {"b": 2}
    R.returncode = 1
    with pytest.raises(RuntimeError):
        bench._child_line(["--workload", "x"], 5)
