"""Every launch plan computes the same steps.  A plan sets, per kernel role, the values per
thread E (4, 8 or 16: the radices of the line transforms) and the threads per workgroup,
hence the lines per workgroup G = threads / (N / E), from 1 up to 64 here, with ragged last
workgroups.  The 3-D passes store their rotated outputs through LDS tiles whose shape and
swizzle follow G, so each plan takes its own store path.  Each run is compared with the
built-in plan (itself compared with the oracle in test_gpu_parity.py) to the rounding of the
different radices: 1e-12 relative on phi, 1e-13 on the modified energy (FP64) after 20 steps.
The last plan also closes every step in a separate kernel instead of the next update kernel.
"""

import math

import numpy as np
import pytest

from paper_2012_15133_amd.inputs import noise_ic

pytestmark = pytest.mark.gpu

PLANS = [
    "inv=4/64,mid=4/64,real=4/64,fwd=4/64",
    "inv=4/256,mid=8/128,real=4/256,fwd=16/256",
    "inv=8/256,mid=8/256,real=8/256,fwd=8/256",
    "inv=16/256,mid=16/128,real=16/128,fwd=8/64",
    "inv=8/128,mid=4/256,real=4/128,fwd=4/128,finsep",
    "inv=4/128,mid=8/512,real=8/128,fwd=8/128",
    "inv=8/512,mid=4/512",
]


def _run(n, phi0, precision, plan, monkeypatch, steps=20):
    from paper_2012_15133_amd import Solver
    if plan:
        monkeypatch.setenv("SPFC_PLAN", plan)
    else:
        monkeypatch.delenv("SPFC_PLAN", raising=False)
    L = tuple(v * math.pi / 4 for v in n)
    s = Solver(n, L, phi0, 0.25, precision=precision, history=64)
    used = s.plan()
    s.step(0.005, steps)
    phi = s.phi().cpu().numpy().astype(np.float64)
    hist = s.history(0, steps + 1)
    assert s.status() == 0
    s.close()
    return phi, hist, used


def _key(used):
    return tuple(sorted((k, tuple(v)) for k, v in used.items()))


@pytest.mark.parametrize("n", [(32, 8, 16), (16, 32, 64), (64, 32), (256, 128)])
def test_plans_agree_fp64(n, monkeypatch):
    phi0 = noise_ic(tuple(reversed(n)), -0.25, 31)
    ref, ref_hist, ref_used = _run(n, phi0, "fp64", "", monkeypatch)
    scale = np.max(np.abs(ref))
    seen = {_key(ref_used)}
    for plan in PLANS:
        phi, hist, used = _run(n, phi0, "fp64", plan, monkeypatch)
        print(n, plan, used, flush=True)
        seen.add(_key(used))
        assert np.max(np.abs(phi - ref)) <= 1e-12 * scale, plan
        for x, y in zip(hist, ref_hist):
            assert abs(x["energy"] - y["energy"]) <= 1e-13 * abs(y["energy"]), plan
    assert len(seen) >= 3   # the plans were taken (some coincide where lines are short)


def test_plans_agree_fp32_3d(monkeypatch):
    n = (32, 16, 32)
    phi0 = noise_ic(tuple(reversed(n)), -0.25, 32)
    ref, ref_hist, _ = _run(n, phi0, "fp32", "", monkeypatch)
    scale = np.max(np.abs(ref))
    for plan in PLANS:
        phi, hist, used = _run(n, phi0, "fp32", plan, monkeypatch)
        print(n, plan, used, flush=True)
        # FP32 fields: a few ulp per transform, different radices round differently
        assert np.max(np.abs(phi - ref)) <= 2e-5 * scale, plan
        for x, y in zip(hist, ref_hist):
            assert abs(x["energy"] - y["energy"]) <= 1e-5 * abs(y["energy"]), plan
