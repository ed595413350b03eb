"""The stored oracle trajectories under tests/golden/ against the oracle that wrote them.

Each file must carry the recipe tests/golden/make_golden.py states for it, and satisfy what
the scheme guarantees along any trajectory: the mean of phi kept (Theorem 2.1) and the
modified energy non-increasing (Theorem 3.1).  The first step of the 1024^2 trajectory is
recomputed by the oracle here (about ten seconds), so a file written by an older oracle
fails; the 256^3 one is checked by its invariants only (one oracle step there takes minutes).
"""

import json
import math
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_golden as MG  # noqa: E402
from oracle import spfc_oracle as O  # noqa: E402
from paper_2012_15133_amd.inputs import noise_ic  # noqa: E402


def _load(which):
    path = os.path.join(HERE, "golden", MG.RUNS[which]["file"])
    if not os.path.exists(path):
        pytest.skip(f"{path} not written")
    d = np.load(path, allow_pickle=False)
    return json.loads(str(d["meta"])), d


@pytest.mark.parametrize("which", sorted(MG.RUNS))
def test_fixture_recipe_and_invariants(which):
    meta, d = _load(which)
    spec = MG.RUNS[which]
    for k in ("n", "epsilon", "dt", "steps", "seed", "mean", "startup", "stride"):
        assert meta[k] == (list(spec[k]) if isinstance(spec[k], tuple) else spec[k]), k
    assert np.allclose(meta["L"], spec["L"], rtol=0, atol=1e-12)
    steps = spec["steps"]
    for key in ("energy", "mean", "r", "xi", "E1", "p1"):
        assert d[key].shape == (steps + 1,), key
        assert np.all(np.isfinite(d[key])), key
    volume = math.prod(spec["L"])
    assert np.all(np.abs(d["mean"] - d["mean"][0]) <= 1e-13)
    assert np.all(np.diff(d["energy"]) <= 1e-12 * d["energy"][:-1])
    assert np.all(d["p1"][1:] <= 0.0) and np.all(d["E1"][1:] >= volume)
    assert sorted(int(k) for k in d["steps_kept"]) == sorted(spec["keep"])
    side = tuple(v // spec["stride"] for v in reversed(spec["n"]))
    for k in spec["keep"]:
        assert d[f"phi_{k}"].shape == side


def test_c2_fixture_first_step_is_the_oracle_s():
    meta, d = _load("c2")
    g = O.Grid(tuple(meta["n"]), tuple(meta["L"]))
    phi0 = noise_ic(g.shape, meta["mean"], meta["seed"])
    ref = O.run(g, O.Params(meta["epsilon"]), phi0, meta["dt"], 1, startup=meta["startup"])
    sl = tuple(slice(None, None, meta["stride"]) for _ in meta["n"])
    # the same code on the same inputs: equal up to the last bits a different CPU's vector
    # math library may change
    assert np.max(np.abs(ref["phi"][sl] - d["phi_1"])) <= 1e-14 * np.max(np.abs(d["phi_1"]))
    for i, rec in enumerate(ref["records"]):
        assert abs(rec["energy"] - d["energy"][i]) <= 1e-14 * d["energy"][i]
        assert abs(rec["r"] - d["r"][i]) <= 1e-14 * d["r"][i]
        assert abs(rec["mean"] - d["mean"][i]) <= 1e-15
