"""Batches of independent runs and graph replay, through the C ABI.

A batch member runs the same kernels with the same reduction order as a single run
of its own grid and parameters, so its field and records must equal the single
run's bit for bit (where the end-of-call update uses the same workgroup count,
i.e. small grids; otherwise the records of the state a call ends on differ by the
summation order only).  Graph replay launches exactly what direct launches would,
so it must reproduce them bit for bit over several calls, with synchronizing
queries between the replays.  One member is also checked against the oracle.
"""

import math

import numpy as np
import pytest

from oracle import spfc_oracle as O
from paper_2012_15133_amd.inputs import noise_ic

pytestmark = pytest.mark.gpu


def _members(specs):
    out = []
    for n, L, eps, mean, seed, prec in specs:
        out.append({"n": n, "L": L, "epsilon": eps, "precision": prec,
                    "phi0": noise_ic(tuple(reversed(n)), mean, seed)})
    return out


SPECS = [
    ((64, 64), (8 * math.pi,) * 2, 0.25, -0.2, 1, "fp64"),
    ((64, 64), (9.0 * math.pi, 7.5 * math.pi), 0.1, -0.3, 2, "fp64"),
    ((32, 32), (4 * math.pi,) * 2, 0.4, -0.1, 3, "fp64"),
    ((64, 64), (8 * math.pi,) * 2, 0.3, 0.0, 4, "fp32"),
    ((64, 64), (6 * math.pi,) * 2, 0.05, -0.35, 5, "fp64"),
    ((16, 16, 16), (4 * math.pi,) * 3, 0.25, -0.25, 6, "fp64"),
]


def _single(m, dt_steps, history, graph=False):
    from paper_2012_15133_amd import Solver
    s = Solver(m["n"], m["L"], m["phi0"], m["epsilon"], precision=m["precision"], history=history, graph=graph)
    for dt, k in dt_steps:
        s.step(dt, k)
    n = s.step_count()
    out = (s.phi().cpu().numpy(), s.history(0, n + 1), s.status())
    s.close()
    return out


def test_batch_members_equal_single_runs_bitwise():
    from paper_2012_15133_amd import Batch
    members = _members(SPECS)
    plan = [(0.01, 12), (0.01, 9), (0.02, 6)]
    b = Batch(members, history=64)
    for dt, k in plan:
        b.step(dt, k)
    assert b.step_count() == 27
    for i, m in enumerate(members):
        print(f"member {i}: n={m['n']} eps={m['epsilon']} {m['precision']}", flush=True)
        phi, hist, flags = _single(m, plan, 64)
        assert np.array_equal(b.phi(i).cpu().numpy(), phi)
        assert b.history(i, 0, 28) == hist
        assert b.status(i) == flags
    b.close()


def test_batch_member_matches_oracle():
    from paper_2012_15133_amd import Batch
    members = _members(SPECS[:3])
    b = Batch(members, history=32)
    b.step(0.01, 20)
    for i in (1, 2):
        m = members[i]
        g = O.Grid(m["n"], m["L"])
        ref = O.run(g, O.Params(m["epsilon"]), m["phi0"], 0.01, 20)
        phi = b.phi(i).cpu().numpy()
        assert np.max(np.abs(phi - ref["phi"])) <= 1e-11 * np.max(np.abs(ref["phi"]))
        for h, r in zip(b.history(i, 0, 21), ref["records"]):
            assert abs(h["energy"] - r["energy"]) <= 1e-12 * abs(r["energy"])
            assert abs(h["mean"] - r["mean"]) <= 1e-14
        e = b.energy(i)
        assert abs(e["modified_energy"] - ref["records"][-1]["energy"]) <= 1e-12 * abs(ref["records"][-1]["energy"])
        assert abs(b.mass(i) - np.mean(m["phi0"])) <= 1e-14
    b.close()


def test_batch_large_members_fields_bitwise():
    """64 members of 128^2 and 4 of 512^2 in one batch: fields equal the single runs bit
    for bit; records to summation-order rounding."""
    from paper_2012_15133_amd import Batch
    rng = np.random.default_rng(7)
    specs = []
    for k in range(64):
        specs.append(((128, 128), (32 * math.pi,) * 2, float(rng.uniform(0.05, 0.5)),
                      float(rng.uniform(-0.4, 0.0)), 100 + k, "fp64"))
    for k in range(4):
        specs.append(((512, 512), (128 * math.pi,) * 2, 0.25, -0.2, 200 + k, "fp64"))
    members = _members(specs)
    b = Batch(members, history=64)
    b.step(0.01, 30)
    for i in (0, 37, 63, 64, 67):
        print(f"member {i}", flush=True)
        phi, hist, flags = _single(members[i], [(0.01, 30)], 64)
        assert np.array_equal(b.phi(i).cpu().numpy(), phi)
        for x, y in zip(b.history(i, 0, 31), hist):
            for key in x:
                assert abs(x[key] - y[key]) <= 1e-13 * max(1.0, abs(y[key])), (i, key)
        assert b.status(i) == flags
    b.close()


def test_batch_member_index_errors():
    from paper_2012_15133_amd import Batch, SpfcError
    b = Batch(_members(SPECS[:2]), history=8)
    with pytest.raises(SpfcError):
        b.status(2)
    with pytest.raises(SpfcError):
        b.history(-1, 0, 1)
    b.close()


# ----------------------------------------------------------------- graph replay

@pytest.mark.parametrize("n,startup", [((64, 64), "sav1"), ((64, 32), "ghost"), ((16, 16, 16), "sav1"),
                                       ((256, 256), "copy")])
def test_graph_replay_equals_direct_launches(n, startup):
    from paper_2012_15133_amd import Solver
    L = tuple(2 * math.pi * v / 8 for v in n)
    phi0 = noise_ic(tuple(reversed(n)), -0.2, 9)
    plan = [(0.01, 1), (0.01, 8), (0.01, 7), (0.02, 11), (0.02, 2), (0.01, 4)]
    runs = []
    for graph in (False, True):
        s = Solver(n, L, phi0, 0.25, startup=startup, history=64, graph=graph)
        snaps = []
        for dt, k in plan:
            s.step(dt, k)
            # eager work and a synchronization between the replays
            snaps.append((s.phi().cpu().numpy(), s.energy()["modified_energy"], s.mass()))
        runs.append((snaps, s.history(0, s.step_count() + 1), s.status()))
        s.close()
    (a, ha, fa), (b, hb, fb) = runs
    for (pa, ea, ma), (pb, eb, mb) in zip(a, b):
        assert np.array_equal(pa, pb)
        assert ea == eb and ma == mb
    assert ha == hb and fa == fb


def test_graph_replay_batch_and_checkpoint():
    from paper_2012_15133_amd import Batch, Solver
    members = _members(SPECS[:4])
    b = Batch(members, history=64, graph=True)
    b.step(0.01, 10)
    b.step(0.01, 13)
    for i in (0, 3):
        phi, hist, _ = _single(members[i], [(0.01, 10), (0.01, 13)], 64)
        assert np.array_equal(b.phi(i).cpu().numpy(), phi)
        assert b.history(i, 0, 24) == hist
    b.close()
    m = members[1]
    s = Solver(m["n"], m["L"], m["phi0"], m["epsilon"], history=64, graph=True)
    s.step(0.01, 10)
    ck = s.save_state()
    s.step(0.01, 10)
    ref = s.phi().cpu().numpy()
    s.load_state(ck)
    s.step(0.01, 10)
    assert np.array_equal(s.phi().cpu().numpy(), ref)
    s.close()


def _batch_snapshots(members, graph, script):
    from paper_2012_15133_amd import Batch
    b = Batch(members, history=96, graph=graph)
    snaps = []
    for what, arg in script:
        if what == "step":
            b.step(*arg)
        elif what == "time":
            b.time_kernels(0.01, reps=3)   # runs from a snapshot and restores the state
        elif what == "profile":
            b.profile(arg)                 # while profiling the steps launch directly
        elif what == "reset":
            b.reset([m["phi0"] for m in members])
        # eager work and synchronizations between the replays
        snaps.append([(b.phi(i).cpu().numpy(), b.energy(i)["modified_energy"], b.mass(i))
                      for i in range(len(members))])
    n = b.step_count()
    out = (snaps, [b.history(i, 0, n + 1) for i in range(len(members))], [b.status(i) for i in range(len(members))])
    b.close()
    return out


def test_graph_replay_whole_batch_equals_direct_launches():
    """Several size classes with graph replay: one graph holds two steady steps of every
    class (each class a branch of its own).  Equal bit for bit to direct launches over
    calls with odd and even step counts, dt changes, kernel timing from a snapshot,
    profiled steps and a reset."""
    specs = [((64, 64), (8 * math.pi,) * 2, 0.25, -0.2, 21, "fp64"),
             ((128, 128), (32 * math.pi,) * 2, 0.1, -0.3, 22, "fp64"),
             ((32, 32), (4 * math.pi,) * 2, 0.4, -0.1, 23, "fp64"),
             ((128, 128), (32 * math.pi,) * 2, 0.3, -0.25, 24, "fp64"),
             ((64, 64), (8 * math.pi,) * 2, 0.2, -0.15, 25, "fp32"),
             ((16, 16, 16), (4 * math.pi,) * 3, 0.25, -0.25, 26, "fp64")]
    members = _members(specs)
    script = [("step", (0.01, 1)), ("step", (0.01, 8)), ("step", (0.01, 7)), ("step", (0.02, 11)),
              ("time", None), ("step", (0.02, 6)), ("profile", True), ("step", (0.02, 4)), ("profile", False),
              ("step", (0.01, 5)), ("reset", None), ("step", (0.01, 9)), ("step", (0.01, 2))]
    direct = _batch_snapshots(members, False, script)
    replay = _batch_snapshots(members, True, script)
    for k, (sa, sb) in enumerate(zip(direct[0], replay[0])):
        for i, ((pa, ea, ma), (pb, eb, mb)) in enumerate(zip(sa, sb)):
            assert np.array_equal(pa, pb), (k, i)
            assert ea == eb and ma == mb, (k, i)
    assert direct[1] == replay[1]
    assert direct[2] == replay[2] == [0] * len(members)


# ----------------------------------------------------------------- launch-plan tuner

def test_tune_keeps_the_run_state():
    """Tuning mid-run restores the state: records so far unchanged, the step count
    unchanged, and the continuation equal to an untuned run up to the rounding of the
    different transform radices."""
    from paper_2012_15133_amd import Solver
    n, L = (128, 64), (16 * math.pi, 8 * math.pi)
    phi0 = noise_ic((64, 128), -0.2, 12)
    a = Solver(n, L, phi0, 0.25, history=128)
    b = Solver(n, L, phi0, 0.25, history=128)
    a.step(0.01, 30)
    b.step(0.01, 30)
    before = a.history(0, 31)
    plan = a.tune(0.01, trial_steps=6)
    print("plan", plan, flush=True)
    assert set(plan) == {"inv", "real", "fwd"}
    assert all(e in (4, 8, 16) and 32 <= t <= 256 for e, t in plan.values())
    assert a.step_count() == 30 and a.history(0, 31) == before
    a.step(0.01, 40)
    b.step(0.01, 40)
    pa, pb = a.phi().cpu().numpy(), b.phi().cpu().numpy()
    assert np.max(np.abs(pa - pb)) <= 1e-12 * np.max(np.abs(pb))
    for x, y in zip(a.history(0, 71), b.history(0, 71)):
        assert abs(x["energy"] - y["energy"]) <= 1e-13 * abs(y["energy"])
    a.close()
    b.close()


def test_batch_tune_then_step_matches_untuned_members():
    from paper_2012_15133_amd import Batch
    members = _members(SPECS)
    b = Batch(members, history=64)
    b.step(0.01, 5)
    b.tune(0.01, trial_steps=4)
    for i in range(len(members)):
        assert set(b.plan(i)) >= {"inv", "real", "fwd"}
    assert b.step_count() == 5
    b.step(0.01, 20)
    for i in (0, 2, 5):
        phi, hist, _ = _single(members[i], [(0.01, 5), (0.01, 20)], 64)
        got = b.phi(i).cpu().numpy()
        assert np.max(np.abs(got - phi)) <= 1e-12 * np.max(np.abs(phi))
        for x, y in zip(b.history(i, 0, 26), hist):
            assert abs(x["energy"] - y["energy"]) <= 1e-13 * abs(y["energy"])
    b.close()


def test_time_kernels_keeps_the_run_state():
    """Back-to-back kernel timing perturbs the older state while it runs and restores
    the snapshot afterwards: the run continues bit for bit as an untimed run."""
    from paper_2012_15133_amd import Solver
    n, L = (128, 128), (16 * math.pi,) * 2
    phi0 = noise_ic((128, 128), -0.2, 14)
    a = Solver(n, L, phi0, 0.25, history=64)
    b = Solver(n, L, phi0, 0.25, history=64)
    a.step(0.01, 12)
    b.step(0.01, 12)
    kt = a.time_kernels(0.01, reps=5)
    names = {k["name"] for k in kt}
    assert {"spec_inv", "real_pass", "spec_fwd"} <= names
    assert all(k["avg_ms"] > 0 and k["launches"] == 1 for k in kt if k["name"] != "step_finalize")
    assert a.step_count() == 12
    a.step(0.01, 9)
    b.step(0.01, 9)
    assert np.array_equal(a.phi().cpu().numpy(), b.phi().cpu().numpy())
    assert a.history(0, 22) == b.history(0, 22)
    assert a.status() == b.status()
    a.close()
    b.close()


def test_phi_all_equals_per_member_fields_bitwise():
    """spfc_batch_get_phi_all (one launch per pass for every 64 members) gives what the
    member-by-member call gives, for a class wider than one launch and a 3-D class."""
    import torch
    from paper_2012_15133_amd import Batch
    from paper_2012_15133_amd.binding import SPFC_FP32, SPFC_FP64, spfc_batch_get_phi_all
    specs = [((32, 32), (4 * math.pi,) * 2, 0.1 + 0.004 * k, -0.2, 100 + k, "fp64") for k in range(70)]
    specs += [((16, 16, 16), (4 * math.pi,) * 3, 0.25, -0.25, 7 + k, "fp32") for k in range(2)]
    members = _members(specs)
    b = Batch(members, history=8)
    b.step(0.01, 5)
    for dt, code in (("fp64", SPFC_FP64), ("fp32", SPFC_FP32)):
        outs = [torch.full(tuple(reversed(m["n"])), float("nan"), device="cuda",
                           dtype=torch.float64 if dt == "fp64" else torch.float32) for m in members]
        spfc_batch_get_phi_all(b.b, [o.data_ptr() for o in outs], code)
        b.stream.synchronize()
        for i in range(len(members)):
            assert torch.equal(outs[i], b.phi(i, dt)), (dt, i)
    same = torch.empty((70, 32, 32), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        b.phi_all(same)          # the batch holds two grid sizes
    b.close()


def test_reset_from_one_tensor_equals_reset_from_a_list():
    """Batch.reset takes either a sequence of fields or one contiguous [members, n_y, n_x]
    float64 device tensor (pointers computed from its stride): same restart, same bits."""
    import torch
    from paper_2012_15133_amd import Batch
    specs = [((64, 64), (8 * math.pi,) * 2, 0.1 + 0.05 * k, -0.2, 60 + k, "fp64") for k in range(4)]
    members = _members(specs)
    a, b = Batch(members, history=8), Batch(members, history=8)
    a.step(0.01, 30)
    fields = a.phi_all(torch.empty((4, 64, 64), dtype=torch.float64, device="cuda")).clone()
    shift = [0.001 * (k + 1) for k in range(4)]
    a.reset(fields, shift)
    b.reset([fields[m].clone() for m in range(4)], shift)
    for x, y in zip(a.energies(), b.energies()):
        assert x["r"] == y["r"] and x["E1"] == y["E1"]
    a.step(0.01, 10)
    b.step(0.01, 10)
    for m in range(4):
        assert torch.equal(a.phi(m), b.phi(m))


def test_reset_restarts_like_init_and_shifts_r():
    import torch
    from paper_2012_15133_amd import Batch
    from paper_2012_15133_amd.binding import SpfcError
    specs = [((64, 64), (8 * math.pi,) * 2, 0.1 + 0.05 * k, -0.2, 40 + k, "fp64") for k in range(4)]
    members = _members(specs)
    b = Batch(members, history=8)
    b.step(0.01, 150)
    before = b.energies()
    fields = b.phi_all(torch.empty((4, 64, 64), dtype=torch.float64, device="cuda"))
    fields = [fields[m].clone() for m in range(4)]
    # a restart without a shift is the same run as a batch started from those fields
    fresh = Batch([dict(m, phi0=f.cpu().numpy()) for m, f in zip(members, fields)], history=8)
    b.reset(fields)
    assert b.step_count() == 0
    b.step(0.01, 20)
    fresh.step(0.01, 20)
    for m in range(4):
        assert torch.equal(b.phi(m), fresh.phi(m))
    # with the shift r - sqrt(E_1) the SAV variable of the state is carried over exactly
    shift = [p["r"] - math.sqrt(p["E1"]) for p in before]
    assert max(abs(s) for s in shift) > 1e-6          # the run has drifted from sqrt(E_1)
    b.reset(fields, shift)
    after = b.energies()
    for p, a in zip(before, after):
        assert a["r"] == pytest.approx(p["r"], rel=1e-13)
        assert a["E1"] == pytest.approx(p["E1"], rel=1e-13)
        assert a["sav_energy"] == pytest.approx(p["sav_energy"], rel=1e-13)
    # a shift that makes r non-positive: error, and that member keeps sqrt(E_1)
    bad = list(shift)
    bad[2] = -2.0 * math.sqrt(before[2]["E1"])
    with pytest.raises(SpfcError):
        b.reset(fields, bad)
    e = b.energies()
    assert e[2]["r"] == pytest.approx(math.sqrt(e[2]["E1"]), rel=1e-15)
    assert e[1]["r"] == pytest.approx(before[1]["r"], rel=1e-13)
    b.close()
    fresh.close()
