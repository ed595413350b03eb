"""Stabilized SAV scheme (closing remarks of Section 5) on the GPU against the oracle.

Same tolerances as the plain FP64 parity tests (1e-11 on phi, 1e-12 on the modified
energy); the stabilization only changes the symbols of the step operator and its
right-hand side and adds one energy term.  The singular-data case compares both
schemes in the regime where the plain one fails (xi < 0): the GPU must follow the
oracle there too.
"""

import math

import numpy as np
import pytest

from oracle import spfc_oracle as O
from paper_2012_15133_amd.inputs import noise_ic

pytestmark = pytest.mark.gpu


def _compare(n, L, eps, A, phi0, dt, steps, startup="sav1", tol_phi=1e-11, tol_e=1e-12):
    from paper_2012_15133_amd import Solver
    g = O.Grid(n, L)
    prm = O.Params(eps, stab=A)
    ref = O.run(g, prm, phi0, dt, steps, startup=startup)
    s = Solver(n, L, phi0, eps, startup=startup, history=steps + 1, stab=A)
    s.step(dt, steps)
    phi = s.phi().cpu().numpy()
    hist = s.history(0, steps + 1)
    rel = np.max(np.abs(phi - ref["phi"])) / np.max(np.abs(ref["phi"]))
    print(f"{n} A={A}: rel Linf {rel:.2e}", flush=True)
    assert rel <= tol_phi
    for k, (h, r) in enumerate(zip(hist, ref["records"])):
        assert abs(h["energy"] - r["energy"]) <= tol_e * abs(r["energy"]), k
        assert abs(h["mean"] - r["mean"]) <= 1e-14 * math.sqrt(k + 1) + 1e-15, k
        if k > 0:
            assert abs(h["xi"] - r["xi"]) <= 1e-11 * max(1.0, abs(r["xi"])), k
    e = s.energy()
    assert abs(e["modified_energy"] - ref["records"][-1]["energy"]) <= tol_e * abs(ref["records"][-1]["energy"])
    flags = s.status()
    s.close()
    return hist, flags


@pytest.mark.parametrize("n,A,startup", [((64, 64), 50.0, "sav1"), ((64, 32), 2.0, "ghost"),
                                         ((16, 16, 16), 5.0, "copy")])
def test_stabilized_trajectory(n, A, startup):
    L = tuple(2 * math.pi * v / 8 for v in n)
    phi0 = noise_ic(tuple(reversed(n)), -0.2, 21)
    if startup == "ghost":
        # smooth data: the ghost start differentiates mu^0 twice more
        phi0 = O.ifftn(O.fftn(phi0) * (O.Grid(n, L).ksq() < 1.0)).real
    hist, flags = _compare(n, L, 0.25, A, phi0, 0.02, 40, startup)
    assert flags == 0
    for a, b in zip(hist[1:], hist[2:]):
        assert b["energy"] <= a["energy"] * (1 + 1e-12)


def test_singular_data_plain_and_stabilized():
    n = (64, 64)
    g = O.Grid(n, (100.0, 100.0))
    phi0 = noise_ic(g.shape, 0.0, 5)
    phi0[32, 32] += 10.0
    hist, _ = _compare(n, (100.0, 100.0), 0.5, 0.0, phi0, 0.01, 30)
    assert min(h["xi"] for h in hist[1:]) < 0.0
    hist, flags = _compare(n, (100.0, 100.0), 0.5, 1e5, phi0, 0.01, 30)
    assert all(abs(h["xi"] - 1.0) <= 0.02 for h in hist[1:])
    assert flags & 1 == 0


def test_stabilized_batch_member_equals_single_run():
    from paper_2012_15133_amd import Batch, Solver
    n, L = (64, 64), (8 * math.pi,) * 2
    members = [{"n": n, "L": L, "epsilon": 0.25, "stab": A, "phi0": noise_ic((64, 64), -0.2, 30 + k)}
               for k, A in enumerate((0.0, 3.0, 300.0))]
    b = Batch(members, history=32)
    b.step(0.01, 25)
    for i, m in enumerate(members):
        s = Solver(n, L, m["phi0"], 0.25, history=32, stab=m["stab"])
        s.step(0.01, 25)
        assert np.array_equal(b.phi(i).cpu().numpy(), s.phi().cpu().numpy())
        assert b.history(i, 0, 26) == s.history(0, 26)
        s.close()
    b.close()
