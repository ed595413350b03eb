"""The paper's numerical experiments on the GPU path (through the C ABI).

Section 5.1 (manufactured solution, a = 0.975 on (0,1)^2): the forcing of the paper,
f = d_t phi_e - Delta mu(phi_e) (its closed form is pinned against sympy in
`test_oracle_pins.py`), is given to the solver as four fixed fields with
time-dependent coefficients; the forced run matches the oracle's forced run and the
error at T = 1 falls like dt^2 (the paper's figure: slope -2).  The run starts with the
first-order SAV step (the paper's start is not stated).

Section 5.2 (square patterns, a = 0.5, L = 100, noise 0.05 (2u - 1)): a short run with
dt 0.01 then 0.02 and the restart at the change, against the oracle; the modified energy
does not rise within a dt segment and the mean of the initial data is kept.
"""

import math

import numpy as np
import pytest

from oracle import spfc_oracle as O
from paper_2012_15133_amd.inputs import noise_ic

pytestmark = pytest.mark.gpu

W = 2.0 * math.pi
A_X1 = 0.975


def _x1_grid(n):
    xs = np.arange(n) / n
    X, Y = np.meshgrid(xs, xs)            # [y, x]
    return X, Y


def _exact(X, Y, t):
    return np.sin(W * X) * np.cos(W * Y) * math.cos(t) / W


def _terms(X, Y):
    sc = lambda p, q: np.sin(p * W * X) * np.cos(q * W * Y)
    return [sc(1, 1), sc(3, 3), sc(3, 1), sc(1, 3)]


def _coef(t, a=A_X1):
    c3 = W ** 3 * math.cos(t) ** 3
    return [-math.sin(t) / W + 2 * W * (a - 4 * W ** 2 + 4 * W ** 4) * math.cos(t) + 2.5 * c3,
            13.5 * c3, 2.5 * c3, -2.5 * c3]


def _forcing(X, Y, t):
    return sum(c * g for c, g in zip(_coef(t), _terms(X, Y)))


def _gpu_x1(n, NT, precision="fp64"):
    from paper_2012_15133_amd import Solver
    X, Y = _x1_grid(n)
    s = Solver((n, n), (1.0, 1.0), _exact(X, Y, 0.0), 1 - A_X1, startup="sav1", precision=precision)
    s.set_forcing(_terms(X, Y))
    dt = 1.0 / NT
    s.step_forced(dt, [_coef((k + 1) * dt) for k in range(NT)])
    phi = s.phi().cpu().numpy()
    s.close()
    return phi, X, Y


def test_x1_forcing_terms_are_the_closed_form():
    """The four-term split used on the GPU is the pinned closed form (host check)."""
    import sys, os
    sys.path.insert(0, os.path.dirname(__file__))
    from test_oracle_pins import forcing_closed_form
    X, Y = _x1_grid(16)
    for t in (0.0, 0.3, 1.0):
        assert np.max(np.abs(_forcing(X, Y, t) - forcing_closed_form(X, Y, t, A_X1))) <= 1e-9 * np.max(
            np.abs(forcing_closed_form(X, Y, t, A_X1)))


def test_x1_forced_run_matches_oracle():
    n, NT = 32, 50
    phi, X, Y = _gpu_x1(n, NT)
    g = O.Grid((n, n), (1.0, 1.0))
    ref = O.run(g, O.Params(1 - A_X1), _exact(X, Y, 0.0), 1.0 / NT, NT, startup="sav1",
                forcing=lambda t: _forcing(X, Y, t), energies=False)["phi"]
    rel = np.linalg.norm(phi - ref) / np.linalg.norm(ref)
    print(f"forced run vs oracle: rel L2 {rel:.2e}")
    assert rel <= 1e-11


def test_x1_second_order_in_time_on_gpu():
    """The paper's setting: n = 128, T = 1, N_T = 100, 200, 400, 800; fitted log-log slopes
    of the l2 and l-infinity errors against the exact solution within [1.9, 2.1]."""
    n = 128
    NTs = [100, 200, 400, 800]
    e2, einf = [], []
    for NT in NTs:
        phi, X, Y = _gpu_x1(n, NT)
        err = phi - _exact(X, Y, 1.0)
        e2.append(math.sqrt(np.sum(err * err) / (n * n)))
        einf.append(float(np.max(np.abs(err))))
    for errs in (e2, einf):
        slope = -np.polyfit(np.log(NTs), np.log(errs), 1)[0]
        print("errors", [f"{e:.3e}" for e in errs], "slope", f"{slope:.3f}")
        assert 1.9 <= slope <= 2.1


def test_forcing_errors():
    from paper_2012_15133_amd import Solver
    from paper_2012_15133_amd.binding import SpfcError
    X, Y = _x1_grid(16)
    s = Solver((16, 16), (1.0, 1.0), _exact(X, Y, 0.0), 1 - A_X1)
    with pytest.raises(ValueError):
        s.step_forced(0.01, [[1.0]])          # no forcing set (binding check)
    s.set_forcing(_terms(X, Y))
    with pytest.raises(ValueError):
        s.step_forced(0.01, [[1.0, 2.0]])     # wrong number of terms
    with pytest.raises(SpfcError):
        s.step_forced(-0.01, [_coef(0.0)])
    s.set_forcing([])                          # removed: plain steps again
    s.step(0.01, 2)
    s.close()
    g = Solver((16, 16), (1.0, 1.0), _exact(X, Y, 0.0), 1 - A_X1, startup="ghost")
    g.set_forcing(_terms(X, Y))
    with pytest.raises(SpfcError):
        g.step_forced(0.01, [_coef(0.01)])     # the ghost start is not offered with forcing
    g.close()


def test_x2_short_run_with_dt_change():
    from paper_2012_15133_amd import Solver
    n, L = 128, 100.0
    phi0 = noise_ic((n, n), 0.0, 21)
    g = O.Grid((n, n), (L, L))
    prm = O.Params(0.5)
    first = O.run(g, prm, phi0, 0.01, 100, startup="copy", energies=False)
    second = O.run(g, prm, first["phi"], 0.02, 100, startup="copy", energies=False)
    s = Solver((n, n), (L, L), phi0, 0.5, startup="copy", history=256)
    s.step(0.01, 100)
    mid = s.phi().cpu().numpy()
    s.step(0.02, 100)
    end = s.phi().cpu().numpy()
    hist = s.history(0, 201)
    for got, ref in ((mid, first["phi"]), (end, second["phi"])):
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"rel L2 vs oracle {rel:.2e}")
        assert rel <= 1e-10
    E = [h["energy"] for h in hist]   # modified energy of each recorded state
    for seg in (E[0:101], E[101:201]):
        assert all(b <= a + 1e-12 * abs(a) for a, b in zip(seg, seg[1:]))
    m0 = float(np.mean(phi0))            # the sample mean of the noise, kept by the scheme
    assert max(abs(h["mean"] - m0) for h in hist) <= 1e-15
    assert s.status() == 0
    s.close()
