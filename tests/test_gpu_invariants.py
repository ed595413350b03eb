"""Properties of the scheme that the GPU path must show at any size, independent of the
oracle (the same invariants pin the oracle in test_oracle_pins.py):

- a uniform state is steady: phi stays constant, E_1 = (1 + 1/c4)|Omega| (eq. energy
  split with the 2|Omega| constant), r and the modified energy stay constant;
- the mean decouples (no cubic term): phi0 + c gives phi^n + c with the same E_1, r and
  xi at every step (the flux and every symbol except the k = 0 mode ignore the mean);
- shifts by whole cells and the x <-> y transpose of a square grid commute with the step;
- linear regime: phi0 = b0 + delta cos(kx) with delta = 1e-6 follows the scalar BDF2
  recurrence of eq. scheme-SAV-1 restricted to one mode (xi = 1 + O(delta^2), flux O(delta^3)).
"""

import math

import numpy as np
import pytest

from paper_2012_15133_amd.inputs import noise_ic

pytestmark = pytest.mark.gpu


def _solver(n, L, phi0, eps=0.25, **kw):
    from paper_2012_15133_amd import Solver
    return Solver(n, L, phi0, eps, **kw)


@pytest.mark.parametrize("n,L", [((64, 64), (8 * math.pi,) * 2), ((16, 16, 16), (4 * math.pi,) * 3)])
def test_uniform_state_is_steady(n, L):
    b0 = -0.3
    phi0 = np.full(tuple(reversed(n)), b0)
    s = _solver(n, L, phi0)
    s.step(0.01, 50)
    phi = s.phi().cpu().numpy()
    volume = float(np.prod(L))
    hist = s.history(1, 50)
    assert np.max(np.abs(phi - b0)) <= 1e-14
    for h in hist:
        assert h["E1"] == pytest.approx(2.0 * volume, rel=1e-13)       # c4 = 1
        assert h["r"] == pytest.approx(math.sqrt(2.0 * volume), rel=1e-13)
        assert h["energy"] == pytest.approx(hist[0]["energy"], rel=1e-13)
        assert h["mean"] == pytest.approx(b0, abs=1e-14)
    assert s.status() == 0
    s.close()


def test_mean_shift_decouples():
    n, L = (64, 64), (8 * math.pi,) * 2
    phi0 = noise_ic((64, 64), -0.2, 21)
    a, b = _solver(n, L, phi0), _solver(n, L, phi0 + 0.1)
    a.step(0.01, 30)
    b.step(0.01, 30)
    assert np.max(np.abs((b.phi().cpu().numpy() - a.phi().cpu().numpy()) - 0.1)) <= 1e-12
    for ha, hb in zip(a.history(1, 30), b.history(1, 30)):
        assert hb["E1"] == pytest.approx(ha["E1"], rel=1e-12)
        assert hb["r"] == pytest.approx(ha["r"], rel=1e-12)
        assert hb["xi"] == pytest.approx(ha["xi"], rel=1e-12)
        assert hb["mean"] == pytest.approx(ha["mean"] + 0.1, abs=1e-13)
    a.close()
    b.close()


def test_shift_and_transpose_commute_with_the_step():
    n, L = (64, 64), (8 * math.pi,) * 2
    phi0 = noise_ic((64, 64), -0.2, 22)

    def run(p):
        s = _solver(n, L, np.ascontiguousarray(p))
        s.step(0.02, 20)
        out = s.phi().cpu().numpy()
        s.close()
        return out

    base = run(phi0)
    shifted = run(np.roll(phi0, (3, -5), axis=(0, 1)))
    assert np.max(np.abs(shifted - np.roll(base, (3, -5), axis=(0, 1)))) <= 1e-12
    transposed = run(phi0.T)
    assert np.max(np.abs(transposed - base.T)) <= 1e-12
    # an x-only field stays x-only
    xonly = run(np.tile(phi0[0:1, :], (64, 1)))
    assert np.max(np.abs(xonly - xonly[0:1, :])) <= 1e-14


@pytest.mark.parametrize("m", [1, 3, 5])
def test_linear_regime_follows_the_scalar_recurrence(m):
    n, L = 32, 8 * math.pi
    k = 2 * math.pi * m / L
    x = np.arange(n) * (L / n)
    d0, b0, dt, steps, a = 1e-6, -0.2, 0.05, 20, 0.75
    phi0 = b0 + d0 * np.cos(k * x)[None, :] * np.ones((n, 1))
    s = _solver((n, n), (L, L), phi0)
    amp = lambda p: 2.0 * np.mean((p[0] - b0) * np.cos(k * x))
    A_prev, A_cur = d0, d0
    for step in range(steps):
        if step == 0:
            a0, a1, a2, Ahat = 1.0, 1.0, 0.0, A_cur          # first-order SAV start
        else:
            a0, a1, a2, Ahat = 1.5, 2.0, -0.5, 2 * A_cur - A_prev
        A_new = (a1 * A_cur + a2 * A_prev + 2 * dt * k ** 4 * Ahat) / (a0 + dt * k * k * (a + k ** 4))
        A_prev, A_cur = A_cur, A_new
        s.step(dt, 1)
        got = amp(s.phi().cpu().numpy())
        assert abs(got - A_cur) <= 1e-9 * abs(A_cur), (step, got, A_cur)
    s.close()
