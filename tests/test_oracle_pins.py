"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these tests compares the oracle with itself: each checks it against a
brute-force definition, a closed form, a symbolic derivation (sympy), an
identity proved in the paper, or an independent library routine.
"""

import math

import numpy as np
import pytest
import sympy as sp

from oracle import spfc_oracle as O
from paper_2012_15133_amd.inputs import noise_ic

RNG = np.random.default_rng(12345)


# ----------------------------------------------------------------- P1: FFT

def brute_dft(x, sign):
    """O(n^2d) DFT straight from the definition sum_j x_j exp(sign 2 pi i m.j/n)."""
    out = np.zeros(x.shape, dtype=np.complex128)
    idx = np.indices(x.shape).reshape(x.ndim, -1).T
    flat = x.reshape(-1)
    for m in idx:
        ph = sum(m[a] * idx[:, a] / x.shape[a] for a in range(x.ndim))
        out[tuple(m)] = np.sum(flat * np.exp(sign * 2j * np.pi * ph))
    return out


@pytest.mark.parametrize("shape", [(8, 8), (16, 8), (4, 16), (8, 4, 2), (8, 8, 8), (2, 2)])
def test_fft_matches_brute_dft(shape):
    x = RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)
    F = O.fftn(x)
    ref = brute_dft(x, -1)
    assert np.max(np.abs(F - ref)) <= 1e-13 * np.max(np.abs(ref))
    inv = O.ifftn(ref)
    assert np.max(np.abs(inv - x)) <= 1e-13 * np.max(np.abs(x))
    # unnormalised inverse direction against the definition as well
    assert np.max(np.abs(inv * x.size - brute_dft(ref, +1))) <= 1e-12 * np.max(np.abs(ref))


def test_fft_parseval_and_library_crosscheck():
    x = RNG.standard_normal((64, 32))
    F = O.fftn(x)
    assert abs(np.sum(np.abs(F) ** 2) / x.size - np.sum(x * x)) <= 1e-12 * np.sum(x * x)
    # independent library routine (pocketfft via numpy), test-only cross-check
    assert np.max(np.abs(F - np.fft.fftn(x))) <= 1e-12 * np.max(np.abs(F))
    y = RNG.standard_normal((16, 16, 16))
    assert np.max(np.abs(O.fftn(y) - np.fft.fftn(y))) <= 1e-12 * np.max(np.abs(np.fft.fftn(y)))


def test_fft_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        O.fftn(np.zeros((6, 8)))


# ----------------------------------------------------------------- P2: derivatives of trig polynomials

def _trig_poly(g, nterms, rng):
    """Random real trig polynomial with |mt| < n/2 per axis, its gradient and Laplacian."""
    xs = np.meshgrid(*[np.arange(n) * h for n, h in zip(g.n, g.h)], indexing="ij")
    xs = [np.transpose(c) for c in xs]         # array order [.., y, x]
    f = np.zeros(g.shape)
    gr = [np.zeros(g.shape) for _ in range(g.dim)]
    lp = np.zeros(g.shape)
    for _ in range(nterms):
        m = [int(rng.integers(-(n // 2) + 1, n // 2)) for n in g.n]
        k = [2 * np.pi * mj / Lj for mj, Lj in zip(m, g.L)]
        c, s = rng.standard_normal(2)
        th = sum(kj * xj for kj, xj in zip(k, xs))
        f += c * np.cos(th) + s * np.sin(th)
        for j in range(g.dim):
            gr[j] += k[j] * (-c * np.sin(th) + s * np.cos(th))
        lp += -sum(kj * kj for kj in k) * (c * np.cos(th) + s * np.sin(th))
    return f, gr, lp


@pytest.mark.parametrize("n,L", [((16, 16), (2.0, 2.0)), ((32, 16), (8 * np.pi, 3.0)),
                                 ((8, 8, 8), (1.0, 1.0, 1.0)), ((16, 8, 4), (5.0, 2.0, 1.5))])
def test_spectral_derivatives_exact_on_trig_polys(n, L):
    g = O.Grid(n, L)
    f, gr, lp = _trig_poly(g, 12, np.random.default_rng(7))
    scale = np.max(np.abs(lp)) + 1.0
    for j, d in enumerate(O.grad(g, f)):
        assert np.max(np.abs(d - gr[j])) <= 1e-12 * scale
    assert np.max(np.abs(O.lap(g, f) - lp)) <= 1e-12 * scale
    assert np.max(np.abs(O.div(g, gr) - lp)) <= 1e-12 * scale
    a = 0.3
    ref = a * f + O.lap(g, O.lap(g, f))
    assert np.max(np.abs(O.L_op(g, O.Params(1 - a), f) - ref)) <= 1e-12 * (np.max(np.abs(ref)) + 1)


def test_nyquist_conventions():
    """Odd-order symbol drops the Nyquist mode, even-order keeps it (reading of the
    even-n grids used in Section 5)."""
    g = O.Grid((8, 8), (2 * np.pi, 2 * np.pi))
    x = np.arange(8)
    cb = np.cos(np.pi * x)[None, :] * np.ones((8, 1))   # (-1)^x: the x-Nyquist mode
    for d in O.grad(g, cb):
        assert np.max(np.abs(d)) < 1e-14
    assert np.max(np.abs(O.lap(g, cb) + 16.0 * cb)) < 1e-12   # -(pi n / L)^2 = -16


def test_summation_by_parts():
    """<f, Delta g> = -<grad f, grad g> and <f, L g> = <L f, g> (eqs. spectral-coll-inner product-3/-4),
    on functions without Nyquist content (where nabla.nabla = Delta holds for even n)."""
    g = O.Grid((16, 16), (3.0, 3.0))
    f, _, _ = _trig_poly(g, 10, np.random.default_rng(1))
    q, _, _ = _trig_poly(g, 10, np.random.default_rng(2))
    lhs = O.inner(g, f, O.lap(g, q))
    rhs = -sum(O.inner(g, a, b) for a, b in zip(O.grad(g, f), O.grad(g, q)))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)
    prm = O.Params(0.25)
    assert abs(O.inner(g, f, O.L_op(g, prm, q)) - O.inner(g, O.L_op(g, prm, f), q)) < 1e-10


# ----------------------------------------------------------------- P3/P4: energies and chemical potential

def test_E1_single_mode_closed_form():
    """phi = A cos(kx), 4m < n: E_1 = |Omega| (3/32 A^4 k^4 - 1/2 A^2 k^2 + 2) (c4 = 1),
    from E_1 = int 1/4|grad phi|^4 - |grad phi|^2 + 2 (eq. energy-SPFC-split-1)."""
    L, n, m, A = 8 * np.pi, 64, 4, 0.7
    g = O.Grid((n, n), (L, L))
    k = 2 * np.pi * m / L
    x = np.arange(n) * g.h[0]
    phi = A * np.cos(k * x)[None, :] * np.ones((n, 1))
    ref = g.volume * (3.0 / 32 * A ** 4 * k ** 4 - 0.5 * A ** 2 * k ** 2 + 2.0)
    assert abs(O.E1(g, O.Params(0.25), phi) - ref) <= 1e-12 * ref


def test_N_single_mode_closed_form():
    """Same mode, 3m < n/2: N = 3/4 A^3 k^4 (cos t - cos 3t) - 2 k^2 A cos t (t = kx)."""
    L, n, m, A = 8 * np.pi, 64, 4, 0.7
    g = O.Grid((n, n), (L, L))
    k = 2 * np.pi * m / L
    th = k * np.arange(n) * g.h[0]
    phi = A * np.cos(th)[None, :] * np.ones((n, 1))
    ref = (0.75 * A ** 3 * k ** 4 * (np.cos(th) - np.cos(3 * th)) - 2 * k * k * A * np.cos(th))[None, :]
    assert np.max(np.abs(O.N_nl(g, O.Params(0.25), phi) - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("dim", [2, 3])
def test_sav_energy_two_mode_closed_form(dim):
    """The SAV energy of Section 5.2, a/2 ||phi||^2 + 1/2 ||Delta_N phi||^2 + r^2, on
    phi = b0 + A cos(k x) + B sin(l y) (k, l below the Nyquist mode, k != 1 != l):
    ||phi||^2 = |Omega| (b0^2 + A^2/2 + B^2/2) and ||Delta phi||^2 = |Omega| (k^4 A^2 + l^4 B^2)/2
    by orthogonality, so the value is |Omega| [a (b0^2 + (A^2 + B^2)/2) + (k^4 A^2 + l^4 B^2)/2] / 2
    + r^2.  A wrong weight on either norm, a Laplacian taken as a gradient, r in place of
    r^2 or a dropped mean all change it."""
    n = (32, 16) if dim == 2 else (16, 8, 8)
    L = (6.0, 2.5) if dim == 2 else (6.0, 2.5, 3.0)
    g = O.Grid(n, L)
    prm = O.Params(0.3)
    b0, A, B, r = -0.3, 0.7, 0.45, 1.9
    k, l = 2 * np.pi * 3 / L[0], 2 * np.pi * 2 / L[1]
    axes = [np.arange(nj) * hj for nj, hj in zip(g.n, g.h)]
    x = axes[0].reshape((1,) * (dim - 1) + (-1,))
    y = axes[1].reshape((1,) * (dim - 2) + (-1, 1))
    phi = (b0 + A * np.cos(k * x) + B * np.sin(l * y)) * np.ones(g.shape)
    ref = 0.5 * g.volume * (prm.a * (b0 ** 2 + 0.5 * (A * A + B * B)) + 0.5 * (k ** 4 * A * A + l ** 4 * B * B)) + r * r
    assert abs(O.sav_energy(g, prm, phi, r) - ref) <= 1e-13 * ref


def _sympy_fields(dim, L, expr_fn, c4):
    xs = sp.symbols("x y z")[:dim]
    phi = expr_fn(*xs)
    grads = [sp.diff(phi, v) for v in xs]
    s = sum(gv ** 2 for gv in grads)
    Nexpr = -c4 * sum(sp.diff(s * gv, v) for gv, v in zip(grads, xs)) + 2 * sum(sp.diff(phi, v, 2) for v in xs)
    lapphi = sum(sp.diff(phi, v, 2) for v in xs)
    dens = sp.Rational(1, 4) * c4 * s ** 2 - s
    return xs, [sp.lambdify(xs, e, "numpy") for e in (phi, Nexpr, dens, lapphi)]


@pytest.mark.parametrize("dim", [2, 3])
def test_E1_N_EN_match_symbolic_on_low_degree_fields(dim):
    """For a trig polynomial whose products stay below the grid's resolution, the pseudo-spectral
    E_1, N_N and E_N equal the continuous ones (sympy), since the trapezoid rule and spectral
    derivatives are exact there (Section 2.1)."""
    L = 2 * np.pi * 3.0
    n = 32 if dim == 2 else 16
    k = 2 * np.pi / L
    c4 = 1.3
    if dim == 2:
        fn = lambda x, y: 0.4 * sp.cos(k * x) + 0.3 * sp.sin(k * (x + 2 * y)) - 0.2 * sp.cos(2 * k * y) + 0.1
    else:
        fn = lambda x, y, z: 0.4 * sp.cos(k * x) + 0.3 * sp.sin(k * (x - y + z)) + 0.25 * sp.cos(k * z) - 0.2
    xs, (fphi, fN, fdens, flap) = _sympy_fields(dim, L, fn, c4)
    g = O.Grid((n,) * dim, (L,) * dim)
    grid = [np.arange(n) * g.h[0]] * dim
    mesh = np.meshgrid(*grid, indexing="ij")
    mesh = [np.transpose(c) for c in mesh]
    ev = lambda f: np.broadcast_to(np.asarray(f(*mesh), dtype=np.float64), g.shape)
    phi, Nref, dens, lp = ev(fphi), ev(fN), ev(fdens), ev(flap)
    prm = O.Params(0.4, c4=c4)
    assert np.max(np.abs(O.N_nl(g, prm, phi) - Nref)) <= 1e-12 * np.max(np.abs(Nref))
    E1ref = g.cell * np.sum(dens) + (1 + 1 / c4) * g.volume
    assert abs(O.E1(g, prm, phi) - E1ref) <= 1e-12 * E1ref
    # E_N = (c4/4)||grad||^4 - ||grad||^2 + a/2||phi||^2 + 1/2||lap||^2  (eq. energy-discrete-spectral)
    ENref = g.cell * np.sum(dens + 0.5 * prm.a * phi * phi + 0.5 * lp * lp)
    assert abs(O.E_N(g, prm, phi) - ENref) <= 1e-12 * abs(ENref)


def test_E1_lower_bound_pointwise():
    """(c4/4) s^2 - s + 1/c4 >= 0 gives E_1 >= |Omega| (eqs. energy-SPFC-split-2-1/-2-2),
    including a field tuned so that |grad phi|^2 is close to the minimiser 2/c4."""
    g = O.Grid((32, 32), (2 * np.pi * 4, 2 * np.pi * 4))
    for c4 in (1.0, 0.5, 3.0):
        prm = O.Params(0.25, c4=c4)
        for A in (0.0, 0.3, math.sqrt(2.0 / c4), 2.5):
            x = np.arange(32) * g.h[0]
            phi = A * np.sin(x)[None, :] * np.ones((32, 1))
            assert O.E1(g, prm, phi) >= g.volume * (1 - 1e-14)


# ----------------------------------------------------------------- the time step

def _c1_like(n=32, seed=1, mean=-0.2, L=8 * np.pi):
    g = O.Grid((n, n), (L, L))
    return g, O.Params(0.25), noise_ic(g.shape, mean, seed)


@pytest.mark.parametrize("startup", ["sav1", "ghost", "copy"])
def test_mass_conservation(startup):
    """Theorem 2.1: the mean of phi^n stays at the mean of phi^0 (for ghost, mean(phi^-1) =
    mean(phi^0) because mean(Delta_N mu) = 0)."""
    g, prm, phi0 = _c1_like()
    out = O.run(g, prm, phi0, 0.01, 30, startup=startup, energies=False)
    m0 = np.mean(phi0)
    # the mean is exact in exact arithmetic; each step may add a few roundings of O(1) values
    eps = np.finfo(np.float64).eps
    for k, rec in enumerate(out["records"]):
        assert abs(rec["mean"] - m0) <= 10 * (k + 1) * eps


def _identity_residual(g, prm, dt, phi_n, phi_nm1, r_n, r_nm1, alpha, extrapolate):
    phi1, r1, info = O.sav_step(g, prm, dt, phi_n, phi_nm1, r_n, r_nm1, alpha=alpha, extrapolate=extrapolate)
    mu = O.mu_of(g, prm, phi1, info["phihat"], r1)
    diss = dt * O.inner(g, O.lap(g, mu), mu)         # = -dt ||grad mu||^2 (eq. eng stab-2-1)
    if extrapolate:
        # Theorem 3.1, eq. eng stab-5
        lhs = (O.modified_energy(g, prm, phi1, phi_n, r1, r_n)
               - O.modified_energy(g, prm, phi_n, phi_nm1, r_n, r_nm1))
        rhs = (-0.25 * O.L_half_sq(g, prm, phi1 - 2 * phi_n + phi_nm1)
               - 0.5 * (r1 - 2 * r_n + r_nm1) ** 2 + diss)
    else:
        # first-order start step from (phi^0, phi^0, r^0, r^0): the same algebra with
        # BDF1 weights gives E(1) - E(0) = 3/2 dt <Delta mu, mu> - 1/4||L^1/2 (phi1-phi0)||^2 - 1/2 (r1-r0)^2
        lhs = (O.modified_energy(g, prm, phi1, phi_n, r1, r_n)
               - O.modified_energy(g, prm, phi_n, phi_n, r_n, r_n))
        rhs = 1.5 * diss - 0.25 * O.L_half_sq(g, prm, phi1 - phi_n) - 0.5 * (r1 - r_n) ** 2
    scale = O.modified_energy(g, prm, phi_n, phi_nm1, r_n, r_nm1)
    return phi1, r1, info, (lhs - rhs) / scale, lhs


@pytest.mark.parametrize("dim", [2, 3])
def test_energy_identity_exact(dim):
    """Theorem 3.1 holds as an identity (not just an inequality) step by step."""
    if dim == 2:
        g, prm, phi0 = _c1_like(n=32)
    else:
        g = O.Grid((8, 8, 8), (4 * np.pi,) * 3)
        prm = O.Params(0.25)
        phi0 = noise_ic(g.shape, -0.25, 3)
    dt = 0.01
    phi_n, phi_nm1, r_n, r_nm1 = O.initial_state(g, prm, dt, phi0, "sav1")
    phi1, r1, info, res, lhs = _identity_residual(g, prm, dt, phi_n, phi_nm1, r_n, r_nm1, O.BDF1, False)
    assert abs(res) <= 1e-12 and lhs <= 0
    phi_nm1, phi_n, r_nm1, r_n = phi_n, phi1, r_n, r1
    for _ in range(6):
        phi1, r1, info, res, lhs = _identity_residual(g, prm, dt, phi_n, phi_nm1, r_n, r_nm1, O.BDF2, True)
        assert abs(res) <= 1e-12
        assert lhs <= 0
        phi_nm1, phi_n, r_nm1, r_n = phi_n, phi1, r_n, r1


def test_energy_identity_ghost_start():
    g, prm, phi0 = _c1_like(n=16)
    dt = 0.02
    phi_n, phi_nm1, r_n, r_nm1 = O.initial_state(g, prm, dt, phi0, "ghost")
    assert abs(np.mean(phi_nm1) - np.mean(phi0)) < 1e-15
    for _ in range(4):
        phi1, r1, info, res, lhs = _identity_residual(g, prm, dt, phi_n, phi_nm1, r_n, r_nm1, O.BDF2, True)
        assert abs(res) <= 1e-12 and lhs <= 0
        phi_nm1, phi_n, r_nm1, r_n = phi_n, phi1, r_n, r1


def test_energy_monotone_solvability_signs():
    """Theorem 3.1 (monotone modified energy), eq. solver-5 (p1 <= 0), eq. energy-SPFC-split-2-2."""
    g, prm, phi0 = _c1_like(n=32, seed=4)
    out = O.run(g, prm, phi0, 0.05, 40)
    recs = out["records"]
    for a, b in zip(recs, recs[1:]):
        assert b["energy"] <= a["energy"]
    for rec in recs[1:]:
        assert rec["p1"] <= 0.0
        assert rec["E1"] >= g.volume


def test_r_update_matches_xi_form():
    """Solving eq. solver-4 for <N, phi^{n+1}> and substituting (eq. solver-6, solver-2) must agree
    with the closed form xi = [rho + (a0 p2 - p_psi)/(2S)] / [a0 (S - dt p1/(2S))] where
    p2 = <N, A^-1 psi>, p_psi = <N, psi>, phi^{n+1} = dt xi A^-1 Delta N + A^-1 psi."""
    g, prm, phi0 = _c1_like(n=16, seed=9)
    dt = 0.03
    out = O.run(g, prm, phi0, dt, 3, energies=False)
    phi_n, phi_nm1, r_n, r_nm1 = out["phi"], out["phi_prev"], out["r"], out["r_prev"]
    phi1, r1, info = O.sav_step(g, prm, dt, phi_n, phi_nm1, r_n, r_nm1)
    a0, a1, a2 = O.BDF2
    psi = a1 * phi_n + a2 * phi_nm1
    rho = a1 * r_n + a2 * r_nm1
    S = math.sqrt(info["E1"])
    Nn = info["N"]
    k2 = g.ksq()
    A = a0 + dt * k2 * (prm.a + k2 * k2)
    b1 = np.real(np.fft.ifftn(-k2 * np.fft.fftn(Nn) / A))
    b2 = np.real(np.fft.ifftn(np.fft.fftn(psi) / A))
    p1, p2, pp = (g.cell * np.sum(Nn * b1), g.cell * np.sum(Nn * b2), g.cell * np.sum(Nn * psi))
    xi = (rho + (a0 * p2 - pp) / (2 * S)) / (a0 * (S - dt * p1 / (2 * S)))
    assert abs(xi * S - r1) <= 1e-13 * abs(r1)
    assert np.max(np.abs(dt * xi * b1 + b2 - phi1)) <= 1e-12 * np.max(np.abs(phi1))


def test_uniform_state_is_fixed_point():
    g = O.Grid((16, 16), (5.0, 5.0))
    prm = O.Params(0.25)
    phi0 = np.full(g.shape, -0.3)
    out = O.run(g, prm, phi0, 0.1, 10)
    assert np.max(np.abs(out["phi"] + 0.3)) < 1e-15
    for rec in out["records"]:
        assert abs(rec["r"] - math.sqrt(2 * g.volume)) < 1e-12
        assert abs(rec["energy"] - out["records"][0]["energy"]) < 1e-12 * rec["energy"]


def test_mean_shift_decouples():
    """With the SPFC nonlinearity depending on grad phi only, phi0 + c evolves as phi + c,
    r and xi unchanged, modified energy shifted by a/2 |Omega| c^2 (Sections 1, 2.2)."""
    g, prm, phi0 = _c1_like(n=16, seed=5, mean=0.0)
    c = 0.17
    a = O.run(g, prm, phi0, 0.02, 8)
    b = O.run(g, prm, phi0 + c, 0.02, 8)
    assert np.max(np.abs((b["phi"] - c) - a["phi"])) <= 1e-12
    for ra, rb in zip(a["records"], b["records"]):
        assert abs(ra["r"] - rb["r"]) <= 1e-12 * ra["r"]
        m0 = np.mean(phi0)
        shift = 0.5 * prm.a * g.volume * ((m0 + c) ** 2 - m0 ** 2)
        assert abs(rb["energy"] - ra["energy"] - shift) <= 1e-11 * ra["energy"]


def test_symmetries():
    """Shift, transpose and reflection equivariance of the scheme; an x-only field stays x-only."""
    g, prm, phi0 = _c1_like(n=16, seed=6)
    run = lambda p: O.run(g, prm, p, 0.02, 6, energies=False)["phi"]
    base = run(phi0)
    assert np.max(np.abs(run(np.roll(phi0, (3, -5), axis=(0, 1))) - np.roll(base, (3, -5), axis=(0, 1)))) < 1e-12
    assert np.max(np.abs(run(phi0.T.copy()) - base.T)) < 1e-12
    refl = lambda p: np.roll(p[:, ::-1], 1, axis=1)          # x_j -> x_{-j}
    assert np.max(np.abs(run(refl(phi0)) - refl(base))) < 1e-12
    xonly = np.tile(phi0[0:1, :], (16, 1))
    out = run(xonly)
    assert np.max(np.abs(out - out[0:1, :])) < 1e-14


@pytest.mark.parametrize("m", [1, 3, 5])
def test_linear_regime_recurrence(m):
    """phi0 = b0 + delta cos(kx), delta = 1e-6: xi = 1 + O(delta^2) and the cubic flux is O(delta^3),
    so the amplitude follows a0 A+ + dt k^2 (a + k^4) A+ = a1 A + a2 A- + 2 dt k^4 Ahat
    (eq. scheme-SAV-1 restricted to one mode)."""
    n, L = 32, 8 * np.pi
    g = O.Grid((n, n), (L, L))
    prm = O.Params(0.25)
    k = 2 * np.pi * m / L
    x = np.arange(n) * g.h[0]
    d0 = 1e-6
    phi0 = -0.2 + d0 * np.cos(k * x)[None, :] * np.ones((n, 1))
    dt, steps = 0.05, 20
    out = O.run(g, prm, phi0, dt, steps, energies=False, keep=set(range(steps + 1)))
    amp = lambda p: 2.0 * np.mean((p[0] + 0.2) * np.cos(k * x))
    A_prev, A_cur = d0, d0
    for nstep in range(steps):
        if nstep == 0:
            a0, a1, a2, Ahat = 1.0, 1.0, 0.0, A_cur
        else:
            a0, a1, a2, Ahat = 1.5, 2.0, -0.5, 2 * A_cur - A_prev
        A_new = (a1 * A_cur + a2 * A_prev + 2 * dt * k ** 4 * Ahat) / (a0 + dt * k * k * (prm.a + k ** 4))
        A_prev, A_cur = A_cur, A_new
        got = amp(out["kept"][nstep + 1])
        assert abs(got - A_cur) <= 1e-9 * abs(A_cur)


# ----------------------------------------------------------------- P14: second order in time (Section 5.1)

OMEGA = 2 * np.pi


def exact_phi(x, y, t):
    """Manufactured solution of Section 5.1 (eq. eqn:init1)."""
    return np.sin(OMEGA * x) * np.cos(OMEGA * y) * np.cos(t) / OMEGA


def forcing_closed_form(x, y, t, a):
    """f = d_t phi_e - Delta mu(phi_e) for eq. equation-SPFC, worked out by hand:
    [-sin t / w + 2 w (a - 4 w^2 + 4 w^4) cos t] s1c1
      + w^3 cos^3 t [5/2 s1c1 + 27/2 s3c3 + 5/2 s3c1 - 5/2 s1c3],  s_p c_q = sin(p w x) cos(q w y)."""
    w = OMEGA
    sc = lambda p, q: np.sin(p * w * x) * np.cos(q * w * y)
    return ((-np.sin(t) / w + 2 * w * (a - 4 * w ** 2 + 4 * w ** 4) * np.cos(t)) * sc(1, 1)
            + w ** 3 * np.cos(t) ** 3 * (2.5 * sc(1, 1) + 13.5 * sc(3, 3) + 2.5 * sc(3, 1) - 2.5 * sc(1, 3)))


def test_forcing_closed_form_is_the_pde_residual():
    """The hand-derived forcing equals d_t phi - Delta mu computed symbolically (sympy)."""
    x, y, t, a = sp.symbols("x y t a")
    w = 2 * sp.pi
    phi = sp.sin(w * x) * sp.cos(w * y) * sp.cos(t) / w
    gx, gy = sp.diff(phi, x), sp.diff(phi, y)
    s = gx ** 2 + gy ** 2
    lapl = lambda e: sp.diff(e, x, 2) + sp.diff(e, y, 2)
    mu = -(sp.diff(s * gx, x) + sp.diff(s * gy, y)) + a * phi + 2 * lapl(phi) + lapl(lapl(phi))
    f = sp.lambdify((x, y, t, a), sp.diff(phi, t) - lapl(mu), "numpy")
    pts = np.random.default_rng(3).random((50, 3))
    for (px, py, pt) in pts:
        ref = f(px, py, pt, 0.975)
        assert abs(forcing_closed_form(px, py, pt, 0.975) - ref) <= 1e-9 * (abs(ref) + 1)


def _mms_errors(NT, n=32):
    g = O.Grid((n, n), (1.0, 1.0))
    prm = O.Params(1 - 0.975)
    xs = np.arange(n) / n
    X, Y = np.meshgrid(xs, xs)            # [y, x]
    dt = 1.0 / NT
    phi0 = exact_phi(X, Y, 0.0)
    phim1 = exact_phi(X, Y, -dt)
    out = O.run(g, prm, phi0, dt, NT, startup="copy", phim1=phim1,
                forcing=lambda t: forcing_closed_form(X, Y, t, prm.a), energies=False)
    err = out["phi"] - exact_phi(X, Y, 1.0)
    return math.sqrt(g.cell * np.sum(err * err)), np.max(np.abs(err))


def test_second_order_temporal_convergence():
    """Section 5.1 / Theorem 4.1: errors fall like dt^2 in discrete l2 and l-infinity
    (fitted log-log slope within [1.9, 2.1]).  n = 32 resolves the manufactured
    solution and its cubic flux exactly, so the error is purely temporal."""
    NTs = [100, 200, 400, 800]
    e2, einf = zip(*[_mms_errors(NT) for NT in NTs])
    for errs in (e2, einf):
        slope = -np.polyfit(np.log(NTs), np.log(errs), 1)[0]
        assert 1.9 <= slope <= 2.1, (slope, errs)


# ----------------------------------------------------------------- quartic term (beta/4) phi^4 (standard PFC, Section 1)

def test_beta_uniform_state():
    """phi = b0 everywhere: every derivative vanishes, so N = beta b0^3, E_1 = |Omega| (beta b0^4 / 4
    + 1 + 1/c4) >= |Omega|, E_N = |Omega| (beta b0^4 / 4 + a b0^2 / 2), and the state is a fixed
    point of the scheme with r constant."""
    g = O.Grid((16, 8), (5.0, 3.0))
    b0, beta, c4 = -0.3, 0.7, 1.3
    prm = O.Params(0.25, c4=c4, beta=beta)
    phi = np.full(g.shape, b0)
    assert np.max(np.abs(O.N_nl(g, prm, phi) - beta * b0 ** 3)) <= 1e-15
    E1 = g.volume * (0.25 * beta * b0 ** 4 + 1.0 + 1.0 / c4)
    assert abs(O.E1(g, prm, phi) - E1) <= 1e-14 * E1 and E1 >= g.volume
    EN = g.volume * (0.25 * beta * b0 ** 4 + 0.5 * prm.a * b0 ** 2)
    assert abs(O.E_N(g, prm, phi) - EN) <= 1e-14 * EN
    out = O.run(g, prm, phi, 0.1, 6)
    assert np.max(np.abs(out["phi"] - b0)) < 1e-15
    for rec in out["records"]:
        assert abs(rec["r"] - math.sqrt(E1)) < 1e-12 * math.sqrt(E1)


def test_beta_single_mode_closed_form():
    """phi = b0 + A cos t (t = k x, 4m < n so phi^4 is resolved): the quartic term adds
    |Omega| beta/4 (b0^4 + 3 b0^2 A^2 + 3 A^4 / 8) to E_1 and
    beta [b0^3 + 3 b0 A^2 / 2 + (3 b0^2 A + 3 A^3 / 4) cos t + (3 b0 A^2 / 2) cos 2t + (A^3 / 4) cos 3t]
    to N (powers of cos t reduced to multiple angles)."""
    L, n, m = 8 * np.pi, 64, 3
    b0, A, beta = -0.25, 0.6, 1.7
    g = O.Grid((n, n), (L, L))
    k = 2 * np.pi * m / L
    t = (k * np.arange(n) * g.h[0])[None, :] * np.ones((n, 1))
    phi = b0 + A * np.cos(t)
    p0, pb = O.Params(0.25), O.Params(0.25, beta=beta)
    dE = g.volume * 0.25 * beta * (b0 ** 4 + 3 * b0 ** 2 * A ** 2 + 3 * A ** 4 / 8)
    assert abs((O.E1(g, pb, phi) - O.E1(g, p0, phi)) - dE) <= 1e-12 * dE
    dN = beta * (b0 ** 3 + 1.5 * b0 * A * A + (3 * b0 * b0 * A + 0.75 * A ** 3) * np.cos(t)
                 + 1.5 * b0 * A * A * np.cos(2 * t) + 0.25 * A ** 3 * np.cos(3 * t))
    assert np.max(np.abs((O.N_nl(g, pb, phi) - O.N_nl(g, p0, phi)) - dN)) <= 1e-13 * np.max(np.abs(dN))
    assert abs((O.E_N(g, pb, phi) - O.E_N(g, p0, phi)) - dE) <= 1e-12 * dE


@pytest.mark.parametrize("beta", [0.0, 0.9])
def test_N_is_the_variation_of_E1(beta):
    """N_N = delta E_1 / delta phi: d/dh E_1(phi + h q) at h = 0 equals <N_N(phi), q> on fields
    without Nyquist content (where nabla.nabla = Delta).  E_1(phi + h q) is a quartic polynomial
    in h, so the central difference carries only an h^2 term and one Richardson step makes it
    exact: a wrong weight between the terms of E_1 and of N fails."""
    g = O.Grid((16, 16), (5.0, 4.0))
    f, _, _ = _trig_poly(g, 6, np.random.default_rng(21))
    q, _, _ = _trig_poly(g, 6, np.random.default_rng(22))
    phi, q = 0.3 * f, 0.2 * q
    prm = O.Params(0.25, c4=1.4, beta=beta)
    D = lambda h: (O.E1(g, prm, phi + h * q) - O.E1(g, prm, phi - h * q)) / (2 * h)
    h = 1e-2
    dE = (4 * D(h / 2) - D(h)) / 3
    ref = O.inner(g, O.N_nl(g, prm, phi), q)
    assert abs(dE - ref) <= 1e-9 * (abs(ref) + 1e-3)


@pytest.mark.parametrize("dim", [2, 3])
def test_beta_energy_identity_exact(dim):
    """Theorem 3.1 as an identity with the quartic term in E_1 (the algebra of the proof does
    not depend on the form of E_1), from the first-order start and then BDF2."""
    if dim == 2:
        g = O.Grid((32, 32), (8 * np.pi,) * 2)
    else:
        g = O.Grid((8, 8, 8), (4 * np.pi,) * 3)
    prm = O.Params(0.25, beta=1.2)
    phi0 = noise_ic(g.shape, -0.3, 31) + 0.2 * np.cos(2 * np.pi * np.arange(g.n[0]) / g.n[0] * 2)
    dt = 0.01
    phi_n, phi_nm1, r_n, r_nm1 = O.initial_state(g, prm, dt, phi0, "sav1")
    phi1, r1, info, res, lhs = _identity_residual(g, prm, dt, phi_n, phi_nm1, r_n, r_nm1, O.BDF1, False)
    assert abs(res) <= 1e-12 and lhs <= 0
    phi_nm1, phi_n, r_nm1, r_n = phi_n, phi1, r_n, r1
    for _ in range(5):
        phi1, r1, info, res, lhs = _identity_residual(g, prm, dt, phi_n, phi_nm1, r_n, r_nm1, O.BDF2, True)
        assert abs(res) <= 1e-12 and lhs <= 0
        assert info["p1"] <= 0.0 and info["E1"] >= g.volume
        phi_nm1, phi_n, r_nm1, r_n = phi_n, phi1, r_n, r1


# ----------------------------------------------------------------- stabilized scheme (end of Section 5)

def _stab_identity_residual(g, prm, dt, phi_n, phi_nm1, r_n, r_nm1, first_order):
    """Exact energy identity of the stabilized scheme, derived from the algebra of Theorem 3.1
    with the regularization -A dt Delta_N (phi^{n+1} - phi^n) in mu (d^{n+1} = phi^{n+1} - phi^n,
    |f|^2 = <f, -Delta_N f>, E_s = E + (A dt / 4)|d|^2):
      BDF2:  E_s^{n+1} - E_s^n = -1/4 ||L^1/2 (d^{n+1} - d^n)||^2 - 1/2 (r^{n+1} - 2r^n + r^{n-1})^2
                                 - A dt |d^{n+1}|^2 - (A dt / 4) |d^{n+1} - d^n|^2 + dt <Delta mu, mu>
      first-order start from (phi^0, phi^0, r^0, r^0):
             E_s^1 - E_s^0 = 3/2 dt <Delta mu, mu> - (5/4) A dt |d^1|^2 - 1/4 ||L^1/2 d^1||^2 - 1/2 (r^1 - r^0)^2."""
    alpha = O.BDF1 if first_order else O.BDF2
    phi1, r1, info = O.sav_step(g, prm, dt, phi_n, phi_nm1, r_n, r_nm1, alpha=alpha, extrapolate=not first_order)
    mu = O.mu_of(g, prm, phi1, info["phihat"], r1, phi_old=phi_n, dt=dt)
    diss = dt * O.inner(g, O.lap(g, mu), mu)
    A = prm.stab
    d1, d0 = phi1 - phi_n, phi_n - phi_nm1
    lhs = (O.stabilized_energy(g, prm, dt, phi1, phi_n, r1, r_n)
           - O.stabilized_energy(g, prm, dt, phi_n, phi_nm1, r_n, r_nm1))
    if first_order:
        rhs = (1.5 * diss - 1.25 * A * dt * O.grad_sq_norm(g, d1) - 0.25 * O.L_half_sq(g, prm, d1)
               - 0.5 * (r1 - r_n) ** 2)
    else:
        rhs = (-0.25 * O.L_half_sq(g, prm, d1 - d0) - 0.5 * (r1 - 2 * r_n + r_nm1) ** 2
               - A * dt * O.grad_sq_norm(g, d1) - 0.25 * A * dt * O.grad_sq_norm(g, d1 - d0) + diss)
    scale = O.stabilized_energy(g, prm, dt, phi_n, phi_nm1, r_n, r_nm1)
    return phi1, r1, (lhs - rhs) / scale, lhs


@pytest.mark.parametrize("dim,A", [(2, 0.5), (2, 50.0), (3, 5.0)])
def test_stabilized_energy_identity_exact(dim, A):
    """The identity holds exactly only with the regularization in mu with this sign and with
    phi^n on the right-hand side: a flipped sign, a term on phi^{n+1} alone or a missing
    phi^n term each leave a residual of the size of the A terms."""
    if dim == 2:
        g = O.Grid((32, 32), (4 * np.pi,) * 2)
        phi0 = noise_ic(g.shape, -0.2, 4)
    else:
        g = O.Grid((8, 8, 8), (4 * np.pi,) * 3)
        phi0 = noise_ic(g.shape, -0.25, 3)
    prm = O.Params(0.25, stab=A)
    dt = 0.02
    phi_n, phi_nm1, r_n, r_nm1 = O.initial_state(g, prm, dt, phi0, "sav1")
    phi1, r1, res, lhs = _stab_identity_residual(g, prm, dt, phi_n, phi_nm1, r_n, r_nm1, True)
    assert abs(res) <= 1e-12 and lhs <= 0
    phi_nm1, phi_n, r_nm1, r_n = phi_n, phi1, r_n, r1
    for _ in range(5):
        phi1, r1, res, lhs = _stab_identity_residual(g, prm, dt, phi_n, phi_nm1, r_n, r_nm1, False)
        assert abs(res) <= 1e-12 and lhs <= 0
        phi_nm1, phi_n, r_nm1, r_n = phi_n, phi1, r_n, r1


def _stab_identity_of(g, prm, dt, phi_n, phi_nm1, r_n, r_nm1, phi1, r1, phihat):
    mu = O.mu_of(g, prm, phi1, phihat, r1, phi_old=phi_n, dt=dt)
    diss = dt * O.inner(g, O.lap(g, mu), mu)
    d1, d0 = phi1 - phi_n, phi_n - phi_nm1
    lhs = (O.stabilized_energy(g, prm, dt, phi1, phi_n, r1, r_n)
           - O.stabilized_energy(g, prm, dt, phi_n, phi_nm1, r_n, r_nm1))
    rhs = (-0.25 * O.L_half_sq(g, prm, d1 - d0) - 0.5 * (r1 - 2 * r_n + r_nm1) ** 2
           - prm.stab * dt * O.grad_sq_norm(g, d1) - 0.25 * prm.stab * dt * O.grad_sq_norm(g, d1 - d0) + diss)
    return (lhs - rhs) / O.stabilized_energy(g, prm, dt, phi_n, phi_nm1, r_n, r_nm1)


def test_stabilized_identity_catches_planted_mistakes():
    """Plant two plausible mistakes in the stabilized step (on the CPU, in the oracle): the
    regularization with the opposite sign, and the regularization acting on phi^{n+1} alone
    (its phi^n part of the right-hand side cancelled through the forcing slot).  The identity
    residual is at rounding level for the correct step and far above it for both plants."""
    g = O.Grid((16, 16), (4 * np.pi,) * 2)
    prm = O.Params(0.25, stab=20.0)
    dt = 0.02
    st = O.run(g, prm, noise_ic(g.shape, -0.2, 6), dt, 3, energies=False)
    state = (st["phi"], st["phi_prev"], st["r"], st["r_prev"])
    good = O.sav_step(g, prm, dt, *state)
    assert abs(_stab_identity_of(g, prm, dt, *state, good[0], good[1], good[2]["phihat"])) <= 1e-12
    flipped = O.sav_step(g, O.Params(0.25, stab=-20.0), dt, *state)
    cancel = -prm.stab * dt * O.lap(g, O.lap(g, state[0]))
    no_old = O.sav_step(g, prm, dt, *state, forcing=cancel)
    for phi1, r1, info in (flipped, no_old):
        assert abs(_stab_identity_of(g, prm, dt, *state, phi1, r1, info["phihat"])) > 1e-8


def _singular_ic(n=64, seed=5):
    g = O.Grid((n, n), (100.0, 100.0))
    phi0 = noise_ic(g.shape, 0.0, seed)
    phi0[n // 2, n // 2] += 10.0
    return g, phi0


def test_singular_initial_data_plain_vs_stabilized():
    """End of Section 5: with a nucleation of magnitude 10 at the centre of (0,100)^2 (a = 0.5,
    the Section 5.2 noise), the plain scheme gives no reasonable solution while the stabilized
    one does.  Measured reading: the plain scheme drives r through zero (xi = r/sqrt(E_1) < 0)
    within a few steps, while with A = 1e5 xi stays within 2 % of 1; both keep the mass and
    a non-increasing modified energy (Theorems 2.1 and 3.1 hold for any data)."""
    g, phi0 = _singular_ic()
    for A, check in ((0.0, lambda xs: min(xs) < 0.0), (1e5, lambda xs: all(abs(x - 1) <= 0.02 for x in xs))):
        out = O.run(g, O.Params(0.5, stab=A), phi0, 0.01, 30)
        recs = out["records"]
        xs = [r["xi"] for r in recs[1:]]
        assert check(xs), (A, min(xs), max(xs))
        for a, b in zip(recs, recs[1:]):
            assert b["energy"] <= a["energy"] * (1 + 1e-13)
        assert abs(recs[-1]["mean"] - np.mean(phi0)) <= 1e-13


# ----------------------------------------------------------------- P5: one full step from a single mode

def test_one_step_from_a_single_mode_closed_form():
    """phi^n = phi^{n-1} = A cos(kappa x) (3m < N/2, so nothing aliases): N = n1 cos + n3 cos 3
    (the P4 closed form), the solves act mode by mode, and every scalar of the step is a
    closed expression in A, kappa, dt, a (derived by hand from eq. scheme-SAV-1:
    A_k phi^{n+1} = psi + dt xi Delta N, a0 r^{n+1} - rho = <N, a0 phi^{n+1} - psi>/(2S)):
    b1 = -k^2 n_k / A_k, b2 = 1.5 A / A_kappa on cos theta; p1, p2, p_psi are |Omega|/2 sums
    of the mode products; xi = [rho + (a0 p2 - p_psi)/(2S)] / [a0 (S - dt p1/(2S))]."""
    n, L, m, A, dt = 64, 8 * math.pi, 4, 0.3, 0.01
    g = O.Grid((n, n), (L, L))
    prm = O.Params(0.25)
    kap = 2 * math.pi * m / L
    X = np.tile(np.arange(n) * L / n, (n, 1))
    phi = A * np.cos(kap * X)
    S = math.sqrt(O.E1(g, prm, phi))
    new, r_new, info = O.sav_step(g, prm, dt, phi, phi, S, S)
    Om, a = L * L, prm.a
    n1, n3 = 0.75 * A ** 3 * kap ** 4 - 2 * kap ** 2 * A, -0.75 * A ** 3 * kap ** 4
    Ak = 1.5 + dt * kap ** 2 * (a + kap ** 4)
    A3 = 1.5 + dt * 9 * kap ** 2 * (a + 81 * kap ** 4)
    p1 = Om / 2 * (-kap ** 2 * n1 ** 2 / Ak - 9 * kap ** 2 * n3 ** 2 / A3)
    p2 = Om / 2 * n1 * 1.5 * A / Ak
    ppsi = Om / 2 * n1 * 1.5 * A
    xi = (1.5 * S + (1.5 * p2 - ppsi) / (2 * S)) / (1.5 * (S - dt * p1 / (2 * S)))
    ref = (dt * xi * (-kap ** 2 * n1 / Ak) + 1.5 * A / Ak) * np.cos(kap * X) \
        + dt * xi * (-9 * kap ** 2 * n3 / A3) * np.cos(3 * kap * X)
    assert np.max(np.abs(new - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert abs(info["p1"] - p1) <= 1e-13 * abs(p1)
    assert abs(info["xi"] - xi) <= 1e-13
    assert abs(r_new - xi * S) <= 1e-13 * S


# ----------------------------------------------------------------- P15: self-convergence, r-consistency

def _smooth(g, seed, amp=0.05, mmax=3):
    rng = np.random.default_rng(seed)
    xs = [np.arange(nj) * hj for nj, hj in zip(g.n, g.h)]
    X, Y = np.meshgrid(xs[0], xs[1])
    phi = np.full(g.shape, -0.2)
    for _ in range(6):
        th = 2 * np.pi * (int(rng.integers(-mmax, mmax + 1)) * X / g.L[0] + int(rng.integers(-mmax, mmax + 1)) * Y / g.L[1])
        phi += amp * rng.uniform(-1, 1) * np.cos(th + rng.uniform(0, 2 * np.pi))
    return phi


@pytest.mark.parametrize("startup,order", [("sav1", 2), ("ghost", 2), ("copy", 1)])
def test_self_convergence_and_r_consistency(startup, order):
    """The 64^2 setup (L = 8 pi, epsilon = 0.25) to T = 1 with dt = 0.02, 0.01, 0.005, 0.0025
    from smooth data (white noise is not in the asymptotic regime at these dt):
    ||phi_dt - phi_dt/2|| / ||phi_dt/2 - phi_dt/4|| ~ 2^order, with order 2 for the
    first-order SAV and the ghost start (Theorem 4.1) and 1 for the copy start (phi^{-1} =
    phi^0 is an O(dt) change of the history: the restart rule of Section 5.2 costs one
    order).  |r - sqrt(E_1(phi))| at T falls at least 3.6x per halving (second order or
    better)."""
    g = O.Grid((64, 64), (8 * math.pi,) * 2)
    prm = O.Params(0.25)
    phi0 = _smooth(g, 7)
    dts = [0.02, 0.01, 0.005, 0.0025]
    phis, gaps = [], []
    for dt in dts:
        out = O.run(g, prm, phi0, dt, int(round(1.0 / dt)), startup=startup, energies=False)
        phis.append(out["phi"])
        gaps.append(abs(out["r"] - math.sqrt(O.E1(g, prm, out["phi"]))))
    lo, hi = (3.6, 4.4) if order == 2 else (1.8, 2.4)
    for i in range(2):
        ratio = np.linalg.norm(phis[i] - phis[i + 1]) / np.linalg.norm(phis[i + 1] - phis[i + 2])
        assert lo <= ratio <= hi, (startup, ratio)
    for i in range(3):
        assert gaps[i] / gaps[i + 1] >= 3.6, (startup, gaps)
