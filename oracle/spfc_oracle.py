"""Plain FP64 CPU oracle for the SAV-BDF2 scheme for the square phase field crystal equation.

TEST INFRASTRUCTURE.  This module exists to check the GPU path; it is not part of
it.  Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import it.  It shares no code with the HIP path: its FFT, its operators,
its energies and its time step are written out here, slowly and literally.

Source: M. Wang, Q. Huang, C. Wang, "A second order accurate scalar auxiliary
variable (SAV) numerical method for the square phase field crystal equation"
(arXiv 2012.15133).  Each function names the passage it follows.

Conventions (readings where the paper is silent or written for odd N only):

* Grid functions are arrays indexed [y, x] (2-D) or [z, y, x] (3-D), x
  fastest.  Spatial axis j = 0, 1, 2 is x, y, z; it is array axis dim-1-j.
  Point j along an axis of n points and length L sits at j*h, h = L/n
  (Section 2.1, generalised from the unit box).
* Inner product <f, g> = (prod_j h_j) * sum f g  (Section 2.1, eq.
  spectral-coll-inner product-1).  Mean = sum f / prod n.
* DFT: F(m) = sum_j f_j exp(-2 pi i m.j / n), inverse divides by prod n.  This is
  the paper's normalised expansion (Section 2.1) up to the constant factor.
* Signed wavenumber index mt = m for m < n/2, m - n for m >= n/2.
  Odd-order (first-derivative) symbol kappa1 = 2 pi mt / L with the Nyquist
  entry m = n/2 set to 0, so that derivatives of real data stay real.
  Even-order symbol kappa2^2 = (2 pi mt / L)^2 keeps the Nyquist entry,
  (pi n / L)^2.  |k|^2 = sum_j kappa2^2 along each axis.  (The paper assumes
  odd n, where neither rule is needed; its experiments use even n.)
* D_j f = F^-1[i kappa1_j F f] (eqs. spectral-coll-2-1/-2-3), Delta_N f =
  F^-1[-|k|^2 F f] (eq. spectral-coll-3), L_N f = F^-1[(a + |k|^4) F f]
  (Section 2.1, eigenvalue a + lambda^2 of L_N, eq. spectral-coll-6).
* The 4-Laplacian energy coefficient c4 multiplies (1/4)|grad phi|^4 (the paper
  has c4 = 1, eq. energy-SPFC).  The constant of E_1 is (1 + 1/c4)|Omega| so
  that E_1 >= |Omega| still holds; at c4 = 1 it is the paper's 2|Omega|
  (Section 2.2, eqs. energy-SPFC-split-1/-2-2).
* |grad phi|^4 is the Euclidean (sum_j (D_j phi)^2)^2, matching the flux
  |grad phi|^2 grad phi of the chemical potential (eq. equation-SPFC).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "fft_axis", "fftn", "ifftn", "Grid", "Params",
    "grad", "div", "lap", "L_op", "inner", "E1", "N_nl", "E_N",
    "L_half_sq", "modified_energy", "sav_energy", "mu_of",
    "sav_step", "initial_state", "run",
]


# ----------------------------------------------------------------- FFT (own code)

def _bit_reverse(n: int) -> np.ndarray:
    bits = n.bit_length() - 1
    idx = np.arange(n)
    rev = np.zeros(n, dtype=np.int64)
    for b in range(bits):
        rev |= ((idx >> b) & 1) << (bits - 1 - b)
    return rev


def fft_axis(x: np.ndarray, axis: int, sign: int) -> np.ndarray:
    """Unnormalised DFT along one axis: X(m) = sum_j x_j exp(sign 2 pi i m j / n).

    Iterative radix-2 decimation in time: permute to bit-reversed order, then
    merge pairs of half-length transforms E, O into X[k] = E[k] + w^k O[k],
    X[k + m] = E[k] - w^k O[k] with w = exp(sign pi i / m).  n must be a power
    of two.  No scaling in either direction.
    """
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    n = x.shape[-1]
    if n & (n - 1):
        raise ValueError("fft_axis: length must be a power of two")
    batch = x.shape[:-1]
    y = x[..., _bit_reverse(n)]
    m = 1
    while m < n:
        w = np.exp(sign * 1j * np.pi * np.arange(m) / m)
        y = y.reshape(batch + (n // (2 * m), 2, m))
        even = y[..., 0, :]
        odd = y[..., 1, :] * w
        y = np.stack((even + odd, even - odd), axis=-2)
        m *= 2
    y = y.reshape(batch + (n,))
    return np.moveaxis(y, -1, axis)


def fftn(f: np.ndarray) -> np.ndarray:
    """Forward DFT over every axis (sign -1, unnormalised)."""
    F = np.asarray(f, dtype=np.complex128)
    for ax in range(F.ndim):
        F = fft_axis(F, ax, -1)
    return F


def ifftn(F: np.ndarray) -> np.ndarray:
    """Inverse DFT over every axis (sign +1), divided by the number of points."""
    f = np.asarray(F, dtype=np.complex128)
    for ax in range(f.ndim):
        f = fft_axis(f, ax, +1)
    return f / f.size


# ----------------------------------------------------------------- grid and symbols

class Grid:
    """Periodic grid Omega_N (Section 2.1), sides L_j, n_j points per axis.

    `n` and `L` are given in spatial order (x, y[, z]).
    """

    def __init__(self, n, L):
        self.n = tuple(int(v) for v in n)
        self.L = tuple(float(v) for v in L)
        if len(self.n) not in (2, 3) or len(self.L) != len(self.n):
            raise ValueError("Grid: dimension must be 2 or 3")
        self.dim = len(self.n)
        self.h = tuple(Lj / nj for Lj, nj in zip(self.L, self.n))
        self.cell = float(np.prod(self.h))          # h^d
        self.volume = float(np.prod(self.L))        # |Omega|
        self.shape = tuple(reversed(self.n))        # array shape, x last
        self.npts = int(np.prod(self.n))

    def _along(self, j: int, v: np.ndarray) -> np.ndarray:
        shp = [1] * self.dim
        shp[self.dim - 1 - j] = self.n[j]
        return v.reshape(shp)

    def _signed(self, j: int) -> np.ndarray:
        nj = self.n[j]
        m = np.arange(nj)
        return np.where(m < nj // 2, m, m - nj).astype(np.float64)

    def kappa1(self, j: int) -> np.ndarray:
        """Odd-order symbol along spatial axis j, Nyquist entry zero."""
        k = 2.0 * np.pi * self._signed(j) / self.L[j]
        if self.n[j] % 2 == 0:
            k[self.n[j] // 2] = 0.0
        return self._along(j, k)

    def kappa2sq(self, j: int) -> np.ndarray:
        """Even-order symbol along spatial axis j (Nyquist kept)."""
        k = 2.0 * np.pi * self._signed(j) / self.L[j]
        return self._along(j, k * k)

    def ksq(self) -> np.ndarray:
        """|k|^2 = sum_j kappa2_j^2, i.e. minus the symbol of Delta_N."""
        out = np.zeros(self.shape)
        for j in range(self.dim):
            out = out + self.kappa2sq(j)
        return out


@dataclass(frozen=True)
class Params:
    """Model parameters: a = 1 - epsilon > 0 (Section 1), c4 > 0 (paper: 1).

    stab = A >= 0 selects the stabilized scheme of the closing remarks of Section 5:
    the regularization -A dt Delta_N (phi^{n+1} - phi^n) is added to the chemical
    potential of the step (A = 0: the scheme eq. scheme-SAV-1 itself).

    beta >= 0 adds (beta/4) phi^4 to the energy density, the quartic term of the
    standard PFC energy (Section 1, eq. energy-PFC), beside the 4-Laplacian term of
    the SPFC energy (paper: 0).  It is convex and nonnegative, so it joins the
    nonlinear part E_1 (which keeps E_1 >= |Omega|) and adds beta phi^3 to N."""
    epsilon: float
    c4: float = 1.0
    stab: float = 0.0
    beta: float = 0.0

    @property
    def a(self) -> float:
        return 1.0 - self.epsilon

    def e1_constant(self, volume: float) -> float:
        return (1.0 + 1.0 / self.c4) * volume


# ----------------------------------------------------------------- operators (Section 2.1)

def grad(g: Grid, f: np.ndarray):
    """nabla_N f = (D_x f, D_y f[, D_z f])  (eqs. spectral-coll-2-1, spectral-coll-3)."""
    F = fftn(f)
    return [ifftn(1j * g.kappa1(j) * F).real for j in range(g.dim)]


def div(g: Grid, v) -> np.ndarray:
    """nabla_N . v = sum_j D_j v_j  (eq. spectral-coll-3)."""
    out = np.zeros(g.shape)
    for j in range(g.dim):
        out = out + ifftn(1j * g.kappa1(j) * fftn(v[j])).real
    return out


def lap(g: Grid, f: np.ndarray) -> np.ndarray:
    """Delta_N f = sum_j D_j^2 f  (eqs. spectral-coll-2-3, spectral-coll-3)."""
    return ifftn(-g.ksq() * fftn(f)).real


def L_op(g: Grid, prm: Params, f: np.ndarray) -> np.ndarray:
    """L_N f = (a I + Delta_N^2) f, eigenvalue a + |k|^4  (Section 2.1, eq. spectral-coll-6)."""
    k2 = g.ksq()
    return ifftn((prm.a + k2 * k2) * fftn(f)).real


def inner(g: Grid, f: np.ndarray, q: np.ndarray) -> float:
    """<f, q> = h^d sum f q  (eq. spectral-coll-inner product-1)."""
    return g.cell * float(np.sum(f * q))


# ----------------------------------------------------------------- energies (Sections 2.1-2.2, 3.1)

def _grad_sq(g: Grid, phi: np.ndarray):
    gr = grad(g, phi)
    s = np.zeros(g.shape)
    for d in gr:
        s = s + d * d
    return gr, s


def E1(g: Grid, prm: Params, phi: np.ndarray) -> float:
    """E_{1,N}(phi) = (c4/4)||nabla_N phi||_4^4 - ||nabla_N phi||_2^2 + (beta/4)||phi||_4^4
    + (1 + 1/c4)|Omega|.

    Section 2.2 (definition after eq. scheme-SAV-1); c4 = 1, beta = 0 gives the paper's form.
    """
    _, s = _grad_sq(g, phi)
    dens = 0.25 * prm.c4 * s * s - s
    if prm.beta != 0.0:
        dens = dens + 0.25 * prm.beta * phi ** 4
    return g.cell * float(np.sum(dens)) + prm.e1_constant(g.volume)


def N_nl(g: Grid, prm: Params, phi: np.ndarray) -> np.ndarray:
    """N_N(phi) = -c4 nabla_N.(|nabla_N phi|^2 nabla_N phi) + 2 Delta_N phi + beta phi^3
    (Section 2.2, after eq. scheme-SAV-1; the variational derivative of E_1)."""
    gr, s = _grad_sq(g, phi)
    out = -prm.c4 * div(g, [s * d for d in gr]) + 2.0 * lap(g, phi)
    if prm.beta != 0.0:
        out = out + prm.beta * phi ** 3
    return out


def E_N(g: Grid, prm: Params, phi: np.ndarray) -> float:
    """Discrete SPFC energy (eq. energy-discrete-spectral):
    (c4/4)||nabla phi||_4^4 + a/2 ||phi||^2 - ||nabla phi||^2 + 1/2 ||Delta_N phi||^2
    (+ (beta/4)||phi||_4^4)."""
    _, s = _grad_sq(g, phi)
    lp = lap(g, phi)
    quartic = 0.25 * prm.beta * float(np.sum(phi ** 4)) if prm.beta != 0.0 else 0.0
    return (g.cell * (float(np.sum(0.25 * prm.c4 * s * s - s)) + quartic)
            + 0.5 * prm.a * inner(g, phi, phi) + 0.5 * inner(g, lp, lp))


def L_half_sq(g: Grid, prm: Params, f: np.ndarray) -> float:
    """||L_N^{1/2} f||^2 = <f, L_N f>  (eq. spectral-coll-inner product-4)."""
    return inner(g, f, L_op(g, prm, f))


def modified_energy(g: Grid, prm: Params, phi1, phi0, r1: float, r0: float) -> float:
    """Modified energy of Theorem 3.1 (eq. discrete energy):
    1/4 (||L^{1/2} phi1||^2 + ||L^{1/2}(2 phi1 - phi0)||^2) + 1/2 (r1^2 + (2 r1 - r0)^2)."""
    return (0.25 * (L_half_sq(g, prm, phi1) + L_half_sq(g, prm, 2.0 * phi1 - phi0))
            + 0.5 * (r1 * r1 + (2.0 * r1 - r0) ** 2))


def grad_sq_norm(g: Grid, f: np.ndarray) -> float:
    """<f, -Delta_N f>: the squared gradient norm with the even-order symbol of Delta_N."""
    return -inner(g, f, lap(g, f))


def stabilized_energy(g: Grid, prm: Params, dt: float, phi1, phi0, r1: float, r0: float) -> float:
    """Modified energy of the stabilized scheme: the energy of Theorem 3.1 plus
    (A dt / 4) <phi1 - phi0, -Delta_N (phi1 - phi0)>.  Derived here from the algebra of
    Theorem 3.1 with the regularization term in mu; it equals modified_energy at A = 0."""
    d = phi1 - phi0
    return modified_energy(g, prm, phi1, phi0, r1, r0) + 0.25 * prm.stab * dt * grad_sq_norm(g, d)


def sav_energy(g: Grid, prm: Params, phi: np.ndarray, r: float) -> float:
    """SAV energy plotted against E_N in Section 5.2: a/2 ||phi||^2 + 1/2 ||Delta_N phi||^2 + r^2."""
    lp = lap(g, phi)
    return 0.5 * prm.a * inner(g, phi, phi) + 0.5 * inner(g, lp, lp) + r * r


def mu_of(g: Grid, prm: Params, phi_new, phihat, r_new: float, phi_old=None, dt: float = 0.0) -> np.ndarray:
    """Chemical potential of the step, mu = L_N phi^{n+1} + r^{n+1}/sqrt(E_1(phihat)) N_N(phihat)
    (Section 3.1, eq. eng stab-1, second line), plus -A dt Delta_N (phi^{n+1} - phi^n) for the
    stabilized scheme (phi_old = phi^n)."""
    mu = L_op(g, prm, phi_new) + (r_new / math.sqrt(E1(g, prm, phihat))) * N_nl(g, prm, phihat)
    if prm.stab != 0.0:
        mu = mu - prm.stab * dt * lap(g, phi_new - phi_old)
    return mu


# ----------------------------------------------------------------- one time step (Section 2.3)

BDF2 = (1.5, 2.0, -0.5)   # (3/2 phi^{n+1} - 2 phi^n + 1/2 phi^{n-1}) / dt   (eq. scheme-SAV-1)
BDF1 = (1.0, 1.0, 0.0)    # (phi^{n+1} - phi^n) / dt: first-order start step (not in the paper)


def sav_step(g: Grid, prm: Params, dt: float, phi_n, phi_nm1, r_n: float, r_nm1: float,
             alpha=BDF2, extrapolate: bool = True, forcing=None):
    """One step of the SAV scheme, solved the way Section 2.3 solves it.

    The scheme (eq. scheme-SAV-1) with time-derivative weights
    alpha = (a0, a1, a2), i.e. (a0 phi^{n+1} - a1 phi^n - a2 phi^{n-1}) / dt,
    and the same weights for r.  BDF2 is alpha = (3/2, 2, -1/2) with the
    extrapolation phihat = 2 phi^n - phi^{n-1}; the first-order start step
    uses alpha = (1, 1, 0) and phihat = phi^n.  `forcing`, if given, is a grid
    function f^{n+1} added to the phi equation only.

    Steps (eqs. solver-1 ... solver-6, written for general alpha):
      1. E = E_{1,N}(phihat), N = N_N(phihat).
      2. A_N = a0 I - dt Delta_N L_N; v = A_N^{-1} Delta_N N.
      3. g = dt Delta_N N (rho/a0 - <N, psi>/(2 a0 sqrt E)) / sqrt E + psi + dt f,
         psi = a1 phi^n + a2 phi^{n-1}, rho = a1 r^n + a2 r^{n-1}
         (for BDF2 this is the right-hand side g_N^n printed before eq. solver-3).
    Stabilized scheme (prm.stab = A > 0): mu gains -A dt Delta_N (phi^{n+1} - phi^n), so
    dt Delta_N mu gains -A dt^2 Delta_N^2 (phi^{n+1} - phi^n): A_N gains + A dt^2 Delta_N^2 and
    the right-hand side of step 3 gains + A dt^2 Delta_N^2 phi^n.  The r equation (eq.
    solver-2) keeps a0 phi^{n+1} - psi, so steps 3 (the constant c) and 6 use psi itself.
      4. LHS = <N, phi^{n+1}> from eq. solver-4:
         (1 - dt/(2E) <N, v>) LHS = <N, A_N^{-1} g>.
      5. phi^{n+1} = dt/(2E) LHS v + A_N^{-1} g   (eq. solver-6).
      6. r^{n+1} = (rho + <N, a0 phi^{n+1} - psi>/(2 sqrt E)) / a0   (eq. solver-2).
    Returns (phi_new, r_new, info) with diagnostics in `info`.
    """
    a0, a1, a2 = alpha
    phihat = 2.0 * phi_n - phi_nm1 if extrapolate else phi_n
    psi = a1 * phi_n + a2 * phi_nm1
    rho = a1 * r_n + a2 * r_nm1

    E = E1(g, prm, phihat)
    sqE = math.sqrt(E)
    Nh = N_nl(g, prm, phihat)

    k2 = g.ksq()
    A = a0 + dt * k2 * (prm.a + k2 * k2)          # symbol of A_N = a0 I - dt Delta_N L_N
    if prm.stab != 0.0:
        A = A + prm.stab * dt * dt * k2 * k2      # + A dt^2 Delta_N^2

    def A_inv(f):
        return ifftn(fftn(f) / A).real

    lapN = lap(g, Nh)
    v = A_inv(lapN)
    rhs = psi if forcing is None else psi + dt * forcing
    if prm.stab != 0.0:
        rhs = rhs + prm.stab * dt * dt * lap(g, lap(g, phi_n))
    c = rho / a0 - inner(g, Nh, psi) / (2.0 * a0 * sqE)
    gN = dt * lapN * (c / sqE) + rhs
    Ag = A_inv(gN)
    p1 = inner(g, Nh, v)
    coef = 1.0 - dt / (2.0 * E) * p1
    LHS = inner(g, Nh, Ag) / coef
    phi_new = dt / (2.0 * E) * LHS * v + Ag
    r_new = (rho + inner(g, Nh, a0 * phi_new - psi) / (2.0 * sqE)) / a0
    info = {"E1": E, "p1": p1, "coef": coef, "LHS": LHS,
            "xi": r_new / sqE, "phihat": phihat, "N": Nh}
    return phi_new, r_new, info


# ----------------------------------------------------------------- start-up and runs

STARTUPS = ("sav1", "ghost", "copy")


def initial_state(g: Grid, prm: Params, dt: float, phi0, startup: str = "sav1", forcing0=None):
    """Two-level initial data (phi^0, phi^{-1}, r^0, r^{-1}).

    * "ghost": phi^{-1} = phi^0 - dt Delta_N mu^0, mu^0 = N_N(phi^0) + L_N phi^0,
      r^0 = sqrt(E_1(phi^0)), r^{-1} = sqrt(E_1(phi^{-1}))  (eq. scheme-SAV-initial-1
      and the sentence after it).  With a forcing f^0, dt f^0 is subtracted as well.
    * "copy": phi^{-1} = phi^0 and r^{-1} = r^0, the restart rule of Section 5.2.
    * "sav1": the same pair as "copy"; the first step is then the first-order
      SAV step (BDF1 weights, phihat = phi^0) instead of BDF2.
    """
    phi0 = np.asarray(phi0, dtype=np.float64)
    r0 = math.sqrt(E1(g, prm, phi0))
    if startup == "ghost":
        mu0 = N_nl(g, prm, phi0) + L_op(g, prm, phi0)
        phim1 = phi0 - dt * lap(g, mu0)
        if forcing0 is not None:
            phim1 = phim1 - dt * forcing0
        rm1 = math.sqrt(E1(g, prm, phim1))
    elif startup in ("copy", "sav1"):
        phim1 = phi0.copy()
        rm1 = r0
    else:
        raise ValueError(f"unknown startup {startup!r}")
    return phi0.copy(), phim1, r0, rm1


def run(g: Grid, prm: Params, phi0, dt: float, nsteps: int, startup: str = "sav1",
        forcing=None, t0: float = 0.0, phim1=None, energies: bool = True, keep=None):
    """Advance `nsteps` steps from phi0 and record per-step diagnostics.

    records[n] (n = 0..nsteps) holds the modified energy E_n = E(phi^n, phi^{n-1},
    r^n, r^{n-1}) (eq. discrete energy; for n = 0 the start-up pair; for the stabilized
    scheme the energy of `stabilized_energy`), the mean
    of phi^n, r^n, and for n >= 1 xi = r^n / sqrt(E_1(phihat)), E_1(phihat) and
    p1 = <N, A_N^{-1} Delta_N N> of the step that produced phi^n.
    `forcing(t)` returns f at time t; it is evaluated at t^{n+1}.
    `phim1`, if given, replaces the start-up phi^{-1} (with r^{-1} = sqrt(E_1)).
    `keep` is an optional set of step indices whose phi^n is returned.
    """
    f0 = forcing(t0) if (forcing is not None and startup == "ghost") else None
    phi_n, phi_nm1, r_n, r_nm1 = initial_state(g, prm, dt, phi0, startup, f0)
    if phim1 is not None:
        phi_nm1 = np.asarray(phim1, dtype=np.float64).copy()
        r_nm1 = math.sqrt(E1(g, prm, phi_nm1))
    records = []

    def record(info=None):
        rec = {"mean": float(np.mean(phi_n)), "r": r_n}
        if energies:
            rec["energy"] = stabilized_energy(g, prm, dt, phi_n, phi_nm1, r_n, r_nm1)
        if info is not None:
            rec.update({"xi": info["xi"], "E1": info["E1"], "p1": info["p1"]})
        records.append(rec)

    record()
    kept = {}
    if keep is not None and 0 in keep:
        kept[0] = phi_n.copy()
    for n in range(nsteps):
        first_order = (n == 0 and startup == "sav1")
        alpha = BDF1 if first_order else BDF2
        fn = forcing(t0 + (n + 1) * dt) if forcing is not None else None
        phi_new, r_new, info = sav_step(g, prm, dt, phi_n, phi_nm1, r_n, r_nm1,
                                        alpha=alpha, extrapolate=not first_order,
                                        forcing=fn)
        phi_nm1, phi_n = phi_n, phi_new
        r_nm1, r_n = r_n, r_new
        record(info)
        if keep is not None and (n + 1) in keep:
            kept[n + 1] = phi_n.copy()
    return {"phi": phi_n, "phi_prev": phi_nm1, "r": r_n, "r_prev": r_nm1,
            "records": records, "kept": kept}
