"""Pins of the surrogate's CPU oracle (oracle/fno_oracle.py) against library routines,
closed forms, invariants and finite differences."""

import math

import numpy as np
import pytest
import torch

from oracle import fno_oracle as F

S = F.FnoShape(n=16, width=4, layers=2, mx=3, my=3, hidden=5)


def test_bf16_rounding_matches_torch():
    x = torch.from_numpy(np.random.default_rng(0).standard_normal(4096) * 10.0 ** np.random.default_rng(1)
                         .integers(-8, 8, 4096))
    ref = x.to(torch.float32).to(torch.bfloat16).to(torch.float64)
    assert torch.equal(F.round_bf16(x), ref)


def test_analysis_matches_numpy_rfft2():
    s = F.FnoShape(n=32, width=1, layers=1, mx=5, my=4)
    v = np.random.default_rng(2).standard_normal((3, 32, 32))
    got = F.analysis(s, torch.from_numpy(v)).numpy()
    R = np.fft.rfft2(v) / (32 * 32)                  # [b, ky, kx]
    kx, ky = F.mode_indices(s)
    assert np.max(np.abs(got - R[:, ky, kx])) <= 1e-15 * 32


def test_synthesis_matches_numpy_irfft2():
    """synth(U) = N^2 irfft2 of the zero-filled half spectrum, for any complex U (including
    kx = 0 entries that are not Hermitian pairs: their real part is what a real inverse keeps)."""
    s = F.FnoShape(n=32, width=1, layers=1, mx=5, my=4)
    rng = np.random.default_rng(3)
    U = rng.standard_normal((2, s.modes)) + 1j * rng.standard_normal((2, s.modes))
    half = np.zeros((2, 32, 17), complex)
    kx, ky = F.mode_indices(s)
    half[:, ky, kx] = U
    ref = np.fft.irfft2(half, s=(32, 32)) * 32 * 32
    got = F.synthesis(s, torch.from_numpy(U)).numpy()
    assert np.max(np.abs(got - ref)) <= 1e-12


def test_synthesis_inverts_analysis_on_band_limited_fields():
    s = F.FnoShape(n=16, width=1, layers=1, mx=3, my=3)
    rng = np.random.default_rng(4)
    half = np.zeros((16, 9), complex)
    kx, ky = F.mode_indices(s)
    half[ky, kx] = rng.standard_normal(s.modes) + 1j * rng.standard_normal(s.modes)
    half[16 - s.my, 0] = 0.0     # (0, -MY) has no retained partner (0, +MY)
    v = np.fft.irfft2(half, s=(16, 16))                # real and band-limited
    back = F.synthesis(s, F.analysis(s, torch.from_numpy(v))).numpy()
    assert np.max(np.abs(back - v)) <= 1e-14


# Standard normal distribution function at a few points, from printed tables of Phi
# (e.g. Abramowitz and Stegun, Table 26.1): gelu(z) = z Phi(z).
PHI_TABLE = [(-3.0, 0.0013498980316301), (-1.0, 0.15865525393145705), (-0.5, 0.30853753872598688),
             (0.0, 0.5), (0.5, 0.69146246127401312), (1.0, 0.84134474606854295),
             (1.96, 0.97500210485177952), (2.0, 0.97724986805182079)]


def test_gelu_against_normal_table_and_independent_routines():
    """The oracle's gelu against z Phi(z) with Phi taken from a table, from scipy's ndtr
    (Cephes, an implementation independent of torch.erf) and torch's own exact gelu."""
    from scipy.special import ndtr
    z = torch.tensor([t[0] for t in PHI_TABLE], dtype=torch.float64)
    ref = torch.tensor([t[0] * t[1] for t in PHI_TABLE], dtype=torch.float64)
    assert torch.max(torch.abs(F.gelu(z) - ref)) <= 1e-15
    w = torch.linspace(-8.0, 8.0, 4001, dtype=torch.float64)
    assert torch.max(torch.abs(F.gelu(w) - w * torch.from_numpy(ndtr(w.numpy())))) <= 4e-16 * 8
    assert torch.max(torch.abs(F.gelu(w) - torch.nn.functional.gelu(w, approximate="none"))) <= 4e-16 * 8
    # limits: gelu(z) -> z for large z, -> 0 for very negative z; gelu'(0) = 1/2
    assert abs(float(F.gelu(torch.tensor(40.0, dtype=torch.float64))) - 40.0) == 0.0
    assert abs(float(F.gelu(torch.tensor(-40.0, dtype=torch.float64)))) <= 1e-300
    h = 1e-6
    d0 = (F.gelu(torch.tensor(h, dtype=torch.float64)) - F.gelu(torch.tensor(-h, dtype=torch.float64))) / (2 * h)
    assert abs(float(d0) - 0.5) <= 1e-10


def test_gelu_prime_and_the_bf16_kept_backward():
    """gelu' against torch's own gelu backward (an implementation independent of the oracle's
    closed form) and a central difference; the layer GELU of the bf16 network differentiates
    at u rounded to bf16 (equal to gelu'(u) where u is a bf16 value, else at the rounded u)."""
    z = torch.linspace(-6.0, 6.0, 2001, dtype=torch.float64, requires_grad=True)
    torch.nn.functional.gelu(z, approximate="none").sum().backward()
    assert torch.max(torch.abs(F.gelu_prime(z.detach()) - z.grad)) <= 1e-15
    h = 1e-5
    fd = (F.gelu(z.detach() + h) - F.gelu(z.detach() - h)) / (2 * h)
    assert torch.max(torch.abs(F.gelu_prime(z.detach()) - fd)) <= 1e-9
    u = torch.tensor([0.1234567, -1.7654321, 2.5, 0.0], dtype=torch.float64, requires_grad=True)
    F._layer_gelu(u, True).sum().backward()
    uq = F.round_bf16(u.detach())
    assert torch.equal(u.grad, F.gelu_prime(uq))
    assert u.grad[2] == F.gelu_prime(torch.tensor(2.5, dtype=torch.float64))   # 2.5 is a bf16 value
    assert u.grad[0] != F.gelu_prime(u.detach()[0])                              # 0.1234567 is not
    assert torch.equal(F._layer_gelu(u.detach(), True), F.gelu(u.detach()))     # forward unchanged


def _batch(s, b=2, seed=5):
    rng = np.random.default_rng(seed)
    phi = torch.from_numpy(-0.2 + 0.05 * rng.standard_normal((b, s.n, s.n)))
    eps = torch.from_numpy(rng.uniform(0.1, 0.4, b))
    tgt = phi + torch.from_numpy(0.01 * rng.standard_normal((b, s.n, s.n)))
    return phi, eps, tgt


def test_mass_is_kept_exactly():
    p = F.init_params(S, 1)
    phi, eps, _ = _batch(S)
    out = F.forward(S, p, phi, eps)
    assert torch.max(torch.abs(out.mean(dim=(1, 2)) - phi.mean(dim=(1, 2)))) <= 1e-15


def test_translation_equivariance():
    """No positional input: circular shifts commute with the network."""
    p = F.init_params(S, 2)
    phi, eps, _ = _batch(S)
    a = F.forward(S, p, torch.roll(phi, (3, 5), (1, 2)), eps)
    b = torch.roll(F.forward(S, p, phi, eps), (3, 5), (1, 2))
    assert torch.max(torch.abs(a - b)) <= 1e-13


def test_gradients_match_finite_differences():
    p = F.init_params(S, 3)
    phi, eps, tgt = _batch(S)
    _, grads = F.loss_and_grads(S, p, phi, eps, tgt)
    rng = np.random.default_rng(6)
    for name in ("Lw", "Lb", "Wr0", "Wi1", "Pw0", "Pb1", "Q1", "q1", "Q2", "q2"):
        t = p[name]
        for _ in range(3):
            idx = tuple(int(rng.integers(0, d)) for d in t.shape)
            h = 1e-6 * max(1.0, abs(float(t[idx])))
            tp = dict(p); tm = dict(p)
            tp[name] = t.clone(); tp[name][idx] += h
            tm[name] = t.clone(); tm[name][idx] -= h
            fd = (float(F.mse(F.forward(S, tp, phi, eps), tgt)) - float(F.mse(F.forward(S, tm, phi, eps), tgt))) / (2 * h)
            g = float(grads[name][idx])
            assert abs(fd - g) <= 1e-6 * max(1e-6, abs(g)) + 1e-12, (name, idx, fd, g)


def test_output_is_band_limited():
    """The increment phi_pred - phi lies in the retained modes (up to the unpaired
    (0, -MY) entry, whose synthesis keeps only its real-part pair)."""
    p = F.init_params(S, 8)
    phi, eps, _ = _batch(S)
    d = (F.forward(S, p, phi, eps) - phi).numpy()
    spec = np.fft.rfft2(d)
    kx, ky = F.mode_indices(S)
    mask = np.zeros(spec.shape[1:], bool)
    mask[ky, kx] = True
    mask[S.my, 0] = True      # conjugate partner of (0, -MY) in the kx = 0 column
    assert np.max(np.abs(spec[:, ~mask])) <= 1e-12 * np.max(np.abs(spec))
