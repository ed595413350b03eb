"""FNO surrogate on the GPU (libspfc_fno.so through its C ABI) against the CPU oracle.

The oracle runs in float64 with bfloat16 rounding at the points where the GPU stores
bfloat16 (activations, the mixing operands), on the same float32 weights.  What
remains is the GPU's FP32 accumulation order: a spectral coefficient summed over
N^2 = 4096 points carries ~1e-4 relative FP32 error where the sum cancels, enough to
flip its bfloat16 rounding (2^-8 relative) for a few percent of the mixing inputs,
and the forward row kernel's matrix-core products carry FP32 operands as bf16 hi + lo
pairs (16 significant bits), which flips a few more roundings of the stored
activations; over four layers that gives ~5e-3 to 1.5e-2 norm-wise relative
differences in the forward pass (bound 2e-2).  Against the unrounded float64 network
the bf16 storage itself moves the increment by ~10 % here; that is reported and
bounded only loosely.  Gradient bounds are derived per block in the test from how
much bf16 rounding moves the oracle's own gradient.
"""

import numpy as np
import pytest
import torch

from conftest import error_report
from oracle import fno_oracle as F

pytestmark = pytest.mark.gpu

N = 64
S = F.FnoShape(n=N)


def _params(seed):
    p = F.init_params(S, seed)
    # the GPU holds float32 weights: give the oracle the same values
    return {k: v.to(torch.float32).to(torch.float64) for k, v in p.items()}


def _batch(b, seed):
    rng = np.random.default_rng(seed)
    phi = torch.from_numpy(-0.2 + 0.1 * rng.standard_normal((b, N, N))).to(torch.float32).to(torch.float64)
    eps = torch.from_numpy(rng.uniform(0.1, 0.4, b)).to(torch.float32).to(torch.float64)
    tgt = (phi + torch.from_numpy(0.05 * rng.standard_normal((b, N, N)))).to(torch.float32).to(torch.float64)
    return phi, eps, tgt


def _rel(a, b):
    return float(torch.linalg.norm((a - b).reshape(-1)) / torch.linalg.norm(b.reshape(-1)))


def test_forward_matches_oracle():
    from paper_2012_15133_amd.surrogate import Surrogate
    p = _params(1)
    phi, eps, _ = _batch(3, 2)
    net = Surrogate(N, p, max_batch=4)
    got = net.forward(phi, eps).cpu().to(torch.float64)
    ref = F.forward(S, p, phi, eps, bf16=True)
    ref64 = F.forward(S, p, phi, eps, bf16=False)
    e_bf = _rel(got - phi, ref - phi)
    e_64 = _rel(got - phi, ref64 - phi)
    print(f"increment rel L2: vs bf16 oracle {e_bf:.2e}, vs fp64 oracle {e_64:.2e}")
    assert e_bf <= 2e-2
    assert e_64 <= 0.3
    # the mean of phi is kept (to FP32 rounding of a sum over N^2 points)
    assert torch.max(torch.abs(got.mean(dim=(1, 2)) - phi.mean(dim=(1, 2)))) <= 1e-6
    net.close()


def _well_conditioned_batch(b, seed):
    """Unit-variance fields and an in-band target increment: the gradients are then not
    dominated by bf16 rounding of nearly cancelling sums (small fluctuations on a large
    mean make the projection gradients swing by ~100 % between a bf16 and a float64
    network, which would test nothing)."""
    rng = np.random.default_rng(seed)
    phi = torch.from_numpy(rng.standard_normal((b, N, N))).to(torch.float32).to(torch.float64)
    eps = torch.from_numpy(rng.uniform(0.1, 0.4, b)).to(torch.float32).to(torch.float64)
    inc = F.synthesis(S, F.analysis(S, torch.from_numpy(rng.standard_normal((b, N, N)))))
    tgt = (phi + 0.3 * N * inc / inc.norm()).to(torch.float32).to(torch.float64)
    return phi, eps, tgt


def test_gradients_match_oracle():
    """Each block of the gradient within half the change bf16 rounding itself makes to the
    oracle's gradient of that block, or within 2e-2 (unit-variance inputs; the reading of
    the n = 256 tests below), of the bf16 oracle; the loss to 1e-3."""
    from paper_2012_15133_amd.surrogate import Surrogate, unflatten
    p = _params(3)
    phi, eps, tgt = _well_conditioned_batch(2, 4)
    net = Surrogate(N, p, max_batch=2, train=True)
    loss, g = net.grads(phi, eps, tgt)
    gg = unflatten(g.cpu().to(torch.float64))
    ref_loss, ref = F.loss_and_grads(S, p, phi, eps, tgt, bf16=True)
    _, ref64 = F.loss_and_grads(S, p, phi, eps, tgt, bf16=False)
    print(f"loss {loss:.6e} vs {ref_loss:.6e}")
    assert abs(loss - ref_loss) <= 1e-3 * ref_loss
    assert abs(float(gg["q2"][0])) <= 1e-2 * float(torch.linalg.norm(ref["Q2"]))   # zero in exact arithmetic
    for k, r in ref.items():
        if k == "q2":
            continue
        e, sens = _rel(gg[k], r), _rel(ref64[k], r)
        print(f"  grad {k:5s} rel L2 {e:.2e}  (bf16 vs float64 oracle {sens:.2e})")
        assert e <= 0.5 * sens or e <= 2e-2, k
    a = torch.cat([gg[k].reshape(-1) for k in ref if k != "q2"])
    b = torch.cat([ref[k].reshape(-1) for k in ref if k != "q2"])
    cos = float(torch.dot(a, b) / (torch.linalg.norm(a) * torch.linalg.norm(b)))
    print(f"gradient cosine {cos:.6f}")
    assert cos >= 0.999
    net.close()


def test_translation_equivariance_and_batch_independence():
    from paper_2012_15133_amd.surrogate import Surrogate
    p = _params(5)
    phi, eps, _ = _batch(4, 6)
    net = Surrogate(N, p, max_batch=4)
    a = net.forward(torch.roll(phi, (8, 16), (1, 2)), eps).cpu().to(torch.float64)
    b = torch.roll(net.forward(phi, eps).cpu().to(torch.float64), (8, 16), (1, 2))
    assert _rel(a - torch.roll(phi, (8, 16), (1, 2)), b - torch.roll(phi, (8, 16), (1, 2))) <= 2e-2
    # a sample's result does not depend on the other samples of the batch
    one = net.forward(phi[2:3], eps[2:3]).cpu().to(torch.float64)
    four = net.forward(phi, eps).cpu().to(torch.float64)
    assert torch.equal(one[0], four[2])
    net.close()


def test_adam_steps_reduce_the_loss():
    """A learnable target: phi plus half of its mean-free low-pass part (|k| < 6), an
    increment inside the retained band that the spectral path can express."""
    from paper_2012_15133_amd.surrogate import Surrogate
    p = _params(7)
    phi, eps, _ = _batch(4, 8)
    k = np.fft.fftfreq(N, 1.0 / N)
    mask = (np.abs(k)[:, None] < 6) & (np.abs(k)[None, :] < 6)
    mask[0, 0] = False
    tgt = phi + 0.5 * torch.from_numpy(np.real(np.fft.ifft2(np.fft.fft2(phi.numpy()) * mask)))
    net = Surrogate(N, p, max_batch=4, train=True)
    d = lambda t: t.to(device="cuda", dtype=torch.float32).contiguous()
    phi_d, eps_d, tgt_d = d(phi), d(eps), d(tgt)
    losses = [float(net.train_step(phi_d, eps_d, tgt_d, 3e-3).item()) for _ in range(80)]
    print("losses", [f"{x:.3e}" for x in losses[::10]])
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.3 * losses[0]
    net.close()


def test_per_kernel_timing_leaves_the_result_unchanged():
    """The per-kernel timing call repeats each launch of a forward pass back to back; the
    launches are idempotent, so its output equals the plain forward pass bit for bit, and
    it reports each kernel role with its launch count per pass."""
    from paper_2012_15133_amd.binding import SpfcError
    from paper_2012_15133_amd.surrogate import Surrogate, spfc_fno_time_forward
    p = _params(9)
    phi, eps, _ = _batch(4, 10)
    net = Surrogate(N, p, max_batch=4)
    ref = net.forward(phi, eps)
    roles, got = net.time_forward(phi, eps, reps=3)
    assert torch.equal(got, ref)
    counts = {k: v[2] for k, v in roles.items()}
    assert counts == {"lift_row": 1, "col_anal": 4, "mix": 4, "col_synth": 4, "layer_row": 3, "last_row": 1,
                      "filter_anal": 1, "filter_synth": 1, "finish": 1}
    assert all(v[0] > 0 and v[1] > 0 for v in roles.values())
    # the output must not alias the input (the last kernel adds the increment to phi)
    x, e = net._inputs(phi, eps)
    with pytest.raises(SpfcError):
        spfc_fno_time_forward(net.h, 4, x.data_ptr(), e.data_ptr(), x.data_ptr(), 2)
    with pytest.raises(SpfcError):
        spfc_fno_time_forward(net.h, 4, x.data_ptr(), e.data_ptr(), ref.data_ptr(), 0)
    net.close()


def test_large_and_small_batches_agree():
    """Batch 64 (2048 planes: the column analysis takes four units per workgroup, one
    wave each) against batches of 4 (few planes: the rows of a unit split over four
    waves): the same samples give the same increments up to FP32 summation order (which
    can flip a bf16 rounding of a mixing operand, as against the oracle; measured 8.8e-4,
    bound 5e-3), and
    both stay within the oracle bound on samples the oracle checks."""
    from paper_2012_15133_amd.surrogate import Surrogate
    p = _params(11)
    phi, eps, _ = _batch(64, 12)
    net = Surrogate(N, p, max_batch=64)
    big = net.forward(phi, eps).cpu().to(torch.float64)
    small = torch.cat([net.forward(phi[i:i + 4], eps[i:i + 4]).cpu().to(torch.float64) for i in range(0, 64, 4)])
    e = _rel(big - phi, small - phi)
    print(f"batch 64 vs batches of 4: increment rel L2 {e:.2e}")
    assert e <= 5e-3
    ref = F.forward(S, p, phi[:2], eps[:2], bf16=True)
    assert _rel(big[:2] - phi[:2], ref - phi[:2]) <= 2e-2
    net.close()


# ----------------------------------------------------------------- n = 256, the size the surrogate runs at
#
# Bound (a reading fixed before these tests ran): the GPU and the bf16 oracle round to
# bf16 at the same points, so they can differ only where the GPU's FP32 summation order
# flips one of those roundings, by one bf16 unit each.  The gap between the bf16 oracle
# and the float64 oracle is the effect of every rounding at once.  A GPU path that rounds
# where the oracle does, and nowhere else, therefore stays within half of that gap: per
# gradient block in relative L2, and on the increment both in relative L2 and point by
# point (its largest pointwise difference against half the largest pointwise bf16 gap).
# An extra rounding, a dropped term or a wrong operand moves the GPU by at least the
# whole gap and fails.  On unit-variance inputs the fixed 2e-2 of the n = 64 tests holds
# as well.

N256 = 256
S256 = F.FnoShape(n=N256)


def _inputs_256(b, seed, regime):
    """"data": the surrogate's inputs, mean -0.2 with 0.05 (2u - 1) noise and epsilon in
    [0.1, 0.4), a target 2e-2 away inside the retained band; "unit": unit-variance fields."""
    rng = np.random.default_rng(seed)
    if regime == "data":
        phi = -0.2 + 0.05 * (2.0 * rng.random((b, N256, N256)) - 1.0)
        amp = 0.02
    else:
        phi = rng.standard_normal((b, N256, N256))
        amp = 0.3
    eps = rng.uniform(0.1, 0.4, b)
    inc = F.synthesis(S256, F.analysis(S256, torch.from_numpy(rng.standard_normal((b, N256, N256)))))
    f = lambda t: torch.as_tensor(t).to(torch.float32).to(torch.float64)
    phi = f(phi)
    return phi, f(eps), f(phi + amp * inc / inc.abs().max())


@pytest.mark.parametrize("regime", ["data", "unit"])
def test_forward_n256_element_by_element(regime):
    from paper_2012_15133_amd.surrogate import Surrogate
    p = _params(13)
    phi, eps, _ = _inputs_256(2, 14, regime)
    net = Surrogate(N256, p, max_batch=2)
    got = net.forward(phi, eps).cpu().to(torch.float64)
    net.close()
    ref = F.forward(S256, p, phi, eps, bf16=True)
    ref64 = F.forward(S256, p, phi, eps, bf16=False)
    d, dr, d64 = got - phi, ref - phi, ref64 - phi
    gap_inf = float((d - dr).abs().max())
    sens_inf = float((dr - d64).abs().max())
    e_bf, sens = _rel(d, dr), _rel(dr, d64)
    error_report(f"fno n=256 forward ({regime})", rel_l2=e_bf, bf16_vs_fp64_l2=sens,
                 max_point_gap=gap_inf, bf16_vs_fp64_max_point=sens_inf)
    assert gap_inf <= 0.5 * sens_inf
    assert e_bf <= 0.5 * sens
    if regime == "unit":
        assert e_bf <= 2e-2
    assert torch.max(torch.abs(got.mean(dim=(1, 2)) - phi.mean(dim=(1, 2)))) <= 1e-6


@pytest.mark.parametrize("regime", ["data", "unit"])
def test_gradients_n256(regime):
    from paper_2012_15133_amd.surrogate import Surrogate, unflatten
    p = _params(15)
    phi, eps, tgt = _inputs_256(2, 16, regime)
    net = Surrogate(N256, p, max_batch=2, train=True)
    loss, g = net.grads(phi, eps, tgt)
    net.close()
    gg = unflatten(g.cpu().to(torch.float64))
    ref_loss, ref = F.loss_and_grads(S256, p, phi, eps, tgt, bf16=True)
    _, ref64 = F.loss_and_grads(S256, p, phi, eps, tgt, bf16=False)
    assert abs(loss - ref_loss) <= 1e-3 * ref_loss
    worst, bad = 0.0, []
    for k, r in ref.items():
        if k == "q2":
            continue
        e, sens = _rel(gg[k], r), _rel(ref64[k], r)
        print(f"  grad {k:5s} rel L2 {e:.2e}  (bf16 vs float64 oracle {sens:.2e})")
        worst = max(worst, e / sens)
        if not (e <= 0.5 * sens or (regime == "unit" and e <= 2e-2)):
            bad.append((k, e, sens))
    error_report(f"fno n=256 gradients ({regime})", worst_block_gap_over_bf16_gap=worst)
    assert not bad, bad
