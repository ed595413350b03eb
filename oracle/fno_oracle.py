"""CPU oracle of the Fourier-neural-operator surrogate (test infrastructure only).

Plain, slow, obviously correct float64 PyTorch-on-CPU code; only tests/, the
package's smoke entry and bench.py's CPU baseline may import it.  Nothing here is
shared with the HIP path.

The surrogate maps phi(t) of an SPFC run (with its epsilon) to phi(t + 50 dt).
Network (a Fourier neural operator: lifting, Fourier layers, projection):

  input      x = (phi, epsilon) per grid point (epsilon broadcast)
  lifting    v0[c] = Lw[c,0] phi + Lw[c,1] epsilon + Lb[c]                  c < width
  layer l    u_l[o] = synth(mix_l(anal(v_l)))[o] + sum_i Pw_l[o,i] v_l[i] + Pb_l[o]
             v_{l+1} = gelu(u_l) for l < L-1, v_L = u_{L-1}
  projection h[k] = gelu(sum_c Q1[k,c] v_L[c] + q1[k]),  out = sum_k Q2[k] h[k] + q2
  filter     out_f = synth(anal(out))   (the increment restricted to the retained modes)
  output     phi_pred = phi + out_f - mean(out_f)   (the mean of phi is kept exactly)

Truncated transforms on an N x N grid (x contiguous), retained modes
kx in [0, MX) and ky in [0, MY) u [N - MY, N), mode index m = kx * 2MY + j with
ky = j (j < MY) or N - 2MY + j (j >= MY):

  anal(v)[m]  = alpha_kx sum_{y,x} v[y,x] exp(-2 pi i (kx x + ky y) / N),  alpha = 1 / N^2
  synth(U)[y,x] = sum_m beta_kx Re(U[m] exp(+2 pi i (kx x + ky y) / N)),   beta = 1 (kx = 0), 2 else
  mix(V)[o,m] = sum_i V[i,m] W[m,i,o]   (complex weights)

synth(anal(v)) = v for a real field band-limited to the retained modes except
(kx, ky) = (0, -MY), whose conjugate partner (0, +MY) is not retained (pinned in
tests).  gelu(z) = z Phi(z) with the normal distribution function Phi.

`bf16=True` rounds (to nearest even) where the GPU path stores bfloat16: the
activations v_l and the operands of the complex mixing (V and W), and, in the
backward pass, the pre-activation u_l of a Fourier layer at which gelu' is taken
(the GPU keeps u_l for the backward pass only as a bf16 copy).
"""

from __future__ import annotations

import functools
import math
from dataclasses import dataclass

import numpy as np
import torch

F64 = torch.float64


@dataclass(frozen=True)
class FnoShape:
    n: int = 256          # grid points per axis
    width: int = 32       # channels of the Fourier layers
    layers: int = 4
    mx: int = 16          # retained kx (half-spectrum axis)
    my: int = 16          # retained |ky| per sign
    hidden: int = 64      # projection hidden width

    @property
    def modes(self) -> int:
        return self.mx * 2 * self.my


# ----------------------------------------------------------------- bf16 rounding

def round_bf16(t: torch.Tensor) -> torch.Tensor:
    """Round to bfloat16 (nearest, ties to even) through float32, back to float64."""
    f = t.detach().to(torch.float32).numpy().astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (r.astype(np.uint32)).view(np.float32).astype(np.float64)
    return torch.from_numpy(out.reshape(f.shape))


class _StraightRound(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x):
        return round_bf16(x)

    @staticmethod
    def backward(ctx, g):
        return g


def _q(t, on: bool):
    return _StraightRound.apply(t) if on else t


# ----------------------------------------------------------------- transforms

def mode_indices(s: FnoShape):
    """(kx, ky) of mode index m = kx * 2MY + j."""
    kx = np.repeat(np.arange(s.mx), 2 * s.my)
    j = np.tile(np.arange(2 * s.my), s.mx)
    ky = np.where(j < s.my, j, s.n - 2 * s.my + j)
    return kx, ky


@functools.lru_cache(maxsize=4)
def _phase(s: FnoShape, sign: float):
    """exp(sign 2 pi i (kx x + ky y) / N) as a [modes, N(y), N(x)] complex tensor."""
    kx, ky = mode_indices(s)
    y = np.arange(s.n)[None, :, None]
    x = np.arange(s.n)[None, None, :]
    ang = 2.0 * math.pi * ((kx[:, None, None] * x) % s.n + (ky[:, None, None] * y) % s.n) / s.n
    return torch.from_numpy(np.exp(sign * 1j * ang))


def analysis(s: FnoShape, v: torch.Tensor, alpha=None) -> torch.Tensor:
    """v [..., N, N] real -> [..., modes] complex, alpha per mode (default 1/N^2)."""
    E = _phase(s, -1.0)
    out = torch.einsum("...yx,myx->...m", v.to(torch.complex128), E)
    a = torch.full((s.modes,), 1.0 / (s.n * s.n), dtype=F64) if alpha is None else alpha
    return out * a


def beta(s: FnoShape) -> torch.Tensor:
    kx, _ = mode_indices(s)
    return torch.from_numpy(np.where(kx == 0, 1.0, 2.0))


def synthesis(s: FnoShape, U: torch.Tensor, b=None) -> torch.Tensor:
    """U [..., modes] complex -> [..., N, N] real: sum_m b_m Re(U_m e^{+i...})."""
    E = _phase(s, +1.0)
    w = beta(s) if b is None else b
    return torch.einsum("...m,myx->...yx", U * w, E).real


# ----------------------------------------------------------------- network

def gelu(z):
    return 0.5 * z * (1.0 + torch.erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    """d/dz [z Phi(z)] = Phi(z) + z phi(z), phi the standard normal density."""
    return 0.5 * (1.0 + torch.erf(z / math.sqrt(2.0))) + z * torch.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


class _GeluKeptBf16(torch.autograd.Function):
    """gelu(u) whose derivative in the backward pass is taken at u rounded to bf16: the GPU
    keeps the pre-activation of a Fourier layer for its backward pass only as a bf16 copy."""

    @staticmethod
    def forward(ctx, u):
        ctx.save_for_backward(round_bf16(u))
        return gelu(u)

    @staticmethod
    def backward(ctx, g):
        (uq,) = ctx.saved_tensors
        return g * gelu_prime(uq)


def _layer_gelu(u, bf16: bool):
    return _GeluKeptBf16.apply(u) if bf16 else gelu(u)


def init_params(s: FnoShape, seed: int = 0) -> dict:
    """Seeded initial weights (uniform, fan-in scaled); float64 tensors."""
    g = torch.Generator().manual_seed(seed)

    def u(shape, scale):
        return (torch.rand(shape, generator=g, dtype=F64) * 2.0 - 1.0) * scale

    c, h = s.width, s.hidden
    p = {"Lw": u((c, 2), 1.0), "Lb": u((c,), 0.1)}
    for l in range(s.layers):
        sc = 1.0 / (c * c)
        p[f"Wr{l}"] = u((s.modes, c, c), sc)
        p[f"Wi{l}"] = u((s.modes, c, c), sc)
        p[f"Pw{l}"] = u((c, c), 1.0 / math.sqrt(c))
        p[f"Pb{l}"] = u((c,), 0.1)
    p["Q1"] = u((h, c), 1.0 / math.sqrt(c))
    p["q1"] = u((h,), 0.1)
    p["Q2"] = u((h,), 1.0 / math.sqrt(h))
    p["q2"] = u((1,), 0.0)
    return p


def forward(s: FnoShape, p: dict, phi: torch.Tensor, eps: torch.Tensor, bf16: bool = False) -> torch.Tensor:
    """phi [B, N, N], eps [B] -> phi_pred [B, N, N]."""
    v = p["Lw"][None, :, 0, None, None] * phi[:, None] + p["Lw"][None, :, 1, None, None] * eps[:, None, None, None] \
        + p["Lb"][None, :, None, None]
    v = _q(v, bf16)
    for l in range(s.layers):
        V = analysis(s, v)                                          # [B, C, M]
        W = torch.complex(_q(p[f"Wr{l}"], bf16), _q(p[f"Wi{l}"], bf16))   # [M, I, O]
        Vq = torch.complex(_q(V.real, bf16), _q(V.imag, bf16))
        U = torch.einsum("bim,mio->bom", Vq, W)
        w = synthesis(s, U)
        u = w + torch.einsum("oi,biyx->boyx", p[f"Pw{l}"], v) + p[f"Pb{l}"][None, :, None, None]
        v = _layer_gelu(u, bf16) if l < s.layers - 1 else u
        v = _q(v, bf16)
    hpre = torch.einsum("kc,bcyx->bkyx", p["Q1"], v) + p["q1"][None, :, None, None]
    out = torch.einsum("k,bkyx->byx", p["Q2"], gelu(hpre)) + p["q2"][0]
    out = synthesis(s, analysis(s, out))
    return phi + out - out.mean(dim=(1, 2), keepdim=True)


def mse(pred: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """Mean over samples and points of the squared error."""
    return ((pred - target) ** 2).mean()


def loss_and_grads(s: FnoShape, p: dict, phi, eps, target, bf16: bool = False):
    """Loss and gradients with respect to every parameter (float64 autograd)."""
    q = {k: v.detach().clone().requires_grad_(True) for k, v in p.items()}
    loss = mse(forward(s, q, phi, eps, bf16), target)
    loss.backward()
    return float(loss.detach()), {k: v.grad.detach().clone() for k, v in q.items()}
