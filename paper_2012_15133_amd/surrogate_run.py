"""The surrogate in use: training data from the GPU SAV-BDF2 solver, training on the GPU,
and jumps of 50 steps judged by the solver, with the plain steps as fallback.

Workload (2-D, as the surrogate is specified): n = 256 points per axis on a box of side
16 pi (h = pi / 16), epsilon ~ U[0.1, 0.4), mean density -0.2 with the noise initial data
of `inputs.noise_ic`, dt = 0.01; the network maps phi(t) to phi(t + 50 dt).  The side is
chosen so that the network's retained modes (|m| < 16, i.e. |k| < 2) hold the pattern's
wavenumber |k| = 1 and its first harmonics; on a box of side 32 pi they would stop at
|k| < 1.

A jump from a running state (phi, r) to the predicted phi' is judged by the SAV energy
of the paper's Section 5.2, Eb(phi, r) = a/2 ||phi||^2 + 1/2 ||Delta_N phi||^2 + r^2, with
the SAV variable carried across the jump as r' = r + sqrt(E_1(phi')) - sqrt(E_1(phi))
(the continuous-time SAV relation keeps r - sqrt(E_1(phi)) constant; a long discrete
run drifts away from r = sqrt(E_1), and its dynamics depend on that drift).  The jump is
accepted when Eb(phi', r') <= Eb(phi, r) for every member and the mean is kept (the
network keeps it by construction).  The prediction is restarted in a second batch of
the same members; an accepted jump makes that batch the running one, a rejected jump
leaves the running batch untouched and it takes the 50 plain steps.
"""

from __future__ import annotations

import math
import time

from .binding import SPFC_E_INVAL, SpfcError
from .inputs import noise_ic, uniform_range

JUMP = 50
DT = 0.01
N = 256
SIDE = 16.0 * math.pi


def members(count: int, seed: int, eps_range=(0.1, 0.4), mean: float = -0.2, n: int = N, side: float = SIDE):
    """Member dicts for `Batch`: seeded epsilon and noise initial data."""
    eps = uniform_range(seed, count, eps_range[0], eps_range[1])
    return [{"n": (n, n), "L": (side, side), "epsilon": float(eps[k]),
             "phi0": noise_ic((n, n), mean, seed * 1000 + k + 1)} for k in range(count)]


def trajectories(mem, snaps: int, warm: int = 0, jump: int = JUMP, dt: float = DT):
    """Run all members together; return float32 device tensors traj [snaps + 1, M, n, n]
    (phi at warm, warm + jump, ... steps) and eps [M]."""
    import torch
    from .binding import Batch
    n = mem[0]["n"][0]
    b = Batch(mem, history=16)
    if warm:
        b.step(dt, warm)
    traj = torch.empty((snaps + 1, len(mem), n, n), dtype=torch.float32, device="cuda")
    b.phi_all(traj[0])
    for s in range(snaps):
        b.step(dt, jump)
        b.phi_all(traj[s + 1])
    b.close()
    eps = torch.tensor([m["epsilon"] for m in mem], dtype=torch.float32, device="cuda")
    return traj, eps


def train(net, traj, eps, iters: int, batch: int, lr: float, seed: int = 0, log_every: int = 100):
    """Adam on random (snapshot, member) pairs, cosine learning-rate decay to lr / 20.
    Returns [(iteration, loss)] sampled every log_every iterations."""
    import torch
    S, M = traj.shape[0] - 1, traj.shape[1]
    g = torch.Generator().manual_seed(seed)
    log = []
    for it in range(iters):
        si = torch.randint(0, S, (batch,), generator=g).to("cuda")
        mi = torch.randint(0, M, (batch,), generator=g).to("cuda")
        phi = traj[si, mi].contiguous()
        tgt = traj[si + 1, mi].contiguous()
        e = eps[mi].contiguous()
        lr_t = lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * it / max(1, iters))))
        loss = net.train_step(phi, e, tgt, lr_t)
        if it % log_every == 0 or it == iters - 1:
            log.append((it, float(loss.item())))
    return log


class Jumper:
    """Advance a SAV run of `batch` (members of one grid size) by jumps of JUMP steps;
    `spare` is a second batch of the same members.  The two swap roles on every accepted
    jump: the running batch is always `self.b`, and it is advanced only through jump() (the
    energies of an accepted state are kept for the next jump)."""

    def __init__(self, batch, spare, net, eps, dt: float = DT, energy_tol: float = 0.0):
        import torch
        self.torch = torch
        self.b = batch
        self.spare = spare
        self.net = net
        self.eps = eps
        self.dt = dt
        self.tol = energy_tol
        n = batch.ns[0][0]
        self.phi = torch.empty((len(batch), n, n), dtype=torch.float32, device="cuda")
        self.pred = torch.empty((len(batch), n, n), dtype=torch.float64, device="cuda")
        self.accepted = 0
        self.rejected = 0
        self._energies = None   # energies of the running batch's state, when known

    def decide(self, before, after):
        """Whether a restart `after` (made with r shifted by r - sqrt(E_1) of `before`)
        is accepted (see module text)."""
        for p, a in zip(before, after):
            good = (math.isfinite(a["sav_energy"])
                    and a["sav_energy"] <= p["sav_energy"] + self.tol * abs(p["sav_energy"])
                    and abs(a["mean"] - p["mean"]) <= 1e-6)
            if not good:
                return False
        return True

    def jump(self) -> bool:
        self.b.phi_all(self.phi)
        before = self._energies if self._energies is not None else self.b.energies()
        self.pred.copy_(self.net.forward(self.phi, self.eps))
        shift = [p["r"] - math.sqrt(p["E1"]) for p in before]
        after = None
        if not bool(self.torch.isfinite(self.pred).all()):
            ok = False       # a non-finite prediction: no jump (its E_1 could overflow to inf, r = inf)
        else:
            try:
                self.spare.reset(self.pred, shift)
            except SpfcError as e:
                if e.status != SPFC_E_INVAL:
                    raise
                ok = False       # a shifted r not positive: no jump
            else:
                # energies of every member even where one is not finite (decide() rejects those)
                after = self.spare.energies(allow_nonfinite=True)
                ok = self.decide(before, after)
        if ok:
            self.accepted += 1
            self.b, self.spare = self.spare, self.b
            self._energies = after      # the new running state's, computed just now
            return True
        self.rejected += 1
        self.b.step(self.dt, JUMP)
        self._energies = None
        return False


def timed(fn, stream):
    """Wall time of fn() on the device: HIP events on `stream` around it."""
    import torch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3, time.perf_counter() - t0
