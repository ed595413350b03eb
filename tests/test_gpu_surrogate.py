"""The FNO surrogate in use: trained on the GPU on trajectories of the GPU SAV solver,
then jumping 50 steps at a time for 64 held-out members, with the SAV energy as judge
and the plain steps as fallback.

What is checked: a rejected jump leaves the run exactly on the plain path (bit for
bit); an accepted jump restarts the run from the prediction with the SAV variable
carried across; after training, every jump over a 300-step stretch is accepted, the
field reached is within 10 % (relative to the change over the stretch) of the plain
run's, and a jump costs less device time than the 50 plain steps it replaces.
Measured with 3000 training iterations: errors of 2-5 % of the change per jump and
2.4 % after 10 jumps; here 1200 iterations keep the test short.
"""

import math

import pytest
import torch

pytestmark = pytest.mark.gpu

M = 64


@pytest.fixture(scope="module")
def trained():
    from paper_2012_15133_amd import surrogate_run as R
    from paper_2012_15133_amd.surrogate import Surrogate, init_params
    mem = R.members(48, seed=11)
    traj, eps = R.trajectories(mem, snaps=40, warm=500)
    net = Surrogate(R.N, init_params(0), max_batch=32, train=True)
    log = R.train(net, traj, eps, iters=1200, batch=32, lr=1e-3, log_every=300)
    print("training loss", [(i, f"{l:.2e}") for i, l in log])
    params = net.params().cpu()
    net.close()
    del traj
    assert log[-1][1] < 0.05 * log[0][1]
    return params


def _held_out(warm):
    from paper_2012_15133_amd import Batch
    from paper_2012_15133_amd import surrogate_run as R
    test = R.members(M, seed=77)
    eps = torch.tensor([m["epsilon"] for m in test], dtype=torch.float32, device="cuda")
    b = Batch(test, history=16)
    b.step(R.DT, warm)
    return test, eps, b


def test_rejected_jumps_stay_on_the_plain_path(trained):
    from paper_2012_15133_amd import Batch
    from paper_2012_15133_amd import surrogate_run as R
    from paper_2012_15133_amd.surrogate import Surrogate
    test, eps, b = _held_out(200)
    plain = Batch(test, history=16)
    plain.step(R.DT, 200)
    net = Surrogate(R.N, trained, max_batch=M)
    J = R.Jumper(b, Batch(test, history=16), net, eps, energy_tol=-1.0)   # no jump can pass
    for _ in range(2):
        assert not J.jump()
    plain.step(R.DT, 2 * R.JUMP)
    assert J.rejected == 2 and J.accepted == 0 and J.b is b
    for m in (0, 17, 63):
        assert torch.equal(J.b.phi(m), plain.phi(m))
    net.close()


def test_accepted_jump_restarts_from_the_prediction(trained):
    from paper_2012_15133_amd import Batch
    from paper_2012_15133_amd import surrogate_run as R
    from paper_2012_15133_amd.surrogate import Surrogate
    test, eps, b = _held_out(300)
    net = Surrogate(R.N, trained, max_batch=M)
    phi = b.phi_all(torch.empty((M, R.N, R.N), dtype=torch.float32, device="cuda"))
    before = b.energies()
    pred = net.forward(phi, eps).to(torch.float64)
    J = R.Jumper(b, Batch(test, history=16), net, eps, energy_tol=1e9)   # every jump passes
    assert J.jump()
    assert J.b is not b and J.b.step_count() == 0
    for m in (0, 31):   # through the solver's forward and inverse transform
        assert torch.allclose(J.b.phi(m), pred[m], rtol=0, atol=1e-13)
    after = J.b.energies()
    for p, a in zip(before, after):
        # r' - sqrt(E_1(phi')) = r - sqrt(E_1(phi))
        assert a["r"] - math.sqrt(a["E1"]) == pytest.approx(p["r"] - math.sqrt(p["E1"]), abs=1e-12 * p["r"])
        assert a["mean"] == pytest.approx(p["mean"], abs=1e-6)
    net.close()


def test_jumps_are_accepted_accurate_and_faster(trained):
    from paper_2012_15133_amd import Batch
    from paper_2012_15133_amd import surrogate_run as R
    from paper_2012_15133_amd.surrogate import Surrogate
    test, eps, b = _held_out(1000)
    plain = Batch(test, history=16)
    plain.step(R.DT, 1000)
    net = Surrogate(R.N, trained, max_batch=M)
    start = plain.phi_all(torch.empty((M, R.N, R.N), dtype=torch.float64, device="cuda")).clone()
    J = R.Jumper(b, Batch(test, history=16), net, eps)
    jumps = 6
    for _ in range(jumps):
        J.jump()
    plain.step(R.DT, jumps * R.JUMP)
    ref = plain.phi_all(torch.empty_like(start))
    got = J.b.phi_all(torch.empty_like(start))
    err = ((got - ref).flatten(1).norm(dim=1) / (ref - start).flatten(1).norm(dim=1))
    print(f"accepted {J.accepted} of {jumps}; error / change: mean {float(err.mean()):.3f}, max {float(err.max()):.3f}")
    assert J.accepted == jumps
    assert float(err.mean()) <= 0.10
    # time of one jump against the 50 plain steps it replaces (wall, synchronized)
    t_plain = R.timed(lambda: plain.step(R.DT, R.JUMP), plain.stream)[1]
    t_jump = R.timed(lambda: J.jump(), J.b.stream)[1]
    print(f"50 plain steps {t_plain * 1e3:.2f} ms, one jump {t_jump * 1e3:.2f} ms (wall)")
    assert t_jump < t_plain
    net.close()


class _BadNet:
    """A stand-in network whose prediction is not finite (overflow or NaN in its output)."""

    def __init__(self, value):
        self.value = value

    def forward(self, phi, eps):
        # float64, so that a huge finite value stays finite and E_1 itself overflows
        out = torch.full(phi.shape, self.value, dtype=torch.float64, device=phi.device)
        out[:, 0, 0] = -self.value
        return out


@pytest.mark.parametrize("value", [float("inf"), float("nan"), 1e200])
def test_nonfinite_or_overflowing_prediction_is_a_rejected_jump(value):
    """A prediction that is not finite, or whose E_1 overflows, is rejected like any other
    failed jump: the run takes the plain steps and stays bit for bit on the plain path."""
    from paper_2012_15133_amd import Batch
    from paper_2012_15133_amd import surrogate_run as R
    test = R.members(6, seed=78)
    eps = torch.tensor([m["epsilon"] for m in test], dtype=torch.float32, device="cuda")
    b, plain = Batch(test, history=16), Batch(test, history=16)
    for x in (b, plain):
        x.step(R.DT, 20)
    J = R.Jumper(b, Batch(test, history=16), _BadNet(value), eps)
    assert not J.jump()
    plain.step(R.DT, R.JUMP)
    assert J.rejected == 1 and J.accepted == 0 and J.b is b
    for m in range(6):
        assert torch.equal(J.b.phi(m), plain.phi(m))
        assert J.b.status(m) == 0
    for x in (J.b, J.spare, plain):
        x.close()
