"""GPU path: precision variants, determinism, checkpoint/resume, restarts, the history
ring, error codes and full-size properties, all through the C ABI."""

import ctypes
import math
import os

import numpy as np
import pytest

from oracle import spfc_oracle as O
from paper_2012_15133_amd.inputs import noise_ic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu

L64 = (8 * math.pi,) * 2


def _solver(n, L, phi0, eps=0.25, **kw):
    from paper_2012_15133_amd import Solver
    return Solver(n, L, phi0, eps, **kw)


def _run(n, L, phi0, dt, steps, **kw):
    s = _solver(n, L, phi0, history=steps + 1, **kw)
    s.step(dt, steps)
    return s, s.history(0, steps + 1), s.phi().cpu().numpy()


# ----------------------------------------------------------------- FP32 fields, FP64 scalars

@pytest.mark.parametrize("n,L,steps,seed", [((64, 64), L64, 200, 1), ((32, 32, 32), (4 * math.pi,) * 3, 40, 3)])
def test_fp32_path_error_report(n, L, steps, seed):
    """FP32 transforms and pointwise work, FP64 reductions and SAV scalar, against the FP64
    oracle.  The paper fixes no FP32 accuracy (parity unpinned); the bounds are the flags of
    the error report: relative L-inf <= 1e-3, modified energy <= 1e-5 relative."""
    g = O.Grid(n, L)
    phi0 = noise_ic(g.shape, -0.2, seed)
    dt = 0.01 if len(n) == 2 else 0.005
    ref = O.run(g, O.Params(0.25), phi0, dt, steps)
    s, hist, phi = _run(n, L, phi0, dt, steps, precision="fp32")
    linf = np.max(np.abs(phi - ref["phi"])) / np.max(np.abs(ref["phi"]))
    e_err = max(abs(h["energy"] - r["energy"]) / r["energy"] for h, r in zip(hist, ref["records"]))
    m_err = max(abs(h["mean"] - r["mean"]) for h, r in zip(hist, ref["records"]))
    print(f"fp32 {n}: rel Linf {linf:.2e}, modified energy rel {e_err:.2e}, mean {m_err:.2e}")
    assert linf <= 1e-3 and e_err <= 1e-5 and m_err <= 1e-6
    assert s.status() & ~8 == 0      # an FP32-noise energy rise may set ENERGY_RISE only
    s.close()


def test_fp32_full_size_2d_sampled():
    n, L = (1024, 1024), (128 * math.pi,) * 2
    g = O.Grid(n, L)
    phi0 = noise_ic(g.shape, -0.2, 2)
    ref = O.run(g, O.Params(0.25), phi0, 0.01, 2, energies=False)
    s, hist, phi = _run(n, L, phi0, 0.01, 2, precision="fp32")
    linf = np.max(np.abs(phi - ref["phi"])) / np.max(np.abs(ref["phi"]))
    print(f"fp32 1024^2 after 2 steps: rel Linf {linf:.2e}")
    assert linf <= 1e-5
    s.close()


# ----------------------------------------------------------------- determinism and checkpoints

def test_bitwise_determinism():
    phi0 = noise_ic((64, 64), -0.2, 1)
    _, h1, p1 = _run((64, 64), L64, phi0, 0.01, 60)
    _, h2, p2 = _run((64, 64), L64, phi0, 0.01, 60)
    assert np.array_equal(p1, p2)
    assert h1 == h2


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_checkpoint_resume_is_bitwise(precision):
    n = (64, 32)
    L = (8 * math.pi, 4 * math.pi)
    phi0 = noise_ic((32, 64), -0.1, 4)
    a = _solver(n, L, phi0, precision=precision, history=128)
    a.step(0.01, 25)
    ck = a.save_state()
    a.step(0.01, 30)
    ref_phi = a.phi().cpu().numpy()
    ref_hist = a.history(25, 31)
    b = _solver(n, L, noise_ic((32, 64), 0.3, 99), precision=precision, history=128)
    b.load_state(ck)
    assert b.step_count() == 25
    b.step(0.01, 30)
    assert np.array_equal(b.phi().cpu().numpy(), ref_phi)
    got = b.history(26, 30)
    for x, y in zip(got, ref_hist[1:]):
        assert x == y
    a.close()
    b.close()


def test_dt_change_restarts_like_the_paper():
    """A new dt restarts the two-step scheme from phi^{-1} = phi^0 with r = sqrt(E_1(phi^0))
    (Section 5.2); the oracle does the same with startup 'copy' from the state reached."""
    n = (32, 32)
    L = (4 * math.pi,) * 2
    g = O.Grid(n, L)
    prm = O.Params(0.25)
    phi0 = noise_ic(g.shape, -0.2, 5)
    first = O.run(g, prm, phi0, 0.01, 15)
    second = O.run(g, prm, first["phi"], 0.02, 15, startup="copy")
    s = _solver(n, L, phi0, history=64)
    s.step(0.01, 15)
    s.step(0.02, 15)
    phi = s.phi().cpu().numpy()
    assert np.max(np.abs(phi - second["phi"])) <= 1e-11 * np.max(np.abs(second["phi"]))
    hist = s.history(16, 15)
    for h, r in zip(hist, second["records"][1:]):
        assert abs(h["energy"] - r["energy"]) <= 1e-12 * r["energy"]
    s.close()


def test_history_ring_and_out_of_range():
    from paper_2012_15133_amd import SpfcError
    phi0 = noise_ic((32, 32), -0.2, 7)
    s = _solver((32, 32), (4 * math.pi,) * 2, phi0, history=16)
    s.step(0.01, 50)
    ok = s.history(35, 16)
    assert len(ok) == 16 and all(np.isfinite(r["energy"]) for r in ok)
    with pytest.raises(SpfcError):
        s.history(30, 5)
    with pytest.raises(SpfcError):
        s.history(45, 10)
    s.close()


# ----------------------------------------------------------------- error codes

def test_error_codes_on_device():
    import torch
    from paper_2012_15133_amd import binding as B
    lib = B.load_library()
    g = B.make_grid((32, 32), (4 * math.pi,) * 2)
    p = B.make_params(0.25)
    nb = B.spfc_workspace_bytes(g, p)
    ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    wsp = (ws.data_ptr() + 255) // 256 * 256
    phi = torch.tensor(noise_ic((32, 32), -0.2, 1), device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    ctx = ctypes.c_void_p()
    assert lib.spfc_init(ctypes.byref(g), ctypes.byref(p), phi.data_ptr(), wsp, nb - 1, stream,
                         ctypes.byref(ctx)) == B.SPFC_E_NOMEM
    bad = phi.clone()
    bad[3, 4] = float("nan")
    assert lib.spfc_init(ctypes.byref(g), ctypes.byref(p), bad.data_ptr(), wsp, nb, stream,
                         ctypes.byref(ctx)) == B.SPFC_E_INVAL
    assert lib.spfc_init(ctypes.byref(g), ctypes.byref(p), phi.data_ptr(), wsp, nb, stream,
                         ctypes.byref(ctx)) == B.SPFC_OK
    assert lib.spfc_step(ctx, 0.0, 1) == B.SPFC_E_INVAL
    assert lib.spfc_step(ctx, float("nan"), 1) == B.SPFC_E_INVAL
    assert lib.spfc_step(ctx, 0.01, -1) == B.SPFC_E_INVAL
    assert lib.spfc_step(ctx, 0.01, 0) == B.SPFC_OK
    out = torch.empty((32, 32), dtype=torch.float64, device="cuda")
    assert lib.spfc_get_phi(ctx, out.data_ptr(), 7) == B.SPFC_E_INVAL
    recs = (B.spfc_record * 2)()
    assert lib.spfc_history(ctx, 1, 2, recs) == B.SPFC_E_STATE
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    assert lib.spfc_save_state(ctx, small.data_ptr(), 16) == B.SPFC_E_STATE
    assert lib.spfc_destroy(ctx) == B.SPFC_OK


def test_nonfinite_flag_is_sticky():
    """Initial data so large that E_1 overflows: the step sets NONFINITE and the energy query
    reports it (condition forced from the host; the kernels just carry inf/NaN)."""
    from paper_2012_15133_amd import binding as B
    phi0 = noise_ic((32, 32), 0.0, 3) * 1e80
    s = _solver((32, 32), (4 * math.pi,) * 2, phi0)
    s.step(0.01, 2)
    assert s.status() & B.SPFC_FLAG_NONFINITE
    e = B.spfc_energy(s.ctx, allow_nonfinite=True)
    assert not math.isfinite(e["E1"]) or not math.isfinite(e["modified_energy"])
    s.close()


# ----------------------------------------------------------------- full 3-D size

def test_3d_full_size_properties():
    """256^3, L = 32 pi, dt = 0.005, FP32 fields: 500 steps; mass conserved to FP32 round-off,
    modified energy non-increasing up to FP32 noise, p1 <= 0, E_1 >= |Omega|, and the first
    steps agree with the FP64 GPU path on the same input."""
    n = (256, 256, 256)
    L = (32 * math.pi,) * 3
    phi0 = noise_ic((256, 256, 256), -0.25, 3)
    s = _solver(n, L, phi0, precision="fp32", history=501)
    s.step(0.005, 500)
    hist = s.history(0, 501)
    m0 = float(np.mean(phi0))
    vol = (32 * math.pi) ** 3
    for k, h in enumerate(hist):
        assert abs(h["mean"] - m0) <= 1e-6
        if k > 0:
            assert h["energy"] <= hist[k - 1]["energy"] * (1 + 1e-6)
            assert h["p1"] <= 0.0
            assert h["E1"] >= vol
    assert s.status() & ~8 == 0
    s.close()
    a = _solver(n, L, phi0, precision="fp32", history=8)
    b = _solver(n, L, phi0, precision="fp64", history=8)
    a.step(0.005, 5)
    b.step(0.005, 5)
    pa, pb = a.phi().cpu().numpy(), b.phi().cpu().numpy()
    rel = np.max(np.abs(pa - pb)) / np.max(np.abs(pb))
    print(f"256^3 fp32 vs fp64 after 5 steps: rel Linf {rel:.2e}")
    assert rel <= 1e-5
    a.close()
    b.close()


def test_3d_512_fp32_largest_grid_properties():
    """The largest 3-D grid of the FP32 path, 512^3 (h = pi/8): 30 steps; mass kept to FP32
    round-off, modified energy not rising beyond FP32 noise, p1 <= 0, E_1 >= |Omega|, no flags
    other than the energy-noise one."""
    n = (512, 512, 512)
    L = (64 * math.pi,) * 3
    phi0 = noise_ic(n, -0.25, 5)
    s = _solver(n, L, phi0, precision="fp32", history=31)
    del phi0
    s.step(0.005, 30)
    hist = s.history(0, 31)
    vol = (64 * math.pi) ** 3
    m0 = hist[0]["mean"]
    for k, h in enumerate(hist):
        assert abs(h["mean"] - m0) <= 1e-6
        if k > 0:
            assert h["energy"] <= hist[k - 1]["energy"] * (1 + 1e-6)
            assert h["p1"] <= 0.0
            assert h["E1"] >= vol
    assert s.status() & ~8 == 0
    s.close()


def test_recovery_from_a_poisoned_state():
    """Failure detection and recovery: a checkpoint is taken, a NaN is planted in one entry
    of a copy of it (from the host, in the saved spectrum), loading that copy and stepping
    sets NONFINITE; loading the good checkpoint clears the state (its flags are the saved
    ones) and the run continues with a smaller dt (restart at the change) exactly as an
    uninterrupted run from the checkpoint does."""
    import torch
    from paper_2012_15133_amd import binding as B
    n, L = (32, 32), (4 * math.pi,) * 2
    phi0 = noise_ic((32, 32), -0.2, 8)
    s = _solver(n, L, phi0, history=64)
    s.step(0.01, 20)
    good = s.save_state().clone()
    bad = good.clone()
    # the checkpoint is an aligned header and two aligned half spectra (17 x 32 complex FP64
    # each here); poison entry 5 of the newest one
    F = 17 * 32 * 16
    off = good.numel() - 2 * ((F + 255) // 256 * 256)
    bad[off + 5 * 16: off + 5 * 16 + 8] = torch.tensor([float("nan")], dtype=torch.float64).view(torch.uint8).to("cuda")
    s.load_state(bad)
    s.step(0.01, 2)
    assert s.status() & B.SPFC_FLAG_NONFINITE
    s.load_state(good)
    assert s.status() == 0
    s.step(0.005, 10)
    ref = _solver(n, L, phi0, history=64)
    ref.load_state(good)
    ref.step(0.005, 10)
    assert s.status() == 0 and s.step_count() == ref.step_count() == 30
    assert torch.equal(s.phi(), ref.phi())
    s.close()
    ref.close()


def test_launch_blocking_debug_mode_gives_the_same_bits():
    """HIP_LAUNCH_BLOCKING=1 (every launch synchronous, so an error is reported by the
    launch that caused it; each launch's status is checked by the library) changes timing
    only: a run in a child process under it equals the normal run bit for bit."""
    import subprocess
    import sys
    code = ("import sys, math, hashlib; sys.path.insert(0, %r)\n"
            "from paper_2012_15133_amd import Solver\n"
            "from paper_2012_15133_amd.inputs import noise_ic\n"
            "s = Solver((64, 64), (8 * math.pi,) * 2, noise_ic((64, 64), -0.2, 1), 0.25)\n"
            "s.step(0.01, 30)\n"
            "print(hashlib.sha256(s.phi().cpu().numpy().tobytes()).hexdigest())\n") % ROOT
    outs = []
    for blocking in ("0", "1"):
        env = dict(os.environ, HIP_LAUNCH_BLOCKING=blocking)
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=240)
        assert r.returncode == 0, r.stderr[-2000:]
        outs.append(r.stdout.strip().splitlines()[-1])
    assert outs[0] == outs[1]
