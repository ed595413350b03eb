"""The allocation-free run (spfc_run_noalloc, through the C ABI) against the same run
through spfc_init + spfc_step + spfc_get_phi + spfc_energy on a caller workspace: the
same kernels and plan, so the same bits.  Two calls in a row, the second on a smaller
grid (the library's array keeps the first call's contents), then a grid too large for
the array, which must be refused."""

import ctypes
import math

import numpy as np
import pytest
import torch

from paper_2012_15133_amd import binding as B
from paper_2012_15133_amd.inputs import noise_ic

pytestmark = pytest.mark.gpu


def _reference(n, L, phi0, eps, dt, steps, precision):
    s = B.Solver(n, L, phi0, eps, precision=precision, history=64)
    s.step(dt, steps)
    e = s.energy()
    phi = s.phi()
    s.close()
    return phi, e


def _noalloc(n, L, phi0, eps, dt, steps, precision):
    grid = B.make_grid(n, L)
    prm = B.make_params(eps, precision=precision, history=64)
    p0 = torch.from_numpy(np.ascontiguousarray(phi0)).to("cuda")
    out = torch.empty_like(p0)
    stream = torch.cuda.current_stream()
    e = B.spfc_run_noalloc(grid, prm, p0.data_ptr(), dt, steps, out.data_ptr(), B.SPFC_FP64, stream.cuda_stream)
    return out, e


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_equals_workspace_run_twice_then_smaller(precision):
    cases = [((256, 128), 0.01, 30, 21), ((64, 64), 0.01, 45, 22), ((16, 32, 16), 0.005, 12, 23)]
    for n, dt, steps, seed in cases:
        L = tuple(v * math.pi / 8 for v in n)
        phi0 = noise_ic(tuple(reversed(n)), -0.2, seed)
        ref_phi, ref_e = _reference(n, L, phi0, 0.25, dt, steps, precision)
        got_phi, got_e = _noalloc(n, L, phi0, 0.25, dt, steps, precision)
        assert torch.equal(got_phi, ref_phi), (n, precision)
        assert got_e == ref_e, (n, precision, got_e, ref_e)
        assert got_e["step"] == steps


def test_noalloc_refuses_grids_beyond_its_array():
    n = (1024, 1024)
    grid = B.make_grid(n, (128 * math.pi,) * 2)
    prm = B.make_params(0.25, precision="fp64", history=64)
    assert B.spfc_workspace_bytes(grid, prm) > B.SPFC_NOALLOC_BYTES
    p0 = torch.zeros((1024, 1024), dtype=torch.float64, device="cuda")
    out = torch.empty_like(p0)
    with pytest.raises(B.SpfcError) as ei:
        B.spfc_run_noalloc(grid, prm, p0.data_ptr(), 0.01, 1, out.data_ptr(), B.SPFC_FP64, 0)
    assert ei.value.status == B.SPFC_E_NOMEM
    # a bad argument is refused before any work
    small = B.make_grid((64, 64), (8 * math.pi,) * 2)
    with pytest.raises(B.SpfcError):
        B.spfc_run_noalloc(small, prm, p0.data_ptr(), -1.0, 1, out.data_ptr(), B.SPFC_FP64, 0)
