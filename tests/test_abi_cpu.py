"""Host-side checks of the HIP library that need no GPU: it loads, it exports every
function include/spfc.h declares, argument validation and workspace sizing, and
the line-FFT schedule of the kernels run thread by thread on the host."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spfc.h")
LIB = os.path.join(ROOT, "paper_2012_15133_amd", "libspfc.so")


def _lib():
    if not os.path.exists(LIB):
        from paper_2012_15133_amd import build as B
        B.build()
    from paper_2012_15133_amd import binding
    return binding


def test_header_declares_and_library_exports_all():
    decl = set(re.findall(r"\b(spfc_[a-z_]+)\s*\(", open(HEADER).read()))
    decl -= {"spfc_ctx"}
    B = _lib()
    assert set(B.EXPORTS) == decl
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (spfc_[a-z_]+)", out))
    assert decl <= exported, decl - exported
    lib = B.load_library()
    for name in decl:
        assert getattr(lib, name) is not None


def test_workspace_and_validation():
    B = _lib()
    g = B.make_grid((1024, 1024), (128 * np.pi,) * 2)
    p = B.make_params(0.25)
    n64 = B.spfc_workspace_bytes(g, p)
    n32 = B.spfc_workspace_bytes(g, B.make_params(0.25, precision="fp32"))
    F = 513 * 1024 * 16
    assert 9 * F <= n64 < 9 * F + 4 * 2 ** 20
    assert n32 < n64
    bad = [
        (B.make_grid((100, 64), (1, 1)), p),
        (B.make_grid((4, 64), (1, 1)), p),
        (B.make_grid((2048, 64), (1, 1)), p),
        (B.make_grid((64, 64), (0.0, 1)), p),
        (B.make_grid((64, 64), (float("nan"), 1)), p),
        (g, B.make_params(1.0)),
        (g, B.make_params(0.25, c4=0.0)),
        (g, B.make_params(0.25, startup=7)),
        (g, B.make_params(0.25, precision=5)),
        (g, B.make_params(0.25, history=0)),
        (g, B.make_params(0.25, stab=-1.0)),
        (g, B.make_params(0.25, stab=float("inf"))),
        (g, B.make_params(0.25, beta=-0.5)),
        (g, B.make_params(0.25, beta=float("nan"))),
    ]
    for gg, pp in bad:
        with pytest.raises(B.SpfcError) as ei:
            B.spfc_workspace_bytes(gg, pp)
        assert ei.value.status == B.SPFC_E_INVAL


def test_init_rejects_null_pointers_without_touching_the_device():
    B = _lib()
    lib = B.load_library()
    g = B.make_grid((64, 64), (1.0, 1.0))
    p = B.make_params(0.25)
    ctx = ctypes.c_void_p()
    assert lib.spfc_init(ctypes.byref(g), ctypes.byref(p), None, None, 0, None, ctypes.byref(ctx)) == B.SPFC_E_INVAL
    assert lib.spfc_init(None, ctypes.byref(p), 1, 256, 1 << 30, None, ctypes.byref(ctx)) == B.SPFC_E_INVAL
    # misaligned workspace
    assert lib.spfc_init(ctypes.byref(g), ctypes.byref(p), 256, 257, 1 << 30, None,
                         ctypes.byref(ctx)) == B.SPFC_E_INVAL
    assert lib.spfc_step(None, 0.01, 1) == B.SPFC_E_INVAL
    assert lib.spfc_destroy(None) == B.SPFC_E_INVAL
    for code in range(6):
        assert B.strerror(code)


def test_batch_workspace_and_validation():
    """Batch sizing: one class per (grid sizes, precision); a class of M members needs
    M times the per-member fields plus one twiddle table; shared run settings only."""
    B = _lib()
    g = B.make_grid((256, 256), (64 * np.pi,) * 2)
    g2 = B.make_grid((256, 256), (70.0, 60.0))
    g3 = B.make_grid((128, 128), (32 * np.pi,) * 2)
    p = B.make_params(0.25, history=64)
    q = B.make_params(0.4, history=64)
    one = B.spfc_workspace_bytes(g, p)
    four = B.spfc_batch_workspace_bytes([g, g2, g, g2], [p, q, q, p])
    F = 129 * 256 * 16
    assert 4 * 9 * F <= four < 4 * one
    assert B.spfc_batch_workspace_bytes([g], [p]) == one
    mixed = B.spfc_batch_workspace_bytes([g, g3, g], [p, p, q])
    assert mixed == B.spfc_batch_workspace_bytes([g, g], [p, q]) + B.spfc_workspace_bytes(g3, p)
    # the fp32 members of the same size are a class of their own
    p32 = B.make_params(0.25, precision="fp32", history=64)
    assert B.spfc_batch_workspace_bytes([g, g], [p, p32]) == one + B.spfc_workspace_bytes(g, p32)
    for grids, params in [([g, g], [p, B.make_params(0.25, startup="ghost", history=64)]),
                          ([g, g], [p, B.make_params(0.25, history=65)]),
                          ([g, B.make_grid((100, 64), (1, 1))], [p, p]),
                          ([g], [B.make_params(1.5, history=64)])]:
        with pytest.raises(B.SpfcError) as ei:
            B.spfc_batch_workspace_bytes(grids, params)
        assert ei.value.status == B.SPFC_E_INVAL
    lib = B.load_library()
    out = ctypes.c_size_t()
    assert lib.spfc_batch_workspace_bytes(0, None, None, ctypes.byref(out)) == B.SPFC_E_INVAL
    bh = ctypes.c_void_p()
    ga, pa = B._arrays([g, g], [p, p])
    assert lib.spfc_batch_init(2, ga, pa, None, 256, 1 << 30, None, ctypes.byref(bh)) == B.SPFC_E_INVAL
    ptrs = (ctypes.c_void_p * 2)(256, 512)
    assert lib.spfc_batch_init(2, ga, pa, ptrs, 257, 1 << 30, None, ctypes.byref(bh)) == B.SPFC_E_INVAL
    assert lib.spfc_batch_init(2, ga, pa, ptrs, 256, 1024, None, ctypes.byref(bh)) == B.SPFC_E_NOMEM
    assert lib.spfc_batch_step(None, 0.01, 1) == B.SPFC_E_INVAL
    assert lib.spfc_batch_destroy(None) == B.SPFC_E_INVAL
    assert lib.spfc_set_graph(None, 1) == B.SPFC_E_INVAL
    rec = (B.spfc_record * 1)()
    assert lib.spfc_batch_history(None, 0, 0, 1, rec) == B.SPFC_E_INVAL


# ----------------------------------------------------------------- line FFT schedule on the host

def _emu():
    from paper_2012_15133_amd import build as B
    path = os.path.join(ROOT, "_build", "libfft_emul.so")
    if not os.path.exists(path):
        path = B.build_emulator()
    lib = ctypes.CDLL(path)
    lib.emu_fft_lines.argtypes = [ctypes.c_int] * 5 + [ctypes.c_void_p] * 2
    return lib


@pytest.mark.parametrize("e", [16, 8, 4])
@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("n", [8, 16, 32, 64, 128, 256, 512, 1024])
def test_line_fft_schedule_matches_dft(fp32, n, e):
    """The Stockham schedule of the kernels (fft_core.hpp), run thread by thread on the
    host, against the DFT definition evaluated by matrix product."""
    lib = _emu()
    rng = np.random.default_rng(n + fp32)
    j = np.arange(n)
    for sign in (-1, 1):
        W = np.exp(sign * 2j * np.pi * (np.outer(j, j) % n) / n)
        for c in (1, 3):
            x = rng.standard_normal((c, n)) + 1j * rng.standard_normal((c, n))
            out = np.zeros((c, n), complex)
            assert lib.emu_fft_lines(fp32, n, e, sign, c, np.ascontiguousarray(x).ctypes.data,
                                     out.ctypes.data) == 0
            ref = x @ W.T
            err = np.max(np.abs(out - ref)) / np.max(np.abs(ref))
            # FFT rounding grows like u log2(n) (u the unit roundoff; twiddles taken as powers
            # of a table entry add a few u each): measured up to 1.1 u log2(n) in both precisions
            bound = 8 * 2.0 ** -24 * np.log2(n) if fp32 else 2e-15 * np.log2(n)
            assert err <= bound, (n, sign, c, err)


def test_fno_header_declares_and_library_exports_all():
    header = os.path.join(ROOT, "include", "spfc_fno.h")
    decl = set(re.findall(r"\b(spfc_fno_[a-z_]+)\s*\(", open(header).read()))
    _lib()
    from paper_2012_15133_amd import surrogate as S
    assert set(S.EXPORTS) == decl
    lib = os.path.join(ROOT, "paper_2012_15133_amd", "libspfc_fno.so")
    out = subprocess.run(["nm", "-D", "--defined-only", lib], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (spfc_fno_[a-z_]+)", out))
    assert decl <= exported, decl - exported


def test_fno_sizes_and_validation_without_a_device():
    _lib()
    from paper_2012_15133_amd import surrogate as S
    assert S.spfc_fno_param_count() == sum(int(np.prod(s)) for _, s in S.param_layout()) == 4200801
    small = S.spfc_fno_workspace_bytes(S.spfc_fno_shape(64, 4, 0))
    train = S.spfc_fno_workspace_bytes(S.spfc_fno_shape(64, 4, 1))
    big = S.spfc_fno_workspace_bytes(S.spfc_fno_shape(256, 64, 1))
    assert small < train < big
    lib = S.load_library()
    n = ctypes.c_size_t()
    for bad in ((100, 4, 0), (64, 0, 0), (64, 129, 0), (64, 4, 2), (512, 4, 0)):
        assert lib.spfc_fno_workspace_bytes(ctypes.byref(S.spfc_fno_shape(*bad)), ctypes.byref(n)) == 1
    h = ctypes.c_void_p()
    assert lib.spfc_fno_init(ctypes.byref(S.spfc_fno_shape(64, 4, 0)), None, 256, 1 << 30, None,
                             ctypes.byref(h)) == 1
    assert lib.spfc_fno_init(ctypes.byref(S.spfc_fno_shape(64, 4, 0)), 256, 257, 1 << 30, None,
                             ctypes.byref(h)) == 1
    assert lib.spfc_fno_init(ctypes.byref(S.spfc_fno_shape(64, 4, 0)), 256, 256, 1024, None,
                             ctypes.byref(h)) == 2
    assert lib.spfc_fno_forward(None, 1, 256, 256, 256) == 1
    assert lib.spfc_fno_destroy(None) == 1


def test_noalloc_limits_and_refusals_without_a_device():
    """The allocation-free run's array holds the grids its header names, and the call refuses
    bad arguments and grids beyond the array before it makes any device call."""
    B = _lib()
    lib = B.load_library()
    fits = [((1024, 512), "fp64"), ((1024, 1024), "fp32"), ((128, 128, 64), "fp32")]
    for n, prec in fits:
        g = B.make_grid(n, (10.0,) * len(n))
        assert B.spfc_workspace_bytes(g, B.make_params(0.25, precision=prec)) <= B.SPFC_NOALLOC_BYTES, n
    big = B.make_grid((1024, 1024), (10.0, 10.0))
    p64 = B.make_params(0.25)
    assert B.spfc_workspace_bytes(big, p64) > B.SPFC_NOALLOC_BYTES
    e = B.spfc_energy_t()
    fake = ctypes.c_void_p(256)   # never dereferenced: every case below is refused first
    st = lib.spfc_run_noalloc(ctypes.byref(big), ctypes.byref(p64), fake, 0.01, 1, fake, B.SPFC_FP64, ctypes.byref(e),
                              None)
    assert st == B.SPFC_E_NOMEM
    small = B.make_grid((64, 64), (10.0, 10.0))
    for args in [(small, p64, None, 0.01, 1, fake, B.SPFC_FP64), (small, p64, fake, 0.0, 1, fake, B.SPFC_FP64),
                 (small, p64, fake, 0.01, -1, fake, B.SPFC_FP64), (small, p64, fake, 0.01, 1, None, B.SPFC_FP64),
                 (small, p64, fake, 0.01, 1, fake, 7), (B.make_grid((100, 64), (1, 1)), p64, fake, 0.01, 1, fake, 0)]:
        g, p, phi, dt, n, out, dtype = args
        assert lib.spfc_run_noalloc(ctypes.byref(g), ctypes.byref(p), phi, dt, n, out, dtype, ctypes.byref(e),
                                    None) == B.SPFC_E_INVAL
