"""ctypes binding of libspfc.so (include/spfc.h): the C ABI calls under the same
names, plus a small `Solver` class that takes device memory and the stream from
PyTorch.  Argument marshalling only: every step of the method runs in the HIP
kernels of the library.  There is no fallback: if the library is missing the
calls raise.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SPFC_LIB", os.path.join(HERE, "libspfc.so"))

SPFC_OK, SPFC_E_INVAL, SPFC_E_NOMEM, SPFC_E_DEVICE, SPFC_E_NONFINITE, SPFC_E_STATE = range(6)
SPFC_FLAG_NONFINITE, SPFC_FLAG_E1_BELOW_OMEGA, SPFC_FLAG_P1_POSITIVE, SPFC_FLAG_ENERGY_RISE = 1, 2, 4, 8
SPFC_STARTUP_SAV1, SPFC_STARTUP_GHOST, SPFC_STARTUP_COPY = 0, 1, 2
SPFC_FP64, SPFC_FP32 = 0, 1
STARTUPS = {"sav1": SPFC_STARTUP_SAV1, "ghost": SPFC_STARTUP_GHOST, "copy": SPFC_STARTUP_COPY}
PRECISIONS = {"fp64": SPFC_FP64, "fp32": SPFC_FP32}

EXPORTS = [
    "spfc_workspace_bytes", "spfc_init", "spfc_step", "spfc_mass", "spfc_energy", "spfc_history",
    "spfc_step_count", "spfc_get_phi", "spfc_state_bytes", "spfc_save_state", "spfc_load_state",
    "spfc_status", "spfc_profile", "spfc_kernel_times", "spfc_strerror", "spfc_destroy", "spfc_set_graph",
    "spfc_batch_workspace_bytes", "spfc_batch_init", "spfc_batch_step", "spfc_batch_set_graph",
    "spfc_batch_step_count", "spfc_batch_status", "spfc_batch_mass", "spfc_batch_energy", "spfc_batch_history",
    "spfc_batch_get_phi", "spfc_batch_destroy", "spfc_batch_profile", "spfc_batch_kernel_times",
    "spfc_tune_bytes", "spfc_tune", "spfc_get_plan", "spfc_batch_tune_bytes", "spfc_batch_tune",
    "spfc_batch_get_plan", "spfc_time_kernels", "spfc_batch_time_kernels", "spfc_batch_reset",
    "spfc_batch_energies", "spfc_batch_get_phi_all", "spfc_forcing_bytes", "spfc_set_forcing",
    "spfc_step_forced", "spfc_run_noalloc",
]

SPFC_NOALLOC_BYTES = 64 << 20


class spfc_grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("L", ctypes.c_double * 3)]


class spfc_params(ctypes.Structure):
    _fields_ = [("epsilon", ctypes.c_double), ("c4", ctypes.c_double), ("startup", ctypes.c_int),
                ("precision", ctypes.c_int), ("history", ctypes.c_int64), ("energy_tol", ctypes.c_double),
                ("stab", ctypes.c_double), ("beta", ctypes.c_double)]


class spfc_record(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("energy", "mean", "r", "xi", "E1", "p1", "S", "reserved")]


class spfc_energy_t(ctypes.Structure):
    _fields_ = [("modified_energy", ctypes.c_double), ("energy", ctypes.c_double),
                ("sav_energy", ctypes.c_double), ("r", ctypes.c_double), ("E1", ctypes.c_double),
                ("mean", ctypes.c_double), ("step", ctypes.c_int64)]


class SpfcError(RuntimeError):
    def __init__(self, call, status):
        self.status = status
        super().__init__(f"{call} failed: {status} ({strerror(status)})")


_lib = None


def load_library(path: str | None = None):
    """Load libspfc.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library not built: {p} is missing (run python -m paper_2012_15133_amd.build)")
    lib = ctypes.CDLL(p)
    vp, sz, i64, dbl, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    P = ctypes.POINTER
    sig = {
        "spfc_workspace_bytes": [P(spfc_grid), P(spfc_params), P(sz)],
        "spfc_init": [P(spfc_grid), P(spfc_params), vp, vp, sz, vp, P(vp)],
        "spfc_step": [vp, dbl, i64],
        "spfc_forcing_bytes": [vp, i32, P(sz)],
        "spfc_set_forcing": [vp, i32, P(vp), vp, sz],
        "spfc_step_forced": [vp, dbl, i64, vp],
        "spfc_mass": [vp, P(dbl)],
        "spfc_energy": [vp, P(spfc_energy_t)],
        "spfc_history": [vp, i64, i64, P(spfc_record)],
        "spfc_step_count": [vp, P(i64)],
        "spfc_get_phi": [vp, vp, i32],
        "spfc_state_bytes": [vp, P(sz)],
        "spfc_save_state": [vp, vp, sz],
        "spfc_load_state": [vp, vp, sz],
        "spfc_status": [vp, P(ctypes.c_uint32)],
        "spfc_profile": [vp, i32],
        "spfc_kernel_times": [vp, i32, P(ctypes.c_char_p), P(dbl), P(i64), P(dbl), P(i32)],
        "spfc_destroy": [vp],
        "spfc_set_graph": [vp, i32],
        "spfc_batch_workspace_bytes": [i32, P(spfc_grid), P(spfc_params), P(sz)],
        "spfc_batch_init": [i32, P(spfc_grid), P(spfc_params), P(vp), vp, sz, vp, P(vp)],
        "spfc_batch_step": [vp, dbl, i64],
        "spfc_batch_set_graph": [vp, i32],
        "spfc_batch_step_count": [vp, P(i64)],
        "spfc_batch_status": [vp, i32, P(ctypes.c_uint32)],
        "spfc_batch_mass": [vp, i32, P(dbl)],
        "spfc_batch_energy": [vp, i32, P(spfc_energy_t)],
        "spfc_batch_history": [vp, i32, i64, i64, P(spfc_record)],
        "spfc_batch_get_phi": [vp, i32, vp, i32],
        "spfc_batch_destroy": [vp],
        "spfc_batch_profile": [vp, i32],
        "spfc_tune_bytes": [vp, P(sz)],
        "spfc_tune": [vp, dbl, i64, vp, sz],
        "spfc_get_plan": [vp, P(i32)],
        "spfc_batch_tune_bytes": [vp, P(sz)],
        "spfc_batch_tune": [vp, dbl, i64, vp, sz],
        "spfc_batch_get_plan": [vp, i32, P(i32)],
        "spfc_time_kernels": [vp, dbl, i32, vp, sz],
        "spfc_batch_time_kernels": [vp, dbl, i32, vp, sz],
        "spfc_batch_reset": [vp, P(vp), P(dbl)],
        "spfc_batch_energies": [vp, P(spfc_energy_t)],
        "spfc_batch_get_phi_all": [vp, P(vp), i32],
        "spfc_batch_kernel_times": [vp, i32, P(ctypes.c_char_p), P(dbl), P(i64), P(dbl), P(i32)],
        "spfc_run_noalloc": [P(spfc_grid), P(spfc_params), vp, dbl, i64, vp, i32, P(spfc_energy_t), vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.spfc_strerror.argtypes = [ctypes.c_int]
    lib.spfc_strerror.restype = ctypes.c_char_p
    if path is None:
        _lib = lib
    return lib


def strerror(status: int) -> str:
    try:
        return load_library().spfc_strerror(int(status)).decode()
    except RuntimeError:
        return f"status {status}"


def _check(call, status):
    if status != SPFC_OK:
        raise SpfcError(call, status)


def make_grid(n, L) -> spfc_grid:
    n = list(n)
    L = list(L)
    g = spfc_grid()
    g.dim = len(n)
    for j in range(3):
        g.n[j] = int(n[j]) if j < len(n) else 1
        g.L[j] = float(L[j]) if j < len(L) else 1.0
    return g


def make_params(epsilon, c4=1.0, startup="sav1", precision="fp64", history=4096, energy_tol=0.0,
                stab=0.0, beta=0.0) -> spfc_params:
    p = spfc_params()
    p.stab = float(stab)
    p.beta = float(beta)
    p.epsilon = float(epsilon)
    p.c4 = float(c4)
    p.startup = STARTUPS[startup] if isinstance(startup, str) else int(startup)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.history = int(history)
    p.energy_tol = float(energy_tol)
    return p


# ------------------------------------------------------------------ thin wrappers, same names as the ABI

def spfc_workspace_bytes(grid: spfc_grid, params: spfc_params) -> int:
    out = ctypes.c_size_t(0)
    _check("spfc_workspace_bytes", load_library().spfc_workspace_bytes(ctypes.byref(grid), ctypes.byref(params),
                                                                       ctypes.byref(out)))
    return out.value


def spfc_init(grid, params, phi0_ptr: int, workspace_ptr: int, workspace_bytes: int, stream_ptr: int):
    ctx = ctypes.c_void_p()
    _check("spfc_init", load_library().spfc_init(ctypes.byref(grid), ctypes.byref(params), phi0_ptr, workspace_ptr,
                                                 workspace_bytes, stream_ptr, ctypes.byref(ctx)))
    return ctx


def spfc_step(ctx, dt: float, n: int):
    _check("spfc_step", load_library().spfc_step(ctx, float(dt), int(n)))


def spfc_forcing_bytes(ctx, terms: int) -> int:
    n = ctypes.c_size_t()
    _check("spfc_forcing_bytes", load_library().spfc_forcing_bytes(ctx, int(terms), ctypes.byref(n)))
    return n.value


def spfc_set_forcing(ctx, terms: int, field_ptrs, buf_ptr: int, buf_bytes: int):
    ptrs = (ctypes.c_void_p * max(1, len(field_ptrs)))(*field_ptrs) if field_ptrs else None
    _check("spfc_set_forcing", load_library().spfc_set_forcing(ctx, int(terms), ptrs, buf_ptr, int(buf_bytes)))


def spfc_step_forced(ctx, dt: float, n: int, coef_ptr: int):
    _check("spfc_step_forced", load_library().spfc_step_forced(ctx, float(dt), int(n), coef_ptr))


def spfc_mass(ctx) -> float:
    m = ctypes.c_double()
    _check("spfc_mass", load_library().spfc_mass(ctx, ctypes.byref(m)))
    return m.value


def spfc_energy(ctx, allow_nonfinite: bool = False) -> dict:
    e = spfc_energy_t()
    st = load_library().spfc_energy(ctx, ctypes.byref(e))
    if not (st == SPFC_OK or (allow_nonfinite and st == SPFC_E_NONFINITE)):
        _check("spfc_energy", st)
    return {k: getattr(e, k) for k, _ in spfc_energy_t._fields_}


def spfc_history(ctx, first: int, count: int) -> list:
    buf = (spfc_record * max(count, 1))()
    _check("spfc_history", load_library().spfc_history(ctx, int(first), int(count), buf))
    return _records(buf, count)


def spfc_step_count(ctx) -> int:
    n = ctypes.c_int64()
    _check("spfc_step_count", load_library().spfc_step_count(ctx, ctypes.byref(n)))
    return n.value


def spfc_get_phi(ctx, out_ptr: int, dtype: int = SPFC_FP64):
    _check("spfc_get_phi", load_library().spfc_get_phi(ctx, out_ptr, int(dtype)))


def spfc_state_bytes(ctx) -> int:
    n = ctypes.c_size_t()
    _check("spfc_state_bytes", load_library().spfc_state_bytes(ctx, ctypes.byref(n)))
    return n.value


def spfc_save_state(ctx, out_ptr: int, nbytes: int):
    _check("spfc_save_state", load_library().spfc_save_state(ctx, out_ptr, int(nbytes)))


def spfc_load_state(ctx, in_ptr: int, nbytes: int):
    _check("spfc_load_state", load_library().spfc_load_state(ctx, in_ptr, int(nbytes)))


def spfc_status(ctx) -> int:
    f = ctypes.c_uint32()
    _check("spfc_status", load_library().spfc_status(ctx, ctypes.byref(f)))
    return f.value


def spfc_profile(ctx, enable: bool):
    _check("spfc_profile", load_library().spfc_profile(ctx, 1 if enable else 0))


def _kernel_times(call, handle) -> list:
    cap = 8
    names = (ctypes.c_char_p * cap)()
    avg = (ctypes.c_double * cap)()
    nl = (ctypes.c_int64 * cap)()
    by = (ctypes.c_double * cap)()
    cnt = ctypes.c_int()
    _check(call, getattr(load_library(), call)(handle, cap, names, avg, nl, by, ctypes.byref(cnt)))
    return [{"name": names[i].decode(), "avg_ms": avg[i], "launches": nl[i], "bytes": by[i]}
            for i in range(min(cnt.value, cap))]


def spfc_kernel_times(ctx) -> list:
    return _kernel_times("spfc_kernel_times", ctx)


def spfc_strerror(status: int) -> str:
    return strerror(status)


def spfc_destroy(ctx):
    _check("spfc_destroy", load_library().spfc_destroy(ctx))


def spfc_set_graph(ctx, enable: bool):
    _check("spfc_set_graph", load_library().spfc_set_graph(ctx, 1 if enable else 0))


def _records(buf, count):
    return [{k: getattr(buf[i], k) for k, _ in spfc_record._fields_ if k != "reserved"} for i in range(count)]


def _arrays(grids, params):
    ga = (spfc_grid * len(grids))(*grids)
    pa = (spfc_params * len(params))(*params)
    return ga, pa


def spfc_batch_workspace_bytes(grids, params) -> int:
    ga, pa = _arrays(grids, params)
    out = ctypes.c_size_t(0)
    _check("spfc_batch_workspace_bytes", load_library().spfc_batch_workspace_bytes(len(grids), ga, pa,
                                                                                   ctypes.byref(out)))
    return out.value


def spfc_batch_init(grids, params, phi0_ptrs, workspace_ptr: int, workspace_bytes: int, stream_ptr: int):
    ga, pa = _arrays(grids, params)
    ptrs = (ctypes.c_void_p * len(phi0_ptrs))(*phi0_ptrs)
    b = ctypes.c_void_p()
    _check("spfc_batch_init", load_library().spfc_batch_init(len(grids), ga, pa, ptrs, workspace_ptr,
                                                             workspace_bytes, stream_ptr, ctypes.byref(b)))
    return b


def spfc_batch_step(b, dt: float, n: int):
    _check("spfc_batch_step", load_library().spfc_batch_step(b, float(dt), int(n)))


def spfc_batch_set_graph(b, enable: bool):
    _check("spfc_batch_set_graph", load_library().spfc_batch_set_graph(b, 1 if enable else 0))


def spfc_batch_step_count(b) -> int:
    n = ctypes.c_int64()
    _check("spfc_batch_step_count", load_library().spfc_batch_step_count(b, ctypes.byref(n)))
    return n.value


def spfc_batch_status(b, member: int) -> int:
    f = ctypes.c_uint32()
    _check("spfc_batch_status", load_library().spfc_batch_status(b, int(member), ctypes.byref(f)))
    return f.value


def spfc_batch_mass(b, member: int) -> float:
    m = ctypes.c_double()
    _check("spfc_batch_mass", load_library().spfc_batch_mass(b, int(member), ctypes.byref(m)))
    return m.value


def spfc_batch_energy(b, member: int, allow_nonfinite: bool = False) -> dict:
    e = spfc_energy_t()
    st = load_library().spfc_batch_energy(b, int(member), ctypes.byref(e))
    if not (st == SPFC_OK or (allow_nonfinite and st == SPFC_E_NONFINITE)):
        _check("spfc_batch_energy", st)
    return {k: getattr(e, k) for k, _ in spfc_energy_t._fields_}


def spfc_batch_history(b, member: int, first: int, count: int) -> list:
    buf = (spfc_record * max(count, 1))()
    _check("spfc_batch_history", load_library().spfc_batch_history(b, int(member), int(first), int(count), buf))
    return _records(buf, count)


def spfc_batch_get_phi(b, member: int, out_ptr: int, dtype: int = SPFC_FP64):
    _check("spfc_batch_get_phi", load_library().spfc_batch_get_phi(b, int(member), out_ptr, int(dtype)))


def spfc_tune_bytes(ctx) -> int:
    n = ctypes.c_size_t()
    _check("spfc_tune_bytes", load_library().spfc_tune_bytes(ctx, ctypes.byref(n)))
    return n.value


def spfc_tune(ctx, dt: float, trial_steps: int, scratch_ptr: int, scratch_bytes: int):
    _check("spfc_tune", load_library().spfc_tune(ctx, float(dt), int(trial_steps), scratch_ptr, int(scratch_bytes)))


def spfc_time_kernels(ctx, dt: float, reps: int, scratch_ptr: int, scratch_bytes: int):
    _check("spfc_time_kernels", load_library().spfc_time_kernels(ctx, float(dt), int(reps), scratch_ptr,
                                                                 int(scratch_bytes)))


def spfc_batch_time_kernels(b, dt: float, reps: int, scratch_ptr: int, scratch_bytes: int):
    _check("spfc_batch_time_kernels", load_library().spfc_batch_time_kernels(b, float(dt), int(reps), scratch_ptr,
                                                                             int(scratch_bytes)))


def _plan(arr):
    keys = ("inv", "real", "fwd", "mid")
    return {k: (arr[2 * i], arr[2 * i + 1]) for i, k in enumerate(keys) if arr[2 * i]}


def spfc_get_plan(ctx) -> dict:
    arr = (ctypes.c_int * 8)()
    _check("spfc_get_plan", load_library().spfc_get_plan(ctx, arr))
    return _plan(arr)


def spfc_batch_tune_bytes(b) -> int:
    n = ctypes.c_size_t()
    _check("spfc_batch_tune_bytes", load_library().spfc_batch_tune_bytes(b, ctypes.byref(n)))
    return n.value


def spfc_batch_tune(b, dt: float, trial_steps: int, scratch_ptr: int, scratch_bytes: int):
    _check("spfc_batch_tune", load_library().spfc_batch_tune(b, float(dt), int(trial_steps), scratch_ptr,
                                                             int(scratch_bytes)))


def spfc_batch_get_plan(b, member: int) -> dict:
    arr = (ctypes.c_int * 8)()
    _check("spfc_batch_get_plan", load_library().spfc_batch_get_plan(b, int(member), arr))
    return _plan(arr)


def spfc_batch_reset(b, phi_ptrs, r_shift=None):
    ptrs = (ctypes.c_void_p * len(phi_ptrs))(*phi_ptrs)
    rr = None if r_shift is None else (ctypes.c_double * len(r_shift))(*[float(x) for x in r_shift])
    _check("spfc_batch_reset", load_library().spfc_batch_reset(b, ptrs, rr))


def spfc_batch_get_phi_all(b, out_ptrs, dtype: int = SPFC_FP64):
    ptrs = (ctypes.c_void_p * len(out_ptrs))(*out_ptrs)
    _check("spfc_batch_get_phi_all", load_library().spfc_batch_get_phi_all(b, ptrs, int(dtype)))


def spfc_batch_energies(b, count: int, allow_nonfinite: bool = False) -> list:
    buf = (spfc_energy_t * count)()
    st = load_library().spfc_batch_energies(b, buf)
    if not (st == SPFC_OK or (allow_nonfinite and st == SPFC_E_NONFINITE)):
        _check("spfc_batch_energies", st)
    return [{k: getattr(buf[i], k) for k, _ in spfc_energy_t._fields_} for i in range(count)]


def spfc_batch_profile(b, enable: bool):
    _check("spfc_batch_profile", load_library().spfc_batch_profile(b, 1 if enable else 0))


def spfc_batch_kernel_times(b) -> list:
    return _kernel_times("spfc_batch_kernel_times", b)


def spfc_batch_destroy(b):
    _check("spfc_batch_destroy", load_library().spfc_batch_destroy(b))


def spfc_run_noalloc(grid, params, phi0_ptr: int, dt: float, n: int, out_ptr: int, dtype: int = SPFC_FP64,
                     stream_ptr: int = 0) -> dict:
    """One run in the library's own per-device array (no allocation); returns the energies
    of phi^n, which is written to out_ptr."""
    e = spfc_energy_t()
    _check("spfc_run_noalloc", load_library().spfc_run_noalloc(ctypes.byref(grid), ctypes.byref(params), phi0_ptr,
                                                               float(dt), int(n), out_ptr, int(dtype),
                                                               ctypes.byref(e), stream_ptr))
    return {k: getattr(e, k) for k, _ in spfc_energy_t._fields_}


# ------------------------------------------------------------------ convenience class (PyTorch memory + stream)

def _stream_for(torch, stream, graph):
    """The caller's stream, else a new one when graphs are wanted (they cannot be
    captured on the null stream), else the current stream."""
    if stream is not None:
        return stream
    if graph:
        return torch.cuda.Stream()
    return torch.cuda.current_stream()


def _device_field(torch, np, phi0, shape):
    if isinstance(phi0, torch.Tensor):
        p0 = phi0.to(device="cuda", dtype=torch.float64).contiguous()
    else:
        p0 = torch.from_numpy(np.ascontiguousarray(np.asarray(phi0, dtype=np.float64))).to("cuda")
    if tuple(p0.shape) != shape:
        raise ValueError(f"phi0 shape {tuple(p0.shape)} != {shape}")
    return p0


class Solver:
    """One run on the current HIP device.  phi0: array of shape (n_y, n_x) or
    (n_z, n_y, n_x) (x fastest), copied to the device as float64."""

    def __init__(self, n, L, phi0, epsilon, c4=1.0, startup="sav1", precision="fp64", history=4096,
                 energy_tol=0.0, stream=None, graph=False, stab=0.0, beta=0.0):
        import numpy as np
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Solver needs a HIP device")
        load_library()
        self.torch = torch
        self.n = tuple(int(v) for v in n)
        self.grid = make_grid(n, L)
        self.params = make_params(epsilon, c4, startup, precision, history, energy_tol, stab, beta)
        self.stream = _stream_for(torch, stream, graph)
        nbytes = spfc_workspace_bytes(self.grid, self.params)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self._ws_bytes = nbytes
        p0 = _device_field(torch, np, phi0, tuple(reversed(self.n)))
        self.ctx = spfc_init(self.grid, self.params, p0.data_ptr(), self._ws_ptr, nbytes, self.stream.cuda_stream)
        del p0
        if graph:
            spfc_set_graph(self.ctx, True)

    def step(self, dt, n=1):
        spfc_step(self.ctx, dt, n)

    def set_forcing(self, fields):
        """f(x, t) = sum_i c_i(t) fields[i](x) from now on (fields: arrays of the grid's
        shape); an empty sequence removes the forcing."""
        import numpy as np
        torch = self.torch
        if len(fields) == 0:
            spfc_set_forcing(self.ctx, 0, [], None, 0)
            self._forcing = None
            self.forcing_terms = 0
            return
        dev = [_device_field(torch, np, f, tuple(reversed(self.n))) for f in fields]
        nb = spfc_forcing_bytes(self.ctx, len(dev))
        buf = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
        ptr = (buf.data_ptr() + 255) // 256 * 256
        spfc_set_forcing(self.ctx, len(dev), [d.data_ptr() for d in dev], ptr, nb)
        self._forcing = buf          # kept while the forcing is in use
        self.forcing_terms = len(dev)

    def step_forced(self, dt, coef):
        """len(coef) steps of size dt; coef[s][i] = c_i at the new time level of step s."""
        import numpy as np
        if not getattr(self, "forcing_terms", 0):
            raise ValueError("no forcing set (set_forcing)")
        c = np.ascontiguousarray(np.asarray(coef, dtype=np.float64).reshape(len(coef), -1))
        if c.shape[1] != self.forcing_terms:
            raise ValueError(f"coefficients have {c.shape[1]} terms, the forcing has {self.forcing_terms}")
        dev = self.torch.from_numpy(c).to("cuda")
        spfc_step_forced(self.ctx, dt, c.shape[0], dev.data_ptr())
        self.stream.synchronize()    # the kernels read the coefficients as they run

    def energy(self):
        return spfc_energy(self.ctx)

    def mass(self):
        return spfc_mass(self.ctx)

    def history(self, first, count):
        return spfc_history(self.ctx, first, count)

    def step_count(self):
        return spfc_step_count(self.ctx)

    def status(self):
        return spfc_status(self.ctx)

    def phi(self, dtype="fp64"):
        torch = self.torch
        shape = tuple(reversed(self.n))
        out = torch.empty(shape, dtype=torch.float64 if dtype == "fp64" else torch.float32, device="cuda")
        spfc_get_phi(self.ctx, out.data_ptr(), SPFC_FP64 if dtype == "fp64" else SPFC_FP32)
        self.stream.synchronize()
        return out

    def save_state(self):
        torch = self.torch
        nb = spfc_state_bytes(self.ctx)
        buf = torch.empty(nb, dtype=torch.uint8, device="cuda")
        spfc_save_state(self.ctx, buf.data_ptr(), nb)
        return buf

    def load_state(self, buf):
        spfc_load_state(self.ctx, buf.data_ptr(), buf.numel())

    def tune(self, dt, trial_steps=20):
        """Choose the fastest launch plan for steps of size dt (the run state is kept)."""
        nb = spfc_tune_bytes(self.ctx)
        scratch = self.torch.empty(nb, dtype=self.torch.uint8, device="cuda")
        spfc_tune(self.ctx, dt, trial_steps, scratch.data_ptr(), nb)
        del scratch
        return spfc_get_plan(self.ctx)

    def plan(self):
        return spfc_get_plan(self.ctx)

    def time_kernels(self, dt, reps=20):
        """Per-launch kernel durations of a steady step (back-to-back launches; the run
        state is kept); same entries as kernel_times()."""
        nb = spfc_tune_bytes(self.ctx)
        scratch = self.torch.empty(nb, dtype=self.torch.uint8, device="cuda")
        spfc_time_kernels(self.ctx, dt, reps, scratch.data_ptr(), nb)
        del scratch
        return spfc_kernel_times(self.ctx)

    def profile(self, enable=True):
        spfc_profile(self.ctx, enable)

    def kernel_times(self):
        return spfc_kernel_times(self.ctx)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            spfc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent runs advanced together on the current HIP device.  members: list of
    dicts with keys n, L, phi0, epsilon and optionally c4, stab, beta and precision; startup,
    history and energy_tol are shared."""

    def __init__(self, members, startup="sav1", history=4096, energy_tol=0.0, stream=None, graph=False):
        import numpy as np
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Batch needs a HIP device")
        load_library()
        self.torch = torch
        self.ns = [tuple(int(v) for v in m["n"]) for m in members]
        self.precisions = [m.get("precision", "fp64") for m in members]
        grids = [make_grid(m["n"], m["L"]) for m in members]
        params = [make_params(m["epsilon"], m.get("c4", 1.0), startup, m.get("precision", "fp64"), history,
                              energy_tol, m.get("stab", 0.0), m.get("beta", 0.0)) for m in members]
        self.stream = _stream_for(torch, stream, graph)
        nbytes = spfc_batch_workspace_bytes(grids, params)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        ws = (self.workspace.data_ptr() + 255) // 256 * 256
        fields = [_device_field(torch, np, m["phi0"], tuple(reversed(n))) for m, n in zip(members, self.ns)]
        self.b = spfc_batch_init(grids, params, [f.data_ptr() for f in fields], ws, nbytes,
                                 self.stream.cuda_stream)
        del fields
        if graph:
            spfc_batch_set_graph(self.b, True)

    def __len__(self):
        return len(self.ns)

    def step(self, dt, n=1):
        spfc_batch_step(self.b, dt, n)

    def step_count(self):
        return spfc_batch_step_count(self.b)

    def status(self, m):
        return spfc_batch_status(self.b, m)

    def mass(self, m):
        return spfc_batch_mass(self.b, m)

    def energy(self, m):
        return spfc_batch_energy(self.b, m)

    def history(self, m, first, count):
        return spfc_batch_history(self.b, m, first, count)

    def reset(self, fields, r_shift=None):
        """Start every member again from new fields (sequence of arrays or tensors, or one
        contiguous float64 device tensor [members, n_y, n_x] when all members have one grid
        size); the SAV variable is sqrt(E_1(field)) plus r_shift[m] when given."""
        import numpy as np
        torch = self.torch
        if isinstance(fields, torch.Tensor) and fields.is_cuda and fields.dtype == torch.float64 \
                and fields.is_contiguous() and fields.dim() == len(self.ns[0]) + 1 and fields.shape[0] == len(self.ns) \
                and all(tuple(reversed(n)) == tuple(fields.shape[1:]) for n in self.ns):
            step = fields[0].numel() * fields.element_size()
            spfc_batch_reset(self.b, [fields.data_ptr() + m * step for m in range(len(self.ns))], r_shift)
            return
        dev = [_device_field(torch, np, f, tuple(reversed(n))) for f, n in zip(fields, self.ns)]
        spfc_batch_reset(self.b, [d.data_ptr() for d in dev], r_shift)
        del dev

    def energies(self, allow_nonfinite=False):
        return spfc_batch_energies(self.b, len(self.ns), allow_nonfinite)

    def phi_all(self, out):
        """Every member's field into out[m] (float32 or float64 device tensor of shape
        [members, n_y, n_x]; all members of one grid size)."""
        dt = SPFC_FP32 if out.dtype == self.torch.float32 else SPFC_FP64
        if not out.is_contiguous() or out.shape[0] != len(self.ns):
            raise ValueError("out must be a contiguous [members, n_y, n_x] tensor")
        step = out[0].numel() * out.element_size()
        spfc_batch_get_phi_all(self.b, [out.data_ptr() + m * step for m in range(len(self.ns))], dt)
        self.stream.synchronize()
        return out

    def phi(self, m, dtype="fp64"):
        torch = self.torch
        out = torch.empty(tuple(reversed(self.ns[m])), dtype=torch.float64 if dtype == "fp64" else torch.float32,
                          device="cuda")
        spfc_batch_get_phi(self.b, m, out.data_ptr(), SPFC_FP64 if dtype == "fp64" else SPFC_FP32)
        self.stream.synchronize()
        return out

    def tune(self, dt, trial_steps=20):
        """Choose the fastest launch plan of every size class (the run state is kept)."""
        nb = spfc_batch_tune_bytes(self.b)
        scratch = self.torch.empty(nb, dtype=self.torch.uint8, device="cuda")
        spfc_batch_tune(self.b, dt, trial_steps, scratch.data_ptr(), nb)
        del scratch

    def plan(self, m):
        return spfc_batch_get_plan(self.b, m)

    def time_kernels(self, dt, reps=20):
        nb = spfc_batch_tune_bytes(self.b)
        scratch = self.torch.empty(nb, dtype=self.torch.uint8, device="cuda")
        spfc_batch_time_kernels(self.b, dt, reps, scratch.data_ptr(), nb)
        del scratch
        return spfc_batch_kernel_times(self.b)

    def profile(self, enable=True):
        spfc_batch_profile(self.b, enable)

    def kernel_times(self):
        return spfc_batch_kernel_times(self.b)

    def close(self):
        if getattr(self, "b", None) is not None:
            spfc_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
