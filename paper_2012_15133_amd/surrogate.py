"""ctypes binding of libspfc_fno.so (include/spfc_fno.h): the C ABI calls under the
same names, the parameter-vector layout, and a `Surrogate` class that holds a
network on the current HIP device with PyTorch memory and streams.  Marshalling
only: every step of the network runs in the library's HIP kernels; there is no
fallback if the library is missing.
"""

from __future__ import annotations

import ctypes
import math
import os

from .binding import SPFC_OK, SpfcError

HERE = os.path.dirname(os.path.abspath(__file__))
FNO_LIB_PATH = os.environ.get("SPFC_FNO_LIB", os.path.join(HERE, "libspfc_fno.so"))

EXPORTS = ["spfc_fno_param_count", "spfc_fno_workspace_bytes", "spfc_fno_init", "spfc_fno_forward",
           "spfc_fno_time_forward", "spfc_fno_grads", "spfc_fno_train_step", "spfc_fno_get_params", "spfc_fno_destroy"]

WIDTH, MODES, HIDDEN, LAYERS = 32, 512, 64, 4


class spfc_fno_shape(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("max_batch", ctypes.c_int), ("train", ctypes.c_int)]


_lib = None


def load_library(path: str | None = None):
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or FNO_LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library not built: {p} is missing (run python -m paper_2012_15133_amd.build)")
    lib = ctypes.CDLL(p)
    vp, sz, i64, i32, f32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64, ctypes.c_int, ctypes.c_float
    P = ctypes.POINTER
    sig = {
        "spfc_fno_param_count": [P(i64)],
        "spfc_fno_workspace_bytes": [P(spfc_fno_shape), P(sz)],
        "spfc_fno_init": [P(spfc_fno_shape), vp, vp, sz, vp, P(vp)],
        "spfc_fno_forward": [vp, i32, vp, vp, vp],
        "spfc_fno_time_forward": [vp, i32, vp, vp, vp, i32, i32, P(ctypes.c_char_p), P(ctypes.c_double),
                                  P(ctypes.c_double), P(i32), P(i32)],
        "spfc_fno_grads": [vp, i32, vp, vp, vp, vp, vp],
        "spfc_fno_train_step": [vp, i32, vp, vp, vp, f32, vp],
        "spfc_fno_get_params": [vp, vp],
        "spfc_fno_destroy": [vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def _check(call, status):
    if status != SPFC_OK:
        raise SpfcError(call, status)


# ------------------------------------------------------------------ wrappers, same names as the ABI

def spfc_fno_param_count() -> int:
    n = ctypes.c_int64()
    _check("spfc_fno_param_count", load_library().spfc_fno_param_count(ctypes.byref(n)))
    return n.value


def spfc_fno_workspace_bytes(shape: spfc_fno_shape) -> int:
    n = ctypes.c_size_t()
    _check("spfc_fno_workspace_bytes", load_library().spfc_fno_workspace_bytes(ctypes.byref(shape), ctypes.byref(n)))
    return n.value


def spfc_fno_init(shape, params_ptr: int, ws_ptr: int, ws_bytes: int, stream_ptr: int):
    h = ctypes.c_void_p()
    _check("spfc_fno_init", load_library().spfc_fno_init(ctypes.byref(shape), params_ptr, ws_ptr, ws_bytes,
                                                         stream_ptr, ctypes.byref(h)))
    return h


def spfc_fno_forward(h, batch: int, phi_ptr: int, eps_ptr: int, out_ptr: int):
    _check("spfc_fno_forward", load_library().spfc_fno_forward(h, int(batch), phi_ptr, eps_ptr, out_ptr))


def spfc_fno_time_forward(h, batch: int, phi_ptr: int, eps_ptr: int, out_ptr: int, reps: int):
    """Per-kernel timing of one forward pass: {role: (avg_ms, bytes, launches)}."""
    cap = 16
    names = (ctypes.c_char_p * cap)()
    ms, nbytes = (ctypes.c_double * cap)(), (ctypes.c_double * cap)()
    launches, count = (ctypes.c_int * cap)(), ctypes.c_int()
    _check("spfc_fno_time_forward", load_library().spfc_fno_time_forward(
        h, int(batch), phi_ptr, eps_ptr, out_ptr, int(reps), cap, names, ms, nbytes, launches, ctypes.byref(count)))
    return {names[i].decode(): (ms[i], nbytes[i], launches[i]) for i in range(min(count.value, cap))}


def spfc_fno_grads(h, batch: int, phi_ptr: int, eps_ptr: int, target_ptr: int, loss_ptr: int, grad_ptr: int):
    _check("spfc_fno_grads", load_library().spfc_fno_grads(h, int(batch), phi_ptr, eps_ptr, target_ptr, loss_ptr,
                                                           grad_ptr))


def spfc_fno_train_step(h, batch: int, phi_ptr: int, eps_ptr: int, target_ptr: int, lr: float, loss_ptr: int):
    _check("spfc_fno_train_step", load_library().spfc_fno_train_step(h, int(batch), phi_ptr, eps_ptr, target_ptr,
                                                                     float(lr), loss_ptr))


def spfc_fno_get_params(h, params_ptr: int):
    _check("spfc_fno_get_params", load_library().spfc_fno_get_params(h, params_ptr))


def spfc_fno_destroy(h):
    _check("spfc_fno_destroy", load_library().spfc_fno_destroy(h))


# ------------------------------------------------------------------ parameter vector

def param_layout():
    """(name, shape) of every block of the parameter vector, in order."""
    c, h = WIDTH, HIDDEN
    out = [("Lw", (c, 2)), ("Lb", (c,))]
    for l in range(LAYERS):
        out += [(f"Wr{l}", (MODES, c, c)), (f"Wi{l}", (MODES, c, c)), (f"Pw{l}", (c, c)), (f"Pb{l}", (c,))]
    out += [("Q1", (h, c)), ("q1", (h,)), ("Q2", (h,)), ("q2", (1,))]
    return out


def flatten(params: dict):
    """Dict of arrays/tensors (any float type, CPU) -> one float32 torch vector."""
    import torch
    return torch.cat([torch.as_tensor(params[k]).reshape(-1).to(torch.float32) for k, _ in param_layout()])


def unflatten(vec) -> dict:
    out, o = {}, 0
    for k, shp in param_layout():
        n = math.prod(shp)
        out[k] = vec[o:o + n].reshape(shp)
        o += n
    return out


def init_params(seed: int = 0) -> dict:
    """Seeded uniform initial weights with fan-in scaling (float32, CPU)."""
    import torch
    g = torch.Generator().manual_seed(seed)
    out = {}
    scales = {"Lw": 1.0, "Lb": 0.1, "Q1": 1.0 / math.sqrt(WIDTH), "q1": 0.1, "Q2": 1.0 / math.sqrt(HIDDEN), "q2": 0.0}
    for k, shp in param_layout():
        if k[:2] in ("Wr", "Wi"):
            s = 1.0 / (WIDTH * WIDTH)
        elif k[:2] == "Pw":
            s = 1.0 / math.sqrt(WIDTH)
        elif k[:2] == "Pb":
            s = 0.1
        else:
            s = scales[k]
        out[k] = (torch.rand(shp, generator=g, dtype=torch.float32) * 2.0 - 1.0) * s
    return out


# ------------------------------------------------------------------ convenience class

class Surrogate:
    """FNO on the current HIP device.  params: flat float32 vector (CPU or device) or a dict."""

    def __init__(self, n: int, params, max_batch: int = 64, train: bool = False, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Surrogate needs a HIP device")
        load_library()
        self.torch = torch
        self.n = int(n)
        self.shape = spfc_fno_shape(self.n, int(max_batch), 1 if train else 0)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        vec = flatten(params) if isinstance(params, dict) else params
        vec = torch.as_tensor(vec, dtype=torch.float32).to("cuda").contiguous()
        if vec.numel() != spfc_fno_param_count():
            raise ValueError(f"parameter vector has {vec.numel()} entries, expected {spfc_fno_param_count()}")
        nb = spfc_fno_workspace_bytes(self.shape)
        self.workspace = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
        ws = (self.workspace.data_ptr() + 255) // 256 * 256
        self.h = spfc_fno_init(self.shape, vec.data_ptr(), ws, nb, self.stream.cuda_stream)
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")

    def _inputs(self, phi, eps):
        torch = self.torch
        phi = torch.as_tensor(phi).to(device="cuda", dtype=torch.float32).contiguous()
        eps = torch.as_tensor(eps).to(device="cuda", dtype=torch.float32).contiguous()
        return phi, eps

    def forward(self, phi, eps):
        """phi [B, n, n], eps [B] -> phi_pred [B, n, n] (float32 device tensor)."""
        phi, eps = self._inputs(phi, eps)
        out = self.torch.empty_like(phi)
        spfc_fno_forward(self.h, phi.shape[0], phi.data_ptr(), eps.data_ptr(), out.data_ptr())
        return out

    def time_forward(self, phi, eps, reps=20):
        """Per-kernel timing of one forward pass (each launch repeated `reps` times back to
        back between HIP events): {role: (avg_ms per launch, algorithmic bytes per launch,
        launches per pass)}, and the forward result."""
        phi, eps = self._inputs(phi, eps)
        out = self.torch.empty_like(phi)
        roles = spfc_fno_time_forward(self.h, phi.shape[0], phi.data_ptr(), eps.data_ptr(), out.data_ptr(), reps)
        return roles, out

    def grads(self, phi, eps, target):
        phi, eps = self._inputs(phi, eps)
        target = self.torch.as_tensor(target).to(device="cuda", dtype=self.torch.float32).contiguous()
        g = self.torch.empty(spfc_fno_param_count(), dtype=self.torch.float32, device="cuda")
        spfc_fno_grads(self.h, phi.shape[0], phi.data_ptr(), eps.data_ptr(), target.data_ptr(), self.loss.data_ptr(),
                       g.data_ptr())
        return float(self.loss.item()), g

    def train_step(self, phi, eps, target, lr):
        """One Adam step on device tensors (float32, contiguous); returns the loss tensor
        (device, not synchronized)."""
        spfc_fno_train_step(self.h, phi.shape[0], phi.data_ptr(), eps.data_ptr(), target.data_ptr(), lr,
                            self.loss.data_ptr())
        return self.loss

    def params(self):
        v = self.torch.empty(spfc_fno_param_count(), dtype=self.torch.float32, device="cuda")
        spfc_fno_get_params(self.h, v.data_ptr())
        return v

    def close(self):
        if getattr(self, "h", None) is not None:
            spfc_fno_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
