"""Python binding of the warm-start network (``include/lbml.h``).

Argument marshalling only: the forward, backward, loss and Adam steps run in
the gfx950 kernels of ``liblbnlm.so`` (BF16 matrix-core GEMMs with FP32
accumulation). PyTorch provides device memory and the stream.
"""
import ctypes as C
from typing import Sequence

import numpy as np

from .lbnlm import load_library

LBML_FUNCTIONS = ["lbml_workspace_bytes", "lbml_param_count", "lbml_create", "lbml_destroy", "lbml_set_params",
                  "lbml_get_params", "lbml_forward", "lbml_mse", "lbml_backward", "lbml_get_grads",
                  "lbml_adam_step", "lbml_train_step", "lbml_last_error"]

_bound = False


def _lib():
    global _bound
    L = load_library()
    if not _bound:
        vp, sz, fp = C.c_void_p, C.c_size_t, C.POINTER(C.c_float)
        ip = C.POINTER(C.c_int32)
        L.lbml_workspace_bytes.argtypes = [C.c_int32, ip, C.c_int32, C.POINTER(sz)]
        L.lbml_param_count.argtypes = [C.c_int32, ip, C.POINTER(sz)]
        L.lbml_create.argtypes = [C.c_int32, ip, C.c_int32, vp, sz, vp, C.POINTER(vp)]
        L.lbml_destroy.argtypes = [vp]
        L.lbml_set_params.argtypes = [vp, fp, sz]
        L.lbml_get_params.argtypes = [vp, fp, sz]
        L.lbml_get_grads.argtypes = [vp, fp, sz]
        L.lbml_forward.argtypes = [vp, vp, C.c_int32, vp]
        L.lbml_mse.argtypes = [vp, vp, vp, C.c_int32, vp, C.POINTER(C.c_double)]
        L.lbml_backward.argtypes = [vp, vp, C.c_int32]
        L.lbml_adam_step.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int32]
        L.lbml_train_step.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float,
                                      C.c_int32, C.POINTER(C.c_double)]
        L.lbml_last_error.argtypes = [vp]
        L.lbml_last_error.restype = C.c_char_p
        for n in LBML_FUNCTIONS[:-1]:
            getattr(L, n).restype = C.c_int32
        _bound = True
    return L


def param_count(dims: Sequence[int]) -> int:
    L = _lib()
    d = (C.c_int32 * len(dims))(*dims)
    out = C.c_size_t(0)
    if L.lbml_param_count(len(dims) - 1, d, C.byref(out)) != 0:
        raise ValueError("bad dims")
    return int(out.value)


def init_params(dims: Sequence[int], seed: int = 0) -> np.ndarray:
    """Uniform fan-in initialisation (limit sqrt(3/fan_in) for SiLU layers,
    sqrt(1/fan_in) for the output layer), zero biases, flat layout of lbml.h."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(len(dims) - 1):
        fan_in, fan_out = dims[l], dims[l + 1]
        lim = np.sqrt((3.0 if l < len(dims) - 2 else 1.0) / fan_in)
        parts.append(rng.uniform(-lim, lim, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


class Net:
    """A network of widths ``dims`` for batches of up to ``max_batch`` rows.

    Its kernels run on ``stream`` (default: torch's current stream, which may
    be the null stream), so that they are ordered with the torch operations
    that produce its inputs and consume its outputs, and with the caching
    allocator that recycles those tensors."""

    def __init__(self, dims: Sequence[int], max_batch: int, stream=None, device="cuda"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("lbml needs a GPU; no CPU fallback exists")
        self.L = _lib()
        self.dims = [int(d) for d in dims]
        self.max_batch = int(max_batch)
        d = (C.c_int32 * len(self.dims))(*self.dims)
        nb = C.c_size_t(0)
        if self.L.lbml_workspace_bytes(len(self.dims) - 1, d, self.max_batch, C.byref(nb)) != 0:
            raise ValueError("bad network shape")
        self.device = torch.device(device)
        self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        st = self.L.lbml_create(len(self.dims) - 1, d, self.max_batch, C.c_void_p(ptr), nb.value,
                                C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != 0:
            raise RuntimeError(f"lbml_create failed ({st})")
        self.h = h
        self.n_params = param_count(self.dims)
        self.t = 0

    def _check(self, st):
        if st != 0:
            raise RuntimeError(f"lbml error {st}: {self.L.lbml_last_error(self.h).decode()}")

    def set_params(self, p: np.ndarray):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.n_params
        self._check(self.L.lbml_set_params(self.h, p.ctypes.data_as(C.POINTER(C.c_float)), p.size))

    def get_params(self) -> np.ndarray:
        p = np.zeros(self.n_params, dtype=np.float32)
        self._check(self.L.lbml_get_params(self.h, p.ctypes.data_as(C.POINTER(C.c_float)), p.size))
        return p

    def get_grads(self) -> np.ndarray:
        g = np.zeros(self.n_params, dtype=np.float32)
        self._check(self.L.lbml_get_grads(self.h, g.ctypes.data_as(C.POINTER(C.c_float)), g.size))
        return g

    def forward(self, x_dev, y_dev=None):
        """x_dev: float32 CUDA tensor [batch, dims[0]]; returns y [batch, dims[-1]]."""
        import torch
        assert x_dev.dtype == torch.float32 and x_dev.is_contiguous() and x_dev.shape[1] == self.dims[0]
        b = x_dev.shape[0]
        if y_dev is None:
            y_dev = torch.empty((b, self.dims[-1]), dtype=torch.float32, device=self.device)
        self._x = x_dev  # must stay alive until backward
        self._check(self.L.lbml_forward(self.h, C.c_void_p(x_dev.data_ptr()), b, C.c_void_p(y_dev.data_ptr())))
        return y_dev

    def mse(self, y_dev, t_dev, dy_dev, want_loss=True):
        loss = C.c_double(0.0)
        self._check(self.L.lbml_mse(self.h, C.c_void_p(y_dev.data_ptr()), C.c_void_p(t_dev.data_ptr()),
                                    y_dev.shape[0], C.c_void_p(dy_dev.data_ptr()),
                                    C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def backward(self, dy_dev):
        self._check(self.L.lbml_backward(self.h, C.c_void_p(dy_dev.data_ptr()), dy_dev.shape[0]))

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        self._check(self.L.lbml_adam_step(self.h, lr, beta1, beta2, eps, self.t))

    def train_step(self, X_dev, Y_dev, idx_dev, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, want_loss=False):
        """lbml_train_step: forward, MSE, backward and Adam on rows idx_dev
        (int32 CUDA tensor) of X_dev / Y_dev (float32 CUDA tensors), in one
        call; returns the batch loss before the update if want_loss."""
        import torch
        assert X_dev.dtype == torch.float32 and X_dev.is_contiguous() and X_dev.shape[1] == self.dims[0]
        assert Y_dev.dtype == torch.float32 and Y_dev.is_contiguous() and Y_dev.shape[1] == self.dims[-1]
        assert idx_dev.dtype == torch.int32 and idx_dev.is_contiguous() and idx_dev.numel() <= self.max_batch
        self.t += 1
        loss = C.c_double(0.0)
        self._check(self.L.lbml_train_step(self.h, C.c_void_p(X_dev.data_ptr()), C.c_void_p(Y_dev.data_ptr()),
                                           C.c_void_p(idx_dev.data_ptr()), idx_dev.numel(), lr, beta1, beta2, eps,
                                           self.t, C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.L.lbml_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
