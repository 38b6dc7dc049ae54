"""Python binding of the lbnlm C ABI (``include/lb.h``).

Argument marshalling only: every step of the solver runs in the gfx950
kernels of ``liblbnlm.so``. PyTorch provides the device workspace and the
stream. There is no CPU path: without the built library, or without a GPU,
creating a :class:`Solver` raises.
"""
import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbnlm.so")

FP64 = 0
FP32_SHIFTED = 1

PROFILES = {"ux": 0, "uy": 1, "sxx": 2, "sxy": 3, "syy": 4, "n1": 5, "pressure": 6,
            "kxy": 7, "trT": 8, "kxx": 9}
SCALARS = {"mass": 32, "momx": 33, "flux": 34, "wall_drag": 35, "umid": 36,
           "residual": 37, "step": 38, "active": 39, "nan": 40}

STATUS = {0: "LB_OK", -1: "LB_EINVAL", -2: "LB_ENOMEM", -3: "LB_EHIP", -4: "LB_EUNSTABLE", -5: "LB_ESTATE"}

# Names of every function include/lb.h declares.
ABI_FUNCTIONS = ["lb_workspace_bytes", "lb_create", "lb_destroy", "lb_step", "lb_observe", "lb_observe_noalloc",
                 "lb_get_state", "lb_set_state", "lb_get_stress", "lb_set_stress", "lb_set_profile",
                 "lb_last_error", "lb_status_string"]


TOP_WALLS = {"halfway": 0, "zou_he": 1}


class LbChannel(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("force", C.c_double), ("tau_lb", C.c_double),
                ("G", C.c_double), ("tau0", C.c_double), ("gamma_c", C.c_double), ("eps", C.c_double),
                ("visc_split", C.c_double), ("t_startup", C.c_int64), ("wall_velocity", C.c_double),
                ("pressure_gradient", C.c_double), ("nn_pressure", C.c_int32), ("top_wall", C.c_int32)]


class LbOptions(C.Structure):
    _fields_ = [("precision", C.c_int32), ("obs_every", C.c_int32), ("strip_rows", C.c_int32),
                ("steady_tol", C.c_double), ("viscoelastic", C.c_int32), ("stress_force", C.c_int32),
                ("steps_per_sweep", C.c_int32)]


class LbError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library():
    """Loads ``liblbnlm.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1310_7450_amd/build.py")
    L = C.CDLL(LIB_PATH)
    vp, dp, sz = C.c_void_p, C.POINTER(C.c_double), C.c_size_t
    L.lb_workspace_bytes.argtypes = [C.POINTER(LbChannel), C.c_int32, C.POINTER(LbOptions), C.POINTER(sz)]
    L.lb_create.argtypes = [C.POINTER(LbChannel), C.c_int32, C.POINTER(LbOptions), vp, sz, vp, C.POINTER(vp)]
    L.lb_destroy.argtypes = [vp]
    L.lb_step.argtypes = [vp, C.c_int64]
    L.lb_observe.argtypes = [vp, C.c_int32, C.c_int32, dp, sz]
    L.lb_observe_noalloc.argtypes = [vp, C.c_int32, C.c_int32, dp, sz]
    L.lb_get_state.argtypes = [vp, C.c_int32, dp, dp]
    L.lb_set_state.argtypes = [vp, C.c_int32, dp, dp, C.c_int64]
    L.lb_get_stress.argtypes = [vp, C.c_int32, dp]
    L.lb_set_stress.argtypes = [vp, C.c_int32, dp]
    L.lb_set_profile.argtypes = [vp, C.c_int32, dp, dp, C.c_int32, C.c_int32]
    L.lb_last_error.argtypes = [vp]
    L.lb_last_error.restype = C.c_char_p
    L.lb_status_string.argtypes = [C.c_int32]
    L.lb_status_string.restype = C.c_char_p
    for name in ["lb_workspace_bytes", "lb_create", "lb_destroy", "lb_step", "lb_observe", "lb_observe_noalloc",
                 "lb_get_state", "lb_set_state", "lb_get_stress", "lb_set_stress", "lb_set_profile"]:
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


@dataclass
class ChannelSpec:
    """Parameters of one channel (lattice units; see ``lb_channel`` in lb.h).
    ``nn_pressure`` None takes the Solver's default; ``top_wall`` is
    "halfway" or "zou_he"."""
    nx: int
    ny: int
    force: float
    tau_lb: float = 1.0
    G: float = 1e-4
    tau0: float = 1e4
    gamma_c: float = 0.1
    eps: float = 0.0
    visc_split: float = 0.0
    t_startup: int = 2 ** 62
    wall_velocity: float = 0.0
    pressure_gradient: float = 0.0
    nn_pressure: Optional[bool] = None
    top_wall: str = "halfway"

    def resolved_nn_pressure(self, default=True):
        return bool(default if self.nn_pressure is None else self.nn_pressure)

    def to_c(self, default_nn_pressure=True):
        return LbChannel(int(self.nx), int(self.ny), float(self.force), float(self.tau_lb), float(self.G),
                         float(self.tau0), float(self.gamma_c), float(self.eps), float(self.visc_split),
                         int(self.t_startup), float(self.wall_velocity), float(self.pressure_gradient),
                         int(self.resolved_nn_pressure(default_nn_pressure)), TOP_WALLS[self.top_wall])


def _dp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def options(precision=FP64, obs_every=1000, strip_rows=0, steady_tol=0.0, viscoelastic=False, stress_force=False,
            steps_per_sweep=0):
    if isinstance(precision, str):
        precision = {"fp64": FP64, "fp32": FP32_SHIFTED, "fp32_shifted": FP32_SHIFTED}[precision]
    return LbOptions(int(precision), int(obs_every), int(strip_rows), float(steady_tol), int(bool(viscoelastic)),
                     int(bool(stress_force)), int(steps_per_sweep))


def channel_array(channels: Sequence[ChannelSpec], default_nn_pressure=True):
    return (LbChannel * len(channels))(*[c.to_c(default_nn_pressure) for c in channels])


def workspace_bytes(channels: Sequence[ChannelSpec], opts: LbOptions, default_nn_pressure=True) -> int:
    L = load_library()
    arr = channel_array(channels, default_nn_pressure)
    out = C.c_size_t(0)
    st = L.lb_workspace_bytes(arr, len(channels), C.byref(opts), C.byref(out))
    if st != 0:
        raise LbError(st, "invalid channels or options")
    return int(out.value)


class Solver:
    """A handle of the C library over ``channels``, on one CUDA/HIP stream.
    ``nn_pressure`` is the value of lb_channel.nn_pressure for every channel
    whose spec leaves it None. ``viscoelastic`` selects the time-integrated
    nonlinear Maxwell stress (lb_options.viscoelastic) in place of the
    instantaneous one; ``stress_force`` makes the stress enter as the force
    density div Sigma^nN (lb_options.stress_force; FP64, nn_pressure False).
    ``steps_per_sweep`` is lb_options.steps_per_sweep (0: two steps per pass
    where eligible, 1: one)."""

    def __init__(self, channels: Sequence[ChannelSpec], precision="fp64", nn_pressure=True,
                 obs_every=1000, strip_rows=0, steady_tol=0.0, stream=None, device="cuda", viscoelastic=False,
                 stress_force=False, steps_per_sweep=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("lbnlm needs a GPU; no CPU fallback exists")
        self.L = load_library()
        self.channels = list(channels)
        self.opts = options(precision, obs_every, strip_rows, steady_tol, viscoelastic, stress_force,
                            steps_per_sweep)
        self.default_nn_pressure = bool(nn_pressure)
        nbytes = workspace_bytes(self.channels, self.opts, self.default_nn_pressure)
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = self.workspace.data_ptr()
        aligned = (ptr + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        arr = channel_array(self.channels, self.default_nn_pressure)
        h = C.c_void_p()
        st = self.L.lb_create(arr, len(self.channels), C.byref(self.opts), C.c_void_p(aligned),
                              nbytes, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != 0:
            raise LbError(st, "lb_create failed")
        self.h = h

    # ------------------------------------------------------------------ calls
    def _check(self, st):
        if st != 0:
            msg = self.L.lb_last_error(self.h).decode()
            raise LbError(st, msg)

    def step(self, n: int):
        self._check(self.L.lb_step(self.h, int(n)))

    def observe(self, ch: int, what: str):
        if what in SCALARS:
            out = np.zeros(1)
            self._check(self.L.lb_observe(self.h, ch, SCALARS[what], _dp(out), 1))
            return float(out[0])
        ny = self.channels[ch].ny
        out = np.zeros(ny)
        self._check(self.L.lb_observe(self.h, ch, PROFILES[what], _dp(out), ny))
        return out

    def observe_noalloc(self, ch: int, what: str):
        """lb_observe_noalloc: the same values as observe(), computed in the
        library's per-GPU static scratch (no allocation on the call)."""
        if what in SCALARS:
            out = np.zeros(1)
            self._check(self.L.lb_observe_noalloc(self.h, ch, SCALARS[what], _dp(out), 1))
            return float(out[0])
        out = np.zeros(self.channels[ch].ny)
        self._check(self.L.lb_observe_noalloc(self.h, ch, PROFILES[what], _dp(out), len(out)))
        return out

    def profiles(self, ch: int):
        return {k: self.observe(ch, k) for k in PROFILES}

    def get_state(self, ch: int):
        c = self.channels[ch]
        pops = np.zeros((9, c.ny, c.nx))
        P = np.zeros((c.ny, c.nx))
        self._check(self.L.lb_get_state(self.h, ch, _dp(pops), _dp(P)))
        return pops, P

    def set_state(self, ch: int, pops, P, t: int):
        pops = np.ascontiguousarray(pops, dtype=np.float64)
        P = np.ascontiguousarray(P, dtype=np.float64)
        c = self.channels[ch]
        assert pops.shape == (9, c.ny, c.nx) and P.shape == (c.ny, c.nx)
        self._check(self.L.lb_set_state(self.h, ch, _dp(pops), _dp(P), int(t)))

    def get_stress(self, ch: int):
        """Stored stress sigma(t-1) of channel ch as [3, ny, nx] (xx, xy, yy);
        viscoelastic handles only."""
        c = self.channels[ch]
        sig = np.zeros((3, c.ny, c.nx))
        self._check(self.L.lb_get_stress(self.h, ch, _dp(sig)))
        return sig

    def set_stress(self, ch: int, sigma):
        sigma = np.ascontiguousarray(sigma, dtype=np.float64)
        c = self.channels[ch]
        assert sigma.shape == (3, c.ny, c.nx)
        self._check(self.L.lb_set_stress(self.h, ch, _dp(sigma)))

    def set_profile(self, ch: int, ux, n1, points="rows"):
        """Warm start of channel ch from u_x and N1 at the lattice rows
        (points="rows") or at Chebyshev-Gauss points (points="chebyshev")."""
        ux = np.ascontiguousarray(ux, dtype=np.float64)
        n1 = np.ascontiguousarray(n1, dtype=np.float64)
        assert ux.shape == n1.shape and ux.ndim == 1
        mode = {"rows": 0, "chebyshev": 1}[points]
        self._check(self.L.lb_set_profile(self.h, ch, _dp(ux), _dp(n1), len(ux), mode))

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.L.lb_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
