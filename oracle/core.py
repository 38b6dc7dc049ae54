"""ctypes binding of the FP64 C oracle (``lb_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The oracle state is the post-streaming population n_i(r, t) of the paper's
Eq. (lbupdate), stored as ``n[9, ny, nx]``, plus the previous stress trace
``P[ny, nx]`` that Eq. (rhoplus) differences against, and, with the
time-integrated (viscoelastic) model, the stress of the previous step
``S[3, ny, nx]`` (xx, xy, yy).
"""
import ctypes as C

import numpy as np

from . import build as _build

_lib = None

FIELDS = ["utx", "uty", "kxx", "kxy", "kyx", "kyy", "sxx", "sxy", "syy",
          "trT", "r", "rho_e", "ux", "uy", "s", "mx", "my", "tauM"]

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
WEIGHTS = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


class OrcParams(C.Structure):
    _fields_ = [("g", C.c_double), ("tau_eff", C.c_double), ("G", C.c_double),
                ("tau", C.c_double), ("gamma_c", C.c_double), ("lam", C.c_double),
                ("t_startup", C.c_longlong), ("nn_pressure", C.c_int), ("uw", C.c_double),
                ("dp", C.c_double), ("ve", C.c_int), ("saf", C.c_int), ("zh", C.c_int)]


def lib():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        L.orc_resolve.argtypes = [C.c_double] * 6 + [C.c_double, C.c_longlong, C.c_int, C.c_double,
                                                     C.c_double, C.c_int, C.c_int, C.c_int,
                                                     C.POINTER(OrcParams)]
        L.orc_resolve.restype = C.c_int
        L.orc_equilibrium.argtypes = [C.c_double] * 3 + [dp]
        L.orc_forcing.argtypes = [C.c_double, dp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, dp]
        L.orc_stress_series.argtypes = [dp, C.c_double, C.c_double, dp]
        L.orc_stress_series.restype = C.c_int
        L.orc_tau_M.argtypes = [dp, C.c_double, C.c_double]
        L.orc_tau_M.restype = C.c_double
        L.orc_stress_ve_step.argtypes = [dp, C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_step.argtypes = [C.POINTER(OrcParams), C.c_int, C.c_int, dp, dp, dp, C.c_longlong, dp, dp, dp,
                               dp]
        L.orc_step.restype = C.c_int
        L.orc_run.argtypes = [C.POINTER(OrcParams), C.c_int, C.c_int, dp, dp, dp, C.c_longlong, C.c_longlong]
        L.orc_run.restype = C.c_longlong
        L.orc_init_rest.argtypes = [C.c_int, C.c_int, dp, dp, dp]
        L.orc_zou_he_top.argtypes = [C.POINTER(OrcParams), C.c_int, C.c_int, dp, C.c_longlong]
        L.orc_wall_drag.argtypes = [C.c_int, C.c_int, dp, C.c_double]
        L.orc_wall_drag.restype = C.c_double
        L.orc_num_fields.restype = C.c_int
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        assert L.orc_num_fields() == len(FIELDS)
        _lib = L
    return _lib


def _p(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def num_threads():
    return int(lib().orc_num_threads())


def set_num_threads(n):
    lib().orc_set_num_threads(int(n))


def equilibrium(rho, ux, uy):
    out = np.zeros(9)
    lib().orc_equilibrium(rho, ux, uy, _p(out))
    return out


def forcing(tau, sbar, r, fx, fy, ux, uy):
    out = np.zeros(9)
    sb = np.ascontiguousarray(sbar, dtype=np.float64)
    lib().orc_forcing(tau, _p(sb), r, fx, fy, ux, uy, _p(out))
    return out


def stress_series(kappa, G, tauM):
    """sigma (xx, xy, yy) of Eq. (sigtsum) and the number of terms (-1: diverged)."""
    k = np.ascontiguousarray(kappa, dtype=np.float64).reshape(2, 2)
    out = np.zeros(3)
    nt = lib().orc_stress_series(_p(k), G, tauM, _p(out))
    return out, nt


def stress_ve_step(kappa, G, tau, gamma_c, sigma_prev):
    """One step of the time-integrated stress (xx, xy, yy) from sigma_prev
    under the velocity gradient kappa[a][b] = d_b u_a."""
    k = np.ascontiguousarray(kappa, dtype=np.float64).reshape(2, 2)
    sp = np.ascontiguousarray(sigma_prev, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_stress_ve_step(_p(k), G, tau, gamma_c, _p(sp), _p(out))
    return out


def tau_M(kappa, tau, gamma_c):
    k = np.ascontiguousarray(kappa, dtype=np.float64).reshape(2, 2)
    return lib().orc_tau_M(_p(k), tau, gamma_c)


TOP_WALLS = {"halfway": 0, "zou_he": 1}


def resolve(tau_lb, G, tau0, gamma_c, eps=0.0, visc_split=0.0, force=0.0,
            t_startup=2 ** 62, nn_pressure=True, wall_velocity=0.0, pressure_drop=0.0, viscoelastic=False,
            stress_force=False, top_wall="halfway"):
    p = OrcParams()
    rc = lib().orc_resolve(tau_lb, G, tau0, gamma_c, eps, visc_split, force,
                           int(t_startup), int(bool(nn_pressure)), float(wall_velocity),
                           float(pressure_drop), int(bool(viscoelastic)), int(bool(stress_force)),
                           TOP_WALLS[top_wall], C.byref(p))
    if rc != 0:
        raise ValueError("invalid channel parameters")
    return p


class Channel:
    """One channel advanced by the oracle. Time ``t`` counts completed steps."""

    def __init__(self, nx, ny, force, tau_lb=1.0, G=1e-4, tau0=1e4, gamma_c=0.1,
                 eps=0.0, visc_split=0.0, t_startup=2 ** 62, nn_pressure=True, wall_velocity=0.0,
                 pressure_gradient=0.0, viscoelastic=False, stress_force=False, top_wall="halfway"):
        """wall_velocity: x velocity of the top wall while t < t_startup
        (planar Couette flow); 0 gives the channel with two fixed walls.
        top_wall: "halfway" (bounce-back on the half link above row ny - 1;
        a moving wall reflects with the wall-momentum term, R9) or "zou_he"
        (Zou and He's velocity boundary on the top node row, R13: the
        channel spans y = -1/2 .. ny - 1).
        pressure_gradient: pressure drop per unit length G_p imposed by
        generalised periodic boundaries (R10: p+ - p- = (nx + 1) G_p between
        the virtual nodes; needs force 0 and nn_pressure False).
        viscoelastic: the time-integrated nonlinear Maxwell stress (R11),
        carried in ``S`` from step to step, in place of the instantaneous one.
        stress_force: the non-Newtonian stress enters as the force density
        div Sigma^nN (R12; needs nn_pressure False)."""
        self.nx, self.ny = int(nx), int(ny)
        self.params = resolve(tau_lb, G, tau0, gamma_c, eps, visc_split, force,
                              t_startup, nn_pressure, wall_velocity, (self.nx + 1) * pressure_gradient,
                              viscoelastic, stress_force, top_wall)
        self.n = np.empty((9, self.ny, self.nx))
        self.P = np.empty((self.ny, self.nx))
        self.S = np.zeros((3, self.ny, self.nx))
        lib().orc_init_rest(self.nx, self.ny, _p(self.n), _p(self.P), _p(self.S))
        self.t = 0
        self._complete_top()

    def _complete_top(self):
        """R13: the top node row's populations entering from outside the
        lattice, completed for the current step."""
        if self.params.zh:
            lib().orc_zou_he_top(C.byref(self.params), self.nx, self.ny, _p(self.n), self.t)

    def set_state(self, n, P, t=None, S=None):
        self.n[...] = n
        self.P[...] = P
        if S is not None:
            self.S[...] = S
        if t is not None:
            self.t = int(t)
        self._complete_top()

    def run(self, steps):
        bad = lib().orc_run(C.byref(self.params), self.nx, self.ny, _p(self.n), _p(self.P), _p(self.S),
                            self.t, int(steps))
        if bad != 0:
            raise RuntimeError(f"oracle: stress series failed at {bad} node-steps")
        self.t += int(steps)

    def fields(self):
        """Per-node observables of the current step, dict name -> [ny, nx]."""
        f = np.empty((len(FIELDS), self.ny, self.nx))
        bad = lib().orc_step(C.byref(self.params), self.nx, self.ny, _p(self.n), _p(self.P), _p(self.S),
                             self.t, None, None, None, _p(f))
        if bad != 0:
            raise RuntimeError("oracle: stress series failed")
        return {name: f[q] for q, name in enumerate(FIELDS)}

    def profiles(self):
        """x-averaged rows of every field."""
        return {k: v.mean(axis=1) for k, v in self.fields().items()}

    def mass(self):
        """sum over nodes of (sum_i n_i - delta rho_prev), delta rho_prev = -(3/2) P."""
        return float(self.n.sum() + 1.5 * self.P.sum()) if self.params.nn_pressure else float(self.n.sum())

    def momentum_x(self):
        return float((CX[:, None, None] * self.n).sum())

    def wall_drag(self):
        """Momentum handed to both walls by the step that produced the state
        (the top wall moved during step t - 1 if t - 1 < t_startup)."""
        uw = self.params.uw if 1 <= self.t and self.t - 1 < self.params.t_startup else 0.0
        return float(lib().orc_wall_drag(self.nx, self.ny, _p(self.n), uw))

    def force_now(self):
        return self.params.g if self.t < self.params.t_startup else 0.0
