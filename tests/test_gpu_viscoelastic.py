"""GPU parity of the time-integrated (viscoelastic) nonlinear Maxwell model
against the FP64 oracle, through the C ABI.

The model is Eq. (gkder) with d_t G = -G / tau_M(t), tau_M from
Eq. (nlmaxwell), stepped with explicit upper-convected terms and implicit
relaxation. The stress of the previous step is part of the state. The GPU
writes the step as the old stress plus its increment and the oracle as one
quotient: equal in exact arithmetic, so FP64 agrees to rounding. Tolerances
as for the instantaneous model: FP64 1e-5, FP32 1e-3 relative L-infinity on
u_x and sigma_xy; states node by node where the run is well conditioned
(G tau <= 0.2).
"""
import dataclasses

import numpy as np
import pytest

from paper_1310_7450_amd import workloads
from paper_1310_7450_amd.lbnlm import ChannelSpec, LbError

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-5
FP32_TOL = 1e-3
ETA_S = 1.0 / 6.0


def solver(channels, **kw):
    from paper_1310_7450_amd import Solver
    return Solver(channels, viscoelastic=True, **kw)


def oracle_channel(orc, spec, nn_pressure=True):
    return orc.Channel(spec.nx, spec.ny, spec.force, tau_lb=spec.tau_lb, G=spec.G, tau0=spec.tau0,
                       gamma_c=spec.gamma_c, eps=spec.eps, visc_split=spec.visc_split,
                       t_startup=spec.t_startup, viscoelastic=True, nn_pressure=nn_pressure,
                       wall_velocity=spec.wall_velocity, pressure_gradient=spec.pressure_gradient,
                       top_wall=spec.top_wall)


def linf(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def compare_profiles(s, ch, o, tol, label):
    """x-averaged u_x, sigma_xy and N1 of GPU channel ch against oracle o."""
    f = o.fields()
    errs = {}
    for name, ref in (("ux", f["ux"]), ("sxy", f["sxy"]), ("n1", f["sxx"] - f["syy"])):
        errs[name] = linf(s.observe(ch, name), ref.mean(axis=1))
    print(f"{label}: " + " ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
    assert errs["ux"] <= tol and errs["sxy"] <= tol, (label, errs)
    assert errs["n1"] <= 10 * tol, (label, errs)
    return errs


@pytest.mark.parametrize("nx,ny", [(1, 16), (4, 33), (64, 7), (100, 37), (130, 5), (8, 1), (128, 9), (192, 5),
                                   (256, 3), (384, 2), (512, 9), (768, 11)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_perturbed_state_parity(orc, nx, ny, precision):
    """Seeded random populations, trace and stress on narrow, aligned-wide,
    ragged-wide and odd lattices (every sweep kernel class): one and several
    steps match the oracle node by node, populations, trace and stress."""
    spec = ChannelSpec(nx=nx, ny=ny, force=3e-6, tau_lb=0.8, G=2e-4, tau0=500.0, gamma_c=0.1,
                       eps=0.01, visc_split=0.3, t_startup=40)
    pops, P = workloads.random_state(nx, ny, seed=nx * 1000 + ny)
    sig = workloads.random_stress(nx, ny, seed=nx * 1000 + ny + 7)
    o = oracle_channel(orc, spec)
    o.set_state(pops, P, t=0, S=sig)
    tol = 1e-12 if precision == "fp64" else 2e-6
    with solver([spec], precision=precision, obs_every=16, strip_rows=4) as s:
        s.set_state(0, pops, P, 0)
        s.set_stress(0, sig)
        assert np.abs(s.get_stress(0) - sig).max() <= (0 if precision == "fp64" else 1e-13)
        for n in [1, 2, 57]:
            s.step(n)
            o.run(n)
            g_pops, g_P = s.get_state(0)
            g_sig = s.get_stress(0)
            err = np.abs(g_pops - o.n).max() / np.abs(o.n - workloads.REST_WEIGHTS[:, None, None]).max()
            perr = np.abs(g_P - o.P).max() / max(np.abs(o.P).max(), 1e-30)
            serr = np.abs(g_sig - o.S).max() / np.abs(o.S).max()
            print(f"{precision} {nx}x{ny} t={o.t}: state {err:.2e} P {perr:.2e} sigma {serr:.2e}", flush=True)
            assert err < tol * 50 and perr < (1e-9 if precision == "fp64" else 1e-3)
            assert serr < (1e-11 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_channel_startup_and_steady_state(orc, precision):
    """x-uniform channels of four widths (narrow, vector, aligned 64-column and
    generic strips) in one handle, from rest: at 300 steps (the stress still
    building up) and at 40,000 steps (steady) each equals the nx = 1 oracle
    run of the time-integrated model, and the steady profile is within 1% of
    the analytic one of Sec. III.B (which both models share)."""
    from oracle import analytic
    ny, g, tau0 = 32, 2e-6, 1e3
    widths = [8, 256, 320, 100]
    specs = [ChannelSpec(nx=w, ny=ny, force=g, tau_lb=1.0, G=1e-4, tau0=tau0, gamma_c=0.1) for w in widths]
    o = oracle_channel(orc, dataclasses.replace(specs[0], nx=1))
    tol = FP64_TOL if precision == "fp64" else FP32_TOL
    with solver(specs, precision=precision, obs_every=100) as s:
        for n, label in ((300, "start-up"), (39700, "steady")):
            s.step(n)
            o.run(n)
            for i, w in enumerate(widths):
                compare_profiles(s, i, o, tol, f"{precision} nx={w} {label} t={o.t}")
                assert np.abs(s.observe(i, "kxx")).max() == 0.0
        want = analytic.steady_profile(ny, g, ETA_S, 1e-4, tau0, 0.1)
        for i in range(len(widths)):
            assert linf(s.observe(i, "ux"), want) < 1e-2


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_large_channel_sampled_rows(orc, precision):
    """The 4096 x 1024 lattice at full size with the time-integrated stress
    (the launch configuration the benchmark times), eps = -0.05: after 2,000
    steps from rest the x-averaged rows equal an nx = 1 oracle run."""
    wl = workloads.large_channel(eps=-0.05)
    spec = wl["channels"][0]
    with solver([spec], precision=precision, obs_every=1000) as s:
        s.step(2000)
        o = oracle_channel(orc, dataclasses.replace(spec, nx=1))
        o.run(2000)
        compare_profiles(s, 0, o, FP32_TOL if precision == "fp32" else FP64_TOL, f"large {precision}")
        assert np.abs(s.observe(0, "kxx")).max() == 0.0


@pytest.mark.parametrize("drive", ["couette", "couette_zou_he", "couette_zou_he_strips", "pressure"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_other_drives_state_parity(orc, drive, precision):
    """The time-integrated stress with a moving top wall (planar Couette
    flow: the half-link wall, and Zou and He's node wall on 64-wide and
    512-wide lattices) and with the pressure drive of generalised periodic
    boundaries: random populations and stress match the oracle after 1, 2
    and 57 steps, across the switch-off at t = 40."""
    nx, ny = {"couette": (64, 9), "couette_zou_he": (64, 9), "couette_zou_he_strips": (512, 9),
              "pressure": (100, 13)}[drive]
    if drive.startswith("couette"):
        kw = dict(wall_velocity=2e-3, top_wall="zou_he" if "zou_he" in drive else "halfway")
    else:
        kw = dict(force=0.0, pressure_gradient=2e-6)
    spec = ChannelSpec(nx=nx, ny=ny, force=kw.pop("force", 0.0), tau_lb=0.8, G=2e-4, tau0=500.0, gamma_c=0.1,
                       eps=0.01, visc_split=0.3, t_startup=40, **kw)
    nnp = drive.startswith("couette")
    pops, P = workloads.random_state(nx, ny, seed=nx + ny)
    sig = workloads.random_stress(nx, ny, seed=nx + ny + 1)
    o = oracle_channel(orc, spec, nn_pressure=nnp)
    o.set_state(pops, P, t=0, S=sig)
    with solver([spec], precision=precision, obs_every=16, strip_rows=4, nn_pressure=nnp) as s:
        s.set_state(0, pops, P, 0)
        s.set_stress(0, sig)
        for n in [1, 2, 57]:
            s.step(n)
            o.run(n)
            g_pops, _ = s.get_state(0)
            err = np.abs(g_pops - o.n).max() / np.abs(o.n - workloads.REST_WEIGHTS[:, None, None]).max()
            serr = np.abs(s.get_stress(0) - o.S).max() / np.abs(o.S).max()
            print(f"{precision} {drive} t={o.t}: state {err:.2e} sigma {serr:.2e}", flush=True)
            assert err < (5e-11 if precision == "fp64" else 1e-4)
            assert serr < (1e-11 if precision == "fp64" else 1e-5)


def test_stress_calls_need_the_option():
    """lb_get_stress / lb_set_stress on a handle of the instantaneous model
    fail with LB_EINVAL and a message."""
    from paper_1310_7450_amd import Solver
    spec = ChannelSpec(nx=8, ny=8, force=1e-6, tau_lb=1.0, G=1e-4, tau0=1e3, gamma_c=0.1)
    with Solver([spec], precision="fp64") as s:
        with pytest.raises(LbError, match="instantaneous"):
            s.get_stress(0)
        with pytest.raises(LbError, match="instantaneous"):
            s.set_stress(0, np.zeros((3, 8, 8)))
