"""GPU parity of the stress-as-force variant (lb_options.stress_force) with
the FP64 oracle's reading R12, through the C ABI.

The divergence of the non-Newtonian stress enters as a force density. The
GPU runs a step as one fused FP64 kernel over tiles of nodes (u~ and Sigma^nN
of the tile and its halo in LDS, then collide-and-stream); observation runs
the same stages as separate node-wise passes. It agrees with the oracle to
rounding (well conditioned, G tau <= 0.2).
"""
import dataclasses

import numpy as np
import pytest

from paper_1310_7450_amd import workloads
from paper_1310_7450_amd.lbnlm import ChannelSpec, LbError

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-5
ETA_S = 1.0 / 6.0


def solver(channels, **kw):
    from paper_1310_7450_amd import Solver
    kw.setdefault("precision", "fp64")
    kw.setdefault("nn_pressure", False)
    return Solver(channels, stress_force=True, **kw)


def oracle_channel(orc, spec):
    return orc.Channel(spec.nx, spec.ny, spec.force, tau_lb=spec.tau_lb, G=spec.G, tau0=spec.tau0,
                       gamma_c=spec.gamma_c, eps=spec.eps, visc_split=spec.visc_split, t_startup=spec.t_startup,
                       nn_pressure=False, wall_velocity=spec.wall_velocity, stress_force=True)


def linf(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


@pytest.mark.parametrize("nx,ny,uw", [(1, 16, 0.0), (4, 33, 0.0), (64, 7, 0.0), (100, 37, 0.0), (8, 1, 0.0),
                                      (8, 2, 0.0), (256, 3, 0.0), (16, 12, 1e-3), (67, 5, 0.0), (68, 4, 0.0),
                                      (128, 37, 0.0), (192, 16, 1e-3), (512, 9, 0.0), (128, 1, 0.0),
                                      (128, 2, 1e-3), (64, 40, 1e-3)])
def test_perturbed_state_parity(orc, nx, ny, uw):
    """Seeded random populations on narrow, wide, odd, one- and two-row
    lattices (and some with a moving top wall): after 1, 2 and 57 steps the
    populations equal the oracle's node by node. The fused kernel's 64 x 8
    tiles wrap their two-node halo columns by a modulo below nx = 68 (67: a
    second tile of three columns) and by one add or subtract from 68 on;
    128 and wider run several tiles per row band and several bands."""
    spec = ChannelSpec(nx=nx, ny=ny, force=3e-6, tau_lb=0.8, G=2e-4, tau0=500.0, gamma_c=0.1, eps=0.01,
                       visc_split=0.3, t_startup=40, wall_velocity=uw)
    pops, P = workloads.random_state(nx, ny, seed=nx * 1000 + ny + 3)
    o = oracle_channel(orc, spec)
    o.set_state(pops, P, t=0)
    with solver([spec], obs_every=16) as s:
        s.set_state(0, pops, P, 0)
        for n in [1, 2, 57]:
            s.step(n)
            o.run(n)
            g_pops, g_P = s.get_state(0)
            err = np.abs(g_pops - o.n).max() / np.abs(o.n - workloads.REST_WEIGHTS[:, None, None]).max()
            print(f"saf {nx}x{ny} uw={uw} t={o.t}: state {err:.2e}", flush=True)
            assert err < 5e-11
            assert np.array_equal(g_P, o.P)


def test_channels_startup_steady_and_observables(orc):
    """Four x-uniform channels of different widths in one handle, from rest:
    at 300 steps and at 40,000 steps (steady) the x-averaged u_x and
    sigma_xy equal the nx = 1 oracle run, the scalars (mass, momentum, wall
    drag, u_mid) agree, and the steady profile is within 1% of the
    analytic one (Sec. III.B)."""
    from oracle import analytic
    ny, g, tau0 = 32, 2e-6, 1e3
    widths = [8, 256, 320, 100]
    specs = [ChannelSpec(nx=w, ny=ny, force=g, tau_lb=1.0, G=1e-4, tau0=tau0, gamma_c=0.1) for w in widths]
    o = oracle_channel(orc, dataclasses.replace(specs[0], nx=1))
    with solver(specs, obs_every=100) as s:
        for n in (300, 39700):
            s.step(n)
            o.run(n)
            f = o.fields()
            for i, w in enumerate(widths):
                e_u = linf(s.observe(i, "ux"), f["ux"][:, 0])
                e_s = linf(s.observe(i, "sxy"), f["sxy"][:, 0])
                print(f"saf nx={w} t={o.t}: ux {e_u:.2e} sxy {e_s:.2e}", flush=True)
                assert e_u < FP64_TOL and e_s < FP64_TOL
                assert np.abs(s.observe(i, "kxx")).max() == 0.0
                assert s.observe(i, "mass") == pytest.approx(o.mass() * w, rel=1e-12)
                assert s.observe(i, "momx") == pytest.approx(o.momentum_x() * w, rel=1e-9)
                assert s.observe(i, "wall_drag") == pytest.approx(o.wall_drag() * w, rel=1e-9)
        want = analytic.steady_profile(ny, g, ETA_S, 1e-4, tau0, 0.1)
        for i in range(len(widths)):
            assert linf(s.observe(i, "ux"), want) < 1e-2


def test_large_channel_sampled_rows(orc):
    """The 4096 x 1024 lattice, eps = -0.05, 2,000 steps from rest: the
    x-averaged rows equal an nx = 1 oracle run."""
    wl = workloads.large_channel(eps=-0.05)
    spec = wl["channels"][0]
    with solver([spec], obs_every=1000) as s:
        s.step(2000)
        o = oracle_channel(orc, dataclasses.replace(spec, nx=1))
        o.run(2000)
        f = o.fields()
        assert linf(s.observe(0, "ux"), f["ux"][:, 0]) < FP64_TOL
        assert linf(s.observe(0, "sxy"), f["sxy"][:, 0]) < FP64_TOL


def test_frozen_channel_keeps_its_state():
    """With steady_tol, the narrow channel freezes first: its state stays
    exactly the same through later steps of odd length (the fused kernel's
    workgroups skip it) while the wide one keeps stepping."""
    specs = [ChannelSpec(nx=8, ny=16, force=2e-6, tau_lb=1.0, G=1e-4, tau0=1e3, gamma_c=0.1),
             ChannelSpec(nx=100, ny=96, force=1e-6, tau_lb=1.0, G=1e-4, tau0=1e3, gamma_c=0.1)]
    with solver(specs, obs_every=200, steady_tol=1e-7) as s:
        while s.observe(0, "active") != 0:
            s.step(200)
        assert s.observe(1, "active") == 1
        t0, t1 = s.observe(0, "step"), s.observe(1, "step")
        pops0, P0 = s.get_state(0)
        wide0, _ = s.get_state(1)
        for n in (1, 2, 3):
            s.step(n)
            pops, P = s.get_state(0)
            assert np.array_equal(pops, pops0) and np.array_equal(P, P0), n
            assert s.observe(0, "step") == t0
        assert s.observe(1, "step") == t1 + 6
        assert not np.array_equal(s.get_state(1)[0], wide0)


@pytest.mark.parametrize("kw", [dict(precision="fp32"), dict(nn_pressure=True), dict(viscoelastic=True)])
def test_rejected_combinations(kw):
    """The stress force needs FP64, no flow-induced density and the
    instantaneous model; lb_create reports LB_EINVAL otherwise."""
    spec = ChannelSpec(nx=8, ny=8, force=1e-6, tau_lb=1.0, G=1e-4, tau0=1e3, gamma_c=0.1)
    with pytest.raises(LbError):
        solver([spec], **kw)


def test_rejected_with_pressure_drive():
    spec = ChannelSpec(nx=8, ny=8, force=0.0, tau_lb=1.0, G=1e-4, tau0=1e3, gamma_c=0.1, pressure_gradient=1e-6)
    with pytest.raises(LbError):
        solver([spec])
