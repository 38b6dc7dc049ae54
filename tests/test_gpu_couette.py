"""Planar Couette flow with a moving top wall (Sec. IV.B): GPU against the
oracle, through the C ABI.

The paper's moving wall is Zou and He's velocity boundary on the top node
row (Sec. II.B, last paragraph; reading R13 of the oracle): it is the wall of
the Couette workload. The half-link wall with the wall-momentum term (R9)
stays as an alternative and is checked the same way. The workload takes the
paper's Fig. stopshear parameters (theta = 100, u0 = 1e-2 L / tau_mu) in the
well-conditioned setting (viscosity split 1/2 without the delta-rho terms),
where GPU and oracle agree to round-off."""
import numpy as np
import pytest

from paper_1310_7450_amd import workloads
from paper_1310_7450_amd.lbnlm import ChannelSpec
from paper_1310_7450_amd.protocol import startup_cessation

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-5
FP32_TOL = 1e-3
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])


def solver(channels, **kw):
    from paper_1310_7450_amd import Solver
    return Solver(channels, **kw)


def oracle_channel(orc, spec, nx=None, nn_pressure=True):
    nnp = spec.nn_pressure if spec.nn_pressure is not None else nn_pressure
    return orc.Channel(spec.nx if nx is None else nx, spec.ny, spec.force, tau_lb=spec.tau_lb, G=spec.G,
                       tau0=spec.tau0, gamma_c=spec.gamma_c, eps=spec.eps, visc_split=spec.visc_split,
                       t_startup=spec.t_startup, nn_pressure=nnp, wall_velocity=spec.wall_velocity,
                       top_wall=spec.top_wall)


def momentum(n):
    return float((CX[:, None, None] * n).sum())


@pytest.mark.parametrize("top_wall", ["zou_he", "halfway"])
@pytest.mark.parametrize("nx,ny", [(1, 16), (8, 9), (64, 7), (100, 13), (128, 9), (192, 5), (256, 6), (512, 11),
                                   (3, 1), (4, 2)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_couette_state_parity(orc, nx, ny, precision, top_wall):
    """Seeded random populations with the top wall moving (u_w = 0.02) and
    stopping at t = 40, on narrow, aligned-wide (FP64 tiles, FP32 vector
    strips of 256 columns, 2 of them at 512), ragged-wide and one- or two-row
    lattices: the state set at t0 = 5 and advanced across the switch matches
    the oracle node by node. The wall drag after each single step equals the
    oracle's momentum budget M(t) + N f - M(t+1) (FP64)."""
    if top_wall == "zou_he" and ny < 2:
        pytest.skip("a Zou-He wall needs two rows")
    spec = ChannelSpec(nx=nx, ny=ny, force=1e-6, tau_lb=0.8, G=2e-4, tau0=500.0, gamma_c=0.1, eps=0.01,
                       visc_split=0.3, t_startup=40, wall_velocity=0.02, top_wall=top_wall)
    pops, P = workloads.random_state(nx, ny, seed=7000 + nx * 100 + ny)
    o = oracle_channel(orc, spec)
    o.set_state(pops, P, t=5)
    tol = 1e-12 if precision == "fp64" else 2e-6
    with solver([spec], precision=precision, obs_every=16, strip_rows=4) as s:
        s.set_state(0, pops, P, 5)
        g_pops, _ = s.get_state(0)
        # a Zou-He wall completes what enters its row from above: compare with
        # the oracle's completed state
        assert np.abs(g_pops - o.n).max() <= (1e-16 if precision == "fp64" else 1e-7)
        for n in [1, 2, 57]:
            if n > 1:
                s.step(n - 1)
                o.run(n - 1)
            m0, f0 = momentum(o.n), o.force_now()
            s.step(1)
            o.run(1)
            g_pops, g_P = s.get_state(0)
            err = np.abs(g_pops - o.n).max() / np.abs(o.n - workloads.REST_WEIGHTS[:, None, None]).max()
            print(f"{precision} {top_wall} {nx}x{ny} t={o.t}: state {err:.2e}", flush=True)
            assert err < tol * 50
            if precision == "fp64":
                drag = s.observe(0, "wall_drag")
                budget = m0 + nx * ny * f0 - momentum(o.n)
                assert drag == pytest.approx(budget, rel=1e-9, abs=1e-15)
                if top_wall == "halfway":
                    assert drag == pytest.approx(o.wall_drag(), rel=1e-9, abs=1e-15)


def plug_rows(u):
    """Rows within 1% of the maximum velocity: the paper's indicator of the
    plug width (Fig. stopprofiles)."""
    return int((u >= 0.99 * u.max()).sum())


@pytest.mark.parametrize("top_wall", ["zou_he", "halfway"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_couette_startup_cessation(orc, precision, top_wall):
    """The Couette workload (8 x 64, theta = 100, Pe = 10): the profile
    through start-up and cessation equals an nx = 1 oracle run; the steady
    start-up profile is the linear one between the fixed half-way wall and
    the moving wall; after the wall stops an intermediate plug forms at the
    formerly moving wall and moves into the channel (its 1%-of-maximum width
    at least twice that of the solvent alone at the same times, the plug
    reaching to within 20 rows of the wall 100 steps after the stop and its
    maximum moving down); and u_mid falls
    below 1e-2 of its value at the switch-off within the Bingham energy
    bound evaluated on the oracle's profile (Pe >= 10)."""
    from oracle import analytic
    wl = workloads.couette_64(top_wall=top_wall)
    spec = wl["channels"][0]
    L = wl["width"]
    ts = wl["startup"]
    tol = FP64_TOL * 1e-4 if precision == "fp64" else FP32_TOL
    o = oracle_channel(orc, spec, nx=1)
    newt = oracle_channel(orc, workloads.couette_64(newtonian=True, top_wall=top_wall)["channels"][0], nx=1)
    checkpoints = [ts // 2, ts, ts + 100, ts + 500, ts + 1000, ts + 2000]
    with solver([spec], precision=precision, obs_every=100) as s:
        argmax, plug_top = [], []
        for t in checkpoints:
            s.step(t - int(s.observe(0, "step")))
            o.run(t - o.t)
            newt.run(t - newt.t)
            ug, uo = s.observe(0, "ux"), o.profiles()["ux"]
            e = np.abs(ug - uo).max() / spec.wall_velocity
            print(f"{precision} {top_wall} t={t}: u_x err {e:.2e} (of u0); plug rows {plug_rows(ug)} "
                  f"(solvent alone {plug_rows(newt.profiles()['ux'])}); argmax {int(ug.argmax())}", flush=True)
            assert e <= tol
            if t == ts:
                # the state at the switch-off; a Zou-He wall row already
                # carries the stopped wall's velocity of this step
                fluid = spec.ny - (1 if top_wall == "zou_he" else 0)
                lin = spec.wall_velocity * (np.arange(fluid) + 0.5) / L
                assert np.abs(ug[:fluid] - lin).max() / spec.wall_velocity < 1e-3
                if top_wall == "zou_he":
                    assert abs(ug[-1]) < 1e-15
                u_ts_oracle = uo.copy()
            if t > ts:
                argmax.append(int(ug.argmax()))
                plug_top.append(int(np.nonzero(ug >= 0.99 * ug.max())[0].max()))
            if t in (ts + 500, ts + 1000):
                assert plug_rows(ug) >= 2 * plug_rows(newt.profiles()["ux"])
        assert plug_top[0] >= spec.ny - 20
        assert all(a >= b for a, b in zip(argmax, argmax[1:]))
    eta_s = (spec.tau_lb - 0.5) / 3.0
    bound = analytic.bingham_stop_bound(u_ts_oracle, eta_s, spec.G * spec.gamma_c, spec.ny, width=L)
    pe = (spec.wall_velocity / L) * spec.tau0 / spec.gamma_c
    with solver([spec], precision=precision, obs_every=100) as s:
        res = startup_cessation(s, ts, wl["cessation"], every=100, thresholds=(1e-2, 1e-3))
    t_stop = res[0]["t_stop"]
    print(f"{precision} {top_wall}: t_stop {t_stop}, Bingham bound {bound:.0f}, Pe {pe:.1f}", flush=True)
    assert pe >= 10 * 0.99 and t_stop[1e-2] is not None and t_stop[1e-2] <= bound
