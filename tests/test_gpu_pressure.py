"""Pressure-driven channels (generalised periodic boundaries, Sec. II.B):
GPU against the oracle, through the C ABI. The inlet/outlet column pass
runs after every sweep; every kernel class meets it at the period's ends."""
import numpy as np
import pytest

from paper_1310_7450_amd import workloads
from paper_1310_7450_amd.lbnlm import ChannelSpec

pytestmark = pytest.mark.gpu

CS2 = 1.0 / 3.0


def solver(channels, **kw):
    from paper_1310_7450_amd import Solver
    return Solver(channels, **kw)


def oracle_channel(orc, spec):
    return orc.Channel(spec.nx, spec.ny, spec.force, tau_lb=spec.tau_lb, G=spec.G, tau0=spec.tau0,
                       gamma_c=spec.gamma_c, eps=spec.eps, visc_split=spec.visc_split, t_startup=spec.t_startup,
                       nn_pressure=False, pressure_gradient=spec.pressure_gradient)


@pytest.mark.parametrize("nx,ny", [(2, 9), (8, 16), (64, 7), (100, 13), (128, 9), (192, 5), (256, 6), (5, 1)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_pressure_state_parity(orc, nx, ny, precision):
    """Seeded random populations (every moment non-zero, x gradients) with
    the pressure drop on until t = 40, then held at zero: the state matches
    the oracle node by node on narrow, aligned-wide and ragged-wide lattices
    and a one-row channel."""
    spec = ChannelSpec(nx=nx, ny=ny, force=0.0, tau_lb=0.8, G=2e-4, tau0=500.0, gamma_c=0.1, eps=0.01,
                       visc_split=0.3, t_startup=40, pressure_gradient=1e-5)
    pops, P = workloads.random_state(nx, ny, seed=9000 + nx * 100 + ny)
    o = oracle_channel(orc, spec)
    o.set_state(pops, P, t=0)
    tol = 1e-12 if precision == "fp64" else 2e-6
    with solver([spec], precision=precision, obs_every=16, strip_rows=4, nn_pressure=False) as s:
        s.set_state(0, pops, P, 0)
        for n in [1, 2, 57]:
            s.step(n)
            o.run(n)
            g_pops, _ = s.get_state(0)
            err = np.abs(g_pops - o.n).max() / np.abs(o.n - workloads.REST_WEIGHTS[:, None, None]).max()
            print(f"{precision} {nx}x{ny} t={o.t}: state {err:.2e}", flush=True)
            assert err < tol * 50


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_pressure_channel_steady(orc, precision):
    """The pressure-driven nlM channel from the linear-density start: the
    x-averaged u_x and sigma_xy equal the oracle's on the same lattice
    (FP64 1e-5, FP32 1e-3 relative), and on the GPU's own state the pressure
    falls along the channel at G_p while on every cut at constant x
    cs2 rho + N1/2 is uniform across y (Fig. channelsigma, lower panel)."""
    wl = workloads.pressure_channel(nx=16, ny=32)
    spec = wl["channels"][0]
    pops, P = workloads.linear_density_state(spec)
    o = oracle_channel(orc, spec)
    o.set_state(pops, P, t=0)
    o.run(30000)
    tol = 1e-5 if precision == "fp64" else 1e-3
    with solver([spec], precision=precision, obs_every=1000, nn_pressure=False) as s:
        s.set_state(0, pops, P, 0)
        s.step(30000)
        po = o.profiles()
        for f in ("ux", "sxy"):
            e = np.abs(s.observe(0, f) - po[f]).max() / np.abs(po[f]).max()
            print(f"{precision} {f}: Linf rel {e:.2e}", flush=True)
            assert e < tol
        g_pops, _ = s.get_state(0)
        rho = g_pops.sum(axis=0)
        n1 = s.observe(0, "n1")
    p = CS2 * rho
    spread = n1.max() - n1.min()
    for x in (0, spec.nx // 2, spec.nx - 1):
        tot = p[:, x] + n1 / 2
        assert tot.max() - tot.min() < 0.1 * spread / 2
    assert p[:, 0].mean() - p[:, -1].mean() == pytest.approx(spec.pressure_gradient * (spec.nx - 1), rel=1e-2)
