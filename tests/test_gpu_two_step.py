"""Two steps per pass over the state (FP32 storage, captured blocks of K
steps, K a multiple of 4) against one step per pass and against the FP64
oracle.

The two-step sweep keeps a strip's rows of step t on chip and applies step
t+1 to them; each node update is the one-step sweep's arithmetic, so the
states agree with one step per pass to FP32 round-off (and, where the
compiler contracts the same products into the same fused operations, bit for
bit). Shapes cover one, two, three and many column strips per row (two-step
strips are at most 248 columns, split as evenly as the width allows in
multiples of 4), ragged row bands, one- and two-row channels, the periodic
wrap of the window around the channel, and handles that mix eligible
channels with others (moving wall, Zou-He top, pressure drive, narrow
widths) whose steps still run one per pass inside the same block."""
import numpy as np
import pytest

from paper_1310_7450_amd import workloads
from paper_1310_7450_amd.lbnlm import ChannelSpec

pytestmark = pytest.mark.gpu


def solver(channels, **kw):
    from paper_1310_7450_amd import Solver
    return Solver(channels, **kw)


def spec(nx, ny, **kw):
    base = dict(force=3e-6, tau_lb=0.8, G=2e-4, tau0=500.0, gamma_c=0.1, eps=0.01, visc_split=0.3, t_startup=20)
    base.update(kw)
    return ChannelSpec(nx=nx, ny=ny, **base)


def run_pair(chans, steps, obs_every, seed=0, strip_rows=0):
    """The same seeded random states advanced by a two-step handle and a
    one-step handle; returns [(state2, state1)] per channel."""
    out = []
    states = [workloads.random_state(c.nx, c.ny, seed=seed + 17 * i) for i, c in enumerate(chans)]
    res = []
    for sps in (0, 1):
        with solver(chans, precision="fp32", obs_every=obs_every, strip_rows=strip_rows, steps_per_sweep=sps) as s:
            for i, (pops, P) in enumerate(states):
                s.set_state(i, pops, P, 0)
            for n in steps:
                s.step(n)
            res.append([s.get_state(i) for i in range(len(chans))])
    for i in range(len(chans)):
        out.append((res[0][i], res[1][i]))
    return out, states


def state_diff(a, b, pops0):
    dev = np.abs(b[0] - workloads.REST_WEIGHTS[:, None, None]).max()
    return np.abs(a[0] - b[0]).max() / dev, np.abs(a[1] - b[1]).max() / max(np.abs(b[1]).max(), 1e-30)


# a few FP32 units of the populations (2.6e-8 each near 0.44) relative to the
# state's deviation from rest (~1e-3); a wrong column, row or wall
# substitution gives O(1)
TOL = 2e-4


@pytest.mark.parametrize("nx,ny", [(256, 1), (256, 2), (512, 3), (512, 37), (768, 16), (1024, 65), (2048, 33),
                                   (4096, 24)])
def test_two_step_matches_one_step(nx, ny):
    """Random x-varying states, 2 blocks of 8 steps plus 3 single steps:
    the two-step handle's populations and traces equal the one-step
    handle's to FP32 round-off (bitwise equality reported)."""
    pairs, st = run_pair([spec(nx, ny)], [16, 3], obs_every=8, seed=nx + ny)
    (a, b), = pairs
    e, ep = state_diff(a, b, st[0][0])
    same = np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    print(f"{nx}x{ny}: two-step vs one-step state {e:.2e} P {ep:.2e} bitwise {same}", flush=True)
    assert e < TOL and ep < 1e-3


def test_two_step_mixed_handle():
    """Eligible channels beside channels that stay one step per pass
    (moving wall, Zou-He top, pressure drive, widths 64, 300 and 192) in one
    handle: every channel equals its one-step run."""
    chans = [spec(512, 20), spec(512, 12, wall_velocity=1e-3), spec(768, 9, top_wall="zou_he", nn_pressure=False),
             spec(256, 7, force=0.0, pressure_gradient=1e-6, nn_pressure=False), spec(64, 10), spec(300, 6),
             spec(1024, 30), spec(192, 5)]
    pairs, st = run_pair(chans, [8, 8, 5], obs_every=8, seed=3)
    for i, (a, b) in enumerate(pairs):
        e, ep = state_diff(a, b, st[i][0])
        print(f"channel {i} ({chans[i].nx}x{chans[i].ny}): state {e:.2e} P {ep:.2e}", flush=True)
        assert e < TOL and ep < 1e-3


def test_two_step_matches_oracle(orc):
    """Against the FP64 oracle node by node after 1 + 2 blocks of 4 steps
    (the first step one per pass, the blocks two per pass) on a 512 x 13
    channel with x gradients."""
    c = spec(512, 13)
    pops, P = workloads.random_state(512, 13, seed=5)
    o = orc.Channel(512, 13, c.force, tau_lb=c.tau_lb, G=c.G, tau0=c.tau0, gamma_c=c.gamma_c, eps=c.eps,
                    visc_split=c.visc_split, t_startup=c.t_startup, nn_pressure=True)
    o.set_state(pops, P, t=0)
    with solver([c], precision="fp32", obs_every=4) as s:
        s.set_state(0, pops, P, 0)
        for n in [3, 8, 4]:
            s.step(n)
            o.run(n)
            g, gP = s.get_state(0)
            err = np.abs(g - o.n).max() / np.abs(o.n - workloads.REST_WEIGHTS[:, None, None]).max()
            perr = np.abs(gP - o.P).max() / np.abs(o.P).max()
            print(f"t={o.t}: state {err:.2e} P {perr:.2e}", flush=True)
            assert err < 1e-4 and perr < 1e-3


@pytest.mark.parametrize("nx", [256, 768, 4096])
def test_two_step_x_uniform_stays_bitwise_uniform(nx):
    """From rest, 3 blocks of 100 steps (with the reference moves between
    blocks): every column of every row stays identical, so every lane of
    every window and every strip boundary computes the same values."""
    with solver([spec(nx, 21, t_startup=2 ** 62)], precision="fp32", obs_every=100) as s:
        s.step(300)
        pops, P = s.get_state(0)
        assert np.array_equal(pops, np.broadcast_to(pops[:, :, :1], pops.shape))
        assert np.array_equal(P, np.broadcast_to(P[:, :1], P.shape))
        assert np.abs(pops - workloads.REST_WEIGHTS[:, None, None]).max() > 0

