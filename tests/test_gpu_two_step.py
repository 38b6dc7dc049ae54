"""Two steps per pass over the state (captured blocks of K steps, K a
multiple of 4) against one step per pass and against the FP64 oracle, in
FP32 (reference-shifted storage) and FP64, at two nodes per lane and, for
FP32 states larger than the last-level cache (streamed with nontemporal
stores) with the instantaneous stress, four.

The two-step sweep keeps a strip's rows of step t on chip and applies step
t+1 to them; each node update is the one-step sweep's arithmetic, so the
states agree with one step per pass to round-off (and, where the compiler
contracts the same products into the same fused operations, bit for bit).
Shapes cover one, two, three and many column strips per row (two-step strips
are at most 124 columns at two nodes per lane and 248 at four, split as
evenly as the width allows in multiples of the nodes per lane), ragged row
bands, states of either size, one- and
two-row channels, the periodic wrap of the window around the channel, and
handles that mix eligible channels with others (pressure drive, other
widths) whose steps still run one per pass inside the same block (in FP64 on
the tile sweep). Moving half-way walls and Zou-He tops run two steps per pass
too, with the wall switched off between the two steps of a launch.

The narrow widths (1, 2, 4, ..., 64: a row in nx lanes, 64 / nx rows per
wavefront) take two steps per pass in their own kernel, which keeps whole
row groups of step t in a ring; their shapes cover every width, strips of a
few groups and of one, channels shorter than a group and ragged last
groups."""
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


def run_pair(chans, steps, obs_every, seed=0, strip_rows=0, precision="fp32"):
    """The same seeded random states advanced by a two-step handle and a
    one-step handle; returns [(state2, state1)] per channel."""
    out = []
    states = [workloads.random_state(c.nx, c.ny, seed=seed + 17 * i) for i, c in enumerate(chans)]
    res = []
    for sps in (0, 1):
        with solver(chans, precision=precision, obs_every=obs_every, strip_rows=strip_rows,
                    steps_per_sweep=sps) as s:
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


# FP32: a few units of the populations (2.6e-8 each near 0.44) relative to
# the state's deviation from rest (~1e-3); FP64: the same in FP64 units. A
# wrong column, row or wall substitution gives O(1)
TOL = {"fp32": (2e-4, 1e-3), "fp64": (1e-11, 1e-9)}
# against the oracle, whose rounding order differs: the perturbed-state
# parity bound (random states amplify round-off over a few tens of steps)
ORACLE_TOL = {"fp32": (1e-4, 1e-3), "fp64": (5e-11, 1e-9)}

# (1024, 6600) in FP32 and (1024, 3300) in FP64 exceed 256 MB per state
# buffer: streamed, FP32 at four nodes per lane
SHAPES = {"fp32": [(256, 1), (256, 2), (512, 3), (512, 37), (768, 16), (1024, 65), (2048, 33), (4096, 24),
                   (1024, 6600)],
          "fp64": [(128, 1), (128, 2), (192, 3), (320, 37), (256, 16), (1024, 65), (4096, 24), (1024, 3300)]}
NARROW = [(1, 40), (1, 3), (2, 33), (4, 17), (8, 511), (8, 1), (8, 6), (16, 9), (16, 200), (32, 70), (32, 2),
          (64, 5), (64, 130)]


@pytest.mark.parametrize("precision,nx,ny", [(p, nx, ny) for p in SHAPES for nx, ny in SHAPES[p] + NARROW])
def test_two_step_matches_one_step(precision, nx, ny):
    """Random x-varying states, 2 blocks of 8 steps plus 3 single steps:
    the two-step handle's populations and traces equal the one-step
    handle's to round-off (bitwise equality reported)."""
    pairs, st = run_pair([spec(nx, ny)], [16, 3], obs_every=8, seed=nx + ny, precision=precision)
    (a, b), = pairs
    e, ep = state_diff(a, b, st[0][0])
    same = np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    print(f"{precision} {nx}x{ny}: two-step vs one-step state {e:.2e} P {ep:.2e} bitwise {same}", flush=True)
    assert e < TOL[precision][0] and ep < TOL[precision][1]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_two_step_mixed_handle(precision):
    """Two-step channels (plain, with a moving wall, with a Zou-He top,
    narrow ones of widths 64 and 8) beside channels that stay one step per
    pass (pressure drive, widths 300 and 192 in FP32; 300 is tiled in FP64)
    in one handle: every channel equals its one-step run."""
    chans = [spec(512, 20), spec(512, 12, wall_velocity=1e-3), spec(768, 9, top_wall="zou_he", nn_pressure=False),
             spec(256, 7, force=0.0, pressure_gradient=1e-6, nn_pressure=False), spec(64, 10), spec(300, 6),
             spec(1024, 30), spec(192, 5), spec(8, 21, wall_velocity=1e-3), spec(8, 9),
             spec(16, 4, force=0.0, pressure_gradient=1e-6, nn_pressure=False)]
    pairs, st = run_pair(chans, [8, 8, 5], obs_every=8, seed=3, precision=precision)
    for i, (a, b) in enumerate(pairs):
        e, ep = state_diff(a, b, st[i][0])
        print(f"{precision} channel {i} ({chans[i].nx}x{chans[i].ny}): state {e:.2e} P {ep:.2e}", flush=True)
        assert e < TOL[precision][0] and ep < TOL[precision][1]


@pytest.mark.parametrize("precision,big", [("fp32", (1024, 6600)), ("fp64", (1024, 3300))])
def test_two_step_streamed_walls(orc, precision, big):
    """A channel large enough to make the state streamed (above 256 MB per
    buffer: FP32 then runs four nodes per lane) beside channels with a
    moving half-way top wall and a Zou-He top, switched off at t = 19
    (inside a two-step launch): every channel equals its one-step run, and
    the wall channels equal the FP64 oracle node by node."""
    kw = dict(wall_velocity=1e-3, t_startup=19, nn_pressure=False)
    chans = [spec(*big), spec(512, 15, **kw), spec(512, 15, top_wall="zou_he", **kw)]
    pairs, st = run_pair(chans, [24, 3], obs_every=8, seed=21, precision=precision)
    for i, (a, b) in enumerate(pairs):
        e, ep = state_diff(a, b, st[i][0])
        print(f"{precision} channel {i} ({chans[i].nx}x{chans[i].ny}): state {e:.2e} P {ep:.2e}", flush=True)
        assert e < TOL[precision][0] and ep < TOL[precision][1]
    for i in (1, 2):
        c = chans[i]
        o = orc.Channel(c.nx, c.ny, c.force, tau_lb=c.tau_lb, G=c.G, tau0=c.tau0, gamma_c=c.gamma_c, eps=c.eps,
                        visc_split=c.visc_split, t_startup=c.t_startup, nn_pressure=False,
                        wall_velocity=c.wall_velocity, top_wall=c.top_wall)
        o.set_state(*st[i], t=0)
        o.run(27)
        eo = np.abs(pairs[i][0][0] - o.n).max() / np.abs(o.n - workloads.REST_WEIGHTS[:, None, None]).max()
        print(f"{precision} {c.top_wall} wall beside a streamed state: vs oracle {eo:.2e}", flush=True)
        assert eo < ORACLE_TOL[precision][0]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_two_step_many_narrow_channels(precision):
    """More narrow channels than the GPU holds two-step workgroups at once
    (1,600 channels of every narrow width, 1 to 7 rows, a few with a moving
    wall), so that every channel is one strip and the strips run in several
    rounds: each channel equals its one-step run."""
    widths = [1, 2, 4, 8, 16, 32, 64]
    chans = [spec(widths[i % 7], 1 + (i * 5) % 7, **({"wall_velocity": 1e-3} if i % 97 == 0 else {}))
             for i in range(1600)]
    pairs, st = run_pair(chans, [8, 4], obs_every=4, seed=11, precision=precision)
    worst = (0.0, 0.0)
    for i, (a, b) in enumerate(pairs):
        e, ep = state_diff(a, b, st[i][0])
        worst = (max(worst[0], e), max(worst[1], ep))
        assert e < TOL[precision][0] and ep < TOL[precision][1], (i, chans[i].nx, chans[i].ny, e, ep)
    print(f"{precision} 1600 narrow channels: worst state {worst[0]:.2e} P {worst[1]:.2e}", flush=True)


@pytest.mark.parametrize("precision,nx", [("fp32", 512), ("fp64", 320), ("fp32", 16), ("fp64", 8), ("fp32", 64)])
def test_two_step_matches_oracle(orc, precision, nx):
    """Against the FP64 oracle node by node after 3 single steps and 3
    blocks of 4 (the blocks two steps per pass) on a channel of 13 rows
    with x gradients."""
    c = spec(nx, 13)
    pops, P = workloads.random_state(nx, 13, seed=5)
    o = orc.Channel(nx, 13, c.force, tau_lb=c.tau_lb, G=c.G, tau0=c.tau0, gamma_c=c.gamma_c, eps=c.eps,
                    visc_split=c.visc_split, t_startup=c.t_startup, nn_pressure=True)
    o.set_state(pops, P, t=0)
    tol = ORACLE_TOL[precision]
    with solver([c], precision=precision, obs_every=4) as s:
        s.set_state(0, pops, P, 0)
        for n in [3, 8, 4]:
            s.step(n)
            o.run(n)
            g, gP = s.get_state(0)
            err = np.abs(g - o.n).max() / np.abs(o.n - workloads.REST_WEIGHTS[:, None, None]).max()
            perr = np.abs(gP - o.P).max() / np.abs(o.P).max()
            print(f"{precision} t={o.t}: state {err:.2e} P {perr:.2e}", flush=True)
            assert err < tol[0] and perr < tol[1]


@pytest.mark.parametrize("precision,nx", [("fp32", 256), ("fp32", 768), ("fp32", 4096), ("fp64", 128),
                                          ("fp64", 320), ("fp64", 4096), ("fp32", 8), ("fp64", 64),
                                          ("fp32", 327680)])
def test_two_step_x_uniform_stays_bitwise_uniform(precision, nx):
    """From rest, 3 blocks of 100 steps (with the reference moves between
    blocks in FP32): every column of every row stays identical, so every lane
    of every window and every strip boundary computes the same values."""
    with solver([spec(nx, 21, t_startup=2 ** 62)], precision=precision, obs_every=100) as s:
        s.step(300)
        pops, P = s.get_state(0)
        assert np.array_equal(pops, np.broadcast_to(pops[:, :, :1], pops.shape))
        assert np.array_equal(P, np.broadcast_to(P[:, :1], P.shape))
        assert np.abs(pops - workloads.REST_WEIGHTS[:, None, None]).max() > 0



@pytest.mark.parametrize("precision,nx,ny", [("fp32", 512, 19), ("fp32", 256, 2), ("fp32", 1024, 40),
                                             ("fp32", 1024, 6600), ("fp64", 192, 19), ("fp64", 128, 1),
                                             ("fp64", 512, 40)])
def test_two_step_viscoelastic_matches_one_step(precision, nx, ny):
    """The time-integrated stress: the stored stress sigma(t) rides in the
    ring beside the populations. From seeded random populations and a seeded
    random stress, 2 blocks of 8 steps plus 3 single steps: populations,
    traces and stresses equal the one-step handle's to round-off."""
    c = spec(nx, ny, G=1e-4, tau0=1e3)
    pops, P = workloads.random_state(nx, ny, seed=nx + 3 * ny)
    rng = np.random.default_rng(nx * ny)
    sig = 1e-6 * rng.standard_normal((3, ny, nx))
    res = []
    for sps in (0, 1):
        with solver([c], precision=precision, obs_every=8, steps_per_sweep=sps, viscoelastic=True) as s:
            s.set_state(0, pops, P, 0)
            s.set_stress(0, sig)
            s.step(16)
            s.step(3)
            res.append((s.get_state(0), s.get_stress(0)))
    (a, sa), (b, sb) = res
    e, ep = state_diff(a, b, pops)
    es = np.abs(sa - sb).max() / np.abs(sb).max()
    print(f"{precision} VE {nx}x{ny}: state {e:.2e} P {ep:.2e} stress {es:.2e}", flush=True)
    assert e < TOL[precision][0] and ep < TOL[precision][1]
    assert es < (1e-4 if precision == "fp32" else 1e-11)


@pytest.mark.parametrize("precision,nx", [("fp32", 512), ("fp64", 192), ("fp32", 8), ("fp64", 32), ("fp32", 64)])
@pytest.mark.parametrize("wall", ["moving", "zou_he"])
def test_two_step_walls_match_one_step_and_oracle(orc, precision, nx, wall):
    """A moving top wall (half-way, u_w = 1e-3) or a Zou-He top moving at
    u_w, switched off at t = 19 (inside a launch: step 18 with the wall, 19
    without): the two-step handle equals the one-step handle to round-off
    and the FP64 oracle within the FP32 or FP64 tolerance, node by node."""
    kw = dict(wall_velocity=1e-3, t_startup=19, nn_pressure=False)
    if wall == "zou_he":
        kw["top_wall"] = "zou_he"
    c = spec(nx, 15, **kw)
    pops, P = workloads.random_state(nx, 15, seed=nx + len(wall))
    res = []
    for sps in (0, 1):
        with solver([c], precision=precision, obs_every=8, steps_per_sweep=sps) as s:
            s.set_state(0, pops, P, 0)
            s.step(24)
            s.step(3)
            res.append(s.get_state(0))
    e, ep = state_diff(res[0], res[1], pops)
    o = orc.Channel(nx, 15, c.force, tau_lb=c.tau_lb, G=c.G, tau0=c.tau0, gamma_c=c.gamma_c, eps=c.eps,
                    visc_split=c.visc_split, t_startup=c.t_startup, nn_pressure=False, wall_velocity=c.wall_velocity,
                    top_wall=c.top_wall)
    o.set_state(pops, P, t=0)
    o.run(27)
    eo = np.abs(res[0][0] - o.n).max() / np.abs(o.n - workloads.REST_WEIGHTS[:, None, None]).max()
    print(f"{precision} {wall} {nx}: two-step vs one-step {e:.2e} (P {ep:.2e}), vs oracle {eo:.2e}", flush=True)
    assert e < TOL[precision][0] and ep < TOL[precision][1]
    assert eo < ORACLE_TOL[precision][0]
