"""lb_observe_noalloc, the allocation-free observation (its scratch in a
per-GPU static device array instead of the handle's workspace), against
lb_observe through the C ABI: every profile and scalar of every channel
equal, on two calls in a row whose second handle is smaller than the first
(the shared array keeps the first call's contents), and the documented
rejections."""
import numpy as np
import pytest

from paper_1310_7450_amd import workloads
from paper_1310_7450_amd.lbnlm import PROFILES, SCALARS, ChannelSpec, LbError

pytestmark = pytest.mark.gpu


def solver(channels, **kw):
    from paper_1310_7450_amd import Solver
    return Solver(channels, **kw)


def compare_all(s):
    for ch in range(len(s.channels)):
        for what in list(PROFILES) + list(SCALARS):
            a = s.observe(ch, what)
            b = s.observe_noalloc(ch, what)
            assert np.array_equal(np.asarray(a), np.asarray(b)), (ch, what, a, b)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_observation_equals_observe(precision):
    big = [ChannelSpec(512, 9, 2e-6, 0.8, 2e-4, 500.0, 0.1, 0.01, 0.3, t_startup=40),
           ChannelSpec(8, 40, 1e-6, 1.0, 1e-4, 1e3, 0.1),
           ChannelSpec(100, 13, 1e-6, 0.9, 1e-4, 1e3, 0.1, -0.02, 0.0),
           ChannelSpec(64, 9, 0.0, 0.8, 2e-4, 500.0, 0.1, wall_velocity=0.02, top_wall="zou_he",
                       nn_pressure=False, visc_split=0.3)]
    with solver(big, precision=precision, obs_every=100, steady_tol=1e-12) as s:
        for i, c in enumerate(big):
            pops, P = workloads.random_state(c.nx, c.ny, seed=50 + i)
            s.set_state(i, pops, P, 0)
        s.step(250)
        print(f"{precision}: first handle, 4 channels", flush=True)
        compare_all(s)
    small = [ChannelSpec(4, 16, 3e-6, 1.0, 1e-4, 1e3, 0.1)]
    with solver(small, precision=precision, obs_every=100) as s:
        s.step(37)
        print(f"{precision}: second handle, 1 channel of 4 x 16", flush=True)
        compare_all(s)


def test_noalloc_rejections():
    tall = [ChannelSpec(8, 2_000_000, 1e-7, 1.0, 1e-4, 1e3, 0.1)]
    with solver(tall, precision="fp32") as s:
        with pytest.raises(LbError, match="scratch") as e:
            s.observe_noalloc(0, "ux")
        assert e.value.status == -1
        assert s.observe_noalloc(0, "step") == 0.0
    saf = [ChannelSpec(64, 8, 1e-6, 1.0, 1e-4, 1e3, 0.1, nn_pressure=False)]
    with solver(saf, precision="fp64", stress_force=True) as s:
        with pytest.raises(LbError, match="stress-force") as e:
            s.observe_noalloc(0, "ux")
        assert e.value.status == -1
