"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances: FP64 storage within 1e-5 relative L-infinity on u_x and sigma_xy
(expected ~1e-12: the two sides differ only in rounding order; the stress
comes from a closed-form solve on the GPU and from summing the series in the
oracle), FP32 shifted storage within 1e-3. L-infinity relative means
max|a - b| / max|b| over the field.

Element-wise parity needs a well-conditioned run. With the explicit stress,
the scheme amplifies round-off without bound once G tau (lattice units)
exceeds about 0.3 at visc_split 0: the 8 x 64, G tau = 1 channel turns a
1e-15 perturbation of the oracle into a 27% change of its own state within
500 steps. Long parity runs therefore use G tau <= 0.2; the G tau = 1
workload is compared exactly over its first steps and statistically after.
"""
import dataclasses

import numpy as np
import pytest

from paper_1310_7450_amd import workloads
from paper_1310_7450_amd.lbnlm import ChannelSpec

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-5
FP32_TOL = 1e-3


def solver(channels, **kw):
    from paper_1310_7450_amd import Solver
    return Solver(channels, **kw)


def linf(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def oracle_channel(orc, spec, nn_pressure=True):
    nnp = spec.nn_pressure if spec.nn_pressure is not None else nn_pressure
    return orc.Channel(spec.nx, spec.ny, spec.force, tau_lb=spec.tau_lb, G=spec.G, tau0=spec.tau0,
                       gamma_c=spec.gamma_c, eps=spec.eps, visc_split=spec.visc_split,
                       t_startup=spec.t_startup, nn_pressure=nnp, wall_velocity=spec.wall_velocity,
                       top_wall=spec.top_wall)


def compare_fields(s, ch, o, tol, label):
    f = o.fields()
    ux_o, sxy_o = f["ux"].mean(axis=1), f["sxy"].mean(axis=1)
    ux_g, sxy_g = s.observe(ch, "ux"), s.observe(ch, "sxy")
    e_u, e_s = linf(ux_g, ux_o), linf(sxy_g, sxy_o)
    print(f"{label}: Linf rel u_x {e_u:.3e}  sigma_xy {e_s:.3e}", flush=True)
    assert e_u <= tol, (label, e_u)
    if np.abs(sxy_o).max() > 0:
        assert e_s <= tol, (label, e_s)
    return e_u, e_s


def test_poiseuille_fp64_state_parity(orc):
    """The 8 x 64 start-up/cessation channel at G tau = 0.2, FP64: full
    population state and previous trace equal the oracle's during start-up,
    at the switch-off and during cessation."""
    wl = workloads.poiseuille_64(tau0=2e3)
    spec = wl["channels"][0]
    o = oracle_channel(orc, spec)
    dev = pdev = 0.0
    with solver([spec], precision="fp64", obs_every=1000) as s:
        for n in [3000, 17000, 20000]:
            s.step(n)
            o.run(n)
            pops, P = s.get_state(0)
            # normalise by the largest deviation from rest seen so far (the
            # fluid is nearly at rest again after the cessation)
            dev = max(dev, np.abs(o.n - workloads.REST_WEIGHTS[:, None, None]).max())
            err = np.abs(pops - o.n).max() / dev
            print(f"t={o.t}: state rel err {err:.3e}  P err {np.abs(P - o.P).max():.3e}", flush=True)
            assert err < 1e-9
            pdev = max(pdev, np.abs(o.P).max())
            assert np.abs(P - o.P).max() <= 1e-9 * pdev
            if o.t <= 20000:
                compare_fields(s, 0, o, FP64_TOL, f"fp64 t={o.t}")


def test_poiseuille_newtonian_fp64(orc):
    spec = workloads.poiseuille_64(newtonian=True)["channels"][0]
    o = oracle_channel(orc, spec)
    with solver([spec], precision="fp64") as s:
        s.step(25000)
        o.run(25000)
        compare_fields(s, 0, o, FP64_TOL, "newtonian")


def test_poiseuille_fp32_shifted(orc):
    """FP32 shifted storage through start-up and into cessation; during the
    cessation the error is measured against the largest velocity and stress
    of the run (the fields decay towards zero)."""
    spec = workloads.poiseuille_64(tau0=2e3)["channels"][0]
    o = oracle_channel(orc, spec)
    umax = smax = 0.0
    with solver([spec], precision="fp32") as s:
        for n in [5000, 15000, 2000, 18000]:
            s.step(n)
            o.run(n)
            pr = o.profiles()
            umax = max(umax, np.abs(pr["ux"]).max())
            smax = max(smax, np.abs(pr["sxy"]).max())
            eu = np.abs(s.observe(0, "ux") - pr["ux"]).max() / umax
            es = np.abs(s.observe(0, "sxy") - pr["sxy"]).max() / smax
            print(f"fp32 t={o.t}: u_x err {eu:.3e} sigma_xy err {es:.3e} (of run max)", flush=True)
            assert eu < FP32_TOL and es < FP32_TOL


@pytest.mark.parametrize("nx,ny", [(1, 16), (2, 9), (4, 33), (16, 20), (64, 7), (3, 12), (100, 37), (130, 5), (63, 2),
                                   (8, 1), (128, 9), (192, 5), (256, 3), (128, 1), (384, 2), (65, 6), (66, 3),
                                   (512, 9), (768, 11)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_perturbed_state_parity(orc, nx, ny, precision):
    """Seeded random populations (every moment non-zero, x gradients present)
    on narrow, aligned-wide (nx a multiple of 64), ragged-wide and odd
    lattices: one and several steps match the oracle node by node; covers the
    lane-group wrap, the edge columns and halo of wide strips, the periodic
    wrap across strips, partial last strips, and one/two-row channels. In
    FP64 the widths that are not powers of two run on 64 x 8 tiles: 3, 63
    and 65 wrap their halo columns by a modulo (65: a second tile of one
    column), 66 and up by one add or subtract, and 100, 130 end in a
    partial tile. In FP32, 512 and 768 run two and three 256-column vector
    strips per row band, with strips of 4 rows stacked four to a workgroup
    and every other band marching the other way, so the x halo between
    strips and the flipped marches meet a state with x gradients."""
    spec = ChannelSpec(nx=nx, ny=ny, force=3e-6, tau_lb=0.8, G=2e-4, tau0=500.0, gamma_c=0.1,
                       eps=0.01, visc_split=0.3, t_startup=40)
    pops, P = workloads.random_state(nx, ny, seed=nx * 1000 + ny)
    o = oracle_channel(orc, spec)
    o.set_state(pops, P, t=0)
    tol = 1e-12 if precision == "fp64" else 2e-6
    with solver([spec], precision=precision, obs_every=16, strip_rows=4) as s:
        s.set_state(0, pops, P, 0)
        g_pops, g_P = s.get_state(0)
        assert np.abs(g_pops - pops).max() <= (0 if precision == "fp64" else 1e-7)
        for n in [1, 2, 57]:
            s.step(n)
            o.run(n)
            g_pops, g_P = s.get_state(0)
            err = np.abs(g_pops - o.n).max() / np.abs(o.n - workloads.REST_WEIGHTS[:, None, None]).max()
            perr = np.abs(g_P - o.P).max() / max(np.abs(o.P).max(), 1e-30)
            print(f"{precision} {nx}x{ny} t={o.t}: state {err:.2e} P {perr:.2e}", flush=True)
            assert err < tol * 50 and perr < (1e-9 if precision == "fp64" else 1e-3)


def test_batched_channels_match_individual_oracles(orc):
    """Channels of different shapes and parameters in one handle advance
    exactly as separate oracle runs (no cross-talk between channels)."""
    specs = [
        ChannelSpec(8, 48, 1e-6, 1.0, 1e-4, 1e3, 0.1, 0.0, 0.0),
        ChannelSpec(8, 33, 2e-6, 0.9, 5e-5, 2e3, 0.1, -0.03, 0.0, t_startup=700),
        ChannelSpec(100, 20, 1e-6, 1.0, 1e-4, 1e3, 0.1, 0.02, 0.25),
        ChannelSpec(4, 64, 5e-7, 1.0, 0.0, 1e4, 0.1),
        ChannelSpec(64, 12, 1e-6, 1.2, 1e-4, 1.5e3, 0.2, 0.0, 0.5),
    ]
    oracles = [oracle_channel(orc, sp) for sp in specs]
    with solver(specs, precision="fp64", obs_every=200) as s:
        s.step(1500)
        for i, o in enumerate(oracles):
            o.run(1500)
            pops, P = s.get_state(i)
            err = np.abs(pops - o.n).max() / np.abs(o.n - workloads.REST_WEIGHTS[:, None, None]).max()
            print(f"channel {i}: state rel err {err:.2e}", flush=True)
            assert err < 1e-9
            compare_fields(s, i, o, FP64_TOL, f"batched ch{i}")


def test_observables_match_oracle(orc):
    """Profiles and channel totals (pressure, N1, kappa_xy, mass, momentum,
    wall drag, centre velocity) agree with the oracle's."""
    spec = ChannelSpec(8, 40, 2e-6, 1.0, 1e-4, 1e3, 0.1)
    o = oracle_channel(orc, spec)
    with solver([spec], precision="fp64") as s:
        s.step(3001)
        o.run(3001)
        f = o.fields()
        pr = {k: v.mean(axis=1) for k, v in f.items()}
        assert linf(s.observe(0, "n1"), pr["sxx"] - pr["syy"]) < 1e-9
        assert linf(s.observe(0, "pressure"), pr["rho_e"] / 3) < 1e-14
        assert linf(s.observe(0, "kxy"), pr["kxy"]) < 1e-9
        assert linf(s.observe(0, "trT"), pr["trT"]) < 1e-9
        assert s.observe(0, "mass") == pytest.approx(o.mass(), rel=1e-14)
        assert s.observe(0, "momx") == pytest.approx(o.momentum_x(), rel=1e-10)
        assert s.observe(0, "wall_drag") == pytest.approx(o.wall_drag(), rel=1e-9)
        ux = pr["ux"]
        assert s.observe(0, "umid") == pytest.approx(0.5 * (ux[19] + ux[20]), rel=1e-10)
        assert s.observe(0, "step") == 3001


def test_bitwise_repeat_and_step_splitting():
    """Two handles give identical states; N steps equal k + (N - k) steps in
    any split across graph boundaries (bitwise)."""
    spec = ChannelSpec(256, 50, 1e-6, 1.0, 1e-4, 1e3, 0.1)
    pops0, P0 = workloads.perturbed_rest_state(256, 50, seed=7)
    states = []
    for split in [[2500], [1000, 1500], [999, 1, 1337, 163], [2500]]:
        with solver([spec], precision="fp32", obs_every=500) as s:
            s.set_state(0, pops0, P0, 0)
            for n in split:
                s.step(n)
            states.append(s.get_state(0))
    for pops, P in states[1:]:
        assert np.array_equal(pops, states[0][0]) and np.array_equal(P, states[0][1])


@pytest.mark.parametrize("precision,nx", [("fp64", 300), ("fp64", 512), ("fp32", 300), ("fp32", 512), ("fp32", 1024)])
def test_x_uniform_stays_bitwise_uniform(precision, nx):
    """A wide x-periodic channel started from rest stays exactly x-uniform:
    every halo lane, edge column and wrapped column computes the same values
    (FP32: also across the moves of the row reference velocities every 100
    steps)."""
    spec = ChannelSpec(nx, 40, 1e-6, 1.0, 1e-4, 1e3, 0.1)
    with solver([spec], precision=precision, obs_every=100) as s:
        s.step(777)
        pops, P = s.get_state(0)
        assert np.array_equal(pops, np.broadcast_to(pops[:, :, :1], pops.shape))
        assert np.abs(s.observe(0, "kxx")).max() == 0.0


def test_mass_conservation_fp64():
    """Hydrodynamic mass conserved to round-off on the GPU (FP64)."""
    spec = ChannelSpec(8, 64, 2e-6, 1.0, 1e-4, 2e3, 0.1)
    with solver([spec], precision="fp64", obs_every=1000) as s:
        m0 = s.observe(0, "mass")
        s.step(10000)
        assert abs(s.observe(0, "mass") - m0) / 512 < 1e-15 * 10000


def test_convergence_freezes_channels(orc):
    """With steady_tol, channels stop once the residual falls below it and
    their final profile matches the oracle run for the same number of steps."""
    specs = [ChannelSpec(8, 16, 2e-6, 1.0, 1e-4, 1e3, 0.1), ChannelSpec(8, 48, 1e-6, 1.0, 1e-4, 1e3, 0.1)]
    with solver(specs, precision="fp64", obs_every=200, steady_tol=1e-7) as s:
        s.step(200000)
        steps = [int(s.observe(i, "step")) for i in range(2)]
        assert all(s.observe(i, "active") == 0 for i in range(2))
        assert steps[0] < steps[1] < 200000
        for i, sp in enumerate(specs):
            o = oracle_channel(orc, sp)
            o.run(steps[i])
            compare_fields(s, i, o, FP64_TOL, f"frozen ch{i} at {steps[i]}")


@pytest.mark.parametrize("nx", [8, 100])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_frozen_channel_survives_odd_steps(precision, nx):
    """A channel frozen by the convergence check keeps its state exactly
    through later steps of odd length, which change the buffer the handle
    reads from; so does a state set on it while frozen. nx = 8 runs the
    narrow strip sweep; nx = 100 the tile sweep in FP64 (whose workgroups
    skip a frozen channel) and the generic strip sweep in FP32."""
    specs = [ChannelSpec(nx, 16, 2e-6, 1.0, 1e-4, 1e3, 0.1), ChannelSpec(nx, 96, 1e-6, 1.0, 1e-4, 1e3, 0.1)]
    with solver(specs, precision=precision, obs_every=200, steady_tol=1e-7) as s:
        while s.observe(0, "active") != 0:
            s.step(200)
        assert s.observe(1, "active") == 1
        t0 = s.observe(0, "step")
        pops0, P0 = s.get_state(0)
        u0 = s.observe(0, "ux")
        for n in (1, 2, 3):
            s.step(n)
            pops, P = s.get_state(0)
            assert np.array_equal(pops, pops0) and np.array_equal(P, P0), n
            assert np.array_equal(s.observe(0, "ux"), u0) and s.observe(0, "step") == t0
        pops1 = pops0.copy()
        pops1[0] += 1e-9
        s.set_state(0, pops1, P0, int(t0))
        s.step(1)
        pops, _ = s.get_state(0)
        assert np.abs(pops - pops1).max() < (1e-16 if precision == "fp64" else 1e-9)


@pytest.mark.parametrize("nnp", [True, False])
def test_warm_start_profile_state(nnp):
    """lb_set_profile writes equilibrium populations at the given u_x with
    rho_e = 1 - (3/2) N1 (rho_e = 1 without the flow-induced density) and
    P = N1, keeping the rest-state mass."""
    spec = ChannelSpec(4, 24, 1e-6, 1.0, 1e-4, 1e3, 0.1, nn_pressure=nnp)
    ux = 1e-3 * np.sin(np.linspace(0.1, 3.0, 24))
    n1 = 1e-6 * np.cos(np.linspace(0, 2, 24))
    with solver([spec], precision="fp64") as s:
        s.set_profile(0, ux, n1)
        pops, P = s.get_state(0)
        assert np.allclose(P, n1[:, None], rtol=0, atol=1e-20)
        rho = pops.sum(axis=0)
        assert np.allclose(rho, ((1 - 1.5 * n1) if nnp else np.ones(24))[:, None], rtol=1e-14)
        mx = (pops[[1, 5, 8]].sum(axis=0) - pops[[3, 6, 7]].sum(axis=0))
        assert np.allclose(mx / rho, ux[:, None], rtol=1e-12, atol=1e-18)
        assert s.observe(0, "mass") == pytest.approx(96.0, rel=1e-14)


@pytest.mark.parametrize("ny", [24, 64, 97])
def test_warm_start_chebyshev_points_exact_for_polynomials(ny):
    """lb_set_profile from values at the 64 Chebyshev-Gauss points
    d_k = cos(pi (2k+1)/128): barycentric interpolation reproduces any
    polynomial of degree < 64 at the rows d = (y - y_c)/H, so a cubic u_x and
    a quadratic N1 come back exactly (to round-off) in the state's moments."""
    n = 64
    dk = np.cos(np.pi * (2 * np.arange(n) + 1) / (2 * n))
    u_of = lambda d: 1e-3 * (1 - d * d) * (1 + 0.3 * d)
    n1_of = lambda d: 2e-6 * (1 - 0.5 * d * d)
    spec = ChannelSpec(2, ny, 1e-6, 1.0, 1e-4, 1e3, 0.1)
    d = (np.arange(ny) - (ny - 1) / 2) / (ny / 2)
    with solver([spec], precision="fp64") as s:
        s.set_profile(0, u_of(dk), n1_of(dk), points="chebyshev")
        pops, P = s.get_state(0)
        rho = pops.sum(axis=0)
        mx = pops[[1, 5, 8]].sum(axis=0) - pops[[3, 6, 7]].sum(axis=0)
        assert np.allclose(P, n1_of(d)[:, None], rtol=1e-11, atol=1e-18)
        assert np.allclose(mx / rho, u_of(d)[:, None], rtol=1e-10, atol=1e-16)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_large_channel_sampled_rows(orc, precision):
    """The 4096 x 1024 lattice at full size, in the launch configuration the
    benchmark times (FP64: a 336 MB state, written with nontemporal stores),
    with eps = -0.05 (G tau = 0.1; the drawn eps = 0.045 gives G tau = 1.2,
    outside the well-conditioned band): the x-uniform run equals an nx = 1
    oracle run row for row (an x-periodic uniform state has no x
    dependence), within the tolerance of the precision."""
    wl = workloads.large_channel(eps=-0.05)
    spec = wl["channels"][0]
    with solver([spec], precision=precision, obs_every=1000) as s:
        s.step(wl["steps"])
        import dataclasses
        o = oracle_channel(orc, dataclasses.replace(spec, nx=1))
        o.run(wl["steps"])
        compare_fields(s, 0, o, FP32_TOL if precision == "fp32" else FP64_TOL, f"large_channel {precision}")
        assert np.abs(s.observe(0, "kxx")).max() == 0.0


def band_rows(u, rows=16):
    """u(y) symmetrised with u(ny-1-y) and averaged over bands of rows."""
    s = 0.5 * (u + u[::-1])
    return s.reshape(-1, rows).mean(axis=1)


def spread_measures(a, b):
    """Pointwise, band-averaged and integrated (flux) differences of two
    row profiles, relative to the second one's maximum and sum."""
    m = np.abs(b).max()
    return (np.abs(a - b).max() / m, np.abs(band_rows(a) - band_rows(b)).max() / m,
            abs(a.sum() - b.sum()) / abs(b.sum()))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_large_channel_as_drawn_statistical(orc, precision):
    """The benchmark's workload exactly as drawn (4096 x 1024, seed 1:
    g = 1.06e-6, eps = +0.045, G_inf tau = 1.21), from rest, 10,000 steps,
    in the launch configuration the benchmark times. At this G_inf tau the
    explicit stress amplifies round-off (two FP64 oracle runs 1e-15 apart
    differ by percents within 100 steps), so: the first 5 steps equal the
    nx = 1 oracle node for node (FP64 to 1e-9, FP32 to its resolution), and
    after 10,000 steps u_x and sigma_xy, pointwise, averaged over 16-row
    bands of the symmetrised profile, and integrated (the flux), lie within
    twice the largest spread of three oracle runs perturbed by 1e-15 (plus
    the FP32 resolution bound 2^-24 K, K = 1000, in FP32)."""
    import dataclasses
    wl = workloads.large_channel()
    spec = wl["channels"][0]
    one = dataclasses.replace(spec, nx=1)
    base = oracle_channel(orc, one)
    pert = []
    for seed in range(3):
        o = oracle_channel(orc, one)
        rng = np.random.default_rng(900 + seed)
        o.set_state(o.n * (1 + 1e-15 * rng.uniform(-1, 1, o.n.shape)), o.P, t=0)
        pert.append(o)
    extra = 0.0 if precision == "fp64" else 2.0 ** -24 * 1000
    with solver([spec], precision=precision, obs_every=1000) as s:
        s.step(5)
        base.run(5)
        f = base.fields()
        for name, tol in (("ux", 1e-9 if precision == "fp64" else 1e-5),
                          ("sxy", 1e-9 if precision == "fp64" else 1e-4)):
            e = linf(s.observe(0, name), f[name].mean(axis=1))
            print(f"{precision} t=5: {name} {e:.2e}", flush=True)
            assert e < tol
        s.step(wl["steps"] - 5)
        base.run(wl["steps"] - 5)
        ref = base.profiles()
        got = {k: s.observe(0, k) for k in ("ux", "sxy")}
    for o in pert:
        o.run(wl["steps"])
    for k in ("ux", "sxy"):
        sp = np.max([spread_measures(o.profiles()[k], ref[k]) for o in pert], axis=0)
        e = spread_measures(got[k], ref[k])
        print(f"{precision} t={wl['steps']} {k}: GPU vs oracle pointwise {e[0]:.2e} band {e[1]:.2e} "
              f"flux {e[2]:.2e}; oracle spread {sp[0]:.2e} {sp[1]:.2e} {sp[2]:.2e}", flush=True)
        assert e[0] <= 2 * sp[0] + extra and e[1] <= 2 * sp[1] + extra and e[2] <= 2 * sp[2] + extra


def test_poiseuille_gtau1_short_exact_long_statistical(orc):
    """The G tau = 1 workload as specified: exact over the first 5 steps
    (round-off has not been amplified yet), then after 20,000 steps the
    x-averaged velocity within 1% of the oracle's (two oracle runs that differ
    by 1e-15 already differ by 0.13% there) and mass conserved."""
    spec = workloads.poiseuille_64()["channels"][0]
    o = oracle_channel(orc, spec)
    with solver([spec], precision="fp64") as s:
        s.step(5)
        o.run(5)
        pops, _ = s.get_state(0)
        assert np.abs(pops - o.n).max() / np.abs(o.n - workloads.REST_WEIGHTS[:, None, None]).max() < 1e-9
        s.step(19995)
        o.run(19995)
        e = linf(s.observe(0, "ux"), o.profiles()["ux"])
        print(f"G tau = 1 at t=20000: u_x Linf rel {e:.3e}", flush=True)
        assert e < 1e-2
        assert abs(s.observe(0, "mass") - 512) < 1e-9


def test_batched_sweep_fp32_reaches_fp64_steady_state(orc):
    """All 256 channels of the batched sweep (nx = 8, ny 32..509, the drawn
    eps, G tau and g) run to residual < 1e-9 in FP32 and in FP64. Every
    channel converges in both. The FP32 steady profiles equal the FP64 ones
    within 5e-5 of max |u_x|: a frozen profile still moves at < 1e-9 max|u|
    per step, and the slowest channel relaxes over ~4e4 steps (H^2 / (pi^2 nu),
    H = 255, nu = 1/6). FP32 resolves the slow last stretch of convergence.
    Channels run as configured (G tau <= 0.3) have FP64 profiles within
    2e-3 of the analytic steady profile of Sec. III.B: the lattice
    discretisation error, largest in the narrowest channels. Stiff channels
    (viscosity split 1/2: relaxation times up to about 20) carry the larger
    wall error of BGK at such relaxation times; theirs is reported."""
    from oracle import analytic
    wl = workloads.batched_sweep()
    chans = wl["channels"]
    prof = {}
    for prec in ("fp32", "fp64"):
        with solver(chans, precision=prec, obs_every=1000, steady_tol=1e-9, strip_rows=16) as s:
            s.step(3_000_000)
            assert all(s.observe(i, "active") == 0 for i in range(len(chans))), prec
            prof[prec] = [s.observe(i, "ux") for i in range(len(chans))]
    d32 = []
    e64 = []
    for i, c in enumerate(chans):
        p = orc.resolve(c.tau_lb, c.G, c.tau0, c.gamma_c, c.eps)
        ua = analytic.steady_profile(c.ny, c.force, (c.tau_lb - 0.5) / 3, p.G, p.tau, c.gamma_c)
        u64 = prof["fp64"][i]
        d32.append(np.abs(prof["fp32"][i] - u64).max() / np.abs(u64).max())
        e64.append(np.abs(u64 - ua).max() / np.abs(ua).max())
    d32, e64 = np.array(d32), np.array(e64)
    lit = np.array([c.visc_split == 0.0 for c in chans])
    print(f"FP32 vs FP64 steady: median {np.median(d32):.2e} max {d32.max():.2e}; FP64 vs analytic: "
          f"as configured ({lit.sum()}) median {np.median(e64[lit]):.2e} max {e64[lit].max():.2e}, "
          f"stiff ({(~lit).sum()}) median {np.median(e64[~lit]):.2e} max {e64[~lit].max():.2e}", flush=True)
    assert d32.max() < 5e-5 and np.median(d32) < 1e-6, (d32.max(), np.median(d32))
    assert e64[lit].max() < 2e-3 and np.median(e64[lit]) < 2e-4, (e64[lit].max(), np.median(e64[lit]))


def load_batched_fixture():
    import importlib.util
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "make_batched_oracle.py")
    spec = importlib.util.spec_from_file_location("make_batched_oracle", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.load()


def test_batched_sweep_per_channel_error_vs_oracle():
    """The batched sweep as configured (256 channels of nx = 8, widths
    32..512, forces, eps and tau0 over the whole box; stiff draws with the
    viscosity split 1/2 and no delta-rho terms) in one FP32 handle, run until
    every channel's residual is below 1e-9: every channel converges, and for
    a width-stratified sample of 34 channels (three per width decile and the
    four widest) the steady u_x and sigma_xy equal the FP64 oracle's steady
    state from rest (tests/golden/batched_sweep_seed2_oracle.txt) within the
    FP32 tolerance 1e-3 (L-infinity relative per channel), after the same
    number of steps to within two checks."""
    wl = workloads.batched_sweep()
    chans = wl["channels"]
    ref = load_batched_fixture()
    assert sorted(ref) == workloads.batched_sample(chans)
    with solver(chans, precision="fp32", obs_every=1000, steady_tol=1e-9, strip_rows=16) as s:
        s.step(3_000_000)
        steps = [int(s.observe(i, "step")) for i in range(len(chans))]
        assert all(s.observe(i, "active") == 0 for i in range(len(chans))), steps
        eu, es = [], []
        for i, (t_o, u_o, s_o) in sorted(ref.items()):
            u, sx = s.observe(i, "ux"), s.observe(i, "sxy")
            eu.append(linf(u, u_o))
            es.append(linf(sx, s_o))
            print(f"channel {i} ny {chans[i].ny} split {chans[i].visc_split}: steps {steps[i]} (oracle {t_o}); "
                  f"u_x {eu[-1]:.2e} sigma_xy {es[-1]:.2e}", flush=True)
            assert abs(steps[i] - t_o) <= 2000
    print(f"per-channel L-inf vs oracle: u_x median {np.median(eu):.2e} max {np.max(eu):.2e}; "
          f"sigma_xy median {np.median(es):.2e} max {np.max(es):.2e}", flush=True)
    assert max(eu) <= FP32_TOL and max(es) <= FP32_TOL


@pytest.mark.parametrize("ny,path", [(104_857, "tiles"), (104_961, "strips")])
def test_fp64_channel_at_the_tile_offset_limit(orc, ny, path):
    """FP64 channels of 4096 x 104,857 nodes (429,494,272: the tile sweep,
    whose in-channel slot offsets then reach 4,294,942,719, just below
    2^32) and of 4096 x 104,961 (beyond 429,496,704 nodes: the strip sweep,
    with 64-bit offsets). About 69 GB of state each. From rest, after 6
    steps the x-averaged u_x and sigma_xy of every row equal the nx = 1
    oracle, the walls included (the top rows sit at the highest offsets)."""
    spec = ChannelSpec(nx=4096, ny=ny, force=1e-6, tau_lb=1.0, G=1e-4, tau0=1e3, gamma_c=0.1, eps=0.02)
    print(f"fp64 4096 x {ny} ({path})", flush=True)
    with solver([spec], precision="fp64", obs_every=6) as s:
        s.step(6)
        o = oracle_channel(orc, dataclasses.replace(spec, nx=1))
        o.run(6)
        compare_fields(s, 0, o, 1e-10, f"fp64 4096 x {ny} ({path})")
        ux = s.observe(0, "ux")
        # the two wall rows mirror each other up to the rounding of their
        # different bounce-back terms (3e-12 of max u_x measured)
        assert np.all(np.isfinite(ux)) and abs(ux[-1] - ux[0]) < 1e-10 * abs(ux).max()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_nan_reported_before_freezing(orc, precision):
    """Failure detection: a NaN set into one channel of a two-channel handle
    makes the next convergence check return LB_EUNSTABLE with the channel's
    'nan' observable set, before the check freezes anything: the other
    channel, at rest and so converged at that check, stays active. After the
    bad channel is reset, the handle carries on: the rest channel freezes at
    the next check, and the reset channel follows the oracle through its
    force switch-off, so host and device agree on every step counter."""
    from paper_1310_7450_amd.lbnlm import LbError
    K = 16
    specs = [ChannelSpec(8, 16, 2e-6, 0.8, 2e-4, 500.0, 0.1, t_startup=40),
             ChannelSpec(8, 12, 0.0, 1.0, 1e-4, 1e3, 0.1)]
    with solver(specs, precision=precision, obs_every=K, steady_tol=1e-9) as s:
        s.step(K)
        pops, P = s.get_state(0)
        pops[3, 5, 2] = np.nan
        s.set_state(0, pops, P, K)
        with pytest.raises(LbError) as e:
            s.step(K)
        assert e.value.status == -4
        assert s.observe(0, "nan") == 1.0
        assert s.observe(1, "nan") == 0.0
        assert s.observe(1, "active") == 1.0 and s.observe(0, "active") == 1.0
        assert s.observe(0, "step") == 2 * K and s.observe(1, "step") == 2 * K
        # reset channel 0 to rest at t = 2K; the force stays on until t = 40
        rest = np.broadcast_to(workloads.REST_WEIGHTS[:, None, None], (9, 16, 8)).copy()
        s.set_state(0, rest, np.zeros((16, 8)), 2 * K)
        s.step(3 * K)
        assert s.observe(1, "active") == 0.0 and s.observe(1, "step") == 3 * K
        assert s.observe(0, "step") == 5 * K
        o = oracle_channel(orc, specs[0])
        o.set_state(rest, np.zeros((16, 8)), t=2 * K)
        o.run(3 * K)
        g_pops, _ = s.get_state(0)
        err = np.abs(g_pops - o.n).max() / np.abs(o.n - workloads.REST_WEIGHTS[:, None, None]).max()
        print(f"{precision}: after the reset, state {err:.2e}", flush=True)
        assert err < (1e-9 if precision == "fp64" else 1e-4)
