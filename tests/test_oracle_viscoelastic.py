"""Pins of the oracle's time-integrated (viscoelastic) nonlinear Maxwell model.

The model is the differential form of Eq. (gkder) with d_t G = -G / tau_M(t)
and tau_M from Eq. (nlmaxwell) at the current velocity gradient, the
time-dependent generalisation Sec. III.A mentions. One step takes the
upper-convected terms explicitly and the relaxation implicitly (the oracle's
reading R11). The pins use what that fixes independently of the code:
- the exact solution of the one-step recursion in simple shear (both
  orientations, so a transposed kappa fails);
- its continuous-time limit, the start-up of the upper-convected Maxwell
  model;
- the fixed point, which must be the series of Eq. (sigtsum) for any kappa;
- channel-level consequences: the same steady state as the instantaneous
  model, mass conservation, and the Newtonian limit.
"""
import math

import numpy as np
import pytest

from oracle import analytic

ETA_S = 1.0 / 6.0  # tau_LB = 1


def iterate(orc, kappa, G, tau, gc, n, s0=(0.0, 0.0, 0.0)):
    s = np.array(s0, dtype=float)
    out = [s.copy()]
    for _ in range(n):
        s = orc.stress_ve_step(kappa, G, tau, gc, s)
        out.append(s.copy())
    return np.array(out)


@pytest.mark.parametrize("orient", ["xy", "yx"])
def test_shear_startup_matches_discrete_closed_form(orc, orient):
    """Simple shear at rate gd from rest. With q = 1/(1 + r), r = 1/tau + gd/gc
    (II_D = gd^2), the recursion has the closed-form solution
    sigma_shear(n) = G gd / r (1 - q^n),
    sigma_flow(n) = 2 gd G gd / r [(1 - q^n)/r - n q^n] along the flow
    direction, and zero across it. Shear along x (kappa_xy = gd) loads
    sigma_xx; shear along y (kappa_yx = gd) loads sigma_yy."""
    G, tau, gc, gd = 1e-4, 800.0, 0.1, 3e-4
    kap = [[0, gd], [0, 0]] if orient == "xy" else [[0, 0], [gd, 0]]
    n = np.arange(4001)
    s = iterate(orc, kap, G, tau, gc, 4000)
    r = 1.0 / tau + gd / gc
    q = 1.0 / (1.0 + r)
    shear = G * gd / r * (1 - q ** n)
    flow = 2 * gd * G * gd / r * ((1 - q ** n) / r - n * q ** n)
    along, across = (0, 2) if orient == "xy" else (2, 0)
    assert np.allclose(s[:, 1], shear, rtol=1e-12, atol=1e-13 * shear.max())
    assert np.allclose(s[:, along], flow, rtol=1e-11, atol=1e-13 * flow.max())
    assert np.abs(s[:, across]).max() == 0.0


@pytest.mark.parametrize("tau", [200.0, 2000.0])
def test_shear_startup_continuous_limit(orc, tau):
    """Upper-convected Maxwell start-up in simple shear at constant tau_M
    (gamma_c -> inf): sigma_xy(t) = G gd tau_M (1 - e^{-t/tau_M}),
    N1(t) = 2 G gd^2 tau_M^2 [1 - (1 + t/tau_M) e^{-t/tau_M}]. The one-step
    scheme is first order: its error is O(dt / tau_M)."""
    G, gd = 1e-4, 1e-4
    n = int(5 * tau)
    s = iterate(orc, [[0, gd], [0, 0]], G, tau, 1e300, n)
    t = np.arange(n + 1) / tau
    sxy = G * gd * tau * (1 - np.exp(-t))
    n1 = 2 * G * gd * gd * tau * tau * (1 - (1 + t) * np.exp(-t))
    e_xy = np.abs(s[:, 1] - sxy).max() / sxy.max()
    e_n1 = np.abs(s[:, 0] - s[:, 2] - n1).max() / n1.max()
    assert e_xy < 1.0 / tau and e_n1 < 2.0 / tau
    assert e_xy > 0.05 / tau  # first order, not better: the scheme is what it says


def test_fixed_point_is_the_series(orc):
    """Eqs. (sigtsum), (smalld): held at a constant kappa (rotation, extension
    and shear mixed), the stress relaxes to the steady sum of the
    instantaneous model, which solves the same fixed-point relation."""
    rng = np.random.default_rng(11)
    G, gc, tau = 1e-4, 0.1, 300.0
    for _ in range(12):
        k = 1e-3 * rng.standard_normal((2, 2))
        tM = orc.tau_M(k, tau, gc)
        want, nt = orc.stress_series(k, G, tM)
        assert nt > 0
        s = np.zeros(3)
        for _ in range(int(60 * tM) + 10):
            s = orc.stress_ve_step(k, G, tau, gc, s)
        assert np.allclose(s, want, rtol=1e-9, atol=1e-12 * np.abs(want).max())


def test_yield_stress_reached_in_time(orc):
    """Eq. (yieldstress): for tau -> inf and steady shear the stress tends to
    the dynamic yield stress G gamma_c, from below (it builds up over tau_M,
    not at once as in the instantaneous model)."""
    G, gc, gd = 1e-4, 0.1, 1e-3
    s = iterate(orc, [[0, gd], [0, 0]], G, math.inf, gc, 3000)
    assert s[1, 1] < 0.02 * G * gc
    assert np.all(np.diff(s[:, 1]) >= 0)
    assert s[-1, 1] == pytest.approx(G * gc, rel=1e-12)


def test_channel_steady_state_equals_instantaneous(orc):
    """Sec. III.B: both models share the steady relation, so the steady LB
    channel is the same (within the remaining transient) and within the
    paper's 1% of the analytic profile of Eq. (maxwellpoiseuille)."""
    ny, g, tau0 = 32, 2e-6, 1e3
    out = {}
    for ve in (False, True):
        ch = orc.Channel(1, ny, g, tau_lb=1.0, G=1e-4, tau0=tau0, gamma_c=0.1, viscoelastic=ve)
        ch.run(40000)
        out[ve] = ch.fields()
    u0, u1 = out[False]["ux"][:, 0], out[True]["ux"][:, 0]
    assert np.abs(u1 - u0).max() < 1e-7 * np.abs(u0).max()
    s0, s1 = out[False]["sxy"][:, 0], out[True]["sxy"][:, 0]
    assert np.abs(s1 - s0).max() < 1e-7 * np.abs(s0).max()
    want = analytic.steady_profile(ny, g, ETA_S, 1e-4, tau0, 0.1)
    assert np.abs(u1 - want).max() / want.max() < 1e-2


def test_channel_stress_lags_at_startup(orc):
    """Early in the start-up the time-integrated shear stress trails the
    instantaneous one (it needs about tau_M to build up), so the fluid first
    responds closer to the solvent alone and runs ahead."""
    ny, g = 32, 2e-6
    runs = {}
    for ve in (False, True):
        ch = orc.Channel(1, ny, g, tau_lb=1.0, G=1e-4, tau0=1e3, gamma_c=0.1, viscoelastic=ve)
        ch.run(300)
        runs[ve] = ch.fields()
    wall = 0
    assert abs(runs[True]["sxy"][wall, 0]) < 0.7 * abs(runs[False]["sxy"][wall, 0])
    assert runs[True]["ux"][ny // 2, 0] > runs[False]["ux"][ny // 2, 0]


def test_channel_mass_conserved(orc):
    """Eq. (rhoj), R1: the hydrodynamic mass is conserved with the
    time-integrated stress as well (round-off per node and step)."""
    ch = orc.Channel(4, 32, 2e-6, tau_lb=1.0, G=1e-4, tau0=2e3, gamma_c=0.1, viscoelastic=True)
    n = ch.nx * ch.ny
    q0 = ch.mass()
    ch.run(5000)
    assert abs(ch.P).max() > 1e-8 and abs(ch.S).max() > 1e-8
    assert abs(ch.mass() - q0) / n < 5e-16 * 5000


def test_zero_modulus_identical_to_newtonian(orc):
    """G = 0: the stress stays zero and the run equals the instantaneous
    model's G = 0 run bit for bit."""
    a = orc.Channel(2, 16, 1e-6, tau_lb=1.0, G=0.0, tau0=1e4, gamma_c=0.1)
    b = orc.Channel(2, 16, 1e-6, tau_lb=1.0, G=0.0, tau0=1e4, gamma_c=0.1, viscoelastic=True)
    a.run(500)
    b.run(500)
    assert np.array_equal(a.n, b.n) and np.array_equal(a.P, b.P)
    assert np.abs(b.S).max() == 0.0
