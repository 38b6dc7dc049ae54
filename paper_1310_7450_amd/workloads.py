"""Seeded synthetic channel workloads shaped like the paper's runs.

Input generation only: this module draws channel parameters and initial
perturbations from seeded numpy generators and holds none of the method's
arithmetic. Both the GPU path and the CPU oracle take their inputs from here.

Named workloads (lattice units, rho0 = 1):

* ``poiseuille_64``: one 8 x 64 channel, g = 1e-6, tau_LB = 1, G = 1e-4,
  tau0 = 1e4 steps, gamma_c = 0.1, eps = 0 (yield-stress-like, theta = 6),
  20,000 start-up steps then 20,000 cessation steps; ``newtonian=True``
  sets G = 0.
* ``large_channel``: one 4096 x 1024 channel, g log-uniform in [1e-7, 1e-5]
  and eps uniform in [-0.05, 0.05] from seed 1, other parameters as above,
  10,000 steps from rest.
* ``batched_sweep``: 256 channels, nx = 8, per channel in order
  ny ~ U{32..512}, log10 g ~ U(-7, -5), eps ~ U(-0.1, 0.1),
  log10 tau0 ~ U(3, 5), from seed 2 (see the function for the low-Mach
  rule and the conditioning policy of stiff draws); ``batched_sample``
  picks a width-stratified sample of it.
* ``transient_scale``: 16 channels of 8192 x 2048, 8 at eps = 0 and 8 at
  eps = +0.02, g = 2 G gamma_c / H (wp H = 2 gamma_c), 50,000 start-up steps
  then cessation.
* ``couette_64``: planar Couette flow, 8 x 64, Zou and He's top wall at u0
  switched on and off, theta = 100 (the paper's Fig. stopshear parameters in
  lattice units).
"""
import numpy as np

from .lbnlm import ChannelSpec

REST_WEIGHTS = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def poiseuille_64(newtonian=False, nx=8, ny=64, tau0=1e4):
    """``tau0`` other than 1e4 gives the same channel at another Maxwell time
    (tau0 = 2e3 puts G tau = 0.2 inside the explicit-stress stable band)."""
    spec = ChannelSpec(nx=nx, ny=ny, force=1e-6, tau_lb=1.0, G=0.0 if newtonian else 1e-4, tau0=tau0,
                       gamma_c=0.1, eps=0.0, visc_split=0.0, t_startup=20000)
    name = "poiseuille_64" + ("_newtonian" if newtonian else "") + ("" if tau0 == 1e4 else f"_tau0_{tau0:g}")
    return {"name": name, "channels": [spec], "startup": 20000, "cessation": 20000}


def large_channel(seed=1, nx=4096, ny=1024, eps=None):
    """``eps`` overrides the drawn separation (the force is still drawn)."""
    rng = np.random.default_rng(seed)
    g = 10.0 ** rng.uniform(-7.0, -5.0)
    e = rng.uniform(-0.05, 0.05)
    if eps is not None:
        e = float(eps)
    spec = ChannelSpec(nx=nx, ny=ny, force=g, tau_lb=1.0, G=1e-4, tau0=1e4, gamma_c=0.1, eps=e)
    return {"name": f"large_channel_{nx}x{ny}" + ("" if eps is None else f"_eps_{e:g}"),
            "channels": [spec], "steps": 10000, "seed": seed}


def perturbed_rest_state(nx, ny, seed, amplitude=1e-4):
    """Populations of a fluid at rest with a seeded density perturbation of
    relative amplitude ``amplitude`` (n_i = a_i (1 + delta)), and P = 0, in the
    layout of ``lb_get_state``: pops[9][ny][nx], P[ny][nx]."""
    rng = np.random.default_rng(seed)
    delta = amplitude * rng.uniform(-1.0, 1.0, size=(ny, nx))
    pops = REST_WEIGHTS[:, None, None] * (1.0 + delta[None, :, :])
    return np.ascontiguousarray(pops), np.zeros((ny, nx))


def random_state(nx, ny, seed, amplitude=1e-3):
    """Rest populations with independent seeded perturbations of every
    population (non-equilibrium content in every moment) and a random
    previous trace; for layout and streaming tests."""
    rng = np.random.default_rng(seed)
    pops = REST_WEIGHTS[:, None, None] * (1.0 + amplitude * rng.uniform(-1, 1, size=(9, ny, nx)))
    P = 1e-6 * rng.uniform(-1, 1, size=(ny, nx))
    return np.ascontiguousarray(pops), np.ascontiguousarray(P)


def random_stress(nx, ny, seed, amplitude=1e-6):
    """Seeded random stress fields sigma[3][ny][nx] (xx, xy, yy) in the layout
    of ``lb_get_stress``, for state tests of the time-integrated model."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(amplitude * rng.uniform(-1, 1, size=(3, ny, nx)))


# Rules of the batched sweep (input recipe; see the design notes). Low Mach
# number: a draw whose solvent-viscosity Poiseuille velocity g H^2 / (2 eta_s)
# exceeds 0.1 is redrawn (the nlM fluid only adds viscosity, so its velocity
# is lower still). Conditioning: the explicit stress with the flow-induced
# density terms and visc_split 0 (the configuration as written) amplifies
# round-off once G_inf tau exceeds about 0.3-0.5 (a measured stability map of
# the scheme); a draw above GTAU_LITERAL_MAX runs instead with the viscosity
# split of Sec. IV at STIFF_SPLIT and without the delta-rho terms, which the
# same map shows well conditioned over the whole box (G_inf tau up to 13).
GTAU_LITERAL_MAX = 0.3
STIFF_SPLIT = 0.5
U_SOLVENT_MAX = 0.1


def _closure(tau0, eps, G=1e-4):
    tau = tau0 * 10.0 ** (min(eps, 0.0) / 0.05)
    return G * (1.0 + max(eps, 0.0) ** 0.5), tau


def batched_sweep(seed=2, n_channels=256, nx=8, tau_lb=1.0, G=1e-4, gamma_c=0.1):
    """Channels drawn in order ny ~ U{32..512}, log10 g ~ U(-7,-5),
    eps ~ U(-0.1, 0.1), log10 tau0 ~ U(3, 5) from ``seed``; a draw with
    g (ny/2)^2 / (2 eta_s) > U_SOLVENT_MAX is redrawn. Draws with
    G_inf tau <= GTAU_LITERAL_MAX run as written (visc_split 0, delta-rho
    terms on), the others with visc_split STIFF_SPLIT and without the
    delta-rho terms. Returns the channels, the number of draws and how many
    channels run in the stiff setting."""
    rng = np.random.default_rng(seed)
    eta_s = (tau_lb - 0.5) / 3.0
    chans, draws, stiff = [], 0, 0
    while len(chans) < n_channels:
        ny = int(rng.integers(32, 513))
        g = 10.0 ** rng.uniform(-7.0, -5.0)
        eps = rng.uniform(-0.1, 0.1)
        tau0 = 10.0 ** rng.uniform(3.0, 5.0)
        draws += 1
        if g * (ny / 2.0) ** 2 / (2 * eta_s) > U_SOLVENT_MAX:
            continue
        Ginf, tau = _closure(tau0, eps, G)
        literal = Ginf * tau <= GTAU_LITERAL_MAX
        stiff += not literal
        chans.append(ChannelSpec(nx=nx, ny=ny, force=g, tau_lb=tau_lb, G=G, tau0=tau0, gamma_c=gamma_c,
                                 eps=eps, visc_split=0.0 if literal else STIFF_SPLIT, nn_pressure=literal))
    return {"name": f"batched_sweep_{n_channels}x{nx}", "channels": chans, "draws": draws, "stiff": stiff,
            "seed": seed, "steady_tol": 1e-9, "obs_every": 1000, "max_steps": 3_000_000}


def batched_sample(channels, per_decile=3, widest=4):
    """Indices of a width-stratified sample of a batch: ``per_decile``
    channels evenly spaced through each tenth of the channels ordered by
    width, plus the ``widest`` widest ones (sorted, without repeats)."""
    order = sorted(range(len(channels)), key=lambda i: (channels[i].ny, i))
    n = len(order)
    pick = set()
    for d in range(10):
        lo, hi = d * n // 10, (d + 1) * n // 10
        for k in range(per_decile):
            pick.add(order[lo + (2 * k + 1) * (hi - lo) // (2 * per_decile)])
    pick.update(order[n - widest:])
    return sorted(pick)


def transient_scale(nx=8192, ny=2048, n_per_eps=8, eps_values=(0.0, 0.02), G=1e-4, tau0=1e4, gamma_c=0.1,
                    tau_lb=1.0):
    """Start-up and cessation at scale: ``n_per_eps`` channels of nx x ny at
    each separation in ``eps_values`` (yield-stress case eps = 0, glass side
    eps = +0.02), the nlM parameters of the 8 x 64 channel, and one force for
    all of them, g = 2 G gamma_c / H (wp H = 2 gamma_c: the wall stress of the
    steady flow is twice the yield stress G gamma_c at eps = 0). The force is
    on for 50,000 steps; cessation runs until u_mid has fallen to 1e-3 of its
    value at the switch-off, for at most 200,000 steps. No draws: every
    channel of one eps is the same channel. ``nx`` = 64 gives the x-reduced
    lattice, which evolves bitwise like the full one from rest (the flow
    stays exactly x-uniform and every column runs the same arithmetic)."""
    H = ny / 2.0
    g = 2.0 * G * gamma_c / H
    chans = [ChannelSpec(nx=nx, ny=ny, force=g, tau_lb=tau_lb, G=G, tau0=tau0, gamma_c=gamma_c, eps=float(e),
                         visc_split=0.0, t_startup=50000)
             for e in eps_values for _ in range(n_per_eps)]
    return {"name": f"transient_scale_{len(chans)}x{nx}x{ny}", "channels": chans, "startup": 50000,
            "cessation_cap": 200000, "stop_fraction": 1e-3, "thresholds": (1e-2, 1e-3, 1e-4)}


def couette_width(ny, top_wall):
    """Distance between the fixed half-way wall (y = -1/2) and the moving
    wall: y = ny - 1/2 for the half-way wall, the node row y = ny - 1 for
    Zou and He's wall."""
    return float(ny) if top_wall == "halfway" else ny - 0.5


def couette_64(nx=8, ny=64, theta=100.0, tau_lb=0.6, G=1e-3, gamma_c=0.1, wall_u_scale=1e-2, startup=60000,
               newtonian=False, top_wall="zou_he"):
    """Planar Couette flow switched on and off (Sec. IV.B, Fig. stopshear):
    the top wall moves with u0 for ``startup`` steps, then stops. The wall is
    Zou and He's velocity boundary on the top node row, as in the paper
    (``top_wall="halfway"`` gives the half-link alternative). The paper's
    parameters in lattice units: theta = G tau / eta_s = 100 and
    u0 = 1e-2 L / tau_mu with tau_mu = eta_s / G and L the channel width,
    i.e. u0 = 1e-2 L G / eta_s (0.0191 here; the wall Peclet number
    gdot tau / gamma_c = 10). tau_lb = 0.6 keeps G tau = 3.3; the viscosity
    split 1/2 without the delta-rho terms is the well-conditioned setting for
    it. ``newtonian=True`` gives the solvent alone (G = 0) as a reference."""
    eta_s = (tau_lb - 0.5) / 3.0
    tau0 = theta * eta_s / G
    L = couette_width(ny, top_wall)
    u0 = wall_u_scale * L * G / eta_s
    spec = ChannelSpec(nx=nx, ny=ny, force=0.0, tau_lb=tau_lb, G=0.0 if newtonian else G, tau0=tau0,
                       gamma_c=gamma_c, eps=0.0, visc_split=0.0 if newtonian else 0.5, t_startup=startup,
                       wall_velocity=u0, nn_pressure=False, top_wall=top_wall)
    return {"name": f"couette_{nx}x{ny}" + ("_newtonian" if newtonian else "") +
            ("" if top_wall == "zou_he" else "_halfway"), "channels": [spec],
            "startup": startup, "cessation": 10000, "nn_pressure": False, "theta": theta, "width": L}


def pressure_channel(nx=64, ny=32, pressure_gradient=2e-6, tau_lb=1.0, G=1e-4, tau0=2e3, gamma_c=0.1,
                     startup=2 ** 62):
    """A channel driven by a pressure drop instead of a body force: the
    generalised periodic boundaries impose G_p = ``pressure_gradient``
    (equivalent to force = G_p), the forcing keeps its stress line only
    (``nn_pressure = 0`` on the handle). G tau = 0.2 keeps the explicit
    stress well conditioned. Start from ``linear_density_state``."""
    spec = ChannelSpec(nx=nx, ny=ny, force=0.0, tau_lb=tau_lb, G=G, tau0=tau0, gamma_c=gamma_c, eps=0.0,
                       visc_split=0.0, t_startup=startup, pressure_gradient=pressure_gradient)
    return {"name": f"pressure_channel_{nx}x{ny}", "channels": [spec], "nn_pressure": False}


def linear_density_state(spec):
    """Rest populations with the density falling linearly along x at the
    slope of the imposed pressure gradient, rho(x) = 1 + 3 G_p ((nx-1)/2 - x)
    (the switch-on pre-initialisation of Sec. II.B, which avoids the
    pressure wave of a sudden jump), and P = 0; layout of lb_get_state."""
    x = np.arange(spec.nx)
    rho = 1.0 + 3.0 * spec.pressure_gradient * ((spec.nx - 1) / 2.0 - x)
    pops = REST_WEIGHTS[:, None, None] * np.broadcast_to(rho[None, None, :], (9, spec.ny, spec.nx))
    return np.ascontiguousarray(pops), np.zeros((spec.ny, spec.nx))
