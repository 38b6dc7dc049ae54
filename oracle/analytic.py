"""Closed forms and quadratures the paper fixes, used to pin the oracle.

TEST INFRASTRUCTURE ONLY.

Lattice units (dx = dt = 1, rho0 = 1). A channel of ``ny`` fluid rows between
half-way bounce-back walls has its walls at y = -1/2 and y = ny - 1/2, half
width H = ny/2 and centre y_c = (ny - 1)/2. ``eta_s`` is the solvent
(high-shear) viscosity carried by the BGK collision, eta_s = (tau_LB - 1/2)/3.
"""
import math

import numpy as np
from scipy import integrate


# ---------------------------------------------------------------- rheology --

def simple_shear(gdot, G, tau, gamma_c):
    """nlM steady stress in simple shear kappa_xy = gdot (Sec. III.A):
    tau_M from Eq. (nlmaxwell) with II_D = gdot^2; sigma_xy = G gdot tau_M,
    N1 = sigma_xx - sigma_yy = 2 G gdot^2 tau_M^2, sigma_yy = 0."""
    tauM = 1.0 / (1.0 / tau + abs(gdot) / gamma_c)
    sxy = G * gdot * tauM
    n1 = 2.0 * G * gdot ** 2 * tauM ** 2
    return {"tauM": tauM, "sxx": n1, "sxy": sxy, "syy": 0.0, "N1": n1}


def planar_extension_sxx(edot, G, tauM):
    """sigma_xx in planar extension kappa = diag(edot, -edot) at fixed tau_M
    (Sec. III.A, the upper-convected Maxwell example): 2 G edot tau /(1 - 2 edot tau),
    valid for edot tau_M < 1/2."""
    return 2.0 * G * edot * tauM / (1.0 - 2.0 * edot * tauM)


def II_D_shear(gdot):
    return gdot ** 2


def II_D_extension(edot):
    return (2.0 * edot) ** 2


# ------------------------------------------------- steady channel profile --

def paper_dvdd(d, wpH, theta, gamma_c):
    """The paper's steady shear rate in the upper channel half,
    Eq. (maxwellpoiseuille), in its dimensionless variables (d = y/H,
    v = u_x tau_0 / H, wp = dp/G, theta = tau/tau_0)."""
    a = wpH * d / 2.0
    b = gamma_c * (1.0 + theta) / (2.0 * theta)
    return -a + b - np.sqrt((a - b) ** 2 + wpH * d * gamma_c / theta)


def shear_rate(a, eta_s, G, tau, gamma_c):
    """Shear rate gdot >= 0 at which the total shear stress
    eta_s gdot + G gdot tau_M(gdot) equals a >= 0 (the quadratic of Sec. III.B
    in lattice units; stable root). tau = inf gives the Bingham limit."""
    a = np.asarray(a, dtype=np.float64)
    if G == 0:
        return a / eta_s
    if math.isinf(tau):
        return np.maximum(a - G * gamma_c, 0.0) / eta_s
    A = eta_s * tau / gamma_c
    B = eta_s + G * tau - a * tau / gamma_c
    return 2.0 * a / (B + np.sqrt(B * B + 4.0 * A * a))


def steady_profile(ny, g, eta_s, G, tau, gamma_c):
    """Analytic steady u_x at the lattice rows y = 0..ny-1 of a body-force
    driven channel: the shear stress at distance xi from the centre is g xi,
    and u(xi) = integral_xi^H gdot(g s) ds with no slip at the walls xi = H."""
    H = ny / 2.0
    yc = (ny - 1) / 2.0
    xi = np.abs(np.arange(ny) - yc)

    def rate(s):
        return float(shear_rate(g * s, eta_s, G, tau, gamma_c))

    kink = G * gamma_c / g if (G > 0 and g > 0) else None
    u = np.empty(ny)
    for k, x0 in enumerate(xi):
        pts = [kink] if kink is not None and x0 < kink < H else None
        val, _ = integrate.quad(rate, x0, H, points=pts, epsabs=0, epsrel=1e-13, limit=400)
        u[k] = val
    return u


def steady_rows(ny, g, eta_s, G, tau, gamma_c):
    """Steady shear rate, sigma_xy and N1 at the lattice rows (signed for the
    lower half, where d_y u_x > 0)."""
    yc = (ny - 1) / 2.0
    dy = np.arange(ny) - yc
    gd = shear_rate(g * np.abs(dy), eta_s, G, tau, gamma_c)
    gd = -np.sign(dy) * gd
    tauM = 1.0 / (1.0 / tau + np.abs(gd) / gamma_c) if G > 0 else np.zeros(ny)
    return {"kxy": gd, "sxy": G * gd * tauM, "N1": 2 * G * gd ** 2 * tauM ** 2}


def newtonian_parabola(ny, g, eta):
    H = ny / 2.0
    yc = (ny - 1) / 2.0
    xi = np.arange(ny) - yc
    return g * (H * H - xi * xi) / (2.0 * eta)


def newtonian_startup(ny, g, eta, t, kmax=2000):
    """Start-up of Newtonian Poiseuille flow from rest (Fourier series of the
    diffusion equation with no slip at xi = +-H): u(xi, t) =
    sum_k 16 g H^2 (-1)^k / (eta pi^3 (2k+1)^3) cos(mu_k xi) (1 - exp(-eta mu_k^2 t)),
    mu_k = (2k+1) pi / (2H)."""
    H = ny / 2.0
    yc = (ny - 1) / 2.0
    xi = np.arange(ny) - yc
    k = np.arange(kmax)
    mu = (2 * k + 1) * math.pi / (2 * H)
    coef = 16 * g * H * H * (-1.0) ** k / (eta * math.pi ** 3 * (2 * k + 1) ** 3)
    return (coef[None, :] * np.cos(np.outer(xi, mu)) * (1 - np.exp(-eta * mu[None, :] ** 2 * t))).sum(axis=1)


def couette_width(ny, top_wall="halfway"):
    """Distance between the fixed wall at y = -1/2 and the moving wall: the
    half link y = ny - 1/2 ("halfway") or the top node row y = ny - 1
    ("zou_he")."""
    return float(ny) if top_wall == "halfway" else ny - 0.5


def newtonian_couette_startup(ny, U, eta, t, kmax=2000, rho0=1.0, top_wall="halfway"):
    """Start-up of planar Couette flow from rest (Sec. IV.B): walls at
    y = -1/2 (at rest) and y = -1/2 + H (moving with U from t = 0), H from
    couette_width, s = (y + 1/2)/H. Steady part U s; the transient solves the
    diffusion equation with zero wall values, starting from -U s, whose sine
    series has coefficients -2U (-1)^(n+1) / (n pi): u = U s - (2U/pi) sum
    (-1)^(n+1)/n sin(n pi s) exp(-(eta/rho0) (n pi/H)^2 t)."""
    H = couette_width(ny, top_wall)
    s = (np.arange(ny) + 0.5) / H
    n = np.arange(1, kmax + 1)[:, None]
    terms = ((-1.0) ** (n + 1) / n) * np.sin(n * math.pi * s[None, :]) * np.exp(
        -(eta / rho0) * (n * math.pi / H) ** 2 * t)
    return U * s - (2 * U / math.pi) * terms.sum(axis=0)


def bingham_stop_bound(u_rows, eta, sigma_y, ny, rho0=1.0, width=None):
    """Upper bound on the stopping time of a Bingham fluid (yield stress
    sigma_y, plastic viscosity eta) released from the profile u_rows in a
    channel of width 2H between no-slip walls (H = ny/2 unless ``width``
    gives 2H; Sec. III.B, finite stopping time). From the energy balance
    (rho0/2) d|u|^2/dt = -eta |u'|^2 - sigma_y |u'|_1 with
    |u'|^2 >= lambda1 |u|^2, lambda1 = (pi/2H)^2, and |u'|_1 >= beta |u|,
    beta = sqrt(2/H): t_f <= rho0/(eta lambda1) ln(1 + eta lambda1 Y0 /(sigma_y beta)),
    Y0 = |u(0)|_2."""
    H = (ny if width is None else width) / 2.0
    lam1 = (math.pi / (2 * H)) ** 2
    beta = math.sqrt(2.0 / H)
    Y0 = float(np.sqrt(np.sum(np.asarray(u_rows) ** 2)))
    return rho0 / (eta * lam1) * math.log1p(eta * lam1 * Y0 / (sigma_y * beta))


def dimensionless(ny, g, eta_s, G, tau, gamma_c, rho0=1.0):
    """Map lattice parameters to the paper's dimensionless groups
    (Sec. III.B): tau_0 = eta_s / G, theta = tau / tau_0, wp H = g H / G,
    Re = rho0 H^2 / (eta_s tau_0)."""
    H = ny / 2.0
    tau_0 = eta_s / G
    return {"tau_0": tau_0, "theta": tau / tau_0, "wpH": g * H / G,
            "Re": rho0 * H * H / (eta_s * tau_0), "H": H}
