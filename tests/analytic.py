"""Analytic references for the isothermal H II region (Sect. 5.1) and the
rate equation (Sect. 4.2).  Test infrastructure."""
import math

import numpy as np


def stromgren_radius(rate, n_H, alpha_B):
    """Eq. stromgren_radius: r_S = (3 N_dot / (4 pi alpha_B n_H^2))^(1/3)."""
    return (3.0 * rate / (4.0 * math.pi * alpha_B * n_H * n_H)) ** (1.0 / 3.0)


def recombination_time(n_H, alpha_B):
    """t_rec = 1 / (alpha_B n_H) (Sect. 4.2, recombination time scale for a
    fully ionised gas, n_e = n_H)."""
    return 1.0 / (alpha_B * n_H)


def front_radius(t, r_s, t_rec):
    """Eq. IFront_pos: r_I = r_S (1 - exp(-t/t_rec))^(1/3)."""
    return r_s * (1.0 - np.exp(-np.asarray(t) / t_rec)) ** (1.0 / 3.0)


def front_velocity(t, r_s, t_rec):
    """Eq. IFront_vel."""
    e = np.exp(-np.asarray(t) / t_rec)
    return r_s / (3.0 * t_rec) * e / (1.0 - e) ** (2.0 / 3.0)


def ionised_volume_radius(volume, x):
    """Radius of the sphere holding the ionised volume sum V_j x_j."""
    return (3.0 / (4.0 * math.pi) * float(np.sum(volume * x))) ** (1.0 / 3.0)


def recombination_only(x0, b, t):
    """Closed form of dx/dt = -b x^2 (rate equation without photons, n_e =
    n_HII, b = alpha_B n_H): x(t) = x0 / (1 + b x0 t)."""
    return x0 / (1.0 + b * x0 * t)


def equilibrium_neutral_fraction(a, b, tau):
    """Root y in (0, 1] of a (1 - exp(-y tau)) = b (1 - y)^2: photo-
    ionisations of a cell with constant incoming flux balance recombinations."""
    from scipy.optimize import brentq
    f = lambda y: a * (-math.expm1(-y * tau)) - b * (1.0 - y) ** 2
    if f(1.0) <= 0.0:
        return 1.0
    return brentq(f, 0.0, 1.0, xtol=1e-300, rtol=1e-15, maxiter=500)


def rate_ode_solution(y0, a, b, tau, t):
    """dy/dt = -a (1 - exp(-y tau)) + b (1 - y)^2 integrated with an
    implicit Runge-Kutta method (Radau IIA) at tight tolerances."""
    from scipy.integrate import solve_ivp
    f = lambda _t, y: [-a * (-math.expm1(-y[0] * tau)) + b * (1.0 - y[0]) ** 2]
    sol = solve_ivp(f, (0.0, t), [y0], method="Radau", rtol=1e-12, atol=1e-15)
    return float(sol.y[0, -1])
