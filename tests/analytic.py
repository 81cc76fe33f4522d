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


def inner_profile_front(rate, n_H, sigma, alpha_B):
    """Radius where x = 0.5 in the equilibrium profile of Eq.
    inner_stromgren_region (monochromatic): (1 - x) rate sigma e^-tau /
    (4 pi r^2) = x^2 n_H alpha_B, dtau/dr = (1 - x) n_H sigma, integrated
    outwards with classical RK4 from r_S/1000 (x -> 1 there)."""
    def x_of(r, tau):
        a = rate * sigma * math.exp(-tau) / (4.0 * math.pi * r * r)
        b = n_H * alpha_B
        return (-a + math.sqrt(a * a + 4.0 * b * a)) / (2.0 * b)
    r_s = stromgren_radius(rate, n_H, alpha_B)
    r, tau, h = 1e-3 * r_s, 0.0, 1e-4 * r_s
    f = lambda r_, t_: (1.0 - x_of(r_, t_)) * n_H * sigma
    while x_of(r, tau) >= 0.5:
        k1 = f(r, tau)
        k2 = f(r + h / 2, tau + h / 2 * k1)
        k3 = f(r + h / 2, tau + h / 2 * k2)
        k4 = f(r + h, tau + h * k3)
        tau += h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        r += h
    return r


def slab_front(flux, n_H, sigma, alpha_B):
    """Depth where x = 0.5 in the 1-D equilibrium of a plane-parallel flux
    entering a uniform slab: sigma F y = alpha_B n_H (1 - y)^2 at each
    depth, dF/dz = -n_H sigma y F, RK4 in steps of 1e17 cm."""
    a = alpha_B * n_H

    def y_of(F):
        c = sigma * F
        return ((2 * a + c) - math.sqrt((2 * a + c) ** 2 - 4 * a * a)) / (2 * a)
    z, F, h = 0.0, flux, 1e17
    f = lambda F_: -n_H * sigma * y_of(F_) * F_
    while 1.0 - y_of(F) >= 0.5:
        k1 = f(F)
        k2 = f(F + h / 2 * k1)
        k3 = f(F + h / 2 * k2)
        k4 = f(F + h * k3)
        F += h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        z += h
    return z


def half_crossing(r, x, width, exclude=None):
    """First outward crossing of x = 0.5 of the profile averaged over shells
    (bins) of the given width, linearly interpolated between bin centres."""
    keep = np.ones(r.shape[0], bool)
    if exclude is not None:
        keep[exclude] = False
    r, x = r[keep], x[keep]
    edges = np.arange(0.0, r.max() + width, width)
    cen, val = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        msk = (r >= a) & (r < b)
        if msk.any():
            cen.append(0.5 * (a + b))
            val.append(float(x[msk].mean()))
    cen, val = np.array(cen), np.array(val)
    i = int(np.argmax(val < 0.5))
    assert i > 0 and val[i] < 0.5, "no crossing"
    return cen[i - 1] + (val[i - 1] - 0.5) / (val[i - 1] - val[i]) * (cen[i] - cen[i - 1])
