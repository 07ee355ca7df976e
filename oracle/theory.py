"""Closed-form results the oracle is checked against.

TEST INFRASTRUCTURE ONLY.  Each function states the textbook result or the
paper passage it writes out.
"""
from __future__ import annotations

import math


def duct_resistance_coefficient(h_over_w, terms=50):
    """Bracketed factor of the rectangular-duct Poiseuille pressure drop
    (Sec. III.A, Eq. 21): [1 - sum_n 192/((2n+1)^5 pi^5) (h/w)
    tanh((2n+1) pi w / (2h))]^-1, h and w the half-height and half-width."""
    s = 0.0
    for n in range(terms):
        k = 2 * n + 1
        s += 192.0 / (k ** 5 * math.pi ** 5) * h_over_w * math.tanh(k * math.pi / (2.0 * h_over_w))
    return 1.0 / (1.0 - s)


def washburn_2d(t, z0, L, H, sigma, theta_deg, mu1, mu2, dP=0.0):
    """Interface position of the 2D capillary intrusion (Sec. III.C, Eqs. 25-26):
    the positive root of (mu1-mu2)/2 z^2 + mu2 L z - (sigma cos(theta) H/6 +
    dP H^2/12) t - (mu1-mu2)/2 z0^2 - mu2 L z0 = 0."""
    a = 0.5 * (mu1 - mu2)
    b = mu2 * L
    drive = sigma * math.cos(math.radians(theta_deg)) * H / 6.0 + dP * H * H / 12.0
    c = -drive * t - a * z0 * z0 - b * z0
    if abs(a) < 1e-300:
        return -c / b
    return (-b + math.sqrt(b * b - 4.0 * a * c)) / (2.0 * a)


def washburn_square_duct(t, z0, L, a, sigma, theta_deg, mu1, mu2, dP=0.0, k=28.45):
    """Liquid length in a square duct of side a filled by capillarity (Sec.
    III.C, the Washburn balance of Eqs. 25-26 with the duct's Poiseuille
    resistance): the mean velocity of a square duct is G a^2 / (k mu) with
    k = 28.45, and the capillary pressure 4 sigma cos(theta) / a, so
    [mu1 z + mu2 (L - z)] dz/dt = (a^2 / k)(4 sigma cos(theta) / a + dP);
    the positive root of the integrated quadratic."""
    A = 0.5 * (mu1 - mu2)
    B = mu2 * L
    drive = (a * a / k) * (4.0 * sigma * math.cos(math.radians(theta_deg)) / a + dP)
    c = -drive * t - A * z0 * z0 - B * z0
    if abs(A) < 1e-300:
        return -c / B
    return (-B + math.sqrt(B * B - 4.0 * A * c)) / (2.0 * A)


def laplace_pressure(sigma, R, dim=3):
    """Young-Laplace jump across a static interface of radius R: 2 sigma / R
    for a sphere, sigma / R for a cylinder."""
    return (2.0 if dim == 3 else 1.0) * sigma / R


def poiseuille_profile(y, y0, y1, force, rho, nu):
    """Plane Poiseuille flow between walls at y0 and y1 driven by a body force
    per unit volume: u(y) = F/(2 rho nu) (y - y0)(y1 - y)."""
    return force / (2.0 * rho * nu) * (y - y0) * (y1 - y)


def taylor_green_decay(nu, k, t):
    """Amplitude factor of a 2D Taylor-Green vortex of wavenumber k in both
    directions: exp(-2 nu k^2 t)."""
    return math.exp(-2.0 * nu * k * k * t)


def cap_angle_from_circle(zc, R, z_wall):
    """Contact angle (through the liquid inside the circle) of a circular cap
    whose circle has centre height zc and radius R over a wall plane z_wall."""
    c = (z_wall - zc) / R
    return math.degrees(math.acos(max(-1.0, min(1.0, c))))


def mixture_dynamic_viscosity(phi, rho_l, rho_g, nu_l, nu_g, mix_tanh, mix_phi=0.1, mix_width=0.001):
    """Dynamic viscosity rho(phi) nu(phi) of the mixture: rho linear in the
    clipped phi (Eq. 9), the relaxation time interpolated between the two
    fluids' by F(phi) (Eqs. 10-12: F = phi; Sec. III.A: F = [tanh((phi -
    mix_phi) / mix_width) + 1] / 2), nu = (tau - 1/2) / 3.  Works on arrays."""
    import numpy as np
    pb = np.clip(np.asarray(phi, dtype=float), 0.0, 1.0)
    rho = rho_g + pb * (rho_l - rho_g)
    F = 0.5 * (np.tanh((pb - mix_phi) / mix_width) + 1.0) if mix_tanh else pb
    tau = (1.0 - F) * (3.0 * nu_g + 0.5) + F * (3.0 * nu_l + 0.5)
    return rho * (tau - 0.5) / 3.0


def poiseuille_intrusion_travel(t, M0, dmu, drive):
    """Distance s travelled in time t by a liquid column in a plane channel
    whose viscous resistance is sum over the channel of the dynamic
    viscosity, M0 + dmu s (dmu = mu_liquid - mu_gas), driven by a pressure
    drop p (per unit height squared over 12, drive = p H^2 / 12): the
    positive root of dmu s^2 / 2 + M0 s = drive t (plane Poiseuille flow,
    mean velocity = p H^2 / (12 mu L))."""
    a = 0.5 * dmu
    if abs(a) < 1e-300:
        return drive * t / M0
    return (-M0 + math.sqrt(M0 * M0 + 4.0 * a * drive * t)) / (2.0 * a)
