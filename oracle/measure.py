"""Post-processing of oracle fields for the physics pins.

TEST INFRASTRUCTURE ONLY: contour extraction, circle fit, interface position.
"""
from __future__ import annotations

import numpy as np


def crossings_1d(v, level=0.5):
    """Fractional indices where the 1-D array v crosses level (linear)."""
    out = []
    for i in range(len(v) - 1):
        a, b = v[i] - level, v[i + 1] - level
        if a == 0.0:
            out.append(float(i))
        elif a * b < 0.0:
            out.append(i + a / (a - b))
    return out


def contour_points_xz(phi_xz, level=0.5, z_min=1):
    """Points (x, z) of the level contour of a 2-D field phi[z, x], taken from
    crossings along every column and every row (z >= z_min)."""
    pts = []
    nz, nx = phi_xz.shape
    for x in range(nx):
        for zf in crossings_1d(phi_xz[z_min:, x], level):
            pts.append((float(x), zf + z_min))
    for z in range(z_min, nz):
        for xf in crossings_1d(phi_xz[z, :], level):
            pts.append((xf, float(z)))
    return np.array(pts)


def fit_circle(pts):
    """Algebraic least-squares circle through points (Kasa fit)."""
    x, y = pts[:, 0], pts[:, 1]
    A = np.column_stack([x, y, np.ones_like(x)])
    b = x * x + y * y
    sol, *_ = np.linalg.lstsq(A, b, rcond=None)
    xc, yc = sol[0] / 2.0, sol[1] / 2.0
    R = np.sqrt(sol[2] + xc * xc + yc * yc)
    return xc, yc, R


def cap_angle_3d(phi, wall_z, cx, cy):
    """Contact angle (degrees) and radius of a sessile cap on the wall plane
    z = wall_z, from its axial x-z section: phi on the plane y = cy (linear
    between the two nearest node planes), the 0.5 contour above the first
    fluid layer and away from the wall-adjacent cells, fitted by a circle;
    the angle is that of the circle meeting the wall plane."""
    from oracle import theory
    y0 = int(np.floor(cy))
    f = cy - y0
    sec = (1.0 - f) * phi[:, y0, :] + f * phi[:, y0 + 1, :]
    pts = contour_points_xz(sec, z_min=1)
    pts = pts[pts[:, 1] > wall_z + 2.0]
    xc, zc, R = fit_circle(pts)
    return theory.cap_angle_from_circle(zc, R, wall_z), float(R)
