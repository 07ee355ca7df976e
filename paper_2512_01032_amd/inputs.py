"""Seeded synthetic workloads for the phase-field LB step.

This module only builds inputs: lattice sizes, physical parameters, solid
masks and initial fields.  It performs none of the method's arithmetic and is
the one module that both the GPU library's callers and the CPU oracle's tests
use, so that both sides start from identical arrays.

Conventions
-----------
* Arrays are numpy, indexed ``[z, y, x]`` (x fastest in memory), node
  ``n = x + nx*(y + ny*z)``.
* ``solid``: uint8, 0 = fluid, ``1 + k`` = solid of material ``k`` (< 16).
* ``faces``: six entries (x-, x+, y-, y+, z-, z+); each is ``None`` (periodic)
  or ``(P, ramp)`` for a pressure face whose layer holds ghost nodes with
  ``P(t) = P + ramp * t``.
* Initial order parameter: the planar equilibrium profile of the conservative
  Allen-Cahn equation (Sec. II.B, Eq. 17), phi = 1 in the liquid, applied to a
  signed distance; nodes sit at integer coordinates, walls half-way between the
  last fluid node and the first solid node.
* Unless a workload states otherwise: M = 1/6 (Sec. IV), W = 4, sigma = 1e-3,
  nu_l = 0.01, density ratio 1000, P_ref = 1/3, and the dynamic-viscosity
  ratio fixes nu_g = nu_l * (rho_l / rho_g) / ratio.  W = 4 rather than the
  W = 2.5 of Sec. IV: with central differences and a density ratio of 1000 the
  step is linearly unstable at W = 2.5 (a growing mode in the gas-side tail of
  the interface, present even with sigma = 0) and stable at W >= 3.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

T_G = 1.0 / 3.0  # D3Q19 lattice temperature; the reference pressure is P_ref = T_G


@dataclasses.dataclass
class Physics:
    rho_l: float = 1.0
    rho_g: float = 0.001
    nu_l: float = 0.01
    nu_g: float = 0.1
    sigma: float = 1e-3
    W: float = 4.0
    M: float = 1.0 / 6.0
    F_ex: tuple = (0.0, 0.0, 0.0)
    mobility_corr: bool = True
    gamma: float = -22.5
    phi_M: float = 0.8
    phi_m: float = 0.2
    D: float = 1e-4
    eps: float = 1e-10
    mix_tanh: bool = False          # Sec. II model: F(phi) = phi
    mix_phi: float = 0.1
    mix_width: float = 0.001
    interface_slip: bool = False    # Sec. III.A optimised model: free slip in the band
    slip_lo: float = 0.5
    slip_hi: float = 0.95
    # wall velocity in the band as a fraction of the tangential fluid
    # velocity: 1 the free slip of Sec. III.A, below 1 a partial slip
    slip_factor: float = 1.0
    P_ref: float = T_G
    # Sec. III.A wall-value blend with the previous step: 0/False off; 1/True
    # with the blended value that step used; 2 with that step's own
    # gradient-derived value
    hysteresis: int = 0
    hyst_beta: float = 0.95
    q_phase: int = 7                # phase-field lattice: 7 (D3Q7) or 19 (D3Q19, as in Sec. II.A)


def optimised(ph: Physics, hysteresis: int = 0) -> Physics:
    """The Sec. III.A model: tanh mixture switch and free slip in the band;
    with hysteresis 1 or 2 also the blend of each wall value with one kept
    from the previous step (factor hyst_beta; see Physics.hysteresis)."""
    return dataclasses.replace(ph, mix_tanh=True, interface_slip=True, hysteresis=hysteresis)


@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    phys: Physics
    phi0: np.ndarray
    solid: Optional[np.ndarray] = None
    # signed distance to the wall surface (> 0 in the fluid) for sub-voxel
    # walls; None: voxel walls half-way between fluid and solid nodes
    sdf: Optional[np.ndarray] = None
    u0: Optional[np.ndarray] = None
    P0: Optional[np.ndarray] = None
    faces: tuple = (None,) * 6
    theta_deg: tuple = (90.0,) * 16
    steps: int = 0
    storage: str = "fp32_shift"
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def n_nodes(self):
        return self.nx * self.ny * self.nz


def _grid(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def tanh_profile(signed_dist, W):
    """phi = 1/2 (1 - tanh(d / (W/2))); d < 0 inside the liquid."""
    return 0.5 * (1.0 - np.tanh(signed_dist / (0.5 * W)))


def visc_ratio_nu_g(nu_l, rho_l, rho_g, ratio):
    return nu_l * (rho_l / rho_g) / ratio


# --------------------------------------------------------------------------- C1
def static_droplet(n=32, R=8.0, W=4.0, steps=200, ratio_mu=100.0, storage="fp64"):
    """Static droplet, plain Sec. II model, periodic cube, droplet centred."""
    ph = Physics(W=W, nu_g=visc_ratio_nu_g(0.01, 1.0, 0.001, ratio_mu))
    x, y, z = _grid(n, n, n)
    c = (n - 1) / 2.0
    r = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
    return Workload("static_droplet_%d" % n, n, n, n, ph, tanh_profile(r - R, W),
                    steps=steps, storage=storage, meta={"R": R, "center": (c, c, c)})


# --------------------------------------------------------------------------- C2
def sessile_droplet(nx=128, ny=128, nz=96, R0=24.0, theta=60.0, top_theta=90.0,
                    steps=20000, storage="fp32_shift", W=4.0):
    """Hemispherical cap on a wetting wall at z = 0 (plane z = 0.5), top wall
    at z = nz-1; x and y periodic; optimised model."""
    ph = optimised(Physics(W=W, nu_g=visc_ratio_nu_g(0.01, 1.0, 0.001, 100.0)))
    x, y, z = _grid(nx, ny, nz)
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - 0.5) ** 2)
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[0] = 1          # material 0: bottom wall
    solid[nz - 1] = 2     # material 1: top wall
    th = [90.0] * 16
    th[0], th[1] = theta, top_theta
    return Workload("sessile_droplet", nx, ny, nz, ph, tanh_profile(r - R0, W), solid=solid,
                    theta_deg=tuple(th), steps=steps, storage=storage,
                    meta={"R0": R0, "theta": theta, "wall_z": 0.5, "center": (cx, cy)})


# --------------------------------------------------------------------------- C3
def capillary_filling(nx=1024, ny=32, nz=32, fill=128, theta=45.0, steps=50000,
                      ratio_mu=50.0, storage="fp32_shift", W=4.0, dP=0.0):
    """Square channel along x, walls at y, z in {0, n-1}, pressure ghosts at
    x = 0 (liquid reservoir side) and x = nx-1, liquid for x < fill."""
    ph = optimised(Physics(W=W, nu_g=visc_ratio_nu_g(0.01, 1.0, 0.001, ratio_mu)))
    x, y, z = _grid(nx, ny, nz)
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[:, 0, :] = 1
    solid[:, ny - 1, :] = 1
    solid[0, :, :] = 1
    solid[nz - 1, :, :] = 1
    th = [90.0] * 16
    th[0] = theta
    faces = ((ph.P_ref + dP, 0.0), (ph.P_ref, 0.0), None, None, None, None)
    phi0 = tanh_profile(x - (fill - 0.5), W)
    return Workload("capillary_filling", nx, ny, nz, ph, phi0, solid=solid, faces=faces,
                    theta_deg=tuple(th), steps=steps, storage=storage,
                    meta={"fill": fill, "theta": theta, "width": ny - 2})


def channel_filling_2d(nx=128, nz=18, fill=30, theta=45.0, ratio_mu=50.0, W=4.0, nu_l=0.01,
                       storage="fp64", dP=0.0):
    """Quasi-2D capillary intrusion (y of width 1, periodic): plates at z = 0
    and z = nz - 1 (material 0, angle theta; channel height nz - 2 between the
    half-way walls), pressure ghosts at P_ref + dP at x = 0 (liquid reservoir
    side) and at P_ref at x = nx - 1, liquid for x < fill; the optimised
    model."""
    ph = optimised(Physics(W=W, nu_l=nu_l, nu_g=visc_ratio_nu_g(nu_l, 1.0, 0.001, ratio_mu)))
    x, y, z = _grid(nx, 1, nz)
    solid = np.zeros((nz, 1, nx), np.uint8)
    solid[0] = 1
    solid[nz - 1] = 1
    th = [90.0] * 16
    th[0] = theta
    faces = ((ph.P_ref + dP, 0.0), (ph.P_ref, 0.0), None, None, None, None)
    phi0 = tanh_profile(x - (fill - 0.5), W)
    return Workload("channel_filling_2d", nx, 1, nz, ph, phi0, solid=solid, faces=faces,
                    theta_deg=tuple(th), storage=storage,
                    meta={"fill": fill, "theta": theta, "H": nz - 2})


# --------------------------------------------------------------------------- C4
def slug_positions(seed=0, start=16, end=256, lo=20, hi=60):
    rng = np.random.default_rng(seed)
    out = []
    pos = start
    while True:
        gap = int(rng.integers(lo, hi + 1))
        length = int(rng.integers(lo, hi + 1))
        a = pos + gap
        b = a + length
        if b >= end:
            break
        out.append((a, b))
        pos = b
    return out


def constricted_duct(nx=256, ny=256, nz=512, step_z=256, theta=120.0, ramp_to=2e-3,
                     ramp_steps=10000, seed=0, steps=10000, storage="fp32_shift", W=4.0,
                     slug_offset=0.0):
    """Square duct along z with walls at x, y in {0, n-1}; from z = step_z on,
    only the centred half-width square is fluid.  z = 0 is a pressure inlet
    ramped linearly by ramp_to over ramp_steps, z = nz-1 an outlet at P_ref.
    Liquid slugs of seeded random length and spacing sit in the wide part;
    slug_offset shifts every slug end along z (a non-zero fraction of a cell
    leaves no slug mid-plane on a node)."""
    ph = optimised(Physics(W=W, nu_g=visc_ratio_nu_g(0.01, 1.0, 0.001, 100.0)))
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[:, 0, :] = 1
    solid[:, ny - 1, :] = 1
    solid[:, :, 0] = 1
    solid[:, :, nx - 1] = 1
    qx0, qx1 = nx // 4, nx - nx // 4
    qy0, qy1 = ny // 4, ny - ny // 4
    narrow = np.ones((ny, nx), np.uint8)
    narrow[qy0:qy1, qx0:qx1] = 0
    solid[step_z:] = np.maximum(solid[step_z:], narrow[None])
    slugs = slug_positions(seed, 16, step_z)
    zc = np.arange(nz, dtype=np.float64)
    phz = np.zeros(nz)
    for a, b in slugs:
        za, zb = a - 0.5 + slug_offset, b - 0.5 + slug_offset
        phz += 0.5 * (np.tanh((zc - za) / (0.5 * W)) - np.tanh((zc - zb) / (0.5 * W)))
    phz = np.clip(phz, 0.0, 1.0)
    phi0 = np.broadcast_to(phz[:, None, None], (nz, ny, nx)).copy()
    th = [90.0] * 16
    th[0] = theta
    faces = (None, None, None, None, (ph.P_ref, ramp_to / ramp_steps), (ph.P_ref, 0.0))
    return Workload("constricted_duct", nx, ny, nz, ph, phi0, solid=solid, faces=faces,
                    theta_deg=tuple(th), steps=steps, storage=storage,
                    meta={"slugs": slugs, "step_z": step_z, "slug_offset": slug_offset})


def duct_sdf(wl, offset=0.3):
    """Signed distance of the constricted duct's fluid region with every wall
    surface moved offset (0 <= offset < 0.5) into the fluid from its half-way
    position: the same solid nodes, every wall link at fraction 0.5 - offset.
    Built from the planes of the wide duct, the narrow square and the step
    face (max of the two parts, min within each)."""
    nx, ny, nz = wl.nx, wl.ny, wl.nz
    step_z = wl.meta["step_z"]
    x, y, z = _grid(nx, ny, nz)
    lo, hi = 0.5 + offset, -1.5 - offset
    wide = np.minimum(np.minimum(x - lo, nx + hi - x), np.minimum(y - lo, ny + hi - y))
    qx0, qx1 = nx // 4, nx - nx // 4
    qy0, qy1 = ny // 4, ny - ny // 4
    narrow = np.minimum(np.minimum(x - (qx0 - 0.5 + offset), (qx1 - 0.5 - offset) - x),
                        np.minimum(y - (qy0 - 0.5 + offset), (qy1 - 0.5 - offset) - y))
    before_step = np.minimum(wide, (step_z - 0.5 - offset) - z)
    sdf = np.maximum(before_step, np.minimum(narrow, wide))
    assert ((sdf <= 0) == (wl.solid > 0)).all()
    return sdf


def wall_cap_2d(theta, nx=64, nz=24, R=11.0, W=4.0, steps=8000, storage="fp64"):
    """Quasi-2D cylindrical cap (y of width 1, periodic) on a wall at z = 0
    (material 0, angle theta) under a neutral wall at z = nz - 1, centred at
    x = (nx - 1)/2, initial radius R about the wall plane z = 0.5; Sec. II
    model."""
    ph = Physics(W=W)
    x, y, z = _grid(nx, 1, nz)
    r = np.sqrt((x - (nx - 1) / 2.0) ** 2 + (z - 0.5) ** 2)
    solid = np.zeros((nz, 1, nx), np.uint8)
    solid[0] = 1
    solid[nz - 1] = 2
    th = [90.0] * 16
    th[0] = theta
    return Workload("cap2d_%g" % theta, nx, 1, nz, ph, tanh_profile(r - R, W), solid=solid,
                    theta_deg=tuple(th), steps=steps, storage=storage,
                    meta={"theta": theta, "wall_z": 0.5})


# --------------------------------------------------------------------------- C5
def droplet_on_wall(e, theta, steps, storage="fp32_shift", W=4.0):
    ph = optimised(Physics(W=W, nu_g=visc_ratio_nu_g(0.01, 1.0, 0.001, 100.0)))
    x, y, z = _grid(e, e, e)
    c = (e - 1) / 2.0
    r = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - 0.5) ** 2)
    solid = np.zeros((e, e, e), np.uint8)
    solid[0] = 1
    solid[e - 1] = 2
    th = [90.0] * 16
    th[0] = theta
    return Workload("droplet_%d" % e, e, e, e, ph, tanh_profile(r - e / 4.0, W), solid=solid,
                    theta_deg=tuple(th), steps=steps, storage=storage,
                    meta={"theta": theta})


def channel_filling(e, theta, steps, storage="fp32_shift", W=4.0):
    nx, ny, nz = 2 * e, e // 2, e // 2
    wl = capillary_filling(nx, ny, nz, fill=e // 4, theta=theta, steps=steps,
                           ratio_mu=100.0, storage=storage, W=W)
    wl.name = "channel_%d" % e
    return wl


@dataclasses.dataclass
class Request:
    index: int
    arrival_s: float
    kind: str
    edge: int
    theta: float
    steps: int
    seed: int

    def workload(self, storage="fp32_shift"):
        if self.kind == "droplet":
            return droplet_on_wall(self.edge, self.theta, self.steps, storage)
        return channel_filling(self.edge, self.theta, self.steps, storage)


def serving_trace(n=256, rate=50.0, seed=1, edges=(32, 48, 64, 96, 128),
                  steps_lo=2000, steps_hi=10000, theta_lo=30.0, theta_hi=150.0):
    """Poisson arrivals (exponential gaps, mean 1/rate); request i draws its
    case from seed 1000 + i."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n):
        r = np.random.default_rng(1000 + i)
        kind = "droplet" if r.random() < 0.5 else "channel"
        edge = int(r.choice(edges))
        theta = float(r.uniform(theta_lo, theta_hi))
        steps = int(r.integers(steps_lo, steps_hi + 1))
        out.append(Request(i, float(t[i]), kind, edge, theta, steps, 1000 + i))
    return out


# ------------------------------------------------------------- small test cases
def random_small(nx, ny, nz, seed, walls=False, open_x=False, storage="fp64",
                 u_amp=0.01, optimised_model=False, subvoxel=False):
    """A small lattice with a random smooth phi field, small random velocity
    and optional walls (y = 0 and z = 0 solid layers of two materials) and
    pressure faces along x; used for parity on tiny grids.  subvoxel (with
    walls): the wall surfaces are wavy sheets inside the cells between the
    solid layers and the first fluid nodes, given by a signed distance, so
    every wall link has its own fraction and the normals tilt."""
    rng = np.random.default_rng(seed)
    ph = Physics(W=4.0, nu_g=0.1)
    if optimised_model:
        ph = optimised(ph)
    x, y, z = _grid(nx, ny, nz)
    # sum of a few random spherical blobs gives interfaces in every direction
    phi = np.zeros((nz, ny, nx))
    for _ in range(3):
        c = rng.uniform(0, [nx, ny, nz])
        R = rng.uniform(1.5, max(2.0, min(nx, ny, nz) / 2.5))
        d = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) - R
        phi = np.maximum(phi, tanh_profile(d, ph.W))
    phi = np.clip(phi + rng.normal(0.0, 1e-3, phi.shape), -0.01, 1.01)
    u0 = rng.normal(0.0, u_amp, (3, nz, ny, nx))
    P0 = ph.P_ref + rng.normal(0.0, 1e-4, (nz, ny, nx))
    solid = None
    th = [90.0] * 16
    faces = [None] * 6
    if walls:
        solid = np.zeros((nz, ny, nx), np.uint8)
        solid[:, 0, :] = 1
        solid[0, :, :] = 2
        # a small obstacle gives concave and convex corners
        solid[nz // 2, ny // 2, nx // 2] = 1
        th[0], th[1] = float(rng.uniform(30, 80)), float(rng.uniform(100, 150))
    sdf = None
    if walls and subvoxel:
        # level sets y = 0.7 + 0.25 sin(kx) (+ a z wave) and z = 0.6 + 0.3 cos(kx):
        # the y = 0, z = 0 layers stay solid, the first fluid layers fluid
        k = 2 * np.pi / nx
        sy = y - (0.7 + 0.25 * np.sin(k * x) + 0.05 * np.cos(2 * np.pi * z / nz))
        sz = z - (0.6 + 0.3 * np.cos(k * x))
        sdf = np.minimum(sy, sz)
        # the obstacle: a sphere of radius 0.8 around its node
        c = (nx // 2, ny // 2, nz // 2)
        so = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) - 0.8
        sdf = np.minimum(sdf, so)
        assert ((sdf <= 0) == (solid > 0)).all()
    if open_x:
        faces[0] = (ph.P_ref + 2e-4, 1e-6)
        faces[1] = (ph.P_ref, 0.0)
    return Workload("random_%dx%dx%d_s%d" % (nx, ny, nz, seed), nx, ny, nz, ph, phi,
                    solid=solid, sdf=sdf, u0=u0, P0=P0, faces=tuple(faces), theta_deg=tuple(th),
                    storage=storage)


def offset_plates(ny, delta, nx=1, nz=1, ph=None, phi0=None, theta=90.0, storage="fp64"):
    """Plates normal to y with their surfaces offset by delta (0 <= delta < 1)
    from the lattice-aligned case: walls at y0 = 0.5 + delta and
    y1 = ny - 1.5 - delta, given by the signed distance min(y - y0, y1 - y);
    nodes at or beyond a surface are solid.  Single phase (phi = 1) unless
    phi0 is given."""
    ph = ph if ph is not None else Physics()
    x, y, z = _grid(nx, ny, nz)
    y0, y1 = 0.5 + delta, ny - 1.5 - delta
    sdf = np.minimum(y - y0, y1 - y)
    solid = (sdf <= 0).astype(np.uint8)
    phi = np.ones((nz, ny, nx)) if phi0 is None else phi0
    return Workload("plates_%d_d%.2f" % (ny, delta), nx, ny, nz, ph, phi, solid=solid, sdf=sdf,
                    theta_deg=(theta,) * 16, storage=storage,
                    meta={"y0": y0, "y1": y1})
