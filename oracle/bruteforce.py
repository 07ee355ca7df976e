"""Whole-lattice NumPy reference of the phase-field LB step for tiny grids.

TEST INFRASTRUCTURE ONLY.  Every array operation acts on the full lattice,
direction by direction: neighbour values come from ``np.roll`` and streaming is
one roll per direction with masks for solid links and pressure ghosts.  This is
a second, structurally different transcription of the same step as the C
oracle (which loops node by node and indexes neighbours explicitly); agreement
between the two pins the C oracle's indexing, wrap-around, bounce-back and
ghost bookkeeping.  Both follow the same reading of the paper, so this file
does not pin the formulas themselves -- the physics tests do that.

Paper parts (same equation numbering as the C oracle):
  phi = sum h (after Eq. 4); gradient/Laplacian (Eq. 16); wetting value
  phi_s,i (Eqs. 17-19); chemical potential (Eq. 9); tau_mix (Eqs. 10-12 and
  the tanh switch of Sec. III.A); moments (after Eq. 15); filtered collision
  (Eqs. 6-8, 13-15); phase-field collision (Eqs. 1-5).
"""
from __future__ import annotations

import numpy as np

C = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
              [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1],
              [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])
WG = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
WH = np.array([1 / 4] + [1 / 8] * 6)
TG, TH = 1.0 / 3.0, 0.25
OPP = np.array([int(np.where((C == -C[i]).all(axis=1))[0][0]) for i in range(19)])


def shifted(a, c, sign):
    """Value of field a at x + sign*c for every x (periodic)."""
    return np.roll(a, shift=(-sign * c[2], -sign * c[1], -sign * c[0]), axis=(-3, -2, -1))


class BruteForce:
    def __init__(self, wl, clamp_a=1e-12):
        self.wl = wl
        ph = wl.phys
        self.ph = ph
        self.clamp_a = clamp_a
        shape = wl.shape
        self.shape = shape
        nz, ny, nx = shape
        solid = np.zeros(shape, np.uint8) if wl.solid is None else wl.solid.astype(np.uint8)
        self.solid = solid > 0
        self.mat = np.where(self.solid, solid.astype(int) - 1, 0)
        # ghosts: non-solid nodes on a pressure-face layer
        self.ghost = np.zeros(shape, bool)
        self.gface = -np.ones(shape, int)
        zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        coord = (xx, yy, zz)
        dims = (nx, ny, nz)
        for f in range(6):
            if wl.faces[f] is None:
                continue
            ax = f // 2
            layer = 0 if f % 2 == 0 else dims[ax] - 1
            on = (coord[ax] == layer) & ~self.solid
            assert not (self.ghost & on).any(), "ghost on two pressure faces"
            self.ghost |= on
            self.gface[on] = f
        self.fluid = ~self.solid & ~self.ghost
        # wall normal
        v = np.zeros((3,) + shape)
        for i in range(1, 19):
            sm = shifted(self.solid, C[i], +1)
            for a in range(3):
                v[a] -= WG[i] * C[i][a] * sm
        nv = np.sqrt((v ** 2).sum(0))
        self.nw = np.where(nv > 0, v / np.where(nv > 0, nv, 1.0), 0.0) * self.fluid
        # sub-voxel walls: link fractions q[i] (where x + c_i is solid) and
        # normals from the signed distance, for fluid nodes with a solid link
        self.q = None
        self.same_step = bool(getattr(wl, "meta", {}).get("subvoxel_same_step", False))
        sdf = getattr(wl, "sdf", None)
        if sdf is not None:
            near = np.zeros(shape, bool)
            self.q = np.full((19,) + shape, 0.5)
            for i in range(1, 19):
                link = shifted(self.solid, C[i], +1) & self.fluid
                near |= link
                far = shifted(sdf, C[i], +1)
                assert (sdf[link] > 0).all() and (far[link] <= 0).all(), "sdf does not straddle"
                self.q[i] = np.where(link, sdf / np.where(link, sdf - far, 1.0), 0.5)
            gsd = np.zeros((3,) + shape)
            for i in range(1, 19):
                for a in range(3):
                    gsd[a] += WG[i] * C[i][a] * (shifted(sdf, C[i], +1) - shifted(sdf, C[i], -1))
            gl = np.sqrt((gsd ** 2).sum(0))
            ok = near & (gl > 0)
            self.nw = np.where(ok, gsd / np.where(ok, gl, 1.0), self.nw)
        self.t = 0
        # initial state
        phi = np.where(self.fluid, wl.phi0, 0.0)
        phi = self._ghost_copy(phi)
        self.phi = phi
        u = np.zeros((3,) + shape) if wl.u0 is None else wl.u0.copy()
        u = u * self.fluid
        P = np.full(shape, ph.P_ref) if wl.P0 is None else wl.P0.copy()
        self.hist = np.zeros((19,) + shape)     # wall values of the last step (hysteresis)
        grad, lap = self._stencil(phi, "set")
        heq = self._heq(phi, u, grad, lap)
        geq, K = self._geq(phi, u, P, grad, lap)
        self.h = heq * self.fluid
        self.g = geq * self.fluid
        self.u = u

    # ------------------------------------------------------------ helpers
    def _face_normal(self, f):
        n = [0, 0, 0]
        n[f // 2] = 1 if f % 2 == 0 else -1
        return np.array(n)

    def _owner_value(self, a):
        """a evaluated at the owner (one step inward) of every ghost node."""
        out = np.zeros_like(a)
        for f in range(6):
            if self.wl.faces[f] is None:
                continue
            m = self.gface == f
            out = np.where(m, shifted(a, self._face_normal(f), +1), out)
        return out

    def _ghost_copy(self, phi):
        return np.where(self.ghost, self._owner_value(phi), phi)

    def _phase_lattice(self):
        """Size, weights and temperature of the phase-field lattice."""
        if getattr(self.ph, "q_phase", 7) == 19:
            return 19, WG, TG
        return 7, WH, TH

    def _rho(self, phi):
        ph = self.ph
        return ph.rho_g + np.clip(phi, 0, 1) * (ph.rho_l - ph.rho_g)

    def _mu(self, phi, lap):
        ph = self.ph
        return 48 * ph.sigma / ph.W * phi * (phi - 1) * (phi - 0.5) - 1.5 * ph.sigma * ph.W * lap

    def _tau(self, phi):
        ph = self.ph
        pb = np.clip(phi, 0, 1)
        F = 0.5 * (np.tanh((pb - ph.mix_phi) / ph.mix_width) + 1) if ph.mix_tanh else pb
        return (1 - F) * (ph.nu_g / TG + 0.5) + F * (ph.nu_l / TG + 0.5)

    @staticmethod
    def _Gamma(w, c, u, T):
        cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2]
        uu = (u ** 2).sum(0)
        return w * (1 + cu / T + cu ** 2 / (2 * T * T) - uu / (2 * T))

    def _stencil(self, phi, hist_mode="eval"):
        """hist_mode (hysteresis only): "set" records the wall values,
        "step" blends them with the recorded ones and records the blend
        (hysteresis 1) or the unblended value (hysteresis 2), "eval" blends
        without recording."""
        ph = self.ph
        nb = np.zeros((19,) + self.shape)
        sol = np.zeros((19,) + self.shape, bool)
        matn = np.zeros((19,) + self.shape, int)
        for i in range(1, 19):
            sol[i] = shifted(self.solid, C[i], +1)
            matn[i] = shifted(self.mat, C[i], +1)
            nb[i] = np.where(sol[i], phi, shifted(phi, C[i], +1))
        # pre-gradient with the neutral value at solid links
        g0 = np.zeros((3,) + self.shape)
        for i in range(1, 19):
            for a in range(3):
                g0[a] += WG[i] * C[i][a] * nb[i] / TG
        nw = self.nw
        ng = (nw * g0).sum(0)
        gt = g0 - nw * ng
        tn = np.sqrt((gt ** 2).sum(0))
        that = gt / (tn + ph.eps)
        a_ = np.clip(2 * phi - 1, -1 + self.clamp_a, 1 - self.clamp_a)
        x_x0 = 0.5 * ph.W * np.arctanh(a_)
        for i in range(1, 19):
            if not sol[i].any():
                continue
            th = np.deg2rad(np.array(self.wl.theta_deg))[matn[i]]
            w = -np.cos(th) * nw + np.sin(th) * that
            d = w[0] * C[i][0] + w[1] * C[i][1] + w[2] * C[i][2]
            ps = 0.5 * (1 + np.tanh((x_x0 + d) / (0.5 * ph.W)))
            if getattr(ph, "hysteresis", False):
                if hist_mode == "set":
                    self.hist[i] = np.where(sol[i], ps, self.hist[i])
                else:
                    fresh = ps
                    ps = ph.hyst_beta * self.hist[i] + (1 - ph.hyst_beta) * fresh
                    if hist_mode == "step":
                        keep = fresh if int(ph.hysteresis) == 2 else ps
                        self.hist[i] = np.where(sol[i], keep, self.hist[i])
            nb[i] = np.where(sol[i], ps, nb[i])
        grad = np.zeros((3,) + self.shape)
        lap = np.zeros(self.shape)
        for i in range(1, 19):
            for a in range(3):
                grad[a] += WG[i] * C[i][a] * nb[i]
            lap += WG[i] * (nb[i] - phi)
        return grad / TG, 2 * lap / TG

    def _heq(self, phi, u, grad, lap):
        ph = self.ph
        gn = np.sqrt((grad ** 2).sum(0))
        nh = grad / (gn + ph.eps)
        QP, WP, TP = self._phase_lattice()
        theta = ph.M / TP * (1 - 4 * (phi - 0.5) ** 2) / ph.W
        if ph.mobility_corr:
            s = lap / (np.abs(lap) + ph.eps)
            Fc = lambda x: np.clip(x, 0.0, 1.0)
            Y1 = np.minimum(Fc((phi - ph.phi_M) / ph.D), Fc((1 - phi) / ph.D))
            Y2 = np.minimum(Fc(phi / ph.D), Fc((ph.phi_m - phi) / ph.D))
            theta = theta + ph.gamma * ph.M / (TP * ph.W) * gn * ((1 + s) * Y1 + (1 - s) * Y2)
        out = np.zeros((QP,) + self.shape)
        for i in range(QP):
            cn = C[i][0] * nh[0] + C[i][1] * nh[1] + C[i][2] * nh[2]
            out[i] = phi * self._Gamma(WP[i], C[i], u, TP) + theta * WP[i] * cn
        return out

    def _geq(self, phi, u, P, grad, lap):
        ph = self.ph
        rho = self._rho(phi)
        mu = self._mu(phi, lap)
        rdif = ph.rho_l - ph.rho_g
        geq = np.zeros((19,) + self.shape)
        K = np.zeros((19,) + self.shape)
        for i in range(19):
            G = self._Gamma(WG[i], C[i], u, TG)
            cg = sum((C[i][a] - u[a]) * grad[a] for a in range(3))
            cf = sum((C[i][a] - u[a]) * ph.F_ex[a] for a in range(3))
            K[i] = ((G - WG[i]) * rdif + G * mu / TG) * cg + G * cf / TG
            geq[i] = rho * G + WG[i] * (P / TG - rho) - 0.5 * K[i]
        return geq, K

    def _moments(self, phi, grad, lap):
        ph = self.ph
        rho = self._rho(phi)
        mu = self._mu(phi, lap)
        j = np.zeros((3,) + self.shape)
        for i in range(19):
            for a in range(3):
                j[a] += C[i][a] * self.g[i]
        u = np.stack([(j[a] + 0.5 * (mu * grad[a] + ph.F_ex[a])) / rho for a in range(3)])
        P = TG * self.g.sum(0) + 0.5 * TG * (ph.rho_l - ph.rho_g) * (u * grad).sum(0)
        return u, P

    def _ghost_pops(self, t):
        ph = self.ph
        phio = self._owner_value(self.phi)
        uo = np.stack([self._owner_value(self.u[a]) for a in range(3)])
        rho = self._rho(phio)
        Pb = np.zeros(self.shape)
        for f in range(6):
            if self.wl.faces[f] is None:
                continue
            P0, ramp = self.wl.faces[f]
            Pb = np.where(self.gface == f, P0 + ramp * t, Pb)
        QP, WP, TP = self._phase_lattice()
        h = np.stack([phio * self._Gamma(WP[i], C[i], uo, TP) for i in range(QP)])
        g = np.stack([rho * self._Gamma(WG[i], C[i], uo, TG) + WG[i] * (Pb / TG - rho)
                      for i in range(19)])
        return h * self.ghost, g * self.ghost

    # ---------------------------------------------------------------- step
    def step(self, n=1):
        for _ in range(n):
            self._one_step()

    def _one_step(self):
        ph = self.ph
        phi = np.where(self.fluid, self.h.sum(0), 0.0)
        phi = self._ghost_copy(phi)
        self.phi = phi
        grad, lap = self._stencil(phi, "step")
        u, P = self._moments(phi, grad, lap)
        u = u * self.fluid
        self.u = u
        geq, K = self._geq(phi, u, P, grad, lap)
        neq = self.g - geq
        Pi = np.zeros((3, 3) + self.shape)
        for i in range(19):
            for a in range(3):
                for b in range(3):
                    Pi[a, b] += C[i][a] * C[i][b] * neq[i]
        omega = 1 - 1 / self._tau(phi)
        gs = np.zeros_like(self.g)
        for i in range(19):
            contr = sum((C[i][a] * C[i][b] - (TG if a == b else 0.0)) * Pi[a, b]
                        for a in range(3) for b in range(3))
            gs[i] = geq[i] + K[i] + omega * WG[i] / (2 * TG * TG) * contr
        heq = self._heq(phi, u, grad, lap)
        QP, WP, TP = self._phase_lattice()
        tau_h = ph.M / TP + 0.5
        hs = self.h - (self.h - heq) / tau_h
        # ghosts hand over equilibria built from their owners' phi and u of this
        # step and the face pressure of the next step
        hg, gg = self._ghost_pops(self.t + 1)
        gs = np.where(self.fluid, gs, gg)
        hs = np.where(self.fluid, hs, hg)
        # slip velocity for the bounce-back inside the interface band
        rho = self._rho(phi)
        band = np.zeros(self.shape, bool)
        if ph.interface_slip:
            band = (phi >= ph.slip_lo) & (phi <= ph.slip_hi)
        un = (self.nw * u).sum(0)
        uw = getattr(ph, "slip_factor", 1.0) * (u - self.nw * un) * band
        hn = np.zeros_like(self.h)
        gn = np.zeros_like(self.g)
        for i in range(19):
            src_solid = shifted(self.solid, C[i], -1)
            io = OPP[i]
            cu = C[io][0] * uw[0] + C[io][1] * uw[1] + C[io][2] * uw[2]
            corr = 2 * WG[io] * rho * cu / TG
            if self.q is None:
                bb = gs[io] - corr
            else:
                # interpolated bounce-back with the wall at fraction q of the
                # link io; below 1/2 the upstream population is this step's
                # incoming g_io, or (same_step) the post-collision g_io one
                # node upstream, with the half-way value where that node is solid
                q = self.q[io]
                hi = gs[io] / (2 * q) + (1 - 1 / (2 * q)) * gs[i] - corr / (2 * q)
                if self.same_step:
                    up = shifted(gs[io], C[i], +1)
                    up_solid = shifted(self.solid, C[i], +1)
                    lo = np.where(up_solid, gs[io] - corr,
                                  2 * q * gs[io] + (1 - 2 * q) * up - corr)
                else:
                    lo = 2 * q * gs[io] + (1 - 2 * q) * self.g[io] - corr
                bb = np.where(q >= 0.5, hi, lo)
            gn[i] = np.where(src_solid, bb, shifted(gs[i], C[i], -1))
            if i < QP:
                hn[i] = np.where(src_solid, hs[io], shifted(hs[i], C[i], -1))
        hn *= self.fluid
        gn *= self.fluid
        self.t += 1
        self.h = hn
        self.g = gn

    # ------------------------------------------------------------- outputs
    def fields(self):
        phi = np.where(self.fluid, self.h.sum(0), 0.0)
        phi = self._ghost_copy(phi)
        self.phi = phi
        grad, lap = self._stencil(phi)
        u, P = self._moments(phi, grad, lap)
        u = u * self.fluid
        Pb = np.zeros(self.shape)
        for f in range(6):
            if self.wl.faces[f] is None:
                continue
            P0, ramp = self.wl.faces[f]
            Pb = np.where(self.gface == f, P0 + ramp * self.t, Pb)
        P = np.where(self.fluid, P, np.where(self.ghost, Pb, 0.0))
        phi = np.where(self.solid, 0.0, phi)
        return phi, P, u

    def pops(self):
        return self.h * self.fluid, self.g * self.fluid
