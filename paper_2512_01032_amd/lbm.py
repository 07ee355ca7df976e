"""Python binding of the C ABI in include/lbm.h (ctypes; argument marshalling only).

The functions keep the C names (lbm_create, lbm_step, lbm_read_fields, ...);
`Lattice` and `Server` wrap them for numpy arrays.  Every step of the method
runs in the HIP kernels of liblbm.so; when the library is missing the import
of this module fails loudly -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblbm.so")

LBM_OK, LBM_PENDING = 0, 1
LBM_E_INVAL, LBM_E_NOMEM, LBM_E_DEVICE, LBM_E_UNSTABLE, LBM_E_STATE = -1, -2, -3, -4, -5
NOALLOC_MAX_DOUBLES = 8 << 20   # LBM_NOALLOC_MAX_DOUBLES
STORAGE = {"fp64": 0, "fp32": 1, "fp32_shift": 2, "fp16_shift_g": 3, "fp16_shift_all": 4}
LBM_PHI, LBM_P, LBM_U, LBM_POP_H, LBM_POP_G = 1, 2, 4, 8, 16
LBM_INIT_FIELDS, LBM_INIT_POPULATIONS = 0, 1

EXPORTED = ("lbm_footprint", "lbm_create", "lbm_step", "lbm_sync", "lbm_step_count",
            "lbm_read_fields", "lbm_read_fields_noalloc", "lbm_reduce", "lbm_set_timing", "lbm_get_timing", "lbm_destroy",
            "lbm_last_error", "lbm_get_info", "lbm_server_create", "lbm_submit", "lbm_poll",
            "lbm_server_drain", "lbm_server_clock", "lbm_result_free", "lbm_server_destroy")

c_int32, c_int64, c_double, c_size_t = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("storage", c_int32),
        ("rho_l", c_double), ("rho_g", c_double), ("nu_l", c_double), ("nu_g", c_double),
        ("sigma", c_double), ("W", c_double), ("M", c_double), ("F_ex", c_double * 3),
        ("mobility_corr", c_int32), ("mc_gamma", c_double), ("mc_phi_M", c_double),
        ("mc_phi_m", c_double), ("mc_D", c_double), ("eps", c_double),
        ("mix", c_int32), ("mix_phi", c_double), ("mix_width", c_double),
        ("friction", c_int32), ("slip_lo", c_double), ("slip_hi", c_double),
        ("P_ref", c_double),
        ("face_bc", c_int32 * 6), ("face_P", c_double * 6), ("face_ramp", c_double * 6),
        ("diag_every", c_int32), ("u_max", c_double),
        ("fp16_log2_scale_h", c_int32), ("fp16_log2_scale_g", c_int32),
        ("hysteresis", c_int32), ("hyst_beta", c_double), ("q_phase", c_int32),
        ("subvoxel", c_int32), ("slip_factor", c_double),
    ]


class lbm_geometry(ctypes.Structure):
    _fields_ = [("solid", ctypes.c_void_p), ("theta_deg", c_double * 16), ("sdf", ctypes.c_void_p)]


class lbm_init(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("phi", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("P", ctypes.c_void_p), ("pops", ctypes.c_void_p), ("step", c_int64)]


class lbm_device_ctx(ctypes.Structure):
    _fields_ = [("arena", ctypes.c_void_p), ("arena_bytes", c_size_t), ("stream", ctypes.c_void_p),
                ("device", c_int32)]


class lbm_diag(ctypes.Structure):
    _fields_ = [("step", c_int64), ("phi_sum", c_double), ("mom", c_double * 3),
                ("u_max", c_double), ("P_liq_mean", c_double), ("P_gas_mean", c_double),
                ("n_nan", c_int64), ("n_liq", c_int64), ("n_gas", c_int64)]


class lbm_info(ctypes.Structure):
    _fields_ = [("n_nodes", c_int64), ("n_fluid", c_int64), ("n_ghost", c_int64),
                ("n_solid", c_int64), ("n_tiles", c_int64), ("footprint", c_size_t),
                ("bytes_per_fluid_update", c_double)]


class lbm_server_cfg(ctypes.Structure):
    _fields_ = [("hbm_budget", c_size_t), ("max_slots", c_int32), ("storage", c_int32),
                ("device", c_int32), ("use_graph", c_int32), ("ticks_per_sync", c_int32),
                ("max_resident_nodes", c_int64)]


class lbm_request(ctypes.Structure):
    _fields_ = [("params", lbm_params), ("geometry", lbm_geometry), ("init", lbm_init),
                ("nsteps", c_int64), ("arrival_s", c_double)]


class lbm_result(ctypes.Structure):
    _fields_ = [("status", c_int32), ("nx", c_int64), ("ny", c_int64), ("nz", c_int64),
                ("phi", ctypes.POINTER(c_double)), ("P", ctypes.POINTER(c_double)),
                ("u", ctypes.POINTER(c_double)), ("diag", lbm_diag),
                ("t_submit_s", c_double), ("t_admit_s", c_double), ("t_finish_s", c_double),
                ("steps", c_int64)]


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("lbm error %d: %s" % (code, msg))
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("liblbm.so is not built (run __graft_entry__.build() or "
                          "python -m paper_2512_01032_amd.build); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    L.lbm_footprint.restype = c_size_t
    L.lbm_footprint.argtypes = [ctypes.POINTER(lbm_params)]
    L.lbm_create.argtypes = [ctypes.POINTER(lbm_params), ctypes.POINTER(lbm_geometry),
                             ctypes.POINTER(lbm_init), ctypes.POINTER(lbm_device_ctx),
                             ctypes.POINTER(vp)]
    L.lbm_step.argtypes = [vp, c_int64]
    L.lbm_sync.argtypes = [vp]
    L.lbm_step_count.restype = c_int64
    L.lbm_step_count.argtypes = [vp]
    L.lbm_read_fields.argtypes = [vp, ctypes.c_uint32, vp, vp, vp, vp]
    L.lbm_read_fields_noalloc.argtypes = [vp, ctypes.c_uint32, vp, vp, vp, vp]
    L.lbm_reduce.argtypes = [vp, ctypes.POINTER(lbm_diag)]
    L.lbm_set_timing.argtypes = [vp, c_int32]
    L.lbm_get_timing.argtypes = [vp, ctypes.POINTER(c_double), ctypes.POINTER(c_double),
                                 ctypes.POINTER(c_int64)]
    L.lbm_destroy.argtypes = [vp]
    L.lbm_last_error.restype = ctypes.c_char_p
    L.lbm_get_info.argtypes = [vp, ctypes.POINTER(lbm_info)]
    L.lbm_server_create.argtypes = [ctypes.POINTER(lbm_server_cfg), ctypes.POINTER(vp)]
    L.lbm_submit.argtypes = [vp, ctypes.POINTER(lbm_request), ctypes.POINTER(ctypes.c_uint64)]
    L.lbm_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(lbm_result)]
    L.lbm_server_drain.argtypes = [vp]
    L.lbm_server_clock.restype = c_double
    L.lbm_server_clock.argtypes = [vp]
    L.lbm_result_free.argtypes = [ctypes.POINTER(lbm_result)]
    L.lbm_server_destroy.argtypes = [vp]
    return L


_L = _load()

# the C entry points under their own names
lbm_footprint = _L.lbm_footprint
lbm_create = _L.lbm_create
lbm_step = _L.lbm_step
lbm_sync = _L.lbm_sync
lbm_step_count = _L.lbm_step_count
lbm_read_fields = _L.lbm_read_fields
lbm_read_fields_noalloc = _L.lbm_read_fields_noalloc
lbm_reduce = _L.lbm_reduce
lbm_set_timing = _L.lbm_set_timing
lbm_get_timing = _L.lbm_get_timing
lbm_destroy = _L.lbm_destroy
lbm_last_error = _L.lbm_last_error
lbm_get_info = _L.lbm_get_info
lbm_server_create = _L.lbm_server_create
lbm_submit = _L.lbm_submit
lbm_poll = _L.lbm_poll
lbm_server_drain = _L.lbm_server_drain
lbm_server_clock = _L.lbm_server_clock
lbm_result_free = _L.lbm_result_free
lbm_server_destroy = _L.lbm_server_destroy


def check(rc):
    if rc < 0:
        raise LbmError(rc, (_L.lbm_last_error() or b"").decode())
    return rc


# ------------------------------------------------------------------ marshalling
def params_from_workload(wl, storage=None, diag_every=0, u_max=0.0):
    """lbm_params from an inputs.Workload (plain field copies)."""
    ph = wl.phys
    p = lbm_params()
    p.nx, p.ny, p.nz = wl.nx, wl.ny, wl.nz
    p.storage = STORAGE[storage or wl.storage]
    p.rho_l, p.rho_g, p.nu_l, p.nu_g = ph.rho_l, ph.rho_g, ph.nu_l, ph.nu_g
    p.sigma, p.W, p.M = ph.sigma, ph.W, ph.M
    for a in range(3):
        p.F_ex[a] = ph.F_ex[a]
    p.mobility_corr = int(ph.mobility_corr)
    p.mc_gamma, p.mc_phi_M, p.mc_phi_m, p.mc_D = ph.gamma, ph.phi_M, ph.phi_m, ph.D
    p.eps = ph.eps
    p.mix = 1 if ph.mix_tanh else 0
    p.mix_phi, p.mix_width = ph.mix_phi, ph.mix_width
    beta = float(getattr(ph, "slip_factor", 1.0))
    p.friction = 0 if not ph.interface_slip else (1 if beta == 1.0 else 2)
    p.slip_lo, p.slip_hi = ph.slip_lo, ph.slip_hi
    p.slip_factor = beta
    p.P_ref = ph.P_ref
    for f in range(6):
        fc = wl.faces[f]
        p.face_bc[f] = 0 if fc is None else 1
        p.face_P[f] = 0.0 if fc is None else fc[0]
        p.face_ramp[f] = 0.0 if fc is None else fc[1]
    p.diag_every = int(diag_every)
    p.u_max = float(u_max)
    p.hysteresis = int(getattr(ph, "hysteresis", 0))
    p.hyst_beta = float(getattr(ph, "hyst_beta", 0.0))
    p.q_phase = int(getattr(ph, "q_phase", 7))
    p.subvoxel = 0 if getattr(wl, "sdf", None) is None else 1
    return p


def _arr(a, dtype=np.float64):
    if a is None:
        return None
    return np.ascontiguousarray(a, dtype=dtype)


class Lattice:
    """One lattice on the GPU through the C ABI."""

    def __init__(self, wl, storage=None, diag_every=0, u_max=0.0, stream=None, arena=None,
                 device=0, pops=None, step=0):
        self.wl = wl
        self.shape = wl.shape
        self.N = wl.n_nodes
        self.params = params_from_workload(wl, storage, diag_every, u_max)
        geo = lbm_geometry()
        self._solid = _arr(wl.solid, np.uint8)
        geo.solid = None if self._solid is None else self._solid.ctypes.data
        self._sdf = _arr(getattr(wl, "sdf", None))
        geo.sdf = None if self._sdf is None else self._sdf.ctypes.data
        for k in range(16):
            geo.theta_deg[k] = wl.theta_deg[k]
        init = lbm_init()
        self._keep = []
        if pops is None:
            phi0, u0, P0 = _arr(wl.phi0), _arr(wl.u0), _arr(wl.P0)
            self._keep += [phi0, u0, P0]
            init.kind = LBM_INIT_FIELDS
            init.phi = phi0.ctypes.data
            init.u = None if u0 is None else u0.ctypes.data
            init.P = None if P0 is None else P0.ctypes.data
        else:
            pp = _arr(pops)
            self._keep.append(pp)
            init.kind = LBM_INIT_POPULATIONS
            init.pops = pp.ctypes.data
            init.step = int(step)
        ctx = lbm_device_ctx()
        ctx.device = device
        ctx.stream = stream
        if arena is not None:
            ctx.arena, ctx.arena_bytes = arena
        h = ctypes.c_void_p()
        check(lbm_create(ctypes.byref(self.params), ctypes.byref(geo), ctypes.byref(init),
                         ctypes.byref(ctx), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def step(self, n=1):
        check(lbm_step(self.h, int(n)))

    def sync(self):
        check(lbm_sync(self.h))

    @property
    def t(self):
        return lbm_step_count(self.h)

    def fields(self):
        phi = np.zeros(self.shape)
        P = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        check(lbm_read_fields(self.h, LBM_PHI | LBM_P | LBM_U, phi.ctypes.data, P.ctypes.data,
                              u.ctypes.data, None))
        return phi, P, u

    def read(self, mask, noalloc=False):
        """lbm_read_fields (or lbm_read_fields_noalloc) of the fields in mask:
        a dict of the arrays asked for."""
        qh = self.params.q_phase if self.params.q_phase else 7
        out = {}
        phi = np.zeros(self.shape) if mask & LBM_PHI else None
        P = np.zeros(self.shape) if mask & LBM_P else None
        u = np.zeros((3,) + self.shape) if mask & LBM_U else None
        nq = (qh if mask & LBM_POP_H else 0) + (19 if mask & LBM_POP_G else 0)
        pops = np.zeros((nq,) + self.shape) if nq else None
        fn = lbm_read_fields_noalloc if noalloc else lbm_read_fields
        check(fn(self.h, mask, None if phi is None else phi.ctypes.data,
                 None if P is None else P.ctypes.data, None if u is None else u.ctypes.data,
                 None if pops is None else pops.ctypes.data))
        for k, v in (("phi", phi), ("P", P), ("u", u), ("pops", pops)):
            if v is not None:
                out[k] = v
        return out

    def pops(self):
        qh = self.params.q_phase if self.params.q_phase else 7
        buf = np.zeros((qh + 19,) + self.shape)
        check(lbm_read_fields(self.h, LBM_POP_H | LBM_POP_G, None, None, None, buf.ctypes.data))
        return buf[:qh], buf[qh:]

    def diagnostics(self):
        d = lbm_diag()
        check(lbm_reduce(self.h, ctypes.byref(d)))
        return {"step": d.step, "phi_sum": d.phi_sum, "mom": tuple(d.mom), "u_max": d.u_max,
                "P_liq_mean": d.P_liq_mean, "P_gas_mean": d.P_gas_mean, "n_nan": d.n_nan,
                "n_liq": d.n_liq, "n_gas": d.n_gas}

    def info(self):
        i = lbm_info()
        check(lbm_get_info(self.h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in lbm_info._fields_}

    def set_timing(self, on=True):
        check(lbm_set_timing(self.h, int(on)))

    def get_timing(self):
        a, b, n = c_double(), c_double(), c_int64()
        check(lbm_get_timing(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(n)))
        return a.value, b.value, n.value


def footprint(wl, storage=None):
    p = params_from_workload(wl, storage)
    return int(lbm_footprint(ctypes.byref(p)))


class Server:
    """Continuous-batching server through the C ABI (lbm_server_*)."""

    def __init__(self, storage="fp32_shift", hbm_budget=0, max_slots=0, use_graph=True,
                 ticks_per_sync=32, device=0, max_resident_nodes=0):
        cfg = lbm_server_cfg()
        cfg.hbm_budget = int(hbm_budget)
        cfg.max_slots = int(max_slots)
        cfg.storage = STORAGE[storage]
        cfg.device = int(device)
        cfg.use_graph = int(bool(use_graph))
        cfg.ticks_per_sync = int(ticks_per_sync)
        cfg.max_resident_nodes = int(max_resident_nodes)
        h = ctypes.c_void_p()
        check(lbm_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lbm_server_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def submit(self, wl, nsteps, arrival_s=0.0):
        """Queue a workload for nsteps steps; the arrays are copied during the call."""
        req = lbm_request()
        req.params = params_from_workload(wl)
        solid = _arr(wl.solid, np.uint8)
        phi0, u0, P0 = _arr(wl.phi0), _arr(wl.u0), _arr(wl.P0)
        req.geometry.solid = None if solid is None else solid.ctypes.data
        sdf = _arr(getattr(wl, "sdf", None))
        req.geometry.sdf = None if sdf is None else sdf.ctypes.data
        for k in range(16):
            req.geometry.theta_deg[k] = wl.theta_deg[k]
        req.init.kind = LBM_INIT_FIELDS
        req.init.phi = phi0.ctypes.data
        req.init.u = None if u0 is None else u0.ctypes.data
        req.init.P = None if P0 is None else P0.ctypes.data
        req.nsteps = int(nsteps)
        req.arrival_s = float(arrival_s)
        t = ctypes.c_uint64()
        check(lbm_submit(self.h, ctypes.byref(req), ctypes.byref(t)))
        return t.value

    def poll(self, ticket):
        """None while pending, else a dict with the request's status, fields,
        diagnostics and server-clock timestamps."""
        r = lbm_result()
        rc = check(lbm_poll(self.h, ctypes.c_uint64(ticket), ctypes.byref(r)))
        if rc == LBM_PENDING:
            return None
        try:
            shape = (r.nz, r.ny, r.nx)
            n = r.nx * r.ny * r.nz
            out = {"status": r.status, "steps": r.steps, "t_submit": r.t_submit_s,
                   "t_admit": r.t_admit_s, "t_finish": r.t_finish_s}
            if r.status == LBM_OK:
                out["phi"] = np.ctypeslib.as_array(r.phi, (n,)).reshape(shape).copy()
                out["P"] = np.ctypeslib.as_array(r.P, (n,)).reshape(shape).copy()
                out["u"] = np.ctypeslib.as_array(r.u, (3 * n,)).reshape((3,) + shape).copy()
                d = r.diag
                out["diag"] = {"step": d.step, "phi_sum": d.phi_sum, "mom": tuple(d.mom),
                               "u_max": d.u_max, "P_liq_mean": d.P_liq_mean,
                               "P_gas_mean": d.P_gas_mean, "n_nan": d.n_nan}
            return out
        finally:
            lbm_result_free(ctypes.byref(r))

    def drain(self):
        check(lbm_server_drain(self.h))

    def clock(self):
        return lbm_server_clock(self.h)
