"""ctypes wrapper of the FP64 CPU oracle (liblbmref.so).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it; the product package never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbmref.so")
SRC = os.path.join(HERE, "lbmref.c")

FACE_NAMES = ("x-", "x+", "y-", "y+", "z-", "z+")


def build(force=False):
    """Compile the oracle with gcc (plain C99 + OpenMP)."""
    if not force and os.path.exists(LIB_PATH) and \
            os.path.getmtime(LIB_PATH) >= os.path.getmtime(SRC):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
           "-ffp-contract=off", "-Wall", "-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("rho_l", ctypes.c_double), ("rho_g", ctypes.c_double),
        ("nu_l", ctypes.c_double), ("nu_g", ctypes.c_double),
        ("sigma", ctypes.c_double), ("W", ctypes.c_double), ("M", ctypes.c_double),
        ("F_ex", ctypes.c_double * 3),
        ("mobility_corr", ctypes.c_int),
        ("gamma", ctypes.c_double), ("phi_M", ctypes.c_double), ("phi_m", ctypes.c_double),
        ("D", ctypes.c_double), ("eps", ctypes.c_double),
        ("mix_tanh", ctypes.c_int), ("mix_phi", ctypes.c_double), ("mix_width", ctypes.c_double),
        ("interface_slip", ctypes.c_int), ("slip_lo", ctypes.c_double),
        ("slip_hi", ctypes.c_double),
        ("P_ref", ctypes.c_double),
        ("face_pressure", ctypes.c_int * 6), ("face_P", ctypes.c_double * 6),
        ("face_ramp", ctypes.c_double * 6),
        ("theta_deg", ctypes.c_double * 16),
        ("clamp_a", ctypes.c_double),
        ("hysteresis", ctypes.c_int), ("hyst_beta", ctypes.c_double),
        ("q_phase", ctypes.c_int),
        ("subvoxel_same_step", ctypes.c_int),
        ("slip_factor", ctypes.c_double),
    ]


class Diag(ctypes.Structure):
    _fields_ = [
        ("phi_sum", ctypes.c_double), ("mom", ctypes.c_double * 3), ("u_max", ctypes.c_double),
        ("P_liq_mean", ctypes.c_double), ("P_gas_mean", ctypes.c_double),
        ("n_nan", ctypes.c_long), ("n_liq", ctypes.c_long), ("n_gas", ctypes.c_long),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        L.lbmref_create.restype = ctypes.c_void_p
        L.lbmref_create.argtypes = [ctypes.POINTER(Params), ctypes.c_void_p, dp, dp, dp, dp]
        L.lbmref_destroy.argtypes = [ctypes.c_void_p]
        L.lbmref_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
        L.lbmref_step_count.argtypes = [ctypes.c_void_p]
        L.lbmref_step_count.restype = ctypes.c_long
        L.lbmref_kinds.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.lbmref_fields.argtypes = [ctypes.c_void_p, dp, dp, dp]
        L.lbmref_pops.argtypes = [ctypes.c_void_p, dp, dp]
        L.lbmref_set_pops.argtypes = [ctypes.c_void_p, dp, dp, ctypes.c_long]
        L.lbmref_diagnostics.argtypes = [ctypes.c_void_p, ctypes.POINTER(Diag)]
        L.lbmref_wet_phi_s.restype = ctypes.c_double
        L.lbmref_wet_phi_s.argtypes = [ctypes.c_double, dp, ctypes.POINTER(ctypes.c_int),
                                       ctypes.c_double, ctypes.c_double]
        L.lbmref_wet_direction.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, dp]
        L.lbmref_dtheta.restype = ctypes.c_double
        L.lbmref_dtheta.argtypes = [ctypes.POINTER(Params), ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double]
        L.lbmref_collide_g_node.argtypes = [ctypes.POINTER(Params), dp, ctypes.c_double, dp,
                                            ctypes.c_double, dp, dp, dp]
        L.lbmref_geq_node.argtypes = [ctypes.POINTER(Params), ctypes.c_double, dp,
                                      ctypes.c_double, dp, ctypes.c_double, dp, dp]
        _lib = L
    return _lib


def _dptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(wl, clamp_a=1e-12):
    ph = wl.phys
    p = Params()
    p.nx, p.ny, p.nz = wl.nx, wl.ny, wl.nz
    p.rho_l, p.rho_g, p.nu_l, p.nu_g = ph.rho_l, ph.rho_g, ph.nu_l, ph.nu_g
    p.sigma, p.W, p.M = ph.sigma, ph.W, ph.M
    for a in range(3):
        p.F_ex[a] = ph.F_ex[a]
    p.mobility_corr = int(ph.mobility_corr)
    p.gamma, p.phi_M, p.phi_m, p.D, p.eps = ph.gamma, ph.phi_M, ph.phi_m, ph.D, ph.eps
    p.mix_tanh, p.mix_phi, p.mix_width = int(ph.mix_tanh), ph.mix_phi, ph.mix_width
    p.interface_slip, p.slip_lo, p.slip_hi = int(ph.interface_slip), ph.slip_lo, ph.slip_hi
    p.P_ref = ph.P_ref
    for f in range(6):
        fc = wl.faces[f]
        p.face_pressure[f] = 0 if fc is None else 1
        p.face_P[f] = 0.0 if fc is None else fc[0]
        p.face_ramp[f] = 0.0 if fc is None else fc[1]
    for k in range(16):
        p.theta_deg[k] = wl.theta_deg[k]
    p.clamp_a = clamp_a
    p.hysteresis = int(getattr(ph, "hysteresis", False))
    p.hyst_beta = getattr(ph, "hyst_beta", 0.0)
    p.q_phase = int(getattr(ph, "q_phase", 7))
    p.subvoxel_same_step = int(getattr(wl, "meta", {}).get("subvoxel_same_step", False))
    p.slip_factor = getattr(ph, "slip_factor", 1.0)
    return p


class Oracle:
    """One lattice on the CPU oracle."""

    def __init__(self, wl, clamp_a=1e-12):
        L = lib()
        self.wl = wl
        self.shape = wl.shape
        self.N = wl.n_nodes
        self.params = make_params(wl, clamp_a)
        self._keep = []
        phi0 = np.ascontiguousarray(wl.phi0, dtype=np.float64)
        u0 = None if wl.u0 is None else np.ascontiguousarray(wl.u0, dtype=np.float64)
        P0 = None if wl.P0 is None else np.ascontiguousarray(wl.P0, dtype=np.float64)
        solid = None if wl.solid is None else np.ascontiguousarray(wl.solid, dtype=np.uint8)
        sdf = getattr(wl, "sdf", None)
        sdf = None if sdf is None else np.ascontiguousarray(sdf, dtype=np.float64)
        self._keep = [phi0, u0, P0, solid, sdf]
        h = L.lbmref_create(ctypes.byref(self.params),
                            None if solid is None else solid.ctypes.data,
                            _dptr(sdf), _dptr(phi0), _dptr(u0), _dptr(P0))
        if not h:
            raise ValueError("oracle rejected the workload %s" % wl.name)
        self.h = ctypes.c_void_p(h)

    def __del__(self):
        if getattr(self, "h", None):
            lib().lbmref_destroy(self.h)
            self.h = None

    def step(self, n=1):
        lib().lbmref_step(self.h, int(n))

    @property
    def t(self):
        return lib().lbmref_step_count(self.h)

    def kinds(self):
        k = np.zeros(self.shape, np.uint8)
        lib().lbmref_kinds(self.h, k.ctypes.data)
        return k

    def fields(self):
        phi = np.zeros(self.shape)
        P = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        lib().lbmref_fields(self.h, _dptr(phi), _dptr(P), _dptr(u))
        return phi, P, u

    def pops(self):
        h = np.zeros((int(getattr(self.wl.phys, "q_phase", 7)),) + self.shape)
        g = np.zeros((19,) + self.shape)
        lib().lbmref_pops(self.h, _dptr(h), _dptr(g))
        return h, g

    def set_pops(self, h, g, step):
        h = np.ascontiguousarray(h, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        lib().lbmref_set_pops(self.h, _dptr(h), _dptr(g), int(step))

    def diagnostics(self):
        d = Diag()
        lib().lbmref_diagnostics(self.h, ctypes.byref(d))
        return {"phi_sum": d.phi_sum, "mom": tuple(d.mom), "u_max": d.u_max,
                "P_liq_mean": d.P_liq_mean, "P_gas_mean": d.P_gas_mean,
                "n_nan": d.n_nan, "n_liq": d.n_liq, "n_gas": d.n_gas}


# ---------------------------------------------------------- single-node helpers
def wet_phi_s(phi_smpl, w, c, W, clamp_a=1e-12):
    w = np.ascontiguousarray(w, dtype=np.float64)
    ci = (ctypes.c_int * 3)(*[int(v) for v in c])
    return lib().lbmref_wet_phi_s(float(phi_smpl), _dptr(w), ci, float(W), float(clamp_a))


def wet_direction(n_w, g0, theta_deg, eps=1e-10):
    n_w = np.ascontiguousarray(n_w, dtype=np.float64)
    g0 = np.ascontiguousarray(g0, dtype=np.float64)
    w = np.zeros(3)
    lib().lbmref_wet_direction(_dptr(n_w), _dptr(g0), float(theta_deg), float(eps), _dptr(w))
    return w


def dtheta(wl, phi, grad_norm, lap):
    p = make_params(wl)
    return lib().lbmref_dtheta(ctypes.byref(p), float(phi), float(grad_norm), float(lap))


def collide_g_node(wl, g_in, phi, grad, lap):
    p = make_params(wl)
    g_in = np.ascontiguousarray(g_in, dtype=np.float64)
    grad = np.ascontiguousarray(grad, dtype=np.float64)
    out = np.zeros(19)
    u = np.zeros(3)
    P = ctypes.c_double()
    lib().lbmref_collide_g_node(ctypes.byref(p), _dptr(g_in), float(phi), _dptr(grad),
                                float(lap), _dptr(out), _dptr(u), ctypes.byref(P))
    return out, u, P.value


def geq_node(wl, phi, u, P, grad, lap):
    p = make_params(wl)
    u = np.ascontiguousarray(u, dtype=np.float64)
    grad = np.ascontiguousarray(grad, dtype=np.float64)
    geq = np.zeros(19)
    K = np.zeros(19)
    lib().lbmref_geq_node(ctypes.byref(p), float(phi), _dptr(u), float(P), _dptr(grad),
                          float(lap), _dptr(geq), _dptr(K))
    return geq, K
