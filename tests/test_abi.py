"""The C-ABI library loads and exports every entry point include/lbm.h
declares; host-side validation works without a GPU (no compute calls)."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("lbm_create", "lbm_step", "lbm_read_fields", "lbm_submit", "lbm_footprint",
                 "lbm_reduce", "lbm_destroy", "lbm_poll"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2512_01032_amd import lbm
    L = ctypes.CDLL(lbm.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert set(lbm.EXPORTED) == set(declared_functions())


def test_struct_sizes_match_header():
    """Compile a tiny C program against include/lbm.h and compare the sizes
    and field offsets the ctypes mirror uses."""
    import subprocess
    import tempfile
    from paper_2512_01032_amd import lbm
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "lbm.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(lbm_params), sizeof(lbm_geometry),
         sizeof(lbm_init), sizeof(lbm_device_ctx), sizeof(lbm_diag), sizeof(lbm_info),
         sizeof(lbm_server_cfg), sizeof(lbm_request), sizeof(lbm_result));
  printf("%zu %zu %zu %zu %zu %zu %zu\n", offsetof(lbm_params, face_bc),
         offsetof(lbm_params, diag_every), offsetof(lbm_params, fp16_log2_scale_g),
         offsetof(lbm_params, hysteresis), offsetof(lbm_params, hyst_beta),
         offsetof(lbm_params, q_phase), offsetof(lbm_params, slip_factor));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        exe = os.path.join(d, "s")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split("\n")
    sizes = [int(v) for v in out[0].split()]
    mine = [ctypes.sizeof(t) for t in (lbm.lbm_params, lbm.lbm_geometry, lbm.lbm_init,
                                       lbm.lbm_device_ctx, lbm.lbm_diag, lbm.lbm_info,
                                       lbm.lbm_server_cfg, lbm.lbm_request, lbm.lbm_result)]
    assert sizes == mine
    offs = [int(v) for v in out[1].split()]
    assert offs == [lbm.lbm_params.face_bc.offset, lbm.lbm_params.diag_every.offset,
                    lbm.lbm_params.fp16_log2_scale_g.offset, lbm.lbm_params.hysteresis.offset,
                    lbm.lbm_params.hyst_beta.offset, lbm.lbm_params.q_phase.offset,
                    lbm.lbm_params.slip_factor.offset]


@pytest.mark.parametrize("field,value", [("nu_l", 0.0), ("W", -1.0), ("rho_g", 0.0), ("nx", 0),
                                         ("storage", 9), ("storage", 4), ("q_phase", 8),
                                         ("hysteresis", 3),
                                         ("hysteresis", -1), ("subvoxel", 2)])
def test_invalid_parameters_rejected_on_host(field, value):
    from paper_2512_01032_amd import inputs, lbm
    wl = inputs.random_small(8, 6, 5, seed=0)
    p = lbm.params_from_workload(wl)
    setattr(p, field, value)
    _create_is_rejected(wl, p)


@pytest.mark.parametrize("friction,beta", [(3, 0.5), (-1, 0.5), (2, 1.5), (2, -0.1), (2, float("nan"))])
def test_invalid_friction_rejected_on_host(friction, beta):
    """An unknown friction model, or a partial-slip factor outside [0, 1]."""
    from paper_2512_01032_amd import inputs, lbm
    wl = inputs.random_small(8, 6, 5, seed=0, optimised_model=True)
    p = lbm.params_from_workload(wl)
    p.friction, p.slip_factor = friction, beta
    _create_is_rejected(wl, p)


def _create_is_rejected(wl, p):
    from paper_2512_01032_amd import lbm
    assert lbm.lbm_footprint(ctypes.byref(p)) == 0
    with pytest.raises(lbm.LbmError) as ei:
        wl2 = wl
        g = lbm.lbm_geometry()
        for k in range(16):
            g.theta_deg[k] = 90.0
        init = lbm.lbm_init()
        phi = wl2.phi0.copy()
        init.phi = phi.ctypes.data
        h = ctypes.c_void_p()
        lbm.check(lbm.lbm_create(ctypes.byref(p), ctypes.byref(g), ctypes.byref(init), None,
                                 ctypes.byref(h)))
    assert ei.value.code == lbm.LBM_E_INVAL


def test_invalid_geometry_rejected_on_host():
    from paper_2512_01032_amd import inputs, lbm
    import numpy as np
    wl = inputs.random_small(8, 6, 5, seed=0)
    wl.theta_deg = (0.0,) + (90.0,) * 15                 # angle outside (0, 180)
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Lattice(wl)
    assert ei.value.code == lbm.LBM_E_INVAL
    wl = inputs.random_small(8, 6, 5, seed=0, open_x=True)
    wl.faces = (wl.faces[0], wl.faces[1], (0.3, 0.0), None, None, None)   # two pressure faces meet
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Lattice(wl)
    assert ei.value.code == lbm.LBM_E_INVAL
    wl = inputs.random_small(8, 6, 5, seed=0, open_x=True)
    s = np.zeros(wl.shape, np.uint8)
    s[:, :, 1] = 1                                      # ghost at x = 0 with a solid owner
    wl.solid = s
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Lattice(wl)
    assert ei.value.code == lbm.LBM_E_INVAL


def test_subvoxel_geometry_rejected_on_host():
    """subvoxel = 1 needs a signed distance, a distance needs subvoxel = 1,
    and a distance that does not straddle a wall link is rejected."""
    from paper_2512_01032_amd import inputs, lbm
    wl = inputs.offset_plates(12, 0.3, nx=8, nz=4)
    sdf = wl.sdf
    wl.sdf = None
    p = lbm.params_from_workload(wl)
    p.subvoxel = 1
    g = lbm.lbm_geometry()
    for k in range(16):
        g.theta_deg[k] = 90.0
    solid = np.ascontiguousarray(wl.solid, np.uint8)
    g.solid = solid.ctypes.data
    init = lbm.lbm_init()
    phi = np.ascontiguousarray(wl.phi0)
    init.phi = phi.ctypes.data
    h = ctypes.c_void_p()
    for bad_sdf, sv in ((None, 1), (sdf, 0)):
        p.subvoxel = sv
        keep = None if bad_sdf is None else np.ascontiguousarray(bad_sdf)
        g.sdf = None if keep is None else keep.ctypes.data
        with pytest.raises(lbm.LbmError) as ei:
            lbm.check(lbm.lbm_create(ctypes.byref(p), ctypes.byref(g), ctypes.byref(init), None,
                                     ctypes.byref(h)))
        assert ei.value.code == lbm.LBM_E_INVAL
    wl.sdf = sdf.copy()
    wl.sdf[0, 1, 0] = -0.1      # a fluid node next to the wall with a negative distance
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Lattice(wl)
    assert ei.value.code == lbm.LBM_E_INVAL
    assert b"straddle" in lbm.lbm_last_error()


def test_footprint_counts_populations():
    from paper_2512_01032_amd import inputs, lbm
    wl = inputs.random_small(64, 16, 16, seed=0)
    n = 64 * 16 * 16
    f32 = lbm.footprint(wl, "fp32_shift")
    f16 = lbm.footprint(wl, "fp16_shift_g")
    f64 = lbm.footprint(wl, "fp64")
    assert f32 >= n * (26 * 4 + 4 + 1 + 4)
    assert f64 >= n * (26 * 8 + 8 + 1 + 4)
    assert f16 >= n * (7 * 4 + 19 * 2 + 4 + 1 + 4)
    assert f16 < f32 < f64
    # the D3Q19 phase lattice stores 12 more h arrays
    import dataclasses
    wl.phys = dataclasses.replace(wl.phys, q_phase=19)
    assert lbm.footprint(wl, "fp32_shift") - f32 >= n * 12 * 4


def test_population_layout_limits():
    """Populations sit in 64-node blocks with rows padded to 64 nodes, in one
    buffer group while a node's populations take at most 104 bytes, else in
    two; each group is addressed with 32-bit offsets, so a lattice whose
    group exceeds 4 GiB is rejected (lbm_footprint returns 0)."""
    from paper_2512_01032_amd import inputs, lbm
    wl = inputs.random_small(8, 6, 5, seed=0)
    p = lbm.params_from_workload(wl)

    def fp(nx, ny, nz, storage):
        p.nx, p.ny, p.nz = nx, ny, nz
        p.storage = lbm.STORAGE[storage]
        return lbm.lbm_footprint(ctypes.byref(p))

    # a 40-wide row stores 64 nodes of populations
    assert fp(40, 16, 16, "fp32_shift") >= 64 * 16 * 16 * 104
    # FP32 on D3Q7: 104 bytes per node in one group, 2^32 / 104 nodes at most
    assert fp(256, 256, 630, "fp32_shift") > 0
    assert fp(256, 256, 631, "fp32_shift") == 0
    # FP64: two groups of 104 bytes per node, the same node limit
    assert fp(256, 256, 630, "fp64") > 0
    assert fp(256, 256, 631, "fp64") == 0
    # FP16 g: 66 bytes per node in one group
    assert fp(256, 256, 992, "fp16_shift_g") > 0
    assert fp(256, 256, 993, "fp16_shift_g") == 0


def test_fp16_phase_storage_rejected_on_host():
    """Storage with the phase-field populations in FP16 (LBM_FP16_SHIFT_ALL)
    has no bounded phi error and is refused by lbm_create, lbm_footprint and
    the server, before any device call."""
    from paper_2512_01032_amd import inputs, lbm
    wl = inputs.random_small(8, 6, 5, seed=0)
    assert lbm.footprint(wl, "fp16_shift_all") == 0
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Lattice(wl, storage="fp16_shift_all")
    assert ei.value.code == lbm.LBM_E_INVAL
    assert b"FP16_SHIFT_ALL" in lbm.lbm_last_error()
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Server(storage="fp16_shift_all")
    assert ei.value.code == lbm.LBM_E_INVAL


def test_lattice_without_fluid_rejected_on_host():
    """A geometry with no fluid node (every node solid) is refused by
    lbm_create with LBM_E_INVAL before any device call."""
    from paper_2512_01032_amd import inputs, lbm
    wl = inputs.random_small(8, 6, 5, seed=0)
    wl.solid = np.ones((wl.nz, wl.ny, wl.nx), np.uint8)
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Lattice(wl, storage="fp64")
    assert ei.value.code == lbm.LBM_E_INVAL
    assert b"no fluid node" in lbm.lbm_last_error()
