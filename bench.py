"""Throughput of the fused phase-field LB step on one MI355X.

Workload: the constricted duct, 256 x 256 x 512 nodes (square duct along z,
step constriction to half width at z = 256, contact angle 120 deg, density
ratio 1000, viscosity ratio 100, seeded liquid slugs, inlet pressure ramp),
synthetic inputs from paper_2512_01032_amd.inputs.constricted_duct().

One step = the phi pass + the fused stream-collide sweep over every node.
`value` is million fluid-node updates per second (MLUPS) with the lattice
resident in HBM, FP32 shifted-population storage; FP16-stored populations
(g in FP16, h in FP32) and the plain FP64 / FP32 storage are reported beside
it, each with max |phi - oracle| after a short run.  The roofline object is
for the sweep kernel (the dominant one): algorithmic bytes = 2 (7 s_h +
19 s_g) per fluid node (every population read once and written once) over
the sweep's average duration measured with HIP events on its stream.  The
CPU baseline is the FP64 oracle on the host cores, on a bounded sample: the
same lattice for a few steps, median of three, on all cores and on one.
The oracle legs (skipped with --no-cpu-baseline) also run the configured
validation workloads at full size and length on the GPU: the sessile droplet
(128 x 128 x 96, 20k steps: contact angle, Laplace pressure), the capillary
filling (1024 x 32 x 32, 50k steps: meniscus position against Washburn) and
the duct itself for 10k steps (max |u|), each against the oracle where its
CPU time allows.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MLUPS + % HBM roofline, FP32 vs FP16-store at stated error; p99 solve latency"
SOURCES = ["paper_2512_01032_amd/csrc/kernels_impl.hpp", "paper_2512_01032_amd/csrc/pflbm.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_traffic_constricted_duct.json")


def kernel_hash():
    """Hash of the kernel sources with comments and blank space removed, so
    that the counter record stays tied to the code, not to its comments."""
    import re
    h = hashlib.sha256()
    for s in SOURCES:
        src = open(os.path.join(ROOT, s)).read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(storage):
    """HBM bytes per sweep launch from the committed rocprofv3 counter runs,
    if they were taken on the current kernel source."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_sweep", {}).get(storage)


def copy_calibration(mib, torch):
    """A plain streaming kernel of known traffic (elementwise negation: reads
    and writes mib MiB), run a few times; its counter readings calibrate
    FETCH_SIZE / WRITE_SIZE against bytes actually moved."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    print("[bench] copy calibration: %d MiB x 3" % mib, file=sys.stderr, flush=True)
    del a, b


_TYPES = {"float": "f32", "f": "f32", "double": "f64", "d": "f64", "_Float16": "f16", "DF16_": "f16"}
_STORAGE = {("f32", "f32", "f32"): "fp32_shift", ("f32", "f32", "f16"): "fp16_shift_g",
            ("f64", "f64", "f64"): "fp64"}


def _sweep_storage(name):
    """Storage mode of a MODE_STEP sweep dispatch from its kernel name
    (demangled or mangled), else None."""
    import re
    m = re.search(r"sweep_kernel<(\w+), (\w+), (\w+), 0,", name)
    if not m:
        m = re.search(r"sweep_kernelI(f|d)(f|d|DF16_)(f|d|DF16_)Li0E", name)
    if not m:
        return None
    return _STORAGE.get(tuple(_TYPES[t] for t in m.groups()))


def _counter_rows(path, counter):
    import csv
    out = []
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") == counter:
            out.append((r["Kernel_Name"], float(r["Counter_Value"]), int(r["Grid_Size"])))
    return out


def fold_traffic(fetch_csv, write_csv, mib):
    """Per-launch HBM bytes of the sweep from FETCH_SIZE and WRITE_SIZE (KiB
    per dispatch), each scaled by the factor that maps the same counter on the
    calibration copy to the bytes it moved."""
    rec = {"kernel_hash": kernel_hash(), "bytes_per_sweep": {}, "fetch_bytes": {},
           "write_bytes": {}, "calibration": {}, "copy_mib": mib}
    for key, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        rows = _counter_rows(path, counter)
        cal = [(v, g) for n, v, g in rows if "neg" in n]
        if not cal:
            raise SystemExit("no calibration copy dispatch in %s" % path)
        # the copy kernel's grid covers n/4 float4 or n floats; its traffic is
        # the tensor size, taken from the largest dispatch (the 1 GiB copies)
        kib = max(v for v, g in cal)
        rec["calibration"][key] = {"counter_kib": kib}
        per = {}
        for n, v, g in rows:
            s = _sweep_storage(n)
            if s is not None:
                per.setdefault(s, []).append(v)
        rec["calibration"][key]["per_storage_dispatches"] = {s: len(v) for s, v in per.items()}
        for s, vals in per.items():
            rec[key + "_bytes"][s] = sum(vals) / len(vals) * 1024.0
    return _finish_fold(rec)


def _finish_fold(rec):
    mib = rec["copy_mib"]
    nbytes = mib * (1 << 20)
    ff = nbytes / (rec["calibration"]["fetch"]["counter_kib"] * 1024.0)
    fw = nbytes / (rec["calibration"]["write"]["counter_kib"] * 1024.0)
    rec["calibration"]["fetch"]["factor"] = ff
    rec["calibration"]["write"]["factor"] = fw
    for s in rec["fetch_bytes"]:
        if s in rec["write_bytes"]:
            rec["bytes_per_sweep"][s] = rec["fetch_bytes"][s] * ff + rec["write_bytes"][s] * fw
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    print(json.dumps(rec["bytes_per_sweep"]))


def fluid_nodes(wl):
    """Nodes that are updated: not solid, not on a pressure-face ghost layer."""
    import numpy as np
    m = np.ones(wl.shape, bool) if wl.solid is None else (wl.solid == 0)
    for f, fc in enumerate(wl.faces):
        if fc is None:
            continue
        ax = 2 - f // 2                        # arrays are [z, y, x]
        idx = [slice(None)] * 3
        idx[ax] = 0 if f % 2 == 0 else -1
        m[tuple(idx)] = False
    return int(m.sum())


def _percentiles(lat):
    import numpy as np
    a = np.asarray(lat)
    return float(np.percentile(a, 50)), float(np.percentile(a, 99))


def serve_batched(trace, wls, budget_gb, cap_nodes):
    """Replay the trace in real time through the batched server."""
    from paper_2512_01032_amd import lbm
    srv = lbm.Server(storage="fp32_shift", hbm_budget=int(budget_gb * 1e9), use_graph=True,
                     ticks_per_sync=32, max_resident_nodes=int(cap_nodes))
    c0 = srv.clock()
    w0 = time.perf_counter()
    tickets = []
    for r, wl in zip(trace, wls):
        delay = r.arrival_s - (time.perf_counter() - w0)
        if delay > 0:
            time.sleep(delay)
        tickets.append(srv.submit(wl, r.steps, arrival_s=r.arrival_s))
    srv.drain()
    lat, work, tf, bad = [], 0, 0.0, 0
    for r, wl, t in zip(trace, wls, tickets):
        res = srv.poll(t)
        if res["status"] != lbm.LBM_OK:
            bad += 1
        lat.append(res["t_finish"] - (c0 + r.arrival_s))
        tf = max(tf, res["t_finish"] - c0)
        work += fluid_nodes(wl) * r.steps
    srv.close()
    p50, p99 = _percentiles(lat)
    return {"budget_GB": budget_gb, "max_resident_nodes": int(cap_nodes), "p50_s": p50,
            "p99_s": p99, "makespan_s": tf, "mlups_aggregate": work / tf / 1e6, "failed": bad}


def serve_one_at_a_time(trace, wls, torch):
    """The same trace, FIFO, one lattice at a time through lbm_create/lbm_step."""
    from paper_2512_01032_amd import lbm
    stream = torch.cuda.current_stream()
    w0 = time.perf_counter()
    lat, work = [], 0
    for r, wl in zip(trace, wls):
        delay = r.arrival_s - (time.perf_counter() - w0)
        if delay > 0:
            time.sleep(delay)
        L = lbm.Lattice(wl, storage="fp32_shift", stream=stream.cuda_stream)
        L.step(r.steps)
        L.fields()
        L.close()
        lat.append(time.perf_counter() - w0 - r.arrival_s)
        work += fluid_nodes(wl) * r.steps
    tf = time.perf_counter() - w0
    p50, p99 = _percentiles(lat)
    return {"p50_s": p50, "p99_s": p99, "makespan_s": tf, "mlups_aggregate": work / tf / 1e6}


def accuracy_leg(storages):
    """Errors of each storage mode against the FP64 oracle on the small
    validation cases: the static droplet (phi after 200 steps; Laplace
    pressure after 3000 steps against the oracle and 2 sigma / R), and the
    equilibrium contact angle of quasi-2D wall caps after 8000 steps."""
    import numpy as np
    from paper_2512_01032_amd import inputs, lbm
    from oracle import measure, ref, theory
    out = {m: {} for m in storages}

    def laplace(d, sigma):
        R = (3.0 * d["phi_sum"] / (4.0 * np.pi)) ** (1.0 / 3.0)
        return d["P_liq_mean"] - d["P_gas_mean"], theory.laplace_pressure(sigma, R)

    wl = inputs.static_droplet()
    print("[bench] accuracy: static droplet, oracle 3000 steps", file=sys.stderr, flush=True)
    o = ref.Oracle(wl)
    o.step(200)
    phi200 = o.fields()[0]
    o.step(2800)
    dP_o, dP_th = laplace(o.diagnostics(), wl.phys.sigma)
    for m in storages:
        g = lbm.Lattice(wl, storage=m)
        g.step(200)
        e200 = float(np.abs(g.fields()[0] - phi200).max())
        g.step(2800)
        dP_g, dP_gth = laplace(g.diagnostics(), wl.phys.sigma)
        g.close()
        out[m]["static_droplet"] = {
            "max_abs_dphi_200_steps": e200,
            "dP_3000_steps": dP_g, "dP_oracle": dP_o, "dP_theory_2sigma_over_R": dP_gth,
            "laplace_rel_err_vs_oracle": abs(dP_g - dP_o) / abs(dP_o),
            "laplace_rel_err_vs_theory": abs(dP_g - dP_gth) / dP_gth}
    for theta in (60.0, 120.0):
        wl = inputs.wall_cap_2d(theta)
        print("[bench] accuracy: wall cap %g deg, oracle 8000 steps" % theta, file=sys.stderr,
              flush=True)

        def angle(phi):
            pts = measure.contour_points_xz(phi[:, 0, :], z_min=1)
            pts = pts[pts[:, 1] > 2.5]
            xc, zc, Rf = measure.fit_circle(pts)
            return theory.cap_angle_from_circle(zc, Rf, wl.meta["wall_z"])
        o = ref.Oracle(wl)
        o.step(wl.steps)
        phi_o = o.fields()[0]
        a_o = angle(phi_o)
        for m in storages:
            g = lbm.Lattice(wl, storage=m)
            g.step(wl.steps)
            phi_g = g.fields()[0]
            g.close()
            a_g = angle(phi_g)
            out[m]["cap_%g" % theta] = {
                "angle_deg": a_g, "angle_oracle_deg": a_o,
                "angle_err_vs_oracle_deg": abs(a_g - a_o), "angle_err_vs_input_deg": abs(a_g - theta),
                "max_abs_dphi": float(np.abs(phi_g - phi_o).max())}
    return out


def configured_sessile(storages, steps, oracle_steps):
    """Sessile droplet, 128 x 128 x 96, 60-degree wall, 20k steps: final
    contact angle and Laplace pressure against theory (Young's angle,
    2 sigma / R of the fitted cap), and phi and the pressure jump against
    the oracle after oracle_steps steps."""
    import numpy as np
    from oracle import measure, ref, theory
    from paper_2512_01032_amd import inputs, lbm
    wl = inputs.sessile_droplet(steps=steps)
    cx, cy = wl.meta["center"]
    print("[bench] configured: sessile droplet, oracle %d steps" % oracle_steps, file=sys.stderr,
          flush=True)
    o = ref.Oracle(wl)
    o.step(oracle_steps)
    phi_o = o.fields()[0]
    do = o.diagnostics()
    fluid = o.kinds() == 0
    del o
    out = {"lattice": "128x128x96", "theta_eq_deg": wl.meta["theta"], "steps": steps,
           "oracle_steps": oracle_steps}
    for m in storages:
        print("[bench] configured: sessile droplet %s, %d steps" % (m, steps), file=sys.stderr,
              flush=True)
        g = lbm.Lattice(wl, storage=m, diag_every=1000, u_max=0.5)
        g.step(oracle_steps)
        phi_g = g.fields()[0]
        dg = g.diagnostics()
        # the liquid's mean pressure relaxes slowly (the cap's breathing
        # mode decays on R^2 / nu_l ~ 1e5 steps): its jump every 2000 steps
        el, t, jumps = 0.0, oracle_steps, []
        while t < steps:
            k = min(2000 - t % 2000, steps - t)
            t0 = time.perf_counter()
            g.step(k)
            g.sync()
            el += time.perf_counter() - t0
            t += k
            dd = g.diagnostics()
            jumps.append(dd["P_liq_mean"] - dd["P_gas_mean"])
        phi = g.fields()[0]
        d = g.diagnostics()
        g.close()
        ang, R = measure.cap_angle_3d(phi, wl.meta["wall_z"], cx, cy)
        dP = d["P_liq_mean"] - d["P_gas_mean"]
        dP_th = theory.laplace_pressure(wl.phys.sigma, R)
        jump_g = dg["P_liq_mean"] - dg["P_gas_mean"]
        jump_o = do["P_liq_mean"] - do["P_gas_mean"]
        out[m] = {"angle_deg": ang, "angle_err_vs_theta_eq_deg": ang - wl.meta["theta"],
                  "cap_radius": R, "dP": dP, "dP_theory_2sigma_over_R": dP_th,
                  "laplace_rel_err_vs_theory": abs(dP - dP_th) / dP_th,
                  "u_max": d["u_max"], "n_nan": d["n_nan"],
                  "max_abs_dphi_vs_oracle": float(np.abs(phi_g - phi_o)[fluid].max()),
                  "dP_vs_oracle_rel": abs(jump_g - jump_o) / abs(jump_o),
                  "dP_every_2000": [float("%.4e" % v) for v in jumps],
                  "seconds": el}
        print("[bench] configured: sessile %s: %s" % (m, json.dumps(out[m])), file=sys.stderr,
              flush=True)
    return out


def configured_filling(storages, steps, every, oracle_steps, t_fit=5000):
    """Capillary filling, 1024 x 32 x 32, 45-degree walls, 50k steps: the
    liquid length (phi volume over the 30 x 30 cross-section) every `every`
    steps, FP32 against FP16 g, against the square-duct Washburn law with
    the static angle from step t_fit on, and the dynamic angle that law
    needs to match the run; phi against the oracle after oracle_steps."""
    import math
    import numpy as np
    from oracle import ref, theory
    from paper_2512_01032_amd import inputs, lbm
    wl = inputs.capillary_filling(steps=steps)
    a = wl.meta["width"]
    L = wl.nx - 2
    ph = wl.phys
    mu1, mu2 = ph.rho_l * ph.nu_l, ph.rho_g * ph.nu_g
    print("[bench] configured: capillary filling, oracle %d steps" % oracle_steps,
          file=sys.stderr, flush=True)
    o = ref.Oracle(wl)
    o.step(oracle_steps)
    phi_o = o.fields()[0]
    fluid = o.kinds() == 0
    del o
    out = {"lattice": "1024x32x32", "theta_deg": wl.meta["theta"], "steps": steps,
           "sample_every": every, "oracle_steps": oracle_steps, "washburn_from_step": t_fit}
    series = {}
    for m in storages:
        print("[bench] configured: capillary filling %s, %d steps" % (m, steps), file=sys.stderr,
              flush=True)
        g = lbm.Lattice(wl, storage=m, diag_every=1000, u_max=0.5)
        zs, dphi = [], None
        t0 = time.perf_counter()
        for k in range(steps // every + 1):
            zs.append(g.diagnostics()["phi_sum"] / (a * a))
            if k * every == oracle_steps:
                dphi = float(np.abs(g.fields()[0] - phi_o)[fluid].max())
            if k < steps // every:
                g.step(every)
        g.sync()
        el = time.perf_counter() - t0
        d = g.diagnostics()
        g.close()
        series[m] = zs
        k0 = t_fit // every
        z_th = theory.washburn_square_duct(steps - t_fit, zs[k0], L, a, ph.sigma, wl.meta["theta"],
                                           mu1, mu2)
        # dynamic angle: the Washburn balance over the fitted window
        dz = zs[-1] - zs[k0]
        zbar = 0.5 * (zs[-1] + zs[k0])
        rate = dz / (steps - t_fit)
        c = (mu1 * zbar + mu2 * (L - zbar)) * rate * 28.45 / (a * 4.0 * ph.sigma)
        th_dyn = math.degrees(math.acos(max(-1.0, min(1.0, c))))
        out[m] = {"z_start": zs[0], "z_at_fit_start": zs[k0], "z_end": zs[-1],
                  "z_end_washburn_static_angle": z_th,
                  "travel_rel_err_vs_washburn": (dz - (z_th - zs[k0])) / (z_th - zs[k0]),
                  "dynamic_angle_deg": th_dyn, "u_max": d["u_max"], "n_nan": d["n_nan"],
                  "max_abs_dphi_vs_oracle": dphi, "seconds": el,
                  "z_every_2500": [round(v, 4) for v in zs[::max(1, 2500 // every)]]}
        print("[bench] configured: filling %s: z %.3f -> %.3f (Washburn %.3f), dyn angle %.2f"
              % (m, zs[0], zs[-1], z_th, th_dyn), file=sys.stderr, flush=True)
    if len(series) == 2:
        s1, s2 = (np.asarray(v) for v in series.values())
        out["max_abs_dz_fp32_vs_fp16g"] = float(np.abs(s1 - s2).max())
    return out


def configured_duct(wl, storages, steps, every=500, ramp_stable=2e-4):
    """The benchmark duct for its configured 10k steps: diagnostics every 50
    steps (NaN check), read every `every` steps.  With the configured inlet
    ramp (2e-3 over 1e4 steps) the gas near the inlet speeds up as the
    pressure rises and the run goes NaN after about 4000 steps, in FP64 as
    in FP32: the method's limit at density ratio 1000, not a precision
    effect.  The ramp is the knob: the full 10k steps are run at a ramp of
    ramp_stable in each storage mode, reporting max |u|, the NaN count, the
    phi mass at the start and the end (the pressure faces exchange mass)
    and the wall time of the graph-replayed steps."""
    import dataclasses
    from paper_2512_01032_amd import inputs, lbm
    out = {"steps": steps, "diag_every": 50}

    def run(w, m, label):
        print("[bench] configured: duct %s %s, %d steps" % (label, m, steps), file=sys.stderr,
              flush=True)
        g = lbm.Lattice(w, storage=m, diag_every=50, u_max=0.0)
        nf = g.info()["n_fluid"]
        d0 = g.diagnostics()
        umax, hist, el, t, nan_by = 0.0, [], 0.0, 0, None
        while t < steps:
            t0 = time.perf_counter()
            g.step(every)
            t += every
            try:
                g.sync()
            except lbm.LbmError as e:
                if e.code != lbm.LBM_E_UNSTABLE:
                    raise
                nan_by = t
                break
            el += time.perf_counter() - t0
            d = g.diagnostics()
            umax = max(umax, d["u_max"])
            hist.append(round(d["u_max"], 5))
        g.close()
        r = {"inlet_ramp_to": w.faces[4][1] * 1e4, "max_u": umax, "nan_by_step": nan_by,
             "u_max_every_%d" % every: hist, "phi_sum_start": d0["phi_sum"]}
        if nan_by is None:
            r["phi_sum_end"] = d["phi_sum"]
            r["n_nan"] = d["n_nan"]
            # graph replay with the FP64 diagnostics every 50 steps and a
            # host read of them every `every` steps
            r["mlups_fluid_with_diagnostics"] = nf * steps / el / 1e6
        print("[bench] configured: duct %s %s: max|u| %.4g, NaN by %s" % (label, m, umax, nan_by),
              file=sys.stderr, flush=True)
        return r

    out["configured_ramp_fp32_shift"] = run(wl, "fp32_shift", "ramp 2e-3")
    w2 = inputs.constricted_duct(slug_offset=wl.meta.get("slug_offset", 0.25), ramp_to=ramp_stable)
    for m in storages:
        out[m] = run(w2, m, "ramp %g" % ramp_stable)
    return out


def cpu_baseline_leg(wl, cpu_steps, repeats=3):
    """The FP64 oracle on the host cores: the benchmark lattice for
    cpu_steps steps, `repeats` times (median), OpenMP over every thread in
    the process's affinity mask; and the same on one thread (a child
    process with OMP_NUM_THREADS=1) over a 256 x 256 x 32 section of the
    duct (planes 40-71: walls, slugs, pressure faces at both ends), one step
    per run.
    Returns the baseline object and the oracle's phi after the first run."""
    import subprocess
    import numpy as np
    from oracle import ref
    cores = len(os.sched_getaffinity(0))
    rates = []
    phi_o = kinds = None
    for r in range(repeats):
        print("[bench] cpu baseline: oracle on %d cores, %d steps (run %d)" % (cores, cpu_steps, r + 1),
              file=sys.stderr, flush=True)
        o = ref.Oracle(wl)
        t0 = time.perf_counter()
        o.step(cpu_steps)
        el = time.perf_counter() - t0
        if phi_o is None:
            kinds = o.kinds()
            phi_o = o.fields()[0]
        nf = int((kinds == 0).sum())
        rates.append(nf * cpu_steps / el / 1e6)
        del o
    child = (
        "import sys, time, json; sys.path.insert(0, %r)\n"
        "from oracle import ref\n"
        "from paper_2512_01032_amd import inputs\n"
        "import dataclasses\n"
        "full = inputs.constricted_duct(slug_offset=0.25)\n"
        "wl = dataclasses.replace(full, nz=32, phi0=full.phi0[40:72].copy(),\n"
        "                         solid=full.solid[40:72].copy())\n"
        "out = []\n"
        "for r in range(%d):\n"
        "    o = ref.Oracle(wl)\n"
        "    nf = int((o.kinds() == 0).sum())\n"
        "    t0 = time.perf_counter(); o.step(1); el = time.perf_counter() - t0\n"
        "    out.append(nf / el / 1e6)\n"
        "print(json.dumps(out))\n" % (ROOT, repeats))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    print("[bench] cpu baseline: oracle on 1 thread, 256x256x32 section", file=sys.stderr, flush=True)
    one = json.loads(subprocess.run([sys.executable, "-c", child], env=env, check=True,
                                    capture_output=True, text=True).stdout.strip().splitlines()[-1])
    base = {"value": float(np.median(rates)), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": "full 256x256x512 duct (slug ends a quarter cell off the nodes), %d steps "
                      "after initialisation, FP64, OpenMP over %d host threads; median of %d runs"
                      % (cpu_steps, cores, repeats),
            "runs_mlups": [round(v, 3) for v in rates],
            "single_core": {"value": float(np.median(one)), "unit": "MLUPS", "cores": 1,
                            "sample": "256x256x32 section of the duct (planes 40-71), "
                                      "1 step after initialisation, FP64, one thread; median of %d"
                                      % repeats,
                            "runs_mlups": [round(v, 3) for v in one]}}
    return base, phi_o, kinds


def serving_leg(args, torch):
    from paper_2512_01032_amd import inputs
    trace = inputs.serving_trace()[:args.serve_requests]
    wls = [r.workload("fp32_shift") for r in trace]
    total = sum(fluid_nodes(wl) * r.steps for r, wl in zip(trace, wls))
    out = {"workload": "serving trace: %d requests, Poisson 50/s, droplet-on-wall e^3 or channel "
                       "2e x e/2 x e/2, e in 32..128, 2000-10000 steps, FP32 shifted" % len(trace),
           "fluid_node_updates": total, "batched": []}
    for leg in [x for x in args.serve_legs.split(",") if x]:
        b, cap = (float(v) for v in leg.split(":"))
        print("[bench] serving: batched, budget %.3g GB, resident-node cap %.3g" % (b, cap),
              file=sys.stderr, flush=True)
        r = serve_batched(trace, wls, b, cap)
        print("[bench] serving: %s" % json.dumps(r), file=sys.stderr, flush=True)
        out["batched"].append(r)
    if not args.no_serve_baseline:
        print("[bench] serving: one at a time", file=sys.stderr, flush=True)
        r = serve_one_at_a_time(trace, wls, torch)
        print("[bench] serving: %s" % json.dumps(r), file=sys.stderr, flush=True)
        out["one_at_a_time"] = r
    return out


def run_gpu(wl, storage, steps, warmup, torch):
    from paper_2512_01032_amd import lbm
    stream = torch.cuda.current_stream()
    lat = lbm.Lattice(wl, storage=storage, stream=stream.cuda_stream)
    info = lat.info()
    lat.step(warmup)
    lat.sync()
    lat.get_timing()
    lat.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    lat.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    phi_ms, sweep_ms, n = lat.get_timing()
    lat.set_timing(False)
    return lat, info, el, phi_ms / max(n, 1), sweep_ms / max(n, 1)


def variants_leg(wl, args, torch):
    """The method's options on the benchmark duct (FP32 shifted storage):
    contact-angle hysteresis (Sec. III.A), the D3Q19 phase lattice,
    sub-voxel walls (every wall surface 0.3 cells into the fluid) and
    partial slip in the interface band (wall velocity half the tangential
    fluid velocity).  Each
    reports fluid MLUPS and the sweep against the HBM roofline with its own
    population bytes per node (the hysteresis history and the wall table
    are reported as extra bytes per near-wall node)."""
    import dataclasses
    from paper_2512_01032_amd import inputs
    out = {}
    names = [v for v in args.variants.split(",") if v]
    for name in names:
        v = dataclasses.replace(wl)
        qh, extra = 7, 0
        if name == "hysteresis":
            v.phys = dataclasses.replace(wl.phys, hysteresis=1, hyst_beta=0.95)
            extra = 2 * 18 * 4
        elif name == "d3q19_phase":
            v.phys = dataclasses.replace(wl.phys, q_phase=19)
            qh = 19
        elif name == "subvoxel":
            v.sdf = inputs.duct_sdf(wl, 0.3)
            extra = 21 * 4
        elif name == "partial_slip":
            v.phys = dataclasses.replace(wl.phys, slip_factor=0.5)
        else:
            raise SystemExit("unknown variant %s" % name)
        print("[bench] variant %s: 5 warmup + %d timed steps" % (name, args.variant_steps),
              file=sys.stderr, flush=True)
        lat, info, el, phi_ms, sweep_ms = run_gpu(v, "fp32_shift", args.variant_steps, 5, torch)
        lat.close()
        b_alg = 2 * (qh * 4 + 19 * 4)
        nf = info["n_fluid"]
        achieved = b_alg * nf / (sweep_ms * 1e-3) / 1e9
        out[name] = {"mlups_fluid": round(nf * args.variant_steps / el / 1e6, 2),
                     "ms_per_step": round(el / args.variant_steps * 1e3, 4),
                     "sweep_ms": round(sweep_ms, 4), "phi_pass_ms": round(phi_ms, 4),
                     "bytes_per_fluid_update": b_alg,
                     "extra_bytes_per_near_wall_update": extra,
                     "sweep_GBs": round(achieved, 1),
                     "sweep_frac_hbm": round(achieved / HBM_PEAK_GBS, 4)}
        print("[bench] variant %s: %.1f MLUPS (fluid), sweep %.3f ms, %.0f GB/s alg"
              % (name, out[name]["mlups_fluid"], sweep_ms, achieved), file=sys.stderr, flush=True)
    return out


def streaming_leg(torch, gib=4, reps=10):
    """Context for the roofline: the HBM rate plain streaming kernels reach on
    this GPU, torch's vectorised elementwise kernels over gib-GiB FP32 tensors:
    an in-place update (each byte read and written once, the traffic shape of
    the in-place AA sweep) and a copy.  Timed with HIP events on torch's
    stream."""
    n = gib << 28
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    out = {"tensor_GiB": gib}
    for name, op in (("in_place_update_GBs", lambda: a.mul_(0.999)), ("copy_GBs", lambda: b.copy_(a))):
        for _ in range(2):
            op()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            op()
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = round(2.0 * 4 * n / (ms * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    print("[bench] streaming ceiling: %s" % json.dumps(out), file=sys.stderr, flush=True)
    return out


def storage_bytes(storage):
    return {"fp64": (8, 8), "fp32": (4, 4), "fp32_shift": (4, 4),
            "fp16_shift_g": (4, 2)}[storage]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--configured", default="sessile,filling,duct",
                    help="configured validation runs of the oracle legs (comma list; empty: skip)")
    ap.add_argument("--sessile-steps", type=int, default=20000)
    ap.add_argument("--filling-steps", type=int, default=50000)
    ap.add_argument("--duct-steps", type=int, default=10000)
    ap.add_argument("--modes", default="fp32_shift,fp16_shift_g,fp32,fp64")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (the calibration "
                         "kernel for the HBM byte counters)")
    ap.add_argument("--serve-requests", type=int, default=256,
                    help="requests of the serving trace to replay (0: skip the serving leg)")
    ap.add_argument("--serve-legs", default="64:16e6,1:0",
                    help="batched server runs as budget_GB:max_resident_nodes pairs "
                         "(0 nodes: no cap)")
    ap.add_argument("--no-serve-baseline", action="store_true",
                    help="skip the one-at-a-time replay of the serving trace")
    ap.add_argument("--variants", default="hysteresis,d3q19_phase,subvoxel,partial_slip",
                    help="options of the method timed on the same duct in FP32 shifted storage "
                         "(comma list; empty: skip)")
    ap.add_argument("--variant-steps", type=int, default=60)
    ap.add_argument("--fold-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="fold two rocprofv3 --pmc counter_collection.csv files (FETCH_SIZE, "
                         "WRITE_SIZE) into the per-launch traffic record and exit")
    args = ap.parse_args()
    if args.fold_traffic:
        fold_traffic(*args.fold_traffic, mib=args.copy_mib or 1024)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the lattice of this workload fits one MI355X and "
              "the multi-GPU (z-slab halo exchange) path is not built; use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2512_01032_amd import inputs
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    if args.copy_mib > 0:
        copy_calibration(args.copy_mib, torch)
    wl = inputs.constricted_duct(slug_offset=0.25)
    modes = args.modes.split(",")
    results = {}
    lattices = {}
    for m in modes:
        print("[bench] %s: %d warmup + %d timed steps" % (m, args.warmup, args.steps),
              file=sys.stderr, flush=True)
        lat, info, el, phi_ms, sweep_ms = run_gpu(wl, m, args.steps, args.warmup, torch)
        sh, sg = storage_bytes(m)
        b_alg = 2 * (7 * sh + 19 * sg)
        nf, nn = info["n_fluid"], info["n_nodes"]
        achieved = b_alg * nf / (sweep_ms * 1e-3) / 1e9
        results[m] = {
            "mlups_fluid": nf * args.steps / el / 1e6,
            "mlups_total_nodes": nn * args.steps / el / 1e6,
            "ms_per_step": el / args.steps * 1e3,
            "phi_pass_ms": phi_ms,
            "sweep_ms": sweep_ms,
            "bytes_per_fluid_update": b_alg,
            "sweep_GBs": achieved,
            "sweep_frac_hbm": achieved / HBM_PEAK_GBS,
            "step_GBs_alg": b_alg * nf * args.steps / el / 1e9,
        }
        # the same number of steps again through lbm_step's captured graphs
        # (no events): the rate a caller of the library sees
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(args.steps)
        lat.sync()
        torch.cuda.synchronize()
        results[m]["mlups_fluid_graph_replay"] = nf * args.steps / (time.perf_counter() - t0) / 1e6
        lattices[m] = lat
        print("[bench] %s: %.1f MLUPS (fluid), sweep %.3f ms, phi %.3f ms, %.0f GB/s alg; "
              "graph replay %.1f MLUPS" % (m, results[m]["mlups_fluid"], sweep_ms, phi_ms, achieved,
                                           results[m]["mlups_fluid_graph_replay"]),
              file=sys.stderr, flush=True)
        if m not in ("fp32_shift", "fp16_shift_g"):
            lat.close()
            del lattices[m]

    primary = results["fp32_shift"]
    variants = variants_leg(wl, args, torch)
    streaming = streaming_leg(torch)
    cpu = None
    errors = {}
    accuracy = None
    configured = None
    if not args.no_cpu_baseline:
        # FP64 oracle on the host cores, bounded sample: this lattice, a few
        # steps; the same steps on the GPU give max |phi - oracle|
        cpu, phi_o, kinds = cpu_baseline_leg(wl, args.cpu_steps)
        fluid = kinds == 0
        from paper_2512_01032_amd import lbm
        for m in ("fp32_shift", "fp16_shift_g"):
            g = lbm.Lattice(wl, storage=m)
            g.step(args.cpu_steps)
            phi_g = g.fields()[0]
            errors[m] = float(np.abs(phi_g - phi_o)[fluid].max())
            g.close()
        del phi_o
        accuracy = accuracy_leg(("fp32_shift", "fp16_shift_g", "fp64"))
        legs = [c for c in args.configured.split(",") if c]
        configured = {}
        red = ("fp32_shift", "fp16_shift_g")
        if "sessile" in legs:
            configured["sessile_droplet"] = configured_sessile(red, args.sessile_steps, 200)
        if "filling" in legs:
            configured["capillary_filling"] = configured_filling(red, args.filling_steps, 500, 500)
        if "duct" in legs:
            configured["constricted_duct"] = configured_duct(wl, red, args.duct_steps)

    serving = serving_leg(args, torch) if args.serve_requests > 0 else None

    sh, sg = storage_bytes("fp32_shift")
    b_alg = 2 * (7 * sh + 19 * sg)
    traffic = measured_traffic("fp32_shift")
    line = {
        "metric": METRIC,
        "value": round(primary["mlups_fluid"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(primary["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "constricted_duct_256x256x512", "storage": "fp32_shift",
                   "slug_offset": 0.25,
                   "nodes": wl.n_nodes, "value_counts": "fluid-node updates",
                   "density_ratio": 1000, "contact_angle_deg": 120},
        "roofline": {"bound": "hbm", "achieved": round(primary["sweep_GBs"], 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(primary["sweep_frac_hbm"], 4),
                     "traffic": traffic,
                     "kernel": "sweep_kernel (fused stream-collide)",
                     "bytes_per_unit": b_alg, "unit_count": "fluid nodes per launch"},
        "cpu_baseline": cpu,
        "streaming_ceiling": dict(streaming, sweep_frac_of_in_place=round(
            primary["sweep_GBs"] / streaming["in_place_update_GBs"], 4)),
        "modes": {m: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
                  for m, r in results.items()},
        "max_abs_dphi_vs_oracle": errors,
        "accuracy_vs_oracle": accuracy,
        "configured_runs": configured,
        "serving": serving,
        "variants": variants,
        "kernel_hash": kernel_hash(),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
