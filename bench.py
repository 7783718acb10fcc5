#!/usr/bin/env python3
"""Throughput of the fused D2Q9 stream-and-collide step on one MI355X.

Default workload: decaying Taylor-Green vortex on a fully periodic 4096 x 4096 lattice
(u0 = 0.01, wavenumber 2 pi / N, tau = 0.6), FP64 populations, dense A-B layout; exactly W
untimed warm-up steps, then K timed steps bracketed by device synchronisation (the paper's
protocol is 100 warm-up + 1000 timed kernel calls).  One JSON line on stdout:

  value     = GLUPS = fluid nodes * K / time / 1e9 of the whole job (one GPU);
  roofline  = algorithmic bytes per step kernel ((18 * pop_bytes + 1) per fluid node)
              / average kernel duration from HIP events on the stream the kernels run
              on, against the MI355X HBM peak (8 TB/s);
  cpu_baseline = the FP64 CPU oracle on the host cores, a bounded number of steps of
              the same 4096^2 workload (about 12 s), plus one step on a single thread;
  variants  = the same measurement for the other storage types (16-bit rows with their
              velocity error against the FP64 run and their mass drift), the AA layout and
              the TRT and MRT collisions; the sparse geometries (4096^2 porous discs at fluid
              fractions 0.9, 0.5, 0.2: dense, tiled and indirect layouts, FP64 and FP32,
              GLUPS per fluid node and time per fluid node against the dense all-fluid
              step); reduced-precision storage at 5000 steps (2048^2 Taylor-Green, 4096^2
              porous discs at 0.5: velocity L2 error against FP64 and the closed form, mass
              drift, GLUPS against the FP32 path); the adjoint against the forward step
              (1024 x 256 channel with drag field, T = 2000, sqrt(T) checkpoints); the copy
              kernel, the open-boundary channels, the end-to-end rate with host transfers and
              the D3Q19 lattice (256^3 three-dimensional Taylor-Green vortex; a 256^3 sphere
              packing at fluid fraction 0.4 in the dense, 4 x 4 x 4-block tiled and
              node-list layouts, time per fluid node against the dense all-fluid step); with
              --suite full also 1024^2 / 2048^2, full-way walls, set-up and view costs and
              the adjoint at 4096^2.
  Each variant states the warm-up it ran ("warmup_steps"): lattices small enough to replay
  their steps as HIP graphs warm up by at least 64 steps, so that the graphs are captured
  before the timed region.

  --suite porous: the headline, the FP32 dense step and the 4096^2 porous-disc rows only
              (the sparse layouts' profiling workload).
  --suite sparse: the paper's sparse-geometry study (Sec. 4.3, Fig. 8): sparse efficiency
              eta_P (Eq. 9) over porosity for regular and random circle obstacles, per layout.
  --suite spheres3: the copy kernel and the D3Q19 256^3 sphere packings (dense A-B, the
              4 x 4 x 4-block tiled layout and the fluid-node list), for the sparse D3Q19
              kernels' counters.

Usage: python bench.py [--gpus 1] [--steps 1000] [--warmup 100]
                       [--suite default|full|headline|porous|sparse|spheres3]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, AMD public specification
METRIC = "GLUPS & % HBM peak (dense/sparse D2Q9, fp64/fp32/16b); adjoint step cost vs fwd"
POP_BYTES = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}
PAPER_CONTEXT = {
    "hardware": "GTX Titan Xp (547.68 GB/s), Taichi dense layout, lid-driven cavity",
    "fp64_dense_max_glups": 2.65, "fp64_dense_max_U_B": 0.696,
    "fp32_dense_max_glups": 5.37, "fp32_dense_max_U_B": 0.705,
    "source": "Table 2",
}


def log(msg):
    sys.stderr.write(msg + "\n")
    sys.stderr.flush()


def algorithmic_bytes_per_node(dtype, drag=False):
    """18 populations moved (read + write) plus the node-type byte (+4 B drag field)."""
    from paper_2108_13241_amd import metrics
    return metrics.bytes_per_node(dtype, drag)


HEADLINE_SOURCES = ("lbm_device.h", "lbm_kernels.hip", "lbm_launch.h")
D3Q19_SOURCES = ("lbm3d_kernels.hip", "lbm3d_launch.h", "lbm_device.h")


def kernel_source_hash(names=HEADLINE_SOURCES):
    """Hash of the sources a kernel is built from (default: the D2Q9 step kernels)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2108_13241_amd", "csrc")
    for name in sorted(names):
        h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_key):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except (OSError, ValueError):
        return None
    rec = data.get(kernel_key)
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def time_steps(lat, steps, warmup, min_warmup=0):
    """(seconds for `steps` steps, per-step ms, warm-up steps run) with HIP events on the
    lattice's stream, after max(warmup, min_warmup) untimed steps.  Lattices that replay
    their steps as HIP graphs (small ones) pass min_warmup = 64, so that both parity graphs
    are captured (a one-time cost of a few ms) before the timed region; each record states
    the warm-up it ran."""
    import torch
    stream = torch.cuda.current_stream()
    warm = max(warmup, min_warmup)
    lat.step(warm)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    lat.step(steps)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    return ms / 1e3, ms / max(steps, 1), warm


def device_velocity(lat):
    """(u_x, u_y) of a D2Q9 lattice as device FP64 tensors [ny, nx] (solid nodes 0)."""
    import torch
    ux = torch.empty((lat.ny, lat.nx), dtype=torch.float64, device="cuda")
    uy = torch.empty_like(ux)
    lat.macroscopic_device(None, ux, uy)
    return ux, uy


def l2_rel(u, ref):
    """Relative L2 distance of velocity fields (tuples of device FP64 tensors; solid nodes
    hold 0 in both, so they add nothing)."""
    import torch
    num = sum(((a - b) ** 2).sum() for a, b in zip(u, ref))
    den = sum((b ** 2).sum() for b in ref)
    return float(torch.sqrt(num / den))


def taylor_green_velocity(n, u0, tau, t):
    """Closed-form Taylor-Green velocity after t steps: the initial field decayed by
    exp(-2 nu k^2 t), nu = (tau - 1/2) / 3 (Eq. 5), k = 2 pi / n; device FP64 tensors."""
    import torch
    k = 2.0 * math.pi / n
    nu = (tau - 0.5) / 3.0
    dec = math.exp(-2.0 * nu * k * k * t)
    x = torch.arange(n, dtype=torch.float64, device="cuda")[None, :]
    y = torch.arange(n, dtype=torch.float64, device="cuda")[:, None]
    return (-u0 * dec * torch.cos(k * x) * torch.sin(k * y),
            u0 * dec * torch.sin(k * x) * torch.cos(k * y))


def measure_dense(lbm, n, dtype, layout, steps, warmup, fields, trt=0.0, mrt=None, ref=None,
                  keep=False):
    """Taylor-Green n^2 throughput.  ref: the FP64 velocity field after the same number of
    steps (device tensors), against which the row's velocity error is stated; keep: also
    return this run's velocity field (for use as such a reference)."""
    import synthetic
    m = synthetic.all_fluid(n, n)
    lat = lbm.Lattice(m, 0.6, dtype=dtype, layout=layout)
    lat.set_trt(trt)
    if mrt is not None:
        lat.set_mrt(mrt)
    lat.init_equilibrium(*fields)
    M0 = lat.mass() if (ref is not None or keep) else None
    secs, ms, warm = time_steps(lat, steps, warmup)
    info = lat.info()
    u = None
    extra = {}
    if ref is not None or keep:
        u = device_velocity(lat)
        extra["mass_drift"] = (lat.mass() - M0) / M0
        if ref is not None:
            extra["l2_err_vs_fp64"] = l2_rel(u, ref)
            extra["l2_err_reference"] = ("FP64 HIP path, same layout, collision and step count "
                                         "(pinned to the oracle by sampled-window parity at "
                                         "4096^2)")
    lat.close()
    nf = info["n_fluid"]
    glups = nf * steps / secs / 1e9
    bpn = algorithmic_bytes_per_node(dtype)
    model = (f" TRT magic={trt:g}" if trt else "") + \
        (" MRT s_e,s_eps,s_q=" + ",".join(f"{v:g}" for v in mrt) if mrt is not None else "")
    row = {"workload": f"taylor-green {n}^2" + model,
           "dtype": dtype, "layout": layout,
           "glups": glups, "ms_per_step": ms, "hbm_gbps": glups * bpn,
           "frac_of_peak": glups * bpn / HBM_PEAK_GBPS,
           "paper_U_B_bytes": 18 * POP_BYTES[dtype], "bytes_per_node": bpn,
           "steps": steps, "warmup_steps": warm, **extra}
    return (row, u) if keep else row


def measure_d3q19(lbm, n, dtype, steps, warmup, layout="dense_ab", mrt=None, ref=None,
                  keep=False):
    """D3Q19 dense A-B (or AA) step on the periodic n^3 three-dimensional Taylor-Green
    vortex.  AA timings cover an even number of steps (odd and even kernels alike).  ref /
    keep: as for measure_dense (velocity fields as device tensors)."""
    import torch

    import synthetic
    m = np.zeros((n, n, n), np.uint8)
    lat = lbm.Lattice3D(m, 0.6, dtype=dtype, layout=layout)
    if mrt is not None:
        lat.set_mrt(mrt)
    lat.init_equilibrium(*synthetic.taylor_green3(n, 0.01))
    M0 = lat.mass() if (ref is not None or keep) else None
    secs, ms, warm = time_steps(lat, steps, warmup)
    nf = lat.info()["n_fluid"]
    u = None
    extra = {}
    if ref is not None or keep:
        fields = [torch.empty((n, n, n), dtype=torch.float64, device="cuda") for _ in range(4)]
        lat.macroscopic_device(*fields)
        u = tuple(fields[1:])
        extra["mass_drift"] = (lat.mass() - M0) / M0
        if ref is not None:
            extra["l2_err_vs_fp64"] = l2_rel(u, ref)
            extra["l2_err_reference"] = "FP64 HIP path, same layout and step count"
        del fields
    lat.close()
    glups = nf * steps / secs / 1e9
    bpn = 38 * POP_BYTES[dtype] + 1
    row = {"workload": f"d3q19 taylor-green {n}^3" + (" MRT" if mrt is not None else ""),
           "dtype": dtype, "layout": layout,
           "glups": glups, "ms_per_step": ms, "hbm_gbps": glups * bpn,
           "frac_of_peak": glups * bpn / HBM_PEAK_GBPS, "bytes_per_node": bpn,
           "steps": steps, "warmup_steps": warm, **extra}
    return (row, u) if keep else row


def measure_end_to_end(lbm, n, fields, steps):
    """The headline workload including its host transfers: re-initialisation from host FP64
    fields (rho, ux, uy uploaded), `steps` steps, and the macroscopic fields read back into
    host arrays.  Reported beside the headline, never as its value."""
    import torch

    import synthetic
    lat = lbm.Lattice(synthetic.all_fluid(n, n), 0.6, dtype="f64", layout="dense_ab")
    lat.init_equilibrium(*fields)
    lat.step(64)
    lat.macroscopic()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.init_equilibrium(*fields)
    t1 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    lat.macroscopic()
    t3 = time.perf_counter()
    lat.close()
    return {"workload": f"taylor-green {n}^2 f64 dense_ab, host fields in and out",
            "steps": steps, "upload_init_s": t1 - t0, "steps_s": t2 - t1,
            "download_macroscopic_s": t3 - t2,
            "glups_incl_host_transfers": n * n * steps / (t3 - t0) / 1e9}


def measure_copy(lbm, nbytes, reps=20):
    """Achievable read+write bandwidth of a plain 16-byte copy kernel (a10)."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    for _ in range(3):
        lbm.copy_kernel(a, b, nbytes)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        lbm.copy_kernel(a, b, nbytes)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    return {"bytes": nbytes, "gbps": 2 * nbytes / s / 1e9, "frac_of_peak": 2 * nbytes / s / 1e9 / HBM_PEAK_GBPS}


def measure_porous(lbm, n, phi, dtype, layout, steps, warmup, mask, wall="halfway",
                   dense_ms_per_node=None):
    """Porous discs (walls at y = 0 and n - 1, periodic x, g_x = 1e-6, tau = 0.6): GLUPS per
    fluid node (Eq. 8 counts non-solid nodes only).  dense_ms_per_node: time per node of the
    dense A-B step on the all-fluid n^2 lattice in the same dtype; the row then states its
    time per fluid node relative to it (the sparse target is 1.3)."""
    lat = lbm.Lattice(mask, 0.6, force=(1e-6, 0.0), dtype=dtype, layout=layout)
    lat.set_bounce_back(wall)
    secs, ms, warm = time_steps(lat, steps, warmup)
    info = lat.info()
    lat.close()
    nf = info["n_fluid"]
    glups = nf * steps / secs / 1e9
    bpn = algorithmic_bytes_per_node(dtype)
    out = {"workload": f"porous discs {n}^2 phi={phi}"
                       + (" full-way bounce-back" if wall == "fullway" else ""),
           "dtype": dtype, "layout": layout,
           "n_fluid": nf, "glups_per_fluid_node": glups, "ms_per_step": ms,
           "frac_of_peak": glups * bpn / HBM_PEAK_GBPS,
           "bytes_moved_per_step": info["bytes_moved_per_step"],
           "steps": steps, "warmup_steps": warm}
    if dense_ms_per_node:
        out["time_per_fluid_node_over_dense_all_fluid"] = (ms / nf) / dense_ms_per_node
    if layout == "tiled16":
        out["tile_occupancy"] = nf / max(1, info["n_tiles"] * 256)
    return out


def porous_rows(lbm, n, steps, warmup, dense_ms_per_node):
    """The n^2 porous discs at fluid fractions 0.9, 0.5 and 0.2 in the dense, tiled and
    indirect layouts, FP64 and FP32 (GLUPS per fluid node and time per fluid node against
    the dense all-fluid step of the same dtype)."""
    import synthetic
    rows = []
    for phi in (0.9, 0.5, 0.2):
        mask, minfo = synthetic.porous_discs(n, phi)
        log(f"[bench]   porous phi={phi}: achieved {minfo['phi_achieved']:.3f}")
        for dtype in ("f64", "f32"):
            for layout in ("dense_ab", "tiled16", "indirect"):
                r = measure_porous(lbm, n, phi, dtype, layout, steps, warmup, mask,
                                   dense_ms_per_node=dense_ms_per_node[dtype])
                r["phi_achieved"] = minfo["phi_achieved"]
                log(f"[bench]   phi={phi} {dtype} {layout}: "
                    f"{r['glups_per_fluid_node']:.2f} GLUPS/fluid, time per fluid node "
                    f"{r['time_per_fluid_node_over_dense_all_fluid']:.2f}x dense")
                rows.append(r)
        del mask
    return rows


def measure_reduced(lbm, case, n, steps=5000):
    """Reduced-precision storage at the stated configuration: `steps` steps from the initial
    state, for FP64 (the reference), FP32, FP16 and BF16 shifted storage.  case "tgv": the
    n^2 Taylor-Green vortex, dense A-B; case "porous": the n^2 porous discs at fluid fraction
    0.5 with g_x = 1e-6, tiled layout.  Each row: GLUPS (timed over the `steps` steps) and its
    ratio to the FP32 path, the velocity field's relative L2 error against the FP64 run and
    (vortex) against the closed-form decay, and the relative mass drift."""
    import torch

    import synthetic
    if case == "tgv":
        mask = synthetic.all_fluid(n, n)
        fields, g, layout = synthetic.taylor_green(n, 0.01), (0.0, 0.0), "dense_ab"
        name = f"reduced precision: taylor-green {n}^2, {steps} steps"
        exact = taylor_green_velocity(n, 0.01, 0.6, steps)
    else:
        mask, _ = synthetic.porous_discs(n, 0.5)
        fields, g, layout = None, (1e-6, 0.0), "tiled16"
        name = f"reduced precision: porous discs {n}^2 phi=0.5 g_x=1e-6, {steps} steps"
        exact = None
    rows, ref = [], None
    for dtype in ("f64", "f32", "f16s", "bf16s"):
        lat = lbm.Lattice(mask, 0.6, force=g, dtype=dtype, layout=layout)
        if fields is not None:
            lat.init_equilibrium(*fields)
        M0 = lat.mass()
        secs, ms, _ = time_steps(lat, steps, 0)
        u = device_velocity(lat)
        drift = (lat.mass() - M0) / M0
        nf = lat.info()["n_fluid"]
        lat.close()
        row = {"workload": name, "dtype": dtype, "layout": layout, "steps": steps,
               "glups": nf * steps / secs / 1e9, "ms_per_step": ms, "mass_drift": drift}
        if ref is None:
            ref = u
        else:
            row["l2_err_vs_fp64"] = l2_rel(u, ref)
            row["l2_err_reference"] = ("FP64 HIP path, same layout and step count (pinned to "
                                       "the oracle by sampled-window parity at 4096^2)")
        if exact is not None:
            row["l2_err_vs_closed_form"] = l2_rel(u, exact)
        rows.append(row)
        if dtype != "f64":
            del u
    f32 = next(r["glups"] for r in rows if r["dtype"] == "f32")
    for r in rows:
        r["glups_over_fp32_path"] = r["glups"] / f32
    del ref, exact
    torch.cuda.empty_cache()
    return rows


def measure_porous3(lbm, n, phi, dtype, layout, steps, warmup, mask, dense_ms_per_node=None):
    """D3Q19 sphere packing (walls in z, body force along x): dense A-B (solid nodes skipped),
    the 4 x 4 x 4-block tiled layout and the fluid-node list, GLUPS per fluid node.
    dense_ms_per_node: time per node of the dense A-B step on the all-fluid n^3 lattice in the
    same dtype; the row then states its time per fluid node relative to it."""
    lat = lbm.Lattice3D(mask, 0.6, force=(1e-6, 0.0, 0.0), dtype=dtype, layout=layout)
    secs, ms, warm = time_steps(lat, steps, warmup)
    info = lat.info()
    lat.close()
    nf = info["n_fluid"]
    glups = nf * steps / secs / 1e9
    bpn = info["bytes_per_fluid_node"]
    out = {"workload": f"d3q19 sphere packing {n}^3 phi={phi}", "dtype": dtype,
           "layout": layout, "n_fluid": nf, "glups_per_fluid_node": glups, "ms_per_step": ms,
           "bytes_per_fluid_node": bpn, "frac_of_peak": glups * bpn / HBM_PEAK_GBPS,
           "steps": steps, "warmup_steps": warm}
    if dense_ms_per_node:
        out["time_per_fluid_node_over_dense_all_fluid"] = (ms / nf) / dense_ms_per_node
    if layout == "tiled16":
        b = (mask.reshape(n // 4, 4, n // 4, 4, n // 4, 4) == 0).any(axis=(1, 3, 5))
        out["block_occupancy"] = nf / max(1, int(b.sum()) * 64)
    return out


def measure_open_channel(lbm, inlet, dtype, layout, steps, warmup, nx=4096, ny=512):
    """The paper's channel cases (Sec. 4.1): chan_v (inlet u = 0.1) or chan_p (inlet
    rho = 1.016, initial 1.008), outlet rho = 1, bounce-back walls, nu = 0.25 (tau = 1.25)."""
    import synthetic
    m, bc, val = synthetic.open_channel(nx, ny, inlet, u_in=0.1, rho_in=1.016)
    lat = lbm.Lattice(m, 1.25, dtype=dtype, layout=layout)
    lat.set_boundaries(bc, val)
    if inlet == "pressure":
        lat.init_equilibrium(np.full((ny, nx), 1.008), None, None)
    secs, ms, _ = time_steps(lat, steps, warmup, min_warmup=64)
    nf = lat.info()["n_fluid"]
    lat.close()
    glups = nf * steps / secs / 1e9
    bpn = algorithmic_bytes_per_node(dtype)
    return {"workload": f"chan_{inlet[0]} {nx}x{ny} (open inlet / outlet)", "dtype": dtype,
            "layout": layout, "glups": glups, "ms_per_step": ms,
            "frac_of_peak": glups * bpn / HBM_PEAK_GBPS,
            "note": "working set partly resident in the 256 MB Infinity Cache"}


def measure_small_channel(lbm, steps=2000):
    """256 x 64 channel (walls at y = 0 and 63, g = 1e-6, tau = 0.8, FP64): a launch-bound
    size; time per step with one launch per step and with steps replayed as HIP graphs."""
    import synthetic
    m = synthetic.channel_mask(256, 64)
    out = {"workload": "channel 256x64 f64 dense_ab (launch-bound)", "steps": steps}
    for name, g in (("launch_per_step", 0), ("hip_graph_32", 32)):
        lat = lbm.Lattice(m, 0.8, force=(1e-6, 0.0), dtype="f64", layout="dense_ab")
        lat.set_graph_steps(g)
        secs, ms, _ = time_steps(lat, steps, 64)
        out[f"us_per_step_{name}"] = ms * 1e3
        lat.close()
    return out


def measure_setup(lbm, mask, dtype="f64"):
    """Geometry preprocessing on the host plus device set-up (lbm_create: planning, uploads,
    allocation, equilibrium initial state) and a re-initialisation alone, per layout."""
    import torch
    out = []
    for layout in ("dense_ab", "dense_aa", "tiled16", "tiled16_all", "indirect"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat = lbm.Lattice(mask, 0.6, dtype=dtype, layout=layout)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lat.init_equilibrium(None, None, None)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        out.append({"layout": layout, "dtype": dtype, "create_s": t1 - t0,
                    "init_equilibrium_s": t2 - t1, "n_fluid": lat.info()["n_fluid"]})
        lat.close()
    return out


def measure_views(lbm, n, fields, reps=20):
    """Macroscopic fields (Eq. 2; device FP64 rho, u_x, u_y) and the FP64 mass reduction on
    the 4096^2 FP64 dense lattice, against their algorithmic bytes: every population read
    once (+ the node type), 24 B written per node for the fields."""
    import torch
    import synthetic
    m = synthetic.all_fluid(n, n)
    lat = lbm.Lattice(m, 0.6, dtype="f64", layout="dense_ab")
    lat.init_equilibrium(*fields)
    out = [torch.empty((n, n), dtype=torch.float64, device="cuda") for _ in range(3)]
    lat.macroscopic_device(*out)
    lat.mass()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        lat.macroscopic_device(*out)
    e1.record()
    torch.cuda.synchronize()
    macro_s = e0.elapsed_time(e1) / 1e3 / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        lat.mass()  # includes the device-to-host copy of the result and a stream sync
    mass_s = (time.perf_counter() - t0) / reps
    lat.close()
    nodes = n * n
    macro_b = nodes * (9 * 8 + 1 + 24)
    mass_b = nodes * (9 * 8 + 1)
    return {"workload": f"views taylor-green {n}^2 f64 dense_ab",
            "macroscopic_ms": macro_s * 1e3, "macroscopic_gbps": macro_b / macro_s / 1e9,
            "macroscopic_frac_of_peak": macro_b / macro_s / 1e9 / HBM_PEAK_GBPS,
            "mass_ms_with_sync": mass_s * 1e3, "mass_gbps": mass_b / mass_s / 1e9}


def measure_sparse_geometry(lbm, geom, dtype, layout, steps, warmup):
    """One of the paper's sparse geometries (Sec. 4.3): pressure inlet / outlet, walls,
    nu = 0.5 (tau = 2); GLUPS counting non-solid nodes only (Eq. 8)."""
    m, bc, val, info = geom
    lat = lbm.Lattice(m, 2.0, dtype=dtype, layout=layout)
    lat.set_boundaries(bc, val)
    secs, ms, _ = time_steps(lat, steps, warmup, min_warmup=64)
    li = lat.info()
    lat.close()
    nf = li["n_fluid"]
    return {"kind": info["kind"], "phi": info.get("phi_target", 1.0),
            "phi_achieved": info["phi_achieved"], "dtype": dtype, "layout": layout,
            "glups_per_fluid_node": nf * steps / secs / 1e9, "ms_per_step": ms,
            "n_tiles": li["n_tiles"] if layout.startswith("tiled16") else None}


def sparse_study(lbm, n, steps, warmup):
    """eta_P (Eq. 9) over porosity for the regular 8 x 8 circle array (phi >= 0.3) and
    random circles r in [8, 256] (Sec. 4.3, Fig. 8), per layout and dtype, against the same
    channel without obstacles (the dense geometry) in the same layout."""
    import synthetic
    from paper_2108_13241_amd import metrics
    layouts = ("dense_ab", "tiled16", "tiled16_all", "indirect")
    dtypes = ("f32", "f64")
    rows = []
    dense = synthetic.open_box(n)
    ref = {}
    for dt in dtypes:
        for lay in layouts:
            r = measure_sparse_geometry(lbm, dense, dt, lay, steps, warmup)
            ref[(dt, lay)] = r["glups_per_fluid_node"]
            r["eta_P"] = 1.0
            rows.append(r)
    log(f"[bench]   dense reference: " + ", ".join(f"{k[0]} {k[1]} {v:.1f}" for k, v in ref.items()))
    geoms = [("regular", phi) for phi in (0.9, 0.8, 0.7, 0.6, 0.5, 0.4, 0.3)] + \
            [("random", phi) for phi in (0.9, 0.8, 0.7, 0.6, 0.5, 0.4, 0.3, 0.2, 0.1)]
    for kind, phi in geoms:
        geom = synthetic.circle_array(n, phi) if kind == "regular" else \
            synthetic.random_circles(n, phi)
        line = []
        for dt in dtypes:
            for lay in layouts:
                r = measure_sparse_geometry(lbm, geom, dt, lay, steps, warmup)
                r["eta_P"] = metrics.sparse_efficiency(r["glups_per_fluid_node"], ref[(dt, lay)])
                rows.append(r)
                line.append(f"{dt} {lay} {r['eta_P']:.2f}")
        log(f"[bench]   {kind} phi={phi}: eta_P " + ", ".join(line))
    return rows


def measure_adjoint(lbm, steps=200, T=2000):
    """Adjoint cost on the 1024 x 256 channel with a drag field, FP32.

    adjoint_over_forward: one adjoint step (adjoint kernel + its dJ/dg partial reduction) per
    host call against one forward step per host call (graph replay off, so both pay the same
    launch path).  checkpointed_*: the drivers as a user runs them, T steps with checkpoints
    every K = ceil(sqrt(T)) (forward with checkpoint copies; backward = segment recompute +
    adjoint), whole-run wall time on the device."""
    import torch

    import synthetic
    nx, ny = 1024, 256
    m = synthetic.channel_mask(nx, ny)
    alpha = synthetic.brinkman_alpha(nx, ny, seed=7, sigma=8.0).astype(np.float32)
    lat = lbm.Lattice(m, 0.8, force=(1e-5, 0.0), dtype="f32", layout="dense_ab")
    lat.set_porosity(alpha)
    lat.set_graph_steps(0)
    fwd_s, fwd_ms, _ = time_steps(lat, steps, 20)
    lat.set_graph_steps(-1)
    _, fwd_graph_ms, _ = time_steps(lat, steps, 64)
    sb = lat.state_bytes()
    state = torch.empty(sb, dtype=torch.uint8, device="cuda")
    lat.save_state(state)
    ab, _ = lat.adjoint_bytes()
    mu = [torch.zeros(ab, dtype=torch.uint8, device="cuda") for _ in range(2)]
    ga = torch.zeros((ny, nx), dtype=torch.float64, device="cuda")
    gg = torch.zeros(2, dtype=torch.float64, device="cuda")
    lat.adjoint_seed_outlet_ux(nx - 1, 1.0, mu[0], ga, gg)
    for k in range(20):
        lat.adjoint_step(state, mu[k % 2], mu[1 - k % 2], ga, gg)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(steps):
        lat.adjoint_step(state, mu[k % 2], mu[1 - k % 2], ga, gg)
    e1.record()
    torch.cuda.synchronize()
    adj_ms = e0.elapsed_time(e1) / steps
    # checkpointed drivers (one untimed forward + backward first: the first backward on a
    # context also creates its auxiliary stream and second segment buffer)
    K = int(math.ceil(math.sqrt(T)))
    ckpt = torch.empty(((T + K - 1) // K) * sb, dtype=torch.uint8, device="cuda")
    seg = torch.empty(K * sb, dtype=torch.uint8, device="cuda")
    lat.init_equilibrium(None, None, None)
    lat.run_checkpointed(T, K, ckpt)
    lat.adjoint_checkpointed(T, K, ckpt, seg, nx - 1, 1.0, ga, gg)
    lat.init_equilibrium(None, None, None)
    torch.cuda.synchronize()
    e0.record()
    lat.run_checkpointed(T, K, ckpt)
    e1.record()
    torch.cuda.synchronize()
    run_ms = e0.elapsed_time(e1)
    ga.zero_()
    gg.zero_()
    torch.cuda.synchronize()
    e0.record()
    lat.adjoint_checkpointed(T, K, ckpt, seg, nx - 1, 1.0, ga, gg)
    e1.record()
    torch.cuda.synchronize()
    back_ms = e0.elapsed_time(e1)
    lat.close()
    del ckpt, seg
    return {"workload": "channel 1024x256 with drag field, f32", "forward_ms_per_step": fwd_ms,
            "forward_graph_replay_ms_per_step": fwd_graph_ms,
            "adjoint_ms_per_step": adj_ms, "adjoint_over_forward": adj_ms / fwd_ms,
            "checkpointed_T": T, "checkpointed_K": K,
            "checkpointed_forward_ms": run_ms, "checkpointed_backward_ms": back_ms,
            "checkpointed_backward_over_forward": back_ms / run_ms}


def measure_adjoint_large(lbm, n=4096, steps=50):
    """Adjoint kernel against the forward step at a size where both are HBM-bound: n x n
    channel with a drag field, FP32 state.  Algorithmic bytes per fluid node: forward 77
    (18 x 4 + type + alpha), adjoint 129 (state 36 + lambda in 36 + lambda out 36 + alpha 4 +
    type 1 + FP64 gradient read-modify-write 16)."""
    import torch

    import synthetic
    m = synthetic.channel_mask(n, n)
    alpha = synthetic.brinkman_alpha(n, n, seed=7, sigma=8.0).astype(np.float32)
    lat = lbm.Lattice(m, 0.8, force=(1e-5, 0.0), dtype="f32", layout="dense_ab")
    lat.set_porosity(alpha)
    fwd_s, fwd_ms, _ = time_steps(lat, steps, 10)
    state = torch.empty(lat.state_bytes(), dtype=torch.uint8, device="cuda")
    lat.save_state(state)
    ab, _ = lat.adjoint_bytes()
    mu = [torch.zeros(ab, dtype=torch.uint8, device="cuda") for _ in range(2)]
    ga = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    gg = torch.zeros(2, dtype=torch.float64, device="cuda")
    lat.adjoint_seed_outlet_ux(n - 1, 1.0, mu[0], ga, gg)
    for k in range(5):
        lat.adjoint_step(state, mu[k % 2], mu[1 - k % 2], ga, gg)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(steps):
        lat.adjoint_step(state, mu[k % 2], mu[1 - k % 2], ga, gg)
    e1.record()
    torch.cuda.synchronize()
    adj_ms = e0.elapsed_time(e1) / steps
    nf = lat.info()["n_fluid"]
    lat.close()
    del state, mu, ga
    return {"workload": f"adjoint channel {n}x{n} with drag field, f32",
            "forward_ms_per_step": fwd_ms, "adjoint_ms_per_step": adj_ms,
            "adjoint_over_forward": adj_ms / fwd_ms,
            "forward_frac_of_peak": nf * 77 / (fwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
            "adjoint_frac_of_peak": nf * 129 / (adj_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(n, fields, budget_s=12.0):
    """The FP64 oracle (as it is) on the host cores, a bounded number of steps; plus one
    step on a single thread."""
    import oracle
    import synthetic
    m = synthetic.all_fluid(n, n)
    f = oracle.init(m, *fields)
    threads = oracle.max_threads()
    f = oracle.run(m, f, 0.6, 1, threads=threads)  # first touch of the buffers
    # per-step cost without the per-call copy and allocation: 4 steps minus 1 step
    t0 = time.perf_counter()
    f = oracle.run(m, f, 0.6, 1, threads=threads)
    t1 = time.perf_counter()
    f = oracle.run(m, f, 0.6, 4, threads=threads)
    t4 = time.perf_counter() - t1
    one = max((t4 - (t1 - t0)) / 3.0, 1e-4)
    steps = int(max(1, min(400, budget_s / one)))
    t0 = time.perf_counter()
    f = oracle.run(m, f, 0.6, steps, threads=threads)
    secs = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.run(m, f, 0.6, 1, threads=1)
    secs1 = time.perf_counter() - t0
    return {"value": n * n * steps / secs / 1e9, "unit": "GLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} steps of the taylor-green {n}^2 FP64 workload "
                      f"({secs:.1f} s, OpenMP over rows)",
            "value_1thread": n * n / secs1 / 1e9, "cpu_model": _cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--suite", default="default",
                    choices=["default", "full", "headline", "porous", "sparse", "spheres3"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-reps", type=int, default=20)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print("bench.py measures one GPU: the step runs on a single MI355X and there is "
              "no multi-GPU path (run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2108_13241_amd as lbm
    import synthetic
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    lbm.load()
    n = args.size
    fields = synthetic.taylor_green(n, 0.01)

    log(f"[bench] headline: taylor-green {n}^2 f64 dense_ab, {args.warmup}+{args.steps} steps")
    keep = args.suite in ("default", "full")
    head = measure_dense(lbm, n, "f64", "dense_ab", args.steps, args.warmup, fields, keep=keep)
    if keep:
        head, u64 = head
    log(f"[bench]   {head['glups']:.2f} GLUPS, {head['hbm_gbps']:.0f} GB/s")
    variants = []
    if args.suite == "sparse":
        variants.extend(sparse_study(lbm, n, max(args.steps // 5, 20), max(args.warmup // 5, 5)))
    if args.suite == "porous":
        f32 = measure_dense(lbm, n, "f32", "dense_ab", args.steps, args.warmup, fields)
        variants.append(f32)
        variants.extend(porous_rows(lbm, n, args.steps, args.warmup,
                                    {"f64": head["ms_per_step"] / (n * n),
                                     "f32": f32["ms_per_step"] / (n * n)}))
    if args.suite == "headline":
        c = measure_copy(lbm, 1 << 30, reps=args.copy_reps)
        log(f"[bench]   copy kernel: {c['gbps']:.0f} GB/s")
        variants.append({"workload": "copy kernel 1 GiB", **c})
    if args.suite in ("default", "full"):
        dense_ms_per_node = {"f64": head["ms_per_step"] / (n * n)}
        for dtype, layout in [("f32", "dense_ab"), ("f64", "dense_aa"), ("f32", "dense_aa"),
                              ("f16s", "dense_ab"), ("bf16s", "dense_ab")]:
            r = measure_dense(lbm, n, dtype, layout, args.steps, args.warmup, fields,
                              ref=u64 if dtype in ("f16s", "bf16s") else None)
            err = f", L2 err vs FP64 {r['l2_err_vs_fp64']:.2e}" if "l2_err_vs_fp64" in r else ""
            log(f"[bench]   {dtype} {layout}: {r['glups']:.2f} GLUPS ({r['frac_of_peak']:.3f}){err}")
            variants.append(r)
            if layout == "dense_ab" and dtype == "f32":
                dense_ms_per_node["f32"] = r["ms_per_step"] / (n * n)
        del u64
        for dtype in ("f64", "f32"):
            r = measure_dense(lbm, n, dtype, "dense_ab", args.steps, args.warmup, fields,
                              trt=3.0 / 16.0)
            log(f"[bench]   {dtype} dense_ab TRT: {r['glups']:.2f} GLUPS ({r['frac_of_peak']:.3f})")
            variants.append(r)
        u_mrt = None
        for dtype in ("f64", "f32", "f16s"):
            r = measure_dense(lbm, n, dtype, "dense_ab", args.steps, args.warmup, fields,
                              mrt=(1.19, 1.4, 1.2), keep=dtype == "f64",
                              ref=u_mrt if dtype == "f16s" else None)
            if dtype == "f64":
                r, u_mrt = r
            err = f", L2 err vs FP64 {r['l2_err_vs_fp64']:.2e}" if "l2_err_vs_fp64" in r else ""
            log(f"[bench]   {dtype} dense_ab MRT: {r['glups']:.2f} GLUPS "
                f"({r['frac_of_peak']:.3f}){err}")
            variants.append(r)
        del u_mrt
        # sparse geometries (porous discs at three fluid fractions; per-fluid-node rates)
        variants.extend(porous_rows(lbm, n, args.steps, args.warmup, dense_ms_per_node))
        # reduced-precision storage at its stated configuration
        for case, nn in (("tgv", 2048), ("porous", n)):
            for r in measure_reduced(lbm, case, nn):
                cf = (f", vs closed form {r['l2_err_vs_closed_form']:.2e}"
                      if "l2_err_vs_closed_form" in r else "")
                ef = f", L2 err vs FP64 {r['l2_err_vs_fp64']:.2e}" if "l2_err_vs_fp64" in r else ""
                log(f"[bench]   {r['workload']} {r['dtype']}: {r['glups']:.2f} GLUPS "
                    f"({r['glups_over_fp32_path']:.2f}x FP32){ef}{cf}, "
                    f"mass drift {r['mass_drift']:.1e}")
                variants.append(r)
        # adjoint against forward (1024 x 256 channel with drag field, T = 2000)
        a = measure_adjoint(lbm)
        log(f"[bench]   adjoint/forward = {a['adjoint_over_forward']:.2f} per step; "
            f"checkpointed backward/forward = {a['checkpointed_backward_over_forward']:.2f}")
        variants.append(a)
        c = measure_copy(lbm, 1 << 30)
        log(f"[bench]   copy kernel: {c['gbps']:.0f} GB/s")
        variants.append({"workload": "copy kernel 1 GiB", **c})
        for inlet in ("velocity", "pressure"):
            r = measure_open_channel(lbm, inlet, "f32", "dense_ab", args.steps, args.warmup)
            log(f"[bench]   {r['workload']} f32: {r['glups']:.2f} GLUPS")
            variants.append(r)
        r = measure_small_channel(lbm)
        log(f"[bench]   channel 256x64: {r['us_per_step_launch_per_step']:.2f} us/step, "
            f"graphs {r['us_per_step_hip_graph_32']:.2f} us/step")
        variants.append(r)
        r = measure_end_to_end(lbm, n, fields, args.steps)
        log(f"[bench]   end to end with host transfers: {r['glups_incl_host_transfers']:.2f} GLUPS "
            f"(upload + init {r['upload_init_s'] * 1e3:.0f} ms, read-back "
            f"{r['download_macroscopic_s'] * 1e3:.0f} ms)")
        variants.append(r)
        u3 = None
        d3_ms_per_node = {}
        for dtype in ("f64", "f32", "f16s"):
            r = measure_d3q19(lbm, 256, dtype, args.steps // 2, args.warmup, keep=dtype == "f64",
                              ref=u3 if dtype == "f16s" else None)
            if dtype == "f64":
                r, u3 = r
            d3_ms_per_node[dtype] = r["ms_per_step"] / 256 ** 3
            err = f", L2 err vs FP64 {r['l2_err_vs_fp64']:.2e}" if "l2_err_vs_fp64" in r else ""
            log(f"[bench]   d3q19 256^3 {dtype}: {r['glups']:.2f} GLUPS "
                f"({r['frac_of_peak']:.3f}){err}")
            variants.append(r)
        del u3
        for dtype in ("f64", "f32"):
            r = measure_d3q19(lbm, 256, dtype, 2 * (args.steps // 4), args.warmup, "dense_aa")
            log(f"[bench]   d3q19 256^3 {dtype} dense_aa: {r['glups']:.2f} GLUPS "
                f"({r['frac_of_peak']:.3f})")
            variants.append(r)
        for dtype in ("f64", "f32"):
            r = measure_d3q19(lbm, 256, dtype, args.steps // 2, args.warmup,
                              mrt=(1.19, 1.4, 1.2, 1.3, 1.2))
            log(f"[bench]   d3q19 256^3 {dtype} MRT: {r['glups']:.2f} GLUPS "
                f"({r['frac_of_peak']:.3f})")
            variants.append(r)
        # sparse D3Q19: sphere packing at fluid fraction 0.4 in the dense, block-tiled and
        # node-list layouts, time per fluid node against the all-fluid dense step above
        m3 = synthetic.random_spheres3(256, 0.4)
        for dtype in ("f64", "f32"):
            for layout in ("dense_ab", "tiled16", "indirect"):
                r = measure_porous3(lbm, 256, 0.4, dtype, layout, args.steps // 2, args.warmup,
                                    m3, dense_ms_per_node=d3_ms_per_node[dtype])
                log(f"[bench]   d3q19 spheres 256^3 phi=0.4 {dtype} {layout}: "
                    f"{r['glups_per_fluid_node']:.2f} GLUPS/fluid, time per fluid node "
                    f"{r['time_per_fluid_node_over_dense_all_fluid']:.2f}x dense")
                variants.append(r)
        del m3
    if args.suite == "spheres3":
        c = measure_copy(lbm, 1 << 30, reps=args.copy_reps)
        log(f"[bench]   copy kernel: {c['gbps']:.0f} GB/s")
        variants.append({"workload": "copy kernel 1 GiB", **c})
    if args.suite in ("full", "spheres3"):
        for phi in (0.7, 0.4):
            m3 = synthetic.random_spheres3(256, phi)
            for dtype in ("f32", "f64"):
                for layout in ("dense_ab", "tiled16", "indirect"):
                    r = measure_porous3(lbm, 256, phi, dtype, layout, args.steps // 2,
                                        args.warmup, m3)
                    log(f"[bench]   d3q19 spheres 256^3 phi={phi} {dtype} {layout}: "
                        f"{r['glups_per_fluid_node']:.2f} GLUPS per fluid node "
                        f"({r['frac_of_peak']:.3f})")
                    variants.append(r)
    if args.suite == "full":
        for nn in (1024, 2048):
            f2 = synthetic.taylor_green(nn, 0.01)
            for dtype in ("f64", "f32"):
                for layout in ("dense_ab", "dense_aa"):
                    r = measure_dense(lbm, nn, dtype, layout, args.steps, args.warmup, f2)
                    log(f"[bench]   {nn} {dtype} {layout}: {r['glups']:.2f} GLUPS")
                    variants.append(r)
        mask_p, _ = synthetic.porous_discs(n, 0.5)
        for dtype in ("f32", "f64"):
            for layout in ("dense_ab", "indirect"):
                r = measure_porous(lbm, n, 0.5, dtype, layout, args.steps // 2, args.warmup // 2,
                                   mask_p, wall="fullway")
                log(f"[bench]   phi=0.5 full-way {dtype} {layout}: "
                    f"{r['glups_per_fluid_node']:.2f} GLUPS/fluid")
                variants.append(r)
        for r in measure_setup(lbm, mask_p):
            log(f"[bench]   create {r['layout']} porous {n}^2: {r['create_s']:.2f} s, "
                f"re-init {r['init_equilibrium_s'] * 1e3:.1f} ms")
            variants.append({"workload": f"setup porous discs {n}^2 phi=0.5", **r})
        v = measure_views(lbm, n, fields)
        log(f"[bench]   macroscopic {v['macroscopic_ms']:.3f} ms ({v['macroscopic_frac_of_peak']:.3f}), "
            f"mass {v['mass_ms_with_sync']:.3f} ms")
        variants.append(v)
        al = measure_adjoint_large(lbm, n)
        log(f"[bench]   adjoint {n}^2: {al['adjoint_ms_per_step'] * 1e3:.1f} us "
            f"({al['adjoint_frac_of_peak']:.3f}) vs forward {al['forward_ms_per_step'] * 1e3:.1f} us "
            f"({al['forward_frac_of_peak']:.3f}): {al['adjoint_over_forward']:.2f}x")
        variants.append(al)

    bpn = algorithmic_bytes_per_node("f64")
    bytes_per_launch = bpn * n * n
    achieved = bytes_per_launch / (head["ms_per_step"] / 1e3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBPS,
                "traffic": measured_traffic("k_step_dense_ab_f64_tgv4096"),
                "kernel": "k_step_dense_ab<F64>", "bytes_per_launch": bytes_per_launch,
                "bytes_per_node": bpn}
    cpu = None
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline(n, fields)
        log(f"[bench]   {cpu['value'] * 1e3:.1f} MLUPS on {cpu['cores']} threads")
    out = {
        "metric": METRIC, "value": head["glups"], "unit": "GLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"taylor-green vortex {n}x{n}, fully periodic, u0=0.01, "
                               f"tau=0.6, dense A-B layout, FP64 populations",
                   "nodes": n * n, "layout": "dense_ab", "tau": 0.6},
        "hbm_frac_of_peak": head["frac_of_peak"],
        "roofline": roofline, "cpu_baseline": cpu, "variants": variants,
        "paper_context": PAPER_CONTEXT,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
