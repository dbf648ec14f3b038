#!/usr/bin/env python3
"""Throughput of the scattered-field PIC step on one MI355X.

A step is one pass of the whole hot path over the full particle set: Yee
update of the scattered field, order-2 gather, closed-form incident field at
every particle, Boris push, Esirkepov deposition, Ampere update with Mur
edges (the tile sort amortized in).  The headline workload is the largest
single-GPU configuration, the 2D3V FP32 form: 4096 x 4096 cells at
lambda/48, 134M cold electrons (32 per cell) in the central 2048^2 cells at
0.02 n_c, a tightly focused radially polarized April beam (w0 = 0.8 lambda,
s = 10, a0 = 30) focused at the box centre, a 3000-step run; the same
workload in plain FP64 is timed beside it.  Further legs: the error of
both forms against the FP64 oracle in a window at the focus, the full
3000-step runs, the 2048 x 1024 FP64 LP run, the 1D run, the 3D step, the
256-member batched sweep and the served sweep.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("particle-pushes/sec (push+deposit+field) FP32 vs FP64 at stated "
          "error; sweep p50/p99")

# Algorithmic HBM bytes per particle push of a whole step: every live
# particle's mutable state read and written once (2 S_p) and 18 field words
# per grid cell (E and B read and written, J written and read), spread over
# the particles: 2 S_p + 18 S_w cells/particle.
#   4096^2 FP32 form: S_p = 24 (cell, two offsets, three momenta), S_w = 4,
#     1/8 cell per particle: 57 B;  the same in FP64: S_p = 40, S_w = 8: 98 B
#   2048 x 1024 FP64: 40 B and 1/8 cell per particle: 98 B
#   1D FP64: 32 B, 1/16 cell per particle: 73 B
#   sweep (FP32): 24 B, about 0.2 cell per particle: 62 B
BALG_RP4096_FP32 = 2 * 24 + 18 * 4 / 8
BALG_RP4096_FP64 = 2 * 40 + 18 * 8 / 8
BALG_LP2048_FP64 = 2 * 40 + 18 * 8 / 8
BALG_1D_FP64 = 2 * 32 + 18 * 8 / 16
# 3D push per particle at 2 ppc: read + write x, y, z, ux, uy, uz (96 B)
# and, per cell, 6 field components read and 3 current components read and
# written (96 B / 2)
PUSH3_BYTES = 96 + 48
PEAK_HBM_GBPS = 8000.0

TRAFFIC_FILES = {
    "fp32": os.path.join(ROOT, "profiles",
                         "push_tiled_f32_rp4096.traffic.txt"),
    "fp64": os.path.join(ROOT, "profiles",
                         "push_tiled_f64_rp4096.traffic.txt"),
}
KERNEL_SOURCES = ("sfpic_push.hip", "sfpic_common.h", "sfpic_device.h",
                  "sfpic_sim.h")
FIELD_COMPS = ("ex", "ey", "ez", "bx", "by", "bz")
G = 3

# The window of the focus error check: cells [c - 12, c + 12)^2 around the
# box centre c of the 4096^2 workload, checked after WINDOW_STEPS steps that
# start when the pulse peak reaches the focus; the oracle takes the
# particles of the window plus a halo of 5 WINDOW_STEPS + 3 cells.  Per
# step a change reaches at most 5 cells further: a particle gathers from
# nodes within 1.5 cells (B-bar through Faraday from half a cell more),
# moves less than a cell and deposits within 2.5 cells of its old position;
# so nothing outside the halo reaches the window in time.
WINDOW_HALF = 12
WINDOW_STEPS = 10
WINDOW_HALO = 5 * WINDOW_STEPS + 3


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2310_11393_amd", "csrc", f),
                  "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(tag):
    """HBM bytes per launch of the push from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, if the kernel sources are the ones
    that were profiled (else None)."""
    try:
        kv = dict(l.strip().split("=", 1) for l in open(TRAFFIC_FILES[tag])
                  if "=" in l)
        if kernel_sources_sha() != kv.get("sources_sha256"):
            return None
        return (float(kv["read_bytes_per_launch"]) +
                float(kv["write_bytes_per_launch"]))
    except (OSError, KeyError, ValueError):
        return None


def focus_window(work):
    """(cells of the window, cells of window + halo, first step): the window
    at the box centre, starting at the step where the pulse peak is at the
    focus."""
    c = work.grid.nx // 2
    w = (c - WINDOW_HALF, c + WINDOW_HALF)
    halo = (w[0] - WINDOW_HALO, w[1] + WINDOW_HALO)
    n0 = int(round(work.incident.t_focus / work.grid.dt))
    return w, halo, n0


def window_particle_ids(work, halo):
    """Ids of the generated particles whose cells lie in halo x halo (ids run
    over plasma rows, then columns, ppc consecutive per cell)."""
    import numpy as np
    sp = work.species[0]
    x0, x1, y0, y1 = sp.region
    ncx = x1 - x0
    rows = []
    for cy in range(max(halo[0], y0), min(halo[1], y1)):
        a = (cy - y0) * ncx + (max(halo[0], x0) - x0)
        b = (cy - y0) * ncx + (min(halo[1], x1) - x0)
        rows.append((a * sp.ppc, (b - a) * sp.ppc))
    return rows


# ---------------------------------------------------------------------------
# CPU legs (the oracle, test infrastructure): run in a child process next
# to the GPU legs; nothing here touches the GPU.
# ---------------------------------------------------------------------------

def _oracle_band_rate(work, rows, steps, warm):
    """Oracle step times over the full grid with the particles of `rows`
    plasma rows centred on the axis, and over the same grid with no
    particles: the particle rate and the field time per step."""
    import numpy as np
    import oracle
    from paper_2310_11393_amd import workloads as wl
    sp = work.species[0]
    x0, x1, y0, y1 = sp.region
    ncx = x1 - x0
    r0 = (y0 + y1) // 2 - rows // 2
    first, count = (r0 - y0) * ncx * sp.ppc, rows * ncx * sp.ppc
    cols = wl.generate_particles(sp, work.grid, first, count)
    vac = oracle.OracleSim(work.grid, work.incident)
    vac.step(warm)
    t = time.perf_counter()
    vac.step(steps)
    t_vac = (time.perf_counter() - t) / steps
    del vac
    sim = oracle.OracleSim(work.grid, work.incident)
    sim.add_species(sp.q, sp.m, sp.weight, *cols)
    del cols
    sim.step(warm)
    runs = []
    for _ in range(3):
        t = time.perf_counter()
        sim.step(steps)
        runs.append((time.perf_counter() - t) / steps)
    runs.sort()
    return count, runs[1], t_vac, r0


def _all_cores_worker(args):
    work_name, rows, offset, steps = args
    from paper_2310_11393_amd import workloads as wl
    import numpy as np
    import oracle
    work = getattr(wl, work_name)()
    sp = work.species[0]
    x0, x1, y0, y1 = sp.region
    ncx = x1 - x0
    r0 = (y0 + y1) // 2 - rows // 2 + offset
    first, count = (r0 - y0) * ncx * sp.ppc, rows * ncx * sp.ppc
    cols = wl.generate_particles(sp, work.grid, first, count)
    vac = oracle.OracleSim(work.grid, work.incident)
    vac.step(1)
    t = time.perf_counter()
    vac.step(steps)
    t_vac = time.perf_counter() - t
    del vac
    sim = oracle.OracleSim(work.grid, work.incident)
    sim.add_species(sp.q, sp.m, sp.weight, *cols)
    del cols
    sim.step(1)
    t = time.perf_counter()
    sim.step(steps)
    return count * steps, time.perf_counter() - t - t_vac


def cpu_legs(out_path, rows, steps, all_cores):
    """The oracle's timing on a bounded sample of the headline workload, its
    run of the focus window (for the error of the GPU forms) and its
    full-length 1D run."""
    import numpy as np
    import oracle
    from paper_2310_11393_amd import workloads as wl
    res = {}
    work = wl.rp_4096_fp32()
    n_full = work.species[0].count()
    t0 = time.perf_counter()
    count, t_band, t_vac, r0 = _oracle_band_rate(work, rows, steps, 1)
    rate = count / max(t_band - t_vac, 1e-9)
    t_full = t_vac + n_full / rate
    res["single"] = {
        "value": n_full / t_full, "unit": "particle-pushes/s", "cores": 1,
        "kind": "oracle",
        "sample": (f"4096x4096 grid with the {count} particles of plasma "
                   f"rows {r0}-{r0 + rows - 1}: one warm-up step, then the "
                   f"median of 3 runs of {steps} steps, {t_band:.2f} s per "
                   f"step; the same grid without particles {t_vac:.2f} s "
                   f"per step; value = the 134M-particle step these give, "
                   f"{t_full:.0f} s ({time.perf_counter() - t0:.0f} s of "
                   f"CPU work)"),
        "particle_rate": rate, "field_s_per_step": t_vac}
    # focus window: the oracle from the generated particles near the focus
    w, halo, n0 = focus_window(work)
    sp = work.species[0]
    parts = [wl.generate_particles(sp, work.grid, a, n) for a, n in
             window_particle_ids(work, halo)]
    cols = [np.concatenate([p[k] for p in parts]) for k in range(5)]
    sim = oracle.OracleSim(work.grid, work.incident)
    sim.add_species(sp.q, sp.m, sp.weight, *cols)
    sim.set_step_index(n0)
    t = time.perf_counter()
    sim.step(WINDOW_STEPS)
    sl = (slice(G + w[0], G + w[1]), slice(G + w[0], G + w[1]))
    win = {c: sim.field(c)[sl].copy() for c in FIELD_COMPS}
    del sim
    res["window"] = {"particles": len(cols[0]), "from_step": n0,
                     "steps": WINDOW_STEPS, "cells": list(w),
                     "s": time.perf_counter() - t}
    # 1D full length
    w1 = wl.plane_pulse_1d()
    sp1 = w1.species[0]
    o1 = oracle.OracleSim(w1.grid, w1.incident)
    o1.add_species(sp1.q, sp1.m, sp1.weight,
                   *wl.generate_particles(sp1, w1.grid))
    t = time.perf_counter()
    o1.step(w1.steps)
    t1 = time.perf_counter() - t
    f1 = {c: o1.field(c).copy() for c in FIELD_COMPS}
    res["pulse1d"] = {"steps": w1.steps, "s": t1,
                      "pushes_per_s": sp1.count() * w1.steps / t1}
    del o1
    # every core: independent oracle processes on disjoint bands
    if all_cores > 1:
        import multiprocessing as mp
        band = max(1, rows // 2)
        jobs = [("rp_4096_fp32", band, (k - all_cores // 2) * band, 2)
                for k in range(all_cores)]
        t = time.perf_counter()
        with mp.get_context("spawn").Pool(all_cores) as pool:
            out = pool.map(_all_cores_worker, jobs)
        rate_all = sum(o[0] / max(o[1], 1e-9) for o in out)
        res["all_cores"] = {
            "processes": all_cores, "cores": all_cores,
            "particle_rate": rate_all,
            "value": n_full / (t_vac + n_full / rate_all),
            "sample": (f"{all_cores} oracle processes at once, each the "
                       f"4096x4096 grid with {band} plasma rows of "
                       f"particles, 2 steps after one warm-up step, its "
                       f"field sweeps timed without particles and taken "
                       f"out; value = the 134M-particle step with the "
                       f"particle work over every process and one field "
                       f"sweep, {time.perf_counter() - t:.0f} s")}
    np.savez(out_path, **{f"win_{c}": v for c, v in win.items()},
             **{f"p1d_{c}": v for c, v in f1.items()})
    with open(out_path + ".json", "w") as f:
        json.dump(res, f)


def host_description():
    cpu = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "sched_cpus": len(os.sched_getaffinity(0)),
            "cpu_model": cpu}


# ---------------------------------------------------------------------------
# GPU legs
# ---------------------------------------------------------------------------

def run_steps(sim, steps, tag, chunks=5):
    """Run `steps` steps timed with events on the sim's stream (torch's
    current stream, which the library launches on)."""
    import torch
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    done, chunk = 0, max(1, steps // chunks)
    while done < steps:
        k = min(chunk, steps - done)
        sim.step(k)
        done += k
        if done < steps:
            sim.sync()
            log(f"{tag}: {done}/{steps} steps")
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1)


def timed_leg(work, precision, steps, warmup, balg, tag, kernel, traffic_tag,
              more_steps=0):
    """K steps after W warm-up steps with per-kernel HIP events, the
    roofline of the push from the algorithmic bytes per push, and
    optionally the rest of the run to `more_steps` steps in all."""
    from paper_2310_11393_amd.binding import Simulation
    log(f"{tag}: creating {work.species[0].count()} particles")
    sim = Simulation(work.grid, work.incident, species=work.species,
                     precision=precision)
    sim.step(warmup)
    sim.sync()
    n0 = sim.particle_count()
    sim.profile(True)
    ms = run_steps(sim, steps, tag)
    stats = sim.profile_read()
    sim.profile(False)
    n1 = sim.particle_count()
    pushes = steps * 0.5 * (n0 + n1)
    launches, push_ms = stats["push"]
    avg_s = push_ms / launches * 1e-3
    n_avg = 0.5 * (n0 + n1)
    achieved = balg * n_avg / avg_s / 1e9
    res = {"pushes_per_s": pushes / (ms * 1e-3), "ms_per_step": ms / steps,
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1),
                        "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                        "frac": round(achieved / PEAK_HBM_GBPS, 4),
                        "traffic": measured_traffic(traffic_tag),
                        "kernel": kernel,
                        "avg_launch_ms": round(avg_s * 1e3, 4),
                        "bytes_per_push": balg,
                        "pushes_per_launch": n_avg},
           "kernel_ms_per_step": {k: round(v[1] / steps, 4)
                                  for k, v in stats.items()}}
    log(f"{tag}: {steps} steps {ms:.1f} ms, {res['pushes_per_s'] / 1e9:.2f} "
        f"G pushes/s; push {avg_s * 1e3:.3f} ms = "
        f"{achieved:.0f} GB/s algorithmic")
    if more_steps > warmup + steps:
        rest = more_steps - warmup - steps
        sim.profile(True)
        ms2 = run_steps(sim, rest, tag + " run", chunks=10)
        st2 = sim.profile_read()
        sim.profile(False)
        n2 = sim.particle_count()
        d = sim.diagnostics()
        tot_ms = ms + ms2
        tot_p = pushes + rest * 0.5 * (n1 + n2)
        res["full_run"] = {
            "steps": steps + rest, "from_step": warmup,
            "pushes_per_s": tot_p / (tot_ms * 1e-3),
            "ms_per_step": tot_ms / (steps + rest),
            "push_avg_launch_ms": round(
                (push_ms + st2["push"][1]) /
                (launches + st2["push"][0]), 4),
            "kernel_ms_per_step": {
                k: round((stats[k][1] + v[1]) / (steps + rest), 4)
                for k, v in st2.items()},
            "n_alive_end": n2, "nonfinite": d["nonfinite"],
            "gauss_residual_rel": d["gauss_residual"] /
            max(d["rho_max"], 1e-300)}
        log(f"{tag}: run to step {more_steps}: "
            f"{res['full_run']['pushes_per_s'] / 1e9:.2f} G pushes/s")
    sim.close()
    return res


def window_fields(work, precision):
    """The GPU side of the focus-window check: the full workload from its
    generated particles, started at the step where the pulse reaches the
    focus, WINDOW_STEPS steps, the window's fields."""
    from paper_2310_11393_amd.binding import Simulation
    w, _halo, n0 = focus_window(work)
    sim = Simulation(work.grid, work.incident, species=work.species,
                     precision=precision)
    sim.set_step_index(n0)
    sim.step(WINDOW_STEPS)
    sl = (slice(G + w[0], G + w[1]), slice(G + w[0], G + w[1]))
    out = {c: sim.read_field(c)[sl].copy() for c in FIELD_COMPS}
    sim.close()
    return out


def rel_l2(a, b):
    import numpy as np
    num = sum(float(np.sum((a[c] - b[c]) ** 2)) for c in FIELD_COMPS)
    den = sum(float(np.sum(b[c] ** 2)) for c in FIELD_COMPS)
    return (num / den) ** 0.5 if den > 0 else None


def lp_2048(steps, warmup, on_nodes):
    """The 2048 x 1024 FP64 LP workload (16.8M electrons, 1 eV), its whole
    run; with on_nodes the incident field sampled on the Yee nodes."""
    from paper_2310_11393_amd import workloads as wl
    from paper_2310_11393_amd.binding import Simulation
    work = wl.lp_2048x1024()
    work.incident.on_nodes = int(on_nodes)
    tag = "LP 2048x1024" + (" on nodes" if on_nodes else "")
    sim = Simulation.from_workload(work)
    sim.step(warmup)
    n0 = sim.particle_count()
    sim.profile(True)
    ms = run_steps(sim, steps, tag)
    st = sim.profile_read()
    sim.profile(False)
    n1 = sim.particle_count()
    d = sim.diagnostics()
    fields = [sim.read_field(c) for c in FIELD_COMPS]
    sim.close()
    launches, push_ms = st["push"]
    avg_s = push_ms / launches * 1e-3
    n_avg = 0.5 * (n0 + n1)
    res = {"workload": ("2D3V FP64, 2048x1024 cells (lambda/32), 16.8M "
                        "electrons 16 ppc 1 eV at 0.05 n_c, April LP beam "
                        "w0=lambda s=20 a0=10" +
                        (", incident field on the Yee nodes" if on_nodes
                         else "")),
           "steps": steps, "from_step": warmup,
           "pushes_per_s": steps * n_avg / (ms * 1e-3),
           "ms_per_step": ms / steps,
           "push_avg_launch_ms": round(avg_s * 1e3, 4),
           "push_hbm_frac": round(BALG_LP2048_FP64 * n_avg / avg_s / 1e9 /
                                  PEAK_HBM_GBPS, 4),
           "kernel_ms_per_step": {k: round(v[1] / steps, 4)
                                  for k, v in st.items()},
           "gauss_residual_rel": d["gauss_residual"] / max(d["rho_max"],
                                                           1e-300),
           "nonfinite": d["nonfinite"]}
    log(f"{tag}: {res['pushes_per_s'] / 1e9:.2f} G pushes/s")
    return res, d, fields


def pulse_1d():
    """The 1D FP64 workload (2048 cells, 32768 electrons), its 2000 steps;
    the end fields for the comparison with the oracle's full run."""
    from paper_2310_11393_amd import workloads as wl
    from paper_2310_11393_amd.binding import Simulation
    work = wl.plane_pulse_1d()
    sim = Simulation.from_workload(work)
    n0 = sim.particle_count()
    ms = run_steps(sim, work.steps, "1D")
    n1 = sim.particle_count()
    f = {c: sim.read_field(c) for c in FIELD_COMPS}
    sim.close()
    n_avg = 0.5 * (n0 + n1)
    return {"workload": ("1D3V FP64, 2048 cells (lambda/32), 32768 cold "
                         "electrons 64 ppc at 0.01 n_c, plane pulse a0=1, "
                         "5 cycles"),
            "steps": work.steps, "pushes_per_s": work.steps * n_avg /
            (ms * 1e-3), "ms_per_step": ms / work.steps,
            "hbm_frac_whole_step": round(BALG_1D_FP64 * n_avg /
                                         (ms / work.steps * 1e-3) / 1e9 /
                                         PEAK_HBM_GBPS, 6)}, f


def three_d(steps=20, warmup=2, cells_per_lambda=16, ppc=2, precision=0):
    """The 3D3V step of Sec. 4 (sfpic3_*): the paper's 2 pi [24, 24, 32]
    box at Delta = 2 pi / cells_per_lambda (16: 512 x 384 x 384 cells; 32,
    the paper's own finer resolution: 1024 x 768 x 768 = 6.0e8 cells), cold
    electrons in the Sec. 3.1 density profile (0.31 n_c peak, ppc per cell
    there), tight April LP beam; FP64, or precision 1: fields and momenta
    stored as float, arithmetic FP64.  Host-timed around synchronized step
    batches (the leg runs for seconds)."""
    import torch
    from paper_2310_11393_amd import workloads as wl
    from paper_2310_11393_amd.binding import Simulation3
    g, sp, inc = wl.paper3d_lp(cells_per_lambda, ppc=ppc)
    n_sp = sp.count(g.dx)
    kind = "FP32 storage" if precision else "FP64"
    tag = f"3D 2pi/{cells_per_lambda} {kind}"
    log(f"{tag}: creating {n_sp / 1e6:.1f}M particles on "
        f"{g.nx}x{g.ny}x{g.nz} cells")
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    sim = Simulation3(g, inc, species=[sp], precision=precision)
    sim.step(warmup)
    sim.sync()
    n0 = sim.diagnostics()["n_alive"]
    torch.cuda.synchronize()
    t = time.perf_counter()
    done, chunk = 0, max(1, steps // 4)
    while done < steps:
        k = min(chunk, steps - done)
        sim.step(k)
        sim.sync()
        done += k
        log(f"{tag}: {done}/{steps} steps")
    sec = time.perf_counter() - t
    d = sim.diagnostics()
    sim.close()
    peak = torch.cuda.max_memory_allocated()
    torch.cuda.empty_cache()
    pushes = steps * 0.5 * (n0 + d["n_alive"])
    res = {"workload": (f"3D3V {kind}, {g.nx}x{g.ny}x{g.nz} cells "
                        f"(2 pi/{cells_per_lambda}), {n_sp / 1e6:.1f}M cold "
                        f"electrons, {ppc} ppc at the 0.31 n_c peak of the "
                        "order-12 super-Gaussian profile, April LP "
                        "w0=0.8 lambda s=20 a0=10"),
           "steps": steps, "pushes_per_s": pushes / sec,
           "ms_per_step": sec / steps * 1e3,
           "device_bytes": peak,
           "push_bytes_per_particle": PUSH3_BYTES,
           "gauss_residual_rel": d["gauss_residual"] / max(d["rho_max"],
                                                           1e-300),
           "nonfinite": d["nonfinite"]}
    log(f"{tag}: {res['pushes_per_s'] / 1e9:.2f} G pushes/s, "
        f"{res['ms_per_step']:.1f} ms/step, {peak / 1e9:.0f} GB")
    return res


def batched_sweep(members=256, steps=800, precision=None):
    """The laser-focus / density sweep as one batch: `members` FP32 (or, with
    precision FP64, plain FP64) 2D3V simulations (grid side 256..1024, 8..32
    ppc, LP / RP, density and beam drawn per member), `steps` steps each,
    tile and sort cadence from the autotuner."""
    from paper_2310_11393_amd import workloads as wl
    from paper_2310_11393_amd.binding import Batch
    if precision is None:
        precision = wl.FP32
    ms = [wl.sweep_member(i, precision=precision) for i in range(members)]
    npart = sum(w.species[0].count() for w in ms)
    kind = "FP32" if precision == wl.FP32 else "FP64"
    log(f"batched sweep ({kind}): {members} members, {npart / 1e6:.1f}M "
        f"particles, {steps} steps each")
    t0 = time.perf_counter()
    b = Batch(ms, nsteps=steps)
    t_create = time.perf_counter() - t0
    b.run()
    st = b.stats()
    failed = sum(1 for i in range(members) if b.result(i)["status"] != 0)
    b.close()
    g = st["groups"][0]
    rate = st["pushes"] / (st["step_ms"] * 1e-3)
    log(f"batched sweep ({kind}): {rate / 1e9:.2f} G pushes/s, tile {g['tile']}, "
        f"cadence {g['sort_every']}")
    return {"workload": (f"{members} {kind} 2D3V sweep members (side 256-1024 "
                         f"cells at lambda/32, 8-32 ppc, n 0.001-0.1 n_c, "
                         f"w0 0.6-2 lambda, a0 5-50, LP/RP), {steps} steps "
                         f"each"),
            "members": members, "particles": npart, "steps": steps,
            "pushes_per_s": rate, "step_ms": st["step_ms"],
            "run_ms": st["run_ms"], "create_s": t_create,
            "failed_members": failed,
            "tile": list(g["tile"]), "sort_every": g["sort_every"],
            "tuned": g["tuned"], "push_workgroups": g["push_workgroups"],
            "graph_launches": st["graph_launches"],
            "tuner_trials": [[list(t[0]), t[1], round(t[2], 4)]
                             for t in g["trials"]]}


def served_sweep(rate=20.0, window=60.0, steps=800, slots=64):
    """Poisson arrivals of sweep requests (10% at 2048^2 x 16 ppc) for
    `window` seconds at `rate` per second, served with continuous batching.
    When the arrivals stop the server is shut down: the percentiles of the
    completed requests are reported with the backlog left, and, for all
    requests, lower bounds of the percentiles that count every unfinished
    request at its age when the window closed."""
    import numpy as np
    from paper_2310_11393_amd import workloads as wl
    from paper_2310_11393_amd.binding import Server
    arrivals = wl.served_sweep(rate=rate, window=window, steps=steps)
    offered = sum(w.species[0].count() * w.steps for _, w in arrivals)
    log(f"served sweep: {len(arrivals)} requests over {window:.0f} s "
        f"(offered {offered / window / 1e9:.1f} G pushes/s), {slots} slots")
    srv = Server(max_slots=slots)
    t0 = time.perf_counter()
    tickets, t_sub = [], []
    last = t0
    backlog = []
    for t_arr, w in arrivals:
        delay = t0 + t_arr - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        t_sub.append(time.perf_counter() - t0)
        tickets.append(srv.submit(w))
        if time.perf_counter() - last > 10.0:
            last = time.perf_counter()
            st = srv.stats()
            backlog.append([round(last - t0, 1), st["queued"]])
            log(f"served sweep: t={last - t0:.0f} s submitted "
                f"{st['submitted']} done {st['completed']} running "
                f"{st['running']} queued {st['queued']}")
    rest = t0 + window - time.perf_counter()
    if rest > 0:
        time.sleep(rest)
    t_end = time.perf_counter() - t0
    st = srv.stats()
    backlog.append([round(t_end, 1), st["queued"]])
    ages = []
    for tk, ts in zip(tickets, t_sub):
        if srv.poll(tk) in (3, 4):  # done or failed
            r = srv.result(tk)
            ages.append(r["t_done"] - r["t_submit"])
        else:
            ages.append(t_end - ts)  # still waiting: a lower bound
    srv.close()
    lb = np.array(ages)
    out = {"workload": (f"Poisson arrivals {rate}/s for {window:.0f} s of "
                        f"FP32 sweep requests ({steps} steps; 10% at "
                        f"2048^2 x 16 ppc), {slots} resident slots"),
           "requests": len(arrivals), "completed": st["completed"],
           "failed": st["failed"], "running_at_end": st["running"],
           "queued_at_end": st["queued"],
           "queue_growth": backlog,
           "offered_pushes_per_s": offered / window,
           "pushes_per_s": st["pushes_per_s"],
           "pushes_per_s_wall": st["pushes"] / t_end,
           "p50_s_completed": st["p50_s"], "p99_s_completed": st["p99_s"],
           "p50_s_all_lower_bound": float(np.percentile(lb, 50)),
           "p99_s_all_lower_bound": float(np.percentile(lb, 99)),
           "stable": st["queued"] <= max(1, 0.05 * len(arrivals)),
           "max_resident": st["max_running"], "window_s": t_end,
           "peak_device_bytes": st["bytes_peak"]}
    if not out["stable"]:
        out["note"] = ("the offered load exceeds what one GPU serves: the "
                       "queue grows for the whole window, so time to result "
                       "is dominated by queueing; the completed-request "
                       "percentiles cover the early arrivals only")
    log(f"served sweep: completed {st['completed']} of {len(arrivals)}, "
        f"queue {st['queued']}, {st['pushes_per_s'] / 1e9:.2f} G pushes/s, "
        f"p50 {st['p50_s']:.1f} s (completed)")
    return out


def calibrate_copy():
    """A plain 1 GiB device-to-device copy, three times: the profiler's
    FETCH_SIZE / WRITE_SIZE of these launches scale the counters of the
    kernels to bytes."""
    import torch
    src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    return 1 << 30


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed FP32 and FP64 steps of the "
                         "4096^2 workload (profiling runs)")
    ap.add_argument("--full-steps", type=int, default=3000,
                    help="run both 4096^2 forms to this many steps (0: no)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=16)
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--cpu-all-cores", type=int, default=-1,
                    help="oracle processes for the every-core rate "
                         "(-1: the CPUs available, at most 16)")
    ap.add_argument("--cpu-legs", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--no-lp", action="store_true",
                    help="skip the 2048x1024 FP64 runs")
    ap.add_argument("--no-1d", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched sweep")
    ap.add_argument("--batch-members", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=800)
    ap.add_argument("--batch-fp64", action="store_true",
                    help="--only-batch: the sweep in plain FP64")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the served sweep")
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-window", type=float, default=60.0)
    ap.add_argument("--serve-steps", type=int, default=800)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--no-3d", action="store_true",
                    help="skip the 3D3V leg (sfpic3_*)")
    ap.add_argument("--steps-3d", type=int, default=20)
    ap.add_argument("--no-3d-paper", action="store_true",
                    help="skip the 3D leg at the paper's 2 pi/32 resolution")
    ap.add_argument("--only-3d", action="store_true",
                    help="only the FP64 3D3V leg at 2 pi/16 (profiling runs)")
    ap.add_argument("--only-serve", action="store_true",
                    help="only the served sweep (--serve-rate, --serve-window, "
                         "--serve-steps, --serve-slots; profiling runs)")
    ap.add_argument("--only-batch", action="store_true",
                    help="only the batched sweep (--batch-members, "
                         "--batch-steps; profiling runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy (3x) "
                         "whose profiler counters calibrate HBM traffic")
    args = ap.parse_args()
    if args.cpu_legs:
        cpu_legs(args.cpu_legs, args.cpu_rows, args.cpu_steps,
                 args.cpu_all_cores)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library runs a simulation "
              "on one GPU and has no path across GPUs (sweeps would place "
              "whole members per GPU, one large run would split into "
              "slabs); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    cpu = None
    tmp = tempfile.mkdtemp(prefix="sfpic_bench_")
    cpu_out = os.path.join(tmp, "oracle.npz")
    if not (args.no_cpu_baseline or args.headline_only):
        n_all = args.cpu_all_cores
        if n_all < 0:
            n_all = min(16, len(os.sched_getaffinity(0)))
        # the oracle legs run on the host next to the GPU legs
        cpu = subprocess.Popen(
            [sys.executable, os.path.abspath(__file__), "--cpu-legs",
             cpu_out, "--cpu-rows", str(args.cpu_rows), "--cpu-steps",
             str(args.cpu_steps), "--cpu-all-cores", str(n_all)],
            stdout=subprocess.DEVNULL)

    import numpy as np
    import torch
    from paper_2310_11393_amd import workloads as wl

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.only_serve:
        print(json.dumps({"served_sweep": served_sweep(
            args.serve_rate, args.serve_window, args.serve_steps,
            args.serve_slots)}), flush=True)
        return
    if args.only_batch:
        from paper_2310_11393_amd import workloads as wl
        prec = wl.FP64 if args.batch_fp64 else wl.FP32
        print(json.dumps({"batched_sweep": batched_sweep(
            args.batch_members, args.batch_steps, prec)}), flush=True)
        return
    if args.only_3d:
        res = {"three_d": three_d(steps=args.steps_3d, warmup=args.warmup)}
        if args.calibrate_copy:
            res["copy_calibration_bytes"] = calibrate_copy()
        print(json.dumps(res), flush=True)
        return
    work = wl.rp_4096_fp32()
    full = 0 if args.headline_only else args.full_steps
    f32 = timed_leg(work, wl.FP32, args.steps, args.warmup, BALG_RP4096_FP32,
                    "4096^2 RP FP32", "push_tiled<float,2>", "fp32", full)
    f64 = timed_leg(work, wl.FP64, args.steps, args.warmup, BALG_RP4096_FP64,
                    "4096^2 RP FP64", "push_tiled<double,2>", "fp64", full)
    value = f32["pushes_per_s"]
    out = {
        "metric": METRIC, "value": value, "unit": "particle-pushes/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": f32["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": ("2D3V FP32 form (int cell + FP32 offset, FP64 "
                                "incident-field phase) scattered-field PIC, "
                                "4096x4096 cells (lambda/48), 134M cold "
                                "electrons 32 ppc at 0.02 n_c in the central "
                                "2048^2, April RP beam w0=0.8 lambda s=10 "
                                "a0=30, 3000-step run"),
                   "grid": [work.grid.nx, work.grid.ny],
                   "particles": work.species[0].count(),
                   "precision": "fp32 form", "parallelism": "single GPU"},
        "roofline": f32["roofline"],
        "kernel_ms_per_step": f32["kernel_ms_per_step"],
        "fp64": {k: f64[k] for k in ("pushes_per_s", "ms_per_step",
                                     "roofline", "kernel_ms_per_step")},
        "fp32_over_fp64": value / f64["pushes_per_s"],
    }
    if full:
        out["full_run"] = {"fp32": f32.get("full_run"),
                           "fp64": f64.get("full_run")}
    if args.headline_only:
        if args.calibrate_copy:
            out["copy_calibration_bytes"] = calibrate_copy()
        print(json.dumps(out), flush=True)
        return
    win = {"fp32": window_fields(work, wl.FP32),
           "fp64": window_fields(work, wl.FP64)}
    log("focus window: GPU fields read")
    if not args.no_lp:
        res, d, ref = lp_2048(1500, args.warmup, False)
        out["lp_2048x1024_fp64"] = res
        res2, d2, f2 = lp_2048(1500, args.warmup, True)
        num = sum(float(np.sum((b - a) ** 2)) for a, b in zip(ref, f2))
        den = sum(float(np.sum(a ** 2)) for a in ref)
        res2["field_rel_l2_vs_closed_form"] = (num / den) ** 0.5
        res2["w_kin_rel_vs_closed_form"] = (d2["w_kin"] - d["w_kin"]) / \
            d["w_kin"]
        out["lp_2048x1024_incident_on_nodes"] = res2
        del ref, f2
    p1d = None
    if not args.no_1d:
        out["plane_pulse_1d"], p1d = pulse_1d()
    if not args.no_3d:
        legs = [("three_d", dict(steps=args.steps_3d)),
                ("three_d_fp32", dict(steps=args.steps_3d, precision=1))]
        if not args.no_3d_paper:
            legs.append(("three_d_paper_resolution",
                         dict(steps=max(2, args.steps_3d // 4),
                              cells_per_lambda=32, ppc=8, precision=1)))
        from paper_2310_11393_amd.binding import SfpicError
        for name, kw in legs:
            try:
                out[name] = three_d(**kw)
            except SfpicError as e:  # e.g. device memory taken by others
                log(f"{name}: {e}")
                out[name] = {"error": str(e)}
                torch.cuda.empty_cache()
    if not args.no_batch:
        out["batched_sweep"] = batched_sweep(args.batch_members,
                                             args.batch_steps)
        # the same sweep in plain FP64: the FP32 form's gain at batch scale
        out["batched_sweep_fp64"] = batched_sweep(args.batch_members,
                                                  args.batch_steps, wl.FP64)
        out["batched_fp32_over_fp64"] = (
            out["batched_sweep"]["pushes_per_s"] /
            out["batched_sweep_fp64"]["pushes_per_s"])
    if not args.no_serve:
        out["served_sweep"] = served_sweep(args.serve_rate,
                                           args.serve_window,
                                           args.serve_steps, args.serve_slots)
    if args.calibrate_copy:
        out["copy_calibration_bytes"] = calibrate_copy()
    if cpu is not None:
        log("waiting for the oracle legs on the host")
        rc = cpu.wait()
        if rc == 0:
            with open(cpu_out + ".json") as f:
                cres = json.load(f)
            arr = np.load(cpu_out)
            owin = {c: arr[f"win_{c}"] for c in FIELD_COMPS}
            base = dict(cres["single"])
            base["host"] = host_description()
            if "all_cores" in cres:
                base["all_cores"] = cres["all_cores"]
            out["cpu_baseline"] = base
            out["error_vs_oracle"] = {
                "fp32_field_rel_l2": rel_l2(win["fp32"], owin),
                "fp64_field_rel_l2": rel_l2(win["fp64"], owin),
                "window": (f"cells [{cres['window']['cells'][0]}, "
                           f"{cres['window']['cells'][1]})^2 at the focus, "
                           f"{WINDOW_STEPS} steps from step "
                           f"{cres['window']['from_step']} (pulse peak at "
                           f"the focus), oracle from the "
                           f"{cres['window']['particles']} particles within "
                           f"{WINDOW_HALO} cells of it")}
            if p1d is not None:
                o1 = {c: arr[f"p1d_{c}"] for c in FIELD_COMPS}
                out["plane_pulse_1d"]["field_rel_l2_vs_oracle_end"] = \
                    rel_l2(p1d, o1)
                out["plane_pulse_1d"]["oracle_pushes_per_s"] = \
                    cres["pulse1d"]["pushes_per_s"]
        else:
            out["cpu_baseline"] = {"error": f"oracle legs exited {rc}"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
