#!/usr/bin/env python3
"""Throughput of the scattered-field PIC step on one MI355X.

A step is one pass of the whole hot path over the full particle set: Yee
update of the scattered field, order-2 gather, closed-form incident field at
every particle, Boris push, Esirkepov deposition, Ampere update with Mur
edges.  The default workload is the 2D3V FP64 case: 2048 x 1024 cells at
lambda/32, 16.8M electrons (16 per cell, 1 eV) in the central 1024 x 1024
cells at 0.05 n_c, a tightly focused linearly polarized April beam (w0 =
lambda, s = 20, a0 = 10) focused at the box centre, 1500 steps.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("particle-pushes/sec (push+deposit+field) FP32 vs FP64 at stated "
          "error; sweep p50/p99")

# Algorithmic work of the push kernel per particle (2D3V, FP64, LP April
# field, closed-form branch), counting an FMA as two flops.
PUSH_BYTES_PARTICLE = 2 * 5 * 8     # read + write x, y, ux, uy, uz (double)
PUSH_BYTES_CELL = (6 + 3) * 8        # gather 6 field planes, deposit 3 planes
PUSH_FLOPS = 790                     # weights 36, gather 126, incident 317,
                                     # Boris 62, advance 16, shapes 60,
                                     # deposit 165, misc 8 (common path)
# 3D push as formulated, per particle: weights 42, gather 648 (6 x 27 taps),
# incident (April, full 3D) ~340, Boris and advance 79, shapes 165, Esirkepov
# 1650 (3 components x 25 transverse weights and 100 prefix terms)
PUSH3_FLOPS = 2924
# 3D: read + write x, y, z, ux, uy, uz (96 B) and, per cell at 2 ppc, 6 field
# components read and 3 current components read and written (96 B / 2)
PUSH3_BYTES = 96 + 48
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBPS = 8000.0


TRAFFIC_FILE = os.path.join(ROOT, "profiles",
                            "push_tiled_f64_lp2048x1024.traffic.txt")
KERNEL_SOURCES = ("sfpic_push.hip", "sfpic_common.h", "sfpic_device.h")


def measured_traffic():
    """HBM bytes per launch of the FP64 push from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, if the kernel sources are the ones
    that were profiled (else None)."""
    import hashlib
    try:
        kv = dict(l.strip().split("=", 1) for l in open(TRAFFIC_FILE)
                  if "=" in l)
        h = hashlib.sha256()
        for f in KERNEL_SOURCES:
            with open(os.path.join(ROOT, "paper_2310_11393_amd", "csrc", f),
                      "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() != kv.get("sources_sha256"):
            return None
        return (float(kv["read_bytes_per_launch"]) +
                float(kv["write_bytes_per_launch"]))
    except (OSError, KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(work, sample_rows=128, steps=3):
    """The FP64 oracle (single thread) on a bounded sample of the same
    workload: the full field grid with the particles of a band of
    `sample_rows` plasma rows centred on the beam axis, `steps` steps."""
    import numpy as np
    import oracle
    from paper_2310_11393_amd import workloads as wl
    sp = work.species[0]
    x0, x1, y0, y1 = sp.region
    mid = (y0 + y1) // 2
    r0 = mid - sample_rows // 2
    ncx = x1 - x0
    first = (r0 - y0) * ncx * sp.ppc
    count = sample_rows * ncx * sp.ppc
    x, y, ux, uy, uz = wl.generate_particles(sp, work.grid, first, count)
    sim = oracle.OracleSim(work.grid, work.incident)
    sim.add_species(sp.q, sp.m, sp.weight, x, y, ux, uy, uz)
    t0 = time.perf_counter()
    sim.step(steps)
    dt = time.perf_counter() - t0
    return {"value": count * steps / dt, "unit": "particle-pushes/s",
            "cores": 1, "kind": "oracle",
            "sample": (f"full {work.grid.nx}x{work.grid.ny} grid, "
                       f"{count} particles (plasma rows {r0}-"
                       f"{r0 + sample_rows - 1}), {steps} steps from t=0, "
                       f"{dt:.1f} s")}


def fp32_vs_fp64(steps=200, err_steps=50):
    """The 4096^2 RP workload (134M particles) in the FP32 form and in plain
    FP64, from the same seeded particles: throughput of each and the relative
    L2 difference of the scattered fields after `err_steps` steps."""
    import numpy as np
    import torch
    from paper_2310_11393_amd import workloads as wl
    from paper_2310_11393_amd.binding import Simulation
    work = wl.rp_4096_fp32()
    res = {"workload": ("2D3V 4096x4096 cells (lambda/48), 134M cold "
                        "electrons 32 ppc at 0.02 n_c, April RP beam "
                        "w0=0.8 lambda s=10 a0=30"),
           "steps": steps}
    fields = {}
    for prec, tag in ((wl.FP32, "fp32"), (wl.FP64, "fp64")):
        log(f"4096^2 RP {tag}: creating {work.species[0].count()} particles")
        sim = Simulation(work.grid, work.incident, species=work.species,
                         precision=prec)
        n0 = sim.particle_count()
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e2 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        sim.step(err_steps)
        e1.record(stream)
        torch.cuda.synchronize()
        fields[tag] = [sim.read_field(c) for c in
                       ("ex", "ey", "ez", "bx", "by", "bz")]
        sim.step(steps - err_steps)
        e2.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) + e1.elapsed_time(e2)
        n1 = sim.particle_count()
        res[tag + "_pushes_per_s"] = steps * 0.5 * (n0 + n1) / (ms * 1e-3)
        res[tag + "_ms_per_step"] = ms / steps
        log(f"4096^2 RP {tag}: {res[tag + '_pushes_per_s'] / 1e9:.2f} G "
            f"pushes/s")
        sim.close()
    num = sum(float(np.sum((a - b) ** 2)) for a, b in
              zip(fields["fp32"], fields["fp64"]))
    den = sum(float(np.sum(b ** 2)) for b in fields["fp64"])
    log(f"4096^2 RP: |F64|^2 = {den:.6e}, |F32 - F64|^2 = {num:.6e} after "
        f"{err_steps} steps")
    res["fp32_vs_fp64_field_rel_l2"] = (num / den) ** 0.5 if den > 0 else None
    res["error_after_steps"] = err_steps
    res["fp32_over_fp64"] = res["fp32_pushes_per_s"] / res["fp64_pushes_per_s"]
    return res


def incident_on_nodes(ref, steps, warmup):
    """The main workload with the incident field sampled on the Yee nodes at
    t^n and gathered with the scattered field (sfpic_incident.on_nodes)
    instead of evaluated in closed form at each particle: throughput, and
    how far its fields and energies end from the main run's after the same
    steps (the price of the O(dx^2) sampling)."""
    import numpy as np
    import torch
    from paper_2310_11393_amd import workloads as wl
    from paper_2310_11393_amd.binding import Simulation
    work = wl.lp_2048x1024()
    work.incident.on_nodes = 1
    log("incident on nodes: creating the same particles")
    sim = Simulation.from_workload(work)
    sim.step(warmup)
    sim.sync()
    n0 = sim.particle_count()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    done, chunk = 0, max(1, steps // 5)
    while done < steps:
        k = min(chunk, steps - done)
        sim.step(k)
        done += k
        sim.sync()
        log(f"incident on nodes: {done}/{steps} steps")
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    n1 = sim.particle_count()
    diag = sim.diagnostics()
    num = den = 0.0
    for c, a in zip(("ex", "ey", "ez", "bx", "by", "bz"), ref["fields"]):
        b = sim.read_field(c)
        num += float(np.sum((b - a) ** 2))
        den += float(np.sum(a ** 2))
    sim.close()
    rd = ref["diag"]
    res = {"workload": "the main workload with on_nodes = 1",
           "steps": steps,
           "pushes_per_s": steps * 0.5 * (n0 + n1) / (ms * 1e-3),
           "ms_per_step": ms / steps,
           "field_rel_l2_vs_main": (num / den) ** 0.5 if den > 0 else None,
           "w_kin_rel_vs_main": (diag["w_kin"] - rd["w_kin"]) / rd["w_kin"],
           "w_em_total_rel_vs_main": ((diag["w_em_total"] - rd["w_em_total"])
                                      / rd["w_em_total"])}
    log(f"incident on nodes: {res['pushes_per_s'] / 1e9:.2f} G pushes/s, "
        f"fields {res['field_rel_l2_vs_main']:.3e} from the main run")
    return res


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
           "push_flops_per_particle": PUSH3_FLOPS,
           "push_bytes_per_particle": PUSH3_BYTES,
           "gauss_residual_rel": d["gauss_residual"] / max(d["rho_max"],
                                                           1e-300),
           "nonfinite": d["nonfinite"]}
    log(f"{tag}: {res['pushes_per_s'] / 1e9:.2f} G pushes/s, "
        f"{res['ms_per_step']:.1f} ms/step, {peak / 1e9:.0f} GB")
    return res


def batched_sweep(members=256, steps=400):
    """The laser-focus / density sweep as one batch: `members` FP32 2D3V
    simulations (grid side 256..1024, 8..32 ppc, LP / RP, density and beam
    drawn per member), `steps` steps each, tile and sort cadence from the
    autotuner."""
    from paper_2310_11393_amd import workloads as wl
    from paper_2310_11393_amd.binding import Batch
    ms = [wl.sweep_member(i) for i in range(members)]
    npart = sum(w.species[0].count() for w in ms)
    log(f"batched sweep: {members} members, {npart / 1e6:.1f}M particles, "
        f"{steps} steps each")
    t0 = time.perf_counter()
    b = Batch(ms, nsteps=steps)
    t_create = time.perf_counter() - t0
    b.run()
    st = b.stats()
    b.close()
    g = st["groups"][0]
    rate = st["pushes"] / (st["step_ms"] * 1e-3)
    log(f"batched sweep: {rate / 1e9:.2f} G pushes/s, tile {g['tile']}, "
        f"cadence {g['sort_every']}")
    return {"workload": (f"{members} FP32 2D3V sweep members (side 256-1024 "
                         f"cells at lambda/32, 8-32 ppc, n 0.001-0.1 n_c, "
                         f"w0 0.6-2 lambda, a0 5-50, LP/RP), {steps} steps "
                         f"each"),
            "members": members, "particles": npart, "steps": steps,
            "pushes_per_s": rate, "step_ms": st["step_ms"],
            "run_ms": st["run_ms"], "create_s": t_create,
            "tile": list(g["tile"]), "sort_every": g["sort_every"],
            "tuned": g["tuned"], "push_workgroups": g["push_workgroups"],
            "graph_launches": st["graph_launches"],
            "tuner_trials": [[list(t[0]), t[1], round(t[2], 4)]
                             for t in g["trials"]]}


def served_sweep(rate=2.0, window=30.0, steps=800, slots=64):
    """Poisson arrivals of sweep requests (10% at 2048^2 x 16 ppc) for
    `window` seconds at `rate` per second, served with continuous batching;
    all arrivals are served to completion (none dropped)."""
    from paper_2310_11393_amd import workloads as wl
    from paper_2310_11393_amd.binding import Server
    arrivals = wl.served_sweep(rate=rate, window=window, steps=steps)
    offered = sum(w.species[0].count() * w.steps for _, w in arrivals)
    log(f"served sweep: {len(arrivals)} requests over {window:.0f} s "
        f"(offered {offered / window / 1e9:.1f} G pushes/s), {slots} slots")
    srv = Server(max_slots=slots)
    t0 = time.perf_counter()
    tickets = []
    last = t0
    for t_arr, w in arrivals:
        delay = t0 + t_arr - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        tickets.append(srv.submit(w))
        if time.perf_counter() - last > 10.0:
            last = time.perf_counter()
            st = srv.stats()
            log(f"served sweep: t={last - t0:.0f} s submitted "
                f"{st['submitted']} done {st['completed']} running "
                f"{st['running']} queued {st['queued']}")
    queued_at_window_end = srv.stats()["queued"]
    last = time.perf_counter()
    for tk in tickets:
        while True:
            try:
                srv.wait(tk, 5.0)
                break
            except Exception as e:  # still running
                if getattr(e, "code", 0) != -6:
                    raise
            if time.perf_counter() - last > 10.0:
                last = time.perf_counter()
                st = srv.stats()
                log(f"served sweep: draining, done {st['completed']}/"
                    f"{len(tickets)} running {st['running']} queued "
                    f"{st['queued']}")
        if time.perf_counter() - last > 10.0:
            last = time.perf_counter()
            st = srv.stats()
            log(f"served sweep: draining, done {st['completed']}/"
                f"{len(tickets)} running {st['running']} queued "
                f"{st['queued']}")
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    log(f"served sweep: p50 {st['p50_s']:.2f} s p99 {st['p99_s']:.2f} s, "
        f"{st['pushes_per_s'] / 1e9:.2f} G pushes/s")
    return {"workload": (f"Poisson arrivals {rate}/s for {window:.0f} s of "
                         f"FP32 sweep requests ({steps} steps; 10% at "
                         f"2048^2 x 16 ppc), {slots} resident slots"),
            "requests": len(arrivals), "completed": st["completed"],
            "failed": st["failed"],
            "offered_pushes_per_s": offered / window,
            "pushes_per_s": st["pushes_per_s"],
            "pushes_per_s_wall": st["pushes"] / wall,
            "p50_s": st["p50_s"], "p99_s": st["p99_s"],
            "mean_s": st["mean_s"], "max_s": st["max_s"],
            "queued_at_window_end": queued_at_window_end,
            # the queue keeps up with the arrivals when at most 5% of them
            # still wait for a slot as the arrivals stop (a backlog that grows
            # over the window leaves far more; the busy rate is not the
            # capacity: a lightly loaded server runs small batches)
            "stable": queued_at_window_end <= max(1, 0.05 * len(arrivals)),
            "max_resident": st["max_running"], "wall_s": wall,
            "peak_device_bytes": st["bytes_peak"]}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=128)
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--no-fp32-compare", action="store_true",
                    help="skip the 4096^2 FP32-form vs FP64 comparison")
    ap.add_argument("--compare-steps", type=int, default=200)
    ap.add_argument("--no-on-nodes", action="store_true",
                    help="skip the run with the incident field sampled on "
                         "the Yee nodes")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched sweep")
    ap.add_argument("--batch-members", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=400)
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the served sweep")
    ap.add_argument("--serve-rate", type=float, default=2.0)
    ap.add_argument("--serve-window", type=float, default=30.0)
    ap.add_argument("--serve-steps", type=int, default=800)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--no-3d", action="store_true",
                    help="skip the 3D3V leg (sfpic3_*)")
    ap.add_argument("--steps-3d", type=int, default=20)
    ap.add_argument("--no-3d-paper", action="store_true",
                    help="skip the 3D leg at the paper's 2 pi/32 resolution")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy (3x) "
                         "whose profiler counters calibrate HBM traffic")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library runs a simulation "
              "on one GPU and has no path across GPUs (sweeps would place "
              "whole members per GPU, one large run would split into "
              "slabs); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2310_11393_amd import workloads as wl
    from paper_2310_11393_amd.binding import Simulation

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    work = wl.lp_2048x1024()
    log(f"workload {work.name}: creating {work.species[0].count()} particles")
    sim = Simulation.from_workload(work)
    sim.step(args.warmup)
    sim.sync()
    log(f"warmup {args.warmup} steps done")
    n0 = sim.particle_count()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    sim.profile(True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    ev0.record(stream)
    done = 0
    chunk = max(1, args.steps // 10)
    while done < args.steps:
        k = min(chunk, args.steps - done)
        sim.step(k)
        done += k
        if done < args.steps:
            sim.sync()
            log(f"{done}/{args.steps} steps")
    ev1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms = ev0.elapsed_time(ev1)
    stats = sim.profile_read()
    sim.profile(False)
    n1 = sim.particle_count()
    diag = sim.diagnostics()
    pushes = args.steps * 0.5 * (n0 + n1)
    value = pushes / (ms * 1e-3)
    log(f"{args.steps} steps in {ms:.1f} ms (wall {t_wall:.2f} s): "
        f"{value / 1e9:.2f} G pushes/s; kernels {stats}")

    # dominant kernel: the particle push
    launches, push_ms = stats["push"]
    avg_s = push_ms / launches * 1e-3
    n_avg = 0.5 * (n0 + n1)
    plasma_cells = n_avg / work.species[0].ppc
    flops = n_avg * PUSH_FLOPS
    bytes_ = n_avg * PUSH_BYTES_PARTICLE + plasma_cells * PUSH_BYTES_CELL
    achieved = flops / avg_s / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3),
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                "traffic": measured_traffic(),
                "kernel": "push_tiled_f64<2>",
                "avg_launch_ms": round(avg_s * 1e3, 4),
                "hbm_achieved_GBps": round(bytes_ / avg_s / 1e9, 1),
                "hbm_frac": round(bytes_ / avg_s / 1e9 / PEAK_HBM_GBPS, 4)}
    out = {
        "metric": METRIC, "value": value, "unit": "particle-pushes/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": ("2D3V FP64 scattered-field PIC, 2048x1024 "
                                "cells (lambda/32), 16.8M electrons 16 ppc "
                                "1 eV at 0.05 n_c, April LP beam w0=lambda "
                                "s=20 a0=10, 1500-step run"),
                   "grid": [work.grid.nx, work.grid.ny],
                   "particles": work.species[0].count(),
                   "precision": "fp64", "parallelism": "single GPU"},
        "roofline": roofline,
        "kernel_ms_per_step": {k: round(v[1] / max(v[0], 1), 4) * (
            v[0] / args.steps) for k, v in stats.items()},
        "checks": {"gauss_residual_rel": diag["gauss_residual"] /
                   max(diag["rho_max"], 1e-300),
                   "nonfinite": diag["nonfinite"], "n_alive": diag["n_alive"]},
    }
    ref = None
    if not args.no_on_nodes:
        ref = {"diag": diag, "fields": [sim.read_field(c) for c in
                                        ("ex", "ey", "ez", "bx", "by",
                                         "bz")]}
    sim.close()
    if ref is not None:
        out["incident_on_nodes"] = incident_on_nodes(ref, args.steps,
                                                     args.warmup)
        del ref
    if not args.no_fp32_compare:
        out["fp32_vs_fp64"] = fp32_vs_fp64(args.compare_steps)
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
    if not args.no_serve:
        out["served_sweep"] = served_sweep(args.serve_rate,
                                           args.serve_window,
                                           args.serve_steps, args.serve_slots)
    if args.calibrate_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 1 << 30
        del src, dst
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample (CPU)")
        out["cpu_baseline"] = cpu_baseline(work, args.cpu_rows,
                                           args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
