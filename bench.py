#!/usr/bin/env python3
"""Benchmark: coupled Mcell-steps/s of the MI355X EM-thermal-mechanical path.

Headline workload: the full-scale one-GPU package, 1024 x 1024 x 128 uniform
1 um cells (134 M cells; Cu ground, BT substrate, 64 x 64 Cu bumps in
underfill, Si interposer with TSVs, polyimide RDL with 8 routing layers of
512 traces, two Si dies, air), every trace driven by its own seeded 256-bit
PRBS-7 burst at 16 EM steps per bit, EM step at CFL 0.9, R = 256 EM steps
per thermal step.

One bench step = one coupling block: 256 EM steps (EM update of Eq. 2-3 with
sigma(T) of Eq. 6, Joule source) and one thermal step (Eq. 4-5).  `value` =
cells * 256 * steps / wall time of the timed blocks (mechanics excluded,
inputs resident in HBM); the headline runs the mixed path (FP32 fields,
FP64 temperature / Joule / CG refinement), and the same blocks are timed on
the FP64 path beside it.  After the timed blocks each precision solves the
thermoelastic system once (Eq. 8, multigrid-preconditioned CG, rtol 1e-8)
and evaluates von Mises (Eq. 9); the solve time, CG DOF-iterations/s and the
mixed-vs-FP64 differences of the temperature rise and the peak von Mises
stress are reported beside the headline.

The roofline of the dominant kernel (the EM march) uses the compulsory bytes
per cell-step of the method (mixed 69 B: e-state 48, material 1, FP32
temperature 4, Joule read-modify-write 16; FP64 97 B: e-state 72, material
1, temperature 8, Joule 16), times the cells of one launch, over the mean
launch time from HIP events recorded on the plan's stream around the EM
launches of every timed block.  Beside it: the same figure on the
implementation's own bytes (mixed 87 B with the leapfrog face field, the e
residual and the sigma-change correction), the counted HBM traffic from the
committed rocprofv3 counter summary (when it was taken on the current
source), and the bandwidth a plain device copy reaches.

Further legs (on by default; --legs selects):
  slice      the 256x256x64 graded slice with a warm-started mechanical solve
             after every thermal step (R = 200), mixed and FP64: coupled rate
             with mechanics, march rate, the mechanical tail per block and
             CG DOF-iterations/s;
  r1         the package at the paper's synchronous schedule R = 1 (a thermal
             step and a conductivity refresh after every EM step);
  temporal   the package with the two-step slab wavefront over 8 z-slabs;
  excitation the package under the excitation scheme of Sec. III-B (52,640
             port edges, closed-form waves sampled on the device);
  batch      64 design variants of uneven size, one batched mixed run against
             64 sequential FP64 runs and a batched FP64 run;
  serve      Poisson arrivals through the continuous-batching server, mixed
             and FP64 (--serve-rates, --serve-requests, --serve-precisions;
             --serve-only runs this leg alone, e.g. the sweep of 256 requests
             at 2, 5, 10 and 20 req/s);
  cpu        the FP64 oracle on the host cores: a bounded window of the
             package (one EM step, Joule and a thermal step), a sample of the
             slice with its thermal step, the full 32x32x16 trace case, the
             oracle's CG DOF-iterations/s on the 32x32x16 case, and one
             application of the slice's stiffness (its Jacobi-PCG rate without
             the element cache).

    python bench.py [--steps K] [--warmup W] [--legs headline,slice,...] [--no-cpu]
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
# Compulsory bytes per cell-step of the coupled march (one cell ~ one node +
# three edges): the method's own state, read and written once per step.
BYTES_PER_CELL_STEP = {"fp64": 97.0, "mixed": 69.0}
# Bytes per cell-step the implementation moves by design: the mixed path
# marches the leapfrog form (face field h in FP32, read + written: 24 B more
# than an increment form), with the 8-bit e residual (6 B) and the
# sigma-change correction K (12 B) that keep it inside the temperature bar;
# an increment form would need 48 B of e-state, this one 24 + 24.
DESIGN_BYTES_PER_CELL_STEP = {"fp64": 97.0, "mixed": 87.0}
KERNEL = {"mixed": "em_march_kernel<float, true>", "fp64": "em_march_kernel<double, false>"}
DEFAULT_LEGS = "headline,slice,r1,temporal,excitation,batch,serve,cpu"
PROFILE_EM = {"mixed": "profiles/em_march_package1024x1024x128_mixed.md",
              "fp64": "profiles/em_march_package1024x1024x128_fp64.md"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed coupling blocks of 256 EM steps")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--legs", default=DEFAULT_LEGS)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle legs")
    ap.add_argument("--batch-variants", type=int, default=64)
    ap.add_argument("--serve-requests", type=int, default=32)
    ap.add_argument("--serve-rates", default="2")
    ap.add_argument("--serve-precisions", default="mixed,fp64")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving leg (a rate sweep) and print its JSON line")
    ap.add_argument("--probe", choices=["em", "em-fp64", "em-slice", "em-slice-fp64", "em-slice-pairs3",
                                        "em-slice-pairs8", "mech", "mech-tail", "copy", "r1", "r1-fp64"],
                    default=None,
                    help="short runs for hardware-counter profiles: 8 EM steps of the package (em, em-fp64) or the "
                         "slice (em-slice, em-slice-fp64; em-slice-pairsS: as 4 slab pairs over S z-slabs), the "
                         "slice's serial block tail after 6 warm blocks, 3 times (mech-tail), 8 coupled steps of the package at R = 1 (r1, r1-fp64), two slice "
                         "coupling blocks with their mechanical solves (mech), or a plain 2 GiB device copy (the "
                         "calibration kernel for FETCH_SIZE / WRITE_SIZE)")
    return ap.parse_args()


def say(*a):
    print(*a, file=sys.stderr, flush=True)


# ---- probes for counter runs ---------------------------------------------------
def probe(kind):
    import torch
    if kind == "copy":
        x = torch.ones(1 << 28, dtype=torch.float64, device="cuda")  # 2 GiB
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"probe": "copy", "bytes_read_per_launch": x.numel() * 8,
                          "bytes_written_per_launch": x.numel() * 8}))
        return
    import workloads as W
    import paper_2603_07038_amd as etm
    if kind == "mech-tail":
        prob = W.config2()
        dt = etm.cfl_dt(prob)
        R = prob.em_per_thermal
        J = prob.sample_J_half(dt, prob.n_em_steps)
        plan = etm.Plan(prob, J, dt=dt, precision=etm.ETM_PREC_MIXED, n_steps=prob.n_em_steps, history=False)
        plan.advance(6 * R)
        plan.sync()
        tails = []
        for _ in range(3):
            plan.advance(R - 1)
            plan.sync()
            t = time.perf_counter()
            plan.advance(1)      # last EM step, thermal step, solve, von Mises
            info = plan.sync()
            tails.append({"ms": round((time.perf_counter() - t) * 1e3, 2), "cg_iters": info["cg_iters"],
                          "cg_outer": info["cg_outer"]})
        print(json.dumps({"probe": kind, "workload": prob.name, "cells": prob.n_cells, "tails": tails}))
        return
    if kind == "mech":
        prob = W.config2()
        dt = etm.cfl_dt(prob)
        R = prob.em_per_thermal
        J = prob.sample_J_half(dt, 2 * R + 2)
        plan = etm.Plan(prob, J, dt=dt, precision=etm.ETM_PREC_MIXED, n_steps=2 * R + 2, history=False)
        plan.advance(2 * R)
        info = plan.sync()
        print(json.dumps({"probe": kind, "workload": prob.name, "cells": prob.n_cells, "em_steps": 2 * R,
                          "mech_solves": info["n_solves"], "cg_iters_total": info["cg_iters_total"]}))
        return
    prob = W.config2() if kind.startswith("em-slice") else W.config3()
    prob.mech_every_thermal = 0
    prob.em_per_thermal = 1 if kind.startswith("r1") else 100000  # else no thermal step inside the probe
    prob.history_stride = 0
    dt = etm.cfl_dt(prob)
    J = prob.sample_J_half(dt, 16)
    prec = etm.ETM_PREC_FP64 if kind.endswith("fp64") else etm.ETM_PREC_MIXED
    slabs = int(kind[len("em-slice-pairs"):]) if kind.startswith("em-slice-pairs") else 0
    plan = etm.Plan(prob, J, dt=dt, precision=prec, n_steps=16, history=False, em_slabs=slabs)
    plan.advance(8)
    plan.sync()
    print(json.dumps({"probe": kind, "workload": prob.name, "cells": prob.n_cells, "em_steps": 8}))


def measured_traffic(prec_name):
    """HBM bytes per launch of the EM march from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the copy-kernel calibration);
    None when no summary exists or the kernel source changed since it was taken."""
    rel = PROFILE_EM.get(prec_name)
    if rel is None or not os.path.exists(os.path.join(ROOT, rel)):
        return None
    fields = {}
    for line in open(os.path.join(ROOT, rel)):
        if ":" in line and line.split(":")[0].strip() in ("traffic_bytes_per_launch", "traffic_source_sha256_16"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_2603_07038_amd", "csrc", "em.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if fields.get("traffic_source_sha256_16") != sha or "traffic_bytes_per_launch" not in fields:
        return None
    return int(fields["traffic_bytes_per_launch"])


def copy_ceiling():
    """Achievable HBM bandwidth of a plain device copy (2 GiB read + 2 GiB
    written per launch), from HIP events: the second ceiling of the march."""
    import torch
    x = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n = 10
    e0.record()
    for _ in range(n):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / n
    gbs = 2 * x.numel() * 8 / t / 1e9
    del x, y
    torch.cuda.empty_cache()
    return {"GBs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
            "kernel": "torch copy_, 2 GiB read + 2 GiB written", "launch_us": round(t * 1e6, 1)}


# ---- the headline: coupled blocks of the package, mixed and FP64 -----------------
def march_blocks(prob, J, dt, prec_name, steps, warmup):
    """W untimed + K timed coupling blocks of one precision, then one
    mechanical solve; returns timings, the temperature and von Mises fields."""
    import torch
    import paper_2603_07038_amd as etm
    prec = etm.ETM_PREC_MIXED if prec_name == "mixed" else etm.ETM_PREC_FP64
    R = prob.em_per_thermal
    plan = etm.Plan(prob, J, dt=dt, precision=prec, n_steps=R * (steps + warmup), history=False, cg_maxit=3000)
    stream = plan.stream
    for _ in range(warmup):
        plan.advance(R)
    plan.sync()
    # Each timed block is issued as R - 1 EM steps and the last step with its
    # thermal step; events on the plan's stream bracket the EM launches.
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in range(steps):
        ev[b][0].record(stream)
        plan.advance(R - 1)
        ev[b][1].record(stream)
        plan.advance(1)
    info = plan.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    em_s = sum(a.elapsed_time(b) for a, b in ev) / 1e3
    launch_s = em_s / (steps * (R - 1))
    cells = prob.n_cells
    # one mechanical solve at the temperature reached, cold start: enqueued,
    # then waited for by etm_sync (wall clock around both)
    _, _, mech_dofs = plan.dofs()
    torch.cuda.synchronize()
    tm = time.perf_counter()
    plan.mech_solve()
    minfo = plan.sync(raise_on_error=False)
    torch.cuda.synchronize()
    mech_wall = time.perf_counter() - tm
    if minfo["status"] != etm.ETM_OK:  # reported, not fatal: the march figures stand
        say(f"[bench] {prec_name} mechanical solve: status {minfo['status']}")
    theta = plan.read(etm.ETM_FIELD_THETA)
    vm = plan.read(etm.ETM_FIELD_VM)
    bpc, dbc = BYTES_PER_CELL_STEP[prec_name], DESIGN_BYTES_PER_CELL_STEP[prec_name]
    achieved = bpc * cells / launch_s / 1e9
    res = {
        "value": cells * R * steps / wall / 1e6,
        "ms_per_step": wall / steps * 1e3,
        "em_kernel_us": launch_s * 1e6,
        "march_only_mcell_steps_per_s": cells / launch_s / 1e6,
        "theta_max": info["theta_max"],
        "em_steps": info["step"],
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(prec_name),
                     "traffic_unit": "bytes/launch", "kernel": KERNEL[prec_name],
                     "bytes_per_cell_step": bpc, "cells_per_launch": cells,
                     "algorithmic_bytes_per_launch": int(bpc * cells), "launch_us": round(launch_s * 1e6, 2),
                     "design_bytes_per_cell_step": dbc,
                     "design_frac": round(dbc * cells / launch_s / 1e9 / HBM_PEAK_GBS, 4)},
        "mechanics": {"solve_s_wall": round(mech_wall, 3), "status": minfo["status"],
                      "cg_iters": minfo["cg_iters"], "cg_outer": minfo["cg_outer"], "mg_levels": minfo["mg_levels"],
                      "cg_relres": minfo["cg_relres"], "dofs": mech_dofs,
                      "cg_dof_iter_per_s": mech_dofs * minfo["cg_iters"] / mech_wall if minfo["cg_iters"] else None,
                      "note": "one cold-started solve, setup of the multigrid hierarchy included"},
    }
    del plan
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res, theta, vm


def headline(steps, warmup):
    import numpy as np
    import workloads as W
    import paper_2603_07038_amd as etm
    prob = W.config3()
    prob.history_stride = 0
    prob.mech_every_thermal = 0
    dt = etm.cfl_dt(prob)
    R = prob.em_per_thermal
    J = prob.sample_J_half(dt, prob.n_em_steps)
    say(f"[bench] headline {prob.name} mixed: {warmup} + {steps} blocks of {R} EM steps")
    mixed, tm, vm_m = march_blocks(prob, J, dt, "mixed", steps, warmup)
    say(f"[bench] headline mixed {mixed['value']:.1f} Mcell-steps/s; FP64 next")
    fp64, tf, vm_f = march_blocks(prob, J, dt, "fp64", steps, warmup)
    say(f"[bench] headline fp64 {fp64['value']:.1f} Mcell-steps/s")
    cmp = {"theta_rel_err": float(np.abs(tm - tf).max() / max(np.abs(tf).max(), 1e-300)),
           "theta_max_K": float(tf.max()),
           "peak_vm_rel_err": abs(float(vm_m.max()) - float(vm_f.max())) / max(float(vm_f.max()), 1e-300),
           "vm_field_rel_err": float(np.abs(vm_m - vm_f).max() / max(float(vm_f.max()), 1e-300)),
           "peak_vm_Pa": float(vm_f.max()), "after_em_steps": (steps + warmup) * R,
           "targets": {"theta": 1e-6, "peak_vm": 1e-5}}
    return prob, dt, mixed, fp64, cmp


# ---- the slice with a mechanical solve after every thermal step -----------------
def slice_leg(steps=3, warmup=1, tail_blocks=5):
    import torch
    import workloads as W
    import paper_2603_07038_amd as etm
    prob = W.config2()
    dt = etm.cfl_dt(prob)
    R = prob.em_per_thermal
    J = prob.sample_J_half(dt, prob.n_em_steps)
    out = {"workload": prob.name, "cells": prob.n_cells, "em_steps_per_block": R, "mech_solve_per_block": True,
           "cg_rtol": prob.cg_rtol}
    for name, prec in (("mixed", etm.ETM_PREC_MIXED), ("fp64", etm.ETM_PREC_FP64)):
        plan = etm.Plan(prob, J, dt=dt, precision=prec, n_steps=prob.n_em_steps)
        stream = plan.stream
        for _ in range(warmup):
            plan.advance(R)
        i0 = plan.sync()
        # blocks in parts: the march (R - 1 steps) and the tail (last EM step,
        # thermal step, mechanical solve and von Mises; a solve that ends an
        # advance call runs without overlap)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(tail_blocks)]
        tail_ms = 0.0
        for e in ev:
            e[0].record(stream)
            plan.advance(R - 1)
            e[1].record(stream)
            plan.sync()
            t = time.perf_counter()
            plan.advance(1)   # the solve runs on the plan's side stream: wall clock up to etm_sync
            plan.sync()
            tail_ms += (time.perf_counter() - t) * 1e3
        i1 = plan.sync()
        torch.cuda.synchronize()
        em_ms = sum(e[0].elapsed_time(e[1]) for e in ev)
        split_iters = i1["cg_iters_total"] - i0["cg_iters_total"]
        # whole blocks in one call: each solve overlaps the next block's EM steps
        torch.cuda.synchronize()
        t = time.perf_counter()
        plan.advance(R * steps)
        plan.sync()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        _, _, dofs = plan.dofs()
        out[name] = {"coupled_with_mechanics_mcell_steps_per_s": round(prob.n_cells * R * steps / wall / 1e6, 1),
                     "ms_per_block": round(wall / steps * 1e3, 2),
                     "march_mcell_steps_per_s": round(prob.n_cells * (R - 1) * tail_blocks / (em_ms / 1e3) / 1e6, 1),
                     "em_kernel_us": round(em_ms * 1e3 / (tail_blocks * (R - 1)), 2),
                     "mech_tail_ms_per_block": round(tail_ms / tail_blocks, 2),
                     "cg_iters_per_block": split_iters / tail_blocks,
                     "cg_dof_iter_per_s": dofs * split_iters / (tail_ms / 1e3) if split_iters else None}
        del plan
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out


def r1_leg(steps=16, warmup=2):
    """The package at R = 1 (the paper's schedule: thermal step and
    conductivity refresh after every EM step) against its EM-only step."""
    import torch
    import workloads as W
    import paper_2603_07038_amd as etm
    prob = W.config3()
    prob.history_stride = 0
    prob.em_per_thermal = 1
    dt = etm.cfl_dt(prob)
    J = prob.sample_J_half(dt, steps + warmup + 1)
    out = {"workload": prob.name, "cells": prob.n_cells, "em_steps": steps}
    for name, prec in (("mixed", etm.ETM_PREC_MIXED), ("fp64", etm.ETM_PREC_FP64)):
        plan = etm.Plan(prob, J, dt=dt, precision=prec, n_steps=steps + warmup, history=False)
        plan.advance(warmup)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(plan.stream)
        plan.advance(steps)
        e1.record(plan.stream)
        plan.sync()
        t = e0.elapsed_time(e1) / 1e3 / steps
        out[name] = {"us_per_coupled_step": round(t * 1e6, 1), "mcell_steps_per_s": round(prob.n_cells / t / 1e6, 1)}
        del plan
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out


def temporal_leg(steps=32, warmup=4, slabs=8):
    """The package's EM march with the two-step slab wavefront (em_slabs = S)."""
    import torch
    import workloads as W
    import paper_2603_07038_amd as etm
    prob = W.config3()
    prob.history_stride = 0
    prob.em_per_thermal = 100000
    dt = etm.cfl_dt(prob)
    J = prob.sample_J_half(dt, steps + warmup + 2)
    plan = etm.Plan(prob, J, dt=dt, precision=etm.ETM_PREC_MIXED, n_steps=steps + warmup + 2, history=False,
                    em_slabs=slabs)
    plan.advance(warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(plan.stream)
    plan.advance(steps)
    e1.record(plan.stream)
    plan.sync()
    t = e0.elapsed_time(e1) / 1e3 / steps
    del plan
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return {"workload": prob.name, "em_slabs": slabs, "us_per_em_step": round(t * 1e6, 1),
            "mcell_steps_per_s": round(prob.n_cells / t / 1e6, 1),
            "frac_of_hbm_peak_69B": round(69.0 * prob.n_cells / t / 1e9 / HBM_PEAK_GBS, 4)}


def excitation_leg(steps=128, warmup=8, t_origin=95e-12):
    """The package under the excitation scheme of Sec. III-B (one closed-form
    wave per port, sampled on the device in blocks of steps), mixed precision,
    in a window where the 5 GHz sine and the 40 GHz burst are on."""
    import torch
    import workloads as W
    import paper_2603_07038_amd as etm
    prob = W.config3(excitation="paper", t_origin=t_origin)
    prob.history_stride = 0
    dt = etm.cfl_dt(prob)
    plan = etm.Plan(prob, None, dt=dt, precision=etm.ETM_PREC_MIXED, n_steps=steps + warmup, history=False,
                    device_waves=True)
    plan.advance(warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(plan.stream)
    plan.advance(steps)
    e1.record(plan.stream)
    info = plan.sync()
    t = e0.elapsed_time(e1) / 1e3 / steps
    window_steps = int(round(300e-12 / dt))
    out = {"workload": prob.name, "cells": prob.n_cells, "port_edges": prob.n_ports, "waves": len(prob.waves),
           "t_origin_s": t_origin, "em_steps": steps, "march_mcell_steps_per_s": round(prob.n_cells / t / 1e6, 1),
           "em_step_us": round(t * 1e6, 1), "theta_max_K": info["theta_max"],
           "host_table_bytes_avoided_300ps": len(prob.waves) * (window_steps + 1) * 8}
    del plan
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def batch_leg(n_variants):
    """The 64-variant batch: batched mixed vs sequential FP64 (and batched FP64)."""
    import numpy as np
    import torch
    import workloads as W
    import paper_2603_07038_amd as etm
    probs = [W.config4_variant(v) for v in range(n_variants)]
    dts = [etm.cfl_dt(p) for p in probs]
    Js = [p.sample_J_half(dt, p.n_em_steps) for p, dt in zip(probs, dts)]
    steps = probs[0].n_em_steps
    assert all(p.n_em_steps == steps for p in probs)
    cell_steps = sum(p.n_cells for p in probs) * steps
    res = {"variants": n_variants, "em_steps": steps, "cells_total": sum(p.n_cells for p in probs)}
    fields = {}

    def batched(prec):
        plans = [etm.Plan(p, J, dt=dt, precision=prec, n_steps=steps, history=False, stream=torch.cuda.Stream())
                 for p, J, dt in zip(probs, Js, dts)]
        b = etm.Batch(len(plans))
        for pl in plans:
            b.attach(pl)
        s = torch.cuda.Stream()
        torch.cuda.synchronize()
        t = time.perf_counter()
        b.advance(steps, s)
        s.synchronize()
        infos = etm.solve_all(plans)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        out = [(pl.read(etm.ETM_FIELD_THETA), pl.read(etm.ETM_FIELD_VM)) for pl in plans]
        del b, plans
        torch.cuda.synchronize()
        return wall, out, infos

    def sequential(prec):
        wall = 0.0
        out = []
        for p, J, dt in zip(probs, Js, dts):
            pl = etm.Plan(p, J, dt=dt, precision=prec, n_steps=steps, history=False)
            torch.cuda.synchronize()
            t = time.perf_counter()
            pl.advance(steps)
            pl.mech_solve()
            pl.sync()
            wall += time.perf_counter() - t
            out.append((pl.read(etm.ETM_FIELD_THETA), pl.read(etm.ETM_FIELD_VM)))
            del pl
        torch.cuda.synchronize()
        return wall, out

    wb, fields["mixed"], _ = batched(etm.ETM_PREC_MIXED)
    ws, fields["fp64"] = sequential(etm.ETM_PREC_FP64)
    wbf, _, _ = batched(etm.ETM_PREC_FP64)
    th_err = max(float(np.abs(a[0] - b[0]).max() / max(np.abs(b[0]).max(), 1e-300))
                 for a, b in zip(fields["mixed"], fields["fp64"]))
    vm_err = max(abs(float(a[1].max()) - float(b[1].max())) / max(float(b[1].max()), 1e-300)
                 for a, b in zip(fields["mixed"], fields["fp64"]))
    res.update({"batched_mixed_s": round(wb, 3), "sequential_fp64_s": round(ws, 3), "batched_fp64_s": round(wbf, 3),
                "speedup_vs_sequential_fp64": round(ws / wb, 2),
                "batched_mixed_mcell_steps_per_s": round(cell_steps / wb / 1e6, 1),
                "sequential_fp64_mcell_steps_per_s": round(cell_steps / ws / 1e6, 1),
                "theta_rel_err_mixed_vs_fp64": th_err, "peak_vm_rel_err_mixed_vs_fp64": vm_err,
                "timing": "wall clock, EM march + thermal + one mechanical solve per variant; plan set-up excluded"})
    torch.cuda.empty_cache()
    return res


def serve_leg(n_requests, rates, precisions=("mixed", "fp64")):
    """Continuous-batching server under Poisson arrivals, mixed and FP64.

    Per rate and precision: latency percentiles, designs/hour and the
    sustained fraction (answered requests per second over the offered rate).
    The knee is the highest rate whose p99 latency stays within twice the p99
    at the lowest rate while at least 90% of the offered rate is sustained."""
    import torch
    import workloads as W
    import paper_2603_07038_amd as etm
    from paper_2603_07038_amd import serve
    probs = [W.config5_request(r) for r in range(n_requests)]
    res = {"requests_per_rate": n_requests, "mean_cells": round(sum(p.n_cells for p in probs) / n_requests),
           "mean_em_steps": round(sum(p.n_em_steps for p in probs) / n_requests),
           "arrivals": "Poisson, seed 5999", "rates": {}}
    precs = {"mixed": etm.ETM_PREC_MIXED, "fp64": etm.ETM_PREC_FP64}
    for rate in rates:
        arrivals = W.poisson_arrivals(rate, n_requests)
        one = {}
        for name in precisions:
            reqs = [serve.Request(p, float(t), r) for r, (p, t) in enumerate(zip(probs, arrivals))]
            srv = serve.Server(max_slots=16, hbm_budget=96e9, precision=precs[name])
            torch.cuda.synchronize()
            t = time.perf_counter()

            last = [0]

            def progress(done, t=t, name=name, last=last):
                if len(done) // 32 > last[0] or len(done) == n_requests:
                    last[0] = len(done) // 32
                    say(f"[serve] {name} {rate} req/s: {len(done)}/{n_requests} answered at "
                        f"{time.perf_counter() - t:.1f} s")
            done = srv.run(reqs, realtime=True, progress=progress)
            wall = time.perf_counter() - t
            summ = serve.summarize(done, wall)
            summ["sustained_frac"] = summ["completed"] / wall / rate if wall > 0 else None
            one[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in summ.items()}
            del srv
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
        res["rates"][str(rate)] = one
    for name in precisions:
        pts = [(float(r), v[name]) for r, v in res["rates"].items() if name in v]
        if len(pts) >= 2:   # a knee needs a sweep
            res[f"knee_{name}_req_per_s"] = serving_knee(pts)
    res["knee_rule"] = "highest rate with p99 <= 2x the p99 at the lowest rate and >= 90% of the offered rate answered"
    return res


def serving_knee(pts):
    """The knee of a serving sweep: ``pts`` is a list of (offered rate,
    summary with "p99_s" and "sustained_frac"); returns the highest rate whose
    p99 latency is at most twice the p99 at the lowest rate while at least
    90 % of the offered rate is answered, or None."""
    pts = sorted(pts, key=lambda x: x[0])
    p99_0 = pts[0][1]["p99_s"]
    ok = [r for r, v in pts if v["p99_s"] <= 2.0 * p99_0 and (v["sustained_frac"] or 0.0) >= 0.9]
    return max(ok) if ok else None


# ---- the FP64 oracle on the host cores -------------------------------------------
def cpu_legs(prob3, dt3):
    """The oracle as it stands on the host's cores (bounded samples)."""
    import numpy as np
    import oracle
    import workloads as W
    cores = oracle.num_threads()
    out = {}
    # the headline workload: one EM step with its Joule source and a thermal step
    J3 = prob3.sample_J_half(dt3, 2)
    o = oracle.Oracle(prob3)
    t = time.perf_counter()
    o.run(dt3, 1, J3, R=1)
    el = time.perf_counter() - t
    head = {"value": round(prob3.n_cells / el / 1e6, 3), "unit": "Mcell-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"1 coupled step (EM update, Joule source, thermal step) of the {prob3.nx}x{prob3.ny}x"
                      f"{prob3.nz} package from a zero state, {el:.1f} s (state allocation included)"}
    del o
    # the slice: 16 EM steps closed by their thermal step
    p2 = W.config2()
    o2 = oracle.Oracle(p2)
    dt2 = o2.cfl_dt()
    J2 = p2.sample_J_half(dt2, 17)
    st, _ = o2.run(dt2, 1, J2, R=16)
    t = time.perf_counter()
    o2.run(dt2, 15, J2, state=st, R=16)
    el2 = time.perf_counter() - t
    out["slice256x256x64_coupled"] = {"mcell_steps_per_s": round(p2.n_cells * 15 / el2 / 1e6, 3),
                                      "sample": "EM steps 2-16 with the thermal step at step 16", "s": round(el2, 2)}
    # the slice's mechanics: one application of K (a Jacobi-PCG iteration's
    # dominant work) with element matrices formed on the fly; the oracle's
    # solver would first cache them (576 doubles per cell, 19 GB here)
    mask2 = o2.mech_mask()
    q2 = np.zeros(tuple(o2.node_shape) + (3,))
    q2[..., 2] = 1e-9
    t = time.perf_counter()
    o2.mech_apply(mask2, q2)
    el_k = time.perf_counter() - t
    dofs2 = 3 * int(np.prod(o2.node_shape))
    out["slice256x256x64_cg"] = {"dof_iter_per_s": round(dofs2 / el_k, 1), "apply_s": round(el_k, 2),
                                 "sample": "one K application (HEX8 elements formed per cell), the cost of a "
                                           "Jacobi-PCG iteration without the element cache"}
    del o2
    # the 32x32x16 trace case in full: 2000 steps at R = 200, one solve
    p1 = W.config1()
    o1 = oracle.Oracle(p1)
    dt1 = o1.cfl_dt()
    J1 = p1.sample_J_half(dt1, p1.n_em_steps)
    t = time.perf_counter()
    st1, _ = o1.run(dt1, p1.n_em_steps, J1)
    el1 = time.perf_counter() - t
    mask = o1.mech_mask()
    t = time.perf_counter()
    q, it, _ = o1.mech_solve(st1["theta"], mask, rtol=p1.cg_rtol)
    elm = time.perf_counter() - t
    # CG DOF-iterations/s: two runs of fixed length (setup cancels)
    th = st1["theta"]
    t = time.perf_counter()
    o1.mech_solve(th, mask, rtol=1e-300, maxit=20)
    ta = time.perf_counter() - t
    t = time.perf_counter()
    o1.mech_solve(th, mask, rtol=1e-300, maxit=220)
    tb = time.perf_counter() - t
    dofs = 3 * int(np.prod(o1.node_shape))
    out["pkg32_full"] = {"mcell_steps_per_s": round(p1.n_cells * p1.n_em_steps / el1 / 1e6, 3),
                         "march_s": round(el1, 3), "mech_solve_s": round(elm, 3), "cg_iters": it,
                         "cg_dof_iter_per_s": round(dofs * 200 / max(tb - ta, 1e-9), 1),
                         "cg_note": "Jacobi-PCG; (220 - 20) iterations from the time difference of two fixed-length "
                                    "solves"}
    head["extra"] = out
    return head


def main():
    a = parse()
    if a.probe:
        probe(a.probe)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import paper_2603_07038_amd as etm
    etm.load()
    torch.cuda.init()
    serve_args = (a.serve_requests, [float(r) for r in a.serve_rates.split(",")], a.serve_precisions.split(","))
    if a.serve_only:
        print(json.dumps({"serving": serve_leg(*serve_args)}))
        return
    legs = set(a.legs.split(","))
    prob, dt, mixed, fp64, cmp = headline(a.steps, a.warmup)
    extra = {"copy_ceiling": copy_ceiling()}
    mixed["roofline"]["frac_of_copy_ceiling"] = round(mixed["roofline"]["achieved"] / extra["copy_ceiling"]["GBs"], 4)
    fp64["roofline"]["frac_of_copy_ceiling"] = round(fp64["roofline"]["achieved"] / extra["copy_ceiling"]["GBs"], 4)
    for leg, fn in (("slice", slice_leg), ("r1", r1_leg), ("temporal", temporal_leg), ("excitation", excitation_leg)):
        if leg in legs:
            say(f"[bench] leg {leg}")
            extra[leg] = fn()
    if "batch" in legs:
        say("[bench] leg batch")
        extra["batch"] = batch_leg(a.batch_variants)
    if "serve" in legs:
        say("[bench] leg serve")
        extra["serving"] = serve_leg(*serve_args)
    cpu = None
    if "cpu" in legs and not a.no_cpu:
        say("[bench] leg cpu")
        cpu = cpu_legs(prob, dt)
    out = {
        "metric": "coupled Mcell-steps/s",
        "value": round(mixed["value"], 2),
        "unit": "Mcell-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(mixed["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": prob.name, "cells": prob.n_cells, "grid": [prob.nx, prob.ny, prob.nz],
                   "em_steps_per_step": prob.em_per_thermal, "thermal_steps_per_step": 1, "dt_s": dt,
                   "precision": "mixed", "mechanics": "reported beside (one solve after the timed blocks)"},
        "march_only_mcell_steps_per_s": round(mixed["march_only_mcell_steps_per_s"], 1),
        "em_kernel_us": round(mixed["em_kernel_us"], 2),
        "roofline": mixed["roofline"],
        "cpu_baseline": cpu,
        "fp64": {"value": round(fp64["value"], 2), "ms_per_step": round(fp64["ms_per_step"], 3),
                 "em_kernel_us": round(fp64["em_kernel_us"], 2), "roofline": fp64["roofline"]},
        "mixed_vs_fp64": cmp,
        "mechanics": {"workload": prob.name, "mixed": mixed["mechanics"], "fp64": fp64["mechanics"]},
    }
    out.update(extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
