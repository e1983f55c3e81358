#!/usr/bin/env python3
"""Benchmark: coupled Mcell-steps/s of the MI355X EM-thermal-mechanical path.

Workload: the 256x256x64 graded package slice (4.19 M cells; substrate with
16 PRBS-7-driven traces, 8x8 microbumps, TSV interposer, two dies), EM step
at CFL 0.9, R = 200 EM steps per thermal step, a warm-started mechanical
solve (rtol 1e-8) after every thermal step.

One bench step = one coupling block: 200 EM steps (EM update + Joule
source), one thermal step, one mechanical solve + von Mises, histories.
`value` = cells * EM steps / wall time of the timed blocks, mechanics
included.  The timed blocks run as one advance call, so each block's
solve runs on the plan's side stream while the next block's EM steps run
(the default `mech_overlap`; results are bitwise those of the serial
order).  The march-only rate, the serial tail of a block and CG
DOF-iterations/s come from two further blocks timed in parts.  The headline runs the mixed path (FP32 fields, FP64 temperature /
Joule / CG refinement); the same blocks are timed on the FP64 path.

Beside the headline, the same JSON line carries:
  fullscale  the 1024x1024x128 package (134 M cells): EM march rate and its
             HBM roofline fraction, mixed and FP64, and mixed with the
             two-step slab wavefront over 8 z-slabs (temporal blocking);
  temporal_blocking  the slice's EM march per step with the two-step slab
             wavefront over 3 and 8 z-slabs against one launch per step;
  excitation the same package under the excitation scheme of Sec. III-B (52,640
             port edges, one closed-form wave per port sampled on the
             device): EM march rate, mixed;
  batch      64 design variants of uneven size (64x64x32 .. 192x192x48,
             2048 EM steps + a mechanical solve each): one batched mixed run
             against 64 sequential FP64 runs and a batched FP64 run, with
             the largest temperature / peak von Mises difference between the
             mixed and FP64 results;
  serving    Poisson arrivals of design requests (sizes log-uniform between
             32^3 and 512x512x64 cells) through the continuous-batching
             server: p50/p99 latency and designs/hour, mixed and FP64.

    python bench.py [--steps K] [--warmup W] [--precision mixed|fp64] [--no-fp64] [--no-cpu]
                    [--legs coupled,fullscale,temporal,excitation,batch,serve] [--serve-requests N] [--serve-rate R]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Compulsory bytes per cell-step of the fused EM step (one cell ~ one node +
# three edges): FP64 e^n, e^{n-1} read + e^{n+1} written (72), material id
# (1), temperature for sigma(T) (8), Joule accumulator read-modify-write (16);
# mixed (leapfrog form): e in FP32 read + written (24) with its 8-bit
# residual (6), face field h in FP32 read + written (24), the sigma-change
# correction K read (12, plans with temperature-dependent conductors), id (1),
# FP32 temperature (4), Joule RMW (16).
BYTES_PER_CELL_STEP = {"fp64": 97.0, "mixed": 87.0}
# Compulsory bytes per DOF-iteration of Jacobi-PCG (vectors u, r, p, w and the
# inverse diagonal streamed once per iteration): FP64 80, FP32 40.
BYTES_PER_DOF_ITER = {"fp64": 80.0, "mixed": 40.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--legs", default="coupled,fullscale,temporal,excitation,batch,serve")
    ap.add_argument("--batch-variants", type=int, default=64)
    ap.add_argument("--serve-requests", type=int, default=32)
    ap.add_argument("--serve-rate", type=float, default=2.0)
    ap.add_argument("--probe", choices=["em", "em-fp64", "em-pair", "mech", "copy"], default=None,
                    help="short runs for hardware-counter profiles: 20 EM steps of the workload (em-pair: as "
                         "10 two-step slab wavefronts over --probe-slabs z-slabs), two coupling blocks with their "
                         "mechanical solves (mech), or a plain 2 GiB device copy (the calibration kernel for "
                         "FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--probe-slabs", type=int, default=3)
    return ap.parse_args()


def probe(kind, slabs=3):
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
    prob = W.config2()
    if kind == "mech":
        dt = etm.cfl_dt(prob)
        R = prob.em_per_thermal
        J = prob.sample_J_half(dt, 2 * R + 2)
        plan = etm.Plan(prob, J, dt=dt, precision=etm.ETM_PREC_MIXED, n_steps=2 * R + 2, history=False)
        plan.advance(2 * R)
        info = plan.sync()
        print(json.dumps({"probe": kind, "workload": prob.name, "cells": prob.n_cells, "em_steps": 2 * R,
                          "mech_solves": info["n_solves"], "cg_iters_total": info["cg_iters_total"]}))
        return
    prob.mech_every_thermal = 0
    prob.em_per_thermal = 256  # 20 steps: no thermal step inside the probe
    dt = etm.cfl_dt(prob)
    J = prob.sample_J_half(dt, 64)
    prec = etm.ETM_PREC_FP64 if kind == "em-fp64" else etm.ETM_PREC_MIXED
    plan = etm.Plan(prob, J, dt=dt, precision=prec, n_steps=64, history=False,
                    em_slabs=slabs if kind == "em-pair" else 0)
    plan.advance(20)
    plan.sync()
    print(json.dumps({"probe": kind, "workload": prob.name, "cells": prob.n_cells, "em_steps": 20,
                      "em_slabs": slabs if kind == "em-pair" else 0}))


PROFILE_EM = {"mixed": "profiles/em_march_slice256x256x64_mixed.md"}


def measured_traffic(prec_name):
    """HBM bytes per launch of the EM march from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the copy-kernel calibration);
    None when no summary exists or the kernel source changed since it was taken."""
    import hashlib
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


def run_precision(prob, J, dt, prec_name, steps, warmup):
    import torch
    import paper_2603_07038_amd as etm
    prec = etm.ETM_PREC_MIXED if prec_name == "mixed" else etm.ETM_PREC_FP64
    R = prob.em_per_thermal
    plan = etm.Plan(prob, J, dt=dt, precision=prec, n_steps=prob.n_em_steps)
    stream = plan.stream
    for _ in range(warmup):
        plan.advance(R)
    info_w = plan.sync()
    # The parts of a block, timed apart on `split` further blocks: the EM
    # march (R - 1 steps back to back) and the tail (last EM step, thermal
    # step, mechanical solve, von Mises; a solve that ends an advance call
    # runs without overlap).
    split = 2
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(split)]
    for b in range(split):
        ev[b][0].record(stream)
        plan.advance(R - 1)
        ev[b][1].record(stream)
        plan.advance(1)
        ev[b][2].record(stream)
    info0 = plan.sync()
    torch.cuda.synchronize()
    em_ms = sum(e[0].elapsed_time(e[1]) for e in ev)
    tail_ms = sum(e[1].elapsed_time(e[2]) for e in ev)
    split_iters = info0["cg_iters_total"] - info_w["cg_iters_total"]
    # The headline: `steps` coupled steps in one advance call; each scheduled
    # solve runs on the plan's side stream while the next block's EM steps
    # run (mech_overlap, the default; the last block's solve ends the call).
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.advance(R * steps)
    info = plan.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cells = prob.n_cells
    em_launch_s = em_ms / 1e3 / (split * (R - 1))
    iters = info["cg_iters_total"] - info0["cg_iters_total"]
    _, _, mech_dofs = plan.dofs()
    res = dict(
        wall_s=wall,
        ms_per_step=wall / steps * 1e3,
        value=cells * R * steps / wall / 1e6,
        march_mcell_steps_per_s=cells * (R - 1) * split / (em_ms / 1e3) / 1e6,
        em_kernel_us=em_launch_s * 1e6,
        tail_ms_per_block=tail_ms / split,
        cg_iters=iters,
        cg_dof_iter_per_s=(mech_dofs * split_iters / (tail_ms / 1e3)) if split_iters else None,
        theta_max=info["theta_max"],
        cg_relres=info["cg_relres"],
        step_reached=info["step"],
    )
    bpc = BYTES_PER_CELL_STEP[prec_name]
    achieved = bpc * cells / em_launch_s / 1e9
    res["fields"] = (plan.read(etm.ETM_FIELD_THETA), plan.read(etm.ETM_FIELD_VM))
    res["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(prec_name),
                       "traffic_unit": "bytes/launch", "algorithmic_bytes_per_launch": int(bpc * cells),
                       "kernel": "em_march_kernel<%s>" % ("float,true" if prec_name == "mixed" else "double,false"),
                       "launch_us": round(em_launch_s * 1e6, 2),
                       "bytes_per_cell_step": bpc, "cells_per_launch": cells}
    del plan
    torch.cuda.synchronize()
    return res


def fullscale_leg(steps=48, warmup=8):
    """EM march of the 1024x1024x128 package, mixed and FP64."""
    import torch
    import workloads as W
    import paper_2603_07038_amd as etm
    prob = W.config3()
    prob.history_stride = 0
    dt = etm.cfl_dt(prob)
    J = prob.sample_J_half(dt, steps + warmup + 2)
    out = {"workload": prob.name, "cells": prob.n_cells}
    for name, prec, slabs in (("mixed", etm.ETM_PREC_MIXED, 0), ("fp64", etm.ETM_PREC_FP64, 0),
                              ("mixed_em_slabs8", etm.ETM_PREC_MIXED, 8)):
        plan = etm.Plan(prob, J, dt=dt, precision=prec, n_steps=steps + warmup + 2, history=False, em_slabs=slabs)
        plan.advance(warmup)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(plan.stream)
        plan.advance(steps)
        e1.record(plan.stream)
        plan.sync()
        t = e0.elapsed_time(e1) / 1e3 / steps
        bpc = BYTES_PER_CELL_STEP[name.split("_")[0]]
        gbs = bpc * prob.n_cells / t / 1e9
        out[name] = {"march_mcell_steps_per_s": round(prob.n_cells / t / 1e6, 1), "em_kernel_us": round(t * 1e6, 1),
                     "achieved_GBs": round(gbs, 1), "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}
        del plan
        torch.cuda.synchronize()
    return out


def temporal_leg(steps=100, warmup=10, slabs=(0, 3, 8)):
    """EM march of the 256x256x64 slice (mixed) with the two-step slab
    wavefront (em_slabs = S) against one launch per step (S = 0); the
    fullscale leg runs the package with S = 8."""
    import torch
    import workloads as W
    import paper_2603_07038_amd as etm
    prob = W.config2()
    prob.mech_every_thermal = 0
    prob.em_per_thermal = 100000
    prob.history_stride = 0
    dt = etm.cfl_dt(prob)
    J = prob.sample_J_half(dt, steps + warmup + 2)
    out = {"workload": prob.name, "cells": prob.n_cells, "em_steps": steps, "us_per_step": {}}
    for S in slabs:
        plan = etm.Plan(prob, J, dt=dt, precision=etm.ETM_PREC_MIXED, n_steps=steps + warmup + 2, history=False,
                        em_slabs=S)
        plan.advance(warmup)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(plan.stream)
        plan.advance(steps)
        e1.record(plan.stream)
        plan.sync()
        out["us_per_step"][str(S)] = round(e0.elapsed_time(e1) * 1e3 / steps, 2)
        del plan
        torch.cuda.synchronize()
    return out


def excitation_leg(steps=256, warmup=8, t_origin=95e-12):
    """EM march of the 1024x1024x128 package under the excitation scheme of
    Sec. III-B (one closed-form wave per port, sampled on the device in blocks
    of steps), mixed precision, in a window where the 5 GHz sine and the
    40 GHz burst are on; the march rate against the tabulated-PRBS package
    of the fullscale leg, and the host table the device sampling avoids for
    the scheme's 300 ps window."""
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
    return res


def serve_leg(n_requests, rate):
    """Continuous-batching server under Poisson arrivals, mixed and FP64."""
    import torch
    import workloads as W
    import paper_2603_07038_amd as etm
    from paper_2603_07038_amd import serve
    arrivals = W.poisson_arrivals(rate, n_requests)
    probs = [W.config5_request(r) for r in range(n_requests)]
    res = {"requests": n_requests, "rate_per_s": rate,
           "mean_cells": round(sum(p.n_cells for p in probs) / n_requests), "arrivals": "Poisson, seed 5999"}
    for name, prec in (("mixed", etm.ETM_PREC_MIXED), ("fp64", etm.ETM_PREC_FP64)):
        reqs = [serve.Request(p, float(t), r) for r, (p, t) in enumerate(zip(probs, arrivals))]
        srv = serve.Server(max_slots=16, hbm_budget=96e9, precision=prec)
        torch.cuda.synchronize()
        t = time.perf_counter()
        done = srv.run(reqs, realtime=True)
        wall = time.perf_counter() - t
        summ = serve.summarize(done, wall)
        res[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in summ.items()}
        del srv
        torch.cuda.synchronize()
    return res


def cpu_baseline(prob, dt, J, budget_s):
    """The FP64 oracle as it stands, on the host cores: EM + Joule march steps
    of the same workload (a bounded sample), in Mcell-steps/s."""
    import oracle
    o = oracle.Oracle(prob)
    t = time.perf_counter()
    st, _ = o.run(dt, 1, J, R=prob.em_per_thermal)
    one = time.perf_counter() - t
    n = max(1, min(int(budget_s / max(one, 1e-3)), 200))
    t = time.perf_counter()
    o.run(dt, n, J, state=st, R=prob.em_per_thermal)
    el = time.perf_counter() - t
    return {"value": round(prob.n_cells * n / el / 1e6, 3), "unit": "Mcell-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{n} EM+Joule steps of the {prob.nx}x{prob.ny}x{prob.nz} slice (FP64 oracle, mechanics "
                      f"and thermal steps not in the sample), {el:.1f} s"}


def main():
    a = parse()
    if a.probe:
        probe(a.probe, a.probe_slabs)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import workloads as W
    import paper_2603_07038_amd as etm
    legs = set(a.legs.split(","))
    prob = W.config2()
    dt = etm.cfl_dt(prob)
    J = prob.sample_J_half(dt, prob.n_em_steps)
    torch.cuda.init()
    head = run_precision(prob, J, dt, a.precision, a.steps, a.warmup)
    other = None
    if not a.no_fp64 and a.precision == "mixed":
        other = run_precision(prob, J, dt, "fp64", a.steps, a.warmup)
    extra = {}
    if "fullscale" in legs:
        extra["fullscale"] = fullscale_leg()
    if "temporal" in legs:
        extra["temporal_blocking"] = temporal_leg()
    if "excitation" in legs:
        extra["excitation"] = excitation_leg()
    if "batch" in legs:
        extra["batch"] = batch_leg(a.batch_variants)
    if "serve" in legs:
        extra["serving"] = serve_leg(a.serve_requests, a.serve_rate)
    cpu = None
    if not a.no_cpu:
        cpu = cpu_baseline(prob, dt, J, a.cpu_seconds)
    out = {
        "metric": "coupled Mcell-steps/s (EM + Joule + thermal march with a warm-started mechanical solve per "
                  "thermal step)",
        "value": round(head["value"], 2),
        "unit": "Mcell-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(head["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if a.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": prob.name, "cells": prob.n_cells, "grid": [prob.nx, prob.ny, prob.nz],
                   "em_steps_per_step": prob.em_per_thermal, "dt_s": dt, "mech_solve_per_step": True,
                   "cg_rtol": prob.cg_rtol, "precision": a.precision},
        "march_mcell_steps_per_s": round(head["march_mcell_steps_per_s"], 1),
        "em_kernel_us": round(head["em_kernel_us"], 2),
        "mech_ms_per_step": round(head["tail_ms_per_block"], 2),
        "cg_iters": head["cg_iters"],
        "cg_dof_iter_per_s": head["cg_dof_iter_per_s"],
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
    }
    out.update(extra)
    if other:
        import numpy as np
        (tm, vm), (tf, vf) = head.pop("fields"), other.pop("fields")
        out["mixed_vs_fp64"] = {
            "theta_rel_err": float(np.abs(tm - tf).max() / max(np.abs(tf).max(), 1e-300)),
            "peak_vm_rel_err": abs(float(vm.max()) - float(vf.max())) / max(float(vf.max()), 1e-300),
            "theta_max_K": float(tf.max()),
            "after_em_steps": (a.warmup + a.steps) * prob.em_per_thermal,
            "targets": {"theta": 1e-6, "peak_vm": 1e-5}}
        out["fp64"] = {"value": round(other["value"], 2), "ms_per_step": round(other["ms_per_step"], 3),
                       "march_mcell_steps_per_s": round(other["march_mcell_steps_per_s"], 1),
                       "em_kernel_us": round(other["em_kernel_us"], 2), "cg_iters": other["cg_iters"],
                       "cg_dof_iter_per_s": other["cg_dof_iter_per_s"], "roofline": other["roofline"]}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
