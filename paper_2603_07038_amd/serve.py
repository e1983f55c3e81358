"""Continuous-batching server for design-variant simulations.

Requests (one package design each) arrive over time.  The server keeps a
batch of bound plans resident on the GPU and advances all of them together
(one launch per EM step over every admitted variant, chunks replayed from
HIP graphs).  At every chunk boundary it

  * admits queued requests, first come first served, while a batch slot is
    free and the summed device footprint stays within the HBM budget;
  * advances every admitted variant by one chunk (or by the fewest steps any
    of them still needs, so each stops exactly at its own step count);
  * retires variants whose EM + thermal march is complete: the variant
    leaves the batch and a worker thread runs its mechanical solve (Eq. 8,
    multigrid-preconditioned CG) and von Mises stress (Eq. 9) on the
    variant's own stream, overlapping with the batched march of the others,
    then reads the results back; the workspace is released and the request's
    latency (arrival -> result on the host) is recorded.

A variant's results do not depend on what it shares the GPU with: the
batched EM step runs the same per-node arithmetic as a solo run.
"""
from __future__ import annotations

import dataclasses
import time
from concurrent.futures import FIRST_COMPLETED, ThreadPoolExecutor
from concurrent.futures import wait as wait_futures
from typing import List, Optional

import numpy as np

from . import ETM_FIELD_THETA, ETM_FIELD_VM, ETM_PREC_MIXED, STATUS_NAMES, Batch, EtmError, Plan, cfl_dt


@dataclasses.dataclass
class Request:
    prob: object          # workloads.Problem
    arrival: float = 0.0  # seconds after the server starts
    rid: int = 0
    opts: Optional[dict] = None  # plan option overrides (e.g. {"cg_maxit": 500})


@dataclasses.dataclass
class Result:
    rid: int
    name: str
    cells: int
    em_steps: int
    arrival: float
    admitted: float
    finished: float
    theta_max: float
    vm_max: float
    cg_iters: int
    cg_relres: float
    theta: Optional[np.ndarray] = None
    vm: Optional[np.ndarray] = None
    status: str = "ok"    # "ok"; "rejected" (footprint above the HBM budget); "error" (see message)
    message: str = ""

    @property
    def latency(self):
        return self.finished - self.arrival


class Server:
    def __init__(self, max_slots: int = 16, hbm_budget: float = 64e9, precision: int = ETM_PREC_MIXED,
                 chunk: int = 256, keep_fields: bool = False, tune_json: Optional[str] = None,
                 solve_workers: int = 4):
        import torch
        self.torch = torch
        self.max_slots = max_slots
        self.hbm_budget = float(hbm_budget)
        self.precision = precision
        self.chunk = int(chunk)
        self.keep_fields = keep_fields
        self.batch = Batch(max_slots, tune_json)
        self.stream = torch.cuda.Stream()
        self.used = 0.0
        self.active = {}   # slot -> [request, plan, admitted time, EM steps enqueued]
        self.solving = []  # [future, request, plan, admitted time]
        self.pool = ThreadPoolExecutor(max_workers=max(1, int(solve_workers)))
        self._t0 = time.perf_counter()
        self.log: List[str] = []

    def _make_plan(self, req: Request):
        p = req.prob
        dt = cfl_dt(p)
        J = p.sample_J_half(dt, p.n_em_steps)
        plan = Plan(p, J, dt=dt, precision=self.precision, n_steps=p.n_em_steps, history=False, bind=False,
                    **(req.opts or {}))
        return plan

    def _reject(self, req: Request, plan, now: float, status: str, message: str) -> Result:
        return Result(rid=req.rid, name=req.prob.name, cells=req.prob.n_cells, em_steps=req.prob.n_em_steps,
                      arrival=req.arrival, admitted=now, finished=now, theta_max=float("nan"), vm_max=float("nan"),
                      cg_iters=0, cg_relres=float("nan"), status=status, message=message)

    def _admit(self, req: Request, plan, now: float) -> bool:
        if len(self.active) >= self.max_slots or self.used + plan.footprint > self.hbm_budget:
            return False
        torch = self.torch
        stream = torch.cuda.Stream()   # the variant's own stream (its solve runs there)
        with torch.cuda.stream(stream):
            ws = torch.empty(plan.footprint + 256, dtype=torch.uint8, device="cuda")
            plan.bind(ws, stream)
        slot = self.batch.attach(plan)
        self.active[slot] = [req, plan, now, 0]
        self.log.append(f"admit {req.rid} slot {slot} stream {stream.cuda_stream:#x} at {now:.3f}")
        self.used += plan.footprint
        return True

    def _finish(self, plan):
        """Worker thread: solve, von Mises, read back; returns (info, theta, vm,
        time, error message or "")."""
        err = ""
        try:
            plan.mech_solve()   # enqueues; its outcome (e.g. ETM_E_NOCONV) comes from etm_sync
        except EtmError as e:
            err = str(e)
        info = plan.sync(raise_on_error=False)
        theta = plan.read(ETM_FIELD_THETA)
        vm = plan.read(ETM_FIELD_VM)
        return info, theta, vm, time.perf_counter() - self._t0, err

    def _retire(self, slot: int):
        req, plan, admitted, _ = self.active.pop(slot)
        self.batch.detach(slot)
        self.log.append(f"retire {req.rid} slot {slot}")
        self.solving.append([self.pool.submit(self._finish, plan), req, plan, admitted])

    def _collect(self, done: List[Result], block: float = 0.0):
        if not self.solving:
            return
        if block > 0.0:
            wait_futures([e[0] for e in self.solving], timeout=block, return_when=FIRST_COMPLETED)
        keep = []
        for fut, req, plan, admitted in self.solving:
            if not fut.done():
                keep.append([fut, req, plan, admitted])
                continue
            try:
                info, theta, vm, finished, err = fut.result()
                if not err and info["status"] != 0:
                    err = f"{STATUS_NAMES.get(info['status'], info['status'])}: reported by etm_sync"
                done.append(Result(rid=req.rid, name=req.prob.name, cells=req.prob.n_cells,
                                   em_steps=req.prob.n_em_steps, arrival=req.arrival, admitted=admitted,
                                   finished=finished, theta_max=float(theta.max()), vm_max=float(vm.max()),
                                   cg_iters=int(info["cg_iters"]), cg_relres=float(info["cg_relres"]),
                                   theta=theta if self.keep_fields else None, vm=vm if self.keep_fields else None,
                                   status="error" if err else "ok", message=err))
            except Exception as e:  # a failure of one request never stops the loop
                now = time.perf_counter() - self._t0
                r = self._reject(req, plan, now, "error", repr(e))
                r.admitted = admitted
                done.append(r)
            finally:
                self.used -= plan.footprint
                plan.ws = None
        self.solving = keep

    def run(self, requests: List[Request], realtime: bool = True, progress=None) -> List[Result]:
        """Serve all requests; arrivals are honoured in wall-clock time when
        ``realtime`` (else every request is available at once).  ``progress``,
        if given, is called with the list of answered requests each time it
        has grown."""
        pending = sorted(requests, key=lambda r: r.arrival)
        queue: List = []
        done: List[Result] = []
        self._t0 = t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        n_seen = 0
        while pending or queue or self.active or self.solving:
            if progress is not None and len(done) != n_seen:
                n_seen = len(done)
                progress(done)
            t = now()
            while pending and (not realtime or pending[0].arrival <= t):
                r = pending.pop(0)
                try:
                    plan = self._make_plan(r)
                except EtmError as e:   # invalid request: answered at once
                    done.append(self._reject(r, None, now(), "error", str(e)))
                    continue
                if plan.footprint > self.hbm_budget:
                    # can never fit: answered at once instead of blocking the queue
                    done.append(self._reject(r, plan, now(), "rejected",
                                             f"needs {plan.footprint} B of device memory, above the "
                                             f"{int(self.hbm_budget)} B budget"))
                    continue
                queue.append((r, plan))
            self._collect(done)
            while queue:
                r, plan = queue[0]
                if not self._admit(r, plan, now()):
                    break
                queue.pop(0)
            if not self.active:
                # nothing to march: wait for a solve to finish or the next arrival
                nxt = max(0.0, pending[0].arrival - now()) if (pending and realtime) else 0.05
                if self.solving:
                    self._collect(done, block=min(max(nxt, 1e-3), 0.05))
                elif pending and realtime:
                    time.sleep(min(nxt, 0.05))
                continue
            n = min([self.chunk] + [ent[0].prob.n_em_steps - ent[3] for ent in self.active.values()])
            if n > 0:
                self.batch.advance(n, self.stream)
            for ent in self.active.values():
                ent[3] += n
            for slot in [s for s, ent in self.active.items() if ent[3] >= ent[0].prob.n_em_steps]:
                self._retire(slot)
        return done


def summarize(results: List[Result], wall: float) -> dict:
    """Latency percentiles and throughput over the requests that finished;
    rejected and failed requests are counted beside them."""
    ok = [r for r in results if r.status == "ok"]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    return {"requests": len(results), "completed": len(ok),
            "rejected": sum(r.status == "rejected" for r in results),
            "failed": sum(r.status == "error" for r in results),
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "designs_per_hour": len(ok) / wall * 3600.0 if wall > 0 else None,
            "cell_steps": int(sum(r.cells * r.em_steps for r in ok)), "wall_s": wall,
            "cg_iters_mean": float(np.mean([r.cg_iters for r in ok])) if ok else None,
            "cg_iters_max": int(max(r.cg_iters for r in ok)) if ok else None}
