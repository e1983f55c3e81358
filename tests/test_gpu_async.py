"""The mechanical solve is enqueue-only: etm_mech_solve and an etm_advance
whose last block schedules a solve return while the solve still runs on the
device; etm_sync waits for it and reports its outcome.  Checked on the
256x256x64 slice after a first solve (which builds the multigrid hierarchy
and may wait for it), with the solve's results against a second plan that
waits after every call."""
import time

import numpy as np
import pytest

import paper_2603_07038_amd as etm
import workloads as W

pytestmark = pytest.mark.gpu


def test_solves_return_before_they_end():
    prob = W.config2()
    prob.em_per_thermal = 20
    prob.mech_every_thermal = 1
    dt = etm.cfl_dt(prob)
    J = prob.sample_J_half(dt, 101)
    plan = etm.Plan(prob, J, dt=dt, precision=etm.ETM_PREC_MIXED, n_steps=100, history=False)
    plan.advance(20)                      # first solve: builds the hierarchy
    plan.sync()
    # a scheduled solve at the end of the call
    t0 = time.perf_counter()
    plan.advance(20)
    t_call = time.perf_counter() - t0
    info = plan.sync()
    t_all = time.perf_counter() - t0
    print(f"[async] advance {t_call * 1e3:.1f} ms, with sync {t_all * 1e3:.1f} ms, cg {info['cg_iters']}", flush=True)
    assert info["n_solves"] == 2 and info["cg_relres"] <= prob.cg_rtol
    assert t_call < 0.6 * t_all
    # an explicit solve for a changed temperature
    th = plan.read(etm.ETM_FIELD_THETA)
    th += np.random.default_rng(5).uniform(0.0, 1.0, th.shape)
    plan.write(etm.ETM_FIELD_THETA, th)
    t0 = time.perf_counter()
    plan.mech_solve()
    t_call = time.perf_counter() - t0
    info = plan.sync()
    t_all = time.perf_counter() - t0
    print(f"[async] mech_solve {t_call * 1e3:.1f} ms, with sync {t_all * 1e3:.1f} ms, cg {info['cg_iters']}",
          flush=True)
    assert info["n_solves"] == 3 and info["cg_relres"] <= prob.cg_rtol
    assert t_call < 0.6 * t_all
    # the same calls, each waited for, give the same results
    ref = etm.Plan(prob, J, dt=dt, precision=etm.ETM_PREC_MIXED, n_steps=100, history=False)
    for call in (lambda: ref.advance(20), lambda: ref.advance(20), lambda: ref.write(etm.ETM_FIELD_THETA, th),
                 ref.mech_solve):
        call()
        ref.sync()
    for f in (etm.ETM_FIELD_UX, etm.ETM_FIELD_UZ, etm.ETM_FIELD_VM, etm.ETM_FIELD_THETA):
        np.testing.assert_array_equal(plan.read(f), ref.read(f))
