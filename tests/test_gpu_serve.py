"""Serving: continuous batching admits requests as slots free up, and each
request's results are the same alone, in the mix, and as a plain solo run."""
import sys

import numpy as np
import pytest

import paper_2603_07038_amd as etm
from paper_2603_07038_amd import serve
import workloads as W

pytestmark = pytest.mark.gpu


def _req(r, nx, ny, nz, bits):
    p = W.package(nx, ny, nz, 7000 + r, bump_pitch_um=20, bump_cells=8, trace_width=2, trace_pitch=4,
                  n_trace_layers=2, max_traces=6, n_bits=bits, steps_per_bit=4, em_per_thermal=256,
                  name=f"req{r}")
    return serve.Request(prob=p, arrival=0.05 * r, rid=r)


def _solo(prob, prec):
    dt = etm.cfl_dt(prob)
    pl = etm.Plan(prob, prob.sample_J_half(dt, prob.n_em_steps), dt=dt, precision=prec, n_steps=prob.n_em_steps,
                  history=False)
    pl.advance(prob.n_em_steps)
    pl.mech_solve()
    pl.sync()
    return pl.read(etm.ETM_FIELD_THETA), pl.read(etm.ETM_FIELD_VM)


@pytest.mark.parametrize("prec", [etm.ETM_PREC_MIXED, etm.ETM_PREC_FP64])
def test_results_same_alone_and_in_the_mix(prec):
    reqs = [_req(0, 40, 36, 32, 128), _req(1, 64, 48, 40, 192), _req(2, 33, 70, 32, 64), _req(3, 50, 50, 36, 128)]
    print(f"[serve] prec={prec} cells={[r.prob.n_cells for r in reqs]}", flush=True)
    # two slots: the later requests wait for a slot and join while others run
    srv = serve.Server(max_slots=2, hbm_budget=64e9, precision=prec, keep_fields=True)
    mix = {r.rid: r for r in srv.run(reqs, realtime=True)}
    assert sorted(mix) == [0, 1, 2, 3]
    bad = []
    for q in reqs:
        alone = serve.Server(max_slots=1, precision=prec, keep_fields=True).run([serve.Request(q.prob, 0.0, q.rid)])[0]
        th, vm = _solo(q.prob, prec)
        m = mix[q.rid]
        for name, r in (("mix", m), ("alone", alone)):
            if not (np.array_equal(r.theta, th) and np.array_equal(r.vm, vm)):
                bad.append((q.rid, name, float(np.abs(r.theta - th).max() / np.abs(th).max())))
        assert m.em_steps == q.prob.n_em_steps
        assert m.cg_relres <= q.prob.cg_rtol
        assert m.latency > 0 and m.finished >= m.admitted >= m.arrival - 1e-9
    print(f"[serve] mismatches (request, run, theta rel err): {bad}", flush=True)
    sys.stdout.flush()
    assert not bad
