"""Serving: continuous batching admits requests as slots free up, and each
request's results are the same alone and in the mix."""
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


@pytest.mark.parametrize("prec", [etm.ETM_PREC_MIXED, etm.ETM_PREC_FP64])
def test_results_same_alone_and_in_the_mix(prec):
    reqs = [_req(0, 40, 36, 32, 128), _req(1, 64, 48, 40, 192), _req(2, 33, 70, 32, 64), _req(3, 50, 50, 36, 128)]
    print(f"[serve] prec={prec} cells={[r.prob.n_cells for r in reqs]}", flush=True)
    # two slots: the later requests wait for a slot and join while others run
    srv = serve.Server(max_slots=2, hbm_budget=64e9, precision=prec, keep_fields=True)
    mix = {r.rid: r for r in srv.run(reqs, realtime=True)}
    assert sorted(mix) == [0, 1, 2, 3]
    for q in reqs:
        alone = serve.Server(max_slots=1, precision=prec, keep_fields=True).run([serve.Request(q.prob, 0.0, q.rid)])[0]
        m = mix[q.rid]
        assert m.em_steps == q.prob.n_em_steps
        np.testing.assert_array_equal(m.theta, alone.theta)
        np.testing.assert_array_equal(m.vm, alone.vm)
        assert m.cg_relres <= q.prob.cg_rtol
        assert m.latency > 0 and m.finished >= m.admitted >= m.arrival - 1e-9
