"""Host logic of the serving measurements (CPU only): the per-rate summary
of answered requests and the knee of a rate sweep."""
import importlib.util
import os

import numpy as np
import pytest

from paper_2603_07038_amd import serve

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _result(rid, latency, status="ok", cg=20, cells=1000, steps=64):
    return serve.Result(rid=rid, name=f"r{rid}", cells=cells, em_steps=steps, arrival=1.0, admitted=1.5,
                        finished=1.0 + latency, theta_max=0.0, vm_max=0.0, cg_iters=cg, cg_relres=1e-9,
                        status=status)


def test_summary_counts_only_answered_requests():
    res = [_result(i, 0.1 * (i + 1), cg=10 + i) for i in range(10)]
    res.append(_result(10, 99.0, status="rejected", cg=0))
    res.append(_result(11, 50.0, status="error", cg=0))
    s = serve.summarize(res, wall=20.0)
    lat = np.array([0.1 * (i + 1) for i in range(10)])
    assert (s["requests"], s["completed"], s["rejected"], s["failed"]) == (12, 10, 1, 1)
    assert s["p50_s"] == pytest.approx(np.percentile(lat, 50))
    assert s["p99_s"] == pytest.approx(np.percentile(lat, 99))
    assert s["mean_s"] == pytest.approx(lat.mean())
    assert s["designs_per_hour"] == pytest.approx(10 / 20.0 * 3600.0)
    assert s["cell_steps"] == 10 * 1000 * 64
    assert s["cg_iters_mean"] == pytest.approx(14.5) and s["cg_iters_max"] == 19


def test_summary_with_nothing_answered():
    s = serve.summarize([_result(0, 1.0, status="rejected")], wall=1.0)
    assert s["completed"] == 0 and s["designs_per_hour"] == 0.0
    assert s["cg_iters_mean"] is None and s["cg_iters_max"] is None


def test_knee_rule():
    knee = _bench().serving_knee
    v = lambda p99, frac: {"p99_s": p99, "sustained_frac": frac}
    # latency within 2x up to 5 req/s, then the queue grows
    assert knee([(10.0, v(28.0, 0.49)), (2.0, v(4.8, 1.01)), (5.0, v(8.5, 0.94)), (20.0, v(39.0, 0.25))]) == 5.0
    # p99 fine but the answered rate falls short at 5 req/s
    assert knee([(2.0, v(4.8, 1.0)), (5.0, v(6.0, 0.85))]) == 2.0
    # the lowest rate itself not sustained: no knee
    assert knee([(2.0, v(4.8, 0.5)), (5.0, v(30.0, 0.2))]) is None
    # a missing sustained fraction counts as not sustained
    assert knee([(2.0, v(1.0, 1.0)), (5.0, v(1.5, None))]) == 2.0
