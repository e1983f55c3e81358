"""The allocation-free batched advance (etm_batch_advance_noalloc): its
results are bitwise those of etm_batch_advance on the same variants (same
kernels, same work-list order), over two calls in a row from the library's
fixed device scratch, the second with a smaller batch than the first, and it
rejects inputs beyond its stated limits before enqueuing anything."""
import numpy as np
import pytest

import paper_2603_07038_amd as etm
import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = (etm.ETM_FIELD_EX, etm.ETM_FIELD_EY, etm.ETM_FIELD_EZ, etm.ETM_FIELD_EX_PREV, etm.ETM_FIELD_THETA,
          etm.ETM_FIELD_PSUM)


def _problems(shapes, seed0, n_steps):
    return [W.random_problem(seed0 + v, *s, n_steps=n_steps, R=[4, 6, 5][v % 3], n_ports=2, amp=3e10,
                             em_bc=(0,) * 6) for v, s in enumerate(shapes)]


def _run(probs, prec, chunks, noalloc):
    dts = [etm.cfl_dt(p) for p in probs]
    n = sum(chunks)
    plans = [etm.Plan(p, p.sample_J_half(dt, n), dt=dt, precision=prec, n_steps=n, history=True)
             for p, dt in zip(probs, dts)]
    b = etm.Batch(8)
    for pl in plans:
        b.attach(pl)
    for c in chunks:
        (b.advance_noalloc if noalloc else b.advance)(c)
    out = []
    for pl in plans:
        info = pl.sync()
        assert info["step"] == n
        out.append([pl.read(f) for f in FIELDS] + [pl.history()])
    del b
    return out


@pytest.mark.parametrize("prec", [etm.ETM_PREC_FP64, etm.ETM_PREC_MIXED])
def test_noalloc_matches_graph_batch_on_two_calls(prec):
    # first call: four uneven variants (several x tiles, a ragged last tile,
    # more z planes than one chunk), thermal steps and history records inside
    big = _problems([(130, 9, 6), (70, 6, 4), (33, 40, 9), (9, 7, 5)], 900, 47)
    # second call: a smaller batch (fewer variants, fewer tiles) after the big
    # one left its descriptors and longer work list in the scratch array
    small = _problems([(5, 5, 9), (20, 3, 4)], 950, 31)
    for name, probs, chunks in (("big", big, (19, 28)), ("small", small, (31,))):
        print(f"[no-alloc] prec={prec} {name} {[p.name for p in probs]} chunks={chunks}", flush=True)
        got = _run(probs, prec, chunks, noalloc=True)
        ref = _run(probs, prec, chunks, noalloc=False)
        for g, r in zip(got, ref):
            for a, b in zip(g, r):
                np.testing.assert_array_equal(a, b)
    # the small batch again, now right after the big one in the same process
    # state: still bitwise
    again = _run(small, prec, (31,), noalloc=True)
    ref = _run(small, prec, (31,), noalloc=False)
    for g, r in zip(again, ref):
        for a, b in zip(g, r):
            np.testing.assert_array_equal(a, b)


def test_noalloc_rejects_beyond_its_limits():
    p = W.random_problem(990, 4, 4, 3, n_steps=8, R=4, n_ports=1, em_bc=(0,) * 6)
    dt = etm.cfl_dt(p)
    J = p.sample_J_half(dt, 8)
    # more variants than the scratch holds descriptors for
    plans = [etm.Plan(p, J, dt=dt, n_steps=8, history=False) for _ in range(65)]
    b = etm.Batch(80)
    for pl in plans:
        b.attach(pl)
    with pytest.raises(etm.EtmError) as ei:
        b.advance_noalloc(4)
    assert ei.value.status == etm.ETM_E_INVAL and "at most 64" in str(ei.value)
    for pl in plans:
        assert pl.sync()["step"] == 0          # nothing was enqueued
    del b
    # a plan that schedules mechanical solves
    q = W.random_problem(991, 4, 4, 3, n_steps=8, R=4, n_ports=1, em_bc=(0,) * 6)
    q.mech_every_thermal = 1
    pl = etm.Plan(q, J, dt=dt, n_steps=8, history=False)
    b = etm.Batch(2)
    b.attach(pl)
    with pytest.raises(etm.EtmError) as ei:
        b.advance_noalloc(4)
    assert ei.value.status == etm.ETM_E_INVAL and "mech_every_thermal" in str(ei.value)
    assert pl.sync()["step"] == 0
