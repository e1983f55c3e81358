"""Batched variants: each variant's fields after a batched run are bitwise
those of its solo run, for both precisions, with uneven sizes, thermal
blocks inside the run and graph-replayed segments."""
import json
import sys

import numpy as np
import pytest

import paper_2603_07038_amd as etm
import workloads as W

pytestmark = pytest.mark.gpu


def _variants(n):
    out = []
    for v in range(n):
        shape = [(9, 7, 5), (70, 6, 4), (33, 40, 3), (5, 5, 9), (130, 9, 6)][v % 5]
        p = W.random_problem(500 + v, *shape, n_steps=60, R=[4, 6, 5][v % 3], n_ports=2, amp=3e10, em_bc=(0,) * 6)
        out.append(p)
    return out


def _state(plan):
    return [plan.read(f) for f in (etm.ETM_FIELD_EX, etm.ETM_FIELD_EY, etm.ETM_FIELD_EZ, etm.ETM_FIELD_THETA,
                                   etm.ETM_FIELD_PSUM)]


def _size_class(p):
    return int(np.floor(np.log2(p.n_cells)))


@pytest.mark.parametrize("prec,layout", [(etm.ETM_PREC_FP64, None), (etm.ETM_PREC_FP64, 0),
                                         (etm.ETM_PREC_MIXED, None), (etm.ETM_PREC_MIXED, 1),
                                         (etm.ETM_PREC_MIXED, 2)])
def test_batch_matches_solo_bitwise(prec, layout):
    """layout None: the default tuning table; 1 / 2: every variant forced to
    runs over the x-fastest plane / row segments (with odd z-chunks); 0 (FP64):
    odd z-chunks from the FP64 chunk map."""
    probs = _variants(5)
    print(f"[batch] prec={prec} layout={layout} variants={[p.name for p in probs]}", flush=True)
    dts = [etm.cfl_dt(p) for p in probs]
    Js = [p.sample_J_half(dt, 60) for p, dt in zip(probs, dts)]
    solo = []
    for p, dt, J in zip(probs, dts, Js):
        pl = etm.Plan(p, J, dt=dt, precision=prec, n_steps=60, history=False)
        pl.advance(23)
        pl.advance(37)
        solo.append(_state(pl))
    classes = sorted({_size_class(p) for p in probs})
    odd = {str(c): [3, 5, 2][c % 3] for c in classes}
    if layout is None:
        b = etm.Batch(8)
    elif layout == 0:
        b = etm.Batch(8, json.dumps({"kchunk_fp64": odd}))
    else:
        b = etm.Batch(8, json.dumps({"kchunk": odd, "layout": {str(c): layout for c in classes}}))
    plans = []
    for p, dt, J in zip(probs, dts, Js):
        pl = etm.Plan(p, J, dt=dt, precision=prec, n_steps=60, history=False)
        b.attach(pl)
        plans.append(pl)
    b.advance(17)
    b.advance(43)
    for pl, ref in zip(plans, solo):
        assert pl.sync()["step"] == 60
        for a, r in zip(_state(pl), ref):
            np.testing.assert_array_equal(a, r)


def test_batch_detach_and_continue_solo():
    probs = _variants(3)
    dts = [etm.cfl_dt(p) for p in probs]
    Js = [p.sample_J_half(dt, 60) for p, dt in zip(probs, dts)]
    ref = etm.Plan(probs[1], Js[1], dt=dts[1], n_steps=60, history=False)
    ref.advance(60)
    b = etm.Batch(4)
    plans = [etm.Plan(p, J, dt=dt, n_steps=60, history=False) for p, dt, J in zip(probs, dts, Js)]
    slots = [b.attach(pl) for pl in plans]
    b.advance(25)
    b.detach(slots[0])
    b.advance(10)
    plans[1].advance(25)   # continue solo
    for a, r in zip(_state(plans[1]), _state(ref)):
        np.testing.assert_array_equal(a, r)
