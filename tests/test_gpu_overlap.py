"""Overlapped mechanical solves (`mech_overlap`, the default): a scheduled
solve runs on a side stream while the EM steps up to the next thermal step
or history record run on the plan's stream.  The solve reads only the
temperature of its own thermal step and the march never reads the
displacement, so every output must be bitwise that of the serial order --
fields, the previous field, temperature, the Joule sum, displacement, von
Mises stress, histories and CG iteration counts -- over many blocks in one
advance call, with history records inside and at thermal steps, with a
solve at every thermal step and at every second one, in both precisions,
and together with the two-step slab wavefront."""
import sys

import numpy as np
import pytest

import paper_2603_07038_amd as etm
import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = [etm.ETM_FIELD_EX, etm.ETM_FIELD_EY, etm.ETM_FIELD_EZ, etm.ETM_FIELD_EX_PREV, etm.ETM_FIELD_EY_PREV,
          etm.ETM_FIELD_EZ_PREV, etm.ETM_FIELD_THETA, etm.ETM_FIELD_PSUM, etm.ETM_FIELD_UX, etm.ETM_FIELD_UY,
          etm.ETM_FIELD_UZ, etm.ETM_FIELD_VM]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _package(seed, every=1, stride=6):
    p = W.package(44, 40, 30, seed, bump_pitch_um=14, bump_cells=6, max_traces=6, em_per_thermal=8)
    p.mech_every_thermal = every
    p.history_stride = stride
    p.probes = np.array([[0, 5, 6, 3], [3, 9, 30, 14]], dtype=np.int64)
    return p


def _run(prob, precision, chunks, **kw):
    dt = etm.cfl_dt(prob)
    n = sum(chunks)
    J = prob.sample_J_half(dt, n + 1)
    pl = etm.Plan(prob, J, dt=dt, precision=precision, n_steps=n, history=True, **kw)
    for c in chunks:
        pl.advance(c)
    info = pl.sync()
    out = {f: pl.read(f) for f in FIELDS}
    out["hist"] = pl.history()
    return out, info


@pytest.mark.parametrize("precision", [etm.ETM_PREC_MIXED, etm.ETM_PREC_FP64])
@pytest.mark.parametrize("every,stride,slabs", [(1, 6, 0), (2, 8, 0), (1, 0, 3)])
def test_overlapped_solves_bitwise_equal_serial(precision, every, stride, slabs):
    p = _package(41, every, stride)
    chunks = [45, 3, 20]               # many blocks per call; a call ending on a thermal step
    _say(f"[overlap] precision={precision} every={every} stride={stride} slabs={slabs}")
    ref, i0 = _run(p, precision, chunks, mech_overlap=0, em_slabs=slabs)
    got, i1 = _run(p, precision, chunks, mech_overlap=1, em_slabs=slabs)
    assert i0["n_solves"] == i1["n_solves"] >= 4 and i0["cg_iters_total"] == i1["cg_iters_total"]
    assert float(np.abs(ref[etm.ETM_FIELD_VM]).max()) > 0.0
    for k in ref:
        np.testing.assert_array_equal(got[k], ref[k], err_msg=f"field {k}")
