"""Temporal blocking of the EM march (two steps as a wavefront over z-slabs,
`em_slabs`): every tile computes what it computes in a one-step launch, so
the state after any number of steps must be bitwise that of one launch per
step -- fields, the previous field, temperature, the Joule sum, the
displacement and von Mises stress, and the history records.  Cases: both
precisions, slab counts from the degenerate 2 (no overlap) to more slabs
than z-chunks, odd step counts, thermal steps and history records that
break pairs, closed-form waves sampled on the device (the wave table must
cover both steps of a pair), and the 256x256x64 slice in the launch
configuration the benchmark times."""
import sys

import numpy as np
import pytest

import paper_2603_07038_amd as etm
import workloads as W

pytestmark = pytest.mark.gpu
PS = 1e-12

FIELDS = [etm.ETM_FIELD_EX, etm.ETM_FIELD_EY, etm.ETM_FIELD_EZ, etm.ETM_FIELD_EX_PREV, etm.ETM_FIELD_EY_PREV,
          etm.ETM_FIELD_EZ_PREV, etm.ETM_FIELD_THETA, etm.ETM_FIELD_PSUM]
MECH = [etm.ETM_FIELD_UX, etm.ETM_FIELD_UY, etm.ETM_FIELD_UZ, etm.ETM_FIELD_VM]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(prob, precision, slabs, chunks, J=None, device_waves=False, history=True):
    dt = etm.cfl_dt(prob)
    n = sum(chunks)
    if J is None and not device_waves:
        J = prob.sample_J_half(dt, n + 1)
    pl = etm.Plan(prob, J, dt=dt, precision=precision, n_steps=n, history=history, device_waves=device_waves,
                  em_slabs=slabs)
    for c in chunks:
        pl.advance(c)
    info = pl.sync()
    out = {f: pl.read(f) for f in FIELDS}
    if prob.mech_every_thermal:
        out.update({f: pl.read(f) for f in MECH})
    if history:
        out["hist"] = pl.history()
    return out, info


def _same(a, b, label):
    for k in a:
        if k == "hist":
            assert a[k].shape == b[k].shape and a[k].shape[0] > 0, label
            np.testing.assert_array_equal(a[k], b[k], err_msg=f"{label} history")
        else:
            np.testing.assert_array_equal(a[k], b[k], err_msg=f"{label} field {k}")


def _package(seed, n=44, nz=30, excitation=None, t_origin=0.0):
    kw = {} if excitation is None else {"excitation": excitation, "t_origin": t_origin}
    p = W.package(n, n - 4, nz, seed, bump_pitch_um=14, bump_cells=6, max_traces=6, em_per_thermal=8, **kw)
    p.mech_every_thermal = 1
    p.history_stride = 5
    p.probes = np.array([[0, 5, 6, 3], [2, 20, 17, 11], [3, 9, 30, 14]], dtype=np.int64)
    return p


@pytest.mark.parametrize("precision", [etm.ETM_PREC_MIXED, etm.ETM_PREC_FP64])
def test_pairs_bitwise_equal_one_step_launches(precision):
    p = _package(31)
    chunks = [7, 12, 1, 19]            # odd counts; thermal steps every 8, records every 5
    ref, info0 = _run(p, precision, 0, chunks)
    assert float(np.abs(ref[etm.ETM_FIELD_THETA]).max()) > 0.0 and info0["n_solves"] >= 4
    for slabs in (2, 3, 5, 64):
        _say(f"[temporal] precision={precision} slabs={slabs}")
        got, info = _run(p, precision, slabs, chunks)
        assert info["step"] == info0["step"] and info["cg_iters_total"] == info0["cg_iters_total"]
        _same(got, ref, f"slabs={slabs}")


def test_pairs_with_device_sampled_waves():
    # a time origin that puts the trigger and the burst inside the window
    p = _package(32, n=40, nz=28, excitation="paper", t_origin=35 * PS)
    p.mech_every_thermal = 0
    chunks = [1021, 6]                 # the pair at steps 1023-1024 crosses a sampled-wave block
    ref, _ = _run(p, etm.ETM_PREC_MIXED, 0, chunks, device_waves=True, history=False)
    assert float(np.abs(ref[etm.ETM_FIELD_EX]).max()) > 0.0
    for slabs in (3, 8):
        _say(f"[temporal] device waves slabs={slabs}")
        got, _ = _run(p, etm.ETM_PREC_MIXED, slabs, chunks, device_waves=True, history=False)
        _same(got, ref, f"device waves slabs={slabs}")


def test_pairs_on_the_full_slice():
    p = W.config2()
    p.mech_every_thermal = 0
    p.history_stride = 0
    chunks = [9]
    _say("[temporal] slice 256x256x64 mixed, slabs=8")
    ref, _ = _run(p, etm.ETM_PREC_MIXED, 0, chunks, history=False)
    got, _ = _run(p, etm.ETM_PREC_MIXED, 8, chunks, history=False)
    _same(got, ref, "slice")

