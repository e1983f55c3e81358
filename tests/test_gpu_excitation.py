"""The excitation scheme of Sec. III-B on the GPU: closed-form waves evaluated
on the device against the same waves sampled on the host (tabulated path)
and against the oracle, which marches with the sampled values; both
precisions and the batched path.  Time origins put the Ricker trigger and
the Gaussian-pulse-train burst inside the simulated window (the 5 GHz sine
runs throughout)."""
import sys

import numpy as np
import pytest

import oracle
import paper_2603_07038_amd as etm
import workloads as W

pytestmark = pytest.mark.gpu
PS = 1e-12
N_STEPS = 300


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _problem(t_origin, seed=11, n=40):
    p = W.package(n, n, 32, seed, bump_pitch_um=14, bump_cells=6, max_traces=8, excitation="paper",
                  t_origin=t_origin, em_per_thermal=64)
    p.n_em_steps = N_STEPS
    return p


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _e_rel(ea, eb):
    s = max(float(np.abs(x).max()) for x in eb)
    return max(float(np.abs(x - y).max()) for x, y in zip(ea, eb)) / s


@pytest.mark.parametrize("t_origin", [35 * PS, 95 * PS])
def test_device_waves_match_sampled_waves_and_oracle_fp64(t_origin):
    p = _problem(t_origin)
    dt = etm.cfl_dt(p)
    J = p.sample_J_half(dt, N_STEPS)
    _say(f"[excitation] fp64 t_origin={t_origin:.3g} ports={p.n_ports} waves={len(p.waves)}")
    a = etm.Plan(p, None, dt=dt, precision=etm.ETM_PREC_FP64, n_steps=N_STEPS, history=False, device_waves=True)
    b = etm.Plan(p, J, dt=dt, precision=etm.ETM_PREC_FP64, n_steps=N_STEPS, history=False)
    a.advance(N_STEPS)
    b.advance(N_STEPS)
    a.sync()
    b.sync()
    st, _ = oracle.Oracle(p).run(dt, N_STEPS, J)
    ea, eb = a.e(), b.e()
    assert max(float(np.abs(x).max()) for x in st["e"]) > 0.0
    d_tab = _e_rel(ea, eb)
    d_orc = _e_rel(ea, st["e"])
    th = _rel(a.read(etm.ETM_FIELD_THETA), st["theta"])
    ps = _rel(a.read(etm.ETM_FIELD_PSUM), st["psum"])
    _say(f"[excitation]   device vs table {d_tab:.2e}  vs oracle e {d_orc:.2e} theta {th:.2e} psum {ps:.2e}")
    assert d_tab < 1e-12
    assert d_orc < 1e-9 and th < 1e-9 and ps < 1e-9


def test_device_waves_mixed_precision_against_oracle():
    p = _problem(95 * PS)
    dt = etm.cfl_dt(p)
    J = p.sample_J_half(dt, N_STEPS)
    a = etm.Plan(p, None, dt=dt, precision=etm.ETM_PREC_MIXED, n_steps=N_STEPS, history=False, device_waves=True)
    a.advance(N_STEPS)
    a.sync()
    st, _ = oracle.Oracle(p).run(dt, N_STEPS, J)
    d = _e_rel(a.e(), st["e"])
    th = _rel(a.read(etm.ETM_FIELD_THETA), st["theta"])
    _say(f"[excitation] mixed vs oracle e {d:.2e} theta {th:.2e}")
    assert d < 1e-5 and th < 1e-6


def test_batch_with_device_waves_matches_solo_bitwise():
    probs = [_problem(35 * PS, seed=21, n=36), _problem(95 * PS, seed=22, n=44)]
    dts = [etm.cfl_dt(p) for p in probs]
    b = etm.Batch(4)
    plans = [etm.Plan(p, None, dt=dt, precision=etm.ETM_PREC_MIXED, n_steps=N_STEPS, history=False,
                      device_waves=True) for p, dt in zip(probs, dts)]
    for pl in plans:
        b.attach(pl)
    b.advance(N_STEPS)
    for pl in plans:
        pl.sync()
    for p, dt, pl in zip(probs, dts, plans):
        solo = etm.Plan(p, None, dt=dt, precision=etm.ETM_PREC_MIXED, n_steps=N_STEPS, history=False,
                        device_waves=True)
        solo.advance(N_STEPS)
        solo.sync()
        for x, y in zip(pl.e(), solo.e()):
            np.testing.assert_array_equal(x, y)
        np.testing.assert_array_equal(pl.read(etm.ETM_FIELD_THETA), solo.read(etm.ETM_FIELD_THETA))
