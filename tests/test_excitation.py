"""The excitation scheme of Sec. III-B (CPU): closed-form facts of each
waveform, the jitter bounds, the port layout (differential pairs, balanced
Ground-Signal-Ground groups) and the library's host-side validation of
closed-form wave records."""
import ctypes as C
import dataclasses

import numpy as np
import pytest

import paper_2603_07038_amd as etm
import workloads as W

PS = 1e-12


def test_ricker_peak_zero_crossings_window_and_zero_mean():
    w = W.Wave("ricker_w", amp=2.5, t0=40 * PS, tau=1.0 / (np.pi * 50e9), t_on=20 * PS, t_off=60 * PS)
    assert w(np.array([40 * PS]))[0] == 2.5
    z = w.tau / np.sqrt(2.0)  # 1 - 2 u^2 = 0
    assert np.allclose(w(np.array([40 * PS - z, 40 * PS + z])), 0.0, atol=1e-14)
    assert np.all(w(np.array([19.99 * PS, 60 * PS, 70 * PS, -1 * PS])) == 0.0)
    # minima of (1 - 2u^2) e^{-u^2} at u^2 = 3/2, value -2 e^{-3/2}
    tm = 40 * PS + np.sqrt(1.5) * w.tau
    assert abs(w(np.array([tm]))[0] / 2.5 + 2.0 * np.exp(-1.5)) < 1e-12
    # zero mean: the window spans +-20 ps = +-3.14 widths, beyond which the
    # wavelet is below 1e-3 of its peak
    t = np.linspace(0, 100 * PS, 400001)
    assert abs(np.trapezoid(w(t), t)) / (2.5 * w.tau) < 2e-3


def test_sine_zeros_period_and_window():
    w = W.Wave("sine_w", amp=3.0, f0=5e9, t0=10 * PS, t_on=10 * PS, t_off=310 * PS)
    T = 1.0 / 5e9
    assert w(np.array([10 * PS]))[0] == 0.0
    assert abs(w(np.array([10 * PS + T / 4]))[0] - 3.0) < 1e-12
    t = np.linspace(20 * PS, 100 * PS, 7)
    assert np.allclose(w(t), w(t + T), atol=1e-12)
    assert w(np.array([9.9 * PS]))[0] == 0.0 and w(np.array([310 * PS]))[0] == 0.0


def test_gaussian_train_pulses_carrier_and_window():
    c = np.array([105, 155, 205]) * PS
    w = W.Wave("gauss_train", amp=1.5, f0=40e9, t0=80 * PS, tau=12 * PS, centers=c, t_on=80 * PS, t_off=230 * PS)
    # at a pulse centre the envelope is 1 (the neighbours add e^{-(50/12)^2} ~ 3e-8)
    for cc in c:
        v = w(np.array([cc]))[0]
        assert abs(v - 1.5 * np.cos(2 * np.pi * 40e9 * (cc - 80 * PS))) < 1.5 * 1e-7
    # halfway between pulses the envelope is 2 e^{-(25/12)^2}
    mid = 130 * PS
    env = w(np.array([mid]))[0] / (1.5 * np.cos(2 * np.pi * 40e9 * (mid - 80 * PS)))
    assert abs(env - 2 * np.exp(-(25 / 12) ** 2)) < 1e-9
    assert np.all(w(np.array([79 * PS, 230 * PS, 300 * PS])) == 0.0)


def test_paper_waves_follow_the_scheme_and_jitter_bounds():
    rng = np.random.Generator(np.random.PCG64(3))
    for _ in range(200):
        fa, fw, sh = W.paper_jitter(rng)
        assert 0.8 <= fa <= 1.2 and 0.9 <= fw <= 1.1 and -10 * PS <= sh <= 10 * PS
        tr = W.trigger_wave(1.0, (fa, fw, sh))
        assert tr.kind == "ricker_w" and tr.t0 == pytest.approx(40 * PS + sh)
        assert tr.t_on == pytest.approx(max(20 * PS + sh, 0)) and tr.t_off == pytest.approx(60 * PS + sh)
        assert tr.tau == pytest.approx(fw / (np.pi * 50e9)) and tr.amp == pytest.approx(fa)
        lg = W.logic_wave(2.0, (fa, fw, sh))
        assert lg.kind == "sine_w" and lg.f0 == 5e9 and lg.t_off == pytest.approx(300 * PS + sh)
        bu = W.burst_wave(2.0, (fa, fw, sh))
        assert bu.kind == "gauss_train" and bu.f0 == 40e9 and len(bu.centers) == 3
        assert np.allclose(bu.centers, (np.array([105, 155, 205]) * PS + sh))
        assert bu.tau == pytest.approx(12 * PS * fw)
        assert bu.t_on == pytest.approx(80 * PS + sh) and bu.t_off == pytest.approx(230 * PS + sh)
    # a later time origin shifts every wave and clips windows at t = 0
    w0 = W.logic_wave(1.0, (1.0, 1.0, 0.0))
    w1 = W.logic_wave(1.0, (1.0, 1.0, 0.0), t_origin=30 * PS)
    assert w1.t_on == 0.0 and w1.t_off == pytest.approx(270 * PS)
    t = np.array([5, 50, 100]) * PS
    expired = W.trigger_wave(1.0, (1.0, 1.0, 0.0), t_origin=95 * PS)
    assert expired.t_on == 0.0 and expired.t_off == 0.0 and not np.any(expired(t))
    assert np.allclose(w1(t), w0(t + 30 * PS))


def test_slice_layout_differential_pairs_and_balanced_gsg_groups():
    p = W.config2(excitation="paper")
    trig = [w for w in p.waves if w.kind == "ricker_w"]
    assert len(trig) == 16
    assert all((w.amp > 0) == (t % 2 == 0) for t, w in enumerate(p.waves[:16]))  # alternating along y
    assert {w.kind for w in p.waves[16:]} == {"sine_w", "gauss_train"}
    bump = p.port_dir[p.port_wave >= 16]
    assert np.all(bump == 0)  # x-directed feeding
    # per bump column the unjittered weights sum to zero (G-S-G current sinking)
    wid = p.port_wave >= 16
    cols = {}
    for i, wt in zip(p.port_i[wid], p.port_weight[wid]):
        cols[int(i)] = cols.get(int(i), 0.0) + float(wt)
    assert len(cols) == 8 and all(abs(v) < 1e-12 for v in cols.values())
    # logic die (left half) sine, HBM die (right half) burst
    for q in np.nonzero(wid)[0]:
        w = p.waves[p.port_wave[q]]
        assert (w.kind == "sine_w") == (p.port_i[q] < 128)
    # deterministic
    p2 = W.config2(excitation="paper")
    assert all(a.amp == b.amp and a.t0 == b.t0 and a.tau == b.tau for a, b in zip(p.waves, p2.waves))


def test_package_layout_has_one_wave_per_port_group():
    p = W.package(64, 64, 32, 5, bump_pitch_um=16, bump_cells=8, excitation="paper")
    kinds = [w.kind for w in p.waves]
    assert set(kinds) == {"ricker_w", "sine_w", "gauss_train"}
    assert np.all(np.isin(p.port_wave, np.arange(len(p.waves))))
    assert len(np.unique(p.port_wave)) == len(p.waves)


def _create(prob, waves=None, **kw):
    L = etm.load()
    inp = etm._Inputs(prob, None, device_waves=True)
    if waves is not None:
        inp.waves = (etm.etm_wave * len(waves))(*waves)
        inp.src.analytic = inp.waves
        inp.src.n_analytic = len(waves)
    o, keep = etm.make_opts(prob, **kw)
    h = C.c_void_p()
    st = L.etm_plan_create(C.byref(inp.mesh), inp.mats, int(prob.props.shape[0]), C.byref(inp.src), C.byref(o),
                           C.byref(h))
    if st == etm.ETM_OK:
        L.etm_plan_destroy(h)
    return st


def test_library_accepts_and_validates_closed_form_waves():
    p = W.package(40, 40, 24, 7, bump_pitch_um=16, bump_cells=8, max_traces=4, excitation="paper")
    assert _create(p) == etm.ETM_OK, etm.load().etm_last_error()
    n = len(p.waves)

    def rec(**kw):
        d = dict(kind=etm.ETM_WAVE_RICKER, n_pulses=0, amp=1.0, t0=1e-12, width=1e-12, freq=0.0, t_on=0.0,
                 t_off=1e-11)
        d.update(kw)
        pt = (C.c_double * 8)(*([1e-12] * 8))
        return etm.etm_wave(d["kind"], d["n_pulses"], d["amp"], d["t0"], d["width"], d["freq"], d["t_on"],
                            d["t_off"], pt)

    good = [rec()] * n
    assert _create(p, good) == etm.ETM_OK
    for bad in (rec(kind=7), rec(kind=etm.ETM_WAVE_GAUSS_TRAIN, n_pulses=0),
                rec(kind=etm.ETM_WAVE_GAUSS_TRAIN, n_pulses=9), rec(width=0.0), rec(t_on=2e-11),
                rec(amp=float("nan"))):
        assert _create(p, [bad] + good[1:]) == etm.ETM_E_INVAL
    # an empty window is a wave that is always zero; a sine needs no width;
    # a train with 1..8 pulses is fine
    assert _create(p, [rec(t_on=1e-11)] + good[1:]) == etm.ETM_OK
    assert _create(p, [rec(kind=etm.ETM_WAVE_SINE, width=0.0, freq=5e9)] + good[1:]) == etm.ETM_OK
    assert _create(p, [rec(kind=etm.ETM_WAVE_GAUSS_TRAIN, n_pulses=8, freq=4e10)] + good[1:]) == etm.ETM_OK
    # a port that names a wave beyond the closed-form list
    assert _create(p, good[:-1]) == etm.ETM_E_INVAL
