"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle,
element by element on the same seeded inputs.

Tolerances: the FP64 path must agree to 1e-9 of the field's max norm (the
two sides differ only in rounding order); the mixed path to 1e-6 on the
temperature rise and 1e-5 on the peak von Mises stress."""
import sys

import numpy as np
import pytest

import oracle
import paper_2603_07038_amd as etm
import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(a, b):
    scale = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / scale)


def e_err(eg, eo):
    scale = max(max(np.abs(x).max() for x in eo), 1e-300)
    return max(float(np.abs(a - b).max()) for a, b in zip(eg, eo)) / scale


def run_pair(prob, n_steps, precision=etm.ETM_PREC_FP64, stride=0):
    o = oracle.Oracle(prob)
    dt = o.cfl_dt()
    J = prob.sample_J_half(dt, n_steps)
    _say(f"[parity] {prob.name} steps={n_steps} prec={precision} R={prob.em_per_thermal}")
    plan = etm.Plan(prob, J, dt=dt, precision=precision, n_steps=n_steps, history=stride > 0)
    plan.advance(n_steps)
    info = plan.sync()
    st, hist = o.run(dt, n_steps, J, stride=stride, probes=prob.probes)
    return plan, o, st, hist, info, dt, J


SHAPES = [(5, 4, 3), (70, 9, 4), (130, 5, 3), (17, 33, 6)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("seed", [1, 2])
def test_fp64_march_matches_oracle(shape, seed):
    prob = W.random_problem(100 * seed + shape[0], *shape, n_steps=48, R=5, n_ports=3, amp=3e10)
    plan, o, st, hist, info, dt, J = run_pair(prob, 48)
    assert info["step"] == 48
    assert e_err(plan.e(), st["e"]) < 1e-9
    assert e_err(plan.e_prev(), st["e_prev"]) < 1e-9
    assert rel_err(plan.read(etm.ETM_FIELD_THETA), st["theta"]) < 1e-9
    assert rel_err(plan.read(etm.ETM_FIELD_PSUM), st["psum"]) < 1e-9


def test_fp64_history_matches_oracle():
    prob = W.random_problem(7, 9, 7, 5, n_steps=40, R=4, n_ports=2, amp=3e10)
    prob.history_stride = 5
    plan, o, st, hist, info, dt, J = run_pair(prob, 40, stride=5)
    hg = plan.history()
    assert hg.shape == hist.shape
    np.testing.assert_array_equal(hg[:, 0], hist[:, 0])
    for col in range(1, hist.shape[1]):
        assert rel_err(hg[:, col], hist[:, col]) < 1e-9, col


def test_pkg32_fp64_full_window():
    """The 32x32x16 PEC package, 2000 steps, R = 200, then the clamped
    mechanical solve: e, theta, displacement and von Mises against the oracle."""
    prob = W.config1()
    plan, o, st, hist, info, dt, J = run_pair(prob, prob.n_em_steps)
    assert e_err(plan.e(), st["e"]) < 1e-9
    assert rel_err(plan.read(etm.ETM_FIELD_THETA), st["theta"]) < 1e-9
    plan.mech_solve()
    info = plan.sync()
    assert info["cg_relres"] <= prob.cg_rtol
    mask = o.mech_mask()
    q, it, rr = o.mech_solve(st["theta"], mask, rtol=1e-12)
    vm_o = o.von_mises(st["theta"], q)
    _say(f"[parity] gpu cg iters {info['cg_iters']} oracle {it}")
    assert rel_err(plan.u(), q) < 1e-6
    assert rel_err(plan.read(etm.ETM_FIELD_VM), vm_o) < 1e-6


@pytest.mark.parametrize("seed,shape,bc", [(1, (6, 5, 4), W.MECH_KINEMATIC), (2, (9, 7, 4), W.MECH_CLAMP_ZMIN),
                                            (3, (70, 6, 3), W.MECH_KINEMATIC)])
def test_mech_solve_matches_oracle(seed, shape, bc):
    prob = W.random_problem(seed, *shape, n_steps=4, R=2, mech_bc=bc, void_top=1)
    prob.cg_rtol = 1e-12
    o = oracle.Oracle(prob)
    dt = o.cfl_dt()
    J = prob.sample_J_half(dt, 4)
    plan = etm.Plan(prob, J, dt=dt, n_steps=4)
    rng = np.random.default_rng(seed)
    th = rng.uniform(0, 30, o.node_shape)
    plan.write(etm.ETM_FIELD_THETA, th)
    plan.mech_solve()
    info = plan.sync()
    f = o.mech_rhs(th, o.mech_mask())
    fg = np.stack([plan.read(etm.ETM_FIELD_FX), plan.read(etm.ETM_FIELD_FY), plan.read(etm.ETM_FIELD_FZ)], -1)
    assert rel_err(fg, f) < 1e-12
    q, it, rr = o.mech_solve(th, o.mech_mask(), rtol=1e-13)
    assert rel_err(plan.u(), q) < 1e-8
    assert rel_err(plan.read(etm.ETM_FIELD_VM), o.von_mises(th, q)) < 1e-8
    # the GPU solution satisfies the oracle's equations
    res = f - o.mech_apply(o.mech_mask(), plan.u())
    assert np.linalg.norm(res) <= 2e-12 * np.linalg.norm(f)


def test_mixed_precision_tolerances_pkg32():
    """Mixed path (FP32 fields in increment form, FP64 temperature and Joule
    accumulation, FP32 CG with FP64 refinement): temperature rise within
    1e-6 and peak von Mises within 1e-5 of the FP64 oracle."""
    prob = W.config1()
    plan, o, st, hist, info, dt, J = run_pair(prob, prob.n_em_steps, precision=etm.ETM_PREC_MIXED)
    th_err = rel_err(plan.read(etm.ETM_FIELD_THETA), st["theta"])
    plan.mech_solve()
    info = plan.sync()
    q, it, rr = o.mech_solve(st["theta"], o.mech_mask(), rtol=1e-12)
    vm_o = o.von_mises(st["theta"], q)
    vm_g = plan.read(etm.ETM_FIELD_VM)
    vm_err = abs(vm_g.max() - vm_o.max()) / vm_o.max()
    _say(f"[parity] mixed theta err {th_err:.3e} e err {e_err(plan.e(), st['e']):.3e} "
         f"peak VM err {vm_err:.3e} field VM err {rel_err(vm_g, vm_o):.3e} cg {info['cg_iters']}/{info['cg_outer']}")
    assert th_err < 1e-6
    assert vm_err < 1e-5


def test_checkpoint_restore_is_bitwise():
    prob = W.random_problem(12, 11, 6, 5, n_steps=30, R=4, n_ports=2, amp=3e10)
    o = oracle.Oracle(prob)
    dt = o.cfl_dt()
    J = prob.sample_J_half(dt, 30)
    a = etm.Plan(prob, J, dt=dt, n_steps=30)
    a.advance(13)
    ck = a.checkpoint()
    a.advance(17)
    ea, tha = a.e(), a.read(etm.ETM_FIELD_THETA)
    b = etm.Plan(prob, J, dt=dt, n_steps=30)
    b.restore(ck)
    b.advance(17)
    for x, y in zip(ea, b.e()):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(tha, b.read(etm.ETM_FIELD_THETA))


def test_chunked_advance_and_rerun_are_bitwise_equal():
    prob = W.random_problem(13, 70, 5, 4, n_steps=24, R=5, n_ports=2, amp=3e10)
    dt = etm.cfl_dt(prob)
    J = prob.sample_J_half(dt, 24)
    a = etm.Plan(prob, J, dt=dt, n_steps=24)
    a.advance(24)
    b = etm.Plan(prob, J, dt=dt, n_steps=24)
    for n in (7, 11, 6):
        b.advance(n)
    for x, y in zip(a.e(), b.e()):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(a.read(etm.ETM_FIELD_THETA), b.read(etm.ETM_FIELD_THETA))


def _mixed_vs_oracle(prob, n_steps):
    o = oracle.Oracle(prob)
    dt = o.cfl_dt()
    J = prob.sample_J_half(dt, n_steps)
    plan = etm.Plan(prob, J, dt=dt, precision=etm.ETM_PREC_MIXED, n_steps=n_steps, history=False)
    plan.advance(n_steps)
    plan.sync()
    st, _ = o.run(dt, n_steps, J)
    return plan, st, o


def test_mixed_leapfrog_accuracy_on_a_prbs_package():
    """A PRBS-driven package over 2048 steps (Norton ports, Cu traces and
    bumps in dielectrics): the FP32 leapfrog state keeps the temperature rise
    within 1e-6 and the field within 1e-5 of the FP64 oracle."""
    prob = W.package(40, 40, 24, 77, bump_pitch_um=20, bump_cells=6, trace_width=2, trace_pitch=4,
                     n_trace_layers=2, max_traces=6, n_bits=128, steps_per_bit=16, em_per_thermal=256)
    plan, st, o = _mixed_vs_oracle(prob, 2048)
    th_err = rel_err(plan.read(etm.ETM_FIELD_THETA), st["theta"])
    ee = e_err(plan.e(), st["e"])
    _say(f"[parity] prbs package mixed theta err {th_err:.3e} e err {ee:.3e}")
    assert th_err < 1e-6
    assert ee < 1e-5
    # e^{n-1} is the previous field of the march
    assert e_err(plan.e_prev(), st["e_prev"]) < 1e-5


def test_mixed_leapfrog_tracks_sigma_of_T_under_strong_heating():
    """The trace case driven 300x harder (tens of mK per thermal block, Cu
    conductivity 3.9e-3/K): the leapfrog correction K keeps the mixed path on
    the three-level scheme of Eq. (2) with sigma(T^n)."""
    prob = W.config1()
    for w in prob.waves:
        w.amp *= 300.0
    plan, st, o = _mixed_vs_oracle(prob, prob.n_em_steps)
    th = st["theta"]
    th_err = rel_err(plan.read(etm.ETM_FIELD_THETA), th)
    _say(f"[parity] strong heating theta max {th.max():.3e} K, mixed theta err {th_err:.3e}")
    assert th.max() > 1e-2
    assert th_err < 1e-6


def test_mixed_e_fields_are_not_writable():
    prob = W.random_problem(3, 6, 5, 4, n_steps=4, R=2)
    plan = etm.Plan(prob, prob.sample_J_half(etm.cfl_dt(prob), 4), precision=etm.ETM_PREC_MIXED, n_steps=4)
    with pytest.raises(etm.EtmError):
        plan.write(etm.ETM_FIELD_EX, np.zeros(plan.field_shape(etm.ETM_FIELD_EX)))
