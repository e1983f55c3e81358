"""GPU parity against the FP64 oracle for the paths that other tests only
compare with another HIP run: the paper's synchronous schedule (one thermal
step per EM step, Sec. II-A and Eq. 5, R = 1), mixed-precision histories,
batched variants, served requests, the two-step slab wavefront and
mechanical solves overlapped with the march.  Each case marches the oracle
on the same seeded inputs and compares element by element.

Bars: FP64 path e, e^{n-1}, theta and the Joule block sum within 1e-9 of
the field's max norm (rounding order only); displacement and von Mises
within 1e-6 after a solve to rtol 1e-8 (the oracle solves to 1e-12).
Mixed path: temperature rise within 1e-6, e within 1e-5 of the field's max
norm, peak von Mises within 1e-5; history columns as stated in the test."""
import functools
import sys

import numpy as np
import pytest

import oracle
import paper_2603_07038_amd as etm
import workloads as W
from paper_2603_07038_amd import serve

pytestmark = pytest.mark.gpu
FP64, MIXED = etm.ETM_PREC_FP64, etm.ETM_PREC_MIXED


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300))


def e_err(eg, eo):
    scale = max(max(np.abs(x).max() for x in eo), 1e-300)
    return max(float(np.abs(a - b).max()) for a, b in zip(eg, eo)) / scale


def check_march(plan, st, prec, label):
    """The march state of a HIP plan against the oracle's state."""
    errs = {"e": e_err(plan.e(), st["e"]), "theta": rel(plan.read(etm.ETM_FIELD_THETA), st["theta"]),
            "psum": rel(plan.read(etm.ETM_FIELD_PSUM), st["psum"])}
    if prec == FP64:
        errs["e_prev"] = e_err(plan.e_prev(), st["e_prev"])
    _say(f"[oracle-paths] {label}: " + " ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    if prec == FP64:
        assert max(errs.values()) < 1e-9, errs
    else:
        assert errs["e"] < 1e-5 and errs["theta"] < 1e-6 and errs["psum"] < 1e-6, errs
    return errs


def oracle_mech(o, theta_o):
    """The oracle's displacement (rtol 1e-12), von Mises and CG iterations."""
    q, it, _ = o.mech_solve(theta_o, o.mech_mask(), rtol=1e-12)
    return q, o.von_mises(theta_o, q), it


def check_mech(ref, u, vm, prec, label):
    q, vm_o, it = ref
    eu, evm = rel(u, q), rel(vm, vm_o)
    epk = abs(float(vm.max()) - float(vm_o.max())) / max(float(vm_o.max()), 1e-300)
    _say(f"[oracle-paths] {label}: u {eu:.2e} vm {evm:.2e} peak vm {epk:.2e} (oracle cg {it})")
    if prec == FP64:
        assert eu < 1e-6 and evm < 1e-6
    else:
        assert epk < 1e-5


# ---- the paper's synchronous schedule: a thermal step after every EM step ----
R1_CASES = [((9, 7, 5), 11), ((70, 6, 4), 12), ((17, 20, 6), 13)]


@pytest.mark.parametrize("prec", [FP64, MIXED])
@pytest.mark.parametrize("shape,seed", R1_CASES)
def test_synchronous_schedule_random_matches_oracle(prec, shape, seed):
    """R = 1 on random heterogeneous problems whose conductors have tcr > 0:
    sigma(theta) of every edge changes at every step (the coefficient refresh
    and, in mixed precision, the leapfrog correction K run every step)."""
    prob = W.random_problem(seed, *shape, n_steps=60, R=1, n_ports=3, amp=6e10, em_bc=(0,) * 6)
    assert (prob.props[:, 2] > 0).any()
    o = oracle.Oracle(prob)
    dt = o.cfl_dt()
    J = prob.sample_J_half(dt, 60)
    plan = etm.Plan(prob, J, dt=dt, precision=prec, n_steps=60, history=False)
    plan.advance(23)
    plan.advance(37)
    assert plan.sync()["step"] == 60
    st, _ = o.run(dt, 60, J, R=1)
    assert float(np.abs(st["theta"]).max()) > 0
    check_march(plan, st, prec, f"R=1 {prob.name} prec={prec}")


@pytest.mark.parametrize("prec", [FP64, MIXED])
def test_synchronous_schedule_pkg32_full_window(prec):
    """The 32x32x16 PEC trace package over its full 2000-step window at R = 1
    (the paper's schedule; the workload's own schedule is R = 200), then the
    clamped mechanical solve."""
    prob, o, dt, J, st, ref = _pkg32_r1_oracle()
    n = prob.n_em_steps
    plan = etm.Plan(prob, J, dt=dt, precision=prec, n_steps=n, history=False)
    plan.advance(n)
    plan.mech_solve()
    info = plan.sync()
    assert info["step"] == n and info["cg_relres"] <= prob.cg_rtol
    check_march(plan, st, prec, f"R=1 pkg32 prec={prec}")
    check_mech(ref, plan.u(), plan.read(etm.ETM_FIELD_VM), prec, f"R=1 pkg32 prec={prec}")


@functools.lru_cache(maxsize=None)
def _pkg32_r1_oracle():
    prob = W.config1()
    prob.em_per_thermal = 1
    o = oracle.Oracle(prob)
    dt = o.cfl_dt()
    J = prob.sample_J_half(dt, prob.n_em_steps)
    st, _ = o.run(dt, prob.n_em_steps, J, R=1)
    return prob, o, dt, J, st, oracle_mech(o, st["theta"])


# ---- histories of the mixed path --------------------------------------------
def test_mixed_history_matches_oracle():
    """Energy W, cumulative Joule energy, max theta and probe samples of the
    mixed path against the oracle's FP64 histories.  W is quadratic in e
    (bar 2e-5 of the column max); the Joule energy and theta columns carry
    the temperature bar (1e-6); e probes the field bar (1e-5)."""
    prob = W.random_problem(7, 9, 7, 5, n_steps=40, R=4, n_ports=2, amp=3e10)
    prob.history_stride = 5
    prob.probes = np.array([[0, 3, 2, 1], [1, 4, 3, 2], [2, 5, 4, 1], [3, 4, 3, 2]], dtype=np.int64)
    o = oracle.Oracle(prob)
    dt = o.cfl_dt()
    J = prob.sample_J_half(dt, 40)
    plan = etm.Plan(prob, J, dt=dt, precision=MIXED, n_steps=40, history=True)
    plan.advance(40)
    plan.sync()
    st, hist = o.run(dt, 40, J, stride=5, probes=prob.probes)
    hg = plan.history()
    assert hg.shape == hist.shape and hg.shape[0] == 8
    np.testing.assert_array_equal(hg[:, 0], hist[:, 0])
    bars = {1: 2e-5, 2: 1e-6, 3: 1e-6, 4: 1e-5, 5: 1e-5, 6: 1e-5, 7: 1e-6}
    errs = {c: rel(hg[:, c], hist[:, c]) for c in bars}
    _say(f"[oracle-paths] mixed history column errors {errs}")
    for c, bar in bars.items():
        assert errs[c] < bar, (c, errs[c])


# ---- batched variants --------------------------------------------------------
@pytest.mark.parametrize("prec", [FP64, MIXED])
def test_batch_variants_match_oracle(prec):
    """Uneven variants in one batch (graph-replayed segments, thermal steps
    at different R), each compared with the oracle's run of that variant."""
    shapes = [(70, 6, 4), (9, 7, 5), (33, 12, 6)]
    probs = [W.random_problem(600 + v, *s, n_steps=50, R=[4, 6, 5][v], n_ports=2, amp=3e10, em_bc=(0,) * 6)
             for v, s in enumerate(shapes)]
    orcs = [oracle.Oracle(p) for p in probs]
    dts = [o.cfl_dt() for o in orcs]
    Js = [p.sample_J_half(dt, 50) for p, dt in zip(probs, dts)]
    plans = [etm.Plan(p, J, dt=dt, precision=prec, n_steps=50, history=False) for p, J, dt in zip(probs, Js, dts)]
    b = etm.Batch(4)
    for pl in plans:
        b.attach(pl)
    b.advance(21)
    b.advance(29)
    for p, o, pl, dt, J in zip(probs, orcs, plans, dts, Js):
        assert pl.sync()["step"] == 50
        st, _ = o.run(dt, 50, J)
        check_march(pl, st, prec, f"batch {p.name} prec={prec}")


# ---- served requests -----------------------------------------------------------
def _request(r, nx, ny, nz, bits):
    p = W.package(nx, ny, nz, 7100 + r, bump_pitch_um=20, bump_cells=8, trace_width=2, trace_pitch=4,
                  n_trace_layers=2, max_traces=6, n_bits=bits, steps_per_bit=4, em_per_thermal=64,
                  name=f"oreq{r}")
    return serve.Request(prob=p, arrival=0.02 * r, rid=r)


SERVED = [(0, 24, 20, 24, 40), (1, 30, 18, 24, 64), (2, 20, 26, 24, 32)]


@functools.lru_cache(maxsize=None)
def _served_oracle(rid):
    p = _request(*SERVED[rid]).prob
    o = oracle.Oracle(p)
    dt = o.cfl_dt()
    st, _ = o.run(dt, p.n_em_steps, p.sample_J_half(dt, p.n_em_steps))
    q, vm, _ = oracle_mech(o, st["theta"])
    return st["theta"], vm


@pytest.mark.parametrize("prec", [FP64, MIXED])
def test_served_requests_match_oracle(prec):
    """Three requests through the continuous-batching server (two slots, so
    one joins while the others run); each result against the oracle's
    march and solve of that request."""
    reqs = [_request(*a) for a in SERVED]
    srv = serve.Server(max_slots=2, hbm_budget=16e9, precision=prec, chunk=48, keep_fields=True)
    done = {r.rid: r for r in srv.run(reqs, realtime=True)}
    assert sorted(done) == [0, 1, 2]
    for q in reqs:
        p, res = q.prob, done[q.rid]
        theta_o, vm_o = _served_oracle(q.rid)
        et = rel(res.theta, theta_o)
        _say(f"[oracle-paths] served {p.name} prec={prec}: theta {et:.2e}")
        assert et < (1e-9 if prec == FP64 else 1e-6)
        evm = rel(res.vm, vm_o)
        epk = abs(res.vm_max - float(vm_o.max())) / float(vm_o.max())
        _say(f"[oracle-paths] served {p.name} prec={prec}: vm {evm:.2e} peak vm {epk:.2e}")
        assert (evm < 1e-6) if prec == FP64 else (epk < 1e-5)


# ---- two-step slab wavefront with overlapped solves ------------------------------
@pytest.mark.parametrize("prec", [FP64, MIXED])
def test_slab_pairs_with_overlapped_solves_match_oracle(prec):
    """The two-step slab wavefront over 3 z-slabs (odd step counts, thermal
    steps every 8 that break pairs) with a mechanical solve after every
    thermal step on the side stream, against the oracle's march and its
    solve of the final temperature."""
    p, dt, J, st, ref = _slab_oracle()
    n = sum(SLAB_CHUNKS)
    plan = etm.Plan(p, J, dt=dt, precision=prec, n_steps=n, history=False, em_slabs=3, mech_overlap=1)
    for c in SLAB_CHUNKS:
        plan.advance(c)
    info = plan.sync()
    assert info["step"] == n and info["n_solves"] == n // 8
    check_march(plan, st, prec, f"slabs=3 overlap prec={prec}")
    check_mech(ref, plan.u(), plan.read(etm.ETM_FIELD_VM), prec, f"slabs=3 overlap prec={prec}")


SLAB_CHUNKS = (45, 3, 20)   # many blocks per call, a call ending on a thermal step, odd counts


@functools.lru_cache(maxsize=None)
def _slab_oracle():
    p = W.package(30, 26, 30, 41, bump_pitch_um=14, bump_cells=6, max_traces=6, em_per_thermal=8)
    p.mech_every_thermal = 1
    o = oracle.Oracle(p)
    dt = o.cfl_dt()
    n = sum(SLAB_CHUNKS)
    J = p.sample_J_half(dt, n + 1)
    st, _ = o.run(dt, n, J)
    return p, dt, J, st, oracle_mech(o, st["theta"])
