"""GPU: the multigrid-preconditioned mechanical solve (through the C ABI)
against the FP64 oracle, against the Jacobi-preconditioned solve, and its
iteration counts.  The preconditioner changes only how CG gets there: the
converged displacement must agree with the oracle's to the solve tolerance."""
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
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def solve(prob, th, precision, precond, coarse=0):
    o = oracle.Oracle(prob)
    dt = o.cfl_dt()
    J = prob.sample_J_half(dt, 4)
    plan = etm.Plan(prob, J, dt=dt, precision=precision, n_steps=4, mech_precond=precond, mg_coarse_dofs=coarse)
    plan.write(etm.ETM_FIELD_THETA, th)
    plan.mech_solve()
    info = plan.sync()
    return plan, info


CASES = [(11, (24, 20, 10), W.MECH_KINEMATIC, 60), (12, (33, 17, 9), W.MECH_CLAMP_ZMIN, 60),
         (13, (40, 9, 6), W.MECH_KINEMATIC, 3)]


@pytest.mark.parametrize("seed,shape,bc,coarse", CASES)
@pytest.mark.parametrize("precision", [etm.ETM_PREC_FP64, etm.ETM_PREC_MIXED])
def test_multigrid_solve_matches_oracle(seed, shape, bc, coarse, precision):
    prob = W.random_problem(seed, *shape, n_steps=4, R=2, mech_bc=bc, void_top=1)
    prob.cg_rtol = 1e-10
    o = oracle.Oracle(prob)
    rng = np.random.default_rng(seed)
    th = rng.uniform(0, 30, o.node_shape)
    _say(f"[mg] {shape} bc={bc} coarse={coarse} prec={precision}")
    plan, info = solve(prob, th, precision, etm.ETM_PRECOND_MG, coarse)
    _say(f"[mg] levels {info['mg_levels']} iters {info['cg_iters']} outer {info['cg_outer']} relres {info['cg_relres']:.2e}")
    assert info["mg_levels"] >= 2
    assert info["cg_relres"] <= prob.cg_rtol
    q, it, rr = o.mech_solve(th, o.mech_mask(), rtol=1e-13)
    assert rel_err(plan.u(), q) < 1e-7
    assert rel_err(plan.read(etm.ETM_FIELD_VM), o.von_mises(th, q)) < 1e-7
    # a few dozen V-cycle iterations, where Jacobi needs hundreds
    assert info["cg_iters"] <= 120


def test_multigrid_and_jacobi_agree_and_multigrid_is_faster():
    prob = W.random_problem(21, 30, 26, 12, n_steps=4, R=2, mech_bc=W.MECH_KINEMATIC, void_top=1)
    prob.cg_rtol = 1e-10
    o = oracle.Oracle(prob)
    th = np.random.default_rng(5).uniform(0, 30, o.node_shape)
    pm, im = solve(prob, th, etm.ETM_PREC_FP64, etm.ETM_PRECOND_MG)
    pj, ij = solve(prob, th, etm.ETM_PREC_FP64, etm.ETM_PRECOND_JACOBI)
    _say(f"[mg] MG {im['cg_iters']} iterations ({im['mg_levels']} levels), Jacobi {ij['cg_iters']}")
    assert rel_err(pm.u(), pj.u()) < 1e-8
    assert im["cg_iters"] * 5 < ij["cg_iters"]


def test_single_level_is_an_exact_solve():
    """A mesh below the coarse threshold is one level solved by its dense
    inverse: CG converges in one or two iterations."""
    prob = W.random_problem(31, 6, 5, 4, n_steps=4, R=2, mech_bc=W.MECH_KINEMATIC, void_top=1)
    prob.cg_rtol = 1e-12
    o = oracle.Oracle(prob)
    th = np.random.default_rng(6).uniform(0, 30, o.node_shape)
    plan, info = solve(prob, th, etm.ETM_PREC_FP64, etm.ETM_PRECOND_MG, 4000)
    assert info["mg_levels"] == 1
    assert info["cg_iters"] <= 2
    q, _, _ = o.mech_solve(th, o.mech_mask(), rtol=1e-13)
    assert rel_err(plan.u(), q) < 1e-9


def test_multigrid_warm_started_solves_in_the_coupled_march():
    """The 32x32x16 trace case with a solve after every thermal step:
    every solve converges and the final field matches the oracle."""
    prob = W.config1()
    prob.mech_every_thermal = 1
    o = oracle.Oracle(prob)
    dt = o.cfl_dt()
    J = prob.sample_J_half(dt, prob.n_em_steps)
    plan = etm.Plan(prob, J, dt=dt, precision=etm.ETM_PREC_MIXED, n_steps=prob.n_em_steps, history=False)
    plan.advance(prob.n_em_steps)
    info = plan.sync()
    _say(f"[mg] pkg32 solves {info['n_solves']} total iters {info['cg_iters_total']} last {info['cg_iters']}")
    assert info["n_solves"] == prob.n_em_steps // prob.em_per_thermal
    st, _ = o.run(dt, prob.n_em_steps, J)
    q, _, _ = o.mech_solve(st["theta"], o.mech_mask(), rtol=1e-12)
    vm_o = o.von_mises(st["theta"], q)
    assert abs(plan.read(etm.ETM_FIELD_VM).max() - vm_o.max()) / vm_o.max() < 1e-5
