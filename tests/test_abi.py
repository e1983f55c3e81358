"""Host-only checks of the C ABI (no GPU needed): the library loads, exports
every symbol the public header declares, and validates inputs on the host."""
import ctypes as C
import json
import os
import re

import numpy as np
import pytest

import oracle
import paper_2603_07038_amd as etm
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(etm_[a-z0-9_]+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    L = etm.load()
    names = _declared_symbols()
    assert len(names) >= 20
    for n in sorted(names):
        assert hasattr(L, n), n


def _create(prob, J=None, **kw):
    L = etm.load()
    inp = etm._Inputs(prob, J)
    o, keep = etm.make_opts(prob, **kw)
    h = C.c_void_p()
    st = L.etm_plan_create(C.byref(inp.mesh), inp.mats, int(prob.props.shape[0]), C.byref(inp.src), C.byref(o),
                           C.byref(h))
    return st, h


def test_dof_counts_of_the_paper_mesh():
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_counts.json")))
    nx, ny, nz = g["mesh_cells"]
    p = W.Problem(name="paper", dx=np.full(nx, 1e-6), dy=np.full(ny, 1e-6), dz=np.full(nz, 1e-6),
                  mat=np.ones((nz, ny, nx), dtype=np.uint8), props=W.package_materials(), waves=[],
                  **W._empty_ports())
    st, h = _create(p)
    assert st == etm.ETM_OK, etm.load().etm_last_error()
    a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
    etm.check(etm.load().etm_plan_dofs(h, C.byref(a), C.byref(b), C.byref(c)))
    assert (a.value, b.value, c.value) == (g["em_dof"], g["thermal_dof"], g["mech_dof"])
    etm.load().etm_plan_destroy(h)


@pytest.mark.parametrize("maker", [W.config1, lambda: W.random_problem(3, 7, 5, 4)])
def test_auto_dt_matches_oracle_cfl(maker):
    p = maker()
    assert abs(etm.cfl_dt(p) / oracle.Oracle(p).cfl_dt() - 1) < 1e-14


def test_footprint_fits_full_scale_package():
    """The 1024x1024x128 package's plan (state, CG vectors and the multigrid
    hierarchy) fits one MI355X's 288 GB with room."""
    nx, ny, nz = 1024, 1024, 128
    p = W.Problem(name="big", dx=np.full(nx, 1e-6), dy=np.full(ny, 1e-6), dz=np.full(nz, 1e-6),
                  mat=np.ones((nz, ny, nx), dtype=np.uint8), props=W.package_materials(), waves=[],
                  **W._empty_ports())
    for prec in (etm.ETM_PREC_FP64, etm.ETM_PREC_MIXED):
        st, h = _create(p, precision=prec)
        assert st == 0
        fp = C.c_size_t()
        etm.load().etm_plan_footprint(h, C.byref(fp))
        assert fp.value < (128e9 if prec == etm.ETM_PREC_FP64 else 80e9)
        etm.load().etm_plan_destroy(h)


def test_validation_errors():
    p = W.random_problem(1, 5, 4, 3, em_bc=(0,) * 6)
    J = p.sample_J_half(1e-15, 10)
    assert _create(p, J)[0] == etm.ETM_OK
    bad = W.random_problem(1, 5, 4, 3, em_bc=(0,) * 6)
    bad.mat = bad.mat.copy()
    bad.mat[0, 0, 0] = 200
    assert _create(bad, J)[0] == etm.ETM_E_INVAL
    # dt above the CFL limit
    lim = etm.cfl_dt(p, 1.0)
    assert _create(p, J, dt=1.01 * lim)[0] == etm.ETM_E_UNSTABLE
    assert _create(p, J, dt=1.01 * lim, force_dt=True)[0] == etm.ETM_OK
    # port outside / on a PEC face
    q = W.random_problem(1, 5, 4, 3, em_bc=(0,) * 6)
    q.port_i = q.port_i.copy()
    q.port_i[0] = 99
    assert _create(q, J)[0] == etm.ETM_E_INVAL
    r = W.random_problem(1, 5, 4, 3, em_bc=(1,) * 6)
    r.port_dir = np.array([0], dtype=np.uint8)
    r.port_i, r.port_j, r.port_k = (np.array([0], dtype=np.int32),) * 3
    r.port_wave, r.port_weight, r.port_g = np.array([0], dtype=np.int32), np.ones(1), np.zeros(1)
    assert _create(r, J)[0] == etm.ETM_E_INVAL
    # thermal step beyond forward-Euler stability
    t = W.random_problem(1, 5, 4, 3, em_bc=(0,) * 6, R=10 ** 9)
    assert _create(t, J)[0] == etm.ETM_E_UNSTABLE
    # bad options
    assert _create(p, J, em_per_thermal=0)[0] == etm.ETM_E_INVAL
    assert _create(p, J, precision=7)[0] == etm.ETM_E_INVAL
    assert _create(p, J, mech_precond=5)[0] == etm.ETM_E_INVAL
    assert _create(p, J, mg_coarse_dofs=2)[0] == etm.ETM_E_INVAL
    assert _create(p, J, mg_coarse_dofs=5000)[0] == etm.ETM_E_INVAL
    assert _create(p, J, mech_precond=etm.ETM_PRECOND_JACOBI)[0] == etm.ETM_OK
    assert _create(p, J, mg_degree=(C.c_int32 * 2)(5, 2))[0] == etm.ETM_E_INVAL
    # temporal blocking of the EM march: 0..64 z-slabs
    assert _create(p, J, em_slabs=-1)[0] == etm.ETM_E_INVAL
    assert _create(p, J, em_slabs=65)[0] == etm.ETM_E_INVAL
    assert _create(p, J, em_slabs=8)[0] == etm.ETM_OK
    assert _create(p, J, mech_overlap=2)[0] == etm.ETM_E_INVAL
    assert _create(p, J, mech_overlap=0)[0] == etm.ETM_OK


def test_calls_before_bind_are_state_errors():
    p = W.random_problem(2, 4, 4, 3)
    st, h = _create(p, p.sample_J_half(1e-15, 10))
    assert st == 0
    L = etm.load()
    assert L.etm_advance(h, 1) == etm.ETM_E_STATE
    assert L.etm_mech_solve(h) == etm.ETM_E_STATE
    L.etm_plan_destroy(h)
