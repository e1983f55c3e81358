"""Pins of the oracle's thermal update (Eq. 4-5) and of the EM-thermal
coupling schedule against closed forms and conservation."""
import numpy as np
import pytest

import oracle
import workloads as W
from test_oracle_em import _problem, _props_uniform


def test_dct_mode_decays_exactly():
    """Uniform material, uniform dz: theta = cos(n pi k / Nz) is an eigenvector
    of the node finite-volume operator with adiabatic ends, so forward Euler
    multiplies it by (1 - dt_th D (4/dz^2) sin^2(n pi / 2Nz)) per step."""
    nz, dz, k, rc = 12, 1.5e-6, 150.0, 1.7e6
    p = _problem(3, 2, nz, d=(0.9e-6, 1.3e-6, dz), props=_props_uniform(k=k, rho_cp=rc))
    o = oracle.Oracle(p)
    D = k / rc
    dt_th = 0.2 * dz * dz / D
    zero = np.zeros(o.node_shape)
    for n in (1, 3, 7):
        kk = np.arange(nz + 1)
        th0 = np.broadcast_to(np.cos(n * np.pi * kk / nz)[:, None, None], o.node_shape).copy()
        g = 1 - dt_th * D * (4 / dz ** 2) * np.sin(n * np.pi / (2 * nz)) ** 2
        th = th0
        for m in range(25):
            th = o.thermal_step(dt_th, th, zero)
        np.testing.assert_allclose(th, g ** 25 * th0, rtol=0, atol=1e-12)


def _slab_series(z, L, D, t, nterms=400):
    n = np.arange(1, nterms + 1)
    c = (2 / (n * np.pi)) * np.sin(n * np.pi / 2)
    return 0.5 + (c[None, :] * np.cos(np.outer(z, n) * np.pi / L) * np.exp(-D * (n * np.pi / L) ** 2 * t)).sum(1)


def test_slab_series_second_order():
    """A 1D slab with adiabatic faces, initially 1 on the lower half and 0
    above, follows theta = 1/2 + sum 2/(n pi) sin(n pi/2) cos(n pi z/L)
    exp(-D (n pi/L)^2 t); the error falls at second order under refinement
    (dt_th scaled with dz^2)."""
    L, k, rc = 40e-6, 100.0, 2e6
    D = k / rc
    t_end = 0.05 * L * L / D
    errs = []
    for nz in (16, 32, 64):
        dz = L / nz
        p = _problem(1, 1, nz, d=(1e-6, 1e-6, dz), props=_props_uniform(k=k, rho_cp=rc))
        o = oracle.Oracle(p)
        z = np.arange(nz + 1) * dz
        th = np.where(z < L / 2, 1.0, np.where(z > L / 2, 0.0, 0.5))
        th = np.broadcast_to(th[:, None, None], o.node_shape).copy()
        dt_th = 0.1 * dz * dz / D
        steps = int(round(t_end / dt_th))
        dt_th = t_end / steps
        zero = np.zeros(o.node_shape)
        for m in range(steps):
            th = o.thermal_step(dt_th, th, zero)
        errs.append(np.abs(th[:, 0, 0] - _slab_series(z, L, D, t_end)).max())
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


def test_uniform_source_heats_linearly():
    """A uniform source P in a uniform block raises theta by P t / (rho c_p)
    everywhere, boundary nodes included."""
    p = _problem(3, 4, 2, d=(np.array([1e-6, 2e-6, 0.5e-6]), 1e-6, np.array([0.7e-6, 1.9e-6])),
                 props=_props_uniform(k=30.0, rho_cp=2.2e6))
    o = oracle.Oracle(p)
    P = np.full(o.node_shape, 3.3e15)
    th = np.zeros(o.node_shape)
    dt_th = 1e-12
    for m in range(10):
        th = o.thermal_step(dt_th, th, P)
    np.testing.assert_allclose(th, 3.3e15 * 10 * dt_th / 2.2e6, rtol=1e-13)


@pytest.mark.parametrize("R", [1, 3, 10])
def test_heat_is_conserved_through_the_coupled_march(R):
    """Adiabatic conduction moves heat but never creates it, so after whole
    thermal blocks the stored heat sum C_n V_n theta_n equals the dissipated
    EM energy dt * sum_steps sum_e sigma_e e_e^2 L A, for any block length."""
    p = W.random_problem(5, 6, 5, 4, n_steps=30, R=R, n_ports=3, amp=3e10)
    o = oracle.Oracle(p)
    dt = o.cfl_dt(0.9)
    st, _ = o.run(dt, p.n_em_steps, p.sample_J_half(dt))
    stored = (o.heat_capacity() * st["theta"]).sum()
    assert st["ejoule"][0] > 0
    assert abs(stored / st["ejoule"][0] - 1) < 1e-12


def test_block_schedule_R1_is_the_synchronous_update():
    """R = 1 is Eq. (5) literally: one step of the march equals an EM step,
    the Joule source at sigma(T^n) and e^{n+1}, and a thermal step over dt."""
    p = W.random_problem(8, 5, 4, 3, n_steps=6, R=1, n_ports=2, amp=5e10)
    o = oracle.Oracle(p)
    dt = o.cfl_dt(0.9)
    Jh = p.sample_J_half(dt)
    st, _ = o.run(dt, 5, Jh)
    e_prev, e_cur, th = [a.copy() for a in st["e_prev"]], [a.copy() for a in st["e"]], st["theta"].copy()
    st, _ = o.run(dt, 1, Jh, state=st)
    e_next = o.em_step(dt, th, e_prev, e_cur, Jh[:, 6], Jh[:, 5])
    P = o.joule(th, e_next)
    th_next = o.thermal_step(dt, th, P)
    for a, b in zip(st["e"], e_next):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_allclose(st["theta"], th_next, rtol=1e-14, atol=1e-300)


def test_chunked_march_equals_single_run():
    """Advancing in chunks that cut through thermal blocks gives the same
    state as one call (the block sum and the step counter carry over)."""
    p = W.random_problem(9, 5, 4, 3, n_steps=24, R=5, n_ports=2, amp=5e10)
    o = oracle.Oracle(p)
    dt = o.cfl_dt(0.9)
    Jh = p.sample_J_half(dt)
    a, _ = o.run(dt, 24, Jh)
    b, _ = o.run(dt, 7, Jh)
    b, _ = o.run(dt, 11, Jh, state=b)
    b, _ = o.run(dt, 6, Jh, state=b)
    for x, y in zip(a["e"], b["e"]):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(a["theta"], b["theta"])
    np.testing.assert_array_equal(a["psum"], b["psum"])
