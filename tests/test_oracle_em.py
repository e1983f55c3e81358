"""Pins of the oracle's EM update (Eq. 1-3) and Joule source against closed
forms and invariants that do not depend on the oracle's own code."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

EPS0 = 8.8541878128e-12
MU0 = 1.25663706212e-6
C2 = 1.0 / (EPS0 * MU0)


def _props_uniform(eps_r=1.0, sigma=0.0, tcr=0.0, k=1.0, rho_cp=1e6, E=100e9, nu=0.3, cte=1e-5):
    return np.array([[eps_r, sigma, tcr, k, rho_cp, E, nu, cte, 0.0]])


def _problem(nx, ny, nz, d=(1e-6, 1e-6, 1e-6), props=None, mat=None, em_bc=(0,) * 6, **kw):
    dx = np.full(nx, d[0]) if np.isscalar(d[0]) else np.asarray(d[0])
    dy = np.full(ny, d[1]) if np.isscalar(d[1]) else np.asarray(d[1])
    dz = np.full(nz, d[2]) if np.isscalar(d[2]) else np.asarray(d[2])
    props = _props_uniform() if props is None else props
    mat = np.zeros((nz, ny, nx), dtype=np.uint8) if mat is None else mat
    ports = W._stack_ports(kw.pop("ports", []))
    return W.Problem(name="t", dx=dx, dy=dy, dz=dz, mat=mat, props=props,
                     waves=kw.pop("waves", []), em_bc=tuple(em_bc), **ports, **kw)


def test_dof_counts_match_paper():
    """Edges on every primal edge (PMC keeps boundary edges), temperature and
    three displacement components on every node: the paper's three DOF counts."""
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")))
    nx, ny, nz = g["mesh_cells"]
    p = _problem(nx, ny, nz)
    o = oracle.Oracle(p)
    lib = oracle.lib()
    em = sum(lib.or_n_edges(o.h, d) for d in range(3))
    nodes = lib.or_n_nodes(o.h)
    assert em == g["em_dof"]
    assert nodes == g["thermal_dof"]
    assert 3 * nodes == g["mech_dof"]
    assert round(g["window_s"] / g["dt_s"]) == 15000


def test_pec_cavity_mode_is_exact_recurrence():
    """E_y = sin(m pi x/a) sin(p pi z/d) in a vacuum PEC box is an eigenvector
    of the discrete curl-curl with lambda = (2/dx)^2 sin^2(m pi dx/2a) +
    (2/dz)^2 sin^2(p pi dz/2d), so Eq. (2) reduces to
    c^{n+1} = (2 - c0^2 dt^2 lambda) c^n - c^{n-1}."""
    nx, ny, nz, m, pm = 10, 4, 8, 2, 3
    dx, dy, dz = 1.0e-6, 0.7e-6, 1.3e-6
    a, d = nx * dx, nz * dz
    p = _problem(nx, ny, nz, d=(dx, dy, dz), em_bc=(1,) * 6)
    o = oracle.Oracle(p)
    dt = o.cfl_dt(0.95)
    xs = np.arange(nx + 1) * dx
    zs = np.arange(nz + 1) * dz
    mode = np.sin(m * np.pi * xs / a)[None, None, :] * np.sin(pm * np.pi * zs / d)[:, None, None]
    mode = np.broadcast_to(mode, o.edge_shapes[1]).copy()
    lam = (2 / dx) ** 2 * np.sin(m * np.pi * dx / (2 * a)) ** 2 + (2 / dz) ** 2 * np.sin(pm * np.pi * dz / (2 * d)) ** 2
    g = 2.0 - C2 * dt * dt * lam
    ex0, ez0 = np.zeros(o.edge_shapes[0]), np.zeros(o.edge_shapes[2])
    e_prev = [ex0, mode.copy(), ez0]
    e_cur = [ex0, mode.copy(), ez0]
    c_prev, c_cur = 1.0, 1.0
    J = np.zeros(1)
    series = [1.0]
    for n in range(300):
        e_next = o.em_step(dt, None, e_prev, e_cur, J, J)
        c_next = g * c_cur - c_prev
        np.testing.assert_allclose(e_next[1], c_next * mode, rtol=0, atol=1e-9 * max(1.0, abs(c_next)))
        assert np.abs(e_next[0]).max() < 1e-9 and np.abs(e_next[2]).max() < 1e-9
        e_prev, e_cur = e_cur, e_next
        c_prev, c_cur = c_cur, c_next
        series.append(c_cur)
    # The discrete resonance approaches the continuum cavity frequency
    # f = c/2 sqrt((m/a)^2 + (p/d)^2) with the second-order dispersion error.
    s = np.array(series)
    cosw = (s[2:] + s[:-2]) / (2 * s[1:-1])
    cosw = np.median(cosw[np.abs(s[1:-1]) > 0.3])
    f_disc = np.arccos(cosw) / (2 * np.pi * dt)
    f_pred = np.arccos(1 - 0.5 * C2 * dt * dt * lam) / (2 * np.pi * dt)
    assert abs(f_disc / f_pred - 1) < 1e-8
    # on this coarse grid (3 half-waves over 8 cells) the dispersion error is a few %
    f_cont = 0.5 * np.sqrt(C2) * np.sqrt((m / a) ** 2 + (pm / d) ** 2)
    assert abs(f_disc / f_cont - 1) < 0.05


def test_cavity_frequency_converges_second_order():
    """Refining the PEC cavity grid moves the discrete resonance toward the
    continuum frequency at second order."""
    errs = []
    for n in (8, 16, 32):
        a = 10e-6
        dx = a / n
        lam = 2 * (2 / dx) ** 2 * np.sin(np.pi * dx / (2 * a)) ** 2
        # measure lambda from the oracle: apply the curl-curl to the mode
        p = _problem(n, 2, n, d=(dx, dx, dx), em_bc=(1,) * 6)
        o = oracle.Oracle(p)
        xs = np.arange(n + 1) * dx
        mode = np.sin(np.pi * xs / a)[None, None, :] * np.sin(np.pi * xs / a)[:, None, None]
        ey = np.broadcast_to(mode, o.edge_shapes[1]).copy()
        s = o.curlcurl([np.zeros(o.edge_shapes[0]), ey, np.zeros(o.edge_shapes[2])])[1]
        inner = np.abs(ey) > 1e-3
        lam_meas = np.median(s[inner] / ey[inner]) * MU0
        assert abs(lam_meas / lam - 1) < 1e-10
        errs.append(abs(np.sqrt(lam_meas) / (np.sqrt(2) * np.pi / a) - 1))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def _random_mat_problem(seed, nx, ny, nz, em_bc, sigma=False):
    rng = np.random.default_rng(seed)
    props = np.zeros((3, 9))
    for m in range(3):
        props[m] = [rng.uniform(1, 12), rng.uniform(1e3, 1e5) if sigma else 0.0, 0, 1, 1e6, 1e11, 0.3, 1e-5, 0]
    mat = rng.integers(0, 3, (nz, ny, nx)).astype(np.uint8)
    d = (rng.uniform(0.5e-6, 2e-6, nx), rng.uniform(0.5e-6, 2e-6, ny), rng.uniform(0.5e-6, 2e-6, nz))
    return _problem(nx, ny, nz, d=d, props=props, mat=mat, em_bc=em_bc)


@pytest.mark.parametrize("em_bc", [(0,) * 6, (1,) * 6, (1, 0, 0, 1, 1, 0)])
def test_curlcurl_symmetric_psd_with_gradient_nullspace(em_bc):
    """S = diag(L*A) * (oracle curl-curl) is symmetric positive semidefinite,
    and every discrete gradient (of a node potential vanishing on PEC faces)
    is in its null space; with all faces PMC the null space is exactly the
    gradients (dimension = nodes - 1) on this simply connected box."""
    p = _random_mat_problem(7, 3, 3, 2, em_bc)
    o = oracle.Oracle(p)
    shapes = o.edge_shapes
    sizes = [int(np.prod(s)) for s in shapes]
    coeffs = [o.edge_coeffs(d) for d in range(3)]
    free = np.concatenate([~c["pec"].ravel() for c in coeffs])
    vol = np.concatenate([c["vol"].ravel() for c in coeffs])
    n = sum(sizes)
    S = np.zeros((n, n))
    for col in range(n):
        if not free[col]:
            continue
        v = np.zeros(n)
        v[col] = 1.0
        parts = np.split(v, np.cumsum(sizes)[:-1])
        out = o.curlcurl([a.reshape(s) for a, s in zip(parts, shapes)])
        S[:, col] = np.concatenate([a.ravel() for a in out]) * vol
    S = S[np.ix_(free, free)]
    scale = np.abs(S).max()
    assert np.abs(S - S.T).max() < 1e-12 * scale
    ev = np.linalg.eigvalsh(0.5 * (S + S.T))
    assert ev.min() > -1e-10 * scale
    # gradients
    rng = np.random.default_rng(3)
    phi = rng.standard_normal(o.node_shape)
    nz, ny, nx = p.nz, p.ny, p.nx
    if em_bc[0]: phi[:, :, 0] = 0
    if em_bc[1]: phi[:, :, nx] = 0
    if em_bc[2]: phi[:, 0, :] = 0
    if em_bc[3]: phi[:, ny, :] = 0
    if em_bc[4]: phi[0] = 0
    if em_bc[5]: phi[nz] = 0
    gx = np.diff(phi, axis=2) / p.dx[None, None, :]
    gy = np.diff(phi, axis=1) / p.dy[None, :, None]
    gz = np.diff(phi, axis=0) / p.dz[:, None, None]
    out = o.curlcurl([gx, gy, gz])
    gnorm = max(np.abs(gx).max(), np.abs(gy).max(), np.abs(gz).max())
    ref = o.curlcurl([gnorm * rng.standard_normal(s) for s in shapes])
    ref_mag = max(np.abs(a).max() for a in ref)
    for a in out:
        assert np.abs(a).max() < 1e-11 * ref_mag
    if all(b == 0 for b in em_bc):
        nullity = int((ev < 1e-9 * scale).sum())
        assert nullity == (nx + 1) * (ny + 1) * (nz + 1) - 1


def test_cfl_step_below_stability_limit():
    """dt at Courant number 1 sits just below 2/sqrt(lambda_max(D_eps^-1 S))
    for a vacuum grid, where lambda_max comes from a dense eigen-solve."""
    p = _problem(4, 3, 3, d=(1e-6, 0.8e-6, 1.2e-6))
    o = oracle.Oracle(p)
    shapes = o.edge_shapes
    sizes = [int(np.prod(s)) for s in shapes]
    n = sum(sizes)
    A = np.zeros((n, n))
    for col in range(n):
        v = np.zeros(n)
        v[col] = 1.0
        parts = np.split(v, np.cumsum(sizes)[:-1])
        out = o.curlcurl([a.reshape(s) for a, s in zip(parts, shapes)])
        A[:, col] = np.concatenate([a.ravel() for a in out]) / EPS0
    lmax = np.abs(np.linalg.eigvals(A)).max()
    dt1 = o.cfl_dt(1.0)
    assert dt1 <= 2 / np.sqrt(lmax) * (1 + 1e-12)
    assert dt1 > 0.75 * 2 / np.sqrt(lmax)


def test_lossless_energy_conserved():
    """Without loss or source Eq. (2) conserves
    W = 1/2 [ (e^{n+1}-e^n)^T D_eps (e^{n+1}-e^n)/dt^2 + e^{n+1 T} S e^n ]."""
    p = _random_mat_problem(11, 6, 5, 4, (1, 0, 0, 1, 0, 1))
    o = oracle.Oracle(p)
    dt = o.cfl_dt(0.9)
    rng = np.random.default_rng(5)
    pec = [o.edge_coeffs(d)["pec"] for d in range(3)]
    e_prev = [np.where(pc, 0.0, rng.standard_normal(s)) for pc, s in zip(pec, o.edge_shapes)]
    e_cur = [np.where(pc, 0.0, a + 0.1 * rng.standard_normal(a.shape)) for pc, a in zip(pec, e_prev)]
    J = np.zeros(1)
    W0 = o.em_energy(dt, e_prev, e_cur)
    assert W0 > 0
    for n in range(400):
        e_next = o.em_step(dt, None, e_prev, e_cur, J, J)
        e_prev, e_cur = e_cur, e_next
    W1 = o.em_energy(dt, e_prev, e_cur)
    assert abs(W1 / W0 - 1) < 1e-11


def test_energy_balance_with_loss_and_ports():
    """With conduction and sources, multiplying Eq. (2) by (e^{n+1}-e^{n-1})
    gives the exact balance
      W^{n+1/2} - W^{n-1/2} = -(1/4dt) sum vol sigma_tot (e^{n+1}-e^{n-1})^2
                              -(1/2dt) sum vol (e^{n+1}-e^{n-1}) dt*dJ/dt."""
    p = W.random_problem(21, 6, 5, 4, n_steps=60, n_ports=4, amp=1e11)
    o = oracle.Oracle(p)
    dt = o.cfl_dt(0.9)
    Jh = p.sample_J_half(dt)
    co = [o.edge_coeffs(d) for d in range(3)]
    gport = [np.zeros(s) for s in o.edge_shapes]
    wport = [[] for _ in range(3)]
    for q in range(p.n_ports):
        d = int(p.port_dir[q])
        idx = (int(p.port_k[q]), int(p.port_j[q]), int(p.port_i[q]))
        gport[d][idx] += p.port_g[q]
        wport[d].append((idx, int(p.port_wave[q]), float(p.port_weight[q])))
    e_prev, e_cur = o.zeros_e(), o.zeros_e()
    W_prev = o.em_energy(dt, e_prev, e_cur)
    checked = 0
    for n in range(p.n_em_steps):
        e_next = o.em_step(dt, None, e_prev, e_cur, Jh[:, n + 1], Jh[:, n])
        W_next = o.em_energy(dt, e_cur, e_next)
        loss, src = 0.0, 0.0
        for d in range(3):
            diff = e_next[d] - e_prev[d]
            loss += (co[d]["vol"] * (co[d]["sig"] + gport[d]) * diff * diff).sum()
            for idx, w, wt in wport[d]:
                src += co[d]["vol"][idx] * diff[idx] * wt * (Jh[w, n + 1] - Jh[w, n]) * dt
        expect = -loss / (4 * dt) - src / (2 * dt * dt)
        scale = max(abs(W_next), abs(W_prev), abs(loss / (4 * dt)), 1e-300)
        assert abs((W_next - W_prev) - expect) <= 1e-9 * scale
        checked += 1
        W_prev = W_next
        e_prev, e_cur = e_cur, e_next
    assert checked == p.n_em_steps and W_prev > 0


def _bar(nx, ny, nz, sigma, tcr, R, n_steps, J0, use_port_g=False):
    d = (np.array([1.0e-6, 0.6e-6, 1.5e-6, 0.9e-6][:nx]), np.array([0.8e-6, 1.2e-6, 1.0e-6][:ny]),
         np.array([1.1e-6, 0.7e-6][:nz]))
    props = _props_uniform(eps_r=2.0, sigma=0.0 if use_port_g else sigma, tcr=tcr, rho_cp=2.5e6)
    ports = []
    # uniform J (and optionally a lumped conductance) on every x-edge
    for k in range(nz + 1):
        for j in range(ny + 1):
            for i in range(nx):
                ports.append((0, i, j, k, 0, 1.0, sigma if use_port_g else 0.0))
    p = _problem(nx, ny, nz, d=d, props=props, ports=ports, waves=[W.Wave("step", amp=J0)],
                 n_em_steps=n_steps, em_per_thermal=R)
    return p


def _bar_closed_form(eps, sigma0, tcr, rho_cp, J0, dt, R, n_steps, heats=True):
    """Closed-form solution of the uniform-bar march: within each thermal
    block the coefficients are constant and J is constant after t = 0, so the
    three-level recurrence has characteristic roots 1 and
    rho = (eps - a)/(eps + a); e^n = A + B rho^(n - n_b) with A, B fixed by the
    block's two starting values; the Joule source sigma e^2 is uniform, so
    the rise is dt/rho_cp times the sum of sigma_b (e^n)^2."""
    e = np.zeros(n_steps + 1)
    theta = 0.0
    thetas = []
    e_m1, e_0 = 0.0, 0.0
    # first step carries the source jump: (eps + a) e^1 = -(eps - a)*0 + 2 eps*0 - dt*J0
    n = 0
    blk_heat = 0.0
    while n < n_steps:
        sig = sigma0 / (1 + tcr * theta)
        a = 0.5 * dt * sig
        rho = (eps - a) / (eps + a)
        nb = n
        if n == 0:
            e[1] = -dt * J0 / (eps + a)
            e_m1, e_0 = 0.0, e[1]
            start = 1
        else:
            e_m1, e_0 = e[n - 1], e[n]
            start = n
        # e^m = A + B rho^(m - start + 1) with m = start-1 -> e_m1, m = start -> e_0
        B = (e_0 - e_m1) / (rho - 1.0)
        A = e_m1 - B
        blk_end = min(nb + R, n_steps)
        for m in range(start, blk_end + 1):
            e[m] = A + B * rho ** (m - start + 1)
        if heats:
            blk_heat = sig * np.sum(e[nb + 1:blk_end + 1] ** 2) * dt / rho_cp
        if blk_end - nb == R:
            theta += blk_heat
            thetas.append(theta)
        n = blk_end
    return e, thetas


@pytest.mark.parametrize("tcr", [0.0, 0.05])
def test_uniform_bar_reduces_to_closed_form(tcr):
    """A uniform conductor with PMC faces and a uniform step current on every
    x-edge: the curl-curl vanishes, the Joule map gives sigma|E|^2 at every
    node (boundary nodes included) and conduction carries nothing, so the 3D
    march must follow the piecewise closed form, sigma(T) coupling included."""
    nx, ny, nz = 4, 3, 2
    sigma, R, n_steps = 2e3, 8, 40
    J0 = 3e11 if tcr else 1e10
    p = _bar(nx, ny, nz, sigma, tcr, R, n_steps, J0)
    o = oracle.Oracle(p)
    dt = o.cfl_dt(0.9)
    st, _ = o.run(dt, n_steps, p.sample_J_half(dt))
    e, thetas = _bar_closed_form(2.0 * EPS0, sigma, tcr, 2.5e6, J0, dt, R, n_steps)
    np.testing.assert_allclose(st["e"][0], e[n_steps], rtol=1e-11)
    np.testing.assert_allclose(st["e_prev"][0], e[n_steps - 1], rtol=1e-11)
    assert np.abs(st["e"][1]).max() == 0 and np.abs(st["e"][2]).max() == 0
    np.testing.assert_allclose(st["theta"], thetas[-1], rtol=1e-11)
    if tcr:
        assert tcr * thetas[-1] > 0.02  # the coupling is exercised


def test_lumped_port_conductance_does_not_heat():
    """The same bar with sigma carried only by the lumped port conductance:
    the field follows the conductor's closed form but no Joule heat appears."""
    nx, ny, nz = 3, 2, 2
    sigma, R, n_steps, J0 = 2e3, 5, 30, 1e10
    p = _bar(nx, ny, nz, sigma, 0.0, R, n_steps, J0, use_port_g=True)
    o = oracle.Oracle(p)
    dt = o.cfl_dt(0.9)
    st, _ = o.run(dt, n_steps, p.sample_J_half(dt))
    e, _ = _bar_closed_form(2.0 * EPS0, sigma, 0.0, 2.5e6, J0, dt, R, n_steps, heats=False)
    np.testing.assert_allclose(st["e"][0], e[n_steps], rtol=1e-11)
    assert np.abs(st["theta"]).max() == 0.0 and st["ejoule"][0] == 0.0


def test_uniform_field_joule_is_sigma_e2_everywhere():
    """A uniform x-field in a uniform conductor gives P = sigma |E|^2 at every
    node, boundary nodes included (the edge-to-node split is volume-exact)."""
    nx, ny, nz = 3, 4, 2
    p = _problem(nx, ny, nz, d=(np.array([1e-6, 2e-6, 0.5e-6]), np.array([1e-6, 0.3e-6, 0.9e-6, 1.1e-6]),
                                np.array([0.7e-6, 1.6e-6])), props=_props_uniform(sigma=123.0))
    o = oracle.Oracle(p)
    E0 = 7.5
    e = [np.full(o.edge_shapes[0], E0), np.zeros(o.edge_shapes[1]), np.zeros(o.edge_shapes[2])]
    P = o.joule(None, e)
    np.testing.assert_allclose(P, 123.0 * E0 * E0, rtol=1e-13)
