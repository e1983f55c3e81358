"""Pins of two oracle parts that uniform media cannot reach.

1. The thermal load of Eq. (8) at a non-uniform temperature.  On a box cell
   with trilinear shape functions and a temperature that is itself trilinear
   (theta = x, y z, x y z in global coordinates), the load
       f_aI = (3 lambda + 2 mu) cte * int dN_a/dx_I theta dV
   factors into 1D integrals that are written out by hand below.  Evaluating
   theta at the centroid, or lumping it at the nodes, changes these numbers.

2. The per-edge material averages of eps, sigma and k (reading c2: area
   weights over the up-to-four cells of an edge).  Whatever the materials, a
   uniform tangential field gives back each cell's own energy and power,
   and a linear temperature gives each x-slab its own conduction flux:
       (a) 1/2 delta^T D_eps delta / dt^2 = 1/2 eps0 E^2 sum_c eps_r,c V_c
       (b) sum_e sigma_e e_e^2 L_e A_e      = E^2 sum_c sigma_c(theta) V_c
       (c) heat leaving the nodes left of a dual face in one thermal step
           = g sum_{cells of the slab} k_c (transverse area of c)
   because every cell owns four edges of each direction and gives each a
   quarter of its transverse area.  An unweighted mean over the cells of an
   edge fails all three on a graded mesh with mixed materials.
"""
import numpy as np
import pytest

import oracle
from test_oracle_em import _problem

EPS0 = 8.8541878128e-12


def _graded_mixed(seed, nx, ny, nz, n_mat=4, tcr=True):
    """Random graded spacings and random per-cell materials (no layering)."""
    rng = np.random.default_rng(seed)
    props = np.zeros((n_mat, 9))
    for m in range(n_mat):
        props[m] = [rng.uniform(1.0, 12.0), rng.uniform(0.0, 6e7), rng.uniform(0.0, 4e-3) if tcr else 0.0,
                    rng.uniform(0.2, 400.0), rng.uniform(1e6, 4e6), rng.uniform(3e9, 150e9),
                    rng.uniform(0.2, 0.42), rng.uniform(2e-6, 40e-6), 0.0]
    mat = rng.integers(0, n_mat, (nz, ny, nx)).astype(np.uint8)
    d = (rng.uniform(0.4e-6, 3e-6, nx), rng.uniform(0.4e-6, 3e-6, ny), rng.uniform(0.4e-6, 3e-6, nz))
    return _problem(nx, ny, nz, d=d, props=props, mat=mat)


def _cell_volumes(p):
    return p.dz[:, None, None] * p.dy[None, :, None] * p.dx[None, None, :]


# ---- 1D integrals on [x0, x0 + h] with phi_0 = (x0 + h - x) / h, phi_1 = (x - x0) / h
def _int_phi(a, m, x0, h):
    """int phi_a(x) x^m dx, m = 0 or 1."""
    if m == 0:
        return h / 2.0
    return x0 * h / 2.0 + (h * h / 6.0 if a == 0 else h * h / 3.0)


def _int_dphi(a, m, x0, h):
    """int phi_a'(x) x^m dx, m = 0 or 1."""
    s = -1.0 if a == 0 else 1.0
    return s if m == 0 else s * (x0 + h / 2.0)


@pytest.mark.parametrize("powers", [(1, 0, 0), (0, 1, 1), (1, 1, 1), (0, 0, 1)])
def test_thermal_load_of_a_trilinear_temperature_matches_the_integral(powers):
    """theta = x^px y^py z^pz (px, py, pz in {0, 1}) on cell (1, 1, 1) of a
    graded 3x3x3 mesh away from the origin: the element load equals the
    product of hand-written 1D integrals."""
    E, nu, cte = 117e9, 0.34, 17e-6
    props = np.array([[1.0, 0.0, 0.0, 1.0, 1e6, E, nu, cte, 0.0]])
    dx, dy, dz = np.array([1.3e-6, 0.7e-6, 2.1e-6]), np.array([0.9e-6, 1.6e-6, 1.1e-6]), np.array([2.4e-6, 0.5e-6, 1.0e-6])
    p = _problem(3, 3, 3, d=(dx, dy, dz), props=props)
    o = oracle.Oracle(p)
    i = j = k = 1
    x0, y0, z0 = dx[0], dy[0], dz[0]
    h = (dx[i], dy[j], dz[k])
    origin = (x0, y0, z0)
    scale = 1e6 ** sum(powers)  # theta of order 1 K over the micrometre cell
    th8 = np.zeros(8)
    for a in range(8):
        ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
        xyz = (x0 + ax * h[0], y0 + ay * h[1], z0 + az * h[2])
        th8[a] = scale * np.prod([xyz[q] ** powers[q] for q in range(3)])
    _, fe = o.hex8_element(i, j, k, th8)
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    beta = (3 * lam + 2 * mu) * cte
    want = np.zeros(24)
    for a in range(8):
        loc = (a & 1, (a >> 1) & 1, (a >> 2) & 1)
        for I in range(3):
            v = beta * scale
            for J in range(3):
                f = _int_dphi if J == I else _int_phi
                v *= f(loc[J], powers[J], origin[J], h[J])
            want[3 * a + I] = v
    np.testing.assert_allclose(fe, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


def test_thermal_load_is_not_the_centroid_or_lumped_value():
    """The same closed form separates the exact load from the two plausible
    slips it guards against (theta at the centroid for every Gauss point,
    theta lumped at each element node): both differ by far more than
    rounding on theta = x y z."""
    E, nu, cte = 130e9, 0.28, 2.6e-6
    props = np.array([[1.0, 0.0, 0.0, 1.0, 1e6, E, nu, cte, 0.0]])
    dx, dy, dz = np.array([1.0e-6, 2.0e-6]), np.array([1.5e-6, 0.5e-6]), np.array([0.8e-6, 1.7e-6])
    p = _problem(2, 2, 2, d=(dx, dy, dz), props=props)
    o = oracle.Oracle(p)
    h = (dx[1], dy[1], dz[1])
    origin = (dx[0], dy[0], dz[0])
    th8 = np.array([1e18 * np.prod([origin[q] + ((a >> q) & 1) * h[q] for q in range(3)]) for a in range(8)])
    _, fe = o.hex8_element(1, 1, 1, th8)
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    beta = (3 * lam + 2 * mu) * cte
    centroid = th8.mean()
    slip = np.zeros(24)
    for a in range(8):
        loc = (a & 1, (a >> 1) & 1, (a >> 2) & 1)
        for I in range(3):
            v = beta * centroid
            for J in range(3):
                v *= _int_dphi(loc[J], 0, origin[J], h[J]) if J == I else _int_phi(loc[J], 0, origin[J], h[J])
            slip[3 * a + I] = v
    assert np.abs(fe - slip).max() > 1e-3 * np.abs(fe).max()


@pytest.mark.parametrize("d", [0, 1, 2])
def test_edge_permittivity_average_gives_back_every_cell_energy(d):
    """(a): e^n = 0, e^{n+1} = E dt on every d-edge (all faces PMC, so every
    edge exists; the curl term vanishes with e^n = 0)."""
    p = _graded_mixed(11 + d, 5, 4, 3)
    o = oracle.Oracle(p)
    dt, E = 1e-15, 3.7e4
    e0 = o.zeros_e()
    e1 = o.zeros_e()
    e1[d][...] = E * dt
    W = o.em_energy(dt, e0, e1)
    eps_r = p.props[p.mat, 0]
    want = 0.5 * EPS0 * E * E * float((eps_r * _cell_volumes(p)).sum())
    assert W == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_edge_conductivity_average_gives_back_every_cell_power(d):
    """(b) at a uniform rise theta: sigma_c(theta) = sigma0_c / (1 + tcr_c theta)
    per cell (Eq. 6), summed with the cell volumes."""
    p = _graded_mixed(21 + d, 4, 5, 3)
    o = oracle.Oracle(p)
    E, th = 2.3e3, 12.5
    e = o.zeros_e()
    e[d][...] = E
    theta = np.full(o.node_shape, th)
    tot = o.joule_total(theta, e)
    sig = p.props[p.mat, 1] / (1.0 + p.props[p.mat, 2] * th)
    want = E * E * float((sig * _cell_volumes(p)).sum())
    assert tot == pytest.approx(want, rel=1e-12)
    # the node form distributes the same total: sum_n P_n V_n
    P = o.joule(theta, e)
    hx = np.concatenate([[p.dx[0] / 2], (p.dx[:-1] + p.dx[1:]) / 2, [p.dx[-1] / 2]])
    hy = np.concatenate([[p.dy[0] / 2], (p.dy[:-1] + p.dy[1:]) / 2, [p.dy[-1] / 2]])
    hz = np.concatenate([[p.dz[0] / 2], (p.dz[:-1] + p.dz[1:]) / 2, [p.dz[-1] / 2]])
    Vn = hz[:, None, None] * hy[None, :, None] * hx[None, None, :]
    assert float((P * Vn).sum()) == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_edge_conductance_average_carries_each_slab_flux(axis):
    """(c): theta = g x_axis, no source.  The heat the nodes with index <= s
    along `axis` lose in one thermal step is the flux through the dual face
    between s and s + 1: g times the sum of k_c times the transverse area of
    the cells of slab s."""
    p = _graded_mixed(31 + axis, 5, 5, 5, tcr=False)
    o = oracle.Oracle(p)
    g = 1e5  # K/m
    coords = [np.concatenate([[0], np.cumsum(w)]) for w in (p.dx, p.dy, p.dz)]
    Z, Y, X = np.meshgrid(coords[2], coords[1], coords[0], indexing="ij")
    theta = g * (X, Y, Z)[axis]
    dt_th = 1e-12
    out = o.thermal_step(dt_th, theta, np.zeros(o.node_shape))
    CV = o.heat_capacity()
    lost = CV * (out - theta) / dt_th  # = -(flux out of each node)
    kc = p.props[p.mat, 3]
    widths = (p.dx, p.dy, p.dz)
    other = [q for q in range(3) if q != axis]
    for s in range(widths[axis].size - 1):
        # node axis index <= s: the region left of the dual face at s + 1/2
        sel = [slice(None)] * 3
        sel[2 - axis] = slice(0, s + 1)
        gained = float(lost[tuple(sel)].sum())
        csel = [slice(None)] * 3
        csel[2 - axis] = s
        area = np.ones(o.cell_shape)
        for q in other:
            shape = [1, 1, 1]
            shape[2 - q] = -1
            area = area * widths[q].reshape(shape)
        want = g * float((kc * area)[tuple(csel)].sum())
        assert gained == pytest.approx(want, rel=1e-10)
