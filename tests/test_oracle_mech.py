"""Pins of the oracle's thermo-mechanics (Eq. 7-9): HEX8 element, thermal
load, constraints, PCG and von Mises against closed forms and dense solves."""
import numpy as np
import pytest

import oracle
import workloads as W
from test_oracle_em import _problem


def _mech_problem(seed, nx, ny, nz, n_mat=3, same_cte=None, void_top=0, graded=True):
    rng = np.random.default_rng(seed)
    props = np.zeros((n_mat + 1, 9))
    props[0] = [1, 0, 0, 0.026, 1.2e3, 0, 0, 0, 1]
    for m in range(1, n_mat + 1):
        props[m] = [1, 0, 0, 1, 1e6, rng.uniform(3e9, 150e9), rng.uniform(0.2, 0.42),
                    same_cte if same_cte else rng.uniform(2e-6, 40e-6), 0]
    mat = rng.integers(1, n_mat + 1, (nz, ny, nx)).astype(np.uint8)
    if void_top:
        mat[nz - void_top:] = 0
    if graded:
        d = (rng.uniform(0.5e-6, 2e-6, nx), rng.uniform(0.5e-6, 2e-6, ny), rng.uniform(0.5e-6, 2e-6, nz))
    else:
        d = (1e-6, 1e-6, 1e-6)
    return _problem(nx, ny, nz, d=d, props=props, mat=mat)


def _dense_K(o, p, theta=None):
    nn = int(np.prod(o.node_shape))
    K = np.zeros((3 * nn, 3 * nn))
    f = np.zeros(3 * nn)
    for k in range(p.nz):
        for j in range(p.ny):
            for i in range(p.nx):
                nodes = [((k + (a >> 2 & 1)) * (p.ny + 1) + j + (a >> 1 & 1)) * (p.nx + 1) + i + (a & 1)
                         for a in range(8)]
                th8 = None if theta is None else np.array([theta.ravel()[n] for n in nodes])
                Ke, fe = o.hex8_element(i, j, k, th8)
                dofs = np.array([3 * n + c for n in nodes for c in range(3)])
                K[np.ix_(dofs, dofs)] += Ke
                f[dofs] += fe
    return K, f


def _node_xyz(p):
    x = np.concatenate([[0], np.cumsum(p.dx)])
    y = np.concatenate([[0], np.cumsum(p.dy)])
    z = np.concatenate([[0], np.cumsum(p.dz)])
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def test_element_is_symmetric_with_six_rigid_modes():
    """The unconstrained stiffness is symmetric and its null space is exactly
    the six rigid-body motions (three translations, three rotations)."""
    p = _mech_problem(1, 2, 2, 2)
    o = oracle.Oracle(p)
    K, _ = _dense_K(o, p)
    s = np.abs(K).max()
    assert np.abs(K - K.T).max() < 1e-12 * s
    ev = np.linalg.eigvalsh(K)
    assert (ev < 1e-10 * s).sum() == 6 and ev.min() > -1e-10 * s
    X, Y, Z = _node_xyz(p)
    modes = []
    for t in range(3):
        u = np.zeros(X.shape + (3,))
        u[..., t] = 1.0
        modes.append(u)
    for (a, b), (A, B) in zip([(0, 1), (1, 2), (2, 0)], [(X, Y), (Y, Z), (Z, X)]):
        u = np.zeros(X.shape + (3,))
        u[..., a] = -B
        u[..., b] = A
        modes.append(u)
    for u in modes:
        assert np.abs(K @ u.ravel()).max() < 1e-10 * s * np.abs(u).max()


def test_patch_test_linear_field_and_uniaxial_von_mises():
    """A uniform material under the affine field u = A x is in equilibrium at
    every interior node, and with eps = diag(e, -nu e, -nu e) the centroid
    stress is uniaxial: von Mises = E |e| in every cell; a pure shear strain
    gamma_xy gives sqrt(3) * mu * gamma."""
    E, nu = 70e9, 0.3
    props = np.array([[1, 0, 0, 1, 1e6, E, nu, 1e-5, 0]])
    d = (np.array([1e-6, 0.5e-6, 1.7e-6]), np.array([0.8e-6, 1.4e-6, 0.6e-6]), np.array([1.2e-6, 0.9e-6]))
    p = _problem(3, 3, 2, d=d, props=props)
    o = oracle.Oracle(p)
    X, Y, Z = _node_xyz(p)
    e = 2e-4
    u = np.stack([e * X, -nu * e * Y, -nu * e * Z], axis=-1)
    none = np.zeros(o.node_shape, dtype=np.uint8)
    y = o.mech_apply(none, u)
    inner = y[1:-1, 1:-1, 1:-1]
    assert np.abs(inner).max() < 1e-9 * np.abs(y).max()
    vm = o.von_mises(np.zeros(o.node_shape), u)
    np.testing.assert_allclose(vm, E * e, rtol=1e-10)
    g = 3e-4
    u = np.stack([g * Y, np.zeros_like(X), np.zeros_like(X)], axis=-1)
    vm, s6 = o.von_mises(np.zeros(o.node_shape), u, want_stress=True)
    mu = E / (2 * (1 + nu))
    np.testing.assert_allclose(vm, np.sqrt(3) * mu * g, rtol=1e-10)
    np.testing.assert_allclose(s6[..., 3], mu * g, rtol=1e-10)


@pytest.mark.parametrize("seed", [3, 4])
def test_free_thermal_expansion_is_stress_free(seed):
    """Any materials sharing one CTE, heated uniformly and held by the
    kinematic mount, expand freely: u = cte*dT*(x - x_c) exactly and the von
    Mises stress vanishes."""
    cte, dT = 12e-6, 40.0
    p = _mech_problem(seed, 5, 4, 3, same_cte=cte)
    o = oracle.Oracle(p)
    th = np.full(o.node_shape, dT)
    mask = o.mech_mask(W.MECH_KINEMATIC)
    q, it, rr = o.mech_solve(th, mask, rtol=1e-13)
    assert it > 0 and rr <= 1e-13
    X, Y, Z = _node_xyz(p)
    kc, jc, ic = np.argwhere(mask == 7)[0]
    assert kc == 0
    ref = np.stack([cte * dT * (X - X[0, jc, ic]), cte * dT * (Y - Y[0, jc, ic]), cte * dT * Z], axis=-1)
    assert np.abs(q - ref).max() < 1e-9 * np.abs(ref).max()
    vm = o.von_mises(th, q)
    E = p.props[1:, 5].max()
    assert vm.max() < 1e-6 * E * cte * dT


def test_laterally_free_bar_held_at_both_ends():
    """nu = 0, a uniform rise dT, u_x held on both x-faces and two more DOFs
    against the remaining rigid motions: sigma_xx = -E cte dT, all other
    stresses zero, so von Mises = E cte dT in every cell."""
    E, cte, dT = 50e9, 25e-6, 10.0
    props = np.array([[1, 0, 0, 1, 1e6, E, 0.0, cte, 0]])
    p = _problem(4, 3, 2, d=(np.array([1e-6, 0.5e-6, 1.2e-6, 0.8e-6]), 1e-6, 1e-6), props=props)
    o = oracle.Oracle(p)
    mask = np.zeros(o.node_shape, dtype=np.uint8)
    mask[:, :, 0] |= 1
    mask[:, :, -1] |= 1
    mask[0, 0, 0] |= 6
    mask[-1, 0, 0] |= 2
    th = np.full(o.node_shape, dT)
    q, it, rr = o.mech_solve(th, mask, rtol=1e-13)
    assert rr <= 1e-13
    vm, s6 = o.von_mises(th, q, want_stress=True)
    np.testing.assert_allclose(s6[..., 0], -E * cte * dT, rtol=1e-9)
    assert np.abs(s6[..., 1:]).max() < 1e-8 * E * cte * dT
    np.testing.assert_allclose(vm, E * cte * dT, rtol=1e-9)


@pytest.mark.parametrize("bc,void_top", [(W.MECH_KINEMATIC, 0), (W.MECH_CLAMP_ZMIN, 1), (W.MECH_KINEMATIC, 1)])
def test_pcg_matches_dense_solve(bc, void_top):
    """The oracle's Jacobi-PCG equals a dense solve of the assembled,
    constrained system; the matrix-free apply and the load equal the dense
    assembly; nodes touched only by void cells are fixed."""
    p = _mech_problem(10 + bc, 3, 3, 3, void_top=void_top)
    o = oracle.Oracle(p)
    rng = np.random.default_rng(2)
    th = rng.uniform(0, 50, o.node_shape)
    mask = o.mech_mask(bc)
    if void_top:
        assert (mask[-1] == 7).all()
    K, f = _dense_K(o, p, th)
    free = np.array([not (mask.ravel()[n] >> c & 1) for n in range(mask.size) for c in range(3)])
    Kff = K[np.ix_(free, free)]
    qd = np.zeros(K.shape[0])
    qd[free] = np.linalg.solve(Kff, f[free])
    q, it, rr = o.mech_solve(th, mask, rtol=1e-14)
    assert it > 0
    np.testing.assert_allclose(q.ravel(), qd, rtol=0, atol=1e-9 * np.abs(qd).max())
    fo = o.mech_rhs(th, mask).ravel()
    np.testing.assert_allclose(fo[free], f[free], rtol=0, atol=1e-12 * np.abs(f).max())
    assert np.all(fo[~free] == 0)
    v = rng.standard_normal(K.shape[0]) * free
    y = o.mech_apply(mask, v.reshape(q.shape)).ravel()
    np.testing.assert_allclose(y[free], (K @ v)[free], rtol=0, atol=1e-12 * np.abs(K @ v).max())


def test_kinematic_mount_nodes():
    """The three mount nodes: nearest-to-centre bottom node (x,y,z), the +x
    edge node at the centre's y (y,z), the +y edge node at the centre's x (z)."""
    p = _problem(4, 6, 2, d=(np.array([1, 1, 3, 1.0]) * 1e-6, 1e-6, 1e-6))
    o = oracle.Oracle(p)
    m = o.mech_mask(W.MECH_KINEMATIC)
    # x nodes 0,1,2,5,6 um: mid 3 um -> nearest node 2 (2 um, lower on tie); y: 6 cells -> node 3
    expect = np.zeros_like(m)
    expect[0, 3, 2] = 7
    expect[0, 3, 4] = 6
    expect[0, 6, 2] = 4
    np.testing.assert_array_equal(m, expect)
