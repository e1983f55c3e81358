"""Full-size parity: the 256x256x64 graded slice and the 1024x1024x128
package, in the launch configuration the benchmark times (automatic tile
z-chunks, one plan per GPU stream), against the oracle on sampled outputs.

The EM + Joule + thermal march is explicit: one EM step couples an edge to
edges at most one cell away, a thermal step a node to its six neighbours.
After n steps the fields at a node therefore depend only on the data within
n cells.  For each sample node the oracle marches a window of n + 3 cells
around it (faces on the true boundary keep their condition, cut faces are
PMC) with the full problem's time step and sources, and every field within
2 nodes of the sample must match the full-size GPU run.  Samples sit on the
x- and y-tile borders of the march kernel, on z-chunk borders, in the ragged
last node column and plane, at the domain corners and next to the
workload's own ports.  A current source ramping up over 1 ps is added at
each sample so that the fields there are non-zero from the first step.  (A
step in the current would kick the odd-even mode the central difference
has in good conductors, where a = dt sigma / (2 eps0) is ~1e4: the edge
field then swings between ~0 and twice its steady value every step, and
the compared values at the low phase are a cancellation of that swing.)

The mechanical solve is checked by properties that hold at any size: the
GPU displacement satisfies the oracle's FP64 equations K u = f to the
solver tolerance, and the von Mises stress of every cell equals the
oracle's evaluation of the same displacement and temperature."""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
import paper_2603_07038_amd as etm
import workloads as W

pytestmark = pytest.mark.gpu

N_STEPS, R = 14, 4        # 3 thermal steps, then 2 steps of pending Joule power
MARGIN = N_STEPS + 3      # window half-width in cells
NEAR = 2                  # compared nodes around each sample


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _samples(prob):
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    s = [(0, 0, 0), (nx, ny, nz), (nx, 0, nz // 2), (63, 3, 7), (64, 4, 8), (127, 5, 16), (128, 2, 15),
         (nx - 1, ny - 1, 31), (nx // 2, ny, 32), (65, ny // 2, nz), (191, 127, 24)]
    if prob.n_ports:
        q = len(prob.port_i) // 2
        s.append((int(prob.port_i[q]) + 1, int(prob.port_j[q]), int(prob.port_k[q])))
    return [(min(i, nx), min(j, ny), min(k, nz)) for i, j, k in s]


def _with_probe_sources(prob, samples, amp=3e10):
    """The problem plus one z-directed current source (a 1 ps linear ramp)
    at each sample node (at the node below it on the top plane)."""
    w = len(prob.waves)
    add = [(2, i, j, min(k, prob.nz - 1), w, amp, 0.0) for i, j, k in samples]
    a = np.array(add, dtype=np.float64)
    return dataclasses.replace(
        prob,
        port_dir=np.concatenate([prob.port_dir, a[:, 0].astype(np.uint8)]),
        port_i=np.concatenate([prob.port_i, a[:, 1].astype(np.int32)]),
        port_j=np.concatenate([prob.port_j, a[:, 2].astype(np.int32)]),
        port_k=np.concatenate([prob.port_k, a[:, 3].astype(np.int32)]),
        port_wave=np.concatenate([prob.port_wave, a[:, 4].astype(np.int32)]),
        port_weight=np.concatenate([prob.port_weight, a[:, 5]]),
        port_g=np.concatenate([prob.port_g, a[:, 6]]),
        waves=list(prob.waves) + [W.Wave("ramp", amp=1.0, rise=1e-12)],
        em_per_thermal=R, mech_every_thermal=0, n_em_steps=N_STEPS, probes=None, history_stride=0)


def _window(prob, s):
    """Sub-problem of the cells within MARGIN of node s; returns it and the
    cell offset of its origin."""
    lo = [max(c - MARGIN, 0) for c in s]
    hi = [min(c + MARGIN, n) for c, n in zip(s, (prob.nx, prob.ny, prob.nz))]
    (i0, j0, k0), (i1, j1, k1) = lo, hi
    keep = []
    for q in range(prob.n_ports):
        d, i, j, k = int(prob.port_dir[q]), int(prob.port_i[q]), int(prob.port_j[q]), int(prob.port_k[q])
        e1 = (i + (d == 0), j + (d == 1), k + (d == 2))
        if i0 <= i and e1[0] <= i1 and j0 <= j and e1[1] <= j1 and k0 <= k and e1[2] <= k1:
            keep.append(q)
    keep = np.array(keep, dtype=np.int64)
    bc = list(prob.em_bc)
    for f, cut in enumerate((i0 > 0, i1 < prob.nx, j0 > 0, j1 < prob.ny, k0 > 0, k1 < prob.nz)):
        if cut:
            bc[f] = W.PMC
    sub = dataclasses.replace(
        prob, name=f"{prob.name}_win{s}", dx=prob.dx[i0:i1].copy(), dy=prob.dy[j0:j1].copy(),
        dz=prob.dz[k0:k1].copy(), mat=np.ascontiguousarray(prob.mat[k0:k1, j0:j1, i0:i1]),
        port_dir=prob.port_dir[keep], port_i=(prob.port_i[keep] - i0).astype(np.int32),
        port_j=(prob.port_j[keep] - j0).astype(np.int32), port_k=(prob.port_k[keep] - k0).astype(np.int32),
        port_wave=prob.port_wave[keep], port_weight=prob.port_weight[keep], port_g=prob.port_g[keep],
        em_bc=tuple(bc))
    return sub, (i0, j0, k0)


def _near(shape, s, org):
    """Index slices (z, y, x) of the nodes within NEAR of node s in a
    full-size field of the given shape, and the same nodes in the window
    whose cell origin is org."""
    full, win = [], []
    for c, n, o in zip(reversed(s), shape, reversed(org)):
        a, b = max(c - NEAR, 0), min(c + NEAR + 1, n)
        full.append(slice(a, b))
        win.append(slice(a - o, b - o))
    return tuple(full), tuple(win)


def _rel(a, b, scale):
    return float(np.abs(a - b).max() / max(scale, 1e-300))


def _march_parity(prob, precision, e_tol, th_tol):
    samples = _samples(prob)
    prob = _with_probe_sources(prob, samples)
    dt = etm.cfl_dt(prob)
    J = prob.sample_J_half(dt, N_STEPS)
    _say(f"[fullsize] {prob.name} {prob.nx}x{prob.ny}x{prob.nz} prec={precision} steps={N_STEPS} R={R}")
    plan = etm.Plan(prob, J, dt=dt, precision=precision, n_steps=N_STEPS, history=False)
    plan.advance(N_STEPS)
    info = plan.sync()
    assert info["step"] == N_STEPS
    eg = plan.e()
    thg = plan.read(etm.ETM_FIELD_THETA)
    pg = plan.read(etm.ETM_FIELD_PSUM)
    del plan
    worst = {"e": 0.0, "theta": 0.0, "psum": 0.0}
    for s in samples:
        sub, org = _window(prob, s)
        o = oracle.Oracle(sub)
        st, _ = o.run(dt, N_STEPS, J, R=R)
        escale = max(float(np.abs(x).max()) for x in st["e"])
        assert escale > 0.0, s
        for c in range(3):
            f, w = _near(eg[c].shape, s, org)
            worst["e"] = max(worst["e"], _rel(eg[c][f], st["e"][c][w], escale))
        f, w = _near(thg.shape, s, org)
        worst["theta"] = max(worst["theta"], _rel(thg[f], st["theta"][w], float(np.abs(st["theta"]).max())))
        worst["psum"] = max(worst["psum"], _rel(pg[f], st["psum"][w], float(np.abs(st["psum"]).max())))
        _say(f"[fullsize]   sample {s} window {sub.nx}x{sub.ny}x{sub.nz} worst so far {worst}")
    assert worst["e"] < e_tol, worst
    assert worst["theta"] < th_tol, worst
    assert worst["psum"] < th_tol, worst


@pytest.mark.parametrize("precision", [etm.ETM_PREC_FP64, etm.ETM_PREC_MIXED])
def test_slice256_march_sampled_against_oracle(precision):
    fp64 = precision == etm.ETM_PREC_FP64
    _march_parity(W.config2(), precision, 1e-9 if fp64 else 1e-5, 1e-9 if fp64 else 1e-6)


@pytest.mark.parametrize("precision", [etm.ETM_PREC_FP64, etm.ETM_PREC_MIXED])
def test_package1024_march_sampled_against_oracle(precision):
    fp64 = precision == etm.ETM_PREC_FP64
    _march_parity(W.config3(), precision, 1e-9 if fp64 else 1e-5, 1e-9 if fp64 else 1e-6)


def test_slice256_mechanics_satisfies_oracle_equations():
    """Mixed-precision solve (FP32 multigrid-PCG inside FP64 refinement) at
    full size: ||f - K u|| / ||f|| from the oracle's FP64 operator, and von
    Mises of every cell from the oracle's evaluation of the same u."""
    prob = W.config2()
    prob = _with_probe_sources(prob, _samples(prob))
    dt = etm.cfl_dt(prob)
    J = prob.sample_J_half(dt, N_STEPS)
    _say(f"[fullsize] {prob.name} mechanics after {N_STEPS} steps")
    plan = etm.Plan(prob, J, dt=dt, precision=etm.ETM_PREC_MIXED, n_steps=N_STEPS, history=False)
    plan.advance(N_STEPS)
    plan.mech_solve()
    info = plan.sync()
    th = plan.read(etm.ETM_FIELD_THETA)
    u = plan.u()
    vm = plan.read(etm.ETM_FIELD_VM)
    del plan
    assert th.max() > 0.0
    o = oracle.Oracle(prob)
    mask = o.mech_mask()
    f = o.mech_rhs(th, mask)
    r = f - o.mech_apply(mask, u)
    relres = float(np.linalg.norm(r) / np.linalg.norm(f))
    vm_err = _rel(vm, o.von_mises(th, u), float(np.abs(vm).max()))
    _say(f"[fullsize]   cg iters {info['cg_iters']} gpu relres {info['cg_relres']:.3e} oracle relres {relres:.3e} "
         f"vm err {vm_err:.3e}")
    assert relres < 2e-8
    assert vm_err < 1e-9
