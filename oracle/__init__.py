"""FP64 CPU oracle of the coupled EM-thermal-mechanical method (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library; the only shared module is ``workloads`` (inputs).

Arrays use natural per-component shapes, C order, x fastest:
  ex (nz+1, ny+1, nx), ey (nz+1, ny, nx+1), ez (nz, ny+1, nx+1),
  node fields (nz+1, ny+1, nx+1), displacement (nz+1, ny+1, nx+1, 3),
  cell fields (nz, ny, nx).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = C.POINTER(C.c_double)
_u8p = C.POINTER(C.c_uint8)
_ip = C.POINTER(C.c_int)
_i64p = C.POINTER(C.c_int64)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Plain C, no fast-math."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall",
                               "-Wno-unused-function", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        L.or_create.restype = C.c_void_p
        L.or_create.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, _u8p, _dp, C.c_int, _ip]
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_set_ports.argtypes = [C.c_void_p, C.c_int, _u8p, _ip, _ip, _ip, _ip, _dp, _dp]
        L.or_n_edges.restype = C.c_int64
        L.or_n_edges.argtypes = [C.c_void_p, C.c_int]
        L.or_n_nodes.restype = C.c_int64
        L.or_n_nodes.argtypes = [C.c_void_p]
        L.or_cfl_dt.restype = C.c_double
        L.or_cfl_dt.argtypes = [C.c_void_p, C.c_double]
        L.or_curlcurl.argtypes = [C.c_void_p] + [_dp] * 6
        L.or_edge_coeffs.argtypes = [C.c_void_p, _dp, C.c_int, _dp, _dp, _dp, _dp, _u8p]
        L.or_em_step.argtypes = [C.c_void_p, C.c_double, _dp] + [_dp] * 9 + [_dp, _dp]
        L.or_joule.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp]
        L.or_joule_total.restype = C.c_double
        L.or_joule_total.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
        L.or_heat_capacity.argtypes = [C.c_void_p, _dp]
        L.or_thermal_step.argtypes = [C.c_void_p, C.c_double, _dp, _dp, _dp]
        L.or_em_energy.restype = C.c_double
        L.or_em_energy.argtypes = [C.c_void_p, C.c_double] + [_dp] * 6
        L.or_run.restype = C.c_int
        L.or_run.argtypes = [C.c_void_p, C.c_double, C.c_int64, C.c_int64, C.c_int, _dp, C.c_int,
                             C.c_int64] + [_dp] * 6 + [_dp, _dp, _dp, C.c_int, C.c_int, _i64p,
                                                       _dp, C.c_int64]
        L.or_hex8_element.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, _dp, _dp, _dp]
        L.or_mech_mask.argtypes = [C.c_void_p, C.c_int, _u8p]
        L.or_mech_rhs.argtypes = [C.c_void_p, _dp, _u8p, _dp]
        L.or_mech_apply.argtypes = [C.c_void_p, _u8p, _dp, _dp]
        L.or_mech_solve.restype = C.c_int
        L.or_mech_solve.argtypes = [C.c_void_p, _dp, _u8p, C.c_double, C.c_int, _dp, _dp]
        L.or_von_mises.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
        L.or_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a, t=_dp):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """One problem's grid, materials and ports held by the C oracle."""

    def __init__(self, prob, em_bc=None):
        L = lib()
        self.prob = prob
        self.nx, self.ny, self.nz = prob.nx, prob.ny, prob.nz
        self._keep = [_f64(prob.dx), _f64(prob.dy), _f64(prob.dz),
                      np.ascontiguousarray(prob.mat, dtype=np.uint8), _f64(prob.props)]
        bc = np.array(prob.em_bc if em_bc is None else em_bc, dtype=np.int32)
        self.h = L.or_create(self.nx, self.ny, self.nz, _p(self._keep[0]), _p(self._keep[1]),
                             _p(self._keep[2]), _p(self._keep[3], _u8p), _p(self._keep[4]),
                             int(prob.props.shape[0]), _p(bc, _ip))
        n = prob.n_ports
        pd = np.ascontiguousarray(prob.port_dir, dtype=np.uint8)
        pi = np.ascontiguousarray(prob.port_i, dtype=np.int32)
        pj = np.ascontiguousarray(prob.port_j, dtype=np.int32)
        pk = np.ascontiguousarray(prob.port_k, dtype=np.int32)
        pw = np.ascontiguousarray(prob.port_wave, dtype=np.int32)
        pwt, pg = _f64(prob.port_weight), _f64(prob.port_g)
        L.or_set_ports(self.h, n, _p(pd, _u8p), _p(pi, _ip), _p(pj, _ip), _p(pk, _ip), _p(pw, _ip),
                       _p(pwt), _p(pg))

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().or_destroy(self.h)
                self.h = None
        except Exception:
            pass

    # shapes
    @property
    def edge_shapes(self):
        nx, ny, nz = self.nx, self.ny, self.nz
        return [(nz + 1, ny + 1, nx), (nz + 1, ny, nx + 1), (nz, ny + 1, nx + 1)]

    @property
    def node_shape(self):
        return (self.nz + 1, self.ny + 1, self.nx + 1)

    @property
    def cell_shape(self):
        return (self.nz, self.ny, self.nx)

    def zeros_e(self):
        return [np.zeros(s) for s in self.edge_shapes]

    def cfl_dt(self, cfl=None):
        return lib().or_cfl_dt(self.h, self.prob.cfl if cfl is None else cfl)

    def curlcurl(self, e):
        e = [_f64(a) for a in e]
        out = self.zeros_e()
        lib().or_curlcurl(self.h, *[_p(a) for a in e], *[_p(a) for a in out])
        return out

    def edge_coeffs(self, d, theta=None):
        shp = self.edge_shapes[d]
        vol, eps, sig, kth = (np.zeros(shp) for _ in range(4))
        pec = np.zeros(shp, dtype=np.uint8)
        lib().or_edge_coeffs(self.h, _p(None if theta is None else _f64(theta)), d, _p(vol), _p(eps),
                             _p(sig), _p(kth), _p(pec, _u8p))
        return dict(vol=vol, eps=eps, sig=sig, kth=kth, pec=pec.astype(bool))

    def em_step(self, dt, theta, e_prev, e_cur, J_new, J_old):
        e_prev = [_f64(a) for a in e_prev]
        e_cur = [_f64(a) for a in e_cur]
        out = self.zeros_e()
        th = None if theta is None else _f64(theta)
        lib().or_em_step(self.h, dt, _p(th), *[_p(a) for a in e_prev], *[_p(a) for a in e_cur],
                         *[_p(a) for a in out], _p(_f64(J_new)), _p(_f64(J_old)))
        return out

    def joule(self, theta, e):
        P = np.zeros(self.node_shape)
        th = None if theta is None else _f64(theta)
        lib().or_joule(self.h, _p(th), *[_p(_f64(a)) for a in e], _p(P))
        return P

    def joule_total(self, theta, e):
        th = None if theta is None else _f64(theta)
        return lib().or_joule_total(self.h, _p(th), *[_p(_f64(a)) for a in e])

    def heat_capacity(self):
        CV = np.zeros(self.node_shape)
        lib().or_heat_capacity(self.h, _p(CV))
        return CV

    def thermal_step(self, dt_th, theta, pbar):
        out = np.zeros(self.node_shape)
        lib().or_thermal_step(self.h, dt_th, _p(_f64(theta)), _p(_f64(pbar)), _p(out))
        return out

    def em_energy(self, dt, e0, e1):
        return lib().or_em_energy(self.h, dt, *[_p(_f64(a)) for a in e0], *[_p(_f64(a)) for a in e1])

    def new_state(self):
        return dict(e=self.zeros_e(), e_prev=self.zeros_e(), theta=np.zeros(self.node_shape),
                    psum=np.zeros(self.node_shape), ejoule=np.zeros(1), step=0)

    def run(self, dt, n_steps, J_half, state=None, R=None, stride=0, probes=None):
        """Advance the coupled EM + Joule + thermal march by n_steps from
        ``state`` (a fresh zero state if None).  Returns (state, history)."""
        p = self.prob
        st = self.new_state() if state is None else state
        R = p.em_per_thermal if R is None else R
        Jh = _f64(J_half)
        nw, ns = Jh.shape
        prb = np.zeros((0, 4), dtype=np.int64) if probes is None else np.ascontiguousarray(probes, dtype=np.int64)
        cap = (n_steps // stride + 1) if stride > 0 else 0
        hist = np.zeros((max(cap, 1), 4 + prb.shape[0]))
        rec = lib().or_run(self.h, dt, st["step"], n_steps, R, _p(Jh), nw, ns,
                           *[_p(a) for a in st["e"]], *[_p(a) for a in st["e_prev"]],
                           _p(st["theta"]), _p(st["psum"]), _p(st["ejoule"]), stride,
                           prb.shape[0], _p(prb, _i64p), _p(hist), cap)
        st["step"] += n_steps
        return st, hist[:rec]

    # -- mechanics ---------------------------------------------------------
    def hex8_element(self, i, j, k, theta8=None):
        Ke = np.zeros((24, 24))
        fe = np.zeros(24)
        lib().or_hex8_element(self.h, i, j, k, _p(None if theta8 is None else _f64(theta8)), _p(Ke), _p(fe))
        return Ke, fe

    def mech_mask(self, mech_bc=None):
        m = np.zeros(self.node_shape, dtype=np.uint8)
        lib().or_mech_mask(self.h, self.prob.mech_bc if mech_bc is None else mech_bc, _p(m, _u8p))
        return m

    def mech_rhs(self, theta, mask):
        f = np.zeros(self.node_shape + (3,))
        lib().or_mech_rhs(self.h, _p(_f64(theta)), _p(np.ascontiguousarray(mask, dtype=np.uint8), _u8p), _p(f))
        return f

    def mech_apply(self, mask, q):
        y = np.zeros(self.node_shape + (3,))
        lib().or_mech_apply(self.h, _p(np.ascontiguousarray(mask, dtype=np.uint8), _u8p), _p(_f64(q)), _p(y))
        return y

    def mech_solve(self, theta, mask, rtol=1e-12, maxit=100000, q0=None):
        q = np.zeros(self.node_shape + (3,)) if q0 is None else _f64(q0).copy()
        rr = np.zeros(1)
        it = lib().or_mech_solve(self.h, _p(_f64(theta)), _p(np.ascontiguousarray(mask, dtype=np.uint8), _u8p),
                                 rtol, maxit, _p(q), _p(rr))
        return q, it, float(rr[0])

    def von_mises(self, theta, q, want_stress=False):
        vm = np.zeros(self.cell_shape)
        s6 = np.zeros(self.cell_shape + (6,)) if want_stress else None
        lib().or_von_mises(self.h, _p(_f64(theta)), _p(_f64(q)), _p(vm), _p(s6))
        return (vm, s6) if want_stress else vm


def num_threads() -> int:
    return int(lib().or_num_threads())
