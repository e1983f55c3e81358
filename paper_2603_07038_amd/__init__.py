"""Python binding of libetm (include/etm.h): the MI355X transient coupled
EM-thermal-mechanical package solver of arXiv 2603.07038, Sec. II.

Argument marshalling only: every step of the method runs in the gfx950 HIP
kernels of libetm.so.  PyTorch provides device memory (one uint8 workspace
tensor per plan) and the HIP stream.  The library must be built in-tree
(``python -m paper_2603_07038_amd.build``); importing this package fails
loudly when it is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libetm.so")

# ---- constants (mirror etm.h) ------------------------------------------------
ETM_OK, ETM_E_INVAL, ETM_E_NOMEM, ETM_E_HIP, ETM_E_UNSTABLE, ETM_E_NOCONV, ETM_E_STATE = 0, -1, -2, -3, -4, -5, -6
ETM_PMC, ETM_PEC = 0, 1
ETM_MECH_KINEMATIC, ETM_MECH_CLAMP_ZMIN = 0, 1
ETM_PREC_FP64, ETM_PREC_MIXED = 0, 1
ETM_PRECOND_JACOBI, ETM_PRECOND_MG = 0, 1
(ETM_FIELD_EX, ETM_FIELD_EY, ETM_FIELD_EZ, ETM_FIELD_EX_PREV, ETM_FIELD_EY_PREV, ETM_FIELD_EZ_PREV,
 ETM_FIELD_THETA, ETM_FIELD_PSUM, ETM_FIELD_UX, ETM_FIELD_UY, ETM_FIELD_UZ, ETM_FIELD_VM,
 ETM_FIELD_FX, ETM_FIELD_FY, ETM_FIELD_FZ) = range(15)
STATUS_NAMES = {0: "ETM_OK", -1: "ETM_E_INVAL", -2: "ETM_E_NOMEM", -3: "ETM_E_HIP", -4: "ETM_E_UNSTABLE",
                -5: "ETM_E_NOCONV", -6: "ETM_E_STATE"}


class etm_material(C.Structure):
    _fields_ = [("eps_r", C.c_double), ("sigma0", C.c_double), ("tcr", C.c_double), ("k", C.c_double),
                ("rho_cp", C.c_double), ("E", C.c_double), ("nu", C.c_double), ("cte", C.c_double),
                ("is_void", C.c_int32), ("reserved", C.c_int32)]


class etm_mesh(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.POINTER(C.c_double)), ("dy", C.POINTER(C.c_double)), ("dz", C.POINTER(C.c_double)),
                ("mat", C.POINTER(C.c_uint8))]


class etm_port(C.Structure):
    _fields_ = [("dir", C.c_int32), ("i", C.c_int32), ("j", C.c_int32), ("k", C.c_int32), ("wave", C.c_int32),
                ("reserved", C.c_int32), ("weight", C.c_double), ("g", C.c_double)]


ETM_WAVE_RICKER, ETM_WAVE_SINE, ETM_WAVE_GAUSS_TRAIN = 1, 2, 3
ETM_WAVE_MAX_PULSES = 8


class etm_wave(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_pulses", C.c_int32), ("amp", C.c_double), ("t0", C.c_double),
                ("width", C.c_double), ("freq", C.c_double), ("t_on", C.c_double), ("t_off", C.c_double),
                ("pulse_t", C.c_double * ETM_WAVE_MAX_PULSES)]


class etm_source(C.Structure):
    _fields_ = [("n_ports", C.c_int64), ("ports", C.POINTER(etm_port)), ("n_waves", C.c_int32),
                ("n_samples", C.c_int64), ("J_half", C.POINTER(C.c_double)), ("n_analytic", C.c_int32),
                ("reserved", C.c_int32), ("analytic", C.POINTER(etm_wave))]


class etm_opts(C.Structure):
    _fields_ = [("dt", C.c_double), ("cfl", C.c_double), ("force_dt", C.c_int32), ("precision", C.c_int32),
                ("em_bc", C.c_int32 * 6), ("em_per_thermal", C.c_int32), ("mech_every_thermal", C.c_int32),
                ("mech_bc", C.c_int32), ("mech_mask", C.POINTER(C.c_uint8)), ("cg_maxit", C.c_int32),
                ("cg_rtol", C.c_double), ("history_stride", C.c_int32), ("n_probes", C.c_int32),
                ("probes", C.POINTER(C.c_int64)), ("history_cap", C.c_int64), ("n_em_steps_hint", C.c_int64),
                ("mech_precond", C.c_int32), ("mg_coarse_dofs", C.c_int32), ("mg_degree", C.c_int32 * 2),
                ("em_slabs", C.c_int32), ("mech_overlap", C.c_int32)]


class etm_run_info(C.Structure):
    _fields_ = [("step", C.c_int64), ("status", C.c_int32), ("cg_iters", C.c_int32), ("cg_outer", C.c_int32),
                ("n_solves", C.c_int32), ("cg_relres", C.c_double), ("theta_max", C.c_double),
                ("ejoule", C.c_double), ("n_records", C.c_int64), ("cg_iters_total", C.c_int64),
                ("mg_levels", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class EtmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_P = C.c_void_p
_lib = None


def load():
    """Load libetm.so; raise if it has not been built (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2603_07038_amd.build`")
    # torch ships its own HIP runtime; load it first so that libetm binds to the
    # same runtime instance as the tensors and streams it is handed.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    sig = {
        "etm_opts_default": [C.POINTER(etm_opts)],
        "etm_cfl_dt": [C.POINTER(etm_mesh), C.c_double, C.POINTER(C.c_double)],
        "etm_plan_create": [C.POINTER(etm_mesh), C.POINTER(etm_material), C.c_int32, C.POINTER(etm_source),
                            C.POINTER(etm_opts), C.POINTER(_P)],
        "etm_plan_footprint": [_P, C.POINTER(C.c_size_t)],
        "etm_plan_dt": [_P, C.POINTER(C.c_double)],
        "etm_plan_dofs": [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
        "etm_plan_bind": [_P, _P, C.c_size_t, _P],
        "etm_advance": [_P, C.c_int64],
        "etm_mech_solve": [_P],
        "etm_sync": [_P, C.POINTER(etm_run_info)],
        "etm_read": [_P, C.c_int32, _P, C.c_size_t, C.c_int32],
        "etm_write": [_P, C.c_int32, _P, C.c_size_t, C.c_int32],
        "etm_read_history": [_P, C.POINTER(C.c_double), C.c_size_t, C.POINTER(C.c_int64)],
        "etm_checkpoint_size": [_P, C.POINTER(C.c_size_t)],
        "etm_checkpoint": [_P, _P, C.c_size_t],
        "etm_restore": [_P, _P, C.c_size_t],
        "etm_batch_create": [C.c_int32, C.c_char_p, C.POINTER(_P)],
        "etm_batch_attach": [_P, _P, C.POINTER(C.c_int32)],
        "etm_batch_detach": [_P, C.c_int32],
        "etm_batch_advance": [_P, C.c_int64, _P],
        "etm_batch_advance_noalloc": [_P, C.c_int64, _P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int32
    L.etm_plan_destroy.argtypes = [_P]
    L.etm_plan_destroy.restype = None
    L.etm_batch_destroy.argtypes = [_P]
    L.etm_batch_destroy.restype = None
    L.etm_last_error.argtypes = []
    L.etm_last_error.restype = C.c_char_p
    _lib = L
    return L


def check(status):
    if status != ETM_OK:
        msg = load().etm_last_error().decode(errors="replace")
        raise EtmError(status, msg)
    return status


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


# ---- marshalling of a workloads.Problem -------------------------------------
class _Inputs:
    """Keeps the ctypes views of a problem's arrays alive for one call."""

    def __init__(self, prob, J_half, device_waves=False):
        self.dx = np.ascontiguousarray(prob.dx, dtype=np.float64)
        self.dy = np.ascontiguousarray(prob.dy, dtype=np.float64)
        self.dz = np.ascontiguousarray(prob.dz, dtype=np.float64)
        self.mat = np.ascontiguousarray(prob.mat, dtype=np.uint8)
        self.mesh = etm_mesh(prob.nx, prob.ny, prob.nz, _dp(self.dx), _dp(self.dy), _dp(self.dz),
                             self.mat.ctypes.data_as(C.POINTER(C.c_uint8)))
        props = np.asarray(prob.props, dtype=np.float64)
        self.mats = (etm_material * props.shape[0])()
        for m, row in enumerate(props):
            self.mats[m] = etm_material(*[float(x) for x in row[:8]], int(row[8] != 0), 0)
        n = prob.n_ports
        self.ports = (etm_port * max(n, 1))()
        for q in range(n):
            self.ports[q] = etm_port(int(prob.port_dir[q]), int(prob.port_i[q]), int(prob.port_j[q]),
                                     int(prob.port_k[q]), int(prob.port_wave[q]), 0, float(prob.port_weight[q]),
                                     float(prob.port_g[q]))
        if device_waves:
            # every wave as a closed-form record evaluated on the device; no table
            self.waves = (etm_wave * max(len(prob.waves), 1))()
            for w, wave in enumerate(prob.waves):
                d = wave.device_params()
                pt = (C.c_double * ETM_WAVE_MAX_PULSES)(*[float(x) for x in d["pulse_t"]][:ETM_WAVE_MAX_PULSES])
                self.waves[w] = etm_wave(d["kind"], d["n_pulses"], float(d["amp"]), float(d["t0"]), float(d["width"]),
                                         float(d["freq"]), float(d["t_on"]), float(d["t_off"]), pt)
            self.J = np.zeros((1, 1))
            self.src = etm_source(n, self.ports, 0, 0, _dp(self.J), len(prob.waves), 0, self.waves)
        else:
            self.J = np.ascontiguousarray(J_half, dtype=np.float64) if J_half is not None else np.zeros((1, 1))
            self.src = etm_source(n, self.ports, int(self.J.shape[0]), int(self.J.shape[1]), _dp(self.J), 0, 0, None)


def make_opts(prob, *, dt=0.0, precision=ETM_PREC_FP64, n_steps=None, mech_mask=None, force_dt=False,
              cg_maxit=200000, history=True, **overrides):
    o = etm_opts()
    check(load().etm_opts_default(C.byref(o)))
    o.dt = float(dt)
    o.cfl = float(prob.cfl)
    o.force_dt = int(bool(force_dt))
    o.precision = int(precision)
    for f in range(6):
        o.em_bc[f] = int(prob.em_bc[f])
    o.em_per_thermal = int(prob.em_per_thermal)
    o.mech_every_thermal = int(prob.mech_every_thermal)
    o.mech_bc = int(prob.mech_bc)
    o.cg_maxit = int(cg_maxit)
    o.cg_rtol = float(prob.cg_rtol)
    keep = []
    if mech_mask is not None:
        mm = np.ascontiguousarray(mech_mask, dtype=np.uint8)
        keep.append(mm)
        o.mech_mask = mm.ctypes.data_as(C.POINTER(C.c_uint8))
    if history and prob.history_stride and prob.history_stride > 0:
        o.history_stride = int(prob.history_stride)
        pr = np.zeros((0, 4), dtype=np.int64) if prob.probes is None else np.ascontiguousarray(prob.probes, dtype=np.int64)
        keep.append(pr)
        o.n_probes = int(pr.shape[0])
        o.probes = pr.ctypes.data_as(C.POINTER(C.c_int64))
    o.n_em_steps_hint = int(prob.n_em_steps if n_steps is None else n_steps)
    for k, v in overrides.items():
        if isinstance(v, (list, tuple)):   # array fields (em_bc, mg_degree)
            v = type(getattr(o, k))(*v)
        setattr(o, k, v)
    return o, keep


def cfl_dt(prob, cfl=None):
    inp = _Inputs(prob, None)
    out = C.c_double()
    check(load().etm_cfl_dt(C.byref(inp.mesh), float(prob.cfl if cfl is None else cfl), C.byref(out)))
    return out.value


class Plan:
    """One design on the GPU: etm_plan_create + a torch workspace + bind."""

    def __init__(self, prob, J_half, *, device="cuda", stream=None, bind=True, device_waves=False, **opt_kw):
        """J_half: sampled waves [n_waves][n_steps + 1] (see Problem.sample_J_half),
        or None with device_waves=True, where every wave of the problem is
        passed as a closed-form record and evaluated on the device."""
        import torch
        L = load()
        self.prob = prob
        inp = _Inputs(prob, J_half, device_waves)
        o, keep = make_opts(prob, **opt_kw)
        h = _P()
        check(L.etm_plan_create(C.byref(inp.mesh), inp.mats, int(prob.props.shape[0]), C.byref(inp.src), C.byref(o),
                                C.byref(h)))
        self.h = h
        self.precision = o.precision
        self.hist_cols = 4 + o.n_probes
        fp = C.c_size_t()
        check(L.etm_plan_footprint(self.h, C.byref(fp)))
        self.footprint = fp.value
        self.ws = None
        self.stream = None
        if bind:
            self.bind(torch.empty(self.footprint + 256, dtype=torch.uint8, device=device), stream)

    def bind(self, ws_tensor, stream=None):
        import torch
        base = ws_tensor.data_ptr()
        off = (-base) % 256
        self.ws = ws_tensor
        self.stream = stream if stream is not None else torch.cuda.current_stream(ws_tensor.device)
        check(load().etm_plan_bind(self.h, C.c_void_p(base + off), self.footprint, C.c_void_p(self.stream.cuda_stream)))

    def __del__(self):
        try:
            if getattr(self, "h", None):
                load().etm_plan_destroy(self.h)
                self.h = None
        except Exception:
            pass

    @property
    def dt(self):
        v = C.c_double()
        check(load().etm_plan_dt(self.h, C.byref(v)))
        return v.value

    def dofs(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        check(load().etm_plan_dofs(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def advance(self, n):
        check(load().etm_advance(self.h, int(n)))

    def mech_solve(self):
        check(load().etm_mech_solve(self.h))

    def sync(self, raise_on_error=True):
        info = etm_run_info()
        st = load().etm_sync(self.h, C.byref(info))
        if raise_on_error:
            check(st)
        return info.as_dict()

    def field_shape(self, field):
        nx, ny, nz = self.prob.nx, self.prob.ny, self.prob.nz
        if field in (ETM_FIELD_EX, ETM_FIELD_EX_PREV):
            return (nz + 1, ny + 1, nx)
        if field in (ETM_FIELD_EY, ETM_FIELD_EY_PREV):
            return (nz + 1, ny, nx + 1)
        if field in (ETM_FIELD_EZ, ETM_FIELD_EZ_PREV):
            return (nz, ny + 1, nx + 1)
        if field == ETM_FIELD_VM:
            return (nz, ny, nx)
        return (nz + 1, ny + 1, nx + 1)

    def read(self, field):
        out = np.empty(self.field_shape(field), dtype=np.float64)
        check(load().etm_read(self.h, int(field), out.ctypes.data, out.nbytes, 0))
        return out

    def write(self, field, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64)
        assert a.shape == self.field_shape(field)
        check(load().etm_write(self.h, int(field), a.ctypes.data, a.nbytes, 0))

    def e(self):
        return [self.read(ETM_FIELD_EX), self.read(ETM_FIELD_EY), self.read(ETM_FIELD_EZ)]

    def e_prev(self):
        return [self.read(ETM_FIELD_EX_PREV), self.read(ETM_FIELD_EY_PREV), self.read(ETM_FIELD_EZ_PREV)]

    def u(self):
        return np.stack([self.read(ETM_FIELD_UX), self.read(ETM_FIELD_UY), self.read(ETM_FIELD_UZ)], axis=-1)

    def history(self, max_rows=1 << 20):
        cap = np.empty((max_rows, self.hist_cols), dtype=np.float64)
        n = C.c_int64()
        check(load().etm_read_history(self.h, _dp(cap), cap.nbytes, C.byref(n)))
        return cap[: n.value].copy()

    def checkpoint(self):
        n = C.c_size_t()
        check(load().etm_checkpoint_size(self.h, C.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        check(load().etm_checkpoint(self.h, buf.ctypes.data, buf.nbytes))
        return buf

    def restore(self, buf):
        check(load().etm_restore(self.h, buf.ctypes.data, buf.nbytes))


def solve_all(plans, workers=8):
    """Mechanical solves of several bound plans at once.  Each solve runs from
    a worker thread on its plan's own stream (the library releases the GIL
    while it waits), so the small solves of a batch overlap on the GPU.
    Returns each plan's run info."""
    from concurrent.futures import ThreadPoolExecutor

    def one(pl):
        pl.mech_solve()
        return pl.sync()

    with ThreadPoolExecutor(max_workers=max(1, int(workers))) as ex:
        return list(ex.map(one, plans))


class Batch:
    """Several bound plans advanced together (etm_batch_*): one launch per EM
    step over all variants, chunks of steps replayed from HIP graphs."""

    def __init__(self, max_slots, tune_json=None):
        """tune_json: the autotuner's table (JSON text); None reads the table
        committed next to this file, if any ("{}" for built-in defaults)."""
        h = _P()
        if tune_json is None:
            path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_gfx950.json")
            if os.path.exists(path):
                with open(path) as f:
                    tune_json = f.read()
        tj = None if tune_json is None else tune_json.encode()
        check(load().etm_batch_create(int(max_slots), tj, C.byref(h)))
        self.h = h
        self.plans = {}

    def attach(self, plan):
        s = C.c_int32()
        check(load().etm_batch_attach(self.h, plan.h, C.byref(s)))
        self.plans[s.value] = plan
        return s.value

    def detach(self, slot):
        check(load().etm_batch_detach(self.h, int(slot)))
        self.plans.pop(slot, None)

    def advance(self, n, stream=None):
        import torch
        st = stream if stream is not None else torch.cuda.current_stream()
        check(load().etm_batch_advance(self.h, int(n), C.c_void_p(st.cuda_stream)))

    def advance_noalloc(self, n, stream=None):
        """etm_batch_advance_noalloc: the same steps from the library's fixed
        device scratch, without any device allocation or graph."""
        import torch
        st = stream if stream is not None else torch.cuda.current_stream()
        check(load().etm_batch_advance_noalloc(self.h, int(n), C.c_void_p(st.cuda_stream)))

    def __del__(self):
        try:
            if getattr(self, "h", None):
                load().etm_batch_destroy(self.h)
                self.h = None
        except Exception:
            pass
