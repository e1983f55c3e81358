"""Seeded synthetic inputs for the coupled EM-thermal-mechanical package solver.

This module is the only code shared by the FP64 oracle and the HIP library.
It describes *inputs only*: a rectilinear voxel mesh, one material id per
cell, a material table, port edges and excitation waveforms (sampled here,
or handed to the library as closed-form records).  It holds
none of the method's arithmetic (no curl-curl, no Joule map, no conduction,
no elasticity); each side derives everything else on its own.

Units are SI throughout (metres, seconds, S/m, W/m/K, J/m^3/K, Pa, 1/K).
Spatial arrays are C-ordered with x fastest: ``mat[k, j, i]``.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

# ---------------------------------------------------------------------------
# Material table.  Columns follow the order below; ``void`` = 1 marks a cell
# that carries no stiffness (air).  Cu/Si/solder E and CTE follow the paper's
# materials list (Sec. III-A); the dielectric, thermal and polymer values,
# which the paper does not list, are typical figures for these materials.
# ---------------------------------------------------------------------------
PROP_COLUMNS = ("eps_r", "sigma0", "tcr", "k", "rho_cp", "E", "nu", "cte", "void")
N_PROP = len(PROP_COLUMNS)

AIR, SI, CU, POLYIMIDE, UNDERFILL, BT = 0, 1, 2, 3, 4, 5
MATERIAL_NAMES = ("air", "Si", "Cu", "polyimide", "underfill", "BT")


def package_materials() -> np.ndarray:
    """The six-class material table used by every package workload."""
    t = np.zeros((6, N_PROP), dtype=np.float64)
    #            eps_r  sigma0   tcr     k      rho_cp   E        nu    cte     void
    t[AIR] = [1.0, 0.0, 0.0, 0.026, 1.2e3, 0.0, 0.0, 0.0, 1.0]
    t[SI] = [11.7, 10.0, 0.0, 148.0, 1.64e6, 130e9, 0.28, 2.6e-6, 0.0]
    t[CU] = [1.0, 5.8e7, 3.9e-3, 400.0, 3.45e6, 117e9, 0.34, 17e-6, 0.0]
    t[POLYIMIDE] = [3.5, 0.0, 0.0, 0.3, 1.55e6, 3e9, 0.34, 40e-6, 0.0]
    t[UNDERFILL] = [3.9, 0.0, 0.0, 0.5, 1.6e6, 8e9, 0.30, 30e-6, 0.0]
    t[BT] = [4.2, 0.0, 0.0, 0.4, 1.9e6, 20e9, 0.28, 15e-6, 0.0]
    return t


# Boundary-condition codes (per face, order -x,+x,-y,+y,-z,+z).
PMC, PEC = 0, 1
MECH_KINEMATIC, MECH_CLAMP_ZMIN = 0, 1

# Probe field codes.
PROBE_EX, PROBE_EY, PROBE_EZ, PROBE_THETA = 0, 1, 2, 3


# ---------------------------------------------------------------------------
# Excitation waveforms.  Each returns the waveform value at times t (array);
# the value is zero for t < 0 (the source is causal), and the windowed kinds
# are zero outside [t_on, t_off) (t_on >= 0 for every workload here).
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Wave:
    kind: str                 # "gauss_cos" | "prbs_trap" | "step" | "ramp" | "sine" | "ricker"
                              # windowed closed forms (also evaluated on the device):
                              # "ricker_w" | "sine_w" | "gauss_train"
    amp: float                # A/m^2 for current sources, V for voltage ports
    f0: float = 0.0           # carrier / sine frequency [Hz]
    t0: float = 0.0           # centre / phase reference [s]
    tau: float = 0.0          # Gaussian or Ricker width [s]
    bitrate: float = 0.0      # [bit/s]
    rise: float = 0.0         # [s]
    bits: Optional[np.ndarray] = None  # NRZ levels 0/1 for prbs_trap
    t_on: float = 0.0         # windowed kinds: zero outside [t_on, t_off)
    t_off: float = np.inf
    centers: Optional[np.ndarray] = None  # gauss_train pulse centres [s]

    WINDOWED = ("ricker_w", "sine_w", "gauss_train")

    def device_params(self) -> dict:
        """The wave as the library's closed-form wave record (windowed kinds only)."""
        if self.kind not in self.WINDOWED:
            raise ValueError(f"wave kind {self.kind} has no closed-form device record")
        c = np.zeros(8) if self.centers is None else np.asarray(self.centers, dtype=np.float64)
        return dict(kind={"ricker_w": 1, "sine_w": 2, "gauss_train": 3}[self.kind],
                    n_pulses=int(len(c)) if self.kind == "gauss_train" else 0, amp=self.amp, t0=self.t0,
                    width=self.tau, freq=self.f0, t_on=self.t_on, t_off=self.t_off, pulse_t=c)

    def __call__(self, t: np.ndarray) -> np.ndarray:
        t = np.asarray(t, dtype=np.float64)
        out = np.zeros_like(t)
        if self.kind in self.WINDOWED:
            on = (t >= self.t_on) & (t < self.t_off)
            tw = t[on]
            if self.kind == "ricker_w":
                u = (tw - self.t0) / self.tau
                a = u * u
                out[on] = self.amp * (1.0 - 2.0 * a) * np.exp(-a)
            elif self.kind == "sine_w":
                out[on] = self.amp * np.sin(2.0 * np.pi * self.f0 * (tw - self.t0))
            else:
                env = np.zeros_like(tw)
                for c in self.centers:
                    u = (tw - c) / self.tau
                    env += np.exp(-(u * u))
                out[on] = self.amp * env * np.cos(2.0 * np.pi * self.f0 * (tw - self.t0))
            return out
        pos = t >= 0.0
        tp = t[pos]
        if self.kind == "gauss_cos":
            s = (tp - self.t0) / self.tau
            out[pos] = self.amp * np.exp(-s * s) * np.cos(2.0 * np.pi * self.f0 * (tp - self.t0))
        elif self.kind == "step":
            out[pos] = self.amp
        elif self.kind == "ramp":
            out[pos] = self.amp * np.minimum(tp / self.rise, 1.0)
        elif self.kind == "sine":
            out[pos] = self.amp * np.sin(2.0 * np.pi * self.f0 * tp)
        elif self.kind == "ricker":
            a = (np.pi * self.f0 * (tp - self.t0)) ** 2
            out[pos] = self.amp * (1.0 - 2.0 * a) * np.exp(-a)
        elif self.kind == "prbs_trap":
            out[pos] = self.amp * nrz_trapezoid(tp, self.bits, 1.0 / self.bitrate, self.rise)
        else:
            raise ValueError(f"unknown wave kind {self.kind}")
        return out


def prbs7(state: int, n: int) -> np.ndarray:
    """n bits of the PRBS-7 sequence x^7 + x^6 + 1 from a non-zero 7-bit seed.

    Fibonacci form: the new bit is b6 XOR b5 of the state, shifted in at the
    bottom; the emitted bit is the new bit.  Period 127.
    """
    if not (0 < state < 128):
        raise ValueError("PRBS-7 state must be in 1..127")
    out = np.empty(n, dtype=np.uint8)
    s = int(state)
    for m in range(n):
        b = ((s >> 6) ^ (s >> 5)) & 1
        s = ((s << 1) | b) & 0x7F
        out[m] = b
    return out


def nrz_trapezoid(t: np.ndarray, bits: np.ndarray, ui: float, rise: float) -> np.ndarray:
    """Unipolar NRZ level (0..1): each bit boundary m*ui starts a linear ramp
    of length ``rise`` from the previous level (0 before the first bit) to
    the new one, then holds.  Beyond the last bit the last level holds."""
    t = np.asarray(t, dtype=np.float64)
    m = np.clip(np.floor(t / ui).astype(np.int64), 0, len(bits) - 1)
    lvl = bits.astype(np.float64)
    prev = np.where(m > 0, lvl[np.maximum(m - 1, 0)], 0.0)
    cur = lvl[m]
    frac = np.clip((t - m * ui) / rise, 0.0, 1.0)
    return prev + (cur - prev) * frac


# ---------------------------------------------------------------------------
# Problem description.
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    name: str
    dx: np.ndarray            # (nx,) cell widths [m]
    dy: np.ndarray            # (ny,)
    dz: np.ndarray            # (nz,)
    mat: np.ndarray           # (nz, ny, nx) uint8 material ids
    props: np.ndarray         # (n_mat, N_PROP) float64
    # port edges: dir 0/1/2 = x/y/z edge starting at node (i, j, k)
    port_dir: np.ndarray
    port_i: np.ndarray
    port_j: np.ndarray
    port_k: np.ndarray
    port_wave: np.ndarray
    port_weight: np.ndarray   # J on the edge = weight * wave(t)
    port_g: np.ndarray        # lumped conductance added to sigma on the edge [S/m]
    waves: List[Wave]
    em_bc: tuple = (PMC,) * 6
    mech_bc: int = MECH_KINEMATIC
    T0: float = 300.0
    cfl: float = 0.9
    n_em_steps: int = 100
    em_per_thermal: int = 1
    mech_every_thermal: int = 0   # 0: one mechanical solve at the end
    cg_rtol: float = 1e-8
    probes: Optional[np.ndarray] = None   # (n_probes, 4) int64: field, i, j, k
    history_stride: int = 0
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nx(self) -> int:
        return int(self.dx.shape[0])

    @property
    def ny(self) -> int:
        return int(self.dy.shape[0])

    @property
    def nz(self) -> int:
        return int(self.dz.shape[0])

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_ports(self) -> int:
        return int(self.port_dir.shape[0])

    def sample_J_half(self, dt: float, n_steps: Optional[int] = None) -> np.ndarray:
        """Excitation sampled at half steps: ``out[w, s] = wave_w((s - 1/2) dt)``
        for s = 0..n_steps, so that step n (making e^{n+1}) uses columns n+1
        and n.  Column 0 is at t = -dt/2 and is zero for every causal wave."""
        n = self.n_em_steps if n_steps is None else int(n_steps)
        bind_step_timing(self, dt)
        t = (np.arange(n + 1, dtype=np.float64) - 0.5) * dt
        out = np.zeros((max(len(self.waves), 1), n + 1), dtype=np.float64)
        for w, wave in enumerate(self.waves):
            out[w] = wave(t)
        return out


# ---------------------------------------------------------------------------
# The excitation scheme of Sec. III-B.  Trace ports form differential pairs
# (alternating polarity along y) driven by a Ricker "trigger"; bump arrays
# are fed as Ground-Signal-Ground groups of x-directed current ports, driven
# by a 5 GHz sine under the logic die and by a 40 GHz carrier under a 3-bit
# Gaussian pulse train under the HBM die.  Every port draws its own
# amplitude, width and time shift (deterministic, seeded), so the pairs and
# groups are not exactly balanced.  Quantities the paper does not give are
# readings: the Ricker peak frequency (50 GHz: below 1e-3 of its peak at the
# window edges), the pulse train's slots (three equal slots of the 80-230 ps
# window, pulses at their centres, 1/e half-width 12 ps) and the bump
# current density.
# ---------------------------------------------------------------------------
TRIGGER_T0, TRIGGER_FP, TRIGGER_WINDOW = 40e-12, 50e9, (20e-12, 60e-12)
LOGIC_F, LOGIC_WINDOW = 5e9, (0.0, 300e-12)
BURST_F, BURST_WINDOW, BURST_BITS, BURST_WIDTH = 40e9, (80e-12, 230e-12), 3, 12e-12
JITTER_AMP, JITTER_WIDTH, JITTER_PHASE = 0.20, 0.10, 10e-12
BUMP_J0 = 1.0e10   # A/m^2 on a signal bump


def paper_jitter(rng) -> tuple:
    """(amplitude factor, width factor, time shift [s]) of one port."""
    return (1.0 + rng.uniform(-JITTER_AMP, JITTER_AMP), 1.0 + rng.uniform(-JITTER_WIDTH, JITTER_WIDTH),
            rng.uniform(-JITTER_PHASE, JITTER_PHASE))


def _window(lo, hi, shift, t_origin):
    # clipped at t = 0: every source is off before the simulation starts (a
    # window that ended before the time origin becomes the empty [0, 0))
    return max(lo + shift - t_origin, 0.0), max(hi + shift - t_origin, 0.0)


def trigger_wave(amp, jit, t_origin=0.0) -> Wave:
    fa, fw, sh = jit
    on, off = _window(*TRIGGER_WINDOW, sh, t_origin)
    return Wave("ricker_w", amp=amp * fa, t0=TRIGGER_T0 + sh - t_origin, tau=fw / (np.pi * TRIGGER_FP),
                t_on=on, t_off=off)


def logic_wave(amp, jit, t_origin=0.0) -> Wave:
    fa, _, sh = jit  # a continuous sine has no pulse width to vary
    on, off = _window(*LOGIC_WINDOW, sh, t_origin)
    return Wave("sine_w", amp=amp * fa, f0=LOGIC_F, t0=LOGIC_WINDOW[0] + sh - t_origin, t_on=on, t_off=off)


def burst_wave(amp, jit, t_origin=0.0) -> Wave:
    fa, fw, sh = jit
    on, off = _window(*BURST_WINDOW, sh, t_origin)
    slot = (BURST_WINDOW[1] - BURST_WINDOW[0]) / BURST_BITS
    c = BURST_WINDOW[0] + (np.arange(BURST_BITS) + 0.5) * slot + sh - t_origin
    return Wave("gauss_train", amp=amp * fa, f0=BURST_F, t0=BURST_WINDOW[0] + sh - t_origin,
                tau=BURST_WIDTH * fw, centers=c, t_on=on, t_off=off)


def gsg_role(b: int, n: int) -> float:
    """Weight of bump b of a column of n along y.  Signal bumps sit at odd b
    with a ground bump on both sides (b + 1 < n) and carry +1; every ground
    bump returns -1/2 for each adjacent signal bump, so the unjittered
    weights of a column sum to zero."""
    sig = lambda q: 0 <= q < n and q % 2 == 1 and q + 1 < n
    if sig(b):
        return 1.0
    return -0.5 * (sig(b - 1) + sig(b + 1))


def gsg_bump_ports(cols, rows, kmid, logic_x, rng, t_origin, waves):
    """x-directed current ports (3x3 edges through the bump centre at height
    kmid) on a bump array with centres cols x rows; bumps left of logic_x
    belong to the logic die, the rest to the HBM die.  Appends one wave per
    bump to ``waves``; returns the port tuples."""
    plist = []
    for ci in cols:
        for b, cj in enumerate(rows):
            role = gsg_role(b, len(rows))
            if role == 0.0:
                continue
            wid = len(waves)
            jit = paper_jitter(rng)
            waves.append(logic_wave(BUMP_J0, jit, t_origin) if ci < logic_x else burst_wave(BUMP_J0, jit, t_origin))
            plist += [(d, i, j, k, w, role * wt, g)
                      for d, i, j, k, w, wt, g in current_port(0, ci - 1, cj - 1, kmid - 1, 2, wid)]
    return plist


def _empty_ports():
    z = np.zeros(0)
    return dict(port_dir=z.astype(np.uint8), port_i=z.astype(np.int32), port_j=z.astype(np.int32),
                port_k=z.astype(np.int32), port_wave=z.astype(np.int32),
                port_weight=z.astype(np.float64), port_g=z.astype(np.float64))


def _stack_ports(plist):
    if not plist:
        return _empty_ports()
    a = np.array(plist, dtype=np.float64)
    return dict(port_dir=a[:, 0].astype(np.uint8), port_i=a[:, 1].astype(np.int32),
                port_j=a[:, 2].astype(np.int32), port_k=a[:, 3].astype(np.int32),
                port_wave=a[:, 4].astype(np.int32), port_weight=a[:, 5].copy(),
                port_g=a[:, 6].copy())


def dual_width(d: np.ndarray) -> np.ndarray:
    """Node-centred widths (half cells at the two ends).  Used here only to
    size the lumped port source (current = V / R_s over the port's area)."""
    n = d.shape[0]
    h = np.zeros(n + 1)
    h[:n] += 0.5 * d
    h[1:] += 0.5 * d
    return h


def voltage_port(dirn, i0, j0, k0, w, wave_id, dx, dy, dz, rs=50.0):
    """Norton form of a voltage source with series resistance ``rs`` across a
    one-cell gap: the (w+1)^2 edges of direction ``dirn`` starting at node
    (i0, j0, k0) carry J = V(t) / (rs * A) and a lumped conductance
    g = L / (rs * A), where A is the port's total cross-section (the sum of
    the edges' node-centred areas) and L the gap length."""
    hx, hy, hz = dual_width(dx), dual_width(dy), dual_width(dz)
    edges = []
    if dirn == 0:
        for k in range(k0, k0 + w + 1):
            for j in range(j0, j0 + w + 1):
                edges.append((j, k, hy[j] * hz[k]))
        L = dx[i0]
        area = sum(e[2] for e in edges)
        return [(0, i0, j, k, wave_id, 1.0 / (rs * area), L / (rs * area)) for j, k, _ in edges]
    if dirn == 1:
        for k in range(k0, k0 + w + 1):
            for i in range(i0, i0 + w + 1):
                edges.append((i, k, hx[i] * hz[k]))
        L = dy[j0]
        area = sum(e[2] for e in edges)
        return [(1, i, j0, k, wave_id, 1.0 / (rs * area), L / (rs * area)) for i, k, _ in edges]
    raise ValueError("voltage ports are x- or y-directed")


def current_port(dirn, i0, j0, k0, w, wave_id):
    """A current-density source (A/m^2 set by the wave) on the (w+1)^2 edges of
    direction ``dirn`` starting at node (i0, j0, k0); no lumped conductance."""
    out = []
    if dirn == 0:
        for k in range(k0, k0 + w + 1):
            for j in range(j0, j0 + w + 1):
                out.append((0, i0, j, k, wave_id, 1.0, 0.0))
    elif dirn == 1:
        for k in range(k0, k0 + w + 1):
            for i in range(i0, i0 + w + 1):
                out.append((1, i, j0, k, wave_id, 1.0, 0.0))
    else:
        for j in range(j0, j0 + w + 1):
            for i in range(i0, i0 + w + 1):
                out.append((2, i, j, k0, wave_id, 1.0, 0.0))
    return out


# ---------------------------------------------------------------------------
# Workload 1: 32x32x16 uniform 1 um voxels, PEC box, one Cu trace.
# ---------------------------------------------------------------------------
def config1(dt_hint: float = 1.7332e-15) -> Problem:
    """32x32x16, 1 um: Si (k 0-3) / polyimide (k 4-11) with one 2x2 Cu trace
    along x (j 15-16, k 7-8, i 2-29, polyimide gap cell at i = 3) / air
    (k 12-15); all faces PEC; bottom face clamped; a Gaussian-modulated
    10 GHz current source on the 9 x-edges spanning the gap; 2000 EM steps at
    CFL 0.9; Joule heat averaged into 10 thermal steps (R = 200); one PCG at
    the end, rtol 1e-8.

    The window (2000 steps, about 3.5 ps) is a small fraction of a 10 GHz
    period, so the Gaussian envelope is placed relative to the window:
    t0 = T/2, tau = T/6 with T = 2000 * dt_hint.
    """
    nx, ny, nz = 32, 32, 16
    um = 1e-6
    mat = np.empty((nz, ny, nx), dtype=np.uint8)
    mat[0:4] = SI
    mat[4:12] = POLYIMIDE
    mat[12:16] = AIR
    mat[7:9, 15:17, 2:30] = CU
    mat[7:9, 15:17, 3] = POLYIMIDE
    T = 2000 * dt_hint
    waves = [Wave("gauss_cos", amp=1e10, f0=10e9, t0=T / 2, tau=T / 6)]
    ports = _stack_ports(current_port(0, 3, 15, 7, 2, 0))
    probes = np.array([[PROBE_EX, 3, 16, 8], [PROBE_EX, 10, 16, 8], [PROBE_THETA, 10, 16, 8],
                       [PROBE_EZ, 16, 16, 10]], dtype=np.int64)
    return Problem(name="pkg32x32x16_pec_trace", dx=np.full(nx, um), dy=np.full(ny, um),
                   dz=np.full(nz, um), mat=mat, props=package_materials(), waves=waves,
                   em_bc=(PEC,) * 6, mech_bc=MECH_CLAMP_ZMIN, n_em_steps=2000,
                   em_per_thermal=200, mech_every_thermal=0, cg_rtol=1e-8, probes=probes,
                   history_stride=100, **ports)


# ---------------------------------------------------------------------------
# Workload 2: 256x256x64 graded package slice.
# ---------------------------------------------------------------------------
def graded_widths(n: int, dmin: float = 1e-6, extra: float = 4e-6) -> np.ndarray:
    i = np.arange(n, dtype=np.float64)
    u = np.abs(2.0 * (i + 0.5) / n - 1.0)
    return dmin + extra * u * u


def config2(seed: int = 2001, excitation: str = "prbs", t_origin: float = 0.0) -> Problem:
    """256x256x64 package slice on a graded rectilinear grid.

    x/y widths 1 + 4u^2 um with u = |2(i+1/2)/N - 1| (1 um in the middle,
    5 um at the rim).  Layers bottom to top (cells, dz):
      Cu ground plane (2, 1 um) / BT substrate with 16 Cu traces along x
      (12, 2 um) / underfill with an 8x8 Cu microbump array (8, 1.5 um) /
      Si interposer with a seeded TSV grid (24, 2 um) / two Si dies with an
      air gap (14, 2 um) / air (4, 2 um).
    TSVs: physical pitch ~ U[20, 40] um, each site present with p = 0.5,
    2x2 cells of Cu through the interposer.  Each trace is driven across a
    one-cell BT gap by a 1 V PRBS-7 trapezoidal burst (5 Gb/s, 20 ps rise)
    through 50 ohm.  PMC on all faces; kinematic mount.  20,000 EM steps,
    R = 200 (100 thermal steps), a PCG solve after every thermal step.

    excitation="paper": the scheme of Sec. III-B instead (closed-form waves,
    one per port, times measured from t_origin): the trace ports become
    differential pairs driven by the Ricker trigger (+-1 V alternating along
    y) and the bumps Ground-Signal-Ground groups under the two dies.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    N, nz = 256, 64
    dx = graded_widths(N)
    dy = graded_widths(N)
    layers = [(CU, 2, 1.0e-6), (BT, 12, 2.0e-6), (UNDERFILL, 8, 1.5e-6), (SI, 24, 2.0e-6),
              (SI, 14, 2.0e-6), (AIR, 4, 2.0e-6)]
    dz = np.concatenate([np.full(n, d) for _, n, d in layers])
    assert dz.shape[0] == nz
    mat = np.empty((nz, N, N), dtype=np.uint8)
    k = 0
    bounds = []
    for m, n, _ in layers:
        mat[k:k + n] = m
        bounds.append((k, k + n))
        k += n
    # 16 traces in the BT layer, 2x2 cells, along x, with a port gap at i = 10.
    kt = bounds[1][0] + 5
    plist, waves = [], []
    for t in range(16):
        j0 = int(round((t + 0.5) * N / 16)) - 1
        mat[kt:kt + 2, j0:j0 + 2, 8:N - 8] = CU
        mat[kt:kt + 2, j0:j0 + 2, 10] = BT
        bits = prbs7(int(rng.integers(1, 128)), 8)
        waves.append(Wave("prbs_trap", amp=1.0, bitrate=5e9, rise=20e-12, bits=bits))
        plist += voltage_port(0, 10, j0, kt, 2, t, dx, dy, dz)
    if excitation == "paper":
        xrng = np.random.Generator(np.random.PCG64(seed + 7919))
        waves = [trigger_wave(1.0 if t % 2 == 0 else -1.0, paper_jitter(xrng), t_origin) for t in range(16)]
    # 8x8 microbumps, 6x6 cells each, through the underfill layer.
    k0, k1 = bounds[2]
    for bj in range(8):
        cj = int(round((bj + 0.5) * N / 8))
        for bi in range(8):
            ci = int(round((bi + 0.5) * N / 8))
            mat[k0:k1, cj - 3:cj + 3, ci - 3:ci + 3] = CU
    if excitation == "paper":
        bumps = [int(round((b + 0.5) * N / 8)) for b in range(8)]
        plist += gsg_bump_ports(bumps, bumps, (k0 + k1) // 2, N // 2, xrng, t_origin, waves)
    # TSV grid in the interposer.
    k0, k1 = bounds[3]
    xn = np.concatenate([[0.0], np.cumsum(dx)])
    pitch = float(rng.uniform(20e-6, 40e-6))
    sites = np.arange(pitch / 2, xn[-1] - pitch / 4, pitch)
    idx = np.clip(np.searchsorted(xn, sites) - 1, 0, N - 2)
    present = rng.random((idx.size, idx.size)) < 0.5
    for a, jj in enumerate(idx):
        for b, ii in enumerate(idx):
            if present[a, b]:
                mat[k0:k1, jj:jj + 2, ii:ii + 2] = CU
    # Two dies with an air gap.
    k0, k1 = bounds[4]
    g0, g1 = int(0.47 * N), int(0.53 * N)
    mat[k0:k1, :, g0:g1] = AIR
    probes = np.array([[PROBE_EX, 10, int(round(0.5 * N / 16)), kt],
                       [PROBE_EX, 64, int(round(0.5 * N / 16)), kt],
                       [PROBE_THETA, 64, int(round(0.5 * N / 16)), kt]], dtype=np.int64)
    if excitation not in ("prbs", "paper"):
        raise ValueError(f"unknown excitation {excitation}")
    return Problem(name="slice256x256x64_graded" + ("_paperexc" if excitation == "paper" else ""), dx=dx, dy=dy, dz=dz, mat=mat,
                   props=package_materials(), waves=waves, em_bc=(PMC,) * 6,
                   mech_bc=MECH_KINEMATIC, n_em_steps=20000, em_per_thermal=200,
                   mech_every_thermal=1, cg_rtol=1e-8, probes=probes, history_stride=1000,
                   meta=dict(tsv_pitch=pitch), **_stack_ports(plist))


# ---------------------------------------------------------------------------
# Workloads 3-5: uniform 1 um package recipe at arbitrary size.
# ---------------------------------------------------------------------------
def package(nx: int, ny: int, nz: int, seed: int, *, bump_pitch_um: float = 16.0,
            bump_cells: int = 8, trace_width: int = 1, trace_pitch: int = 2,
            n_trace_layers: int = 8, max_traces: Optional[int] = None, n_bits: int = 256,
            steps_per_bit: int = 16, em_per_thermal: int = 256, name: str = "package",
            excitation: str = "prbs", t_origin: float = 0.0) -> Problem:
    """Uniform 1 um package voxelisation, layer thicknesses scaled from the
    128-cell stack: Cu ground (2) / BT (30) / Cu bumps in underfill (16) /
    Si interposer with TSVs under the bumps (32) / polyimide RDL with
    ``n_trace_layers`` routing layers of traces alternating x/y (32) / two Si
    dies with an air gap (12) / air (4).  Every trace is driven across a
    one-cell gap near its start by its own seeded PRBS-7 burst (1 V through
    50 ohm, rise = a quarter bit).

    excitation="paper": the scheme of Sec. III-B instead (closed-form waves,
    one per port, times measured from t_origin): the traces become
    differential pairs driven by the Ricker trigger (+-1 V alternating in
    trace order) and every bump column a Ground-Signal-Ground line, under
    the logic die (left half) or the HBM die (right half)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    um = 1e-6
    dx, dy, dz = np.full(nx, um), np.full(ny, um), np.full(nz, um)
    base = [(CU, 2), (BT, 30), (UNDERFILL, 16), (SI, 32), (POLYIMIDE, 32), (SI, 12), (AIR, 4)]
    scale = nz / 128.0
    th = [max(1, int(round(n * scale))) for _, n in base]
    th[-1] += nz - sum(th)
    if th[-1] < 1:
        th[4] += th[-1] - 1
        th[-1] = 1
    mat = np.empty((nz, ny, nx), dtype=np.uint8)
    k, bounds = 0, []
    for (m, _), n in zip(base, th):
        mat[k:k + n] = m
        bounds.append((k, k + n))
        k += n
    # bumps + TSVs under them
    p = max(int(round(bump_pitch_um)), bump_cells + 2)
    bc = min(bump_cells, p - 2)
    k0, k1 = bounds[2]
    t0, t1 = bounds[3]
    for cj in range(p // 2, ny - bc // 2, p):
        for ci in range(p // 2, nx - bc // 2, p):
            j0, i0 = cj - bc // 2, ci - bc // 2
            mat[k0:k1, j0:j0 + bc, i0:i0 + bc] = CU
            mat[t0:t1, cj - 1:cj + 1, ci - 1:ci + 1] = CU
    # RDL traces
    r0, r1 = bounds[4]
    lay_th = max(1, (r1 - r0) // max(n_trace_layers, 1))
    plist, waves = [], []
    w = trace_width
    for r in range(n_trace_layers):
        kk = r0 + r * lay_th + (lay_th - 1) // 2
        if kk + w > r1:
            break
        along_x = (r % 2 == 0)
        span = ny if along_x else nx
        pitch = max(trace_pitch, w + 1)
        starts = list(range(1, span - w - 1, pitch))
        for s in starts:
            if max_traces is not None and len(waves) >= max_traces:
                break
            wid = len(waves)
            bits = prbs7(int(rng.integers(1, 128)), n_bits)
            # bit period given in EM steps; bind_step_timing() converts it
            waves.append(Wave("prbs_trap", amp=1.0, bitrate=0.0, rise=0.0, bits=bits))
            if along_x:
                mat[kk:kk + w, s:s + w, 2:nx - 2] = CU
                mat[kk:kk + w, s:s + w, 4] = POLYIMIDE
                plist += voltage_port(0, 4, s, kk, w, wid, dx, dy, dz)
            else:
                mat[kk:kk + w, 2:ny - 2, s:s + w] = CU
                mat[kk:kk + w, 4, s:s + w] = POLYIMIDE
                plist += voltage_port(1, s, 4, kk, w, wid, dx, dy, dz)
    if excitation == "paper":
        xrng = np.random.Generator(np.random.PCG64(seed + 7919))
        waves = [trigger_wave(1.0 if t % 2 == 0 else -1.0, paper_jitter(xrng), t_origin) for t in range(len(waves))]
        cols = list(range(p // 2, nx - bc // 2, p))
        rows = list(range(p // 2, ny - bc // 2, p))
        plist += gsg_bump_ports(cols, rows, (k0 + k1) // 2, nx // 2, xrng, t_origin, waves)
    elif excitation != "prbs":
        raise ValueError(f"unknown excitation {excitation}")
    # dies with a gap
    d0, d1 = bounds[5]
    g0, g1 = int(0.48 * nx), int(0.52 * nx)
    if g1 > g0:
        mat[d0:d1, :, g0:g1] = AIR
    n_steps = n_bits * steps_per_bit
    n_steps -= n_steps % em_per_thermal if n_steps >= em_per_thermal else 0
    pr = np.array([[PROBE_THETA, nx // 2, ny // 2, (r0 + r1) // 2]], dtype=np.int64)
    prob = Problem(name=name, dx=dx, dy=dy, dz=dz, mat=mat, props=package_materials(),
                   waves=waves, em_bc=(PMC,) * 6, mech_bc=MECH_KINEMATIC,
                   n_em_steps=max(n_steps, em_per_thermal), em_per_thermal=em_per_thermal,
                   mech_every_thermal=0, cg_rtol=1e-8, probes=pr, history_stride=256,
                   meta=dict(steps_per_bit=steps_per_bit), **_stack_ports(plist))
    return prob


def bind_step_timing(p: Problem, dt: float) -> Problem:
    """Workloads whose bit period is given in EM steps get their physical bit
    rate and rise (a quarter bit) once the time step is known."""
    spb = p.meta.get("steps_per_bit")
    if spb:
        for wv in p.waves:
            if wv.kind == "prbs_trap" and wv.bitrate == 0.0:
                ui = spb * dt
                wv.bitrate = 1.0 / ui
                wv.rise = 0.25 * ui
    return p


def config3(seed: int = 3001, excitation: str = "prbs", t_origin: float = 0.0) -> Problem:
    """1024x1024x128 full-scale one-GPU package: 6 material classes, 64x64
    bumps of 8x8 cells at 16-cell pitch, 8 RDL routing layers x 512 traces
    (width 1, pitch 2, alternating x/y) = 4096 traces, each with a 256-bit
    PRBS-7 burst at 16 steps per bit (4096 EM steps), R = 256.
    excitation="paper": the Sec. III-B scheme on the same geometry."""
    return package(1024, 1024, 128, seed, bump_pitch_um=16, bump_cells=8, trace_width=1,
                   trace_pitch=2, n_trace_layers=8, n_bits=256, steps_per_bit=16,
                   em_per_thermal=256, name="package1024x1024x128" + ("_paperexc" if excitation == "paper" else ""),
                   excitation=excitation, t_origin=t_origin)


def config4_variant(v: int) -> Problem:
    """Design variant v of the 64-variant batch: Nx, Ny ~ U{64..192},
    Nz ~ U{32..48}, bump pitch ~ U[20, 50] um, trace width ~ U[2, 8] um,
    128-bit PRBS-7 per trace at 16 steps per bit, R = 256."""
    rng = np.random.Generator(np.random.PCG64(4000 + v))
    nx, ny = int(rng.integers(64, 193)), int(rng.integers(64, 193))
    nz = int(rng.integers(32, 49))
    pitch = float(rng.uniform(20, 50))
    w = int(rng.integers(2, 9))
    return package(nx, ny, nz, 4000 + v, bump_pitch_um=pitch, bump_cells=max(2, int(pitch) // 2),
                   trace_width=w, trace_pitch=2 * w, n_trace_layers=4, max_traces=64,
                   n_bits=128, steps_per_bit=16, em_per_thermal=256,
                   name=f"variant{v}_{nx}x{ny}x{nz}")


def config5_request(r: int) -> Problem:
    """Serving request r: s ~ U[0, 1], Nx = Ny = round(32 * 16^s),
    Nz = round(32 * 2^s) (cells log-uniform from 32^3 to 512x512x64), burst
    length ~ U{64..1024} bits at 4 steps per bit, R = 256."""
    rng = np.random.Generator(np.random.PCG64(5000 + r))
    s = float(rng.random())
    n = int(round(32 * 16 ** s))
    nz = int(round(32 * 2 ** s))
    bits = int(rng.integers(64, 1025))
    pitch = float(rng.uniform(20, 50))
    w = int(rng.integers(2, 9))
    return package(n, n, nz, 5000 + r, bump_pitch_um=pitch, bump_cells=max(2, int(pitch) // 2),
                   trace_width=w, trace_pitch=2 * w, n_trace_layers=4, max_traces=32,
                   n_bits=bits, steps_per_bit=4, em_per_thermal=256,
                   name=f"request{r}_{n}x{n}x{nz}")


def poisson_arrivals(rate: float, n: int, seed: int = 5999) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


# ---------------------------------------------------------------------------
# Small random problems for parity tests.
# ---------------------------------------------------------------------------
def random_problem(seed: int, nx: int, ny: int, nz: int, *, n_mat: int = 4, graded: bool = True,
                   em_bc=None, mech_bc: int = MECH_KINEMATIC, n_steps: int = 40, R: int = 4,
                   n_ports: int = 2, void_top: int = 1, amp: float = 1e9) -> Problem:
    """A heterogeneous random problem: random spacings (0.5-2 um), random
    materials (the last ``void_top`` layers are air), random port edges with
    Gaussian-modulated sources, some with lumped conductance."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if graded:
        dx = rng.uniform(0.5e-6, 2e-6, nx)
        dy = rng.uniform(0.5e-6, 2e-6, ny)
        dz = rng.uniform(0.5e-6, 2e-6, nz)
    else:
        dx, dy, dz = np.full(nx, 1e-6), np.full(ny, 1e-6), np.full(nz, 1e-6)
    props = np.zeros((n_mat + 1, N_PROP))
    props[0] = [1.0, 0.0, 0.0, 0.026, 1.2e3, 0.0, 0.0, 0.0, 1.0]
    for m in range(1, n_mat + 1):
        cond = rng.random() < 0.5
        props[m] = [rng.uniform(1, 12), rng.uniform(1e5, 6e7) if cond else rng.uniform(0, 20),
                    rng.uniform(0, 5e-3) if cond else 0.0, rng.uniform(0.2, 400),
                    rng.uniform(1e6, 4e6), rng.uniform(3e9, 150e9), rng.uniform(0.2, 0.4),
                    rng.uniform(2e-6, 40e-6), 0.0]
    mat = rng.integers(1, n_mat + 1, size=(nz, ny, nx)).astype(np.uint8)
    if void_top > 0:
        mat[nz - void_top:] = 0
    waves, plist = [], []
    T = n_steps * 1.5e-15
    if em_bc is None:
        em_bc = tuple(int(b) for b in rng.integers(0, 2, 6))

    def pick(n, along, lo_pec, hi_pec):
        if along:
            return int(rng.integers(0, n))
        cand = [v for v in range(n + 1) if not ((v == 0 and lo_pec) or (v == n and hi_pec))]
        return int(cand[rng.integers(0, len(cand))])

    for p in range(n_ports):
        waves.append(Wave("gauss_cos", amp=amp * rng.uniform(0.5, 2.0), f0=rng.uniform(5e9, 50e9),
                          t0=T * rng.uniform(0.2, 0.6), tau=T * rng.uniform(0.1, 0.3)))
        d = int(rng.integers(0, 3))
        i = pick(nx, d == 0, em_bc[0], em_bc[1])
        j = pick(ny, d == 1, em_bc[2], em_bc[3])
        k = pick(nz, d == 2, em_bc[4], em_bc[5])
        g = float(rng.uniform(0, 1e3)) if rng.random() < 0.5 else 0.0
        plist.append((d, i, j, k, p, float(rng.uniform(0.5, 1.5)), g))
    probes = np.array([[PROBE_EX, 0, 0, 0], [PROBE_THETA, nx // 2, ny // 2, nz // 2]], dtype=np.int64)
    return Problem(name=f"random{seed}_{nx}x{ny}x{nz}", dx=dx, dy=dy, dz=dz, mat=mat, props=props,
                   waves=waves, em_bc=tuple(em_bc), mech_bc=mech_bc, n_em_steps=n_steps,
                   em_per_thermal=R, mech_every_thermal=0, cg_rtol=1e-10, probes=probes,
                   history_stride=max(1, n_steps // 4), **_stack_ports(plist))
