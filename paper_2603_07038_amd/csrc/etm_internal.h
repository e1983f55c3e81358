// Private declarations shared by the host plan and the gfx950 kernels.
//
// Device layout: every per-node, per-edge and per-cell array uses one padded
// node-shaped index  n = k*sz + j*sy + i  (x fastest, row pitch sy a multiple
// of 16 elements, plane pitch sz = sy*(ny+1)).  The x-edge, y-edge and
// z-edge starting at node (i,j,k) and the cell whose low corner is node
// (i,j,k) all live at index n of their own arrays; entries that do not exist
// (i == nx for an x-edge, ...) are kept at zero and never updated.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "etm.h"

namespace etm {

constexpr double kEps0 = 8.8541878128e-12;
constexpr double kMu0 = 1.25663706212e-6;
constexpr double kC0 = 299792458.0;
constexpr int kPad = 16;        // row pitch multiple (elements)
constexpr int kMatStride = 16;  // doubles per material row on the device

// Device material row (scaled for the EM update at the plan's dt).
enum MatCol {
  MC_EPSR = 0,    // relative permittivity
  MC_SIGS = 1,    // sigma0 * dt / (2 eps0): the a-coefficient of Eq. (3) per unit eps0
  MC_TCR = 2,     // temperature coefficient of resistance (Eq. 6)
  MC_K = 3,       // thermal conductivity
  MC_RHOCP = 4,   // volumetric heat capacity
  MC_LAMBDA = 5,  // Lame lambda
  MC_MU = 6,      // Lame mu
  MC_BETA = 7,    // (3 lambda + 2 mu) * cte: thermal stress per unit rise
  MC_CTE = 8,
  MC_VOID = 9,    // 1 for a cell without stiffness
};

// Grid description passed by value to every kernel.
struct DevGrid {
  int nx, ny, nz;
  int n_mat;
  int64_t sy, sz, ntot;  // row pitch, plane pitch, padded node count
  const double *dx, *dy, *dz;     // cell widths
  const double *idx, *idy, *idz;  // 1 / width
  const double *hx, *hy, *hz;     // node-centred widths (half cells at the ends)
  const double *ihx, *ihy, *ihz;  // 1 / node-centred width
  const double *al[3], *ah[3];    // per axis: alpha_lo, alpha_hi on nodes (dual-width shares)
  const double *geo;              // base of all 1D tables (dx, dy, dz, idx, ..., ihz, axl, axh, ..., azh)
  uint32_t cs;                    // element stride between the x, y, z components of a field (march kernel)
  const uint8_t *mat;             // cell material ids
  const uint8_t *flags;           // per node: bit d = the d-edge from this node is a port edge
  const double *mtab;             // n_mat rows of kMatStride
  int pec;                        // bit f = face f (-x,+x,-y,+y,-z,+z) is PEC
  int layout;                     // mixed march waves: kLayoutAuto (by row length), kLayoutRuns, kLayoutRows
};
// Work layouts of the mixed-precision march: a wave takes a run of 62
// consecutive nodes of the plane numbered x fastest, or a 62-node segment of
// one row (4 rows per block); automatic picks runs for rows shorter than 512
// nodes.  Results are bitwise the same in every layout.
enum { kLayoutAuto = 0, kLayoutRuns = 1, kLayoutRows = 2 };

// A closed-form wave as stored on the device: kind, n_pulses, amp, t0,
// width, freq, t_on, t_off, pulse centres.  The waves are sampled on the
// device in blocks of kWaveBlock steps, into a table of samples
// s = base .. base + kWaveBlock (J at (s - 1/2) dt) that the march kernels
// read like a tabulated wave; the march kernels themselves carry no
// transcendental code.
constexpr int kWaveStride = 16;
constexpr int kWaveBlock = 1024;

// Port edges, sorted by key = dir * ntot + node.  Entry p has lumped
// conductance gs[p] (scaled like MC_SIGS) and source terms
// [start[p], start[p+1]) of (wave, weight * dt / eps0).
struct DevPorts {
  int n_edges;
  const int64_t *key;
  const double *gs;
  const int32_t *start;
  const int32_t *wave;
  const double *wt;
  const double *J;    // [n_table][n_samples]
  int64_t n_samples;
  const double *Ja;   // closed-form wave n_table + a, sample s: Ja[a * (kWaveBlock + 1) + s - a_base]
  int64_t a_base;
  int n_table;        // tabulated waves
  double *er;         // eps_r of each port edge (written by the coefficient kernel)
};

// Scalars kept on the device.  A plan holds three sets: the march's (Joule
// energy, max temperature, watchdog status, records), the inner CG's (rz,
// alpha, beta, done, iters, tol2, budget) and the mechanical solve's control
// block (fnorm2, tol2 = the FP64 target, rr = the true residual, done = the
// solve's state, iters = inner iterations of all passes, outer = FP64
// residual evaluations, pass_iters).  Every kernel of a solve that is gated
// by a set returns at once while its `done` is nonzero.
constexpr int kMaxPasses = 16;
struct DevScalars {
  double ejoule;      // dissipated energy of completed thermal blocks [J]
  double theta_max;
  int32_t status;     // first asynchronous error
  int32_t pad0;
  int64_t n_records;
  // CG
  double rz, pw, alpha, beta, rr, tol2;
  int32_t done, iters;
  double fnorm2;
  // solve control: outer passes, iteration limit, inner budget
  int32_t outer, maxit, budget, mixed;
  double inner_rtol2;
  int32_t pass_iters[kMaxPasses];
  int32_t restart;    // inner CG: a new inner solve is due (set by the FP64 check, taken by the setup)
  int32_t pad2;
};
// States of a solve's control block (its `done`).
enum { kSolveRunning = 0, kSolveConverged = 1, kSolveGaveUp = 3 };

// Reduction partials: per block, up to 4 doubles.
constexpr int kRedWidth = 4;
// Per-node flag bits besides the port bits (1 << d for a port on own edge d):
// a cell around the node conducts (sigma0 != 0), so an edge incident to the
// node may carry a loss term and Joule heat; such a cell's conductivity also
// depends on temperature (tcr != 0), so the mixed path's K may be nonzero.
// Without them every incident edge has a = 0 and K = 0, which the march
// takes without reading them.
constexpr uint8_t kFlagSigma = 8, kFlagTcr = 16;
// Rows after a kernel's own partials that a two-stage reduction uses for its
// first stage.
constexpr int64_t kFinalizeRows = 512;

// ---- launchers (kernels in em.hip, mech.hip) ------------------------------
struct EmLaunch {
  DevGrid g;
  DevPorts ports;
  int precision;          // ETM_PREC_FP64 / ETM_PREC_MIXED
  int acc_joule;          // add the Joule power of the input field e^n to psum
  int kchunk;             // z planes per block (0 = automatic)
  int pad0;
  double c2dt2;           // (c0 dt)^2
  double cdt;             // c0 dt (leapfrog form)
  double jf;              // eps0 / dt: Joule factor on e^2 * L * sigma_s-area sums
  int64_t step;           // n of the step being made (e^{n} -> e^{n+1})
  // FP64: e0 = e^n, e1 = e^{n-1}, out = e^{n+1}
  // MIXED: e0 = e^n (float), e1 = h^{n-1/2} (faces), out0 / out1 = e^{n+1}, h^{n+1/2}
  const void *e0[3];
  const void *e1[3];
  void *out0[3];
  void *out1[3];
  const double *theta;    // FP64 rise (FP64 path)
  const float *theta32;   // FP32 copy (mixed path)
  double *psum;
  const void *coef;       // per node, 6 components at stride cs (see launch_coef)
  const float *K;         // MIXED: per-edge correction for sigma changes (null when sigma never changes)
  int8_t *elo;            // MIXED: 8-bit residual of e below its FP32 value (updated in place)
};
hipError_t launch_em_step(const EmLaunch &L, hipStream_t s);
// Steps n and n + 1 as a wavefront over z-slabs (La: step n, Lb: step n + 1).
hipError_t launch_em_pair_schedule(const EmLaunch &La, const EmLaunch &Lb, int n_slabs, hipStream_t s);
// Samples s = base .. base + kWaveBlock of n closed-form waves (records of
// kWaveStride doubles at aw) into Ja[w * (kWaveBlock + 1) + s - base].
hipError_t launch_wave_sample(const double *aw, int n, double dt, int64_t base, double *Ja, hipStream_t s);
// Refresh the per-node coefficients of the own x, y, z edges for the current
// temperature (FP64 arithmetic, rounded once to the field precision):
//   FP64:  [eps_r x, y, z, a x, y, z]
//   mixed: [eps_r x, y, z, 2a x, y, z]
// with a = dt sigma(T) / (2 eps0) of the materials (port conductances are
// added in the march); also the eps_r of every port edge.
// Mixed path: with K set, also K += (a_new - a_old) (e_cur + e_prev) on every
// edge whose a changes (e_cur = e^n, e_prev = e^{n-1}; components at stride cs).
struct CoefK {
  float *K = nullptr;
  const float *e_cur = nullptr, *e_prev = nullptr;
  int tcr_only = 0;  // a refresh after a temperature change: only nodes with kFlagTcr can change
};
hipError_t launch_coef(const DevGrid &g, const DevPorts &P, int precision, const void *theta, void *coef, CoefK ck,
                       hipStream_t s);
// Tile counts of the march kernels (x segments, y rows of blocks, z chunks)
// and the default z-chunk, per precision.
void em_tiles(const DevGrid &g, int precision, int kchunk, int *ntx, int *nty, int *nkc);
int em_kchunk(const DevGrid &g, int precision);

// One variant of a batch: its grid, constants and state buffers; the step
// offset within the advance call is read from a device counter.
struct BatchVar {
  EmLaunch L;             // grid, ports, constants and psum (field pointers unused)
  const void *e[3][3];    // FP64: three rotating e buffers; MIXED: sets 0..1
  const void *h[2][3];    // MIXED: face-field sets
  const double *theta[2];
  const float *theta32;
  int64_t step0;          // plan step at the start of the advance call
  int cur0, th0, R, kchunk, acc_joule0, pad1;
};
hipError_t launch_em_batched(const BatchVar *vars, const int4 *items, int n_items, const int64_t *step_ctr,
                             int precision, hipStream_t s);
hipError_t launch_step_ctr(int64_t *ctr, int64_t v, int set, hipStream_t s);

struct ThermalLaunch {
  DevGrid g;
  const void *coef;       // edge coefficients (for the pending Joule power)
  int precision;
  int acc_joule;          // add the pending Joule power of the current field first
  double dt;              // EM step
  double jf;
  int R;                  // EM steps in the block
  const void *e[3];       // current field (for the pending Joule power)
  const double *theta_in;
  double *theta_out;
  float *theta32;         // refreshed copy (mixed path; also its sigma(T) input)
  double *psum;           // zeroed
  double *partials;       // per block: [energy, max]
  DevScalars *sc;
};
hipError_t launch_thermal(const ThermalLaunch &L, hipStream_t s);
hipError_t launch_joule_flush(const DevGrid &g, int precision, const void *const *e, const void *coef, double *psum,
                              double jf, hipStream_t s);

struct DiagLaunch {
  DevGrid g;
  int precision;
  double c2dt2, dt;
  const void *e_new[3];   // e^{n+1}
  const void *e_old[3];   // e^n
  const double *theta;
  const double *psum;
  double *partials;
  DevScalars *sc;
  double *hist_row;       // row to write
  int n_probes;
  const int64_t *probes;  // device: [field, node index] pairs
  int64_t step;
  int64_t cap, rec;
};
hipError_t launch_diag(const DiagLaunch &L, hipStream_t s);

hipError_t launch_pack(const void *src, int src_f32, int64_t sy, int64_t sz, int ni, int nj, int nk,
                       double *dst, hipStream_t s);
hipError_t launch_unpack(const double *src, int ni, int nj, int nk, void *dst, int dst_f32, int64_t sy,
                         int64_t sz, hipStream_t s);
hipError_t launch_fill(void *dst, int64_t n_bytes, hipStream_t s);

// Mechanics.
struct MechGrid {
  DevGrid g;
  const uint8_t *fixed;   // per node: bit c = DOF c fixed
};
hipError_t launch_mech_diag(const MechGrid &M, double *dinv[3], hipStream_t s);
hipError_t launch_mech_rhs(const MechGrid &M, const double *theta, double *f[3], double *partials,
                           DevScalars *sc, double rtol, hipStream_t s);
// Start of a solve, after launch_mech_rhs wrote ctl->fnorm2 and ctl->tol2:
// reset the control block (maxit, inner relative tolerance of the mixed
// path's corrections) and the inner scalars; a zero load gives u = 0 and a
// converged solve at once.
hipError_t launch_solve_init(DevScalars *ctl, DevScalars *scm, int maxit, double inner_rtol2, int mixed,
                             double *u[3], int64_t n, hipStream_t s);
// The solve's FP64 check: r64 = f - K u64 and |r|^2 (skipped once the solve
// is done), then on the device: book the inner iterations of the pass that
// just ended, stop when |r| <= rtol |f| (converged) or when the iteration
// limit is reached or a pass made no progress (gave up), else set the next
// pass's inner tolerance and budget.
hipError_t launch_residual_check(const MechGrid &M, const double *f[3], const double *u[3], double *r[3],
                                 double *partials, DevScalars *ctl, DevScalars *scm, const DevScalars *gate,
                                 hipStream_t s);
// Gate words of a solve's two phases (their `done` = skip): gR for the
// restart of the inner CG (skip unless the solve runs and a restart is due),
// gF for the FP64 check and the refinement update (skip unless the solve
// runs and the inner CG has finished).
hipError_t launch_solve_gates(const DevScalars *ctl, const DevScalars *scm, DevScalars *gR, DevScalars *gF,
                              hipStream_t s);
// CG building blocks (T = double or float vectors; scalars in double).  The
// setups take the solve's control block as a gate: once the solve is done
// they mark the inner CG done, so a whole enqueued pass becomes a no-op.
template <typename T>
struct CgVecs {
  T *u[3], *r[3], *p[3], *w[3];
  const T *dinv[3];
};
template <typename T>
hipError_t launch_cg_setup(const MechGrid &M, const CgVecs<T> &v, const T *rhs[3], double *partials,
                           DevScalars *sc, const DevScalars *gate, hipStream_t s);
template <typename T>
hipError_t launch_cg_iteration(const MechGrid &M, const CgVecs<T> &v, double *partials, DevScalars *sc,
                               hipStream_t s);
// FP64 true residual r64 = f - K u64, its norm into sc (rr), for refinement.
hipError_t launch_residual64(const MechGrid &M, const double *f[3], const double *u[3], double *r[3],
                             double *partials, DevScalars *sc, hipStream_t s);
// Vector helpers of the refinement; gate (may be null) as above.
hipError_t launch_vec_cast(const void *src, int src_f32, void *dst, int dst_f32, int64_t n, const DevScalars *gate,
                           hipStream_t s);
hipError_t launch_vec_zero32(float *x, int64_t n, const DevScalars *gate, hipStream_t s);
hipError_t launch_vec_axpy64(double *y, const float *x, int64_t n, const DevScalars *gate, hipStream_t s);  // y += x
// u_c <- 0 at every fixed DOF c of the plan's constraints
hipError_t launch_mask_fixed(const MechGrid &M, int c, double *u, hipStream_t s);
// u <- w0 u + w1 uprev + w2 uprev2, uprev2 <- uprev, uprev <- previous u
hipError_t launch_extrapolate(double *u[3], double *uprev[3], double *uprev2[3], const double w[3], int64_t n,
                              hipStream_t s);
hipError_t launch_von_mises(const MechGrid &M, const double *theta, const double *u[3], double *vm,
                            hipStream_t s);

// One CG iteration's operator half: w = K p, alpha = rz / (p . w) into sc.
template <typename T>
hipError_t launch_cg_apply_alpha(const MechGrid &M, const CgVecs<T> &v, double *partials, DevScalars *sc,
                                 hipStream_t s);

// ---- Geometric multigrid preconditioner (mg.hip) ---------------------------
// Levels l = 0 (the mesh) .. nlev-1.  Level l+1 keeps every second node of
// level l along each axis that still has more than one cell (plus the last
// node when the cell count is odd); prolongation P interpolates linearly in
// the node coordinates, so it reproduces rigid-body motions on graded grids.
// Coarse operators are Galerkin products A_{l+1} = P^T A_l P with A_0 = K
// restricted to the free DOFs, stored as symmetric 27-point 3x3-block
// stencils; the smoother is Chebyshev on nodal-block-Jacobi, and the
// coarsest level is solved with a dense inverse.
constexpr int kMgMaxLevels = 16;
constexpr int kMgDeg = 4;   // most Chebyshev steps before (and after) the coarse correction
// Block b of nb is dispatched to XCD b % 8; give each XCD a contiguous
// range of logical tiles so that neighbouring tiles share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb / 8, r = nb % 8, x = b % 8, pos = b / 8;
  return x * q + (x < r ? x : r) + pos;
}

constexpr int kMgUpper = 14;  // stored stencil blocks: the centre and the 13 offsets after it
// Entry (r, c) of stored stencil block q of node `node` on a level of n nodes:
// the three entries of a block row are contiguous, so a wave reads a row of
// 64 consecutive nodes as one 768-byte span.
inline __host__ __device__ int64_t stencil_idx(int q, int r, int c, int64_t n, int64_t node) {
  return ((int64_t(q) * 3 + r) * n + node) * 3 + c;
}

template <typename T>
struct V3 {
  T *c[3];
};

struct MgAxis {            // fine-side interpolation table of one axis
  const int32_t *lo;       // per fine node: lower coarse node of its interval
  const double *w;         // weight of that node (1 - w on the next one)
  const int32_t *cpos;     // per coarse node: its fine node
};

template <typename T>
struct MgLevel {
  int nx, ny, nz;          // cells
  int64_t sy, sz, n;       // node strides; n = entries per component of the level's vectors
  const T *A;              // stencil blocks (coarse levels; level 0 when it is the coarsest): row r of block q
                           // at node n is A[((q * 3 + r) * n_nodes + n) * 3 + (0..2)] (see stencil_idx)
  T *Dinv;                 // [6][n] inverse nodal diagonal block (xx, yy, zz, xy, yz, xz); dead rows zero
  uint8_t *dead;           // per node: bit c = DOF c outside the space (fixed, or no stiffness)
  V3<T> xa, xb, d, b;      // smoother iterates, Chebyshev direction, right-hand side (coarse levels)
  MgAxis ax[3];            // interpolation from level + 1 (unused on the coarsest level)
  int deg;                 // Chebyshev steps on this level (1..kMgDeg)
  double c1[kMgDeg], c2[kMgDeg];
};

template <typename T>
struct MgDev {
  int nlev;
  MechGrid M;              // level-0 operator (matrix free)
  MgLevel<T> L[kMgMaxLevels];
  T *Ainv;                 // coarsest level: dense inverse over the live DOFs (symmetric, nlive^2)
  int32_t *live;           // coarsest level: live DOF codes, node * 3 + component
  int nlive;
  double *lam;             // [kMgMaxLevels] largest eigenvalue estimates of Dinv A per level
  double *scale;           // power-iteration normaliser
};

// Set-up: Galerkin operators of every level, nodal inverses and dead masks.
template <typename T>
hipError_t launch_mg_build(const MgDev<T> &G, hipStream_t s);
// Power iteration for the largest eigenvalue of Dinv A on level l (into G.lam[l]).
template <typename T>
hipError_t launch_mg_power(const MgDev<T> &G, int l, int iters, double *partials, hipStream_t s);
// z = M^{-1} b (one V-cycle); returns where z lives (level-0 xa or xb).
template <typename T>
hipError_t launch_mg_vcycle(const MgDev<T> &G, V3<T> b, const DevScalars *sc, V3<T> *z, hipStream_t s);
// Preconditioned CG with the V-cycle (vectors as for Jacobi CG; z in level-0 buffers).
template <typename T>
hipError_t launch_cgmg_setup(const MgDev<T> &G, const CgVecs<T> &v, const T *rhs[3], double *partials,
                             DevScalars *sc, DevScalars *gate, hipStream_t s);
template <typename T>
hipError_t launch_cgmg_iteration(const MgDev<T> &G, const CgVecs<T> &v, double *partials, DevScalars *sc,
                                 hipStream_t s);

int reduce_blocks(int64_t ntot);

}  // namespace etm
