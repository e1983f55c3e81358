// Private host-side plan of the library (shared by plan.cpp and batch.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <string>
#include <vector>

#include "etm_internal.h"

namespace etm {
// A host-side roctx range over a scope (the enqueue of a phase, or a wait):
// EM steps, thermal step, mechanical solve, settle, batch advance.  Seen by
// rocprofv3 --marker-trace; a call without a tool attached does nothing.
struct Range {
  explicit Range(const char *name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range &) = delete;
  Range &operator=(const Range &) = delete;
};
}  // namespace etm

namespace etm {
etm_status fail(etm_status s, const std::string &msg);
struct Region {
  size_t off = 0, bytes = 0;
};
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace etm

#define HIP_TRY(expr)                                                                                      \
  do {                                                                                                     \
    hipError_t e_ = (expr);                                                                                \
    if (e_ != hipSuccess) return etm::fail(ETM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)



using namespace etm;

// One level of the mechanical multigrid hierarchy (host view).
struct MgHostLevel {
  int nx = 0, ny = 0, nz = 0;          // cells
  int64_t sy = 0, sz = 0, n = 0;       // node strides, entries per vector component
  Region A, Dinv, dead, xa, xb, d, b;  // device regions (A: coarse levels only)
  size_t tab[3][3] = {};               // offsets in r_mgtab of lo, w, cpos per axis (from level + 1)
  int deg = 2;
  double c1[kMgDeg] = {}, c2[kMgDeg] = {};
};

// a_base of a plan whose closed-form wave table holds no valid block
constexpr int64_t kNoWaveBlock = -(int64_t(1) << 62);

struct etm_plan {
  // ---- inputs (deep copies)
  int nx = 0, ny = 0, nz = 0, n_mat = 0;
  std::vector<double> dx, dy, dz;
  std::vector<uint8_t> mat_nat;
  std::vector<etm_material> mats;
  int n_waves = 0;
  int64_t n_samples = 0;
  std::vector<double> J;
  int n_analytic = 0;
  std::vector<double> aw;  // closed-form waves, kWaveStride doubles each
  int64_t a_base = kNoWaveBlock;  // first sample of the device table of closed-form waves
  etm_opts opts{};
  double dt = 0;
  int prec = ETM_PREC_FP64, R = 1;
  // ---- layout
  int64_t sy = 0, sz = 0, ntot = 0;
  dim3 ngrid;
  int64_t nblocks_node = 0;
  // ---- host tables
  std::vector<double> geo;  // dx,dy,dz,idx,idy,idz (n each), hx,hy,hz,ihx,ihy,ihz (n+1 each)
  size_t geo_off[18] = {};
  std::vector<double> mtab;
  std::vector<uint8_t> mat_pad, flags, fixed;
  std::vector<int64_t> pe_key;
  std::vector<double> pe_gs, pw_wt;
  std::vector<int32_t> pe_start, pw_wave;
  std::vector<int64_t> probes_dev;  // [field, padded index]
  int64_t hist_cap = 0;
  int hist_cols = 4;
  // ---- workspace regions
  Region r_geo, r_mtab, r_mat, r_flags, r_fixed, r_pkey, r_pgs, r_pstart, r_pwave, r_pwt, r_J, r_probes, r_per, r_aw, r_Ja;
  Region r_coef[6];     // per-node edge coefficients: eps_r x/y/z, a x/y/z (field precision)
  Region r_e[3][3];     // FP64: three rotating e buffers;  MIXED: [0..1] e sets, [2] unused
  Region r_h[2][3];     // MIXED: face-field sets h^{n-1/2} (x-, y-, z-normal faces)
  Region r_K[3];        // MIXED: per-edge correction of the leapfrog form for sigma changes
  Region r_elo;         // MIXED: 8-bit residual of e (3 components at stride comp_stride)
  Region r_theta[2], r_theta32, r_psum, r_part, r_sc, r_hist;
  Region r_partm, r_scm, r_ctl, r_thsolve;  // the mechanical solve's partials, scalars, control block, temperature
  Region r_gR, r_gF;                        // its gate words (restart phase, finish phase)
  Region r_u64[3], r_f64[3], r_r64[3], r_p64[3], r_w64[3], r_dinv64[3], r_uprev64[3], r_uprev2_64[3];
  Region r_u32[3], r_r32[3], r_p32[3], r_w32[3], r_dinv32[3], r_rhs32[3];
  Region r_vm, r_stage;
  // multigrid preconditioner of the mechanical CG
  std::vector<MgHostLevel> mg;         // empty with the Jacobi preconditioner
  std::vector<char> mg_tab;            // interpolation tables (uploaded at bind)
  Region r_mgtab, r_mglive, r_mgainv, r_mgsc;
  int mg_nlive = 0;
  bool mg_ready = false;
  size_t footprint = 0;
  // ---- bound state
  char *ws = nullptr;
  hipStream_t stream = nullptr;
  // side stream of overlapped mechanical solves, and the events that order
  // it against the plan's stream (created at the first bind): ev_main after
  // a thermal step, ev_copy once a solve has read the temperature, ev_solve
  // at the end of a solve's last enqueued passes
  hipStream_t mstream = nullptr;
  hipEvent_t ev_main = nullptr, ev_copy = nullptr, ev_solve = nullptr;
  bool bound = false;
  DevScalars *sc_host = nullptr;   // pinned
  DevScalars *ctl_host = nullptr;  // pinned copy of the solve's control block (written by the device)
  bool solve_pending = false;      // a solve is enqueued and not yet settled
  int solve_enqueued = 0;          // inner iterations enqueued for it so far
  int solve_rounds = 0;            // passes added to it at settle
  int pass_plan_n = 0;             // passes to enqueue for the next solve (0: no history yet)
  int pass_plan[kMaxPasses] = {};  // inner iterations of each
  int64_t step = 0;
  int cur = 0;      // FP64: e^n = buffer cur; MIXED: set cur
  int th_cur = 0;
  int64_t rec = 0;
  int64_t n_thermal = 0;
  int n_solves = 0, cg_iters = 0, cg_outer = 0;
  int64_t sol_t[3] = {-1, -1, -1};  // thermal-step count at the last three mechanical solves
  int64_t cg_total = 0;
  double cg_relres = 0;
  etm_status host_status = ETM_OK;
  std::string host_msg;
  bool dinv_ready = false;
  bool joule_pending = false;  // Joule power of the current field not yet in psum
  int kchunk = 0;              // z planes per EM block (0 = automatic)
  int layout = 0;              // mixed march work layout (kLayoutAuto unless a batch's tuning table sets it)
  int64_t comp_stride = 0;     // elements between the x, y, z components of a field
  bool has_tcr = false;        // some conducting material has a temperature coefficient

  template <typename T>
  T *ptr(const Region &r) const { return reinterpret_cast<T *>(ws + r.off); }

  DevGrid dev_grid() const {
    DevGrid g;
    g.nx = nx; g.ny = ny; g.nz = nz; g.n_mat = n_mat;
    g.sy = sy; g.sz = sz; g.ntot = ntot;
    const double *gb = ptr<double>(r_geo);
    g.dx = gb + geo_off[0]; g.dy = gb + geo_off[1]; g.dz = gb + geo_off[2];
    g.idx = gb + geo_off[3]; g.idy = gb + geo_off[4]; g.idz = gb + geo_off[5];
    g.hx = gb + geo_off[6]; g.hy = gb + geo_off[7]; g.hz = gb + geo_off[8];
    g.ihx = gb + geo_off[9]; g.ihy = gb + geo_off[10]; g.ihz = gb + geo_off[11];
    g.al[0] = gb + geo_off[12]; g.ah[0] = gb + geo_off[13];
    g.al[1] = gb + geo_off[14]; g.ah[1] = gb + geo_off[15];
    g.al[2] = gb + geo_off[16]; g.ah[2] = gb + geo_off[17];
    g.geo = gb;
    g.cs = 0;
    g.mat = ptr<uint8_t>(r_mat);
    g.flags = ptr<uint8_t>(r_flags);
    g.mtab = ptr<double>(r_mtab);
    int pec = 0;
    for (int f = 0; f < 6; ++f) if (opts.em_bc[f] == ETM_PEC) pec |= 1 << f;
    g.pec = pec;
    g.layout = layout;
    return g;
  }
  DevPorts dev_ports() const {
    DevPorts p;
    p.n_edges = int(pe_key.size());
    p.key = ptr<int64_t>(r_pkey);
    p.gs = ptr<double>(r_pgs);
    p.start = ptr<int32_t>(r_pstart);
    p.wave = ptr<int32_t>(r_pwave);
    p.wt = ptr<double>(r_pwt);
    p.J = ptr<double>(r_J);
    p.n_samples = n_samples;
    p.Ja = ptr<double>(r_Ja);
    p.a_base = a_base;
    p.n_table = n_waves;
    p.er = ptr<double>(r_per);
    return p;
  }
  MechGrid mech_grid() const {
    MechGrid m;
    m.g = dev_grid();
    m.fixed = ptr<uint8_t>(r_fixed);
    return m;
  }
  DevScalars *sc() const { return ptr<DevScalars>(r_sc); }
  DevScalars *scm() const { return ptr<DevScalars>(r_scm); }
  DevScalars *ctl() const { return ptr<DevScalars>(r_ctl); }
  int64_t nidx(int i, int j, int k) const { return int64_t(k) * sz + int64_t(j) * sy + i; }
};


namespace etm {
EmLaunch em_launch_template(const etm_plan *p);
etm_status em_one_step(etm_plan *p);
// Refill the device table of closed-form wave samples if it does not cover the
// next `ahead` (<= kWaveBlock) EM steps of the plan.
etm_status ensure_waves(etm_plan *p, int64_t ahead);
etm_status thermal_one(etm_plan *p);
etm_status joule_flush(etm_plan *p);
etm_status coef_refresh(etm_plan *p, bool update_k);
etm_status diag_record(etm_plan *p, int old_cur);
// Enqueue a mechanical solve (no wait once the multigrid hierarchy exists).
etm_status mech_solve_impl(etm_plan *p);
// Wait for an enqueued solve to be decided (adding passes if it needs more);
// a solve that gave up sets host_status = ETM_E_NOCONV.
etm_status solve_settle(etm_plan *p);
}  // namespace etm
