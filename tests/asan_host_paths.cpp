// Host paths of the C ABI under AddressSanitizer and LeakSanitizer, on a
// machine without a GPU: plan creation (valid inputs and every class of
// rejected input), footprint, step and DOF queries, destruction, and batch
// creation with well-formed and malformed tuning JSON (parsed before the
// batch asks the runtime for a device; without a GPU the call then fails
// and must release everything).  Built host-only by test_asan_host.py.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "etm.h"

static int g_fail = 0;
#define CHECK(c)                                                              \
  do {                                                                        \
    if (!(c)) {                                                               \
      std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #c);    \
      ++g_fail;                                                               \
    }                                                                         \
  } while (0)

struct Case {
  int nx = 8, ny = 6, nz = 5;
  std::vector<double> dx, dy, dz;
  std::vector<uint8_t> mat;
  std::vector<etm_material> mats;
  std::vector<etm_port> ports;
  std::vector<double> J;
  std::vector<etm_wave> waves;
  std::vector<int64_t> probes;
  std::vector<uint8_t> mask;
  etm_mesh mesh{};
  etm_source src{};
  etm_opts opts{};

  Case() {
    for (int i = 0; i < nx; ++i) dx.push_back(1e-6 * (1.0 + 0.1 * i));
    for (int j = 0; j < ny; ++j) dy.push_back(1e-6 * (1.5 - 0.05 * j));
    for (int k = 0; k < nz; ++k) dz.push_back(2e-6);
    for (int c = 0; c < nx * ny * nz; ++c) mat.push_back(uint8_t(c / (nx * ny) == nz - 1 ? 2 : (c * 7) % 2));
    mats.push_back({11.7, 10.0, 0.0, 148.0, 1.63e6, 130e9, 0.28, 2.6e-6, 0, 0});
    mats.push_back({1.0, 5.8e7, 3.9e-3, 400.0, 3.45e6, 117e9, 0.34, 17e-6, 0, 0});
    mats.push_back({1.0, 0.0, 0.0, 0.026, 1.2e3, 1.0, 0.0, 0.0, 1, 0});
    ports.push_back({0, 1, 2, 2, 0, 0, 1.0, 0.0});
    ports.push_back({2, 3, 3, 1, 1, 0, 1.0, 0.02});
    for (int s = 0; s < 32; ++s) J.push_back(s ? 1e9 * std::sin(0.3 * s) : 0.0);
    etm_wave w{};
    w.kind = ETM_WAVE_GAUSS_TRAIN;
    w.n_pulses = 3;
    w.amp = 1e9; w.t0 = 0.0; w.width = 1e-12; w.freq = 1e10; w.t_on = 0.0; w.t_off = 1e-9;
    w.pulse_t[0] = 1e-12; w.pulse_t[1] = 3e-12; w.pulse_t[2] = 5e-12;
    waves.push_back(w);
    ports.push_back({1, 4, 1, 2, 1, 0, 0.5, 0.0});  // wave 1: sampled wave 1 (two sampled waves below)
    ports.push_back({0, 2, 4, 3, 2, 0, 1.0, 0.0});  // wave 2: the analytic wave
    for (int s = 0; s < 32; ++s) J.push_back(0.5 * J[s]);
    int64_t pr[8] = {0, 1, 2, 2, 3, 4, 3, 2};
    probes.assign(pr, pr + 8);
    mask.assign(size_t(nx + 1) * (ny + 1) * (nz + 1), 0);
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i <= nx; ++i) mask[size_t(j) * (nx + 1) + i] = 7;
    refresh();
  }
  void refresh() {
    mesh.nx = nx; mesh.ny = ny; mesh.nz = nz;
    mesh.dx = dx.data(); mesh.dy = dy.data(); mesh.dz = dz.data(); mesh.mat = mat.data();
    src.n_ports = int64_t(ports.size()); src.ports = ports.data();
    src.n_waves = 2; src.n_samples = 32; src.J_half = J.data();
    src.n_analytic = int32_t(waves.size()); src.analytic = waves.data();
    etm_opts_default(&opts);
    opts.precision = ETM_PREC_MIXED;
    opts.em_per_thermal = 4;
    opts.history_stride = 2;
    opts.n_probes = 2;
    opts.probes = probes.data();
    opts.n_em_steps_hint = 40;
    opts.mech_mask = mask.data();
  }
  etm_status create(etm_plan **p) { return etm_plan_create(&mesh, mats.data(), int32_t(mats.size()), &src, &opts, p); }
};

static void expect_inval(const char *what, Case &c, etm_status want = ETM_E_INVAL) {
  etm_plan *p = reinterpret_cast<etm_plan *>(0x1);
  const etm_status st = c.create(&p);
  if (st != want || p != nullptr || std::strlen(etm_last_error()) == 0) {
    std::fprintf(stderr, "%s: status %d, plan %p, message '%s'\n", what, int(st), (void *)p, etm_last_error());
    ++g_fail;
  }
}

int main() {
  // valid plans in both precisions and with both preconditioners
  for (int prec = 0; prec < 2; ++prec)
    for (int pc = 0; pc < 2; ++pc) {
      Case c;
      c.opts.precision = prec ? ETM_PREC_FP64 : ETM_PREC_MIXED;
      c.opts.mech_precond = pc ? ETM_PRECOND_JACOBI : ETM_PRECOND_MG;
      c.opts.em_slabs = 2;
      etm_plan *p = nullptr;
      CHECK(c.create(&p) == ETM_OK && p != nullptr);
      size_t fp = 0;
      double dt = 0;
      int64_t nem = 0, nth = 0, nme = 0;
      CHECK(etm_plan_footprint(p, &fp) == ETM_OK && fp > 0);
      CHECK(etm_plan_dt(p, &dt) == ETM_OK && dt > 0);
      CHECK(etm_plan_dofs(p, &nem, &nth, &nme) == ETM_OK && nth == int64_t(9) * 7 * 6 && nem > 0 && nme > 0);
      size_t ck = 0;
      CHECK(etm_checkpoint_size(p, &ck) == ETM_OK && ck > 0);
      etm_plan_destroy(p);
    }
  etm_plan_destroy(nullptr);
  double dt = 0;
  {
    Case c;
    CHECK(etm_cfl_dt(&c.mesh, 0.9, &dt) == ETM_OK && dt > 0);
    CHECK(etm_cfl_dt(nullptr, 0.9, &dt) != ETM_OK);
  }
  // rejected inputs: every one returns its status, leaves *out null, sets a
  // message and frees what creation had allocated so far
  { Case c; c.nx = 0; c.refresh(); expect_inval("nx = 0", c); }
  { Case c; c.mat[17] = 3; expect_inval("material id out of range", c); }
  { Case c; c.dx[3] = -1e-6; expect_inval("negative width", c); }
  { Case c; c.dz[2] = NAN; expect_inval("NaN width", c); }
  { Case c; c.mats[1].nu = 0.5; expect_inval("nu = 0.5", c); }
  { Case c; c.mats[0].rho_cp = 0.0; expect_inval("rho_cp = 0", c); }
  { Case c; c.opts.em_per_thermal = 0; expect_inval("R = 0", c); }
  { Case c; c.opts.mg_degree[1] = 5; expect_inval("mg degree", c); }
  { Case c; c.opts.em_slabs = 65; expect_inval("em_slabs", c); }
  { Case c; c.opts.mech_overlap = 2; expect_inval("mech_overlap", c); }
  { Case c; c.opts.cfl = 1.5; expect_inval("cfl", c); }
  { Case c; c.opts.dt = 1.0; expect_inval("dt above CFL", c, ETM_E_UNSTABLE); }
  { Case c; c.ports[1].k = c.nz + 1; expect_inval("port outside the mesh", c); }
  { Case c; c.ports[0].wave = 7; expect_inval("port wave index", c); }
  { Case c; c.waves[0].kind = 9; expect_inval("wave kind", c); }
  { Case c; c.waves[0].n_pulses = ETM_WAVE_MAX_PULSES + 1; expect_inval("pulse count", c); }
  { Case c; c.waves[0].width = 0.0; expect_inval("wave width", c); }
  { Case c; c.probes[5] = 40; expect_inval("probe outside the mesh", c); }
  { Case c; c.src.J_half = nullptr; expect_inval("null J_half", c); }
  { Case c; std::vector<etm_material> many(257, c.mats[0]); c.mats = many; expect_inval("n_mat = 257", c); }
  {
    Case c;
    etm_plan *p = nullptr;
    CHECK(etm_plan_create(nullptr, c.mats.data(), 3, &c.src, &c.opts, &p) == ETM_E_INVAL && !p);
    CHECK(etm_plan_create(&c.mesh, c.mats.data(), 3, &c.src, &c.opts, nullptr) == ETM_E_INVAL);
    size_t fp = 0;
    CHECK(etm_plan_footprint(nullptr, &fp) == ETM_E_INVAL);
  }
  // batch creation: the tuning JSON is parsed first, then the device is
  // queried; malformed JSON is ignored, never read out of bounds
  const char *tunes[] = {
      nullptr, "", "{}", "{\"kchunk\": {\"17\": 8, \"33\": 16}}", "{\"kchunk\": {\"17\": 8, ",
      "{\"kchunk\"", "{\"kchunk\": {", "{\"kchunk\": {\"", "{\"kchunk\": {\"5\"", "{\"kchunk\": {\"5\":",
      "{\"kchunk\": {\"5\": 999, \"6\": -1, \"x\": \"y\"}}", "\"kchunk\":}", "{\"kchunk\": {\"1\": 4}, \"kchunk\": 3}",
      "{\"kchunk\": {\"17\": 8}, \"layout\": {\"17\": 2, \"18\": 1, \"19\": 7}}", "{\"layout\": {\"",
      "{\"layout\"", "{\"layout\": {\"3\": }",
      "{\"kchunk\": {\"17\": 6}, \"kchunk_fp64\": {\"17\": 24, \"20\": 2, \"21\": 0}}", "{\"kchunk_fp64\": {",
  };
  for (const char *t : tunes) {
    etm_batch *b = reinterpret_cast<etm_batch *>(0x1);
    const etm_status st = etm_batch_create(4, t, &b);
    if (st == ETM_OK) {
      CHECK(b != nullptr);
      etm_batch_destroy(b);
    } else {
      CHECK(b == nullptr && std::strlen(etm_last_error()) > 0);
    }
  }
  std::string big = "{\"kchunk\": {";
  for (int q = 0; q < 2000; ++q) big += "\"" + std::to_string(q) + "\": " + std::to_string(q % 130) + ", ";
  big += "\"2000\": 1}}";
  {
    etm_batch *b = nullptr;
    if (etm_batch_create(4, big.c_str(), &b) == ETM_OK) etm_batch_destroy(b);
  }
  {
    etm_batch *b = nullptr;
    CHECK(etm_batch_create(0, nullptr, &b) != ETM_OK && !b);
  }
  etm_batch_destroy(nullptr);
  if (g_fail) {
    std::fprintf(stderr, "%d check(s) failed\n", g_fail);
    return 1;
  }
  std::printf("ALL OK\n");
  return 0;
}
