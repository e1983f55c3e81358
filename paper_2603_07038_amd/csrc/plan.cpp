// Host side of the C ABI declared in include/etm.h: input validation, derived
// tables, DOF maps and constraints, workspace layout, the coupling schedule
// of arXiv 2603.07038 Sec. II-A (EM step, Joule source, thermal step every R
// EM steps) and the CG driver for Sec. II-B.  All GPU work goes through the
// launchers in em.hip / mech.hip on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "etm_internal.h"
#include "plan.h"

using namespace etm;

namespace etm {
namespace {
thread_local std::string g_err;
}  // namespace
etm_status fail(etm_status s, const std::string &msg) {
  g_err = msg;
  return s;
}
}  // namespace etm

namespace {

// Node-centred widths: half cells at the two ends.
std::vector<double> dual(const std::vector<double> &d) {
  std::vector<double> h(d.size() + 1, 0.0);
  for (size_t i = 0; i < d.size(); ++i) { h[i] += 0.5 * d[i]; h[i + 1] += 0.5 * d[i]; }
  return h;
}

double cfl_limit(const double *dx, int nx, const double *dy, int ny, const double *dz, int nz) {
  double mx = 1e300, my = 1e300, mz = 1e300;
  for (int i = 0; i < nx; ++i) mx = std::min(mx, dx[i]);
  for (int j = 0; j < ny; ++j) my = std::min(my, dy[j]);
  for (int k = 0; k < nz; ++k) mz = std::min(mz, dz[k]);
  return 1.0 / (kC0 * std::sqrt(1.0 / (mx * mx) + 1.0 / (my * my) + 1.0 / (mz * mz)));
}

// Index of the node nearest the midpoint of a 1D node row (lower on a tie).
int nearest_mid(const std::vector<double> &d) {
  double tot = 0;
  for (double v : d) tot += v;
  const double mid = 0.5 * tot;
  double x = 0, best = 1e300;
  int bi = 0;
  for (size_t i = 0; i <= d.size(); ++i) {
    const double dist = std::fabs(x - mid);
    if (dist < best) { best = dist; bi = int(i); }
    if (i < d.size()) x += d[i];
  }
  return bi;
}

etm_status validate_and_copy(etm_plan *p, const etm_mesh *mesh, const etm_material *mats, int32_t n_mat,
                             const etm_source *src, const etm_opts *opts) {
  if (!mesh || !mats || !opts) return fail(ETM_E_INVAL, "null mesh, materials or options");
  if (mesh->nx < 1 || mesh->ny < 1 || mesh->nz < 1) return fail(ETM_E_INVAL, "mesh dimensions must be >= 1");
  if ((int64_t)mesh->nx * mesh->ny * mesh->nz > (int64_t(1) << 34)) return fail(ETM_E_INVAL, "mesh too large");
  if (!mesh->dx || !mesh->dy || !mesh->dz || !mesh->mat) return fail(ETM_E_INVAL, "null mesh array");
  if (n_mat < 1 || n_mat > 256) return fail(ETM_E_INVAL, "n_mat must be in 1..256");
  p->nx = mesh->nx; p->ny = mesh->ny; p->nz = mesh->nz; p->n_mat = n_mat;
  p->dx.assign(mesh->dx, mesh->dx + p->nx);
  p->dy.assign(mesh->dy, mesh->dy + p->ny);
  p->dz.assign(mesh->dz, mesh->dz + p->nz);
  for (auto *v : {&p->dx, &p->dy, &p->dz})
    for (double w : *v)
      if (!(w > 0.0) || !std::isfinite(w)) return fail(ETM_E_INVAL, "cell widths must be finite and > 0");
  const size_t nc = size_t(p->nx) * p->ny * p->nz;
  p->mat_nat.assign(mesh->mat, mesh->mat + nc);
  for (size_t c = 0; c < nc; ++c)
    if (p->mat_nat[c] >= n_mat) return fail(ETM_E_INVAL, "material id out of range at cell " + std::to_string(c));
  p->mats.assign(mats, mats + n_mat);
  for (int m = 0; m < n_mat; ++m) {
    const etm_material &q = mats[m];
    if (!(q.eps_r >= 1.0) || q.sigma0 < 0 || q.k < 0 || !(q.rho_cp > 0))
      return fail(ETM_E_INVAL, "material " + std::to_string(m) + ": need eps_r >= 1, sigma0 >= 0, k >= 0, rho_cp > 0");
    if (!q.is_void && (!(q.E > 0) || !(q.nu > -1.0 && q.nu < 0.5)))
      return fail(ETM_E_INVAL, "material " + std::to_string(m) + ": need E > 0 and -1 < nu < 0.5");
  }
  p->opts = *opts;
  if (opts->precision != ETM_PREC_FP64 && opts->precision != ETM_PREC_MIXED) return fail(ETM_E_INVAL, "bad precision");
  for (int f = 0; f < 6; ++f)
    if (opts->em_bc[f] != ETM_PMC && opts->em_bc[f] != ETM_PEC) return fail(ETM_E_INVAL, "bad em_bc");
  if (opts->em_per_thermal < 1) return fail(ETM_E_INVAL, "em_per_thermal must be >= 1");
  if (opts->mech_every_thermal < 0) return fail(ETM_E_INVAL, "mech_every_thermal must be >= 0");
  if (opts->mech_bc != ETM_MECH_KINEMATIC && opts->mech_bc != ETM_MECH_CLAMP_ZMIN) return fail(ETM_E_INVAL, "bad mech_bc");
  if (opts->cg_maxit < 1 || !(opts->cg_rtol > 0)) return fail(ETM_E_INVAL, "cg_maxit >= 1 and cg_rtol > 0 required");
  if (opts->history_stride < 0 || opts->n_probes < 0 || (opts->n_probes > 0 && !opts->probes))
    return fail(ETM_E_INVAL, "bad history options");
  if (opts->mech_precond != ETM_PRECOND_JACOBI && opts->mech_precond != ETM_PRECOND_MG)
    return fail(ETM_E_INVAL, "bad mech_precond");
  if (opts->mg_coarse_dofs == 0) p->opts.mg_coarse_dofs = 800;
  if (p->opts.mg_coarse_dofs < 3 || p->opts.mg_coarse_dofs > 4000)
    return fail(ETM_E_INVAL, "mg_coarse_dofs must be 0 (default) or 3..4000");
  for (int q = 0; q < 2; ++q) {
    if (opts->mg_degree[q] == 0) p->opts.mg_degree[q] = q == 0 ? 3 : 2;
    if (p->opts.mg_degree[q] < 1 || p->opts.mg_degree[q] > kMgDeg)
      return fail(ETM_E_INVAL, "mg_degree entries must be 0 (default) or 1..4");
  }
  if (opts->em_slabs < 0 || opts->em_slabs > 64) return fail(ETM_E_INVAL, "em_slabs must be 0..64");
  if (opts->mech_overlap != 0 && opts->mech_overlap != 1) return fail(ETM_E_INVAL, "mech_overlap must be 0 or 1");
  p->prec = opts->precision;
  p->R = opts->em_per_thermal;
  // time step
  const double lim = cfl_limit(p->dx.data(), p->nx, p->dy.data(), p->ny, p->dz.data(), p->nz);
  if (opts->dt > 0) {
    p->dt = opts->dt;
    if (p->dt > lim * (1.0 + 1e-12) && !opts->force_dt)
      return fail(ETM_E_UNSTABLE, "dt " + std::to_string(p->dt) + " exceeds the CFL limit " + std::to_string(lim));
  } else {
    if (!(opts->cfl > 0 && opts->cfl <= 1.0)) return fail(ETM_E_INVAL, "cfl must be in (0, 1]");
    p->dt = opts->cfl * lim;
  }
  // sources
  p->n_waves = src ? src->n_waves : 0;
  p->n_samples = src ? src->n_samples : 0;
  p->n_analytic = src ? src->n_analytic : 0;
  if (p->n_waves < 0 || p->n_samples < 0 || p->n_analytic < 0) return fail(ETM_E_INVAL, "negative wave counts");
  if (p->n_waves > 0 && p->n_samples > 0) {
    if (!src->J_half) return fail(ETM_E_INVAL, "null J_half");
    p->J.assign(src->J_half, src->J_half + size_t(p->n_waves) * p->n_samples);
  } else {
    p->n_waves = 0;
    p->n_samples = 0;
  }
  p->aw.clear();
  if (p->n_analytic > 0) {
    if (!src->analytic) return fail(ETM_E_INVAL, "null analytic wave array");
    for (int w = 0; w < p->n_analytic; ++w) {
      const etm_wave &a = src->analytic[w];
      const std::string where = "analytic wave " + std::to_string(w) + ": ";
      if (a.kind != ETM_WAVE_RICKER && a.kind != ETM_WAVE_SINE && a.kind != ETM_WAVE_GAUSS_TRAIN)
        return fail(ETM_E_INVAL, where + "unknown kind");
      const int np = a.kind == ETM_WAVE_GAUSS_TRAIN ? a.n_pulses : 0;
      if (a.kind == ETM_WAVE_GAUSS_TRAIN && (np < 1 || np > ETM_WAVE_MAX_PULSES))
        return fail(ETM_E_INVAL, where + "n_pulses must be in 1..8");
      bool fin = std::isfinite(a.amp) && std::isfinite(a.t0) && std::isfinite(a.width) && std::isfinite(a.freq) &&
                 std::isfinite(a.t_on) && std::isfinite(a.t_off);
      for (int q = 0; q < np; ++q) fin = fin && std::isfinite(a.pulse_t[q]);
      if (!fin) return fail(ETM_E_INVAL, where + "non-finite parameter");
      if (a.kind != ETM_WAVE_SINE && !(a.width > 0)) return fail(ETM_E_INVAL, where + "width must be > 0");
      if (!(a.t_on <= a.t_off)) return fail(ETM_E_INVAL, where + "t_on must be <= t_off");
      const double rec[8] = {double(a.kind), double(np), a.amp, a.t0, a.width, a.freq, a.t_on, a.t_off};
      p->aw.insert(p->aw.end(), rec, rec + 8);
      for (int q = 0; q < kWaveStride - 8; ++q) p->aw.push_back(q < np ? a.pulse_t[q] : 0.0);
    }
  }
  if (src && src->n_ports > 0) {
    if (!src->ports) return fail(ETM_E_INVAL, "null port array");
    if (p->n_waves + p->n_analytic < 1) return fail(ETM_E_INVAL, "ports need sampled or closed-form waves");
  }
  return ETM_OK;
}

// Linear interpolation of one axis from its next coarser level: the coarse
// nodes are every second node (plus the last one when the cell count is
// odd); fine node i lies in [cpos[lo], cpos[lo+1]] with weight w on lo.
// An axis of one cell is kept as it is.
void mg_axis(const std::vector<double> &x, std::vector<int32_t> &lo, std::vector<double> &w,
             std::vector<int32_t> &cpos, std::vector<double> &xc, bool keep) {
  const int n = int(x.size()) - 1;
  cpos.clear();
  if (keep || n <= 1) {
    for (int i = 0; i <= n; ++i) cpos.push_back(i);
  } else {
    for (int i = 0; i <= n; i += 2) cpos.push_back(i);
    if (cpos.back() != n) cpos.push_back(n);
  }
  lo.assign(n + 1, 0);
  w.assign(n + 1, 1.0);
  int I = 0;
  for (int i = 0; i <= n; ++i) {
    while (I + 1 < int(cpos.size()) && cpos[I + 1] <= i) ++I;
    lo[i] = I;
    w[i] = cpos[I] == i ? 1.0 : (x[cpos[I + 1]] - x[i]) / (x[cpos[I + 1]] - x[cpos[I]]);
  }
  xc.resize(cpos.size());
  for (size_t q = 0; q < cpos.size(); ++q) xc[q] = x[cpos[q]];
}

// Levels of the mechanical multigrid: coarsen until a level has at most
// mg_coarse_dofs DOF.  Level 0 uses the plan's padded layout, coarser levels
// a dense one.
void mg_levels(etm_plan *p) {
  p->mg.clear();
  p->mg_tab.clear();
  if (p->opts.mech_precond != ETM_PRECOND_MG) return;
  std::vector<double> xs[3];
  const std::vector<double> *d[3] = {&p->dx, &p->dy, &p->dz};
  for (int a = 0; a < 3; ++a) {
    xs[a].assign(1, 0.0);
    for (double h : *d[a]) xs[a].push_back(xs[a].back() + h);
  }
  MgHostLevel L0;
  L0.deg = p->opts.mg_degree[0];
  L0.nx = p->nx; L0.ny = p->ny; L0.nz = p->nz;
  L0.sy = p->sy; L0.sz = p->sz; L0.n = p->ntot;
  p->mg.push_back(L0);
  auto put = [&](const void *src, size_t bytes) {
    const size_t o = align256(p->mg_tab.size());
    p->mg_tab.resize(o + bytes);
    std::memcpy(p->mg_tab.data() + o, src, bytes);
    return o;
  };
  std::vector<int32_t> lo, cpos;
  std::vector<double> w, xc;
  for (;;) {
    const MgHostLevel F = p->mg.back();
    const int64_t dofs = 3 * int64_t(F.nx + 1) * (F.ny + 1) * (F.nz + 1);
    const bool coarsest = dofs <= p->opts.mg_coarse_dofs || (F.nx <= 1 && F.ny <= 1 && F.nz <= 1) ||
                          int(p->mg.size()) == kMgMaxLevels;
    const bool identity = coarsest && p->mg.size() == 1;  // level 0 assembles its own stencil
    if (coarsest && !identity) break;
    int cells[3];
    for (int a = 0; a < 3; ++a) {
      mg_axis(xs[a], lo, w, cpos, xc, identity);
      p->mg.back().tab[a][0] = put(lo.data(), lo.size() * 4);
      p->mg.back().tab[a][1] = put(w.data(), w.size() * 8);
      p->mg.back().tab[a][2] = put(cpos.data(), cpos.size() * 4);
      cells[a] = int(cpos.size()) - 1;
      xs[a] = xc;
    }
    if (identity) break;
    MgHostLevel C;
    C.deg = p->opts.mg_degree[1];
    C.nx = cells[0]; C.ny = cells[1]; C.nz = cells[2];
    C.sy = C.nx + 1; C.sz = C.sy * (C.ny + 1); C.n = C.sz * (C.nz + 1);
    p->mg.push_back(C);
  }
}

etm_status derive(etm_plan *p, const etm_source *src) {
  const int nx = p->nx, ny = p->ny, nz = p->nz;
  p->sy = ((nx + 1 + kPad - 1) / kPad) * kPad;
  p->sz = p->sy * (ny + 1);
  p->ntot = p->sz * (nz + 1);
  p->ngrid = dim3((nx + 1 + 63) / 64, (ny + 1 + 3) / 4, nz + 1);
  p->nblocks_node = int64_t(p->ngrid.x) * p->ngrid.y * p->ngrid.z;
  // geometry table
  const std::vector<double> hx = dual(p->dx), hy = dual(p->dy), hz = dual(p->dz);
  const std::vector<double> *parts[18];
  std::vector<double> idx(nx), idy(ny), idz(nz), ihx(nx + 1), ihy(ny + 1), ihz(nz + 1);
  // Share of a node's dual width on each side: alpha_lo(i) = dx[i-1] / (2 hx[i]),
  // alpha_hi(i) = dx[i] / (2 hx[i]) (0 for a missing cell).  Products of two
  // of them are the area weights of an edge's (up to four) cells.
  auto alphas = [](const std::vector<double> &d, const std::vector<double> &h, std::vector<double> &lo,
                   std::vector<double> &hi) {
    const size_t n = d.size();
    lo.assign(n + 1, 0.0);
    hi.assign(n + 1, 0.0);
    for (size_t q = 0; q <= n; ++q) {
      if (q > 0) lo[q] = d[q - 1] / (2.0 * h[q]);
      if (q < n) hi[q] = d[q] / (2.0 * h[q]);
    }
  };
  std::vector<double> axl, axh, ayl, ayh, azl, azh;
  for (int i = 0; i < nx; ++i) idx[i] = 1.0 / p->dx[i];
  for (int j = 0; j < ny; ++j) idy[j] = 1.0 / p->dy[j];
  for (int k = 0; k < nz; ++k) idz[k] = 1.0 / p->dz[k];
  for (int i = 0; i <= nx; ++i) ihx[i] = 1.0 / hx[i];
  for (int j = 0; j <= ny; ++j) ihy[j] = 1.0 / hy[j];
  for (int k = 0; k <= nz; ++k) ihz[k] = 1.0 / hz[k];
  parts[0] = &p->dx; parts[1] = &p->dy; parts[2] = &p->dz;
  parts[3] = &idx; parts[4] = &idy; parts[5] = &idz;
  parts[6] = &hx; parts[7] = &hy; parts[8] = &hz;
  parts[9] = &ihx; parts[10] = &ihy; parts[11] = &ihz;
  alphas(p->dx, hx, axl, axh);
  alphas(p->dy, hy, ayl, ayh);
  alphas(p->dz, hz, azl, azh);
  parts[12] = &axl; parts[13] = &axh; parts[14] = &ayl; parts[15] = &ayh; parts[16] = &azl; parts[17] = &azh;
  p->geo.clear();
  for (int q = 0; q < 18; ++q) {
    p->geo_off[q] = p->geo.size();
    p->geo.insert(p->geo.end(), parts[q]->begin(), parts[q]->end());
  }
  // material rows
  p->mtab.assign(size_t(p->n_mat) * kMatStride, 0.0);
  for (int m = 0; m < p->n_mat; ++m) {
    const etm_material &q = p->mats[m];
    double *row = &p->mtab[size_t(m) * kMatStride];
    row[MC_EPSR] = q.eps_r;
    row[MC_SIGS] = q.sigma0 * p->dt / (2.0 * kEps0);
    row[MC_TCR] = q.tcr;
    row[MC_K] = q.k;
    row[MC_RHOCP] = q.rho_cp;
    if (!q.is_void) {
      const double lam = q.E * q.nu / ((1 + q.nu) * (1 - 2 * q.nu)), mu = q.E / (2 * (1 + q.nu));
      row[MC_LAMBDA] = lam;
      row[MC_MU] = mu;
      row[MC_BETA] = (3 * lam + 2 * mu) * q.cte;
      row[MC_CTE] = q.cte;
    }
    row[MC_VOID] = q.is_void ? 1.0 : 0.0;
  }
  // explicit thermal bound: forward Euler is stable when R dt lambda_max <= 2;
  // Gershgorin with the per-cell mediant bound gives
  // lambda_max <= 4 max_c (k/rho_cp)_c (1/dx^2 + 1/dy^2 + 1/dz^2)_min.
  {
    std::vector<char> used(p->n_mat, 0);
    for (uint8_t m : p->mat_nat) used[m] = 1;
    double dmax = 0;
    for (int m = 0; m < p->n_mat; ++m) if (used[m]) dmax = std::max(dmax, p->mats[m].k / p->mats[m].rho_cp);
    double mx = *std::min_element(p->dx.begin(), p->dx.end()), my = *std::min_element(p->dy.begin(), p->dy.end()),
           mz = *std::min_element(p->dz.begin(), p->dz.end());
    const double lam = 4.0 * dmax * (1 / (mx * mx) + 1 / (my * my) + 1 / (mz * mz));
    if (p->R * p->dt * lam > 2.0 && !p->opts.force_dt)
      return fail(ETM_E_UNSTABLE, "thermal step R*dt exceeds the forward-Euler bound");
  }
  {
    std::vector<char> used(p->n_mat, 0);
    for (uint8_t m : p->mat_nat) used[m] = 1;
    p->has_tcr = false;
    for (int m = 0; m < p->n_mat; ++m)
      if (used[m] && p->mats[m].tcr != 0.0 && p->mats[m].sigma0 != 0.0) p->has_tcr = true;
  }
  // padded cell ids
  p->mat_pad.assign(p->ntot, 0);
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      std::memcpy(&p->mat_pad[p->nidx(0, j, k)], &p->mat_nat[(size_t(k) * ny + j) * nx], nx);
  // conducting (and temperature-dependent) cells mark their eight corner
  // nodes: every edge incident to a node lies in the node's eight cells
  p->flags.assign(p->ntot, 0);
  {
    uint8_t mbits[256] = {};
    for (int m = 0; m < p->n_mat; ++m)
      if (p->mats[m].sigma0 != 0.0) mbits[m] = uint8_t(kFlagSigma | (p->mats[m].tcr != 0.0 ? kFlagTcr : 0));
    // per cell row: the bits of each node of the row's line (a node takes
    // the cells on both sides), then or-ed into the four node lines that
    // bound the row
    std::vector<uint8_t> nb(size_t(nx) + 1);
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j) {
        const uint8_t *row = &p->mat_nat[(size_t(k) * ny + j) * nx];
        uint8_t any = 0, prev = 0;
        for (int i = 0; i < nx; ++i) {
          const uint8_t b = mbits[row[i]];
          nb[i] = uint8_t(prev | b);
          prev = b;
          any |= b;
        }
        nb[nx] = prev;
        if (!any) continue;
        for (int c = 0; c < 4; ++c) {
          uint8_t *line = &p->flags[p->nidx(0, j + (c & 1), k + (c >> 1))];
          for (int i = 0; i <= nx; ++i) line[i] |= nb[i];
        }
      }
  }
  // ports
  p->pe_key.clear(); p->pe_gs.clear(); p->pe_start.clear(); p->pw_wave.clear(); p->pw_wt.clear();
  if (src && src->n_ports > 0) {
    struct PE { int64_t key; int wave; double wt, g; };
    std::vector<PE> list;
    list.reserve(size_t(src->n_ports));
    for (int64_t q = 0; q < src->n_ports; ++q) {
      const etm_port &pt = src->ports[q];
      const int d = pt.dir;
      if (d < 0 || d > 2) return fail(ETM_E_INVAL, "port " + std::to_string(q) + ": dir must be 0..2");
      const int ni = nx + (d != 0), nj = ny + (d != 1), nk = nz + (d != 2);
      if (pt.i < 0 || pt.i >= ni || pt.j < 0 || pt.j >= nj || pt.k < 0 || pt.k >= nk)
        return fail(ETM_E_INVAL, "port " + std::to_string(q) + ": edge outside the mesh");
      if (pt.wave < 0 || pt.wave >= p->n_waves + p->n_analytic)
        return fail(ETM_E_INVAL, "port " + std::to_string(q) + ": wave out of range");
      if (!std::isfinite(pt.weight) || !(pt.g >= 0)) return fail(ETM_E_INVAL, "port " + std::to_string(q) + ": bad weight/g");
      const int *b = p->opts.em_bc;
      const bool pec = (d != 0 && ((pt.i == 0 && b[0]) || (pt.i == nx && b[1]))) ||
                       (d != 1 && ((pt.j == 0 && b[2]) || (pt.j == ny && b[3]))) ||
                       (d != 2 && ((pt.k == 0 && b[4]) || (pt.k == nz && b[5])));
      if (pec) return fail(ETM_E_INVAL, "port " + std::to_string(q) + ": edge lies on a PEC face");
      const int64_t node = p->nidx(pt.i, pt.j, pt.k);
      list.push_back({int64_t(d) * p->ntot + node, pt.wave, pt.weight, pt.g});
      p->flags[node] |= uint8_t(1 << d);
    }
    std::stable_sort(list.begin(), list.end(), [](const PE &a, const PE &b) { return a.key < b.key; });
    for (size_t q = 0; q < list.size(); ++q) {
      if (q == 0 || list[q].key != list[q - 1].key) {
        p->pe_key.push_back(list[q].key);
        p->pe_gs.push_back(0.0);
        p->pe_start.push_back(int32_t(p->pw_wave.size()));
      }
      p->pe_gs.back() += list[q].g * p->dt / (2.0 * kEps0);
      p->pw_wave.push_back(list[q].wave);
      p->pw_wt.push_back(list[q].wt * p->dt / kEps0);
    }
    p->pe_start.push_back(int32_t(p->pw_wave.size()));
  } else {
    p->pe_start.push_back(0);
  }
  // mechanical constraints
  p->fixed.assign(p->ntot, 0);
  std::vector<uint8_t> solid(p->ntot, 0);
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        if (p->mats[p->mat_nat[(size_t(k) * ny + j) * nx + i]].is_void) continue;
        for (int c = 0; c < 8; ++c) solid[p->nidx(i + (c & 1), j + ((c >> 1) & 1), k + (c >> 2))] = 1;
      }
  for (int k = 0; k <= nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i <= nx; ++i) {
        const int64_t n = p->nidx(i, j, k);
        p->fixed[n] = solid[n] ? 0 : 7;
      }
  if (p->opts.mech_mask) {
    for (int k = 0; k <= nz; ++k)
      for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i)
          p->fixed[p->nidx(i, j, k)] |= p->opts.mech_mask[(size_t(k) * (ny + 1) + j) * (nx + 1) + i] & 7;
  } else if (p->opts.mech_bc == ETM_MECH_CLAMP_ZMIN) {
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i <= nx; ++i) p->fixed[p->nidx(i, j, 0)] = 7;
  } else {
    const int ic = nearest_mid(p->dx), jc = nearest_mid(p->dy);
    p->fixed[p->nidx(ic, jc, 0)] |= 7;
    p->fixed[p->nidx(nx, jc, 0)] |= 6;
    p->fixed[p->nidx(ic, ny, 0)] |= 4;
  }
  // probes
  p->probes_dev.clear();
  for (int q = 0; q < p->opts.n_probes; ++q) {
    const int64_t *pr = p->opts.probes + 4 * q;
    const int f = int(pr[0]);
    const int64_t i = pr[1], j = pr[2], k = pr[3];
    if (f < 0 || f > 3) return fail(ETM_E_INVAL, "probe field must be 0..3");
    const int ni = nx + (f != 0), nj = ny + (f != 1), nk = nz + (f != 2);
    if (i < 0 || j < 0 || k < 0 || i >= ni || j >= nj || k >= nk) return fail(ETM_E_INVAL, "probe outside the mesh");
    p->probes_dev.push_back(f);
    p->probes_dev.push_back(p->nidx(int(i), int(j), int(k)));
  }
  p->hist_cols = 4 + p->opts.n_probes;
  if (p->opts.history_stride > 0) {
    p->hist_cap = p->opts.history_cap > 0 ? p->opts.history_cap
                                          : std::max<int64_t>(1, p->opts.n_em_steps_hint / p->opts.history_stride + 1);
  } else {
    p->hist_cap = 0;
  }
  mg_levels(p);
  // workspace layout
  size_t off = 0;
  auto take = [&](Region &r, size_t bytes) { r.off = off; r.bytes = align256(std::max<size_t>(bytes, 1)); off += r.bytes; };
  const size_t N = size_t(p->ntot);
  take(p->r_geo, p->geo.size() * 8);
  take(p->r_mtab, p->mtab.size() * 8);
  take(p->r_mat, N);
  take(p->r_flags, N);
  take(p->r_fixed, N);
  take(p->r_pkey, p->pe_key.size() * 8);
  take(p->r_pgs, p->pe_gs.size() * 8);
  take(p->r_pstart, p->pe_start.size() * 4);
  take(p->r_pwave, p->pw_wave.size() * 4);
  take(p->r_pwt, p->pw_wt.size() * 8);
  take(p->r_per, p->pe_key.size() * 8);
  take(p->r_J, p->J.size() * 8);
  take(p->r_aw, p->aw.size() * 8);
  take(p->r_Ja, size_t(p->n_analytic) * (kWaveBlock + 1) * 8);
  take(p->r_probes, p->probes_dev.size() * 8);
  for (int c = 0; c < 6; ++c) take(p->r_coef[c], N * (p->prec == ETM_PREC_FP64 ? 8 : 4));
  if (p->prec == ETM_PREC_FP64) {
    for (int b = 0; b < 3; ++b) for (int c = 0; c < 3; ++c) take(p->r_e[b][c], N * 8);
  } else {
    for (int b = 0; b < 2; ++b) for (int c = 0; c < 3; ++c) take(p->r_e[b][c], N * 4);
    for (int b = 0; b < 2; ++b) for (int c = 0; c < 3; ++c) take(p->r_h[b][c], N * 4);
    for (int c = 0; c < 3; ++c) take(p->r_K[c], N * 4);
    take(p->r_elo, 3 * align256(N * 4) / 4);
    take(p->r_theta32, N * 4);
  }
  take(p->r_theta[0], N * 8);
  take(p->r_theta[1], N * 8);
  take(p->r_psum, N * 8);
  take(p->r_part, size_t(std::max<int64_t>(p->nblocks_node, 1024) + kFinalizeRows) * kRedWidth * 8);
  take(p->r_sc, sizeof(DevScalars));
  // the mechanical solve owns its partials, scalars and temperature copy, so
  // that it can run beside the march on another stream
  take(p->r_partm, size_t(std::max<int64_t>(p->nblocks_node, 1024)) * kRedWidth * 8);
  take(p->r_scm, sizeof(DevScalars));
  take(p->r_ctl, sizeof(DevScalars));
  take(p->r_gR, sizeof(DevScalars));
  take(p->r_gF, sizeof(DevScalars));
  take(p->r_thsolve, N * 8);
  take(p->r_hist, size_t(p->hist_cap) * p->hist_cols * 8);
  for (int c = 0; c < 3; ++c) {
    take(p->r_u64[c], N * 8); take(p->r_f64[c], N * 8); take(p->r_r64[c], N * 8); take(p->r_dinv64[c], N * 8);
    take(p->r_uprev64[c], N * 8);
    take(p->r_uprev2_64[c], N * 8);
  }
  if (p->prec == ETM_PREC_FP64) {
    for (int c = 0; c < 3; ++c) { take(p->r_p64[c], N * 8); take(p->r_w64[c], N * 8); }
  } else {
    for (int c = 0; c < 3; ++c) {
      take(p->r_u32[c], N * 4); take(p->r_r32[c], N * 4); take(p->r_p32[c], N * 4);
      take(p->r_w32[c], N * 4); take(p->r_dinv32[c], N * 4); take(p->r_rhs32[c], N * 4);
    }
  }
  take(p->r_vm, N * 8);
  take(p->r_stage, N * 8);
  if (!p->mg.empty()) {
    const size_t tsz = p->prec == ETM_PREC_FP64 ? 8 : 4;
    const int nlev = int(p->mg.size());
    for (int l = 0; l < nlev; ++l) {
      MgHostLevel &L = p->mg[l];
      const size_t n = size_t(L.n);
      if (l > 0 || nlev == 1) take(L.A, size_t(kMgUpper) * 9 * n * tsz);
      take(L.Dinv, 6 * n * tsz);
      take(L.dead, n);
      take(L.xa, 3 * n * tsz);
      take(L.xb, 3 * n * tsz);
      take(L.d, 3 * n * tsz);
      if (l > 0) take(L.b, 3 * n * tsz);
    }
    const MgHostLevel &C = p->mg.back();
    const size_t dofs = 3 * size_t(C.nx + 1) * (C.ny + 1) * (C.nz + 1);
    take(p->r_mglive, dofs * 4);
    take(p->r_mgainv, dofs * dofs * tsz);
    take(p->r_mgtab, p->mg_tab.size());
    take(p->r_mgsc, (kMgMaxLevels + 2) * 8);
  }
  p->footprint = off;
  // the march kernel addresses the x, y, z components of a field from one
  // base with a fixed stride: check the layout gives one
  {
    const size_t esz = p->prec == ETM_PREC_FP64 ? 8 : 4;
    p->comp_stride = int64_t((p->r_e[0][1].off - p->r_e[0][0].off) / esz);
    for (int b = 0; b < (p->prec == ETM_PREC_FP64 ? 3 : 2); ++b)
      for (int c = 1; c < 3; ++c)
        if (p->r_e[b][c].off - p->r_e[b][c - 1].off != size_t(p->comp_stride) * esz) return fail(ETM_E_INVAL, "layout");
    if (p->prec == ETM_PREC_MIXED)
      for (int b = 0; b < 2; ++b)
        for (int c = 1; c < 3; ++c)
          if (p->r_h[b][c].off - p->r_h[b][c - 1].off != size_t(p->comp_stride) * esz) return fail(ETM_E_INVAL, "layout");
    if (p->prec == ETM_PREC_MIXED)
      for (int c = 1; c < 3; ++c)
        if (p->r_K[c].off - p->r_K[c - 1].off != size_t(p->comp_stride) * esz) return fail(ETM_E_INVAL, "layout");
    for (int c = 1; c < 6; ++c)
      if (p->r_coef[c].off - p->r_coef[c - 1].off != size_t(p->comp_stride) * esz) return fail(ETM_E_INVAL, "layout");
    // the march kernels index component c of a field as c * stride + node in
    // 32 bits (coefficients up to c = 5)
    if (p->ntot + 5 * p->comp_stride >= (int64_t(1) << 32))
      return fail(ETM_E_INVAL, "mesh too large for 32-bit node offsets (padded nodes must stay below 7.1e8)");
  }
  return ETM_OK;
}

struct FieldDesc {
  int ni, nj, nk;
};

FieldDesc field_shape(const etm_plan *p, int field) {
  switch (field) {
    case ETM_FIELD_EX: case ETM_FIELD_EX_PREV: return {p->nx, p->ny + 1, p->nz + 1};
    case ETM_FIELD_EY: case ETM_FIELD_EY_PREV: return {p->nx + 1, p->ny, p->nz + 1};
    case ETM_FIELD_EZ: case ETM_FIELD_EZ_PREV: return {p->nx + 1, p->ny + 1, p->nz};
    case ETM_FIELD_VM: return {p->nx, p->ny, p->nz};
    default: return {p->nx + 1, p->ny + 1, p->nz + 1};
  }
}

// Pointer and element type of a state field on the device.
const void *field_ptr(const etm_plan *p, int field, int *is_f32) {
  *is_f32 = 0;
  const bool mixed = p->prec == ETM_PREC_MIXED;
  switch (field) {
    case ETM_FIELD_EX: case ETM_FIELD_EY: case ETM_FIELD_EZ:
      *is_f32 = mixed;
      return p->ws + p->r_e[p->cur][field - ETM_FIELD_EX].off;
    case ETM_FIELD_EX_PREV: case ETM_FIELD_EY_PREV: case ETM_FIELD_EZ_PREV:
      if (mixed) { *is_f32 = 1; return p->ws + p->r_e[1 - p->cur][field - ETM_FIELD_EX_PREV].off; }
      return p->ws + p->r_e[(p->cur + 2) % 3][field - ETM_FIELD_EX_PREV].off;
    case ETM_FIELD_THETA: return p->ws + p->r_theta[p->th_cur].off;
    case ETM_FIELD_PSUM: return p->ws + p->r_psum.off;
    case ETM_FIELD_UX: case ETM_FIELD_UY: case ETM_FIELD_UZ: return p->ws + p->r_u64[field - ETM_FIELD_UX].off;
    case ETM_FIELD_VM: return p->ws + p->r_vm.off;
    case ETM_FIELD_FX: case ETM_FIELD_FY: case ETM_FIELD_FZ: return p->ws + p->r_f64[field - ETM_FIELD_FX].off;
  }
  return nullptr;
}

}  // namespace

namespace etm {

// Pointers of the current / previous / next e state.
static void em_pointers(const etm_plan *p, EmLaunch &L) {
  if (p->prec == ETM_PREC_FP64) {
    const int c = p->cur, prv = (c + 2) % 3, nxt = (c + 1) % 3;
    for (int d = 0; d < 3; ++d) {
      L.e0[d] = p->ws + p->r_e[c][d].off;
      L.e1[d] = p->ws + p->r_e[prv][d].off;
      L.out0[d] = p->ws + p->r_e[nxt][d].off;
      L.out1[d] = nullptr;
    }
  } else {
    const int s = p->cur, o = 1 - s;
    for (int d = 0; d < 3; ++d) {
      L.e0[d] = p->ws + p->r_e[s][d].off;
      L.e1[d] = p->ws + p->r_h[s][d].off;
      L.out0[d] = p->ws + p->r_e[o][d].off;
      L.out1[d] = p->ws + p->r_h[o][d].off;
    }
  }
}

EmLaunch em_launch_template(const etm_plan *p) {
  EmLaunch L;
  std::memset(&L, 0, sizeof(L));
  L.g = p->dev_grid();
  L.ports = p->dev_ports();
  L.precision = p->prec;
  L.kchunk = p->kchunk;
  L.c2dt2 = (kC0 * p->dt) * (kC0 * p->dt);
  L.cdt = kC0 * p->dt;
  L.jf = kEps0 / p->dt;
  L.step = p->step;
  L.theta = p->ptr<double>(p->r_theta[p->th_cur]);
  L.theta32 = p->prec == ETM_PREC_MIXED ? p->ptr<float>(p->r_theta32) : nullptr;
  L.psum = p->ptr<double>(p->r_psum);
  L.g.cs = uint32_t(p->comp_stride);
  L.coef = p->ws + p->r_coef[0].off;
  L.K = (p->prec == ETM_PREC_MIXED && p->has_tcr) ? p->ptr<float>(p->r_K[0]) : nullptr;
  L.elo = p->prec == ETM_PREC_MIXED ? p->ptr<int8_t>(p->r_elo) : nullptr;
  return L;
}

// Edge coefficients for the current temperature.  With update_k (the
// temperature changed between two EM steps of a running march) the mixed
// path also books the change of a into its leapfrog correction K; at bind and
// restore the coefficients are only (re)computed.
etm_status coef_refresh(etm_plan *p, bool update_k) {
  DevGrid g = p->dev_grid();
  g.cs = uint32_t(p->comp_stride);
  const void *th = p->prec == ETM_PREC_MIXED ? (const void *)p->ptr<float>(p->r_theta32)
                                             : (const void *)p->ptr<double>(p->r_theta[p->th_cur]);
  CoefK ck;
  ck.tcr_only = update_k ? 1 : 0;
  if (update_k && p->prec == ETM_PREC_MIXED) {
    ck.K = p->ptr<float>(p->r_K[0]);
    ck.e_cur = p->ptr<float>(p->r_e[p->cur][0]);
    ck.e_prev = p->ptr<float>(p->r_e[1 - p->cur][0]);
  }
  HIP_TRY(launch_coef(g, p->dev_ports(), p->prec, th, p->ws + p->r_coef[0].off, ck, p->stream));
  return ETM_OK;
}

// One EM step e^n -> e^{n+1}; the Joule power of e^n is added to the block
// sum when it is still pending.
// Make the device table of closed-form wave samples cover the next `ahead`
// EM steps (samples step .. step + ahead); refill it from the current step
// when it does not.  Enqueued on the plan's stream before those steps.
etm_status ensure_waves(etm_plan *p, int64_t ahead) {
  if (p->n_analytic == 0) return ETM_OK;
  if (p->a_base <= p->step && p->step + ahead <= p->a_base + kWaveBlock) return ETM_OK;
  HIP_TRY(launch_wave_sample(p->ptr<double>(p->r_aw), p->n_analytic, p->dt, p->step, p->ptr<double>(p->r_Ja),
                             p->stream));
  p->a_base = p->step;
  return ETM_OK;
}

etm_status em_one_step(etm_plan *p) {
  etm_status st;
  if ((st = ensure_waves(p, 1)) != ETM_OK) return st;
  EmLaunch L = em_launch_template(p);
  L.acc_joule = p->joule_pending ? 1 : 0;
  em_pointers(p, L);
  HIP_TRY(launch_em_step(L, p->stream));
  p->cur = p->prec == ETM_PREC_FP64 ? (p->cur + 1) % 3 : 1 - p->cur;
  p->step++;
  p->joule_pending = true;
  return ETM_OK;
}

// Index of the state buffer that held the field one step before the current
// one (after a step or a pair of steps).
static int previous_state(const etm_plan *p) {
  return p->prec == ETM_PREC_FP64 ? (p->cur + 2) % 3 : 1 - p->cur;
}

// Steps n and n + 1 as a wavefront over z-slabs (temporal blocking); the
// state afterwards is that of two em_one_step calls, bitwise.
etm_status em_two_steps(etm_plan *p) {
  etm_status st;
  if ((st = ensure_waves(p, 2)) != ETM_OK) return st;
  EmLaunch La = em_launch_template(p);
  La.acc_joule = p->joule_pending ? 1 : 0;
  em_pointers(p, La);
  const int c0 = p->cur;
  p->cur = p->prec == ETM_PREC_FP64 ? (c0 + 1) % 3 : 1 - c0;
  EmLaunch Lb = La;
  em_pointers(p, Lb);
  p->cur = p->prec == ETM_PREC_FP64 ? (c0 + 2) % 3 : c0;
  HIP_TRY(launch_em_pair_schedule(La, Lb, p->opts.em_slabs, p->stream));
  p->step += 2;
  p->joule_pending = true;
  return ETM_OK;
}

static void current_e(const etm_plan *p, const void *e[3]) {
  for (int d = 0; d < 3; ++d) e[d] = p->ws + p->r_e[p->cur][d].off;
}

// Add the Joule power of the current field to the block sum (so that the
// sum is complete whenever the host can look at it).
etm_status joule_flush(etm_plan *p) {
  if (!p->joule_pending) return ETM_OK;
  const void *e[3];
  current_e(p, e);
  DevGrid g = p->dev_grid();
  g.cs = uint32_t(p->comp_stride);
  HIP_TRY(launch_joule_flush(g, p->prec, e, p->ws + p->r_coef[0].off, p->ptr<double>(p->r_psum), kEps0 / p->dt,
                             p->stream));
  p->joule_pending = false;
  return ETM_OK;
}

etm_status diag_record(etm_plan *p, int old_cur) {
  etm_status st = joule_flush(p);
  if (st != ETM_OK) return st;
  // after the step: new state is p->cur, old is old_cur
  DiagLaunch D;
  D.g = p->dev_grid();
  D.precision = p->prec;
  D.c2dt2 = (kC0 * p->dt) * (kC0 * p->dt);
  D.dt = p->dt;
  for (int d = 0; d < 3; ++d) {
    D.e_new[d] = p->ws + p->r_e[p->cur][d].off;
    D.e_old[d] = p->ws + p->r_e[old_cur][d].off;
  }
  D.theta = p->ptr<double>(p->r_theta[p->th_cur]);
  D.psum = p->ptr<double>(p->r_psum);
  D.partials = p->ptr<double>(p->r_part);
  D.sc = p->sc();
  D.hist_row = p->ptr<double>(p->r_hist) + std::min(p->rec, std::max<int64_t>(p->hist_cap - 1, 0)) * p->hist_cols;
  D.n_probes = p->opts.n_probes;
  D.probes = p->ptr<int64_t>(p->r_probes);
  D.step = p->step;
  D.cap = p->hist_cap;
  D.rec = p->rec;
  HIP_TRY(launch_diag(D, p->stream));
  if (p->rec < p->hist_cap) p->rec++;
  return ETM_OK;
}

etm_status thermal_one(etm_plan *p) {
  ThermalLaunch T;
  T.g = p->dev_grid();
  T.precision = p->prec;
  T.acc_joule = p->joule_pending ? 1 : 0;
  T.dt = p->dt;
  T.jf = kEps0 / p->dt;
  T.R = p->R;
  current_e(p, T.e);
  T.theta_in = p->ptr<double>(p->r_theta[p->th_cur]);
  T.theta_out = p->ptr<double>(p->r_theta[1 - p->th_cur]);
  T.theta32 = p->prec == ETM_PREC_MIXED ? p->ptr<float>(p->r_theta32) : nullptr;
  T.psum = p->ptr<double>(p->r_psum);
  T.partials = p->ptr<double>(p->r_part);
  T.sc = p->sc();
  T.g.cs = uint32_t(p->comp_stride);
  T.coef = p->ws + p->r_coef[0].off;
  HIP_TRY(launch_thermal(T, p->stream));
  p->th_cur = 1 - p->th_cur;
  p->n_thermal++;
  p->joule_pending = false;
  if (p->has_tcr) return coef_refresh(p, true);
  return ETM_OK;
}

namespace {

etm_status poll_scalars(etm_plan *p) {
  HIP_TRY(hipMemcpyAsync(p->sc_host, p->sc(), sizeof(DevScalars), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return ETM_OK;
}

template <typename T>
MgDev<T> mg_dev(const etm_plan *p) {
  MgDev<T> G{};
  G.nlev = int(p->mg.size());
  G.M = p->mech_grid();
  const char *tb = p->ws + p->r_mgtab.off;
  for (int l = 0; l < G.nlev; ++l) {
    const MgHostLevel &H = p->mg[l];
    MgLevel<T> &L = G.L[l];
    L.nx = H.nx; L.ny = H.ny; L.nz = H.nz;
    L.sy = H.sy; L.sz = H.sz; L.n = H.n;
    L.A = H.A.bytes ? p->ptr<T>(H.A) : nullptr;
    L.Dinv = p->ptr<T>(H.Dinv);
    L.dead = p->ptr<uint8_t>(H.dead);
    auto v3 = [&](const Region &r) {
      V3<T> v{};
      if (r.bytes)
        for (int c = 0; c < 3; ++c) v.c[c] = p->ptr<T>(r) + c * H.n;
      return v;
    };
    L.xa = v3(H.xa); L.xb = v3(H.xb); L.d = v3(H.d); L.b = v3(H.b);
    for (int a = 0; a < 3; ++a) {
      L.ax[a].lo = reinterpret_cast<const int32_t *>(tb + H.tab[a][0]);
      L.ax[a].w = reinterpret_cast<const double *>(tb + H.tab[a][1]);
      L.ax[a].cpos = reinterpret_cast<const int32_t *>(tb + H.tab[a][2]);
    }
    L.deg = H.deg;
    for (int k = 0; k < kMgDeg; ++k) { L.c1[k] = H.c1[k]; L.c2[k] = H.c2[k]; }
  }
  G.Ainv = p->ptr<T>(p->r_mgainv);
  G.live = p->ptr<int32_t>(p->r_mglive);
  G.nlive = p->mg_nlive;
  G.lam = p->ptr<double>(p->r_mgsc);
  G.scale = G.lam + kMgMaxLevels;
  return G;
}

// Chebyshev steps for the interval [lo, hi] = [0.03, 1.1] * lambda (lambda
// the power-iteration estimate of lambda_max(Dinv A)): the three-term
// recurrence of Chebyshev acceleration of Richardson iteration,
// d_0 = r / theta, d_k = c1_k d_{k-1} + c2_k Dinv r_k.  The error polynomial
// stays below 1 in magnitude up to hi + lo and grows beyond it, so the
// smoother (and with it the V-cycle as a CG preconditioner) is safe only
// while lambda_max < 1.13 lambda.  The estimate is a lower bound; after
// kMgPowerIters steps it is within about 4 % of lambda_max on the graded
// package meshes (12 steps: 10 % low).  A smaller lo damps more of the
// middle of the spectrum for the same degree: lo = 0.03 saves 2-3 CG
// iterations per solve against 0.1.
void cheb_coefs(double lam, int deg, double *c1, double *c2) {
  for (int k = 0; k < kMgDeg; ++k) c1[k] = c2[k] = 0.0;
  if (!(lam > 0.0) || !std::isfinite(lam)) return;
  const double hi = 1.1 * lam, lo = 0.03 * lam;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  double rho = 1.0 / sigma;
  c2[0] = 1.0 / theta;
  for (int k = 1; k < deg; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    c1[k] = rn * rho;
    c2[k] = 2.0 * rn / delta;
    rho = rn;
  }
}

// Dense inverse of the coarsest operator over its live DOFs (FP64 Cholesky on
// the host).  A DOF whose pivot vanishes (its coarse basis function adds
// nothing the others do not span) is dropped and the factorisation redone.
template <typename T>
void coarse_inverse(const MgHostLevel &H, const std::vector<T> &A, const std::vector<uint8_t> &dead,
                    std::vector<int32_t> &live, std::vector<T> &inv) {
  std::vector<int64_t> cand;
  for (int k = 0; k <= H.nz; ++k)
    for (int j = 0; j <= H.ny; ++j)
      for (int i = 0; i <= H.nx; ++i) {
        const int64_t n = k * H.sz + j * H.sy + i;
        for (int c = 0; c < 3; ++c)
          if (!(dead[n] >> c & 1)) cand.push_back(n * 3 + c);
      }
  std::vector<char> drop(cand.size(), 0);
  const int64_t N = H.n;
  for (;;) {
    std::vector<int32_t> col(size_t(3 * N), -1);
    live.clear();
    for (size_t q = 0; q < cand.size(); ++q)
      if (!drop[q]) { col[cand[q]] = int32_t(live.size()); live.push_back(int32_t(cand[q])); }
    const int m = int(live.size());
    std::vector<double> D(size_t(m) * m, 0.0);
    for (int k = 0; k <= H.nz; ++k)
      for (int j = 0; j <= H.ny; ++j)
        for (int i = 0; i <= H.nx; ++i) {
          const int64_t n = k * H.sz + j * H.sy + i;
          for (int o = 0; o < 27; ++o) {
            const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
            if (i + ox < 0 || i + ox > H.nx || j + oy < 0 || j + oy > H.ny || k + oz < 0 || k + oz > H.nz) continue;
            const int64_t nb = n + ox + oy * H.sy + oz * H.sz;
            double B[9];
            if (o >= 13) {
              for (int e = 0; e < 9; ++e) B[e] = double(A[stencil_idx(o - 13, e / 3, e % 3, N, n)]);
            } else {
              for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) B[r * 3 + c] = double(A[stencil_idx(13 - o, c, r, N, nb)]);
            }
            for (int r = 0; r < 3; ++r) {
              const int rr = col[n * 3 + r];
              if (rr < 0) continue;
              for (int c = 0; c < 3; ++c) {
                const int cc = col[nb * 3 + c];
                if (cc >= 0) D[size_t(rr) * m + cc] = B[r * 3 + c];
              }
            }
          }
        }
    for (int r = 0; r < m; ++r)
      for (int c = r + 1; c < m; ++c) {
        const double a = 0.5 * (D[size_t(r) * m + c] + D[size_t(c) * m + r]);
        D[size_t(r) * m + c] = D[size_t(c) * m + r] = a;
      }
    double dmax = 0.0;
    for (int r = 0; r < m; ++r) dmax = std::max(dmax, D[size_t(r) * m + r]);
    // Cholesky D = L L^T, row by row (L in the lower triangle of D)
    int bad = -1;
    for (int r = 0; r < m && bad < 0; ++r) {
      double *Lr = &D[size_t(r) * m];
      for (int c = 0; c <= r; ++c) {
        const double *Lc = &D[size_t(c) * m];
        double sum = Lr[c];
        for (int q = 0; q < c; ++q) sum -= Lr[q] * Lc[q];
        if (c < r) {
          Lr[c] = sum / Lc[c];
        } else if (sum > 1e-13 * dmax) {
          Lr[r] = std::sqrt(sum);
        } else {
          bad = r;
        }
      }
    }
    if (bad >= 0) {
      size_t q = 0, seen = 0;
      for (; q < cand.size(); ++q)
        if (!drop[q] && int(seen++) == bad) break;
      drop[q] = 1;
      continue;
    }
    // X = L^{-1}, kept by columns: Xt[c][r] = X[r][c]
    std::vector<double> Xt(size_t(m) * m, 0.0);
    for (int c = 0; c < m; ++c) {
      double *x = &Xt[size_t(c) * m];
      x[c] = 1.0 / D[size_t(c) * m + c];
      for (int r = c + 1; r < m; ++r) {
        const double *Lr = &D[size_t(r) * m];
        double sum = 0.0;
        for (int q = c; q < r; ++q) sum += Lr[q] * x[q];
        x[r] = -sum / Lr[r];
      }
    }
    // D^{-1} = X^T X: entry (r, c) = sum_{q >= max(r,c)} X[q][r] X[q][c]
    inv.assign(size_t(m) * m, T(0));
    for (int r = 0; r < m; ++r)
      for (int c = r; c < m; ++c) {
        const double *xr = &Xt[size_t(r) * m], *xc = &Xt[size_t(c) * m];
        double sum = 0.0;
        for (int q = c; q < m; ++q) sum += xr[q] * xc[q];
        inv[size_t(r) * m + c] = inv[size_t(c) * m + r] = T(sum);
      }
    return;
  }
}

constexpr int kMgPowerIters = 32;  // power steps per level for the Chebyshev interval (cheb_coefs)

template <typename T>
etm_status mg_setup(etm_plan *p) {
  MgDev<T> G = mg_dev<T>(p);
  HIP_TRY(launch_mg_build<T>(G, p->stream));
  double *part = p->ptr<double>(p->r_partm);
  for (int l = 0; l + 1 < G.nlev; ++l) HIP_TRY(launch_mg_power<T>(G, l, kMgPowerIters, part, p->stream));
  const MgHostLevel &H = p->mg.back();
  std::vector<double> lam(kMgMaxLevels, 0.0);
  std::vector<T> A(size_t(kMgUpper) * 9 * H.n);
  std::vector<uint8_t> dead(H.n);
  HIP_TRY(hipMemcpyAsync(lam.data(), G.lam, kMgMaxLevels * 8, hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipMemcpyAsync(A.data(), p->ptr<T>(H.A), A.size() * sizeof(T), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipMemcpyAsync(dead.data(), p->ptr<uint8_t>(H.dead), dead.size(), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  std::vector<int32_t> live;
  std::vector<T> inv;
  coarse_inverse<T>(H, A, dead, live, inv);
  if (!live.empty()) {
    HIP_TRY(hipMemcpyAsync(p->ptr<int32_t>(p->r_mglive), live.data(), live.size() * 4, hipMemcpyHostToDevice,
                           p->stream));
    HIP_TRY(hipMemcpyAsync(p->ptr<T>(p->r_mgainv), inv.data(), inv.size() * sizeof(T), hipMemcpyHostToDevice,
                           p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
  }
  p->mg_nlive = int(live.size());
  for (int l = 0; l + 1 < int(p->mg.size()); ++l) cheb_coefs(lam[l], p->mg[l].deg, p->mg[l].c1, p->mg[l].c2);
  p->mg_ready = true;
  return ETM_OK;
}

}  // namespace

namespace {

// One enqueue group of a solve: n_pass passes of iters[q] inner CG
// iterations each, then von Mises, the copy of the control block to pinned
// host memory and the completion event.  A pass is
//   [restart phase] (re)start an inner CG -- only when the device's last
//       FP64 check asked for one: mixed, K c = r64 in FP32 from c = 0 (the
//       iterative-refinement correction); FP64, CG on K u = f from the
//       current u;
//   iters[q] inner iterations (no-ops once the inner CG has finished);
//   [finish phase] once the inner CG has finished: mixed, u64 += c; the FP64
//       residual check that decides the solve or asks for a restart.
// An inner CG still running at the end of a pass goes on in the next one.
// Every kernel is a no-op once the device has decided the solve.
template <typename T>
etm_status enqueue_passes(etm_plan *p, int n_pass, const int *iters) {
  const MechGrid M = p->mech_grid();
  const int64_t N = p->ntot;
  const bool mixed = sizeof(T) == 4;
  const bool use_mg = !p->mg.empty();
  double *u64[3], *f64[3], *r64[3];
  for (int c = 0; c < 3; ++c) {
    u64[c] = p->ptr<double>(p->r_u64[c]); f64[c] = p->ptr<double>(p->r_f64[c]); r64[c] = p->ptr<double>(p->r_r64[c]);
  }
  const double *cf64[3] = {f64[0], f64[1], f64[2]};
  const double *cu64[3] = {u64[0], u64[1], u64[2]};
  DevScalars *scm = p->scm(), *ctl = p->ctl(), *gR = p->ptr<DevScalars>(p->r_gR), *gF = p->ptr<DevScalars>(p->r_gF);
  double *part = p->ptr<double>(p->r_partm);
  CgVecs<T> v;
  const T *rhs[3];
  for (int c = 0; c < 3; ++c) {
    if (mixed) {
      v.u[c] = (T *)p->ptr<float>(p->r_u32[c]); v.r[c] = (T *)p->ptr<float>(p->r_r32[c]);
      v.p[c] = (T *)p->ptr<float>(p->r_p32[c]); v.w[c] = (T *)p->ptr<float>(p->r_w32[c]);
      v.dinv[c] = (const T *)p->ptr<float>(p->r_dinv32[c]);
      rhs[c] = (const T *)p->ptr<float>(p->r_rhs32[c]);
    } else {
      v.u[c] = (T *)u64[c]; v.r[c] = (T *)r64[c];
      v.p[c] = (T *)p->ptr<double>(p->r_p64[c]); v.w[c] = (T *)p->ptr<double>(p->r_w64[c]);
      v.dinv[c] = (const T *)p->ptr<double>(p->r_dinv64[c]);
      rhs[c] = (const T *)f64[c];
    }
  }
  const MgDev<T> G = use_mg ? mg_dev<T>(p) : MgDev<T>{};
  for (int q = 0; q < n_pass; ++q) {
    HIP_TRY(launch_solve_gates(ctl, scm, gR, gF, p->stream));
    if (mixed)
      for (int c = 0; c < 3; ++c) {
        HIP_TRY(launch_vec_cast(r64[c], 0, (void *)rhs[c], 1, N, gR, p->stream));
        HIP_TRY(launch_vec_zero32((float *)v.u[c], N, gR, p->stream));
      }
    if (use_mg) HIP_TRY(launch_cgmg_setup<T>(G, v, rhs, part, scm, gR, p->stream));
    else HIP_TRY(launch_cg_setup<T>(M, v, rhs, part, scm, gR, p->stream));
    for (int it = 0; it < iters[q]; ++it) {
      if (use_mg) HIP_TRY(launch_cgmg_iteration<T>(G, v, part, scm, p->stream));
      else HIP_TRY(launch_cg_iteration<T>(M, v, part, scm, p->stream));
    }
    HIP_TRY(launch_solve_gates(ctl, scm, gR, gF, p->stream));
    if (mixed)
      for (int c = 0; c < 3; ++c) HIP_TRY(launch_vec_axpy64(u64[c], (const float *)v.u[c], N, gF, p->stream));
    HIP_TRY(launch_residual_check(M, cf64, cu64, r64, part, ctl, scm, gF, p->stream));
  }
  HIP_TRY(launch_von_mises(M, p->ptr<double>(p->r_thsolve), cu64, p->ptr<double>(p->r_vm), p->stream));
  HIP_TRY(hipMemcpyAsync(p->ctl_host, ctl, sizeof(DevScalars), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipEventRecord(p->ev_solve, p->stream));
  return ETM_OK;
}

etm_status enqueue_passes_any(etm_plan *p, int n_pass, const int *iters) {
  return p->prec == ETM_PREC_FP64 ? enqueue_passes<double>(p, n_pass, iters) : enqueue_passes<float>(p, n_pass, iters);
}

}  // namespace

// Enqueue a mechanical solve of Eq. (8) for the current temperature and the
// von Mises stress of Eq. (9) on the plan's stream; returns without waiting
// (apart from the first solve of a plan, which builds the multigrid
// hierarchy).  The passes enqueued follow the previous solve's iteration
// counts; solve_settle adds more if the device has not decided the solve.
etm_status mech_solve_impl(etm_plan *p) {
  etm_status st;
  if ((st = solve_settle(p)) != ETM_OK) return st;  // the previous solve owns u and the scalars
  Range r("etm:mech_solve_enqueue");
  const MechGrid M = p->mech_grid();
  const int64_t N = p->ntot;
  double *u64[3], *f64[3], *r64[3], *dinv64[3];
  for (int c = 0; c < 3; ++c) {
    u64[c] = p->ptr<double>(p->r_u64[c]); f64[c] = p->ptr<double>(p->r_f64[c]);
    r64[c] = p->ptr<double>(p->r_r64[c]); dinv64[c] = p->ptr<double>(p->r_dinv64[c]);
  }
  const bool use_mg = !p->mg.empty();
  if (use_mg && !p->mg_ready) {
    st = p->prec == ETM_PREC_FP64 ? mg_setup<double>(p) : mg_setup<float>(p);
    if (st != ETM_OK) return st;
  }
  if (!p->dinv_ready) {
    HIP_TRY(launch_mech_diag(M, dinv64, p->stream));
    if (p->prec == ETM_PREC_MIXED)
      for (int c = 0; c < 3; ++c)
        HIP_TRY(launch_vec_cast(dinv64[c], 0, p->ptr<float>(p->r_dinv32[c]), 1, N, nullptr, p->stream));
    p->dinv_ready = true;
  }
  // Initial guess: the last solution, extrapolated in time through the ones
  // before it (a Lagrange polynomial in the thermal-step counts of up to the
  // last three solves: quadratic once three exist).  Only the starting point
  // of CG changes; convergence is still judged on the FP64 residual of the
  // new system.
  double *uprev[3], *uprev2[3];
  for (int c = 0; c < 3; ++c) {
    uprev[c] = p->ptr<double>(p->r_uprev64[c]);
    uprev2[c] = p->ptr<double>(p->r_uprev2_64[c]);
  }
  const int64_t tn = p->n_thermal;
  if (p->sol_t[0] >= 0 && tn != p->sol_t[0]) {
    const double x = double(tn), t0 = double(p->sol_t[0]), t1 = double(p->sol_t[1]), t2 = double(p->sol_t[2]);
    double w[3] = {1.0, 0.0, 0.0};
    if (p->sol_t[2] >= 0 && t2 < t1 && t1 < t0) {
      w[0] = (x - t1) * (x - t2) / ((t0 - t1) * (t0 - t2));
      w[1] = (x - t0) * (x - t2) / ((t1 - t0) * (t1 - t2));
      w[2] = (x - t0) * (x - t1) / ((t2 - t0) * (t2 - t1));
    } else if (p->sol_t[1] >= 0 && t1 < t0) {
      w[0] = (x - t1) / (t0 - t1);
      w[1] = (x - t0) / (t1 - t0);
    }
    HIP_TRY(launch_extrapolate(u64, uprev, uprev2, w, N, p->stream));
    p->sol_t[2] = p->sol_t[1];
    p->sol_t[1] = p->sol_t[0];
    p->sol_t[0] = tn;
  } else if (p->sol_t[0] < 0) {
    p->sol_t[0] = tn;
  }
  // the solve's own copy of the temperature (von Mises reads it at the end)
  const double *theta = p->ptr<double>(p->r_theta[p->th_cur]);
  HIP_TRY(hipMemcpyAsync(p->ptr<double>(p->r_thsolve), theta, size_t(N) * 8, hipMemcpyDeviceToDevice, p->stream));
  HIP_TRY(launch_mech_rhs(M, theta, f64, p->ptr<double>(p->r_partm), p->ctl(), p->opts.cg_rtol, p->stream));
  HIP_TRY(hipEventRecord(p->ev_copy, p->stream));  // the temperature is no longer read after this
  const double inner_rtol = 1e-5;
  HIP_TRY(launch_solve_init(p->ctl(), p->scm(), p->opts.cg_maxit, inner_rtol * inner_rtol,
                            p->prec == ETM_PREC_MIXED ? 1 : 0, u64, N, p->stream));
  const double *cf64[3] = {f64[0], f64[1], f64[2]};
  const double *cu64[3] = {u64[0], u64[1], u64[2]};
  DevScalars *gR = p->ptr<DevScalars>(p->r_gR), *gF = p->ptr<DevScalars>(p->r_gF);
  HIP_TRY(launch_solve_gates(p->ctl(), p->scm(), gR, gF, p->stream));
  HIP_TRY(launch_residual_check(M, cf64, cu64, r64, p->ptr<double>(p->r_partm), p->ctl(), p->scm(), gF,
                                p->stream));
  // passes as the last solve needed them (a first solve: a few of a typical length)
  int iters[kMaxPasses];
  int n_pass = p->pass_plan_n;
  if (n_pass <= 0) {
    n_pass = p->prec == ETM_PREC_MIXED ? 3 : 1;
    for (int q = 0; q < n_pass; ++q) iters[q] = p->prec == ETM_PREC_MIXED ? 16 : 48;
  } else {
    for (int q = 0; q < n_pass; ++q) iters[q] = p->pass_plan[q];
  }
  if ((st = enqueue_passes_any(p, n_pass, iters)) != ETM_OK) return st;
  p->solve_enqueued = 0;
  p->solve_rounds = 0;
  for (int q = 0; q < n_pass; ++q) p->solve_enqueued += iters[q];
  p->solve_pending = true;
  p->n_solves++;
  return ETM_OK;
}

// Wait for the pending solve (through its event and the pinned copy of the
// control block), adding passes while the device has not decided it;
// record its counts and plan the next solve's passes.  A solve that gave up
// sets ETM_E_NOCONV, reported by etm_sync; only HIP errors are returned.
etm_status solve_settle(etm_plan *p) {
  if (!p->solve_pending) return ETM_OK;
  Range r("etm:mech_solve_settle");
  for (;;) {
    HIP_TRY(hipEventSynchronize(p->ev_solve));
    const DevScalars c = *p->ctl_host;
    if (c.done == kSolveRunning) {
      // one more pass, on the plan's stream after what was enqueued.  Its
      // length grows with the round trips already taken (8, 16, 32, ...
      // iterations up to the work enqueued so far): a solve that is just
      // short of its plan pays few skipped iterations, a long one few round
      // trips.
      HIP_TRY(hipStreamWaitEvent(p->stream, p->ev_solve, 0));
      const int add = std::min(std::max(8, p->solve_enqueued), 8 << std::min(p->solve_rounds, 8));
      etm_status st = enqueue_passes_any(p, 1, &add);
      if (st != ETM_OK) {
        p->solve_pending = false;
        return st;
      }
      p->solve_enqueued += add;
      p->solve_rounds += 1;
      continue;
    }
    p->solve_pending = false;
    p->cg_iters = c.iters;
    p->cg_outer = c.outer;
    p->cg_total += c.iters;
    p->cg_relres = c.fnorm2 > 0 ? std::sqrt(c.rr / c.fnorm2) : 0.0;
    // the next solve's passes: each one iteration (and 1/16) longer than
    // this solve's.  An iteration enqueued but not needed still launches its
    // kernels, which exit at once (about 0.3 ms per iteration on a 4M-node
    // mesh); one missing ends the pass early and costs a restart.
    int n = 0;
    for (int q = 0; q + 1 < c.outer && q < kMaxPasses; ++q) {
      if (c.pass_iters[q] <= 0) break;
      p->pass_plan[n++] = c.pass_iters[q] + c.pass_iters[q] / 16 + 1;
    }
    if (c.done == kSolveConverged && n > 0) p->pass_plan_n = n;
    if (c.done != kSolveConverged && p->host_status == ETM_OK) {
      p->host_status = ETM_E_NOCONV;
      p->host_msg = "mechanical CG did not converge: relres " + std::to_string(p->cg_relres) + " after " +
                    std::to_string(c.iters) + " iterations";
    }
    return ETM_OK;
  }
}

}  // namespace etm

// =============================== C ABI ======================================
extern "C" {

etm_status etm_opts_default(etm_opts *o) {
  if (!o) return fail(ETM_E_INVAL, "null opts");
  std::memset(o, 0, sizeof(*o));
  o->dt = 0.0;
  o->cfl = 0.9;
  o->precision = ETM_PREC_FP64;
  o->em_per_thermal = 1;
  o->mech_every_thermal = 0;
  o->mech_bc = ETM_MECH_KINEMATIC;
  o->cg_maxit = 200000;
  o->cg_rtol = 1e-8;
  o->mech_precond = ETM_PRECOND_MG;
  o->mg_coarse_dofs = 800;
  o->mg_degree[0] = 3;
  o->mg_degree[1] = 2;
  o->mech_overlap = 1;
  return ETM_OK;
}

etm_status etm_cfl_dt(const etm_mesh *mesh, double cfl, double *dt) {
  if (!mesh || !dt || !mesh->dx || !mesh->dy || !mesh->dz || mesh->nx < 1 || mesh->ny < 1 || mesh->nz < 1)
    return fail(ETM_E_INVAL, "bad mesh");
  if (!(cfl > 0)) return fail(ETM_E_INVAL, "cfl must be > 0");
  *dt = cfl * cfl_limit(mesh->dx, mesh->nx, mesh->dy, mesh->ny, mesh->dz, mesh->nz);
  return ETM_OK;
}

etm_status etm_plan_create(const etm_mesh *mesh, const etm_material *mats, int32_t n_mat, const etm_source *src,
                           const etm_opts *opts, etm_plan **out) {
  if (!out) return fail(ETM_E_INVAL, "null out");
  *out = nullptr;
  etm_plan *p = nullptr;
  try {
    p = new etm_plan();
    etm_status st = validate_and_copy(p, mesh, mats, n_mat, src, opts);
    if (st == ETM_OK) st = derive(p, src);
    if (st != ETM_OK) { delete p; return st; }
    p->opts.mech_mask = nullptr;  // copied into p->fixed
    p->opts.probes = nullptr;     // copied into probes_dev
  } catch (const std::bad_alloc &) {
    delete p;
    return fail(ETM_E_NOMEM, "host allocation failed");
  } catch (...) {
    delete p;
    return fail(ETM_E_INVAL, "unexpected error in plan creation");
  }
  *out = p;
  return ETM_OK;
}

etm_status etm_plan_footprint(const etm_plan *p, size_t *bytes) {
  if (!p || !bytes) return fail(ETM_E_INVAL, "null argument");
  *bytes = p->footprint;
  return ETM_OK;
}

etm_status etm_plan_dt(const etm_plan *p, double *dt) {
  if (!p || !dt) return fail(ETM_E_INVAL, "null argument");
  *dt = p->dt;
  return ETM_OK;
}

etm_status etm_plan_dofs(const etm_plan *p, int64_t *em, int64_t *thermal, int64_t *mech) {
  if (!p) return fail(ETM_E_INVAL, "null plan");
  const int64_t nx = p->nx, ny = p->ny, nz = p->nz;
  const int64_t nodes = (nx + 1) * (ny + 1) * (nz + 1);
  if (em) *em = nx * (ny + 1) * (nz + 1) + (nx + 1) * ny * (nz + 1) + (nx + 1) * (ny + 1) * nz;
  if (thermal) *thermal = nodes;
  if (mech) *mech = 3 * nodes;
  return ETM_OK;
}

etm_status etm_plan_bind(etm_plan *p, void *ws, size_t bytes, void *stream) {
  if (!p || !ws) return fail(ETM_E_INVAL, "null plan or workspace");
  if (bytes < p->footprint) return fail(ETM_E_NOMEM, "workspace smaller than the footprint");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(ETM_E_INVAL, "workspace must be 256-byte aligned");
  p->ws = static_cast<char *>(ws);
  p->stream = static_cast<hipStream_t>(stream);
  if (p->solve_pending) {  // a solve of the previous binding still writes its control block
    HIP_TRY(hipEventSynchronize(p->ev_solve));
    p->solve_pending = false;
  }
  if (!p->mstream) HIP_TRY(hipStreamCreateWithFlags(&p->mstream, hipStreamNonBlocking));
  if (!p->ev_main) HIP_TRY(hipEventCreateWithFlags(&p->ev_main, hipEventDisableTiming));
  if (!p->ev_copy) HIP_TRY(hipEventCreateWithFlags(&p->ev_copy, hipEventDisableTiming));
  if (!p->ev_solve) HIP_TRY(hipEventCreateWithFlags(&p->ev_solve, hipEventDisableTiming));
  if (!p->sc_host) HIP_TRY(hipHostMalloc((void **)&p->sc_host, sizeof(DevScalars), hipHostMallocDefault));
  if (!p->ctl_host) HIP_TRY(hipHostMalloc((void **)&p->ctl_host, sizeof(DevScalars), hipHostMallocDefault));
  std::memset(p->sc_host, 0, sizeof(DevScalars));
  std::memset(p->ctl_host, 0, sizeof(DevScalars));
  HIP_TRY(launch_fill(p->ws, int64_t(p->footprint), p->stream));
  auto up = [&](const Region &r, const void *src, size_t n) -> etm_status {
    if (n) HIP_TRY(hipMemcpyAsync(p->ws + r.off, src, n, hipMemcpyHostToDevice, p->stream));
    return ETM_OK;
  };
  etm_status st;
  if ((st = up(p->r_geo, p->geo.data(), p->geo.size() * 8)) ||
      (st = up(p->r_mtab, p->mtab.data(), p->mtab.size() * 8)) ||
      (st = up(p->r_mat, p->mat_pad.data(), p->mat_pad.size())) ||
      (st = up(p->r_flags, p->flags.data(), p->flags.size())) ||
      (st = up(p->r_fixed, p->fixed.data(), p->fixed.size())) ||
      (st = up(p->r_pkey, p->pe_key.data(), p->pe_key.size() * 8)) ||
      (st = up(p->r_pgs, p->pe_gs.data(), p->pe_gs.size() * 8)) ||
      (st = up(p->r_pstart, p->pe_start.data(), p->pe_start.size() * 4)) ||
      (st = up(p->r_pwave, p->pw_wave.data(), p->pw_wave.size() * 4)) ||
      (st = up(p->r_pwt, p->pw_wt.data(), p->pw_wt.size() * 8)) ||
      (st = up(p->r_J, p->J.data(), p->J.size() * 8)) ||
      (st = up(p->r_aw, p->aw.data(), p->aw.size() * 8)) ||
      (st = up(p->r_probes, p->probes_dev.data(), p->probes_dev.size() * 8)) ||
      (st = up(p->r_mgtab, p->mg_tab.data(), p->mg_tab.size())))
    return st;
  p->bound = true;
  p->a_base = kNoWaveBlock;
  if ((st = coef_refresh(p, false)) != ETM_OK) return st;
  HIP_TRY(hipStreamSynchronize(p->stream));
  p->step = 0; p->cur = 0; p->th_cur = 0; p->rec = 0; p->n_thermal = 0;
  p->n_solves = 0; p->cg_iters = 0; p->cg_outer = 0; p->cg_total = 0; p->cg_relres = 0;
  p->sol_t[0] = p->sol_t[1] = p->sol_t[2] = -1;
  p->host_status = ETM_OK;
  p->host_msg.clear();
  p->dinv_ready = false;
  p->mg_ready = false;
  p->joule_pending = false;
  p->pass_plan_n = 0;
  return ETM_OK;
}

etm_status etm_advance(etm_plan *p, int64_t n) {
  if (!p) return fail(ETM_E_INVAL, "null plan");
  if (!p->bound) return fail(ETM_E_STATE, "plan is not bound");
  if (n < 0) return fail(ETM_E_INVAL, "negative step count");
  Range r_call("etm_advance");
  etm_status st;
  const int64_t hs = p->opts.history_stride;
  auto history_due = [&](int64_t s) { return hs > 0 && s % hs == 0; };
  int64_t q = 0;
  // One EM step, or a pair when enabled, at most `limit` steps, and nothing
  // is due after the first of the two.
  auto march = [&](int64_t limit) -> etm_status {
    Range r("etm:em_step");
    const bool pair = p->opts.em_slabs >= 2 && limit >= 2 && (p->step + 1) % p->R != 0 && !history_due(p->step + 1);
    const etm_status s2 = pair ? em_two_steps(p) : em_one_step(p);
    if (s2 == ETM_OK) q += pair ? 2 : 1;
    return s2;
  };
  while (q < n) {
    if ((st = march(n - q)) != ETM_OK) return st;
    const int old = previous_state(p);
    bool hist = history_due(p->step);
    if (p->step % p->R == 0) {
      {
        Range r("etm:thermal_step");
        if ((st = thermal_one(p)) != ETM_OK) return st;
      }
      if (p->opts.mech_every_thermal > 0 && p->n_thermal % p->opts.mech_every_thermal == 0) {
        if (p->opts.mech_overlap) {
          // The record of this step first (it does not read the mechanics,
          // and the steps enqueued next replace the state it reads).
          if (hist && (st = diag_record(p, old)) != ETM_OK) return st;
          hist = false;
          HIP_TRY(hipEventRecord(p->ev_main, p->stream));
          // Enqueue the EM steps that need nothing else before them: short of
          // the next thermal step and the next history record, within this
          // call.  They read the edge coefficients and the fields, never the
          // temperature buffer the solve reads or anything the solve writes.
          for (;;) {
            const int64_t s_th = (p->step / p->R + 1) * p->R;
            const int64_t s_h = hs > 0 ? (p->step / hs + 1) * hs : INT64_MAX;
            const int64_t allowed = std::min<int64_t>(n - q, std::min(s_th, s_h) - p->step - 1);
            if (allowed <= 0) break;
            if ((st = march(allowed)) != ETM_OK) return st;
          }
          // The solve on the side stream, after the thermal step.  It owns
          // its vectors, scalars and a copy of the temperature, so the
          // plan's stream waits only until that copy is taken (the next
          // thermal step may not overwrite the temperature before).
          HIP_TRY(hipStreamWaitEvent(p->mstream, p->ev_main, 0));
          hipStream_t main_stream = p->stream;
          p->stream = p->mstream;
          st = mech_solve_impl(p);
          p->stream = main_stream;
          HIP_TRY(hipStreamWaitEvent(p->stream, p->ev_copy, 0));
        } else {
          st = mech_solve_impl(p);
        }
        if (st != ETM_OK && st != ETM_E_NOCONV) return st;
      }
    }
    if (hist && (st = diag_record(p, old)) != ETM_OK) return st;
  }
  return joule_flush(p);
}

etm_status etm_mech_solve(etm_plan *p) {
  if (!p) return fail(ETM_E_INVAL, "null plan");
  if (!p->bound) return fail(ETM_E_STATE, "plan is not bound");
  return mech_solve_impl(p);
}

etm_status etm_sync(etm_plan *p, etm_run_info *info) {
  if (!p) return fail(ETM_E_INVAL, "null plan");
  if (!p->bound) return fail(ETM_E_STATE, "plan is not bound");
  etm_status st = solve_settle(p);
  if (st == ETM_OK) st = poll_scalars(p);
  if (st != ETM_OK) return st;
  const DevScalars &s = *p->sc_host;
  if (info) {
    info->step = p->step;
    info->status = p->host_status != ETM_OK ? p->host_status : s.status;
    info->cg_iters = p->cg_iters;
    info->cg_outer = p->cg_outer;
    info->n_solves = p->n_solves;
    info->cg_relres = p->cg_relres;
    info->theta_max = s.theta_max;
    info->ejoule = s.ejoule;
    info->n_records = p->rec;
    info->cg_iters_total = p->cg_total;
    info->mg_levels = p->mg_ready ? int32_t(p->mg.size()) : 0;
    info->reserved = 0;
  }
  if (s.status != ETM_OK) return fail(s.status, "non-finite field detected on the device");
  if (p->host_status != ETM_OK) return fail(p->host_status, p->host_msg);
  return ETM_OK;
}

etm_status etm_read(const etm_plan *p, int32_t field, void *dst, size_t bytes, int32_t dst_is_device) {
  if (!p || !dst) return fail(ETM_E_INVAL, "null argument");
  if (!p->bound) return fail(ETM_E_STATE, "plan is not bound");
  {  // a pending solve writes u, von Mises and f: let it finish (its outcome is reported by etm_sync)
    etm_status s0 = solve_settle(const_cast<etm_plan *>(p));
    if (s0 != ETM_OK) return s0;
  }
  if (field < ETM_FIELD_EX || field > ETM_FIELD_FZ) return fail(ETM_E_INVAL, "unknown field");
  const FieldDesc fd = field_shape(p, field);
  const size_t need = size_t(fd.ni) * fd.nj * fd.nk * 8;
  if (bytes != need) return fail(ETM_E_INVAL, "dst size " + std::to_string(bytes) + " != " + std::to_string(need));
  int f32 = 0;
  const void *src = field_ptr(p, field, &f32);
  double *stage = p->ptr<double>(p->r_stage);
  HIP_TRY(launch_pack(src, f32, p->sy, p->sz, fd.ni, fd.nj, fd.nk, dst_is_device ? (double *)dst : stage, p->stream));
  if (!dst_is_device) {
    HIP_TRY(hipMemcpyAsync(dst, stage, need, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
  }
  return ETM_OK;
}

etm_status etm_write(etm_plan *p, int32_t field, const void *src, size_t bytes, int32_t src_is_device) {
  if (!p || !src) return fail(ETM_E_INVAL, "null argument");
  if (!p->bound) return fail(ETM_E_STATE, "plan is not bound");
  {
    etm_status s0 = solve_settle(p);
    if (s0 != ETM_OK) return s0;
  }
  if (field < ETM_FIELD_EX || field > ETM_FIELD_UZ || field == ETM_FIELD_VM)
    return fail(ETM_E_INVAL, "field is not writable");
  if (p->prec == ETM_PREC_MIXED && field >= ETM_FIELD_EX && field <= ETM_FIELD_EZ_PREV)
    return fail(ETM_E_INVAL, "the mixed path keeps (e, h) as its state: its e fields are set by etm_restore only");
  const FieldDesc fd = field_shape(p, field);
  const size_t need = size_t(fd.ni) * fd.nj * fd.nk * 8;
  if (bytes != need) return fail(ETM_E_INVAL, "src size mismatch");
  double *stage = p->ptr<double>(p->r_stage);
  const void *from = src;
  if (src_is_device) {
    HIP_TRY(hipMemcpyAsync(stage, from, need, hipMemcpyDeviceToDevice, p->stream));
  } else {
    HIP_TRY(hipMemcpyAsync(stage, from, need, hipMemcpyHostToDevice, p->stream));
  }
  int f32 = 0;
  void *dstp = const_cast<void *>(field_ptr(p, field, &f32));
  HIP_TRY(launch_unpack(stage, fd.ni, fd.nj, fd.nk, dstp, f32, p->sy, p->sz, p->stream));
  if (field == ETM_FIELD_THETA && p->prec == ETM_PREC_MIXED)
    HIP_TRY(launch_unpack(stage, fd.ni, fd.nj, fd.nk, p->ptr<float>(p->r_theta32), 1, p->sy, p->sz, p->stream));
  if (field == ETM_FIELD_THETA && p->has_tcr) {
    etm_status st = coef_refresh(p, true);
    if (st != ETM_OK) return st;
  }
  if (field >= ETM_FIELD_UX && field <= ETM_FIELD_UZ) {
    // a fixed DOF carries no displacement: clear what was written there
    // (the solves would otherwise take it as a prescribed displacement)
    HIP_TRY(launch_mask_fixed(p->mech_grid(), field - ETM_FIELD_UX, static_cast<double *>(dstp), p->stream));
    // the next solve's starting point comes from this displacement
    HIP_TRY(hipMemcpyAsync(p->ptr<double>(p->r_uprev64[field - ETM_FIELD_UX]), dstp, size_t(p->ntot) * 8,
                           hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(hipMemcpyAsync(p->ptr<double>(p->r_uprev2_64[field - ETM_FIELD_UX]), dstp, size_t(p->ntot) * 8,
                           hipMemcpyDeviceToDevice, p->stream));
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  return ETM_OK;
}

etm_status etm_read_history(const etm_plan *p, double *dst, size_t bytes, int64_t *n_rows) {
  if (!p || (!dst && bytes)) return fail(ETM_E_INVAL, "null argument");
  if (!p->bound) return fail(ETM_E_STATE, "plan is not bound");
  const size_t row = size_t(p->hist_cols) * 8;
  const int64_t rows = std::min<int64_t>(p->rec, int64_t(bytes / row));
  if (rows > 0) {
    HIP_TRY(hipMemcpyAsync(dst, p->ptr<double>(p->r_hist), size_t(rows) * row, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
  }
  if (n_rows) *n_rows = rows;
  return ETM_OK;
}

extern "C++" {  // helpers of the checkpoint entry points (C++ linkage)
namespace {
struct CkptHeader {
  uint64_t magic;
  int64_t step, rec, n_thermal, cg_total;
  int32_t cur, th_cur, prec, n_solves;
  int64_t ntot;
  int64_t sol_t[3];
};
constexpr uint64_t kMagic = 0x45544d434b505431ull;

std::vector<const Region *> state_regions(const etm_plan *p) {
  std::vector<const Region *> r;
  for (int b = 0; b < 3; ++b) for (int c = 0; c < 3; ++c) if (p->r_e[b][c].bytes) r.push_back(&p->r_e[b][c]);
  if (p->prec == ETM_PREC_MIXED) {
    for (int b = 0; b < 2; ++b) for (int c = 0; c < 3; ++c) r.push_back(&p->r_h[b][c]);
    for (int c = 0; c < 3; ++c) r.push_back(&p->r_K[c]);
    r.push_back(&p->r_elo);
    r.push_back(&p->r_theta32);
  }
  r.push_back(&p->r_theta[0]);
  r.push_back(&p->r_theta[1]);
  r.push_back(&p->r_psum);
  r.push_back(&p->r_sc);
  r.push_back(&p->r_hist);
  for (int c = 0; c < 3; ++c) r.push_back(&p->r_u64[c]);
  for (int c = 0; c < 3; ++c) r.push_back(&p->r_uprev64[c]);
  for (int c = 0; c < 3; ++c) r.push_back(&p->r_uprev2_64[c]);
  return r;
}
}  // namespace
}  // extern "C++"

etm_status etm_checkpoint_size(const etm_plan *p, size_t *bytes) {
  if (!p || !bytes) return fail(ETM_E_INVAL, "null argument");
  size_t s = sizeof(CkptHeader);
  for (const Region *r : state_regions(p)) s += r->bytes;
  *bytes = s;
  return ETM_OK;
}

etm_status etm_checkpoint(const etm_plan *p, void *dst, size_t bytes) {
  if (!p || !dst) return fail(ETM_E_INVAL, "null argument");
  if (!p->bound) return fail(ETM_E_STATE, "plan is not bound");
  {
    etm_status s0 = solve_settle(const_cast<etm_plan *>(p));
    if (s0 != ETM_OK) return s0;
  }
  size_t need = 0;
  etm_checkpoint_size(p, &need);
  if (bytes < need) return fail(ETM_E_NOMEM, "checkpoint buffer too small");
  CkptHeader h{kMagic, p->step, p->rec, p->n_thermal, p->cg_total, p->cur, p->th_cur, p->prec, p->n_solves, p->ntot,
               {p->sol_t[0], p->sol_t[1], p->sol_t[2]}};
  char *o = static_cast<char *>(dst);
  std::memcpy(o, &h, sizeof(h));
  o += sizeof(h);
  for (const Region *r : state_regions(p)) {
    HIP_TRY(hipMemcpyAsync(o, p->ws + r->off, r->bytes, hipMemcpyDeviceToHost, p->stream));
    o += r->bytes;
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  return ETM_OK;
}

etm_status etm_restore(etm_plan *p, const void *src, size_t bytes) {
  if (!p || !src) return fail(ETM_E_INVAL, "null argument");
  if (!p->bound) return fail(ETM_E_STATE, "plan is not bound");
  {
    etm_status s0 = solve_settle(p);
    if (s0 != ETM_OK) return s0;
  }
  size_t need = 0;
  etm_checkpoint_size(p, &need);
  if (bytes < need) return fail(ETM_E_INVAL, "checkpoint too small");
  CkptHeader h;
  std::memcpy(&h, src, sizeof(h));
  if (h.magic != kMagic || h.prec != p->prec || h.ntot != p->ntot) return fail(ETM_E_INVAL, "checkpoint does not match the plan");
  const char *o = static_cast<const char *>(src) + sizeof(h);
  for (const Region *r : state_regions(p)) {
    HIP_TRY(hipMemcpyAsync(p->ws + r->off, o, r->bytes, hipMemcpyHostToDevice, p->stream));
    o += r->bytes;
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  p->step = h.step; p->rec = h.rec; p->n_thermal = h.n_thermal; p->cg_total = h.cg_total;
  p->cur = h.cur; p->th_cur = h.th_cur; p->n_solves = h.n_solves;
  p->sol_t[0] = h.sol_t[0]; p->sol_t[1] = h.sol_t[1]; p->sol_t[2] = h.sol_t[2];
  p->host_status = ETM_OK;
  p->joule_pending = false;
  p->a_base = kNoWaveBlock;
  return coef_refresh(p, false);
}

void etm_plan_destroy(etm_plan *p) {
  if (!p) return;
  if (p->solve_pending && p->ev_solve) (void)hipEventSynchronize(p->ev_solve);  // its copy targets ctl_host
  if (p->mstream) (void)hipStreamSynchronize(p->mstream);
  if (p->ev_main) (void)hipEventDestroy(p->ev_main);
  if (p->ev_copy) (void)hipEventDestroy(p->ev_copy);
  if (p->ev_solve) (void)hipEventDestroy(p->ev_solve);
  if (p->mstream) (void)hipStreamDestroy(p->mstream);
  if (p->sc_host) (void)hipHostFree(p->sc_host);
  if (p->ctl_host) (void)hipHostFree(p->ctl_host);
  delete p;
}

const char *etm_last_error(void) { return g_err.c_str(); }

}  // extern "C"
