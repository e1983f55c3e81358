// gfx950 kernels of the coupled EM + Joule + thermal march (arXiv 2603.07038,
// Sec. II-A): the explicit central-difference EM update of Eq. (2)-(3) with
// sigma(T) from Eq. (6), the Joule source D_sigma e^2, the forward-Euler
// conduction step of Eq. (5), and the history diagnostics.
//
// Scaled form used on the device (both precisions).  Dividing Eq. (2) for an
// edge by eps0 and by the edge volume L*A gives
//   (er + a) e^{n+1} = 2 er e^n - (c0 dt)^2 (C e^n) - (er - a) e^{n-1} - jd
// with er the edge's mean relative permittivity, a = dt sigma_e / (2 eps0)
// (port conductances included), C the purely geometric curl-curl
// (curl mu0^-1 curl = C / mu0) and jd = dt (J^{n+1/2} - J^{n-1/2}) / eps0.
// The mixed path carries (e, delta = e^{n+1} - e^n) in FP32 and updates
//   (er + a) delta^{n+1/2} = (er - a) delta^{n-1/2} - (c0 dt)^2 C e^n - jd,
//   e^{n+1} = e^n + delta^{n+1/2},
// which is the same recurrence rearranged so that FP32 rounding is not
// integrated twice.
//
// One thread owns one node: it updates the x-, y- and z-edges that start at
// the node and gathers the Joule power of all six edges that meet there.  The
// three low-side edges belong to neighbouring threads, so their new values
// are recomputed locally (the state is double/ping-pong buffered, so this
// reads only old values) instead of being exchanged with atomics; the result
// is deterministic.
#include "etm_internal.h"

namespace etm {

namespace {

constexpr int BX = 64, BY = 4;

template <typename T>
struct Ld1 {
  const T *a;
  __device__ __forceinline__ T operator[](int64_t i) const { return a[i]; }
};
template <typename T>
struct LdDiff {  // a - b (e^n recovered from e^{n+1} and delta in the mixed diagnostics)
  const T *a, *b;
  __device__ __forceinline__ T operator[](int64_t i) const { return a[i] - b[i]; }
};

// ---- geometric curl-curl (C e) at the edge of direction D starting at node
// (i,j,k) = index n.  h on a primal face = circulation / area (mu0 dropped);
// faces outside the domain carry zero (PMC truncation).
template <typename T, typename LD>
__device__ __forceinline__ T curl_x(const DevGrid &g, const LD &ex, const LD &ey, const LD &ez, int i, int j,
                                    int k, int64_t n) {
  const T idxi = T(g.idx[i]);
  T s = T(0);
  if (j < g.ny) s += ((ex[n] - ex[n + g.sy]) * T(g.idy[j]) + (ey[n + 1] - ey[n]) * idxi) * T(g.ihy[j]);
  if (j > 0)
    s -= ((ex[n - g.sy] - ex[n]) * T(g.idy[j - 1]) + (ey[n - g.sy + 1] - ey[n - g.sy]) * idxi) * T(g.ihy[j]);
  if (k < g.nz) s -= ((ez[n] - ez[n + 1]) * idxi + (ex[n + g.sz] - ex[n]) * T(g.idz[k])) * T(g.ihz[k]);
  if (k > 0)
    s += ((ez[n - g.sz] - ez[n - g.sz + 1]) * idxi + (ex[n] - ex[n - g.sz]) * T(g.idz[k - 1])) * T(g.ihz[k]);
  return s;
}

template <typename T, typename LD>
__device__ __forceinline__ T curl_y(const DevGrid &g, const LD &ex, const LD &ey, const LD &ez, int i, int j,
                                    int k, int64_t n) {
  const T idyj = T(g.idy[j]);
  T s = T(0);
  // + [hx(k) - hx(k-1)] / hz
  if (k < g.nz) s += ((ez[n + g.sy] - ez[n]) * idyj - (ey[n + g.sz] - ey[n]) * T(g.idz[k])) * T(g.ihz[k]);
  if (k > 0)
    s -= ((ez[n - g.sz + g.sy] - ez[n - g.sz]) * idyj - (ey[n] - ey[n - g.sz]) * T(g.idz[k - 1])) * T(g.ihz[k]);
  // - [hz(i) - hz(i-1)] / hx
  if (i < g.nx) s -= ((ex[n] - ex[n + g.sy]) * idyj + (ey[n + 1] - ey[n]) * T(g.idx[i])) * T(g.ihx[i]);
  if (i > 0)
    s += ((ex[n - 1] - ex[n - 1 + g.sy]) * idyj + (ey[n] - ey[n - 1]) * T(g.idx[i - 1])) * T(g.ihx[i]);
  return s;
}

template <typename T, typename LD>
__device__ __forceinline__ T curl_z(const DevGrid &g, const LD &ex, const LD &ey, const LD &ez, int i, int j,
                                    int k, int64_t n) {
  const T idzk = T(g.idz[k]);
  T s = T(0);
  // + [hy(i) - hy(i-1)] / hx
  if (i < g.nx) s += ((ez[n] - ez[n + 1]) * T(g.idx[i]) + (ex[n + g.sz] - ex[n]) * idzk) * T(g.ihx[i]);
  if (i > 0)
    s -= ((ez[n - 1] - ez[n]) * T(g.idx[i - 1]) + (ex[n - 1 + g.sz] - ex[n - 1]) * idzk) * T(g.ihx[i]);
  // - [hx(j) - hx(j-1)] / hy
  if (j < g.ny) s -= ((ez[n + g.sy] - ez[n]) * T(g.idy[j]) - (ey[n + g.sz] - ey[n]) * idzk) * T(g.ihy[j]);
  if (j > 0)
    s += ((ez[n] - ez[n - g.sy]) * T(g.idy[j - 1]) - (ey[n - g.sy + g.sz] - ey[n - g.sy]) * idzk) * T(g.ihy[j]);
  return s;
}

template <typename T, int D, typename LD>
__device__ __forceinline__ T curl_d(const DevGrid &g, const LD &ex, const LD &ey, const LD &ez, int i, int j,
                                    int k, int64_t n) {
  if (D == 0) return curl_x<T>(g, ex, ey, ez, i, j, k, n);
  if (D == 1) return curl_y<T>(g, ex, ey, ez, i, j, k, n);
  return curl_z<T>(g, ex, ey, ez, i, j, k, n);
}

// ---- edge materials: sums over the up-to-four cells around the edge of
// (quarter of the transverse dual area in the cell) * property.  Divided by
// the dual area they give the area-weighted means; sigma per cell follows
// Eq. (6) at the edge-midpoint rise.
template <typename T, int D>
__device__ __forceinline__ void edge_sums(const DevGrid &g, int i, int j, int k, int64_t n, T th, T &epsA,
                                          T &sigA) {
  epsA = T(0);
  sigA = T(0);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    int a0 = (c & 1) - 1, b0 = (c >> 1) - 1;  // offsets -1/0 in the two transverse directions
    int ii = i, jj = j, kk = k;
    T w;
    if (D == 0) {
      jj = j + a0; kk = k + b0;
      if (jj < 0 || jj >= g.ny || kk < 0 || kk >= g.nz) continue;
      w = T(0.25) * T(g.dy[jj]) * T(g.dz[kk]);
    } else if (D == 1) {
      ii = i + a0; kk = k + b0;
      if (ii < 0 || ii >= g.nx || kk < 0 || kk >= g.nz) continue;
      w = T(0.25) * T(g.dx[ii]) * T(g.dz[kk]);
    } else {
      ii = i + a0; jj = j + b0;
      if (ii < 0 || ii >= g.nx || jj < 0 || jj >= g.ny) continue;
      w = T(0.25) * T(g.dx[ii]) * T(g.dy[jj]);
    }
    const int m = g.mat[n + (ii - i) + (jj - j) * g.sy + (kk - k) * g.sz];
    const double *row = g.mtab + m * kMatStride;
    epsA += w * T(row[MC_EPSR]);
    T s = T(row[MC_SIGS]);
    const T t = T(row[MC_TCR]);
    if (t != T(0)) s = s / (T(1) + t * th);
    sigA += w * s;
  }
}

__device__ __forceinline__ int find_port(const DevPorts &P, int64_t key) {
  int lo = 0, hi = P.n_edges - 1;
  while (lo <= hi) {
    int mid = (lo + hi) >> 1;
    int64_t km = P.key[mid];
    if (km == key) return mid;
    if (km < key) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

template <typename T>
struct EmPtrs {
  const T *e[3];    // e^n
  const T *aux[3];  // FP64: e^{n-1};  mixed: delta^{n-1/2}
  T *oe[3];         // e^{n+1}
  T *oaux[3];       // mixed: delta^{n+1/2}
};

__device__ __forceinline__ bool pec_edge(const DevGrid &g, int D, int i, int j, int k) {
  const int b = g.pec;
  if (D != 0 && ((i == 0 && (b & 1)) || (i == g.nx && (b & 2)))) return true;
  if (D != 1 && ((j == 0 && (b & 4)) || (j == g.ny && (b & 8)))) return true;
  if (D != 2 && ((k == 0 && (b & 16)) || (k == g.nz && (b & 32)))) return true;
  return false;
}

// New value of one edge; sigA (material conductance sum, for the Joule
// source) and the increment are returned by reference.
template <typename T, int D, bool INC>
__device__ __forceinline__ T edge_new(const EmLaunch &L, const EmPtrs<T> &p, const T *th, int i, int j, int k,
                                      int64_t n, T &sigA, T &delta) {
  const DevGrid &g = L.g;
  if (pec_edge(g, D, i, j, k)) { sigA = T(0); delta = T(0); return T(0); }
  const int64_t nb = n + (D == 0 ? 1 : D == 1 ? g.sy : g.sz);
  const T th_e = T(0.5) * (th[n] + th[nb]);
  T epsA;
  edge_sums<T, D>(g, i, j, k, n, th_e, epsA, sigA);
  const T iA = D == 0 ? T(g.ihy[j] * g.ihz[k]) : D == 1 ? T(g.ihx[i] * g.ihz[k]) : T(g.ihx[i] * g.ihy[j]);
  const T er = epsA * iA;
  T a = sigA * iA;
  T jd = T(0);
  if (g.flags[n] & (1 << D)) {
    const int q = find_port(L.ports, int64_t(D) * g.ntot + n);
    if (q >= 0) {
      a += T(L.ports.gs[q]);
      double acc = 0.0;
      const int64_t s1 = L.step + 1, s0 = L.step, ns = L.ports.n_samples;
      for (int t = L.ports.start[q]; t < L.ports.start[q + 1]; ++t) {
        const double *Jw = L.ports.J + int64_t(L.ports.wave[t]) * ns;
        const double j1 = s1 < ns ? Jw[s1] : 0.0, j0 = s0 < ns ? Jw[s0] : 0.0;
        acc += L.ports.wt[t] * (j1 - j0);
      }
      jd = T(acc);
    }
  }
  Ld1<T> ex{p.e[0]}, ey{p.e[1]}, ez{p.e[2]};
  const T cc = curl_d<T, D>(g, ex, ey, ez, i, j, k, n);
  const T e0 = p.e[D][n];
  const T inv = T(1) / (er + a);
  if (INC) {
    delta = ((er - a) * p.aux[D][n] - T(L.c2dt2) * cc - jd) * inv;
    return e0 + delta;
  } else {
    const T en = (T(2) * er * e0 - T(L.c2dt2) * cc - (er - a) * p.aux[D][n] - jd) * inv;
    delta = en - e0;
    return en;
  }
}

template <typename T, bool INC>
__global__ __launch_bounds__(256) void em_step_kernel(EmLaunch L, EmPtrs<T> p, const T *th) {
  const DevGrid &g = L.g;
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  if (i > g.nx || j > g.ny) return;
  const int64_t n = int64_t(k) * g.sz + int64_t(j) * g.sy + i;
  T jsum = T(0), s, d;
  if (i < g.nx) {
    const T e1 = edge_new<T, 0, INC>(L, p, th, i, j, k, n, s, d);
    p.oe[0][n] = e1;
    if (INC) p.oaux[0][n] = d;
    jsum += e1 * e1 * T(g.dx[i]) * s;
  }
  if (j < g.ny) {
    const T e1 = edge_new<T, 1, INC>(L, p, th, i, j, k, n, s, d);
    p.oe[1][n] = e1;
    if (INC) p.oaux[1][n] = d;
    jsum += e1 * e1 * T(g.dy[j]) * s;
  }
  if (k < g.nz) {
    const T e1 = edge_new<T, 2, INC>(L, p, th, i, j, k, n, s, d);
    p.oe[2][n] = e1;
    if (INC) p.oaux[2][n] = d;
    jsum += e1 * e1 * T(g.dz[k]) * s;
  }
  if (i > 0) {
    const T e1 = edge_new<T, 0, INC>(L, p, th, i - 1, j, k, n - 1, s, d);
    jsum += e1 * e1 * T(g.dx[i - 1]) * s;
  }
  if (j > 0) {
    const T e1 = edge_new<T, 1, INC>(L, p, th, i, j - 1, k, n - g.sy, s, d);
    jsum += e1 * e1 * T(g.dy[j - 1]) * s;
  }
  if (k > 0) {
    const T e1 = edge_new<T, 2, INC>(L, p, th, i, j, k - 1, n - g.sz, s, d);
    jsum += e1 * e1 * T(g.dz[k - 1]) * s;
  }
  // P_n = sum_e 1/2 sigma_e e^2 L A / V_n  =  jf * sum_e e^2 L sigA / V_n
  L.psum[n] += double(jsum) * L.jf * (g.ihx[i] * g.ihy[j] * g.ihz[k]);
}

// ---- block reductions (wave64 shuffles, then LDS across the 4 waves) -------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

template <int NS, int NM>
__device__ __forceinline__ void block_reduce_store(const double (&sums)[NS], const double (&maxs)[NM],
                                                   double *out) {
  __shared__ double red[4][NS + NM];
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  const int lane = tid & 63, wv = tid >> 6;
  double v[NS + NM];
#pragma unroll
  for (int q = 0; q < NS; ++q) v[q] = wave_sum(sums[q]);
#pragma unroll
  for (int q = 0; q < NM; ++q) v[NS + q] = wave_max(maxs[q]);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NS + NM; ++q) red[wv][q] = v[q];
  __syncthreads();
  if (tid == 0) {
    const int nw = (blockDim.x * blockDim.y + 63) / 64;
#pragma unroll
    for (int q = 0; q < NS + NM; ++q) {
      double acc = red[0][q];
      for (int w = 1; w < nw; ++w) acc = q < NS ? acc + red[w][q] : fmax(acc, red[w][q]);
      out[q] = acc;
    }
  }
}

// ---- thermal step, Eq. (5) ---------------------------------------------------
// C_n V_n (theta' - theta) = dt*psum*V_n - R*dt*sum_e G_e (theta_n - theta_m),
// G_e = sum over the edge's cells of (quarter transverse area) k_c / L,
// C_n V_n = sum over the node's cell octants of rho_cp * octant volume.
__global__ __launch_bounds__(256) void thermal_kernel(ThermalLaunch L) {
  const DevGrid &g = L.g;
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  double e_part = 0.0, m_part = 0.0;
  if (i <= g.nx && j <= g.ny) {
    const int64_t n = int64_t(k) * g.sz + int64_t(j) * g.sy + i;
    const double t0 = L.theta_in[n];
    double CV = 0.0, gx0 = 0, gx1 = 0, gy0 = 0, gy1 = 0, gz0 = 0, gz1 = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int ox = c & 1, oy = (c >> 1) & 1, oz = c >> 2;
      const int ii = i - 1 + ox, jj = j - 1 + oy, kk = k - 1 + oz;
      if (ii < 0 || ii >= g.nx || jj < 0 || jj >= g.ny || kk < 0 || kk >= g.nz) continue;
      const double *row = g.mtab + g.mat[n + (ox - 1) + (oy - 1) * g.sy + (oz - 1) * g.sz] * kMatStride;
      const double ddx = g.dx[ii], ddy = g.dy[jj], ddz = g.dz[kk], kc = row[MC_K];
      CV += row[MC_RHOCP] * 0.125 * ddx * ddy * ddz;
      // this cell touches the node's x-edge on side ox, y-edge on side oy, z-edge on side oz
      const double wx = 0.25 * ddy * ddz * kc / ddx, wy = 0.25 * ddx * ddz * kc / ddy, wz = 0.25 * ddx * ddy * kc / ddz;
      if (ox) gx1 += wx; else gx0 += wx;
      if (oy) gy1 += wy; else gy0 += wy;
      if (oz) gz1 += wz; else gz0 += wz;
    }
    double flux = 0.0;
    if (i > 0) flux += gx0 * (t0 - L.theta_in[n - 1]);
    if (i < g.nx) flux += gx1 * (t0 - L.theta_in[n + 1]);
    if (j > 0) flux += gy0 * (t0 - L.theta_in[n - g.sy]);
    if (j < g.ny) flux += gy1 * (t0 - L.theta_in[n + g.sy]);
    if (k > 0) flux += gz0 * (t0 - L.theta_in[n - g.sz]);
    if (k < g.nz) flux += gz1 * (t0 - L.theta_in[n + g.sz]);
    const double V = g.hx[i] * g.hy[j] * g.hz[k];
    const double ps = L.psum[n];
    const double tn = t0 + (L.dt * ps * V - double(L.R) * L.dt * flux) / CV;
    L.theta_out[n] = tn;
    L.psum[n] = 0.0;
    if (L.theta32) L.theta32[n] = float(tn);
    e_part = L.dt * ps * V;
    m_part = tn;
  }
  const double s[1] = {e_part}, m[1] = {m_part};
  const int64_t b = (int64_t(blockIdx.z) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  block_reduce_store<1, 1>(s, m, L.partials + b * kRedWidth);
}

// Sum partials [nb][kRedWidth] in a fixed order (one block of 256).
__device__ void reduce_partials(const double *part, int64_t nb, int n_sum, int n_max, double *out) {
  __shared__ double red[4][kRedWidth];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double v[kRedWidth];
  for (int q = 0; q < kRedWidth; ++q) v[q] = q < n_sum ? 0.0 : -1.0e300;
  for (int64_t b = tid; b < nb; b += blockDim.x)
    for (int q = 0; q < n_sum + n_max; ++q) v[q] = q < n_sum ? v[q] + part[b * kRedWidth + q] : fmax(v[q], part[b * kRedWidth + q]);
  for (int q = 0; q < n_sum + n_max; ++q) v[q] = q < n_sum ? wave_sum(v[q]) : wave_max(v[q]);
  if (lane == 0)
    for (int q = 0; q < n_sum + n_max; ++q) red[wv][q] = v[q];
  __syncthreads();
  if (tid == 0)
    for (int q = 0; q < n_sum + n_max; ++q) {
      double acc = red[0][q];
      for (int w = 1; w < (int)(blockDim.x / 64); ++w) acc = q < n_sum ? acc + red[w][q] : fmax(acc, red[w][q]);
      out[q] = acc;
    }
}

__global__ __launch_bounds__(256) void thermal_finalize(const double *part, int64_t nb, DevScalars *sc) {
  __shared__ double out[kRedWidth];
  reduce_partials(part, nb, 1, 1, out);
  if (threadIdx.x == 0) {
    sc->ejoule += out[0];
    sc->theta_max = out[1];
    if (!isfinite(out[0]) || !isfinite(out[1])) { if (sc->status == 0) sc->status = ETM_E_UNSTABLE; }
  }
}

// ---- diagnostics -------------------------------------------------------------
// W = eps0/(2 dt^2) sum_e L A [ er delta^2 + (c0 dt)^2 e^{n+1} (C e^n) ]
template <typename T, bool INC>
__global__ __launch_bounds__(256) void diag_kernel(DiagLaunch L) {
  const DevGrid &g = L.g;
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  double w_part = 0.0, j_part = 0.0, m_part = -1.0e300;
  if (i <= g.nx && j <= g.ny) {
    const int64_t n = int64_t(k) * g.sz + int64_t(j) * g.sy + i;
    const T *en[3] = {(const T *)L.e_new[0], (const T *)L.e_new[1], (const T *)L.e_new[2]};
    const T *eo[3] = {(const T *)L.e_old[0], (const T *)L.e_old[1], (const T *)L.e_old[2]};
    double acc = 0.0;
    for (int D = 0; D < 3; ++D) {
      if ((D == 0 && i == g.nx) || (D == 1 && j == g.ny) || (D == 2 && k == g.nz)) continue;
      if (pec_edge(g, D, i, j, k)) continue;
      double cc;
      if (INC) {
        LdDiff<T> ex{en[0], eo[0]}, ey{en[1], eo[1]}, ez{en[2], eo[2]};
        cc = D == 0 ? double(curl_x<T>(g, ex, ey, ez, i, j, k, n)) : D == 1 ? double(curl_y<T>(g, ex, ey, ez, i, j, k, n))
                                                                          : double(curl_z<T>(g, ex, ey, ez, i, j, k, n));
      } else {
        Ld1<T> ex{eo[0]}, ey{eo[1]}, ez{eo[2]};
        cc = D == 0 ? double(curl_x<T>(g, ex, ey, ez, i, j, k, n)) : D == 1 ? double(curl_y<T>(g, ex, ey, ez, i, j, k, n))
                                                                          : double(curl_z<T>(g, ex, ey, ez, i, j, k, n));
      }
      double epsA, sigA;
      if (D == 0) edge_sums<double, 0>(g, i, j, k, n, 0.0, epsA, sigA);
      else if (D == 1) edge_sums<double, 1>(g, i, j, k, n, 0.0, epsA, sigA);
      else edge_sums<double, 2>(g, i, j, k, n, 0.0, epsA, sigA);
      const double Lh = D == 0 ? g.dx[i] : D == 1 ? g.dy[j] : g.dz[k];
      const double A = D == 0 ? g.hy[j] * g.hz[k] : D == 1 ? g.hx[i] * g.hz[k] : g.hx[i] * g.hy[j];
      const double e1 = double(en[D][n]);
      const double dl = INC ? double(eo[D][n]) : e1 - double(eo[D][n]);
      // er * L * A = epsA * L (epsA already carries the area)
      acc += epsA * Lh * dl * dl + L.c2dt2 * Lh * A * e1 * cc;
    }
    w_part = acc;
    j_part = L.psum[n] * (g.hx[i] * g.hy[j] * g.hz[k]);
    m_part = L.theta[n];
  }
  const double s[2] = {w_part, j_part}, m[1] = {m_part};
  const int64_t b = (int64_t(blockIdx.z) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  block_reduce_store<2, 1>(s, m, L.partials + b * kRedWidth);
}

template <typename T>
__global__ __launch_bounds__(256) void diag_finalize(DiagLaunch L, int64_t nb) {
  __shared__ double out[kRedWidth];
  reduce_partials(L.partials, nb, 2, 1, out);
  if (threadIdx.x == 0) {
    const double W = out[0] * kEps0 / (2.0 * L.dt * L.dt);
    if (!isfinite(W)) { if (L.sc->status == 0) L.sc->status = ETM_E_UNSTABLE; }
    if (L.rec < L.cap) {
      double *row = L.hist_row;
      row[0] = double(L.step);
      row[1] = W;
      row[2] = L.sc->ejoule + L.dt * out[1];
      row[3] = out[2];
      for (int q = 0; q < L.n_probes; ++q) {
        const int f = int(L.probes[2 * q]);
        const int64_t idx = L.probes[2 * q + 1];
        row[4 + q] = f == 3 ? L.theta[idx] : double(((const T *)L.e_new[f])[idx]);
      }
      L.sc->n_records = L.rec + 1;
    }
  }
}

// ---- layout conversion and fills -------------------------------------------
__global__ void pack_kernel(const void *src, int src_f32, int64_t sy, int64_t sz, int ni, int nj, int nk,
                            double *dst) {
  const int64_t total = int64_t(ni) * nj * nk;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    const int i = int(t % ni);
    const int64_t r = t / ni;
    const int j = int(r % nj), k = int(r / nj);
    const int64_t s = int64_t(k) * sz + int64_t(j) * sy + i;
    dst[t] = src_f32 ? double(((const float *)src)[s]) : ((const double *)src)[s];
  }
}

__global__ void unpack_kernel(const double *src, int ni, int nj, int nk, void *dst, int dst_f32, int64_t sy,
                              int64_t sz) {
  const int64_t total = int64_t(ni) * nj * nk;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    const int i = int(t % ni);
    const int64_t r = t / ni;
    const int j = int(r % nj), k = int(r / nj);
    const int64_t s = int64_t(k) * sz + int64_t(j) * sy + i;
    if (dst_f32) ((float *)dst)[s] = float(src[t]); else ((double *)dst)[s] = src[t];
  }
}

__global__ void fill_kernel(uint32_t *dst, int64_t n_words) {
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n_words; t += int64_t(gridDim.x) * blockDim.x)
    dst[t] = 0u;
}

inline dim3 node_grid(const DevGrid &g) {
  return dim3((g.nx + 1 + BX - 1) / BX, (g.ny + 1 + BY - 1) / BY, g.nz + 1);
}

}  // namespace

int reduce_blocks(int64_t) { return 0; }

hipError_t launch_em_step(const EmLaunch &L, hipStream_t s) {
  const dim3 grid = node_grid(L.g), block(BX, BY, 1);
  if (L.precision == ETM_PREC_FP64) {
    EmPtrs<double> p;
    for (int d = 0; d < 3; ++d) {
      p.e[d] = (const double *)L.e0[d];
      p.aux[d] = (const double *)L.e1[d];
      p.oe[d] = (double *)L.out0[d];
      p.oaux[d] = nullptr;
    }
    hipLaunchKernelGGL((em_step_kernel<double, false>), grid, block, 0, s, L, p, L.theta);
  } else {
    EmPtrs<float> p;
    for (int d = 0; d < 3; ++d) {
      p.e[d] = (const float *)L.e0[d];
      p.aux[d] = (const float *)L.e1[d];
      p.oe[d] = (float *)L.out0[d];
      p.oaux[d] = (float *)L.out1[d];
    }
    hipLaunchKernelGGL((em_step_kernel<float, true>), grid, block, 0, s, L, p, L.theta32);
  }
  return hipGetLastError();
}

hipError_t launch_thermal(const ThermalLaunch &L, hipStream_t s) {
  const dim3 grid = node_grid(L.g), block(BX, BY, 1);
  hipLaunchKernelGGL(thermal_kernel, grid, block, 0, s, L);
  const int64_t nb = int64_t(grid.x) * grid.y * grid.z;
  hipLaunchKernelGGL(thermal_finalize, dim3(1), dim3(256), 0, s, (const double *)L.partials, nb, L.sc);
  return hipGetLastError();
}

hipError_t launch_diag(const DiagLaunch &L, hipStream_t s) {
  const dim3 grid = node_grid(L.g), block(BX, BY, 1);
  const int64_t nb = int64_t(grid.x) * grid.y * grid.z;
  if (L.precision == ETM_PREC_FP64) {
    hipLaunchKernelGGL((diag_kernel<double, false>), grid, block, 0, s, L);
    hipLaunchKernelGGL((diag_finalize<double>), dim3(1), dim3(256), 0, s, L, nb);
  } else {
    hipLaunchKernelGGL((diag_kernel<float, true>), grid, block, 0, s, L);
    hipLaunchKernelGGL((diag_finalize<float>), dim3(1), dim3(256), 0, s, L, nb);
  }
  return hipGetLastError();
}

hipError_t launch_pack(const void *src, int src_f32, int64_t sy, int64_t sz, int ni, int nj, int nk, double *dst,
                       hipStream_t s) {
  const int64_t total = int64_t(ni) * nj * nk;
  if (total <= 0) return hipSuccess;
  const int blocks = int(std::min<int64_t>((total + 255) / 256, 65536));
  hipLaunchKernelGGL(pack_kernel, dim3(blocks), dim3(256), 0, s, src, src_f32, sy, sz, ni, nj, nk, dst);
  return hipGetLastError();
}

hipError_t launch_unpack(const double *src, int ni, int nj, int nk, void *dst, int dst_f32, int64_t sy, int64_t sz,
                         hipStream_t s) {
  const int64_t total = int64_t(ni) * nj * nk;
  if (total <= 0) return hipSuccess;
  const int blocks = int(std::min<int64_t>((total + 255) / 256, 65536));
  hipLaunchKernelGGL(unpack_kernel, dim3(blocks), dim3(256), 0, s, src, ni, nj, nk, dst, dst_f32, sy, sz);
  return hipGetLastError();
}

hipError_t launch_fill(void *dst, int64_t n_bytes, hipStream_t s) {
  const int64_t words = n_bytes / 4;
  if (words <= 0) return hipSuccess;
  const int blocks = int(std::min<int64_t>((words + 255) / 256, 65536));
  hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(256), 0, s, (uint32_t *)dst, words);
  return hipGetLastError();
}

}  // namespace etm
