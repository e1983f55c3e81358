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
// The mixed path marches the same scheme as leapfrog on (e^n, h^{n-1/2}),
// both stored in FP32 and combined in FP64, with an 8-bit residual that
// extends the stored e below its FP32 rounding (em_march_row_yee).  Edge
// coefficients are always formed in FP64 and rounded once.
//
// March kernels.  A block owns a column of 4 rows of nodes and marches up a
// chunk of z planes (FP64: 64 x 4 nodes staged in LDS with a one-node halo;
// mixed: one barrier-free wave per row of 62 nodes).  A node updates the x-,
// y- and z-edges that start at it.  The Joule source is gathered one step late: the
// node sums sigma e^2 L A over its six incident edges of the *input* field
// e^n, which the stencil already holds, so no edge update is recomputed.
// The power of the last step of a thermal block is added by the thermal
// kernel (or by a flush kernel at the end of an advance call) before
// temperature changes.
#include <algorithm>

#include "etm_internal.h"

namespace etm {

namespace {

constexpr int BX = 64, BY = 4;             // threads per block (x, y)
constexpr int TXH = BX + 2, TYH = BY + 2;  // staged tile with halo

// ---- field accessors: value of component c at node offset (di, dj, dk) --
template <typename T>
struct GAcc {  // global memory around node n
  const T *e[3];
  int64_t n, sy, sz;
  __device__ __forceinline__ T raw(int c, int di, int dj, int dk) const { return e[c][n + di + dj * sy + dk * sz]; }
  __device__ __forceinline__ double operator()(int c, int di, int dj, int dk) const { return double(raw(c, di, dj, dk)); }
};
template <typename T>
struct SAcc {  // LDS ring: slot[dk+1] holds plane k+dk
  const T (*sh)[3][TYH][TXH];
  int slot[3];
  int li, lj;
  __device__ __forceinline__ T raw(int c, int di, int dj, int dk) const { return sh[slot[dk + 1]][c][lj + dj][li + di]; }
  __device__ __forceinline__ double operator()(int c, int di, int dj, int dk) const { return double(raw(c, di, dj, dk)); }
};

// ---- geometric curl-curl (C e) at the edge of direction D starting at node
// (i,j,k).  h on a primal face = circulation / area (mu0 dropped); faces
// outside the domain carry zero (PMC truncation).
template <typename T, typename A>
__device__ __forceinline__ T curl_x(const DevGrid &g, const A &E, int i, int j, int k) {
  const T idxi = T(g.idx[i]);
  T s = T(0);
  if (j < g.ny) s += ((E.raw(0, 0, 0, 0) - E.raw(0, 0, 1, 0)) * T(g.idy[j]) + (E.raw(1, 1, 0, 0) - E.raw(1, 0, 0, 0)) * idxi) * T(g.ihy[j]);
  if (j > 0) s -= ((E.raw(0, 0, -1, 0) - E.raw(0, 0, 0, 0)) * T(g.idy[j - 1]) + (E.raw(1, 1, -1, 0) - E.raw(1, 0, -1, 0)) * idxi) * T(g.ihy[j]);
  if (k < g.nz) s -= ((E.raw(2, 0, 0, 0) - E.raw(2, 1, 0, 0)) * idxi + (E.raw(0, 0, 0, 1) - E.raw(0, 0, 0, 0)) * T(g.idz[k])) * T(g.ihz[k]);
  if (k > 0) s += ((E.raw(2, 0, 0, -1) - E.raw(2, 1, 0, -1)) * idxi + (E.raw(0, 0, 0, 0) - E.raw(0, 0, 0, -1)) * T(g.idz[k - 1])) * T(g.ihz[k]);
  return s;
}
template <typename T, typename A>
__device__ __forceinline__ T curl_y(const DevGrid &g, const A &E, int i, int j, int k) {
  const T idyj = T(g.idy[j]);
  T s = T(0);
  if (k < g.nz) s += ((E.raw(2, 0, 1, 0) - E.raw(2, 0, 0, 0)) * idyj - (E.raw(1, 0, 0, 1) - E.raw(1, 0, 0, 0)) * T(g.idz[k])) * T(g.ihz[k]);
  if (k > 0) s -= ((E.raw(2, 0, 1, -1) - E.raw(2, 0, 0, -1)) * idyj - (E.raw(1, 0, 0, 0) - E.raw(1, 0, 0, -1)) * T(g.idz[k - 1])) * T(g.ihz[k]);
  if (i < g.nx) s -= ((E.raw(0, 0, 0, 0) - E.raw(0, 0, 1, 0)) * idyj + (E.raw(1, 1, 0, 0) - E.raw(1, 0, 0, 0)) * T(g.idx[i])) * T(g.ihx[i]);
  if (i > 0) s += ((E.raw(0, -1, 0, 0) - E.raw(0, -1, 1, 0)) * idyj + (E.raw(1, 0, 0, 0) - E.raw(1, -1, 0, 0)) * T(g.idx[i - 1])) * T(g.ihx[i]);
  return s;
}
template <typename T, typename A>
__device__ __forceinline__ T curl_z(const DevGrid &g, const A &E, int i, int j, int k) {
  const T idzk = T(g.idz[k]);
  T s = T(0);
  if (i < g.nx) s += ((E.raw(2, 0, 0, 0) - E.raw(2, 1, 0, 0)) * T(g.idx[i]) + (E.raw(0, 0, 0, 1) - E.raw(0, 0, 0, 0)) * idzk) * T(g.ihx[i]);
  if (i > 0) s -= ((E.raw(2, -1, 0, 0) - E.raw(2, 0, 0, 0)) * T(g.idx[i - 1]) + (E.raw(0, -1, 0, 1) - E.raw(0, -1, 0, 0)) * idzk) * T(g.ihx[i]);
  if (j < g.ny) s -= ((E.raw(2, 0, 1, 0) - E.raw(2, 0, 0, 0)) * T(g.idy[j]) - (E.raw(1, 0, 0, 1) - E.raw(1, 0, 0, 0)) * idzk) * T(g.ihy[j]);
  if (j > 0) s += ((E.raw(2, 0, 0, 0) - E.raw(2, 0, -1, 0)) * T(g.idy[j - 1]) - (E.raw(1, 0, -1, 1) - E.raw(1, 0, -1, 0)) * idzk) * T(g.ihy[j]);
  return s;
}

__device__ __forceinline__ bool pec_edge(const DevGrid &g, int D, int i, int j, int k) {
  const int b = g.pec;
  if (D != 0 && ((i == 0 && (b & 1)) || (i == g.nx && (b & 2)))) return true;
  if (D != 1 && ((j == 0 && (b & 4)) || (j == g.ny && (b & 8)))) return true;
  if (D != 2 && ((k == 0 && (b & 16)) || (k == g.nz && (b & 32)))) return true;
  return false;
}

// ---- 1D tables, from one base pointer (dx, dy, dz, idx, idy, idz, hx, hy, hz,
// ihx, ihy, ihz, then alpha_lo / alpha_hi per axis on nodes).
struct Geo {
  const double *dx, *dy, *dz, *idx, *idy, *idz, *ihx, *ihy, *ihz, *axl, *axh, *ayl, *ayh, *azl, *azh;
  __device__ __forceinline__ Geo(const double *g, int nx, int ny, int nz) {
    dx = g; dy = dx + nx; dz = dy + ny;
    idx = dz + nz; idy = idx + nx; idz = idy + ny;
    const double *hx = idz + nz, *hy = hx + nx + 1, *hz = hy + ny + 1;
    ihx = hz + nz + 1; ihy = ihx + nx + 1; ihz = ihy + ny + 1;
    axl = ihz + nz + 1; axh = axl + nx + 1; ayl = axh + nx + 1; ayh = ayl + ny + 1;
    azl = ayh + ny + 1; azh = azl + nz + 1;
  }
};

// ---- edge coefficients from the cells around a node -----------------------
// Cell (i-1+ox, j-1+oy, k-1+oz) touches the node's x-edge on side ox (the
// edge starting at the node if ox = 1, the low-side edge i-1 if ox = 0), its
// y-edge on side oy and its z-edge on side oz.  An edge property is the mean
// over its cells weighted by the share of the edge's dual area in each cell;
// on a rectilinear grid that share factors into alpha_y(oy) * alpha_z(oz)
// for an x-edge (alpha = half the cell width over the node's dual width, 0 for
// a cell outside the mesh).  sigma follows Eq. (6) per cell at the
// edge-midpoint rise.  Returned: the normalised conductance
// a = dt sigma / (2 eps0) and (own edges) the mean eps_r.  FP64 with explicit
// FMAs and contraction off, so every kernel that calls it gets the same bits.
struct CellV {
  double er, sg;  // eps_r, sigma0 * dt / (2 eps0)
  int tf, m;      // sigma depends on temperature; material id
};

template <int D, typename CELL, typename TCR, typename TH>
__device__ __forceinline__ double edge_coef(int side, const double (&ax)[2], const double (&ay)[2],
                                            const double (&az)[2], const CELL &cell, const TCR &tcr_of, const TH &th,
                                            double *er_out) {
#pragma clang fp contract(off)
  double er = 0.0, sg = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int p0 = q & 1, p1 = q >> 1;  // offsets in the two transverse directions
    const int ox = D == 0 ? side : p0, oy = D == 1 ? side : (D == 0 ? p0 : p1), oz = D == 2 ? side : p1;
    const double w = D == 0 ? ay[oy] * az[oz] : D == 1 ? ax[ox] * az[oz] : ax[ox] * ay[oy];
    const CellV v = cell(ox, oy, oz);
    double s0 = v.sg;
    if (v.tf && w != 0.0) {
      const double t0 = th(0, 0, 0);
      const double t1 = D == 0 ? th(side ? 1 : -1, 0, 0) : D == 1 ? th(0, side ? 1 : -1, 0) : th(0, 0, side ? 1 : -1);
      s0 = s0 / (1.0 + tcr_of(v.m) * (0.5 * (t0 + t1)));
    }
    sg = fma(w, s0, sg);
    if (er_out) er = fma(w, v.er, er);
  }
  if (er_out) *er_out = er;
  return sg;
}

// Joule power density at the node from its six incident edges of field e:
//   P_n = sum_e 1/2 sigma_e e^2 L A / V_n = jf * sum_e a_e e^2 (L / dual width),
// with L / dual width = 2 alpha on the edge's side (0 for a missing edge).
// a[0..5], v[0..5]: own x, y, z then low-side x, y, z.
__device__ __forceinline__ double node_joule(const double (&a)[6], const double (&ax)[2], const double (&ay)[2],
                                             const double (&az)[2], const double (&v)[6], double jf) {
#pragma clang fp contract(off)
  double s = 0.0;
  s = fma(ax[1] * a[0], v[0] * v[0], s);
  s = fma(ay[1] * a[1], v[1] * v[1], s);
  s = fma(az[1] * a[2], v[2] * v[2], s);
  s = fma(ax[0] * a[3], v[3] * v[3], s);
  s = fma(ay[0] * a[4], v[4] * v[4], s);
  s = fma(az[0] * a[5], v[5] * v[5], s);
  return (2.0 * jf) * s;
}

// Conductances of the three low-side edges (for the Joule source).
template <typename CELL, typename TCR, typename TH>
__device__ __forceinline__ void low_coefs(const double (&ax)[2], const double (&ay)[2], const double (&az)[2],
                                          const CELL &cell, const TCR &tcr_of, const TH &th, double (&a)[6]) {
  a[3] = edge_coef<0>(0, ax, ay, az, cell, tcr_of, th, nullptr);
  a[4] = edge_coef<1>(0, ax, ay, az, cell, tcr_of, th, nullptr);
  a[5] = edge_coef<2>(0, ax, ay, az, cell, tcr_of, th, nullptr);
}

// The 8 cells around node (i,j,k) from global memory (cells outside the
// mesh read as material 0; their weights are 0).
struct GCell {
  const uint8_t *m;
  const double *mtab;
  int64_t n, sy, sz;
  int i, j, k, nx, ny, nz;
  __device__ __forceinline__ CellV operator()(int ox, int oy, int oz) const {
    const int ci = i - 1 + ox, cj = j - 1 + oy, ck = k - 1 + oz;
    const bool ok = !(ci < 0 || ci >= nx || cj < 0 || cj >= ny || ck < 0 || ck >= nz);
    const int mm = ok ? int(m[n + (ox - 1) + (oy - 1) * sy + (oz - 1) * sz]) : 0;
    const double *row = mtab + mm * kMatStride;
    CellV v;
    v.er = row[MC_EPSR];
    v.sg = row[MC_SIGS];
    v.tf = (row[MC_TCR] != 0.0 && v.sg != 0.0) ? 1 : 0;
    v.m = mm;
    return v;
  }
};
struct GTcr {
  const double *mtab;
  __device__ __forceinline__ double operator()(int m) const { return mtab[m * kMatStride + MC_TCR]; }
};
// The temperatures an own edge of the node reads, loaded beforehand: the
// node's and its +x, +y, +z neighbours'.
struct PTh {
  double t[4];
  __device__ __forceinline__ double operator()(int di, int dj, int dk) const {
    return di > 0 ? t[1] : dj > 0 ? t[2] : dk > 0 ? t[3] : t[0];
  }
};

// The per-material EM constants in LDS: eps_r, the scaled conductance
// (stored negated where sigma depends on T, so one load gives both) and the
// temperature coefficient.  Loaded once per block; every thread of the block
// must reach the barrier.
constexpr int kMatMax = 256;
struct LdsMat {
  double er[kMatMax], sg[kMatMax], tcr[kMatMax];
};
__device__ __forceinline__ void lds_mat_load(const DevGrid &g, LdsMat &M) {
  const int tid = threadIdx.x + threadIdx.y * blockDim.x, nt = blockDim.x * blockDim.y;
  for (int m = tid; m < g.n_mat; m += nt) {
    const double *row = g.mtab + m * kMatStride;
    const bool tf = row[MC_TCR] != 0.0 && row[MC_SIGS] != 0.0;
    M.er[m] = row[MC_EPSR];
    M.sg[m] = tf ? -row[MC_SIGS] : row[MC_SIGS];
    M.tcr[m] = row[MC_TCR];
  }
  __syncthreads();
}
// The 8 cells around a node by id (index ox + 2 oy + 4 oz), values from LDS;
// the same CellV as GCell gives for the same ids.
struct LCell {
  const LdsMat *M;
  int id[8];
  __device__ __forceinline__ CellV operator()(int ox, int oy, int oz) const {
    const int m = id[ox + 2 * oy + 4 * oz];
    const double sg = M->sg[m];
    CellV v;
    v.er = M->er[m];
    v.sg = fabs(sg);
    v.tf = sg < 0.0 ? 1 : 0;
    v.m = m;
    return v;
  }
};
struct LTcr {
  const LdsMat *M;
  __device__ __forceinline__ double operator()(int m) const { return M->tcr[m]; }
};

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

// Value at time t of a closed-form wave (the excitation scheme of Sec. III-B):
// a Ricker wavelet, a sine, or a Gaussian pulse train on a carrier, zero
// outside [t_on, t_off).  Record: kind, n_pulses, amp, t0, width, freq,
// t_on, t_off, pulse centres.
__device__ __forceinline__ double wave_value(const double *w, double t) {
  if (!(t >= w[6] && t < w[7])) return 0.0;
  const int kind = int(w[0]);
  const double amp = w[2], t0 = w[3], width = w[4], f = w[5];
  if (kind == ETM_WAVE_RICKER) {
    const double u = (t - t0) / width;
    const double a = u * u;
    return amp * (1.0 - 2.0 * a) * exp(-a);
  }
  if (kind == ETM_WAVE_SINE) return amp * sin(2.0 * M_PI * f * (t - t0));
  double env = 0.0;
  const int np = int(w[1]);
  for (int q = 0; q < np; ++q) {
    const double u = (t - w[8 + q]) / width;
    env += exp(-(u * u));
  }
  return amp * env * cos(2.0 * M_PI * f * (t - t0));
}

// Samples s = base .. base + kWaveBlock of every closed-form wave: J at
// t = (s - 1/2) dt, the same instants as a tabulated wave's samples.
__global__ __launch_bounds__(256) void wave_sample_kernel(const double *aw, int n, double dt, int64_t base,
                                                          double *Ja) {
  const int64_t per = kWaveBlock + 1;
  const int64_t id = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (id >= int64_t(n) * per) return;
  const int64_t w = id / per, q = id - w * per;
  Ja[id] = wave_value(aw + w * kWaveStride, (double(base + q) - 0.5) * dt);
}

// Source and lumped conductance of port edge q (from find_port) at this step.
// Port source of EM step n at an edge: jd = dt (J^{n+1/2} - J^{n-1/2}) / eps0
// (three-level form), jn = dt J^{n+1/2} / eps0 (leapfrog form), and the
// lumped conductance g (scaled like the a-coefficient).  J^{n+1/2} is the
// sampled value n+1 of a tabulated wave, or of a closed-form wave (sampled on
// the device, see wave_sample_kernel).
struct PortTerm {
  double jd, jn, g;
};
__device__ __forceinline__ PortTerm port_terms(const DevPorts &P, int q, int64_t step) {
  PortTerm r{0.0, 0.0, 0.0};
  if (q < 0) return r;
  r.g = P.gs[q];
  const int64_t s1 = step + 1, s0 = step, ns = P.n_samples;
  for (int t = P.start[q]; t < P.start[q + 1]; ++t) {
    const int w = P.wave[t];
    double j1, j0;
    if (w < P.n_table) {
      const double *Jw = P.J + int64_t(w) * ns;
      j1 = s1 < ns ? Jw[s1] : 0.0;
      j0 = s0 < ns ? Jw[s0] : 0.0;
    } else {
      const double *Jw = P.Ja + int64_t(w - P.n_table) * (kWaveBlock + 1) - P.a_base;
      j1 = Jw[s1];
      j0 = Jw[s0];
    }
    r.jd += P.wt[t] * (j1 - j0);
    r.jn += P.wt[t] * j1;
  }
  return r;
}

// The mixed path keeps each e component as an FP32 value plus an 8-bit
// residual: e = hi + lo * ulp(hi) / 256.  The stencil reads hi; the own-edge
// accumulation e^{n+1} = e^n + (e^{n+1} - e^n) runs on the full value, so
// the per-step rounding of e (which otherwise dominates the error of the
// temperature rise over long windows) is 256 times smaller.
// log2 of ulp(hi) / 256 (subnormals share the smallest binade's ulp)
__device__ __forceinline__ int lo_exp(float hi) {
  const int E = int((__float_as_uint(hi) >> 23) & 0xFFu);
  return max(E, 1) - 158;
}
__device__ __forceinline__ double e_join(float hi, int8_t lo) { return double(hi) + ldexp(double(lo), lo_exp(hi)); }
__device__ __forceinline__ void e_split(double x, float &hi, int8_t &lo) {
  hi = float(x);
  const double r = rint(ldexp(x - double(hi), -lo_exp(hi)));  // exact scaling by a power of two
  lo = int8_t(fmax(-128.0, fmin(127.0, r)));
}

// Face value of the leapfrog field h^{n+1/2} = h^{n-1/2} + c0 dt (curl e^n)
// (per unit area), from the face's four edge values in the fixed order
// (a - b) s + (c - d) t.  Every thread that needs a face computes it with
// this one expression, so a face computed at a tile or chunk border is
// bitwise the value its owner stores.
__device__ __forceinline__ float hface(float hold, float a, float b, double s, float c, float d, double t,
                                       double cdt) {
  const double q = __builtin_fma(double(a) - double(b), s, (double(c) - double(d)) * t);
  return float(__builtin_fma(cdt, q, double(hold)));
}

// 1/x in FP64: hardware reciprocal and two Newton steps (full precision).
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// LDS staging of one block: three e planes (k-1, k, k+1) of the 64 x 4 node
// column with a one-node halo.
template <typename T>
struct MarchSmem {
  T e[3][3][TYH][TXH];
};

template <typename T>
struct EmPtrs {
  const T *e;    // e^n (component c at + c*cs)
  const T *aux;  // FP64: e^{n-1};  mixed: h^{n-1/2} (faces: x-normal, y-normal, z-normal at + c*cs)
  T *oe;         // e^{n+1}
  T *oaux;       // mixed: h^{n+1/2}
};

// Joule power density at node n from the stored coefficients of its six
// incident edges and their field values v (own x, y, z, low x, y, z).  The
// same code serves the march kernel and the flush / thermal kernels.
// The mixed path stores 2a, so its conductances are halved (exactly) here.
template <typename T>
__device__ __forceinline__ double joule_from_coef(const T *cf, uint32_t cs, uint32_t n, uint32_t sy, uint32_t sz,
                                                  int i, int j, int k, const double (&ax)[2], const double (&ay)[2],
                                                  const double (&az)[2], const double (&v)[6], double jf) {
  const double h = sizeof(T) == 4 ? 0.5 : 1.0;
  const double a6[6] = {h * double(cf[3 * cs + n]), h * double(cf[4 * cs + n]), h * double(cf[5 * cs + n]),
                        i > 0 ? h * double(cf[3 * cs + n - 1]) : 0.0, j > 0 ? h * double(cf[4 * cs + n - sy]) : 0.0,
                        k > 0 ? h * double(cf[5 * cs + n - sz]) : 0.0};
  return node_joule(a6, ax, ay, az, v, jf);
}

// ---- FP64: the three-level form of Eq. (2)-(3) on (e^n, e^{n-1}) -----------
// One block: the 64 x 4 node column (tx, ty) over the z planes of chunk kc.
// Per plane: stage e plane k+1, update the own edges of the nodes of plane
// k from their stored coefficients, and gather the Joule power of e^n at the
// node from its six incident edges.
template <typename T>
__device__ __forceinline__ void em_march_tile(const EmLaunch &L, const EmPtrs<T> &p, int64_t step, int tx, int ty,
                                              int kc, int kchunk, int acc_joule, MarchSmem<T> &S) {
  const DevGrid &g = L.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const uint32_t sy = uint32_t(g.sy), sz = uint32_t(g.sz), cs = g.cs;
  const Geo G(g.geo, nx, ny, nz);
  const T *cf = static_cast<const T *>(L.coef);
  const int lx = threadIdx.x, ly = threadIdx.y, tid = ly * BX + lx;
  const int i0 = tx * BX, j0 = ty * BY;
  const int i = i0 + lx, j = j0 + ly;
  const int k0 = kc * kchunk, k1 = min(k0 + kchunk, nz + 1);
  auto load_plane = [&](int kk, int slot) {
    for (int t = tid; t < TYH * TXH; t += BX * BY) {
      const int r = t / TXH, c = t - r * TXH;
      const int gi = i0 - 1 + c, gj = j0 - 1 + r;
      const bool ok = kk >= 0 && kk <= nz && gi >= 0 && gi <= nx && gj >= 0 && gj <= ny;
      const uint32_t q = uint32_t(kk) * sz + uint32_t(gj) * sy + uint32_t(gi);
      S.e[slot][0][r][c] = ok ? p.e[q] : T(0);
      S.e[slot][1][r][c] = ok ? p.e[cs + q] : T(0);
      S.e[slot][2][r][c] = ok ? p.e[2 * cs + q] : T(0);
    }
  };
  // per-thread x / y factors (clamped indices; masks select the valid terms)
  const bool active = i <= nx && j <= ny;
  const int ic = min(i, nx), jc = min(j, ny);
  const double ax[2] = {G.axl[ic], G.axh[ic]}, ay[2] = {G.ayl[jc], G.ayh[jc]};
  const T idx_i = T(G.idx[min(ic, nx - 1)]), idx_m = T(G.idx[max(ic - 1, 0)]), ihx_i = T(G.ihx[ic]);
  const T idy_j = T(G.idy[min(jc, ny - 1)]), idy_m = T(G.idy[max(jc - 1, 0)]), ihy_j = T(G.ihy[jc]);
  const T vi0 = T(i > 0), vi1 = T(i < nx), vj0 = T(j > 0), vj1 = T(j < ny);
  const T c2 = T(L.c2dt2);
  const int pec = g.pec;
  const bool pec_i = (i == 0 && (pec & 1)) || (i == nx && (pec & 2));
  const bool pec_j = (j == 0 && (pec & 4)) || (j == ny && (pec & 8));
  // Plane k + 2 is fetched into registers while plane k is computed and
  // written to LDS at the top of the next iteration, so a block's global
  // loads overlap its own arithmetic instead of stalling at the barrier.
  constexpr int NPF = (TYH * TXH + BX * BY - 1) / (BX * BY);
  T pf[NPF][3];
  auto fetch = [&](int kk) {
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      const int t = tid + q * BX * BY;
      const int r = t / TXH, c = t - r * TXH;
      const int gi = i0 - 1 + c, gj = j0 - 1 + r;
      const bool ok = t < TYH * TXH && kk >= 0 && kk <= nz && gi >= 0 && gi <= nx && gj >= 0 && gj <= ny;
      const uint32_t qq = ok ? uint32_t(kk) * sz + uint32_t(gj) * sy + uint32_t(gi) : 0u;
      pf[q][0] = ok ? p.e[qq] : T(0);
      pf[q][1] = ok ? p.e[cs + qq] : T(0);
      pf[q][2] = ok ? p.e[2 * cs + qq] : T(0);
    }
  };
  auto commit = [&](int slot) {
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      const int t = tid + q * BX * BY;
      if (t < TYH * TXH) {
        const int r = t / TXH, c = t - r * TXH;
        S.e[slot][0][r][c] = pf[q][0];
        S.e[slot][1][r][c] = pf[q][1];
        S.e[slot][2][r][c] = pf[q][2];
      }
    }
  };
  int s_m = 0, s_0 = 1, s_p = 2;
  load_plane(k0 - 1, s_m);
  load_plane(k0, s_0);
  fetch(k0 + 1);
  for (int k = k0; k < k1; ++k) {
    commit(s_p);
    __syncthreads();
    if (k + 2 <= k1) fetch(k + 2);
    if (active) {
      const uint32_t n = uint32_t(k) * sz + uint32_t(j) * sy + uint32_t(i);
      const bool pec_k = (k == 0 && (pec & 16)) || (k == nz && (pec & 32));
      auto E = [&](int c, int di, int dj, int dk) -> T {
        const int sl = dk < 0 ? s_m : dk > 0 ? s_p : s_0;
        return S.e[sl][c][ly + 1 + dj][lx + 1 + di];
      };
      const uint8_t fla = g.flags[n], fl = fla & 7;
      const bool sg = fla & kFlagSigma;
      const T e0x = E(0, 0, 0, 0), e0y = E(1, 0, 0, 0), e0z = E(2, 0, 0, 0);
      const bool pec_d[3] = {pec_j || pec_k, pec_i || pec_k, pec_i || pec_j};
      const T idz_k = T(G.idz[min(k, nz - 1)]), idz_m = T(G.idz[max(k - 1, 0)]), ihz_k = T(G.ihz[k]);
      const T vk0 = T(k > 0), vk1 = T(k < nz);
      // curl-curl of e^n on the three own edges (faces outside the mesh masked to 0)
      const T hz_c = (e0x - E(0, 0, 1, 0)) * idy_j + (E(1, 1, 0, 0) - e0y) * idx_i;        // hz(i, j)
      const T hy_c = (e0z - E(2, 1, 0, 0)) * idx_i + (E(0, 0, 0, 1) - e0x) * idz_k;        // hy(i, k)
      const T hx_c = (E(2, 0, 1, 0) - e0z) * idy_j - (E(1, 0, 0, 1) - e0y) * idz_k;        // hx(j, k)
#pragma unroll
      for (int D = 0; D < 3; ++D) {
        const bool exists = D == 0 ? i < nx : D == 1 ? j < ny : k < nz;
        if (!exists) continue;
        const uint32_t o = D * cs + n;
        if (pec_d[D]) {
          p.oe[o] = T(0);
          continue;
        }
        T cc;
        if (D == 0) {
          const T hz_jm = (E(0, 0, -1, 0) - e0x) * idy_m + (E(1, 1, -1, 0) - E(1, 0, -1, 0)) * idx_i;
          const T hy_km = (E(2, 0, 0, -1) - E(2, 1, 0, -1)) * idx_i + (e0x - E(0, 0, 0, -1)) * idz_m;
          cc = (vj1 * hz_c - vj0 * hz_jm) * ihy_j - (vk1 * hy_c - vk0 * hy_km) * ihz_k;
        } else if (D == 1) {
          const T hx_km = (E(2, 0, 1, -1) - E(2, 0, 0, -1)) * idy_j - (e0y - E(1, 0, 0, -1)) * idz_m;
          const T hz_im = (E(0, -1, 0, 0) - E(0, -1, 1, 0)) * idy_j + (e0y - E(1, -1, 0, 0)) * idx_m;
          cc = (vk1 * hx_c - vk0 * hx_km) * ihz_k - (vi1 * hz_c - vi0 * hz_im) * ihx_i;
        } else {
          const T hy_im = (E(2, -1, 0, 0) - e0z) * idx_m + (E(0, -1, 0, 1) - E(0, -1, 0, 0)) * idz_k;
          const T hx_jm = (e0z - E(2, 0, -1, 0)) * idy_m - (E(1, 0, -1, 1) - E(1, 0, -1, 0)) * idz_k;
          cc = (vi1 * hy_c - vi0 * hy_im) * ihx_i - (vj1 * hx_c - vj0 * hx_jm) * ihy_j;
        }
        const T e0 = D == 0 ? e0x : D == 1 ? e0y : e0z;
        T er = cf[D * cs + n], a = sg ? cf[(3 + D) * cs + n] : T(0), jd = T(0);
        if (fl & (1 << D)) {
          const int q = find_port(L.ports, int64_t(D) * g.ntot + n);
          const PortTerm pt = port_terms(L.ports, q, step);
          a = T(double(a) + pt.g);
          jd = T(pt.jd);
        }
        const T inv = T(rcp64(double(er) + double(a)));
        p.oe[o] = (T(2) * er * e0 - c2 * cc - (er - a) * p.aux[o] - jd) * inv;
      }
      if (acc_joule && sg) {
        const double az[2] = {G.azl[k], G.azh[k]};
        const double v[6] = {double(e0x), double(e0y), double(e0z), double(E(0, -1, 0, 0)), double(E(1, 0, -1, 0)),
                             double(E(2, 0, 0, -1))};
        const double P = joule_from_coef(cf, cs, n, sy, sz, i, j, k, ax, ay, az, v, L.jf);
        if (P != 0.0) L.psum[n] += P;
      }
    }
    __syncthreads();
    const int t = s_m;
    s_m = s_0; s_0 = s_p; s_p = t;
  }
}

// ---- mixed: the same scheme as leapfrog on (e^n, h^{n-1/2}) ----------------
// Both fields are stored in FP32 and combined in FP64:
//   h^{n+1/2} = h^{n-1/2} + c0 dt curl e^n                       (faces)
//   (er + a) (e^{n+1} - e^n) = -2a e^n - c0 dt curl^T h^{n+1/2} - jn + K
// Eliminating h gives Eq. (2) exactly; K (per edge, zero until sigma changes)
// carries the difference the three-level form keeps when a changes at a
// thermal step.  Rounding errors of h reach e only through curl^T, so they
// never feed the gradient (static-charge) modes the curl-curl leaves
// undamped in dielectrics; the increment form e^{n+1} - e^n stored in FP32
// lets them accumulate.

// Per-node inputs of one plane for the edge update.
struct YeeNode {
  float er[3], a2[3], K[3];
  float a2xm, a2ym;  // 2a of the x-edge at i-1 and the y-edge at j-1 (Joule)
  int8_t lo[3];
  uint8_t fl;
};

// One wave per run of nodes, no barriers.  A wave owns WX = 62 consecutive
// nodes of a plane numbered x fastest (a run may cross the end of a row) and
// marches up its z-chunk on its own: lanes 0 and 63 overlap the neighbouring
// runs, so every x-neighbour a face or the Joule gather needs is one lane
// away (whole-wave DPP shifts).  The rows j - 1 and j + 1 of each lane's node
// are read directly (their own waves read the same lines, so they are L2
// hits), and the faces of row j - 1 that the edge update needs are
// recomputed in-wave with the same expression their owner uses.  No LDS and
// no barriers: each wave's loads for the next plane are in flight while it
// computes the current one, and its neighbours on the SIMD fill the gaps.
constexpr int WX = 62;

// Rows shorter than this are marched as runs over the x-fastest plane (no
// idle lanes at row ends); longer rows in tiles of BY rows, whose waves read
// each other's rows j +- 1 from the same L2 lines.  Measured on gfx950: the
// runs take the 256x256x64 slice from 125 to 113 us per step and a
// 608x608x64 package from 743 to 674 us, the tiles keep the 1024x1024x128
// package at 3.23 ms (3.35 ms as runs).
constexpr int kRunMaxRow = 1024;
__host__ __device__ inline bool em_runs(const DevGrid &g) {
  return g.layout == kLayoutRuns || (g.layout != kLayoutRows && g.nx + 1 < kRunMaxRow);
}

__device__ __forceinline__ float lane_next(float v) {  // value of lane + 1 (0 past the last lane)
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ float lane_prev(float v) {  // value of lane - 1 (0 before the first lane)
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}

struct RowE {  // e of one row and plane (x, y, z components)
  float x, y, z;
};

__device__ __forceinline__ void em_march_row_yee(const EmLaunch &L, const EmPtrs<float> &p, int64_t step, int ts,
                                                 int tr, int kc, int kchunk, int acc_joule) {
  const DevGrid &g = L.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const uint32_t sy = uint32_t(g.sy), sz = uint32_t(g.sz), cs = g.cs;
  const int lane = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.y));
  // Runs (short rows, em_runs): wave w owns the nodes t = WX w .. WX w + WX - 1
  // of the plane numbered x fastest (t = j (nx + 1) + i); lane L holds
  // t = WX w - 1 + L.  A run may cross the end of a row (the lane after node
  // (nx, j) holds (0, j + 1)): every term that would read across -- the faces
  // at i = nx, and through them the faces and x-edge at i - 1 of node 0 --
  // does not exist and is masked, so short rows leave no lanes idle.
  // Tiles (long rows): wave `wave` of block (ts, tr) owns nodes
  // i = WX ts .. WX ts + WX - 1 of row j = BY tr + wave; lane L holds
  // i = WX ts - 1 + L.  Either way lanes 0 and 63 overlap the neighbouring
  // waves and every x-neighbour is one lane away.
  const int nx1 = nx + 1, nplane = nx1 * (ny + 1);
  int tc;
  bool inb;
  if (em_runs(g)) {
    const int w = ts * BY + wave;
    if (WX * w >= nplane) return;  // the whole wave is past the plane
    const int t = WX * w - 1 + lane;
    inb = t >= 0 && t < nplane;
    tc = min(max(t, 0), nplane - 1);
  } else {
    const int jr = tr * BY + wave;
    if (jr > ny) return;
    const int ir = WX * ts - 1 + lane;
    inb = ir >= 0 && ir <= nx;
    tc = jr * nx1 + min(max(ir, 0), nx);
  }
  const Geo G(g.geo, nx, ny, nz);
  const float *cf = static_cast<const float *>(L.coef);
  const float *Kp = L.K;
  int8_t *elo = L.elo;
  const double cdt = L.cdt;
  const int j = tc / nx1, ic = tc - j * nx1;                // (clamped for lanes off the plane)
  const int i = inb ? ic : -1;
  const bool own = lane >= 1 && lane <= WX && inb;          // node updated by this lane
  const int k0 = kc * kchunk, k1 = min(k0 + kchunk, nz + 1);
  const bool jm_ok = j > 0, jp_ok = j < ny;                 // rows j - 1, j + 1 exist
  const uint32_t rj = uint32_t(j) * sy + uint32_t(ic);
  const uint32_t rm = jm_ok ? rj - sy : rj, rp = jp_ok ? rj + sy : rj;

  auto ld = [&](const float *base, int kk, uint32_t r, bool ok) -> float {
    const bool v = ok && inb && kk >= 0 && kk <= nz;
    const float x = base[v ? uint32_t(kk) * sz + r : 0u];
    return v ? x : 0.0f;
  };
  auto row3 = [&](int kk, uint32_t r, bool ok) -> RowE {
    return RowE{ld(p.e, kk, r, ok), ld(p.e + cs, kk, r, ok), ld(p.e + 2 * cs, kk, r, ok)};
  };

  // per-lane x and y factors
  const double dxi = G.idx[min(ic, nx - 1)], dhx = G.ihx[ic];
  const double ax[2] = {G.axl[ic], G.axh[ic]};
  const double dyj = G.idy[min(j, ny - 1)], dym = G.idy[max(j - 1, 0)], dhy = G.ihy[j];
  const double ay[2] = {G.ayl[j], G.ayh[j]};
  const int pec = g.pec;
  const bool pec_i = (i == 0 && (pec & 1)) || (i == nx && (pec & 2));
  const bool pec_j = (j == 0 && (pec & 4)) || (j == ny && (pec & 8));
  // faces that exist (independent of the plane, apart from k < nz)
  const bool fz = inb && i < nx && j < ny;         // z-normal (i, j)
  const bool fzm = inb && i < nx && jm_ok;         // z-normal (i, j - 1)
  const bool fy = inb && i < nx;                   // y-normal (i, j, k), k < nz
  const bool fx = inb && j < ny;                   // x-normal (i, j, k), k < nz
  const bool fxm = inb && jm_ok;                   // x-normal (i, j - 1, k), k < nz

  // A node with no conducting cell around it has 2a = 0 on its own edges,
  // on the y-edge of its j - 1 neighbour and (through the previous lane and
  // plane) on the other incident edges, and K = 0: a wave none of whose
  // nodes has a conducting cell skips those loads.  The test is wave-wide
  // (a scalar branch) and reads flags loaded one plane ahead, so no load
  // waits behind it; gating the loads lane by lane measured slower.
  auto load_flags = [&](int kk) -> uint8_t { return g.flags[uint32_t(min(kk, nz)) * sz + rj] & (7 | kFlagSigma); };
  auto load_node = [&](int kk, uint8_t flk, YeeNode &c) {
    const uint32_t n = uint32_t(kk) * sz + rj;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      c.er[d] = cf[d * cs + n];
      c.lo[d] = elo[d * cs + n];
    }
    c.fl = flk;
    c.a2xm = 0.0f;  // from the previous lane
    if (__any(flk & kFlagSigma)) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        c.a2[d] = cf[(3 + d) * cs + n];
        c.K[d] = Kp ? Kp[d * cs + n] : 0.0f;
      }
      c.a2ym = cf[4 * cs + uint32_t(kk) * sz + rm];
    } else {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        c.a2[d] = 0.0f;
        c.K[d] = 0.0f;
      }
      c.a2ym = 0.0f;
    }
  };
  struct Hold {
    float x, y, z, xm, zm;  // old faces at (i, j, k) and at (i, j - 1, k)
  };
  auto load_hold = [&](int kk, Hold &h) {
    const uint32_t kz = uint32_t(min(kk, nz)) * sz, n = kz + rj, m = kz + rm;
    h.x = p.aux[n];
    h.y = p.aux[cs + n];
    h.z = p.aux[2 * cs + n];
    h.xm = p.aux[m];
    h.zm = p.aux[2 * cs + m];
  };

  // ---- prologue
  RowE c0 = row3(k0, rj, true), m0 = row3(k0, rm, jm_ok);
  RowE c1 = row3(k0 + 1, rj, true), m1 = row3(k0 + 1, rm, jm_ok);
  float p0x = ld(p.e, k0, rp, jp_ok), p0z = ld(p.e + 2 * cs, k0, rp, jp_ok);
  float p1x = ld(p.e, k0 + 1, rp, jp_ok), p1z = ld(p.e + 2 * cs, k0 + 1, rp, jp_ok);
  YeeNode nd;
  load_node(k0, load_flags(k0), nd);
  uint8_t fl_next = load_flags(k0 + 1);  // flags of the plane after nd's
  Hold ho;
  load_hold(k0, ho);
  float ezm = 0.0f, hy_km = 0.0f, hx_km = 0.0f, a2zm = 0.0f;
  if (k0 > 0) {
    // the x- and y-edges of plane k0 need the x- and y-normal faces of plane k0 - 1
    const RowE cm = row3(k0 - 1, rj, true);
    const float pmz = ld(p.e + 2 * cs, k0 - 1, rp, jp_ok);
    const uint32_t n = uint32_t(k0 - 1) * sz + rj;
    const double dzm = G.idz[k0 - 1];
    const float hy = hface(p.aux[cs + n], cm.z, lane_next(cm.z), dxi, c0.x, cm.x, dzm, cdt);
    const float hx = hface(p.aux[n], pmz, cm.z, dyj, cm.y, c0.y, dzm, cdt);
    hy_km = fy ? hy : 0.0f;
    hx_km = fx ? hx : 0.0f;
    ezm = cm.z;
    a2zm = cf[5 * cs + n];
  }

#pragma unroll 2
  for (int k = k0; k < k1; ++k) {
    // next plane's e in flight while this plane is computed
    RowE c2{0.0f, 0.0f, 0.0f}, m2{0.0f, 0.0f, 0.0f};
    float p2x = 0.0f, p2z = 0.0f;
    if (k + 2 <= k1) {
      c2 = row3(k + 2, rj, true);
      m2 = row3(k + 2, rm, jm_ok);
      p2x = ld(p.e, k + 2, rp, jp_ok);
      p2z = ld(p.e + 2 * cs, k + 2, rp, jp_ok);
    }
    const uint32_t n = uint32_t(k) * sz + rj;
    const double dzk = G.idz[min(k, nz - 1)], dhz = G.ihz[k];
    const double az[2] = {G.azl[k], G.azh[k]};
    const bool kin = k < nz;
    // h^{n+1/2}: own faces and the z- and x-normal faces of row j - 1
    const float ey_n = lane_next(c0.y), ez_n = lane_next(c0.z), eym_n = lane_next(m0.y);
    float hz_c = hface(ho.z, c0.x, p0x, dyj, ey_n, c0.y, dxi, cdt);
    float hy_c = hface(ho.y, c0.z, ez_n, dxi, c1.x, c0.x, dzk, cdt);
    float hx_c = hface(ho.x, p0z, c0.z, dyj, c0.y, c1.y, dzk, cdt);
    float hz_jm = hface(ho.zm, m0.x, c0.x, dym, eym_n, m0.y, dxi, cdt);
    float hx_jm = hface(ho.xm, c0.z, m0.z, dym, m0.y, m1.y, dzk, cdt);
    hz_c = fz ? hz_c : 0.0f;
    hy_c = (fy && kin) ? hy_c : 0.0f;
    hx_c = (fx && kin) ? hx_c : 0.0f;
    hz_jm = fzm ? hz_jm : 0.0f;
    hx_jm = (fxm && kin) ? hx_jm : 0.0f;
    const float hz_im = lane_prev(hz_c), hy_im = lane_prev(hy_c);
    if (own && fz) p.oaux[2 * cs + n] = hz_c;
    if (own && fy && kin) p.oaux[cs + n] = hy_c;
    if (own && fx && kin) p.oaux[n] = hx_c;
    if (k + 1 < k1) load_hold(k + 1, ho);

    // e^{n+1} on the own x-, y-, z-edges
    const bool pec_k = (k == 0 && (pec & 16)) || (k == nz && (pec & 32));
    const bool pec_d[3] = {pec_j || pec_k, pec_i || pec_k, pec_i || pec_j};
    const bool ex_d[3] = {own && i < nx, own && j < ny, own && kin};
    const double cc[3] = {
        (double(hz_c) - double(hz_jm)) * dhy - (double(hy_c) - double(hy_km)) * dhz,
        (double(hx_c) - double(hx_km)) * dhz - (double(hz_c) - double(hz_im)) * dhx,
        (double(hy_c) - double(hy_im)) * dhx - (double(hx_c) - double(hx_jm)) * dhy};
    const float e0[3] = {c0.x, c0.y, c0.z};
#pragma unroll
    for (int D = 0; D < 3; ++D) {
      // 1/(er + a) is formed here in FP64 from the stored er and 2a, so the
      // recurrence is exactly Eq. (2) for the stored pair: two separately
      // rounded FP32 coefficients would perturb the multiplier (er - a) /
      // (er + a) of the odd-even mode of good conductors (a ~ 1e4) by ~1e-7
      // per step.
      double er = double(nd.er[D]), a2 = double(nd.a2[D]), jn = 0.0;
      if (nd.fl & (1 << D)) {
        const int q = find_port(L.ports, int64_t(D) * g.ntot + n);
        if (q >= 0) {
          const PortTerm pt = port_terms(L.ports, q, step);
          a2 = 2.0 * (0.5 * a2 + pt.g);
          er = L.ports.er[q];
          jn = pt.jn;
        }
      }
      const double inv = rcp64(er + 0.5 * a2);
      // the loss term takes the full e (FP32 part + residual): in a good
      // conductor 2a / (er + a) ~ 2, so a residual left out of it would come
      // back into e at FP32 size every step
      const double ef = e_join(e0[D], nd.lo[D]);
      const double dl = -(a2 * ef + cdt * cc[D] + jn - double(nd.K[D])) * inv;
      float eh;
      int8_t el;
      e_split(ef + dl, eh, el);
      if (pec_d[D]) {
        eh = 0.0f;
        el = 0;
      }
      if (ex_d[D]) {
        p.oe[D * cs + n] = eh;
        elo[D * cs + n] = el;
      }
    }
    // Joule power of e^n at the node, from its six incident edges
    const float a2xm = lane_prev(nd.a2[0]), exm = lane_prev(c0.x);
    if (acc_joule && own && (nd.fl & kFlagSigma)) {
      const double a6[6] = {0.5 * double(nd.a2[0]), 0.5 * double(nd.a2[1]), 0.5 * double(nd.a2[2]),
                            i > 0 ? 0.5 * double(a2xm) : 0.0, jm_ok ? 0.5 * double(nd.a2ym) : 0.0,
                            k > 0 ? 0.5 * double(a2zm) : 0.0};
      const double v[6] = {double(c0.x), double(c0.y), double(c0.z), double(exm), double(m0.y), double(ezm)};
      const double P = node_joule(a6, ax, ay, az, v, L.jf);
      // one thread per node: the add is not contended and its result is the plain sum
      if (P != 0.0) unsafeAtomicAdd(L.psum + n, P);
    }
    ezm = c0.z;
    hy_km = hy_c;
    hx_km = hx_c;
    a2zm = nd.a2[2];
    if (k + 1 < k1) {
      load_node(k + 1, fl_next, nd);
      fl_next = load_flags(k + 2);
    }
    c0 = c1; c1 = c2;
    m0 = m1; m1 = m2;
    p0x = p1x; p0z = p1z; p1x = p2x; p1z = p2z;
  }
}

template <typename T, bool YEE>
__device__ __forceinline__ void march_tile(const EmLaunch &L, const EmPtrs<T> &p, int64_t step, int tx, int ty, int kc,
                                           int kchunk, int acc_joule) {
  if constexpr (YEE) {
    em_march_row_yee(L, p, step, tx, ty, kc, kchunk, acc_joule);
  } else {
    __shared__ MarchSmem<T> S;
    em_march_tile<T>(L, p, step, tx, ty, kc, kchunk, acc_joule, S);
  }
}

template <typename T, bool YEE>
__global__ __launch_bounds__(256) void em_march_kernel(EmLaunch L, EmPtrs<T> p, int ntx, int nty, int nkc, int kchunk,
                                                       int acc_joule) {
  const int nb = ntx * nty * nkc;
  const int b = xcd_remap(blockIdx.x, nb);
  const int tx = b % ntx, ty = (b / ntx) % nty, kc = b / (ntx * nty);
  march_tile<T, YEE>(L, p, L.step, tx, ty, kc, kchunk, acc_joule);
}

// ---- two steps as a wavefront over z-slabs (temporal blocking) -------------
// One launch runs the tiles of two z-ranges of chunks: blocks [0, nA) make
// step n on chunks [kcA, kcA + nkcA) with pointer set pa, blocks [nA, nb)
// make step n + 1 on chunks [kcB, kcB + nkcB) with pb.  The host orders the
// launches so that the n + 1 range runs only after the step-n tiles it
// reads (its own slab and the planes next to it) are complete and after
// every step-n tile that reads the planes it overwrites; see
// launch_em_pair_schedule.  Each tile computes exactly what it computes in
// a one-step launch, so the two steps are bitwise those of two launches.
template <typename T, bool YEE>
__global__ __launch_bounds__(256) void em_march_pair_kernel(EmLaunch L, EmPtrs<T> pa, EmPtrs<T> pb, int ntx, int nty,
                                                            int kcA, int nkcA, int kcB, int nkcB, int kchunk,
                                                            int acc_a) {
  const int cols = ntx * nty, nA = cols * nkcA, nb = nA + cols * nkcB;
  const int b = xcd_remap(blockIdx.x, nb);
  const bool second = b >= nA;
  const int r = second ? b - nA : b;
  const int tx = r % ntx, ty = (r / ntx) % nty, kc = (second ? kcB : kcA) + r / cols;
  if (second)
    march_tile<T, YEE>(L, pb, L.step + 1, tx, ty, kc, kchunk, 1);
  else
    march_tile<T, YEE>(L, pa, L.step, tx, ty, kc, kchunk, acc_a);
}

// ---- batched: one launch walks the (variant, tile) list of all variants ----
// Item = (variant, tile x, tile y, z chunk).  The step offset s is read from
// device memory so that a captured chunk of steps can be replayed.  Held to
// 4 waves per SIMD (at most 128 VGPRs): the FP64 instance otherwise takes
// 129 and drops to 3, which cost about 8 % of the served designs per hour.
template <typename T, bool YEE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void em_march_batched(const BatchVar *vars, const int4 *items, int n_items,
                                                        const int64_t *step_ctr) {
  const int b = xcd_remap(blockIdx.x, n_items);
  const int4 it = items[b];
  const BatchVar &V = vars[it.x];
  const int64_t s = *step_ctr;
  const int64_t step = V.step0 + s;
  EmPtrs<T> p;
  if (YEE) {
    const int cur = int((V.cur0 + s) & 1), o = 1 - cur;
    p.e = (const T *)V.e[cur][0];
    p.aux = (const T *)V.h[cur][0];
    p.oe = (T *)V.e[o][0];
    p.oaux = (T *)V.h[o][0];
  } else {
    const int cur = int((V.cur0 + s) % 3), prv = (cur + 2) % 3, nxt = (cur + 1) % 3;
    p.e = (const T *)V.e[cur][0];
    p.aux = (const T *)V.e[prv][0];
    p.oe = (T *)V.e[nxt][0];
    p.oaux = nullptr;
  }
  const int acc = (s == 0) ? V.acc_joule0 : int(step % V.R != 0);
  march_tile<T, YEE>(V.L, p, step, it.y, it.z, it.w, V.kchunk, acc);
}

__global__ void step_ctr_kernel(int64_t *ctr, int64_t v, int set) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *ctr = set ? v : *ctr + v;
}

// ---- block reductions (wave64 shuffles, then LDS across the waves) --------
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
__device__ __forceinline__ void block_reduce_store(const double (&sums)[NS], const double (&maxs)[NM], double *out) {
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

inline dim3 node_grid(const DevGrid &g) { return dim3((g.nx + 1 + BX - 1) / BX, (g.ny + 1 + BY - 1) / BY, g.nz + 1); }

// Node tiles of BX x BY nodes of one plane, one block each, as a 1D grid
// whose logical tile t = (tile row * tiles per row + tile) * planes + k runs
// through the planes of one column of tiles first; each XCD takes a
// contiguous range of t.  The blocks that read a plane's values as their z
// neighbours then run beside the block that owns it, on the same L2.
inline dim3 node_grid_z(const DevGrid &g) {
  const dim3 d = node_grid(g);
  return dim3(d.x * d.y * d.z);
}
__device__ __forceinline__ void node_tile_z(const DevGrid &g, int &i, int &j, int &k) {
  const int nbx = (g.nx + 1 + BX - 1) / BX, nk = g.nz + 1;
  const int t = xcd_remap(int(blockIdx.x), int(gridDim.x));
  k = t % nk;
  const int c = t / nk;
  i = (c % nbx) * BX + int(threadIdx.x);
  j = (c / nbx) * BY + int(threadIdx.y);
}

// Joule of the current field (the deferred last step) at node (i,j,k), with
// the same arithmetic as the march kernel (missing low-side edges read 0).
template <typename T>
__device__ __forceinline__ double pending_joule(const DevGrid &g, const T *const *e, const T *cf, int i, int j, int k,
                                                int64_t n, double jf) {
  const double ax[2] = {g.al[0][i], g.ah[0][i]}, ay[2] = {g.al[1][j], g.ah[1][j]}, az[2] = {g.al[2][k], g.ah[2][k]};
  const double v[6] = {double(e[0][n]), double(e[1][n]), double(e[2][n]), i > 0 ? double(e[0][n - 1]) : 0.0,
                       j > 0 ? double(e[1][n - g.sy]) : 0.0, k > 0 ? double(e[2][n - g.sz]) : 0.0};
  return joule_from_coef(cf, g.cs, uint32_t(n), uint32_t(g.sy), uint32_t(g.sz), i, j, k, ax, ay, az, v, jf);
}

// Per-node coefficients of the own x, y, z edges: eps_r and the normalised
// material conductance a = dt sigma(T) / (2 eps0), formed in FP64 from the
// cells around the node (their ids read once, the material table in LDS) and
// stored at the field precision.  An edge that does not exist keeps eps_r =
// 1 and a = 0 and reads no temperature.
template <typename T>
__global__ __launch_bounds__(256) void coef_kernel(DevGrid g, DevPorts P, const T *th, T *cf, CoefK ck) {
  __shared__ LdsMat MT;
  int i, j, k;
  node_tile_z(g, i, j, k);
  const bool in = i <= g.nx && j <= g.ny;
  const int64_t n = in ? int64_t(k) * g.sz + int64_t(j) * g.sy + i : 0;
  // after a temperature change only edges next to a cell whose sigma depends
  // on it change (eps_r never does); a block without such a node leaves
  // before it loads the material table
  const bool work = in && (!ck.tcr_only || (g.flags[n] & kFlagTcr));
  if (!__syncthreads_or(work)) return;
  lds_mat_load(g, MT);
  if (!work) return;
  const double ax[2] = {g.al[0][i], g.ah[0][i]}, ay[2] = {g.al[1][j], g.ah[1][j]}, az[2] = {g.al[2][k], g.ah[2][k]};
  LCell CL;
  CL.M = &MT;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int ox = q & 1, oy = (q >> 1) & 1, oz = q >> 2;
    const int ci = i - 1 + ox, cj = j - 1 + oy, ck2 = k - 1 + oz;
    const bool ok = ci >= 0 && ci < g.nx && cj >= 0 && cj < g.ny && ck2 >= 0 && ck2 < g.nz;
    CL.id[q] = ok ? int(g.mat[n + (ox - 1) + (oy - 1) * g.sy + (oz - 1) * g.sz]) : 0;
  }
  const LTcr TC{&MT};
  const bool ex[3] = {i < g.nx, j < g.ny, k < g.nz};
  // every load up front: the temperatures the own edges may read and, for a
  // K update, the old 2a, K and the two fields (clamped where an edge does
  // not exist), so none waits behind a branch
  const PTh TH{{double(th[n]), double(th[ex[0] ? n + 1 : n]), double(th[ex[1] ? n + g.sy : n]),
                double(th[ex[2] ? n + g.sz : n])}};
  const uint32_t cs = g.cs;
  float a2o[3] = {0.0f, 0.0f, 0.0f}, Ko[3] = {0.0f, 0.0f, 0.0f}, ec[3] = {0.0f, 0.0f, 0.0f},
        ep[3] = {0.0f, 0.0f, 0.0f};
  if (sizeof(T) == 4 && ck.K) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const uint32_t o = d * cs + uint32_t(n);
      a2o[d] = float(cf[(3 + d) * cs + n]);
      Ko[d] = ck.K[o];
      ec[d] = ck.e_cur[o];
      ep[d] = ck.e_prev[o];
    }
  }
  double er[3] = {1.0, 1.0, 1.0}, a[3] = {0.0, 0.0, 0.0};
  if (ex[0]) a[0] = edge_coef<0>(1, ax, ay, az, CL, TC, TH, &er[0]);
  if (ex[1]) a[1] = edge_coef<1>(1, ax, ay, az, CL, TC, TH, &er[1]);
  if (ex[2]) a[2] = edge_coef<2>(1, ax, ay, az, CL, TC, TH, &er[2]);
  const uint8_t fl = g.flags[n];
  for (int d = 0; d < 3; ++d) {
    const double e = er[d] > 0.0 ? er[d] : 1.0;  // an edge without cells keeps a harmless 1
    if (sizeof(T) == 4) {
      const float a2 = float(2.0 * a[d]);
      if (ck.K && ex[d]) {
        // leapfrog form: a changed from a_old to a between e_prev = e^{n-1}
        // and e_cur = e^n; K += (a - a_old) (e^n + e^{n-1})
        if (a2 != a2o[d]) {
          const uint32_t o = d * cs + uint32_t(n);
          ck.K[o] = float(double(Ko[d]) + 0.5 * (double(a2) - double(a2o[d])) * (double(ec[d]) + double(ep[d])));
        }
      }
      cf[d * cs + n] = T(e);
      cf[(3 + d) * cs + n] = T(a2);
    } else {
      cf[d * cs + n] = T(e);
      cf[(3 + d) * cs + n] = T(a[d]);
    }
    if (fl & (1 << d)) {
      const int q = find_port(P, int64_t(d) * g.ntot + n);
      if (q >= 0) P.er[q] = e;
    }
  }
}

// ---- thermal step, Eq. (5) ------------------------------------------------
// C_n V_n (theta' - theta) = dt*psum*V_n - R*dt*sum_e G_e (theta_n - theta_m),
// G_e = sum over the edge's cells of (quarter transverse area) k_c / L,
// C_n V_n = sum over the node's cell octants of rho_cp * octant volume.
// The pending Joule power of the block's last EM step is added first, with
// the conductivity of the temperature the block ran at.
// The thermal constants (k, rho c_p) of every material in LDS.
struct LdsTherm {
  double k[kMatMax], rc[kMatMax];
};
__device__ __forceinline__ void lds_therm_load(const DevGrid &g, LdsTherm &M) {
  const int tid = threadIdx.x + threadIdx.y * blockDim.x, nt = blockDim.x * blockDim.y;
  for (int m = tid; m < g.n_mat; m += nt) {
    M.k[m] = g.mtab[m * kMatStride + MC_K];
    M.rc[m] = g.mtab[m * kMatStride + MC_RHOCP];
  }
  __syncthreads();
}

// The thermal step of node (i, j, k) in two parts: every load is issued
// first (out-of-mesh neighbours, cells and edges read the node's own entry
// at a clamped index and are masked to zero afterwards, so no load sits
// behind a branch), then the arithmetic, in the same order as with branches
// (adding the masked zeros leaves the sums unchanged).
struct ThermIn {
  double dxs[2], dys[2], dzs[2], ixs[2], iys[2], izs[2], V;
  int id[8];
  double t0, txl, txh, tyl, tyh, tzl, tzh, ps;
  double ax[2], ay[2], az[2], a6[6], v[6];
};
template <typename T>
__device__ __forceinline__ void thermal_load(const ThermalLaunch &L, const T *const *e, const T *cf, int i, int j,
                                             int k, int64_t n, ThermIn &q) {
  const DevGrid &g = L.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int64_t sy = g.sy, sz = g.sz;
  const bool xl = i > 0, xh = i < nx, yl = j > 0, yh = j < ny, zl = k > 0, zh = k < nz;
  const int il = xl ? i - 1 : 0, ih = xh ? i : nx - 1, jl = yl ? j - 1 : 0, jh = yh ? j : ny - 1;
  const int kl = zl ? k - 1 : 0, kh = zh ? k : nz - 1;
  q.dxs[0] = g.dx[il]; q.dxs[1] = g.dx[ih]; q.dys[0] = g.dy[jl]; q.dys[1] = g.dy[jh];
  q.dzs[0] = g.dz[kl]; q.dzs[1] = g.dz[kh];
  q.ixs[0] = g.idx[il]; q.ixs[1] = g.idx[ih]; q.iys[0] = g.idy[jl]; q.iys[1] = g.idy[jh];
  q.izs[0] = g.idz[kl]; q.izs[1] = g.idz[kh];
  q.V = g.hx[i] * g.hy[j] * g.hz[k];
  const bool vx[2] = {xl, xh}, vy[2] = {yl, yh}, vz[2] = {zl, zh};
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int ox = c & 1, oy = (c >> 1) & 1, oz = c >> 2;
    const bool ok = vx[ox] && vy[oy] && vz[oz];
    const int m = int(g.mat[ok ? n + (ox - 1) + (oy - 1) * sy + (oz - 1) * sz : n]);
    q.id[c] = ok ? m : -1;
  }
  q.t0 = L.theta_in[n];
  q.txl = L.theta_in[xl ? n - 1 : n]; q.txh = L.theta_in[xh ? n + 1 : n];
  q.tyl = L.theta_in[yl ? n - sy : n]; q.tyh = L.theta_in[yh ? n + sy : n];
  q.tzl = L.theta_in[zl ? n - sz : n]; q.tzh = L.theta_in[zh ? n + sz : n];
  q.ps = L.psum[n];
  if (L.acc_joule) {
    // the pending Joule power of the current field (as joule_from_coef)
    const uint32_t cs = g.cs;
    const double h = sizeof(T) == 4 ? 0.5 : 1.0;
    q.ax[0] = g.al[0][i]; q.ax[1] = g.ah[0][i]; q.ay[0] = g.al[1][j]; q.ay[1] = g.ah[1][j];
    q.az[0] = g.al[2][k]; q.az[1] = g.ah[2][k];
    const double exl = double(e[0][xl ? n - 1 : n]), eyl = double(e[1][yl ? n - sy : n]),
                 ezl = double(e[2][zl ? n - sz : n]);
    const double a3 = double(cf[3 * cs + (xl ? n - 1 : n)]), a4 = double(cf[4 * cs + (yl ? n - sy : n)]),
                 a5 = double(cf[5 * cs + (zl ? n - sz : n)]);
    q.v[0] = double(e[0][n]); q.v[1] = double(e[1][n]); q.v[2] = double(e[2][n]);
    q.v[3] = xl ? exl : 0.0; q.v[4] = yl ? eyl : 0.0; q.v[5] = zl ? ezl : 0.0;
    q.a6[0] = h * double(cf[3 * cs + n]); q.a6[1] = h * double(cf[4 * cs + n]); q.a6[2] = h * double(cf[5 * cs + n]);
    q.a6[3] = xl ? h * a3 : 0.0; q.a6[4] = yl ? h * a4 : 0.0; q.a6[5] = zl ? h * a5 : 0.0;
  }
}

__device__ __forceinline__ void thermal_node(const ThermalLaunch &L, const LdsTherm &M, const ThermIn &q, int i,
                                             int j, int k, int64_t n, double &e_part, double &m_part) {
  const DevGrid &g = L.g;
  double ps = q.ps;
  if (L.acc_joule) {
    const double P = node_joule(q.a6, q.ax, q.ay, q.az, q.v, L.jf);
    if (P != 0.0) ps += P;
  }
  double CV = 0.0, gx0 = 0, gx1 = 0, gy0 = 0, gy1 = 0, gz0 = 0, gz1 = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int ox = c & 1, oy = (c >> 1) & 1, oz = c >> 2;
    const bool ok = q.id[c] >= 0;
    const int m = ok ? q.id[c] : 0;
    const double ddx = q.dxs[ox], ddy = q.dys[oy], ddz = q.dzs[oz], kc = M.k[m];
    const double cv = M.rc[m] * 0.125 * ddx * ddy * ddz;
    const double wx = 0.25 * ddy * ddz * kc * q.ixs[ox], wy = 0.25 * ddx * ddz * kc * q.iys[oy],
                 wz = 0.25 * ddx * ddy * kc * q.izs[oz];
    if (ok) {
      CV += cv;
      if (ox) gx1 += wx; else gx0 += wx;
      if (oy) gy1 += wy; else gy0 += wy;
      if (oz) gz1 += wz; else gz0 += wz;
    }
  }
  const double t0 = q.t0;
  double flux = 0.0;
  if (i > 0) flux += gx0 * (t0 - q.txl);
  if (i < g.nx) flux += gx1 * (t0 - q.txh);
  if (j > 0) flux += gy0 * (t0 - q.tyl);
  if (j < g.ny) flux += gy1 * (t0 - q.tyh);
  if (k > 0) flux += gz0 * (t0 - q.tzl);
  if (k < g.nz) flux += gz1 * (t0 - q.tzh);
  const double tn = t0 + (L.dt * ps * q.V - double(L.R) * L.dt * flux) / CV;
  L.theta_out[n] = tn;
  L.psum[n] = 0.0;
  if (L.theta32) L.theta32[n] = float(tn);
  e_part = L.dt * ps * q.V;
  m_part = tn;
}

// One thread per node, one block per 64 x 4 node tile of a plane (node_tile_z
// order).  The node's loads are issued before the block loads the material
// table into LDS and meets at the barrier.
template <typename T>
__global__ __launch_bounds__(256) void thermal_kernel(ThermalLaunch L, const T *e0, const T *e1, const T *e2,
                                                      const T *cf) {
  __shared__ LdsTherm MT;
  const DevGrid &g = L.g;
  int i, j, k;
  node_tile_z(g, i, j, k);
  const bool in = i <= g.nx && j <= g.ny;
  const int64_t n = in ? int64_t(k) * g.sz + int64_t(j) * g.sy + i : 0;
  ThermIn q;
  if (in) {
    const T *e[3] = {e0, e1, e2};
    thermal_load<T>(L, e, cf, i, j, k, n, q);
  }
  lds_therm_load(g, MT);
  double e_part = 0.0, m_part = -1.0e300;
  if (in) {
    thermal_node(L, MT, q, i, j, k, n, e_part, m_part);
    // the max reduction (fmax) drops NaN: carry a non-finite temperature
    // in the energy sum, which the finalize kernel checks
    if (!isfinite(m_part)) e_part = m_part - m_part;
  }
  const double s[1] = {e_part}, m[1] = {m_part};
  block_reduce_store<1, 1>(s, m, L.partials + int64_t(blockIdx.x) * kRedWidth);
}

// Add the pending Joule power of the current field to psum.
template <typename T>
__global__ __launch_bounds__(256) void joule_flush_kernel(DevGrid g, const T *e0, const T *e1, const T *e2,
                                                          const T *cf, double *psum, double jf) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  if (i > g.nx || j > g.ny) return;
  const int64_t n = int64_t(k) * g.sz + int64_t(j) * g.sy + i;
  const T *e[3] = {e0, e1, e2};
  const double P = pending_joule<T>(g, e, cf, i, j, k, n, jf);
  if (P != 0.0) psum[n] += P;
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

// First stage of a two-stage reduction: block b folds rows [b per, (b+1) per)
// of the partials, in a fixed order, into row b of out.
__global__ __launch_bounds__(256) void reduce_rows_kernel(const double *part, int64_t nb, int64_t per, int n_sum,
                                                          int n_max, double *out) {
  __shared__ double o[kRedWidth];
  const int64_t b0 = int64_t(blockIdx.x) * per, b1 = b0 + per < nb ? b0 + per : nb;
  reduce_partials(part + b0 * kRedWidth, b1 > b0 ? b1 - b0 : 0, n_sum, n_max, o);
  if (threadIdx.x == 0)
    for (int q = 0; q < n_sum + n_max; ++q) out[int64_t(blockIdx.x) * kRedWidth + q] = o[q];
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
template <typename T>
__global__ __launch_bounds__(256) void diag_kernel(DiagLaunch L) {
  const DevGrid &g = L.g;
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  double w_part = 0.0, j_part = 0.0, m_part = -1.0e300;
  if (i <= g.nx && j <= g.ny) {
    const int64_t n = int64_t(k) * g.sz + int64_t(j) * g.sy + i;
    const T *en[3] = {(const T *)L.e_new[0], (const T *)L.e_new[1], (const T *)L.e_new[2]};
    const T *eo[3] = {(const T *)L.e_old[0], (const T *)L.e_old[1], (const T *)L.e_old[2]};
    const double ax[2] = {g.al[0][i], g.ah[0][i]}, ay[2] = {g.al[1][j], g.ah[1][j]}, az[2] = {g.al[2][k], g.ah[2][k]};
    GCell CL{g.mat, g.mtab, n, g.sy, g.sz, i, j, k, g.nx, g.ny, g.nz};
    GTcr TC{g.mtab};
    auto zero_th = [](int, int, int) { return 0.0; };
    double er3[3];
    (void)edge_coef<0>(1, ax, ay, az, CL, TC, zero_th, &er3[0]);
    (void)edge_coef<1>(1, ax, ay, az, CL, TC, zero_th, &er3[1]);
    (void)edge_coef<2>(1, ax, ay, az, CL, TC, zero_th, &er3[2]);
    double acc = 0.0;
    for (int D = 0; D < 3; ++D) {
      if ((D == 0 && i == g.nx) || (D == 1 && j == g.ny) || (D == 2 && k == g.nz)) continue;
      if (pec_edge(g, D, i, j, k)) continue;
      GAcc<T> E{{eo[0], eo[1], eo[2]}, n, g.sy, g.sz};
      const double cc = D == 0 ? double(curl_x<T>(g, E, i, j, k))
                               : D == 1 ? double(curl_y<T>(g, E, i, j, k)) : double(curl_z<T>(g, E, i, j, k));
      const double Lh = D == 0 ? g.dx[i] : D == 1 ? g.dy[j] : g.dz[k];
      const double A = D == 0 ? g.hy[j] * g.hz[k] : D == 1 ? g.hx[i] * g.hz[k] : g.hx[i] * g.hy[j];
      const double e1 = double(en[D][n]);
      const double dl = e1 - double(eo[D][n]);
      acc += Lh * A * (er3[D] * dl * dl + L.c2dt2 * e1 * cc);
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
__global__ void pack_kernel(const void *src, int src_f32, int64_t sy, int64_t sz, int ni, int nj, int nk, double *dst) {
  const int64_t total = int64_t(ni) * nj * nk;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    const int i = int(t % ni);
    const int64_t r = t / ni;
    const int j = int(r % nj), k = int(r / nj);
    const int64_t s = int64_t(k) * sz + int64_t(j) * sy + i;
    dst[t] = src_f32 ? double(((const float *)src)[s]) : ((const double *)src)[s];
  }
}

__global__ void unpack_kernel(const double *src, int ni, int nj, int nk, void *dst, int dst_f32, int64_t sy, int64_t sz) {
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

}  // namespace

void em_tiles(const DevGrid &g, int precision, int kchunk, int *ntx, int *nty, int *nkc) {
  if (precision == ETM_PREC_MIXED && em_runs(g)) {
    // BY runs of WX nodes of the x-fastest plane per block, one row of blocks
    const int64_t plane = int64_t(g.nx + 1) * (g.ny + 1), per = int64_t(WX) * BY;
    *ntx = int((plane + per - 1) / per);
    *nty = 1;
  } else if (precision == ETM_PREC_MIXED) {
    // BY rows of WX nodes per block
    *ntx = (g.nx + 1 + WX - 1) / WX;
    *nty = (g.ny + 1 + BY - 1) / BY;
  } else {
    // BX x BY node tiles
    *ntx = (g.nx + 1 + BX - 1) / BX;
    *nty = (g.ny + 1 + BY - 1) / BY;
  }
  *nkc = (g.nz + 1 + kchunk - 1) / kchunk;
}

int em_kchunk(const DevGrid &g, int precision) {
  // Planes per block, from sweeps on gfx950 in both precisions: on the
  // 256x256x64 slice 6 planes beat 4, 8, 10, 12 and 16 (124 against 131 us
  // per mixed step at 8), on the 1024x1024x128 package 12 beat 8, 16, 24
  // and 32 (3.27 against 3.48 ms at 16).  Long chunks on many columns, short
  // ones otherwise, and shorter still (down to 4) while a launch would have
  // fewer than 2048 blocks to spread over the 256 CUs.
  int ntx, nty, nkc;
  em_tiles(g, precision, 1, &ntx, &nty, &nkc);
  const int64_t cols = int64_t(ntx) * nty;
  int kc = cols * ((g.nz + 1 + 11) / 12) >= 8192 ? 12 : 6;
  while (kc > 4 && cols * ((g.nz + 1 + kc - 1) / kc) < 2048) kc = std::max(4, kc - 2);
  return kc;
}

hipError_t launch_em_step(const EmLaunch &L, hipStream_t s) {
  int ntx, nty, nkc;
  const int kc = L.kchunk > 0 ? L.kchunk : em_kchunk(L.g, L.precision);
  em_tiles(L.g, L.precision, kc, &ntx, &nty, &nkc);
  const int nb = ntx * nty * nkc;
  const dim3 block(BX, BY, 1);
  if (L.precision == ETM_PREC_FP64) {
    EmPtrs<double> p{(const double *)L.e0[0], (const double *)L.e1[0], (double *)L.out0[0], nullptr};
    hipLaunchKernelGGL((em_march_kernel<double, false>), dim3(nb), block, 0, s, L, p, ntx, nty, nkc, kc, L.acc_joule);
  } else {
    EmPtrs<float> p{(const float *)L.e0[0], (const float *)L.e1[0], (float *)L.out0[0], (float *)L.out1[0]};
    hipLaunchKernelGGL((em_march_kernel<float, true>), dim3(nb), block, 0, s, L, p, ntx, nty, nkc, kc, L.acc_joule);
  }
  return hipGetLastError();
}

// Steps n and n + 1 (La: pointers and Joule flag of step n; Lb: pointers of
// step n + 1) as a wavefront over n_slabs z-slabs of whole chunks.  Launch t
// runs step n on slab t + 1 (slabs 0 and 1 in launch 0) and step n + 1 on
// slab t - 1 (slabs S - 2 and S - 1 in the last launch), so step n + 1 on a
// slab follows step n on that slab and its two neighbours, and no step-n
// tile still to run reads a plane step n + 1 overwrites (slab s + 2 reads
// down to the last plane of slab s + 1 only).  S launches for the two steps.
hipError_t launch_em_pair_schedule(const EmLaunch &La, const EmLaunch &Lb, int n_slabs, hipStream_t s) {
  int ntx, nty, nkc;
  const int kc = La.kchunk > 0 ? La.kchunk : em_kchunk(La.g, La.precision);
  em_tiles(La.g, La.precision, kc, &ntx, &nty, &nkc);
  const int S = std::max(2, std::min(n_slabs, nkc));
  auto first = [&](int q) { return int(int64_t(q) * nkc / S); };  // first chunk of slab q
  const dim3 block(BX, BY, 1);
  for (int t = 0; t < S; ++t) {
    // step-n slabs [a0, a1), step-(n + 1) slabs [b0, b1) of this launch
    int a0 = 0, a1 = 0, b0 = 0, b1 = 0;
    if (t == 0) {
      a1 = 2;
    } else if (t == S - 1) {
      b0 = S - 2;
      b1 = S;
    } else {
      a0 = t + 1; a1 = t + 2;
      b0 = t - 1; b1 = t;
    }
    const int kcA = a0 < a1 ? first(a0) : 0, nkcA = a0 < a1 ? first(a1) - first(a0) : 0;
    const int kcB = b0 < b1 ? first(b0) : 0, nkcB = b0 < b1 ? first(b1) - first(b0) : 0;
    const int nb = ntx * nty * (nkcA + nkcB);
    if (nb == 0) continue;
    if (La.precision == ETM_PREC_FP64) {
      EmPtrs<double> pa{(const double *)La.e0[0], (const double *)La.e1[0], (double *)La.out0[0], nullptr};
      EmPtrs<double> pb{(const double *)Lb.e0[0], (const double *)Lb.e1[0], (double *)Lb.out0[0], nullptr};
      hipLaunchKernelGGL((em_march_pair_kernel<double, false>), dim3(nb), block, 0, s, La, pa, pb, ntx, nty, kcA, nkcA,
                         kcB, nkcB, kc, La.acc_joule);
    } else {
      EmPtrs<float> pa{(const float *)La.e0[0], (const float *)La.e1[0], (float *)La.out0[0], (float *)La.out1[0]};
      EmPtrs<float> pb{(const float *)Lb.e0[0], (const float *)Lb.e1[0], (float *)Lb.out0[0], (float *)Lb.out1[0]};
      hipLaunchKernelGGL((em_march_pair_kernel<float, true>), dim3(nb), block, 0, s, La, pa, pb, ntx, nty, kcA, nkcA,
                         kcB, nkcB, kc, La.acc_joule);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_em_batched(const BatchVar *vars, const int4 *items, int n_items, const int64_t *step_ctr,
                             int precision, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  if (precision == ETM_PREC_FP64)
    hipLaunchKernelGGL((em_march_batched<double, false>), dim3(n_items), dim3(BX, BY), 0, st, vars, items, n_items,
                       step_ctr);
  else
    hipLaunchKernelGGL((em_march_batched<float, true>), dim3(n_items), dim3(BX, BY), 0, st, vars, items, n_items,
                       step_ctr);
  return hipGetLastError();
}

hipError_t launch_wave_sample(const double *aw, int n, double dt, int64_t base, double *Ja, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t total = int64_t(n) * (kWaveBlock + 1);
  hipLaunchKernelGGL(wave_sample_kernel, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, aw, n, dt, base, Ja);
  return hipGetLastError();
}

hipError_t launch_step_ctr(int64_t *ctr, int64_t v, int set, hipStream_t s) {
  hipLaunchKernelGGL(step_ctr_kernel, dim3(1), dim3(64), 0, s, ctr, v, set);
  return hipGetLastError();
}

hipError_t launch_thermal(const ThermalLaunch &L, hipStream_t s) {
  const dim3 grid = node_grid_z(L.g), block(BX, BY, 1);
  if (L.precision == ETM_PREC_FP64)
    hipLaunchKernelGGL((thermal_kernel<double>), grid, block, 0, s, L, (const double *)L.e[0], (const double *)L.e[1],
                       (const double *)L.e[2], (const double *)L.coef);
  else
    hipLaunchKernelGGL((thermal_kernel<float>), grid, block, 0, s, L, (const float *)L.e[0], (const float *)L.e[1],
                       (const float *)L.e[2], (const float *)L.coef);
  const int64_t nb = int64_t(grid.x) * grid.y * grid.z;
  if (nb > 4 * kFinalizeRows) {
    // two stages: rows [nb, nb + kFinalizeRows) of the partials hold the first
    const int64_t per = (nb + kFinalizeRows - 1) / kFinalizeRows, nb2 = (nb + per - 1) / per;
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(unsigned(nb2)), dim3(256), 0, s, (const double *)L.partials, nb, per,
                       1, 1, L.partials + nb * kRedWidth);
    hipLaunchKernelGGL(thermal_finalize, dim3(1), dim3(256), 0, s, (const double *)(L.partials + nb * kRedWidth),
                       nb2, L.sc);
  } else {
    hipLaunchKernelGGL(thermal_finalize, dim3(1), dim3(256), 0, s, (const double *)L.partials, nb, L.sc);
  }
  return hipGetLastError();
}

hipError_t launch_joule_flush(const DevGrid &g, int precision, const void *const *e, const void *coef, double *psum,
                              double jf, hipStream_t s) {
  const dim3 grid = node_grid(g), block(BX, BY, 1);
  if (precision == ETM_PREC_FP64)
    hipLaunchKernelGGL((joule_flush_kernel<double>), grid, block, 0, s, g, (const double *)e[0], (const double *)e[1],
                       (const double *)e[2], (const double *)coef, psum, jf);
  else
    hipLaunchKernelGGL((joule_flush_kernel<float>), grid, block, 0, s, g, (const float *)e[0], (const float *)e[1],
                       (const float *)e[2], (const float *)coef, psum, jf);
  return hipGetLastError();
}

hipError_t launch_coef(const DevGrid &g, const DevPorts &P, int precision, const void *theta, void *coef, CoefK ck,
                       hipStream_t s) {
  const dim3 grid = node_grid_z(g), block(BX, BY, 1);
  if (precision == ETM_PREC_FP64)
    hipLaunchKernelGGL((coef_kernel<double>), grid, block, 0, s, g, P, (const double *)theta, (double *)coef,
                       CoefK{nullptr, nullptr, nullptr, ck.tcr_only});
  else
    hipLaunchKernelGGL((coef_kernel<float>), grid, block, 0, s, g, P, (const float *)theta, (float *)coef, ck);
  return hipGetLastError();
}

hipError_t launch_diag(const DiagLaunch &L, hipStream_t s) {
  const dim3 grid = node_grid(L.g), block(BX, BY, 1);
  const int64_t nb = int64_t(grid.x) * grid.y * grid.z;
  if (L.precision == ETM_PREC_FP64) {
    hipLaunchKernelGGL((diag_kernel<double>), grid, block, 0, s, L);
    hipLaunchKernelGGL((diag_finalize<double>), dim3(1), dim3(256), 0, s, L, nb);
  } else {
    hipLaunchKernelGGL((diag_kernel<float>), grid, block, 0, s, L);
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
