// gfx950 kernels of the thermoelastic solve (arXiv 2603.07038, Sec. II-B):
// the HEX8 stiffness of Eq. (8) applied matrix-free, its thermal load, the
// CG building blocks (nodal Jacobi preconditioning here, the multigrid
// V-cycle in mg.hip; together they replace the paper's closed AMG solver),
// the device-side outer loop of a solve (FP64 residual checks, refinement
// updates, stop decisions), and the centroid von Mises stress of Eq. (9).
//
// Box elements.  Every cell is an axis-aligned box, so with trilinear shape
// functions N_a = phi_ax(x) phi_ay(y) phi_az(z) each entry of the element
// matrices factors into 1D integrals
//   m(a,b) = int phi_a phi_b  = h/3 (a == b) or h/6,
//   k(a,b) = int phi_a' phi_b' = +1/h or -1/h,
//   int phi_a' phi_b = s_a / 2   (s_0 = -1, s_1 = +1),
// and the 2x2x2 Gauss rule of the paper integrates all of them exactly
// (at most quadratic per axis).  With A^IJ_ab = int dN_a/dx_I dN_b/dx_J,
// the 3x3 block of the element stiffness is
//   K_IJ(a,b) = lambda A^IJ + mu A^JI + delta_IJ mu (A^xx + A^yy + A^zz),
// and the thermal load is f_aI = (3 lambda + 2 mu) cte sum_b theta_b
// int dN_a/dx_I N_b  (theta trilinear, as at the Gauss points).
//
// One thread owns one node and gathers the rows of its 8 cells (no atomics).
// Vectors are SoA node-shaped arrays; fixed DOFs hold zero and their rows
// return zero, which restricts the operator to the free DOFs.
#include <algorithm>

#include "etm_internal.h"
#include "mech_common.h"

namespace etm {

namespace {

using namespace mech;

__global__ __launch_bounds__(256) void mech_diag_kernel(MechGrid M, double *d0, double *d1, double *d2) {
  const DevGrid &g = M.g;
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  if (i > g.nx || j > g.ny) return;
  const int64_t n = int64_t(k) * g.sz + int64_t(j) * g.sy + i;
  double sx = 0, sy = 0, sz = 0;
  for (int c = 0; c < 8; ++c) {
    const int ox = c & 1, oy = (c >> 1) & 1, oz = c >> 2;
    const int ci = i - 1 + ox, cj = j - 1 + oy, ck = k - 1 + oz;
    if (ci < 0 || ci >= g.nx || cj < 0 || cj >= g.ny || ck < 0 || ck >= g.nz) continue;
    const double *row = g.mtab + g.mat[n + (ox - 1) + (oy - 1) * g.sy + (oz - 1) * g.sz] * kMatStride;
    if (row[MC_VOID] != 0.0) continue;
    const double lam = row[MC_LAMBDA], mu = row[MC_MU];
    const double hx = g.dx[ci], hy = g.dy[cj], hz = g.dz[ck];
    const double Axx = (1.0 / hx) * (hy / 3.0) * (hz / 3.0), Ayy = (hx / 3.0) * (1.0 / hy) * (hz / 3.0),
                 Azz = (hx / 3.0) * (hy / 3.0) * (1.0 / hz);
    const double Lp = mu * (Axx + Ayy + Azz);
    sx += (lam + mu) * Axx + Lp;
    sy += (lam + mu) * Ayy + Lp;
    sz += (lam + mu) * Azz + Lp;
  }
  const uint8_t f = M.fixed[n];
  d0[n] = (f & 1) || sx == 0.0 ? 0.0 : 1.0 / sx;
  d1[n] = (f & 2) || sy == 0.0 ? 0.0 : 1.0 / sy;
  d2[n] = (f & 4) || sz == 0.0 ? 0.0 : 1.0 / sz;
}

// Thermal load with fixed rows zeroed; partial ||f||^2 per block.
__global__ __launch_bounds__(256) void mech_rhs_kernel(MechGrid M, const double *theta, double *f0, double *f1,
                                                       double *f2, double *partials) {
  const DevGrid &g = M.g;
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  double nrm = 0.0;
  if (i <= g.nx && j <= g.ny) {
    const int64_t n = int64_t(k) * g.sz + int64_t(j) * g.sy + i;
    double fx = 0, fy = 0, fz = 0;
    for (int c = 0; c < 8; ++c) {
      const int ox = c & 1, oy = (c >> 1) & 1, oz = c >> 2;
      const int ci = i - 1 + ox, cj = j - 1 + oy, ck = k - 1 + oz;
      if (ci < 0 || ci >= g.nx || cj < 0 || cj >= g.ny || ck < 0 || ck >= g.nz) continue;
      const int64_t nb0 = n + (ox - 1) + (oy - 1) * g.sy + (oz - 1) * g.sz;
      const double *row = g.mtab + g.mat[nb0] * kMatStride;
      if (row[MC_VOID] != 0.0) continue;
      const double beta = row[MC_BETA];
      const double hx = g.dx[ci], hy = g.dy[cj], hz = g.dz[ck];
      const int ax = 1 - ox, ay = 1 - oy, az = 1 - oz;
      const double gx = ax ? 0.5 : -0.5, gy = ay ? 0.5 : -0.5, gz = az ? 0.5 : -0.5;
      double sx = 0, sy = 0, sz = 0;
      for (int b = 0; b < 8; ++b) {
        const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
        const double th = theta[nb0 + bx + by * g.sy + bz * g.sz];
        const double mx = hx * (ax == bx ? 1.0 / 3.0 : 1.0 / 6.0), my = hy * (ay == by ? 1.0 / 3.0 : 1.0 / 6.0),
                     mz = hz * (az == bz ? 1.0 / 3.0 : 1.0 / 6.0);
        sx += th * my * mz;
        sy += th * mx * mz;
        sz += th * mx * my;
      }
      fx += beta * gx * sx;
      fy += beta * gy * sy;
      fz += beta * gz * sz;
    }
    const uint8_t fl = M.fixed[n];
    if (fl & 1) fx = 0;
    if (fl & 2) fy = 0;
    if (fl & 4) fz = 0;
    f0[n] = fx; f1[n] = fy; f2[n] = fz;
    nrm = fx * fx + fy * fy + fz * fz;
  }
  const double v[1] = {nrm};
  const int64_t b = (int64_t(blockIdx.z) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  block_sums<1>(v, partials + b * kRedWidth);
}

__global__ __launch_bounds__(256) void rhs_finalize(const double *part, int64_t nb, DevScalars *sc, double rtol) {
  __shared__ double out[1];
  sum_partials<1>(part, nb, out);
  if (threadIdx.x == 0) {
    sc->fnorm2 = out[0];
    sc->tol2 = rtol * rtol * out[0];
  }
}

// ---- CG -----------------------------------------------------------------------
// Jacobi-CG start: r = b - K u, z = Dinv r, p = z; partial r.z and r.r.
template <typename T>
struct EpiJacobiStart {
  CgVecs<T> v;
  const T *b0, *b1, *b2;
  struct Pre { T b[3], d[3]; };
  __device__ Pre load(int64_t n) const {
    return Pre{{b0[n], b1[n], b2[n]}, {v.dinv[0][n], v.dinv[1][n], v.dinv[2][n]}};
  }
  __device__ void operator()(int64_t n, const T y[3], const T *, const Pre &q, double *red) const {
    const T rx = q.b[0] - y[0], ry = q.b[1] - y[1], rz = q.b[2] - y[2];
    const T zx = q.d[0] * rx, zy = q.d[1] * ry, zz = q.d[2] * rz;
    v.r[0][n] = rx; v.r[1][n] = ry; v.r[2][n] = rz;
    v.p[0][n] = zx; v.p[1][n] = zy; v.p[2][n] = zz;
    red[0] += double(rx) * double(zx) + double(ry) * double(zy) + double(rz) * double(zz);
    red[1] += double(rx) * double(rx) + double(ry) * double(ry) + double(rz) * double(rz);
  }
};

__global__ __launch_bounds__(256) void cg_setup_finalize(const double *part, int64_t nb, DevScalars *sc,
                                                         const DevScalars *gate) {
  if (gate && gate->done) return;  // no restart due: the inner CG goes on (or the solve is over)
  __shared__ double out[2];
  sum_partials<2>(part, nb, out);
  if (threadIdx.x == 0) {
    sc->rz = out[0];
    sc->rr = out[1];
    sc->iters = 0;
    sc->done = (out[1] <= sc->tol2) ? 1 : 0;
    sc->alpha = sc->beta = 0.0;
    sc->restart = 0;
  }
}

// w = K p; partial p.w.
template <typename T>
struct EpiApplyDot {
  T *w0, *w1, *w2;
  struct Pre {};
  __device__ Pre load(int64_t) const { return Pre{}; }
  __device__ void operator()(int64_t n, const T y[3], const T xc[3], const Pre &, double *red) const {
    w0[n] = y[0]; w1[n] = y[1]; w2[n] = y[2];
    red[0] += double(xc[0]) * double(y[0]) + double(xc[1]) * double(y[1]) + double(xc[2]) * double(y[2]);
  }
};

__global__ __launch_bounds__(256) void cg_alpha_finalize(const double *part, int64_t nb, DevScalars *sc) {
  if (sc->done) return;
  __shared__ double out[1];
  sum_partials<1>(part, nb, out);
  if (threadIdx.x == 0) {
    sc->pw = out[0];
    sc->alpha = out[0] > 0.0 ? sc->rz / out[0] : 0.0;
    if (!(out[0] > 0.0)) sc->done = 2;  // breakdown: stop (the host re-checks the true residual)
  }
}

template <typename T>
__global__ __launch_bounds__(256) void cg_update_kernel(CgVecs<T> v, int64_t ntot, const DevScalars *sc,
                                                        double *partials) {
  if (sc->done) return;
  const T alpha = T(sc->alpha);
  double rz = 0.0, rr = 0.0;
  for (int64_t n = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; n < ntot; n += int64_t(gridDim.x) * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T p = v.p[c][n];
      v.u[c][n] += alpha * p;
      const T r = v.r[c][n] - alpha * v.w[c][n];
      v.r[c][n] = r;
      const T z = v.dinv[c][n] * r;
      rz += double(r) * double(z);
      rr += double(r) * double(r);
    }
  }
  const double s[2] = {rz, rr};
  block_sums<2>(s, partials + int64_t(blockIdx.x) * kRedWidth);
}

__global__ __launch_bounds__(256) void cg_beta_finalize(const double *part, int64_t nb, DevScalars *sc) {
  if (sc->done) return;
  __shared__ double out[2];
  sum_partials<2>(part, nb, out);
  if (threadIdx.x == 0) {
    sc->iters += 1;
    sc->rr = out[1];
    if (out[1] <= sc->tol2 || !(out[0] > 0.0) || sc->iters >= sc->budget) {
      sc->done = 1;
    } else {
      sc->beta = out[0] / sc->rz;
      sc->rz = out[0];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void cg_p_kernel(CgVecs<T> v, int64_t ntot, const DevScalars *sc) {
  if (sc->done) return;
  const T beta = T(sc->beta);
  for (int64_t n = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; n < ntot; n += int64_t(gridDim.x) * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 3; ++c) v.p[c][n] = v.dinv[c][n] * v.r[c][n] + beta * v.p[c][n];
  }
}

// r64 = f - K u64; partial |r|^2.
struct EpiResidual64 {
  const double *f0, *f1, *f2;
  double *r0, *r1, *r2;
  struct Pre { double f[3]; };
  __device__ Pre load(int64_t n) const { return Pre{{f0[n], f1[n], f2[n]}}; }
  __device__ void operator()(int64_t n, const double y[3], const double *, const Pre &q, double *red) const {
    const double rx = q.f[0] - y[0], ry = q.f[1] - y[1], rz = q.f[2] - y[2];
    r0[n] = rx; r1[n] = ry; r2[n] = rz;
    red[0] += rx * rx + ry * ry + rz * rz;
  }
};

__global__ __launch_bounds__(256) void residual_finalize(const double *part, int64_t nb, DevScalars *sc) {
  __shared__ double out[1];
  sum_partials<1>(part, nb, out);
  if (threadIdx.x == 0) sc->rr = out[0];
}

// The outer loop of a solve, decided on the device after each FP64 residual
// that follows a finished inner CG (the host only enqueues passes): book the
// inner iterations, then stop (converged: |r|^2 <= tol2; gave up: iteration
// limit reached, or an inner solve made no iteration) or ask for a new inner
// solve with its tolerance -- mixed: max(inner_rtol2 |r|^2, tol2 / 4) on the
// FP32 correction; FP64: tol2 on CG restarted from the current u -- and its
// iteration budget.
__global__ __launch_bounds__(256) void residual_check_finalize(const double *part, int64_t nb, DevScalars *ctl,
                                                               DevScalars *scm, const DevScalars *gate) {
  if (gate->done) return;
  __shared__ double out[1];
  sum_partials<1>(part, nb, out);
  if (threadIdx.x == 0) {
    const int it = scm->iters, pass = ctl->outer - 1;
    if (pass >= 0 && pass < kMaxPasses) ctl->pass_iters[pass] = it;
    ctl->iters += it;
    scm->iters = 0;
    ctl->rr = out[0];
    ctl->outer += 1;
    if (out[0] <= ctl->tol2) {
      ctl->done = kSolveConverged;
    } else if (ctl->iters >= ctl->maxit || (pass >= 0 && it == 0)) {
      ctl->done = kSolveGaveUp;
    } else {
      scm->tol2 = ctl->mixed ? fmax(ctl->inner_rtol2 * out[0], 0.25 * ctl->tol2) : ctl->tol2;
      scm->budget = ctl->maxit - ctl->iters;
      scm->restart = 1;
    }
  }
}

__global__ void solve_gates_kernel(const DevScalars *ctl, const DevScalars *scm, DevScalars *gR, DevScalars *gF) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    gR->done = (ctl->done || !scm->restart) ? 1 : 0;
    gF->done = (ctl->done || !scm->done) ? 1 : 0;
  }
}

// Start of a solve (ctl->fnorm2 and ctl->tol2 are set): a zero load is
// solved by u = 0 at once.
__global__ void solve_init_kernel(DevScalars *ctl, DevScalars *scm, int maxit, double inner_rtol2, int mixed) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->done = ctl->fnorm2 == 0.0 ? kSolveConverged : kSolveRunning;
    ctl->rr = 0.0;
    ctl->outer = 0;
    ctl->iters = 0;
    ctl->maxit = maxit;
    ctl->mixed = mixed;
    ctl->inner_rtol2 = inner_rtol2;
    for (int q = 0; q < kMaxPasses; ++q) ctl->pass_iters[q] = 0;
    scm->iters = 0;
    scm->done = 1;      // no inner CG running: the first FP64 check runs
    scm->restart = 0;
    scm->budget = maxit;
  }
}
__global__ void zero_if_no_load_kernel(double *u0, double *u1, double *u2, int64_t n, const DevScalars *ctl) {
  if (ctl->fnorm2 != 0.0) return;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x)
    u0[t] = u1[t] = u2[t] = 0.0;
}

__global__ void cast_kernel(const void *src, int src_f32, void *dst, int dst_f32, int64_t n, const DevScalars *gate) {
  if (gate && gate->done) return;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x) {
    const double x = src_f32 ? double(((const float *)src)[t]) : ((const double *)src)[t];
    if (dst_f32) ((float *)dst)[t] = float(x); else ((double *)dst)[t] = x;
  }
}

// u_c <- 0 at every node whose DOF c is fixed.
__global__ void mask_fixed_kernel(const uint8_t *fixed, int c, double *u, int64_t n) {
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x)
    if (fixed[t] >> c & 1) u[t] = 0.0;
}

// u <- w0 u + w1 u_prev + w2 u_prev2, u_prev2 <- u_prev, u_prev <- old u.
struct Hist3 {
  double *u[3], *v[3], *q[3];
};
__global__ void extrapolate_kernel(Hist3 H, double w0, double w1, double w2, int64_t n) {
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double a = H.u[c][t], b = H.v[c][t], d = H.q[c][t];
      H.u[c][t] = w0 * a + w1 * b + w2 * d;
      H.q[c][t] = b;
      H.v[c][t] = a;
    }
  }
}

__global__ void axpy64_kernel(double *y, const float *x, int64_t n, const DevScalars *gate) {
  if (gate && gate->done) return;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x)
    y[t] += double(x[t]);
}

__global__ void zero32_kernel(float *x, int64_t n, const DevScalars *gate) {
  if (gate && gate->done) return;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x)
    x[t] = 0.0f;
}

// Eq. (9) at the centroid: strain B(0) u_e (dN_a/dx = s_ax / (4 hx) there),
// thermal strain cte * mean nodal rise, isotropic Hooke's law.
__global__ __launch_bounds__(256) void von_mises_kernel(MechGrid M, const double *theta, const double *u0,
                                                        const double *u1, const double *u2, double *vm) {
  const DevGrid &g = M.g;
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  if (i >= g.nx || j >= g.ny || k >= g.nz) return;
  const int64_t n = int64_t(k) * g.sz + int64_t(j) * g.sy + i;
  const double *row = g.mtab + g.mat[n] * kMatStride;
  if (row[MC_VOID] != 0.0) { vm[n] = 0.0; return; }
  const double qx = 0.25 * g.idx[i], qy = 0.25 * g.idy[j], qz = 0.25 * g.idz[k];
  double exx = 0, eyy = 0, ezz = 0, gxy = 0, gyz = 0, gzx = 0, th = 0;
  for (int a = 0; a < 8; ++a) {
    const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
    const int64_t na = n + ax + ay * g.sy + az * g.sz;
    const double dxa = (ax ? qx : -qx), dya = (ay ? qy : -qy), dza = (az ? qz : -qz);
    const double ux = u0[na], uy = u1[na], uz = u2[na];
    exx += dxa * ux; eyy += dya * uy; ezz += dza * uz;
    gxy += dya * ux + dxa * uy;
    gyz += dza * uy + dya * uz;
    gzx += dxa * uz + dza * ux;
    th += theta[na];
  }
  th *= 0.125;
  const double et = row[MC_CTE] * th;
  exx -= et; eyy -= et; ezz -= et;
  const double lam = row[MC_LAMBDA], mu = row[MC_MU];
  const double tr = lam * (exx + eyy + ezz);
  const double sx = tr + 2 * mu * exx, sy = tr + 2 * mu * eyy, sz = tr + 2 * mu * ezz;
  const double txy = mu * gxy, tyz = mu * gyz, tzx = mu * gzx;
  const double a1 = sx - sy, a2 = sy - sz, a3 = sz - sx;
  vm[n] = sqrt(0.5 * (a1 * a1 + a2 * a2 + a3 * a3 + 6.0 * (txy * txy + tyz * tyz + tzx * tzx)));
}

inline int flat_blocks(int64_t n) { return int(std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024))); }

}  // namespace

hipError_t launch_mech_diag(const MechGrid &M, double *dinv[3], hipStream_t s) {
  hipLaunchKernelGGL(mech_diag_kernel, node_grid(M.g), dim3(BX, BY), 0, s, M, dinv[0], dinv[1], dinv[2]);
  return hipGetLastError();
}

hipError_t launch_mech_rhs(const MechGrid &M, const double *theta, double *f[3], double *partials,
                           DevScalars *sc, double rtol, hipStream_t s) {
  const dim3 grid = node_grid(M.g);
  hipLaunchKernelGGL(mech_rhs_kernel, grid, dim3(BX, BY), 0, s, M, theta, f[0], f[1], f[2], partials);
  hipLaunchKernelGGL(rhs_finalize, dim3(1), dim3(256), 0, s, (const double *)partials,
                     int64_t(grid.x) * grid.y * grid.z, sc, rtol);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_setup(const MechGrid &M, const CgVecs<T> &v, const T *rhs[3], double *partials,
                           DevScalars *sc, const DevScalars *gate, hipStream_t s) {
  const T *x[3] = {v.u[0], v.u[1], v.u[2]};
  hipError_t e = launch_hex8<T, 2>(M, x, EpiJacobiStart<T>{v, rhs[0], rhs[1], rhs[2]}, partials, gate, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cg_setup_finalize, dim3(1), dim3(256), 0, s, (const double *)partials,
                     cell_blocks(M.g, cell_kchunk(M.g)), sc, gate);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_iteration(const MechGrid &M, const CgVecs<T> &v, double *partials, DevScalars *sc,
                               hipStream_t s) {
  hipError_t e = launch_cg_apply_alpha<T>(M, v, partials, sc, s);
  if (e != hipSuccess) return e;
  const int fb = flat_blocks(M.g.ntot);
  hipLaunchKernelGGL((cg_update_kernel<T>), dim3(fb), dim3(256), 0, s, v, M.g.ntot, (const DevScalars *)sc, partials);
  hipLaunchKernelGGL(cg_beta_finalize, dim3(1), dim3(256), 0, s, (const double *)partials, int64_t(fb), sc);
  hipLaunchKernelGGL((cg_p_kernel<T>), dim3(fb), dim3(256), 0, s, v, M.g.ntot, (const DevScalars *)sc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_apply_alpha(const MechGrid &M, const CgVecs<T> &v, double *partials, DevScalars *sc,
                                 hipStream_t s) {
  const T *x[3] = {v.p[0], v.p[1], v.p[2]};
  hipError_t e = launch_hex8<T, 1>(M, x, EpiApplyDot<T>{v.w[0], v.w[1], v.w[2]}, partials, sc, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cg_alpha_finalize, dim3(1), dim3(256), 0, s, (const double *)partials,
                     cell_blocks(M.g, cell_kchunk(M.g)), sc);
  return hipGetLastError();
}

template hipError_t launch_cg_apply_alpha<double>(const MechGrid &, const CgVecs<double> &, double *, DevScalars *,
                                                  hipStream_t);
template hipError_t launch_cg_apply_alpha<float>(const MechGrid &, const CgVecs<float> &, double *, DevScalars *,
                                                 hipStream_t);
template hipError_t launch_cg_setup<double>(const MechGrid &, const CgVecs<double> &, const double *[3], double *,
                                            DevScalars *, const DevScalars *, hipStream_t);
template hipError_t launch_cg_setup<float>(const MechGrid &, const CgVecs<float> &, const float *[3], double *,
                                           DevScalars *, const DevScalars *, hipStream_t);
template hipError_t launch_cg_iteration<double>(const MechGrid &, const CgVecs<double> &, double *, DevScalars *,
                                                hipStream_t);
template hipError_t launch_cg_iteration<float>(const MechGrid &, const CgVecs<float> &, double *, DevScalars *,
                                               hipStream_t);

hipError_t launch_residual64(const MechGrid &M, const double *f[3], const double *u[3], double *r[3],
                             double *partials, DevScalars *sc, hipStream_t s) {
  hipError_t e =
      launch_hex8<double, 1>(M, u, EpiResidual64{f[0], f[1], f[2], r[0], r[1], r[2]}, partials, nullptr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(residual_finalize, dim3(1), dim3(256), 0, s, (const double *)partials,
                     cell_blocks(M.g, cell_kchunk(M.g)), sc);
  return hipGetLastError();
}

hipError_t launch_residual_check(const MechGrid &M, const double *f[3], const double *u[3], double *r[3],
                                 double *partials, DevScalars *ctl, DevScalars *scm, const DevScalars *gate,
                                 hipStream_t s) {
  hipError_t e =
      launch_hex8<double, 1>(M, u, EpiResidual64{f[0], f[1], f[2], r[0], r[1], r[2]}, partials, gate, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(residual_check_finalize, dim3(1), dim3(256), 0, s, (const double *)partials,
                     cell_blocks(M.g, cell_kchunk(M.g)), ctl, scm, gate);
  return hipGetLastError();
}

hipError_t launch_solve_gates(const DevScalars *ctl, const DevScalars *scm, DevScalars *gR, DevScalars *gF,
                              hipStream_t s) {
  hipLaunchKernelGGL(solve_gates_kernel, dim3(1), dim3(64), 0, s, ctl, scm, gR, gF);
  return hipGetLastError();
}

hipError_t launch_solve_init(DevScalars *ctl, DevScalars *scm, int maxit, double inner_rtol2, int mixed,
                             double *u[3], int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(solve_init_kernel, dim3(1), dim3(64), 0, s, ctl, scm, maxit, inner_rtol2, mixed);
  hipLaunchKernelGGL(zero_if_no_load_kernel, dim3(flat_blocks(n)), dim3(256), 0, s, u[0], u[1], u[2], n,
                     (const DevScalars *)ctl);
  return hipGetLastError();
}

hipError_t launch_vec_cast(const void *src, int src_f32, void *dst, int dst_f32, int64_t n, const DevScalars *gate,
                           hipStream_t s) {
  hipLaunchKernelGGL(cast_kernel, dim3(flat_blocks(n)), dim3(256), 0, s, src, src_f32, dst, dst_f32, n, gate);
  return hipGetLastError();
}

hipError_t launch_vec_zero32(float *x, int64_t n, const DevScalars *gate, hipStream_t s) {
  hipLaunchKernelGGL(zero32_kernel, dim3(flat_blocks(n)), dim3(256), 0, s, x, n, gate);
  return hipGetLastError();
}

hipError_t launch_extrapolate(double *u[3], double *uprev[3], double *uprev2[3], const double w[3], int64_t n,
                              hipStream_t s) {
  Hist3 H;
  for (int c = 0; c < 3; ++c) { H.u[c] = u[c]; H.v[c] = uprev[c]; H.q[c] = uprev2[c]; }
  hipLaunchKernelGGL(extrapolate_kernel, dim3(flat_blocks(n)), dim3(256), 0, s, H, w[0], w[1], w[2], n);
  return hipGetLastError();
}

hipError_t launch_mask_fixed(const MechGrid &M, int c, double *u, hipStream_t s) {
  hipLaunchKernelGGL(mask_fixed_kernel, dim3(flat_blocks(M.g.ntot)), dim3(256), 0, s, M.fixed, c, u, M.g.ntot);
  return hipGetLastError();
}

hipError_t launch_vec_axpy64(double *y, const float *x, int64_t n, const DevScalars *gate, hipStream_t s) {
  hipLaunchKernelGGL(axpy64_kernel, dim3(flat_blocks(n)), dim3(256), 0, s, y, x, n, gate);
  return hipGetLastError();
}

hipError_t launch_von_mises(const MechGrid &M, const double *theta, const double *u[3], double *vm, hipStream_t s) {
  hipLaunchKernelGGL(von_mises_kernel, node_grid(M.g), dim3(BX, BY), 0, s, M, theta, u[0], u[1], u[2], vm);
  return hipGetLastError();
}

}  // namespace etm
