// Geometric multigrid preconditioner for the thermoelastic system of Eq. (8)
// on gfx950, and the preconditioned CG built on it.
//
// The paper solves Eq. (8) with an algebraic multigrid preconditioner; the
// mesh here is rectilinear, so the hierarchy is geometric and built on the
// device:
//   * coarse nodes are every second node along each axis (plus the last node
//     of an odd axis); prolongation P is trilinear in the node coordinates,
//     so P reproduces linear fields, and with them rigid-body motions, on
//     graded spacings;
//   * A_1 = P^T K P is formed directly from the HEX8 cells.  For a box cell
//     each of the nine 3x3 sub-blocks of the element stiffness is a product
//     of three 1D factors, so the weighted sum over a cell's 8x8 node pairs
//     separates into three 2x2 bilinear forms (cells that touch a fixed DOF
//     take the explicit pair loop, which applies the mask);
//   * deeper levels are stencil products A_{l+1} = P^T A_l P;
//   * every coarse operator is kept as a symmetric 27-point stencil of 3x3
//     blocks: the centre and the 13 offsets after it are stored, the other
//     13 blocks are the transposes stored at the neighbour;
//   * smoothing is Chebyshev on the nodal 3x3-block Jacobi operator, with the
//     top of the spectrum bounded from below by a Rayleigh quotient after a
//     fixed number of power steps; the same polynomial before and after the
//     coarse correction keeps the V-cycle symmetric, so it is a valid CG
//     preconditioner while the interval covers the spectrum;
//   * stencil blocks are stored row by row: the three entries of a block
//     row are contiguous, so a node's block is three 12-byte loads;
//   * the coarsest level is solved exactly with a dense inverse built on the
//     host once per plan.
// Level 0 is applied matrix free (the same HEX8 apply as the CG operator).
#include <algorithm>

#include "etm_internal.h"
#include "mech_common.h"

namespace etm {

namespace {

using namespace mech;

// Node (i, j, k) of the thread in a level launched on lgrid: each plane's
// (nx + 1) x (ny + 1) nodes are numbered x fastest and cut into blocks of
// BX * BY threads, so the coarse levels' short rows (129, 65, 33 nodes) fill
// the waves instead of leaving up to half of each 64-wide row tile idle;
// the blocks are taken in XCD-contiguous order, so the blocks holding the
// rows j - 1, j, j + 1 of a plane share an L2.  Threads past the end of the
// plane get j > ny.
__device__ __forceinline__ void plane_node(int nx, int &i, int &j, int &k) {
  const int nbx = int(gridDim.x);
  const int lb = xcd_remap(int(blockIdx.z) * nbx + int(blockIdx.x), nbx * int(gridDim.z));
  const int t = (lb % nbx) * (BX * BY) + int(threadIdx.y) * BX + int(threadIdx.x);
  k = lb / nbx;
  j = t / (nx + 1);
  i = t - j * (nx + 1);
}

// Offsets of the 27-point stencil: o = (oz+1)*9 + (oy+1)*3 + (ox+1);
// o = 13 is the centre and 26 - o is the opposite offset.
__device__ __forceinline__ void off3(int o, int &ox, int &oy, int &oz) {
  ox = o % 3 - 1;
  oy = (o / 3) % 3 - 1;
  oz = o / 9 - 1;
}

// 1D prolongation weight of coarse node I at fine node i.
__device__ __forceinline__ double p1(const MgAxis &a, int i, int I) {
  const int lo = a.lo[i];
  const double w = a.w[i];
  return I == lo ? w : (I == lo + 1 ? 1.0 - w : 0.0);
}

// Block (row comp, col comp) of A(n, n + offset o) from the symmetric storage.
template <typename T>
__device__ __forceinline__ void stencil_block(const MgLevel<T> &L, int64_t n, int o, double B[9]) {
  const int64_t N = L.n;
  if (o >= 13) {
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) B[r * 3 + c] = double(L.A[stencil_idx(o - 13, r, c, N, n)]);
  } else {
    int ox, oy, oz;
    off3(o, ox, oy, oz);
    const int64_t m = n + ox + oy * L.sy + oz * L.sz;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) B[r * 3 + c] = double(L.A[stencil_idx(13 - o, c, r, N, m)]);
  }
}

// y = A x at node (i,j,k) of a stencil level, the 27 offsets in order.  The
// offsets of one row (ox = -1, 0, 1) are loaded together before they are
// used: an offset outside the level reads the node's own entries (always
// finite) with x = 0, so no load waits behind a branch and a row's loads
// overlap (nine round trips to memory per node instead of 27).  The rows
// stay a loop: unrolled, all 27 offsets' loads are hoisted together and take
// 177 registers (2 waves per SIMD).  Adding the masked zeros leaves the
// sums unchanged.
template <typename T>
__device__ __forceinline__ void stencil_apply(const MgLevel<T> &L, int i, int j, int k, int64_t n, const V3<T> &x,
                                              T y[3]) {
  const int64_t N = L.n;
  T y0 = T(0), y1 = T(0), y2 = T(0);
#pragma unroll 1
  for (int r = 0; r < 9; ++r) {
    const int oy = r % 3 - 1, oz = r / 3 - 1;
    const int jj = j + oy, kk = k + oz;
    const bool row_ok = jj >= 0 && jj <= L.ny && kk >= 0 && kk <= L.nz;
    T xv[3][3], R[3][3][3];
    bool tr[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int ox = c - 1, o = r * 3 + c;
      const int ii = i + ox;
      const bool ok = row_ok && ii >= 0 && ii <= L.nx;
      const int64_t m = ok ? n + ox + oy * L.sy + oz * L.sz : n;
      tr[c] = o < 13;  // stored at the lower neighbour: use its transpose
      const int q = tr[c] ? 13 - o : o - 13;
      const int64_t p = tr[c] ? m : n;
#pragma unroll
      for (int d = 0; d < 3; ++d) xv[c][d] = x.c[d][m];
#pragma unroll
      for (int rr = 0; rr < 3; ++rr)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) R[c][rr][cc] = L.A[stencil_idx(q, rr, cc, N, p)];
      if (!ok) xv[c][0] = xv[c][1] = xv[c][2] = T(0);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T x0 = xv[c][0], x1 = xv[c][1], x2 = xv[c][2];
      T B[3][3];
#pragma unroll
      for (int rr = 0; rr < 3; ++rr)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) B[rr][cc] = tr[c] ? R[c][cc][rr] : R[c][rr][cc];
      y0 += B[0][0] * x0 + B[0][1] * x1 + B[0][2] * x2;
      y1 += B[1][0] * x0 + B[1][1] * x1 + B[1][2] * x2;
      y2 += B[2][0] * x0 + B[2][1] * x1 + B[2][2] * x2;
    }
  }
  y[0] = y0; y[1] = y1; y[2] = y2;
}

// Inverse of the live part of a symmetric 3x3 block (dead rows/columns zero).
// out = (xx, yy, zz, xy, yz, xz).
__device__ __forceinline__ void inv3_live(const double Bin[9], uint8_t dead, double out[6]) {
  double B[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) B[e] = Bin[e];
#pragma unroll
  for (int c = 0; c < 3; ++c)
    if (dead >> c & 1) {
#pragma unroll
      for (int q = 0; q < 3; ++q) { B[c * 3 + q] = 0.0; B[q * 3 + c] = 0.0; }
      B[c * 3 + c] = 1.0;
    }
  const double a = B[0], b = 0.5 * (B[1] + B[3]), c = 0.5 * (B[2] + B[6]);
  const double d = B[4], e = 0.5 * (B[5] + B[7]), f = B[8];
  // adjugate of [[a b c][b d e][c e f]]
  const double A00 = d * f - e * e, A01 = c * e - b * f, A02 = b * e - c * d;
  const double A11 = a * f - c * c, A12 = b * c - a * e, A22 = a * d - b * b;
  const double det = a * A00 + b * A01 + c * A02;
  double C[6];
  if (det > 0.0 && a > 0.0 && d > 0.0 && f > 0.0) {
    const double id = 1.0 / det;
    C[0] = A00 * id; C[1] = A11 * id; C[2] = A22 * id; C[3] = A01 * id; C[4] = A12 * id; C[5] = A02 * id;
  } else {  // not positive definite: point Jacobi on the positive diagonal
    C[0] = a > 0.0 ? 1.0 / a : 0.0; C[1] = d > 0.0 ? 1.0 / d : 0.0; C[2] = f > 0.0 ? 1.0 / f : 0.0;
    C[3] = C[4] = C[5] = 0.0;
  }
  const bool dx = dead & 1, dy = dead & 2, dz = dead & 4;
  out[0] = dx ? 0.0 : C[0];
  out[1] = dy ? 0.0 : C[1];
  out[2] = dz ? 0.0 : C[2];
  out[3] = (dx || dy) ? 0.0 : C[3];
  out[4] = (dy || dz) ? 0.0 : C[4];
  out[5] = (dx || dz) ? 0.0 : C[5];
}

// ---- set-up -------------------------------------------------------------------

// Nodal diagonal blocks of K on level 0 (sum over the node's cells of the
// element block K_e(a,a)), the dead mask (fixed DOFs and DOFs without
// stiffness) and the inverse of the live part.
template <typename T>
__global__ __launch_bounds__(256) void mg_diag0_kernel(MechGrid M, T *Dinv, int64_t dn, uint8_t *dead) {
  const DevGrid &g = M.g;
  int i, j, k;
  plane_node(g.nx, i, j, k);
  if (i > g.nx || j > g.ny) return;
  const int64_t n = int64_t(k) * g.sz + int64_t(j) * g.sy + i;
  double B[9] = {};
  for (int c = 0; c < 8; ++c) {
    const int ox = c & 1, oy = (c >> 1) & 1, oz = c >> 2;
    const int ci = i - 1 + ox, cj = j - 1 + oy, ck = k - 1 + oz;
    if (ci < 0 || ci >= g.nx || cj < 0 || cj >= g.ny || ck < 0 || ck >= g.nz) continue;
    const double *row = g.mtab + g.mat[n + (ox - 1) + (oy - 1) * g.sy + (oz - 1) * g.sz] * kMatStride;
    if (row[MC_VOID] != 0.0) continue;
    const double lam = row[MC_LAMBDA], mu = row[MC_MU];
    const double hx = g.dx[ci], hy = g.dy[cj], hz = g.dz[ck];
    const double gx = ox ? -0.5 : 0.5, gy = oy ? -0.5 : 0.5, gz = oz ? -0.5 : 0.5;  // node is corner 1-o of the cell
    const double mx = hx / 3.0, my = hy / 3.0, mz = hz / 3.0;
    const double Axx = (1.0 / hx) * my * mz, Ayy = mx * (1.0 / hy) * mz, Azz = mx * my * (1.0 / hz);
    const double Axy = gx * gy * mz, Axz = gx * my * gz, Ayz = mx * gy * gz;
    const double Lp = mu * (Axx + Ayy + Azz);
    B[0] += (lam + mu) * Axx + Lp;
    B[4] += (lam + mu) * Ayy + Lp;
    B[8] += (lam + mu) * Azz + Lp;
    B[1] += (lam + mu) * Axy;
    B[2] += (lam + mu) * Axz;
    B[5] += (lam + mu) * Ayz;
  }
  B[3] = B[1]; B[6] = B[2]; B[7] = B[5];
  const uint8_t dd = M.fixed[n] | (B[0] > 0.0 ? 0 : 1) | (B[4] > 0.0 ? 0 : 2) | (B[8] > 0.0 ? 0 : 4);
  double out[6];
  inv3_live(B, dd, out);
  dead[n] = dd;
#pragma unroll
  for (int e = 0; e < 6; ++e) Dinv[e * dn + n] = T(out[e]);
}

// Nodal blocks of a stencil level: centre block, dead mask, inverse.
template <typename T>
__global__ __launch_bounds__(256) void mg_diag_kernel(MgLevel<T> L) {
  int i, j, k;
  plane_node(L.nx, i, j, k);
  if (i > L.nx || j > L.ny) return;
  const int64_t n = int64_t(k) * L.sz + int64_t(j) * L.sy + i;
  double B[9];
  stencil_block<T>(L, n, 13, B);
  const uint8_t dd = (B[0] > 0.0 ? 0 : 1) | (B[4] > 0.0 ? 0 : 2) | (B[8] > 0.0 ? 0 : 4);
  double out[6];
  inv3_live(B, dd, out);
  L.dead[n] = dd;
#pragma unroll
  for (int e = 0; e < 6; ++e) L.Dinv[e * L.n + n] = T(out[e]);
}

// Weighted sum over one HEX8 cell of P(a,I) K_e(a,b) P(b,J) (3x3 block),
// a, b over the cell's nodes; pa / pb are the per-axis weights of the
// cell's low and high node for the row and column coarse node.
__device__ __forceinline__ void cell_galerkin(const DevGrid &g, const uint8_t *dead0, int ci, int cj, int ck,
                                              const double (&pa)[3][2], const double (&pb)[3][2], double acc[9]) {
  const int64_t nb0 = int64_t(ck) * g.sz + int64_t(cj) * g.sy + ci;
  const double *row = g.mtab + g.mat[nb0] * kMatStride;
  if (row[MC_VOID] != 0.0) return;
  const double lam = row[MC_LAMBDA], mu = row[MC_MU];
  const double h[3] = {g.dx[ci], g.dy[cj], g.dz[ck]};
  uint8_t anyd = 0;
#pragma unroll
  for (int a = 0; a < 8; ++a) anyd |= dead0[nb0 + (a & 1) + ((a >> 1) & 1) * g.sy + (a >> 2) * g.sz];
  if (!anyd) {
    // per axis: sum_ab pa_a pb_b f(a,b) for the 1D mass, stiffness and the
    // two mixed factors int phi_a' phi_b (= s_a/2) and int phi_a phi_b' (= s_b/2)
    double Mf[3], Kf[3], Gf[3], Gt[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double a0 = pa[d][0], a1 = pa[d][1], b0 = pb[d][0], b1 = pb[d][1];
      Mf[d] = h[d] * ((a0 * b0 + a1 * b1) * (1.0 / 3.0) + (a0 * b1 + a1 * b0) * (1.0 / 6.0));
      Kf[d] = (a0 - a1) * (b0 - b1) / h[d];
      Gf[d] = 0.5 * (a1 - a0) * (b0 + b1);
      Gt[d] = 0.5 * (a0 + a1) * (b1 - b0);
    }
    const double Sxx = Kf[0] * Mf[1] * Mf[2], Syy = Mf[0] * Kf[1] * Mf[2], Szz = Mf[0] * Mf[1] * Kf[2];
    const double Sxy = Gf[0] * Gt[1] * Mf[2], Syx = Gt[0] * Gf[1] * Mf[2];
    const double Sxz = Gf[0] * Mf[1] * Gt[2], Szx = Gt[0] * Mf[1] * Gf[2];
    const double Syz = Mf[0] * Gf[1] * Gt[2], Szy = Mf[0] * Gt[1] * Gf[2];
    const double Lp = mu * (Sxx + Syy + Szz);
    acc[0] += (lam + mu) * Sxx + Lp;
    acc[1] += lam * Sxy + mu * Syx;
    acc[2] += lam * Sxz + mu * Szx;
    acc[3] += lam * Syx + mu * Sxy;
    acc[4] += (lam + mu) * Syy + Lp;
    acc[5] += lam * Syz + mu * Szy;
    acc[6] += lam * Szx + mu * Sxz;
    acc[7] += lam * Szy + mu * Syz;
    acc[8] += (lam + mu) * Szz + Lp;
    return;
  }
  for (int a = 0; a < 8; ++a) {
    const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
    const double wa = pa[0][ax] * pa[1][ay] * pa[2][az];
    if (wa == 0.0) continue;
    const uint8_t da = dead0[nb0 + ax + ay * g.sy + az * g.sz];
    const double gax = ax ? 0.5 : -0.5, gay = ay ? 0.5 : -0.5, gaz = az ? 0.5 : -0.5;
    for (int b = 0; b < 8; ++b) {
      const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
      const double wb = pb[0][bx] * pb[1][by] * pb[2][bz];
      if (wb == 0.0) continue;
      const uint8_t db = dead0[nb0 + bx + by * g.sy + bz * g.sz];
      const bool sx = ax == bx, sy = ay == by, sz = az == bz;
      const double mx = h[0] * (sx ? 1.0 / 3.0 : 1.0 / 6.0), my = h[1] * (sy ? 1.0 / 3.0 : 1.0 / 6.0),
                   mz = h[2] * (sz ? 1.0 / 3.0 : 1.0 / 6.0);
      const double kx = (sx ? 1.0 : -1.0) / h[0], ky = (sy ? 1.0 : -1.0) / h[1], kz = (sz ? 1.0 : -1.0) / h[2];
      const double gbx = bx ? 0.5 : -0.5, gby = by ? 0.5 : -0.5, gbz = bz ? 0.5 : -0.5;
      const double Axx = kx * my * mz, Ayy = mx * ky * mz, Azz = mx * my * kz;
      const double Axy = gax * gby * mz, Ayx = gay * gbx * mz;
      const double Axz = gax * my * gbz, Azx = gaz * my * gbx;
      const double Ayz = mx * gay * gbz, Azy = mx * gaz * gby;
      const double Lp = mu * (Axx + Ayy + Azz);
      const double E[9] = {(lam + mu) * Axx + Lp, lam * Axy + mu * Ayx, lam * Axz + mu * Azx,
                           lam * Ayx + mu * Axy, (lam + mu) * Ayy + Lp, lam * Ayz + mu * Azy,
                           lam * Azx + mu * Axz, lam * Azy + mu * Ayz, (lam + mu) * Azz + Lp};
      const double w = wa * wb;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        if (da >> r & 1) continue;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (db >> c & 1) continue;
          acc[r * 3 + c] += w * E[r * 3 + c];
        }
      }
    }
  }
}

// Coarse stencil of level 1 straight from the HEX8 cells of level 0.  One
// thread per (coarse node, stored offset q); blockIdx.z = K * kMgUpper + q.
template <typename T>
__global__ __launch_bounds__(256) void mg_galerkin0_kernel(MechGrid M, const uint8_t *dead0, MgAxis ax, MgAxis ay,
                                                           MgAxis az, int cnx, int cny, int cnz, int64_t csy,
                                                           int64_t csz, int64_t cn, T *A) {
  const DevGrid &g = M.g;
  const int I = blockIdx.x * BX + threadIdx.x, J = blockIdx.y * BY + threadIdx.y;
  const int K = blockIdx.z / kMgUpper, q = blockIdx.z % kMgUpper;
  if (I > cnx || J > cny) return;
  int ox, oy, oz;
  off3(q + 13, ox, oy, oz);
  const int I2 = I + ox, J2 = J + oy, K2 = K + oz;
  double acc[9] = {};
  if (I2 >= 0 && I2 <= cnx && J2 >= 0 && J2 <= cny && K2 >= 0 && K2 <= cnz) {
    const int fi = ax.cpos[I], fj = ay.cpos[J], fk = az.cpos[K];
    for (int ck = max(fk - 2, 0); ck <= min(fk + 1, g.nz - 1); ++ck) {
      double pa[3][2], pb[3][2];
      pa[2][0] = p1(az, ck, K); pa[2][1] = p1(az, ck + 1, K);
      pb[2][0] = p1(az, ck, K2); pb[2][1] = p1(az, ck + 1, K2);
      if ((pa[2][0] == 0.0 && pa[2][1] == 0.0) || (pb[2][0] == 0.0 && pb[2][1] == 0.0)) continue;
      for (int cj = max(fj - 2, 0); cj <= min(fj + 1, g.ny - 1); ++cj) {
        pa[1][0] = p1(ay, cj, J); pa[1][1] = p1(ay, cj + 1, J);
        pb[1][0] = p1(ay, cj, J2); pb[1][1] = p1(ay, cj + 1, J2);
        if ((pa[1][0] == 0.0 && pa[1][1] == 0.0) || (pb[1][0] == 0.0 && pb[1][1] == 0.0)) continue;
        for (int ci = max(fi - 2, 0); ci <= min(fi + 1, g.nx - 1); ++ci) {
          pa[0][0] = p1(ax, ci, I); pa[0][1] = p1(ax, ci + 1, I);
          pb[0][0] = p1(ax, ci, I2); pb[0][1] = p1(ax, ci + 1, I2);
          if ((pa[0][0] == 0.0 && pa[0][1] == 0.0) || (pb[0][0] == 0.0 && pb[0][1] == 0.0)) continue;
          cell_galerkin(g, dead0, ci, cj, ck, pa, pb, acc);
        }
      }
    }
  }
  const int64_t node = int64_t(K) * csz + int64_t(J) * csy + I;
#pragma unroll
  for (int e = 0; e < 9; ++e) A[stencil_idx(q, e / 3, e % 3, cn, node)] = T(acc[e]);
}

// Coarse stencil of level l+1 from the stencil of level l (F).
template <typename T>
__global__ __launch_bounds__(256) void mg_galerkin_kernel(MgLevel<T> F, int cnx, int cny, int cnz, int64_t csy,
                                                          int64_t csz, int64_t cn, T *A) {
  const int I = blockIdx.x * BX + threadIdx.x, J = blockIdx.y * BY + threadIdx.y;
  const int K = blockIdx.z / kMgUpper, q = blockIdx.z % kMgUpper;
  if (I > cnx || J > cny) return;
  int ox, oy, oz;
  off3(q + 13, ox, oy, oz);
  const int I2 = I + ox, J2 = J + oy, K2 = K + oz;
  double acc[9] = {};
  if (I2 >= 0 && I2 <= cnx && J2 >= 0 && J2 <= cny && K2 >= 0 && K2 <= cnz) {
    const int fi0 = F.ax[0].cpos[I], fj0 = F.ax[1].cpos[J], fk0 = F.ax[2].cpos[K];
    for (int fk = max(fk0 - 1, 0); fk <= min(fk0 + 1, F.nz); ++fk) {
      const double wk = p1(F.ax[2], fk, K);
      if (wk == 0.0) continue;
      double bz[3];
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const int gk = fk + t - 1;
        bz[t] = (gk >= 0 && gk <= F.nz) ? p1(F.ax[2], gk, K2) : 0.0;
      }
      for (int fj = max(fj0 - 1, 0); fj <= min(fj0 + 1, F.ny); ++fj) {
        const double wj = p1(F.ax[1], fj, J);
        if (wj == 0.0) continue;
        double by[3];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          const int gj = fj + t - 1;
          by[t] = (gj >= 0 && gj <= F.ny) ? p1(F.ax[1], gj, J2) : 0.0;
        }
        for (int fi = max(fi0 - 1, 0); fi <= min(fi0 + 1, F.nx); ++fi) {
          const double wi = p1(F.ax[0], fi, I);
          if (wi == 0.0) continue;
          double bx[3];
#pragma unroll
          for (int t = 0; t < 3; ++t) {
            const int gi = fi + t - 1;
            bx[t] = (gi >= 0 && gi <= F.nx) ? p1(F.ax[0], gi, I2) : 0.0;
          }
          const double wa = wi * wj * wk;
          const int64_t fn = int64_t(fk) * F.sz + int64_t(fj) * F.sy + fi;
          for (int o = 0; o < 27; ++o) {
            int dx, dy, dz;
            off3(o, dx, dy, dz);
            const double wb = bx[dx + 1] * by[dy + 1] * bz[dz + 1];
            if (wb == 0.0) continue;
            double B[9];
            stencil_block<T>(F, fn, o, B);
            const double w = wa * wb;
#pragma unroll
            for (int e = 0; e < 9; ++e) acc[e] += w * B[e];
          }
        }
      }
    }
  }
  const int64_t node = int64_t(K) * csz + int64_t(J) * csy + I;
#pragma unroll
  for (int e = 0; e < 9; ++e) A[stencil_idx(q, e / 3, e % 3, cn, node)] = T(acc[e]);
}

// Deterministic start vector of the power iteration (dead DOFs zero).
template <typename T>
__global__ __launch_bounds__(256) void mg_start_kernel(MgLevel<T> L, V3<T> v) {
  int i, j, k;
  plane_node(L.nx, i, j, k);
  if (i > L.nx || j > L.ny) return;
  const int64_t n = int64_t(k) * L.sz + int64_t(j) * L.sy + i;
  const uint8_t dd = L.dead[n];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    uint32_t h = uint32_t(n) * 2654435761u ^ uint32_t(c + 1) * 2246822519u;
    h ^= h >> 15; h *= 2246822519u; h ^= h >> 13; h *= 3266489917u; h ^= h >> 16;
    const double r = double(h) * (1.0 / 4294967296.0) - 0.5;
    v.c[c][n] = (dd >> c & 1) ? T(0) : T(r);
  }
}

// Power iteration for lambda_max(Dinv A).  With u = scale * v (unit length
// after the first step), y = A u and z = Dinv y, the kernel stores w = z and
// sums z.y, u.y and |z|^2.  Dinv A is self-adjoint in the A inner product,
// so z.y / u.y = <u, Dinv A u>_A / <u, u>_A is a Rayleigh quotient: a lower
// bound of lambda_max whose error falls as (lambda_2 / lambda_1)^(2k), twice
// the rate of the norm ratio |z|.
__device__ __forceinline__ void power_sums(const double u[3], const double y[3], const double z[3], double red[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    red[0] += z[c] * y[c];
    red[1] += u[c] * y[c];
    red[2] += z[c] * z[c];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void mg_power_kernel(MgLevel<T> L, V3<T> v, V3<T> w,
                                                       const double *scale, double *partials) {
  int i, j, k;
  plane_node(L.nx, i, j, k);
  double red[3] = {0.0, 0.0, 0.0};
  if (i <= L.nx && j <= L.ny) {
    const int64_t n = int64_t(k) * L.sz + int64_t(j) * L.sy + i;
    T y[3];
    stencil_apply<T>(L, i, j, k, n, v, y);
    const T s = T(*scale);
    const int64_t N = L.n;
    const T d00 = L.Dinv[n], d11 = L.Dinv[N + n], d22 = L.Dinv[2 * N + n];
    const T d01 = L.Dinv[3 * N + n], d12 = L.Dinv[4 * N + n], d02 = L.Dinv[5 * N + n];
    const T z0 = s * (d00 * y[0] + d01 * y[1] + d02 * y[2]);
    const T z1 = s * (d01 * y[0] + d11 * y[1] + d12 * y[2]);
    const T z2 = s * (d02 * y[0] + d12 * y[1] + d22 * y[2]);
    w.c[0][n] = z0; w.c[1][n] = z1; w.c[2][n] = z2;
    const double u[3] = {double(s) * double(v.c[0][n]), double(s) * double(v.c[1][n]), double(s) * double(v.c[2][n])};
    const double ys[3] = {double(s) * double(y[0]), double(s) * double(y[1]), double(s) * double(y[2])};
    const double zd[3] = {double(z0), double(z1), double(z2)};
    power_sums(u, ys, zd, red);
  }
  const int64_t b = (int64_t(blockIdx.z) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  block_sums<3>(red, partials + b * kRedWidth);
}

__global__ void mg_power_finalize(const double *part, int64_t nb, double *lam, double *scale) {
  __shared__ double out[3];
  sum_partials<3>(part, nb, out);
  if (threadIdx.x == 0) {
    const double zn = sqrt(out[2]);
    *lam = out[1] > 0.0 ? out[0] / out[1] : 0.0;
    *scale = zn > 0.0 ? 1.0 / zn : 0.0;
  }
}

__global__ void mg_scalar_set(double *p, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// ---- V-cycle --------------------------------------------------------------------

// First Chebyshev step from x = 0 at node n: d = x = c2 Dinv b.
template <typename T>
__device__ __forceinline__ void first_step(const MgLevel<T> &L, int64_t n, T b0, T b1, T b2, T c2) {
  const int64_t N = L.n;
  const T d00 = L.Dinv[n], d11 = L.Dinv[N + n], d22 = L.Dinv[2 * N + n];
  const T d01 = L.Dinv[3 * N + n], d12 = L.Dinv[4 * N + n], d02 = L.Dinv[5 * N + n];
  const T z0 = c2 * (d00 * b0 + d01 * b1 + d02 * b2);
  const T z1 = c2 * (d01 * b0 + d11 * b1 + d12 * b2);
  const T z2 = c2 * (d02 * b0 + d12 * b1 + d22 * b2);
  L.d.c[0][n] = z0; L.d.c[1][n] = z1; L.d.c[2][n] = z2;
  L.xa.c[0][n] = z0; L.xa.c[1][n] = z1; L.xa.c[2][n] = z2;
}

// One Chebyshev step: r = b - A x_in (r = b when first: x_in = 0),
// d = c1 d + c2 Dinv r, x_out = x_in + d.
template <typename T>
__global__ __launch_bounds__(256) void mg_smooth_kernel(MgLevel<T> L, V3<T> b, V3<T> xin, V3<T> xout,
                                                        T c1, T c2, int first, const DevScalars *sc) {
  if (sc && sc->done) return;
  int i, j, k;
  plane_node(L.nx, i, j, k);
  if (i > L.nx || j > L.ny) return;
  const int64_t n = int64_t(k) * L.sz + int64_t(j) * L.sy + i;
  T r[3];
  if (first) {
    r[0] = b.c[0][n]; r[1] = b.c[1][n]; r[2] = b.c[2][n];
  } else {
    T y[3];
    stencil_apply<T>(L, i, j, k, n, xin, y);
    r[0] = b.c[0][n] - y[0]; r[1] = b.c[1][n] - y[1]; r[2] = b.c[2][n] - y[2];
  }
  const int64_t N = L.n;
  const T d00 = L.Dinv[n], d11 = L.Dinv[N + n], d22 = L.Dinv[2 * N + n];
  const T d01 = L.Dinv[3 * N + n], d12 = L.Dinv[4 * N + n], d02 = L.Dinv[5 * N + n];
  const T z[3] = {d00 * r[0] + d01 * r[1] + d02 * r[2], d01 * r[0] + d11 * r[1] + d12 * r[2],
                  d02 * r[0] + d12 * r[1] + d22 * r[2]};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T dn = c2 * z[c];
    if (c1 != T(0)) dn += c1 * L.d.c[c][n];
    L.d.c[c][n] = dn;
    xout.c[c][n] = (first ? T(0) : xin.c[c][n]) + dn;
  }
}

// r = b - A x.
template <typename T>
__global__ __launch_bounds__(256) void mg_resid_kernel(MgLevel<T> L, V3<T> b, V3<T> x, V3<T> r,
                                                       const DevScalars *sc) {
  if (sc && sc->done) return;
  int i, j, k;
  plane_node(L.nx, i, j, k);
  if (i > L.nx || j > L.ny) return;
  const int64_t n = int64_t(k) * L.sz + int64_t(j) * L.sy + i;
  T y[3];
  stencil_apply<T>(L, i, j, k, n, x, y);
#pragma unroll
  for (int c = 0; c < 3; ++c) r.c[c][n] = b.c[c][n] - y[c];
}

// b_C = P^T r_F (one thread per coarse node).  With smooth != 0 the coarse
// level's first Chebyshev step (x = 0, so pointwise) follows at once:
// d_C = x_C = c2 Dinv_C b_C.
template <typename T>
__global__ __launch_bounds__(256) void mg_restrict_kernel(MgLevel<T> F, V3<T> r, MgLevel<T> C, int smooth, T c2,
                                                          const DevScalars *sc) {
  if (sc && sc->done) return;
  int I, J, K;
  plane_node(C.nx, I, J, K);
  if (I > C.nx || J > C.ny) return;
  const int fi0 = F.ax[0].cpos[I], fj0 = F.ax[1].cpos[J], fk0 = F.ax[2].cpos[K];
  // the 1D weights of the three fine nodes around the coarse node on each
  // axis first (0 outside the level), then per fine plane its nine nodes'
  // loads together, summed in the order fk, fj, fi where a zero weight adds
  // nothing
  double wi[3], wj[3], wk[3];
  int fi[3], fj[3], fk[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    fi[q] = fi0 - 1 + q; fj[q] = fj0 - 1 + q; fk[q] = fk0 - 1 + q;
    const bool oi = fi[q] >= 0 && fi[q] <= F.nx, oj = fj[q] >= 0 && fj[q] <= F.ny, ok = fk[q] >= 0 && fk[q] <= F.nz;
    if (!oi) fi[q] = fi0;
    if (!oj) fj[q] = fj0;
    if (!ok) fk[q] = fk0;
    wi[q] = oi ? p1(F.ax[0], fi[q], I) : 0.0;
    wj[q] = oj ? p1(F.ax[1], fj[q], J) : 0.0;
    wk[q] = ok ? p1(F.ax[2], fk[q], K) : 0.0;
  }
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll 1
  for (int qk = 0; qk < 3; ++qk) {
    if (wk[qk] == 0.0) continue;
    double rv[9][3];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int64_t fn = int64_t(fk[qk]) * F.sz + int64_t(fj[t / 3]) * F.sy + fi[t % 3];
#pragma unroll
      for (int c = 0; c < 3; ++c) rv[t][c] = double(r.c[c][fn]);
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const double wjj = wj[t / 3], wii = wi[t % 3];
      if (wjj == 0.0 || wii == 0.0) continue;
      const double w = wii * wjj * wk[qk];
      a0 += w * rv[t][0];
      a1 += w * rv[t][1];
      a2 += w * rv[t][2];
    }
  }
  const int64_t cn = int64_t(K) * C.sz + int64_t(J) * C.sy + I;
  const uint8_t dd = C.dead[cn];
  const T b0 = (dd & 1) ? T(0) : T(a0), b1 = (dd & 2) ? T(0) : T(a1), b2 = (dd & 4) ? T(0) : T(a2);
  C.b.c[0][cn] = b0;
  C.b.c[1][cn] = b1;
  C.b.c[2][cn] = b2;
  if (smooth) first_step<T>(C, cn, b0, b1, b2, c2);
}

// x_F += P x_C on the live DOFs of F (one thread per fine node).
template <typename T>
__global__ __launch_bounds__(256) void mg_prolong_kernel(MgLevel<T> F, V3<T> x, MgLevel<T> C, V3<T> xc,
                                                         const DevScalars *sc) {
  if (sc && sc->done) return;
  int i, j, k;
  plane_node(F.nx, i, j, k);
  if (i > F.nx || j > F.ny) return;
  const int64_t n = int64_t(k) * F.sz + int64_t(j) * F.sy + i;
  const int lx = F.ax[0].lo[i], ly = F.ax[1].lo[j], lz = F.ax[2].lo[k];
  const double wx[2] = {F.ax[0].w[i], 1.0 - F.ax[0].w[i]};
  const double wy[2] = {F.ax[1].w[j], 1.0 - F.ax[1].w[j]};
  const double wz[2] = {F.ax[2].w[k], 1.0 - F.ax[2].w[k]};
  // the eight corners' loads first (a corner of weight 0 may lie past the
  // last coarse node: it reads the first corner instead), then the sums in
  // corner order, where a zero weight adds nothing
  double w[8], xv[8][3];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int tx = t & 1, ty = (t >> 1) & 1, tz = t >> 2;
    w[t] = wx[tx] * wy[ty] * wz[tz];
    const int64_t cn = w[t] != 0.0 ? int64_t(lz + tz) * C.sz + int64_t(ly + ty) * C.sy + (lx + tx)
                                   : int64_t(lz) * C.sz + int64_t(ly) * C.sy + lx;
#pragma unroll
    for (int c = 0; c < 3; ++c) xv[t][c] = double(xc.c[c][cn]);
  }
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    if (w[t] == 0.0) continue;
    a0 += w[t] * xv[t][0];
    a1 += w[t] * xv[t][1];
    a2 += w[t] * xv[t][2];
  }
  const uint8_t dd = F.dead[n];
  if (!(dd & 1)) x.c[0][n] += T(a0);
  if (!(dd & 2)) x.c[1][n] += T(a1);
  if (!(dd & 4)) x.c[2][n] += T(a2);
}

template <typename T>
__global__ __launch_bounds__(256) void mg_zero_kernel(MgLevel<T> L, V3<T> x, const DevScalars *sc) {
  if (sc && sc->done) return;
  int i, j, k;
  plane_node(L.nx, i, j, k);
  if (i > L.nx || j > L.ny) return;
  const int64_t n = int64_t(k) * L.sz + int64_t(j) * L.sy + i;
  x.c[0][n] = T(0); x.c[1][n] = T(0); x.c[2][n] = T(0);
}

// Coarsest level: x[live] = Ainv b[live] (Ainv symmetric, read by
// columns).  b[live] is staged in LDS; each block owns 32 rows and splits
// every row's sum over 8 thread groups, reduced in a fixed order.
constexpr int kDenseRows = 32, kDenseParts = 8;
template <typename T>
__global__ __launch_bounds__(256) void mg_dense_kernel(const T *Ainv, const int32_t *live, int nl, V3<T> b, V3<T> x,
                                                       const DevScalars *sc) {
  if (sc && sc->done) return;
  extern __shared__ double bs[];
  __shared__ double red[kDenseParts][kDenseRows];
  for (int j = threadIdx.x; j < nl; j += blockDim.x) {
    const int code = live[j];
    bs[j] = double(b.c[code % 3][code / 3]);
  }
  __syncthreads();
  const int lane = threadIdx.x % kDenseRows, part = threadIdx.x / kDenseRows;
  const int r = blockIdx.x * kDenseRows + lane;
  double acc = 0.0;
  if (r < nl) {
    // eight loads in flight, summed in the same order
    int j = part;
    for (; j + 7 * kDenseParts < nl; j += 8 * kDenseParts) {
      double a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = double(Ainv[int64_t(j + u * kDenseParts) * nl + r]);
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += a[u] * bs[j + u * kDenseParts];
    }
    for (; j < nl; j += kDenseParts) acc += double(Ainv[int64_t(j) * nl + r]) * bs[j];
  }
  red[part][lane] = acc;
  __syncthreads();
  if (part == 0 && r < nl) {
    double sum = red[0][lane];
#pragma unroll
    for (int q = 1; q < kDenseParts; ++q) sum += red[q][lane];
    const int cr = live[r];
    x.c[cr % 3][cr / 3] = T(sum);
  }
}

// ---- level 0 on the cell-based HEX8 apply -----------------------------------------

// Chebyshev step on level 0 (x_in = the applied vector): r = b - K x_in,
// d = c1 d + c2 Dinv r, x_out = x_in + d.
template <typename T>
__device__ __forceinline__ void dinv_load(const MgLevel<T> &L, int64_t n, T D[6]) {
#pragma unroll
  for (int e = 0; e < 6; ++e) D[e] = L.Dinv[e * L.n + n];
}

template <typename T>
__device__ __forceinline__ void dinv_apply(const T D[6], const T r[3], T z[3]) {
  z[0] = D[0] * r[0] + D[3] * r[1] + D[5] * r[2];
  z[1] = D[3] * r[0] + D[1] * r[1] + D[4] * r[2];
  z[2] = D[5] * r[0] + D[4] * r[1] + D[2] * r[2];
}

template <typename T>
struct EpiSmooth0 {
  MgLevel<T> L;
  V3<T> b, xout;
  T c1, c2;
  struct Pre { T b[3], D[6], d[3]; };
  __device__ Pre load(int64_t n) const {
    Pre q;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      q.b[c] = b.c[c][n];
      q.d[c] = c1 != T(0) ? L.d.c[c][n] : T(0);
    }
    dinv_load<T>(L, n, q.D);
    return q;
  }
  __device__ void operator()(int64_t n, const T y[3], const T xc[3], const Pre &q, double *) const {
    const T r[3] = {q.b[0] - y[0], q.b[1] - y[1], q.b[2] - y[2]};
    T z[3];
    dinv_apply<T>(q.D, r, z);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T dn = c2 * z[c] + c1 * q.d[c];
      L.d.c[c][n] = dn;
      xout.c[c][n] = xc[c] + dn;
    }
  }
};

// The last post-smoothing step of a V-cycle that CG applies to its residual
// b = r: also the dot product r . z of the result z = x_out (per-block sums
// into the partials), so no separate pass reads r and z again.
template <typename T>
struct EpiSmooth0Dot : EpiSmooth0<T> {
  __device__ void operator()(int64_t n, const T y[3], const T xc[3], const typename EpiSmooth0<T>::Pre &q,
                             double *red) const {
    const T r[3] = {q.b[0] - y[0], q.b[1] - y[1], q.b[2] - y[2]};
    T z[3];
    dinv_apply<T>(q.D, r, z);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T dn = this->c2 * z[c] + this->c1 * q.d[c];
      this->L.d.c[c][n] = dn;
      const T xo = xc[c] + dn;
      this->xout.c[c][n] = xo;
      red[0] += double(q.b[c]) * double(xo);
    }
  }
};

template <typename T>
struct EpiResid0 {
  V3<T> b, r;
  struct Pre { T b[3]; };
  __device__ Pre load(int64_t n) const { return Pre{{b.c[0][n], b.c[1][n], b.c[2][n]}}; }
  __device__ void operator()(int64_t n, const T y[3], const T *, const Pre &q, double *) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) r.c[c][n] = q.b[c] - y[c];
  }
};

template <typename T>
struct EpiPower0 {
  MgLevel<T> L;
  V3<T> w;
  const double *scale;
  struct Pre { T D[6]; };
  __device__ Pre load(int64_t n) const {
    Pre q;
    dinv_load<T>(L, n, q.D);
    return q;
  }
  // the power step of mg_power_kernel on the matrix-free level (sums z.y, u.y, |z|^2)
  __device__ void operator()(int64_t n, const T y[3], const T xc[3], const Pre &q, double *red) const {
    T z[3];
    dinv_apply<T>(q.D, y, z);
    const T s = T(*scale);
    double u[3], ys[3], zd[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      z[c] *= s;
      w.c[c][n] = z[c];
      u[c] = double(s) * double(xc[c]);
      ys[c] = double(s) * double(y[c]);
      zd[c] = double(z[c]);
    }
    power_sums(u, ys, zd, red);
  }
};

// CG start on level 0: r = b - K u, |r|^2, and the first smoothing step.
template <typename T>
struct EpiStart0 {
  CgVecs<T> v;
  const T *b0, *b1, *b2;
  MgLevel<T> L0;
  int smooth;
  T c2;
  struct Pre { T b[3]; };
  __device__ Pre load(int64_t n) const { return Pre{{b0[n], b1[n], b2[n]}}; }
  __device__ void operator()(int64_t n, const T y[3], const T *, const Pre &q, double *red) const {
    const T r0 = q.b[0] - y[0], r1 = q.b[1] - y[1], r2 = q.b[2] - y[2];
    v.r[0][n] = r0; v.r[1][n] = r1; v.r[2][n] = r2;
    red[0] += double(r0) * double(r0) + double(r1) * double(r1) + double(r2) * double(r2);
    if (smooth) first_step<T>(L0, n, r0, r1, r2, c2);
  }
};

// ---- CG with the V-cycle ------------------------------------------------------------

// Start of an inner CG (a restart of the solve).  With a gate: skipped while
// the gate says so (the inner CG already running goes on); when it runs, the
// gate then tells the rest of the setup whether the inner CG has work.
__global__ void cgmg_start_finalize(const double *part, int64_t nb, DevScalars *sc, DevScalars *gate) {
  if (gate && gate->done) return;
  __shared__ double out[1];
  sum_partials<1>(part, nb, out);
  if (threadIdx.x == 0) {
    sc->rr = out[0];
    sc->iters = 0;
    sc->done = (out[0] <= sc->tol2) ? 1 : 0;
    sc->alpha = sc->beta = sc->rz = 0.0;
    sc->restart = 0;
    if (gate) gate->done = sc->done;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void cgmg_dot_kernel(MechGrid M, CgVecs<T> v, V3<T> z, const DevScalars *sc,
                                                       double *partials) {
  if (sc->done) return;
  const DevGrid &g = M.g;
  int i, j, k;
  plane_node(g.nx, i, j, k);
  double rz = 0.0;
  if (i <= g.nx && j <= g.ny) {
    const int64_t n = int64_t(k) * g.sz + int64_t(j) * g.sy + i;
#pragma unroll
    for (int c = 0; c < 3; ++c) rz += double(v.r[c][n]) * double(z.c[c][n]);
  }
  const double s[1] = {rz};
  const int64_t b = (int64_t(blockIdx.z) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  block_sums<1>(s, partials + b * kRedWidth);
}

// rz_new = r . z; beta = rz_new / rz (first: none).  A non-positive r . z
// means the preconditioned residual vanished or M^{-1} lost definiteness:
// stop; the caller checks the true residual.
__global__ void cgmg_rz_finalize(const double *part, int64_t nb, DevScalars *sc, int first, const DevScalars *gate) {
  if (gate ? gate->done : sc->done) return;
  __shared__ double out[1];
  sum_partials<1>(part, nb, out);
  if (threadIdx.x == 0) {
    const double rzn = out[0];
    if (!(rzn > 0.0)) {
      sc->done = 1;
      return;
    }
    sc->beta = first ? 0.0 : rzn / sc->rz;
    sc->rz = rzn;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void cgmg_p_kernel(CgVecs<T> v, V3<T> z, int64_t ntot, const DevScalars *sc,
                                                     int first, const DevScalars *gate) {
  if (gate ? gate->done : sc->done) return;
  const T beta = T(sc->beta);
  for (int64_t n = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; n < ntot; n += int64_t(gridDim.x) * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 3; ++c) v.p[c][n] = first ? z.c[c][n] : z.c[c][n] + beta * v.p[c][n];
  }
}

// u += alpha p, r -= alpha w, |r|^2; with smooth != 0 also the level-0
// first Chebyshev step on r (padding entries have Dinv = 0).
template <typename T>
__global__ __launch_bounds__(256) void cgmg_update_kernel(CgVecs<T> v, int64_t ntot, MgLevel<T> L0, int smooth, T c2,
                                                          const DevScalars *sc, double *partials) {
  if (sc->done) return;
  const T alpha = T(sc->alpha);
  double rr = 0.0;
  for (int64_t n = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; n < ntot; n += int64_t(gridDim.x) * blockDim.x) {
    T r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      v.u[c][n] += alpha * v.p[c][n];
      r[c] = v.r[c][n] - alpha * v.w[c][n];
      v.r[c][n] = r[c];
      rr += double(r[c]) * double(r[c]);
    }
    if (smooth) first_step<T>(L0, n, r[0], r[1], r[2], c2);
  }
  const double s[1] = {rr};
  block_sums<1>(s, partials + int64_t(blockIdx.x) * kRedWidth);
}

__global__ void cgmg_rr_finalize(const double *part, int64_t nb, DevScalars *sc) {
  if (sc->done) return;
  __shared__ double out[1];
  sum_partials<1>(part, nb, out);
  if (threadIdx.x == 0) {
    sc->iters += 1;
    sc->rr = out[0];
    if (out[0] <= sc->tol2 || sc->iters >= sc->budget) sc->done = 1;
  }
}

inline int flat_blocks(int64_t n) { return int(std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024))); }

// One thread per node of a plane (plane_node), blockIdx.z the plane.
template <typename T>
inline dim3 lgrid(const MgLevel<T> &L) {
  const int64_t plane = int64_t(L.nx + 1) * (L.ny + 1);
  return dim3(unsigned((plane + BX * BY - 1) / (BX * BY)), 1, L.nz + 1);
}

template <typename T>
inline int64_t lblocks(const MgLevel<T> &L) {
  const dim3 g = lgrid(L);
  return int64_t(g.x) * g.y * g.z;
}

template <typename T>
hipError_t smooth(const MgDev<T> &G, int l, V3<T> b, V3<T> xin, V3<T> xout, int step, int first,
                  const DevScalars *sc, hipStream_t s, double *dot_partials = nullptr) {
  const MgLevel<T> &L = G.L[l];
  const T c1 = T(L.c1[step]), c2 = T(L.c2[step]);
  if (l == 0 && !first && dot_partials)
    return launch_hex8<T, 1>(G.M, xin.c, EpiSmooth0Dot<T>{{L, b, xout, c1, c2}}, dot_partials, sc, s);
  if (l == 0 && !first)
    return launch_hex8<T, 0>(G.M, xin.c, EpiSmooth0<T>{L, b, xout, c1, c2}, nullptr, sc, s);
  hipLaunchKernelGGL((mg_smooth_kernel<T>), lgrid(L), dim3(BX, BY), 0, s, L, b, xin, xout, c1, c2, first, sc);
  return hipGetLastError();
}

// Coarse levels get their first smoothing step inside the restriction, and
// level 0 inside the CG kernel that forms r (first_done).
template <typename T>
hipError_t vcycle_level(const MgDev<T> &G, int l, V3<T> b, const DevScalars *sc, V3<T> *out, hipStream_t s,
                        bool first_done, double *dot_partials = nullptr) {
  const MgLevel<T> &L = G.L[l];
  hipError_t e;
  if (l == G.nlev - 1) {
    hipLaunchKernelGGL((mg_zero_kernel<T>), lgrid(L), dim3(BX, BY), 0, s, L, L.xa, sc);
    if (G.nlive > 0)
      hipLaunchKernelGGL((mg_dense_kernel<T>), dim3((G.nlive + kDenseRows - 1) / kDenseRows), dim3(256),
                         size_t(G.nlive) * sizeof(double), s, (const T *)G.Ainv, (const int32_t *)G.live, G.nlive, b,
                         L.xa, sc);
    *out = L.xa;
    return hipGetLastError();
  }
  V3<T> xc = L.xa, xo = L.xb;
  if (!first_done && (e = smooth(G, l, b, xo, xc, 0, 1, sc, s)) != hipSuccess) return e;
  for (int k = 1; k < L.deg; ++k) {
    if ((e = smooth(G, l, b, xc, xo, k, 0, sc, s)) != hipSuccess) return e;
    std::swap(xc, xo);
  }
  if (l == 0) {
    if ((e = launch_hex8<T, 0>(G.M, xc.c, EpiResid0<T>{b, xo}, nullptr, sc, s)) != hipSuccess) return e;
  } else {
    hipLaunchKernelGGL((mg_resid_kernel<T>), lgrid(L), dim3(BX, BY), 0, s, L, b, xc, xo, sc);
  }
  const MgLevel<T> &C = G.L[l + 1];
  const int fuse = l + 2 < G.nlev;  // the coarse level smooths (it is not the coarsest)
  hipLaunchKernelGGL((mg_restrict_kernel<T>), lgrid(C), dim3(BX, BY), 0, s, L, xo, C, fuse, T(C.c2[0]), sc);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  V3<T> xcoarse;
  if ((e = vcycle_level(G, l + 1, C.b, sc, &xcoarse, s, fuse != 0)) != hipSuccess) return e;
  hipLaunchKernelGGL((mg_prolong_kernel<T>), lgrid(L), dim3(BX, BY), 0, s, L, xc, C, xcoarse, sc);
  for (int k = 0; k < L.deg; ++k) {
    // with dot_partials (level 0 of a CG step): the last step also forms b . out
    double *dp = (l == 0 && k + 1 == L.deg) ? dot_partials : nullptr;
    if ((e = smooth(G, l, b, xc, xo, k, 0, sc, s, dp)) != hipSuccess) return e;
    std::swap(xc, xo);
  }
  *out = xc;
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_mg_build(const MgDev<T> &G, hipStream_t s) {
  const MgLevel<T> &L0 = G.L[0];
  hipLaunchKernelGGL((mg_diag0_kernel<T>), lgrid(L0), dim3(BX, BY), 0, s, G.M, L0.Dinv, L0.n, L0.dead);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (G.nlev == 1) {  // level 0 is the coarsest: assemble its stencil (identity tables)
    dim3 grid((L0.nx + 1 + BX - 1) / BX, (L0.ny + 1 + BY - 1) / BY, (L0.nz + 1) * kMgUpper);
    hipLaunchKernelGGL((mg_galerkin0_kernel<T>), grid, dim3(BX, BY), 0, s, G.M, (const uint8_t *)L0.dead, L0.ax[0],
                       L0.ax[1], L0.ax[2], L0.nx, L0.ny, L0.nz, L0.sy, L0.sz, L0.n, const_cast<T *>(L0.A));
    return hipGetLastError();
  }
  for (int l = 0; l + 1 < G.nlev; ++l) {
    const MgLevel<T> &F = G.L[l], &C = G.L[l + 1];
    dim3 grid((C.nx + 1 + BX - 1) / BX, (C.ny + 1 + BY - 1) / BY, (C.nz + 1) * kMgUpper);
    if (l == 0)
      hipLaunchKernelGGL((mg_galerkin0_kernel<T>), grid, dim3(BX, BY), 0, s, G.M, (const uint8_t *)F.dead, F.ax[0],
                         F.ax[1], F.ax[2], C.nx, C.ny, C.nz, C.sy, C.sz, C.n, const_cast<T *>(C.A));
    else
      hipLaunchKernelGGL((mg_galerkin_kernel<T>), grid, dim3(BX, BY), 0, s, F, C.nx, C.ny, C.nz, C.sy, C.sz, C.n,
                         const_cast<T *>(C.A));
    hipLaunchKernelGGL((mg_diag_kernel<T>), lgrid(C), dim3(BX, BY), 0, s, C);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
hipError_t launch_mg_power(const MgDev<T> &G, int l, int iters, double *partials, hipStream_t s) {
  const MgLevel<T> &L = G.L[l];
  hipLaunchKernelGGL((mg_start_kernel<T>), lgrid(L), dim3(BX, BY), 0, s, L, L.xa);
  hipLaunchKernelGGL(mg_scalar_set, dim3(1), dim3(64), 0, s, G.scale, 1.0);
  V3<T> v = L.xa, w = L.xb;
  const int64_t nb = l == 0 ? cell_blocks(G.M.g, cell_kchunk(G.M.g)) : lblocks(L);
  for (int it = 0; it < iters; ++it) {
    if (l == 0) {
      hipError_t e = launch_hex8<T, 3>(G.M, v.c, EpiPower0<T>{L, w, (const double *)G.scale}, partials, nullptr, s);
      if (e != hipSuccess) return e;
    } else {
      hipLaunchKernelGGL((mg_power_kernel<T>), lgrid(L), dim3(BX, BY), 0, s, L, v, w, (const double *)G.scale,
                         partials);
    }
    hipLaunchKernelGGL(mg_power_finalize, dim3(1), dim3(256), 0, s, (const double *)partials, nb, G.lam + l,
                       G.scale);
    std::swap(v, w);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mg_vcycle(const MgDev<T> &G, V3<T> b, const DevScalars *sc, V3<T> *z, hipStream_t s) {
  return vcycle_level(G, 0, b, sc, z, s, false);
}

template <typename T>
hipError_t launch_cgmg_setup(const MgDev<T> &G, const CgVecs<T> &v, const T *rhs[3], double *partials,
                             DevScalars *sc, DevScalars *gate, hipStream_t s) {
  const MgLevel<T> &L0 = G.L[0];
  const int64_t nb = lblocks(L0);
  const int fuse = G.nlev > 1;
  const T *u[3] = {v.u[0], v.u[1], v.u[2]};
  hipError_t e0 = launch_hex8<T, 1>(G.M, u, EpiStart0<T>{v, rhs[0], rhs[1], rhs[2], L0, fuse, T(L0.c2[0])}, partials,
                                    gate, s);
  if (e0 != hipSuccess) return e0;
  hipLaunchKernelGGL(cgmg_start_finalize, dim3(1), dim3(256), 0, s, (const double *)partials,
                     cell_blocks(G.M.g, cell_kchunk(G.M.g)), sc, gate);
  // the rest of the setup runs only after a restart that left work to do
  const DevScalars *g2 = gate ? (const DevScalars *)gate : (const DevScalars *)sc;
  V3<T> r{{v.r[0], v.r[1], v.r[2]}}, z;
  // with more than one level the V-cycle's last level-0 step forms r . z
  hipError_t e = vcycle_level(G, 0, r, g2, &z, s, fuse != 0, fuse ? partials : nullptr);
  if (e != hipSuccess) return e;
  if (!fuse) hipLaunchKernelGGL((cgmg_dot_kernel<T>), lgrid(L0), dim3(BX, BY), 0, s, G.M, v, z, g2, partials);
  hipLaunchKernelGGL(cgmg_rz_finalize, dim3(1), dim3(256), 0, s, (const double *)partials,
                     fuse ? cell_blocks(G.M.g, cell_kchunk(G.M.g)) : nb, sc, 1, g2);
  hipLaunchKernelGGL((cgmg_p_kernel<T>), dim3(flat_blocks(L0.n)), dim3(256), 0, s, v, z, L0.n,
                     (const DevScalars *)sc, 1, g2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cgmg_iteration(const MgDev<T> &G, const CgVecs<T> &v, double *partials, DevScalars *sc,
                                 hipStream_t s) {
  const MgLevel<T> &L0 = G.L[0];
  const int64_t nb = lblocks(L0);
  hipError_t e = launch_cg_apply_alpha<T>(G.M, v, partials, sc, s);
  if (e != hipSuccess) return e;
  const int fb = flat_blocks(L0.n);
  const int fuse = G.nlev > 1;
  hipLaunchKernelGGL((cgmg_update_kernel<T>), dim3(fb), dim3(256), 0, s, v, L0.n, L0, fuse, T(L0.c2[0]),
                     (const DevScalars *)sc, partials);
  hipLaunchKernelGGL(cgmg_rr_finalize, dim3(1), dim3(256), 0, s, (const double *)partials, int64_t(fb), sc);
  V3<T> r{{v.r[0], v.r[1], v.r[2]}}, z;
  // with more than one level the V-cycle's last level-0 step forms r . z
  if ((e = vcycle_level(G, 0, r, sc, &z, s, fuse != 0, fuse ? partials : nullptr)) != hipSuccess) return e;
  if (!fuse)
    hipLaunchKernelGGL((cgmg_dot_kernel<T>), lgrid(L0), dim3(BX, BY), 0, s, G.M, v, z, (const DevScalars *)sc,
                       partials);
  hipLaunchKernelGGL(cgmg_rz_finalize, dim3(1), dim3(256), 0, s, (const double *)partials,
                     fuse ? cell_blocks(G.M.g, cell_kchunk(G.M.g)) : nb, sc, 0, (const DevScalars *)nullptr);
  hipLaunchKernelGGL((cgmg_p_kernel<T>), dim3(fb), dim3(256), 0, s, v, z, L0.n, (const DevScalars *)sc, 0,
                     (const DevScalars *)nullptr);
  return hipGetLastError();
}

#define ETM_MG_INST(T)                                                                                     \
  template hipError_t launch_mg_build<T>(const MgDev<T> &, hipStream_t);                                   \
  template hipError_t launch_mg_power<T>(const MgDev<T> &, int, int, double *, hipStream_t);               \
  template hipError_t launch_mg_vcycle<T>(const MgDev<T> &, V3<T>, const DevScalars *, V3<T> *, hipStream_t); \
  template hipError_t launch_cgmg_setup<T>(const MgDev<T> &, const CgVecs<T> &, const T *[3], double *,    \
                                           DevScalars *, DevScalars *, hipStream_t);                       \
  template hipError_t launch_cgmg_iteration<T>(const MgDev<T> &, const CgVecs<T> &, double *, DevScalars *, \
                                               hipStream_t);
ETM_MG_INST(double)
ETM_MG_INST(float)
#undef ETM_MG_INST

}  // namespace etm
