// Device helpers shared by the mechanics kernels (mech.hip) and the
// multigrid preconditioner (mg.hip): node-grid launch shape, wave64 and block
// reductions in FP64, and the matrix-free HEX8 stiffness of Eq. (8) applied
// cell by cell.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "etm_internal.h"

namespace etm {
namespace mech {

constexpr int BX = 64, BY = 4;

inline dim3 node_grid(const DevGrid &g) { return dim3((g.nx + 1 + BX - 1) / BX, (g.ny + 1 + BY - 1) / BY, g.nz + 1); }

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block sums of NS values into out[0..NS) (any block size that is a multiple of 64, <= 1024).
template <int NS>
__device__ __forceinline__ void block_sums(const double (&v)[NS], double *out) {
  __shared__ double red[16][NS];
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  const int lane = tid & 63, wv = tid >> 6;
  double r[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) r[q] = wsum(v[q]);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NS; ++q) red[wv][q] = r[q];
  __syncthreads();
  if (tid == 0) {
    const int nw = (blockDim.x * blockDim.y) / 64;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      double acc = red[0][q];
      for (int w = 1; w < nw; ++w) acc += red[w][q];
      out[q] = acc;
    }
  }
}

// Fixed-order sum of partials[nb][kRedWidth] columns 0..NS-1 by one block of 256.
template <int NS>
__device__ __forceinline__ void sum_partials(const double *part, int64_t nb, double *out) {
  double v[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) v[q] = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += blockDim.x)
#pragma unroll
    for (int q = 0; q < NS; ++q) v[q] += part[b * kRedWidth + q];
  block_sums<NS>(v, out);
}

// ---- cell-based HEX8 apply ---------------------------------------------------
// For a box cell the element stiffness is a sum of Kronecker products of 1D
// 2x2 factors: mass m(a,b) = int phi_a phi_b, stiffness k = int phi_a' phi_b',
// and the mixed g = int phi_a' phi_b, g^T.  In the per-axis basis
// (sum, difference) = (v0 + v1, v1 - v0) each factor is diagonal or a swap:
//   m: diag(h/2, h/6)   k: diag(0, 2/h)   g: sum -> difference   g^T: difference -> sum
// so K_e u = H^-1 D H u with H the tensor sum/difference transform, and D
// has 24 diagonal entries and 24 single-entry couplings between components.

// Forward transform of 8 corner values (index ax + 2 ay + 4 az) in place.
template <typename T>
__device__ __forceinline__ void haar3(T v[8]) {
#pragma unroll
  for (int a = 0; a < 8; a += 2) { const T s = v[a] + v[a + 1], d = v[a + 1] - v[a]; v[a] = s; v[a + 1] = d; }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int a = (q & 1) | ((q & 2) << 1);
    const T s = v[a] + v[a + 2], d = v[a + 2] - v[a]; v[a] = s; v[a + 2] = d;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) { const T s = v[a] + v[a + 4], d = v[a + 4] - v[a]; v[a] = s; v[a + 4] = d; }
}

// Inverse transform without its factor 1/8 (folded into the operator).
template <typename T>
__device__ __forceinline__ void ihaar3(T v[8]) {
#pragma unroll
  for (int a = 0; a < 4; ++a) { const T s = v[a], d = v[a + 4]; v[a] = s - d; v[a + 4] = s + d; }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int a = (q & 1) | ((q & 2) << 1);
    const T s = v[a], d = v[a + 2]; v[a] = s - d; v[a + 2] = s + d;
  }
#pragma unroll
  for (int a = 0; a < 8; a += 2) { const T s = v[a], d = v[a + 1]; v[a] = s - d; v[a + 1] = s + d; }
}

// (ux, uy, uz) <- K_e (ux, uy, uz) for a box cell of widths h and Lame
// constants lam, mu (corner index ax + 2 ay + 4 az).
template <typename T>
__device__ __forceinline__ void hex8_cell(T ux[8], T uy[8], T uz[8], T hx, T hy, T hz, T lam, T mu) {
  haar3(ux); haar3(uy); haar3(uz);
  const T mx[2] = {hx * T(0.5), hx * T(1.0 / 6.0)}, my[2] = {hy * T(0.5), hy * T(1.0 / 6.0)},
          mz[2] = {hz * T(0.5), hz * T(1.0 / 6.0)};
  const T kx = T(2) / hx, ky = T(2) / hy, kz = T(2) / hz;
  const T el = T(0.125) * lam, em = T(0.125) * mu;
  T vx[8], vy[8], vz[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const int px = p & 1, py = (p >> 1) & 1, pz = p >> 2;
    const T t1 = px ? kx * my[py] * mz[pz] : T(0);
    const T t2 = py ? mx[px] * ky * mz[pz] : T(0);
    const T t3 = pz ? mx[px] * my[py] * kz : T(0);
    const T s = t1 + t2 + t3;
    vx[p] = (el * t1 + em * (s + t1)) * ux[p];
    vy[p] = (el * t2 + em * (s + t2)) * uy[p];
    vz[p] = (el * t3 + em * (s + t3)) * uz[p];
  }
#pragma unroll
  for (int pz = 0; pz < 2; ++pz) {  // x-y coupling: (sum x, diff y) <-> (diff x, sum y)
    const int ai = 2 + 4 * pz, ao = 1 + 4 * pz;
    const T l = el * mz[pz], m = em * mz[pz];
    vx[ao] += l * uy[ai]; vx[ai] += m * uy[ao];
    vy[ai] += l * ux[ao]; vy[ao] += m * ux[ai];
  }
#pragma unroll
  for (int py = 0; py < 2; ++py) {  // x-z coupling
    const int ai = 2 * py + 4, ao = 1 + 2 * py;
    const T l = el * my[py], m = em * my[py];
    vx[ao] += l * uz[ai]; vx[ai] += m * uz[ao];
    vz[ai] += l * ux[ao]; vz[ao] += m * ux[ai];
  }
#pragma unroll
  for (int px = 0; px < 2; ++px) {  // y-z coupling
    const int ai = px + 4, ao = px + 2;
    const T l = el * mx[px], m = em * mx[px];
    vy[ao] += l * uz[ai]; vy[ai] += m * uz[ao];
    vz[ai] += l * uy[ao]; vz[ao] += m * uy[ai];
  }
  ihaar3(vx); ihaar3(vy); ihaar3(vz);
#pragma unroll
  for (int a = 0; a < 8; ++a) { ux[a] = vx[a]; uy[a] = vy[a]; uz[a] = vz[a]; }
}

// y = K x over the mesh, cell by cell, with an epilogue per node.
// A block of CX x CY threads owns a tile of CX x CY cells and the
// (CX-1) x (CY-1) nodes whose four in-plane cells all lie in the tile, and
// marches up z over kchunk node planes: for each cell layer it stages the
// next node plane of x in LDS (three-plane ring), every thread applies its
// cell's K_e and stores the 24 results in LDS, and each owned node adds the
// corners of its four cells in a fixed order, so y is deterministic.
// Fixed DOFs give zero rows; x is taken as zero on them.  The next x plane
// and the material id of the cell below it are fetched one layer ahead,
// right after the layer's first barrier; the
// Lame constants come from a per-block LDS copy of the material table (mu
// stored as -1 for a void material), so no global load sits between the
// barrier and the cell work.  The epilogue's own inputs (Epi::load) and the
// node's fixed-DOF bits are issued before the cell work.  The epilogue sees
// (n, y, x at the node, its prefetched inputs, per-thread partial sums).
constexpr int CX = 32, CY = 8;
constexpr int kMatMaxMech = 256;  // material ids are 8-bit

inline dim3 cell_grid(const DevGrid &g, int kchunk) {
  return dim3((g.nx + 1 + CX - 2) / (CX - 1), (g.ny + 1 + CY - 2) / (CY - 1), (g.nz + 1 + kchunk - 1) / kchunk);
}
inline int cell_kchunk(const DevGrid &g) {
  const int64_t tiles = int64_t((g.nx + 1 + CX - 2) / (CX - 1)) * ((g.ny + 1 + CY - 2) / (CY - 1));
  const int64_t want = std::max<int64_t>(1, (tiles * (g.nz + 1)) / 4096);
  return int(std::max<int64_t>(4, std::min<int64_t>(32, want)));
}

template <typename T, int NS, class Epi>
__global__ __launch_bounds__(CX * CY) void hex8_cell_kernel(MechGrid M, const T *x0, const T *x1, const T *x2,
                                                             int kchunk, Epi epi, double *partials,
                                                             const DevScalars *sc) {
  if (sc && sc->done) return;
  const DevGrid &g = M.g;
  constexpr int PL = (CY + 1) * (CX + 1);          // nodes per staged plane
  constexpr int PT = (PL + CX * CY - 1) / (CX * CY);  // plane entries per thread
  __shared__ T xs[3][3][CY + 1][CX + 1];
  __shared__ T co[24][CY][CX];
  __shared__ T lm_tab[2][kMatMaxMech];
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * CX + tx;
  for (int m = tid; m < g.n_mat; m += CX * CY) {
    const double *row = g.mtab + m * kMatStride;
    lm_tab[0][m] = T(row[MC_LAMBDA]);
    lm_tab[1][m] = row[MC_VOID] == 0.0 ? T(row[MC_MU]) : T(-1);
  }
  // logical tile of this block: XCD-contiguous, x fastest, so tiles that
  // share cache lines at their x and y borders share an L2
  const int nbx = int(gridDim.x), nby = int(gridDim.y);
  const int lb = xcd_remap((int(blockIdx.z) * nby + int(blockIdx.y)) * nbx + int(blockIdx.x), nbx * nby * int(gridDim.z));
  const int bx = lb % nbx, by = (lb / nbx) % nby, bz = lb / (nbx * nby);
  const int i0 = bx * (CX - 1), j0 = by * (CY - 1);
  const int k0 = bz * kchunk, k1 = min(k0 + kchunk, g.nz + 1);
  const int ci = i0 - 1 + tx, cj = j0 - 1 + ty;
  const bool cin = ci >= 0 && ci < g.nx && cj >= 0 && cj < g.ny;
  const int ni = i0 + tx, nj = j0 + ty;
  const bool own = tx < CX - 1 && ty < CY - 1 && ni <= g.nx && nj <= g.ny;
  const T hx = cin ? T(g.dx[ci]) : T(1), hy = cin ? T(g.dy[cj]) : T(1);
  const T *xv[3] = {x0, x1, x2};
  double red[NS > 0 ? NS : 1];
#pragma unroll
  for (int q = 0; q < (NS > 0 ? NS : 1); ++q) red[q] = 0.0;
  // plane k of x into registers (this thread's share), then into LDS
  T pf[PT][3];
  int pm = -1, mid = -1;  // material id of cell (ci, cj, k - 1): fetched with plane k
  auto fetch = [&](int k) {
    const bool cl = cin && k >= 1 && k <= g.nz;
    pm = cl ? int(g.mat[int64_t(k - 1) * g.sz + int64_t(cj) * g.sy + ci]) : -1;
#pragma unroll
    for (int e = 0; e < PT; ++e) {
      const int t = tid + e * CX * CY;
      const int r = t / (CX + 1), c = t - r * (CX + 1);
      const int i = i0 - 1 + c, j = j0 - 1 + r;
      const bool ok = t < PL && k >= 0 && k <= g.nz && i >= 0 && i <= g.nx && j >= 0 && j <= g.ny;
      const int64_t n = ok ? int64_t(k) * g.sz + int64_t(j) * g.sy + i : 0;
#pragma unroll
      for (int q = 0; q < 3; ++q) pf[e][q] = ok ? xv[q][n] : T(0);
    }
  };
  auto stage = [&](int k) {
    mid = pm;
    T(*dst)[CY + 1][CX + 1] = xs[(k + 3) % 3];
#pragma unroll
    for (int e = 0; e < PT; ++e) {
      const int t = tid + e * CX * CY;
      if (t < PL) {
        const int r = t / (CX + 1), c = t - r * (CX + 1);
#pragma unroll
        for (int q = 0; q < 3; ++q) dst[q][r][c] = pf[e][q];
      }
    }
  };
  T acc[3] = {T(0), T(0), T(0)};
  fetch(k0 - 1);
  stage(k0 - 1);
  fetch(k0);
  for (int ck = k0 - 1; ck < k1; ++ck) {
    stage(ck + 1);        // plane ck + 1 (fetched during the previous layer)
    const int m = mid;    // cell layer ck (staged with plane ck + 1)
    const T hz = m >= 0 ? T(g.dz[ck]) : T(1);
    __syncthreads();
    // issued after the barrier (which waits for every load in flight), so
    // they are in flight while this layer computes
    if (ck + 2 <= k1) fetch(ck + 2);
    const int64_t n = int64_t(ck) * g.sz + int64_t(nj) * g.sy + ni;
    const bool emit = own && ck >= k0;
    typename Epi::Pre pre;
    uint8_t fix = 0;
    if (emit) {
      pre = epi.load(n);
      fix = M.fixed[n];
    }
    T ux[8], uy[8], uz[8];
    T lam = T(0), mu = T(-1);
    if (m >= 0) {
      lam = lm_tab[0][m];
      mu = lm_tab[1][m];
    }
    const bool live = mu >= T(0);
    if (live) {
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
        const T(*pl)[CY + 1][CX + 1] = xs[(ck + az + 3) % 3];
        ux[a] = pl[0][ty + ay][tx + ax];
        uy[a] = pl[1][ty + ay][tx + ax];
        uz[a] = pl[2][ty + ay][tx + ax];
      }
      hex8_cell<T>(ux, uy, uz, hx, hy, hz, lam, mu);
    } else {
#pragma unroll
      for (int a = 0; a < 8; ++a) ux[a] = uy[a] = uz[a] = T(0);
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      co[a * 3 + 0][ty][tx] = ux[a];
      co[a * 3 + 1][ty][tx] = uy[a];
      co[a * 3 + 2][ty][tx] = uz[a];
    }
    __syncthreads();
    if (own) {
      // node (ni, nj) is corner (1,1) of cell (tx,ty), (0,1) of (tx+1,ty),
      // (1,0) of (tx,ty+1) and (0,0) of (tx+1,ty+1)
      T y[3], top[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        y[q] = acc[q] + co[3 * 3 + q][ty][tx] + co[2 * 3 + q][ty][tx + 1] + co[1 * 3 + q][ty + 1][tx] +
               co[0 * 3 + q][ty + 1][tx + 1];
        top[q] = co[7 * 3 + q][ty][tx] + co[6 * 3 + q][ty][tx + 1] + co[5 * 3 + q][ty + 1][tx] +
                 co[4 * 3 + q][ty + 1][tx + 1];
      }
      if (emit) {
        if (fix & 1) y[0] = T(0);
        if (fix & 2) y[1] = T(0);
        if (fix & 4) y[2] = T(0);
        const T(*pl)[CY + 1][CX + 1] = xs[(ck + 3) % 3];
        const T xc[3] = {pl[0][ty + 1][tx + 1], pl[1][ty + 1][tx + 1], pl[2][ty + 1][tx + 1]};
        epi(n, y, xc, pre, red);
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) acc[q] = top[q];
    }
  }
  if constexpr (NS > 0) {
    const int64_t b = (int64_t(blockIdx.z) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    block_sums<NS>(red, partials + b * kRedWidth);
  }
}

inline int64_t cell_blocks(const DevGrid &g, int kchunk) {
  const dim3 d = cell_grid(g, kchunk);
  return int64_t(d.x) * d.y * d.z;
}

template <typename T, int NS, class Epi>
inline hipError_t launch_hex8(const MechGrid &M, const T *const x[3], Epi epi, double *partials, const DevScalars *sc,
                              hipStream_t s) {
  const int kc = cell_kchunk(M.g);
  hipLaunchKernelGGL((hex8_cell_kernel<T, NS, Epi>), cell_grid(M.g, kc), dim3(CX, CY), 0, s, M, x[0], x[1], x[2], kc,
                     epi, partials, sc);
  return hipGetLastError();
}

}  // namespace mech
}  // namespace etm
