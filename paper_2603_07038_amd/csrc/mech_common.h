// Device helpers shared by the mechanics kernels (mech.hip) and the
// multigrid preconditioner (mg.hip): node-grid launch shape, wave64 and block
// reductions in FP64, and the matrix-free HEX8 stiffness of Eq. (8).
#pragma once
#include <hip/hip_runtime.h>

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

// K_e rows of local node a applied to the cell's nodal vectors, accumulated
// into y.  pv[3] point at the node-shaped input arrays; nb0 is the index of
// the cell's low corner node.
template <typename T>
__device__ __forceinline__ void cell_rows(const DevGrid &g, int ci, int cj, int ck, int ax, int ay, int az,
                                          int64_t nb0, const T *const *pv, T &yx, T &yy, T &yz) {
  const double *row = g.mtab + g.mat[nb0] * kMatStride;
  if (row[MC_VOID] != 0.0) return;
  const T lam = T(row[MC_LAMBDA]), mu = T(row[MC_MU]);
  const T hx = T(g.dx[ci]), hy = T(g.dy[cj]), hz = T(g.dz[ck]);
  const T ihx = T(g.idx[ci]), ihy = T(g.idy[cj]), ihz = T(g.idz[ck]);
  const T gax = ax ? T(0.5) : T(-0.5), gay = ay ? T(0.5) : T(-0.5), gaz = az ? T(0.5) : T(-0.5);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
    const int64_t nb = nb0 + bx + by * g.sy + bz * g.sz;
    const T px = pv[0][nb], py = pv[1][nb], pz = pv[2][nb];
    const bool sx = ax == bx, sy = ay == by, sz = az == bz;
    const T mx = hx * (sx ? T(1.0 / 3.0) : T(1.0 / 6.0)), my = hy * (sy ? T(1.0 / 3.0) : T(1.0 / 6.0)),
            mz = hz * (sz ? T(1.0 / 3.0) : T(1.0 / 6.0));
    const T kx = sx ? ihx : -ihx, ky = sy ? ihy : -ihy, kz = sz ? ihz : -ihz;
    const T gbx = bx ? T(0.5) : T(-0.5), gby = by ? T(0.5) : T(-0.5), gbz = bz ? T(0.5) : T(-0.5);
    const T Axx = kx * my * mz, Ayy = mx * ky * mz, Azz = mx * my * kz;
    const T Lp = mu * (Axx + Ayy + Azz);
    const T Axy = gax * gby * mz, Ayx = gay * gbx * mz;
    const T Axz = gax * my * gbz, Azx = gaz * my * gbx;
    const T Ayz = mx * gay * gbz, Azy = mx * gaz * gby;
    yx += ((lam + mu) * Axx + Lp) * px + (lam * Axy + mu * Ayx) * py + (lam * Axz + mu * Azx) * pz;
    yy += (lam * Ayx + mu * Axy) * px + ((lam + mu) * Ayy + Lp) * py + (lam * Ayz + mu * Azy) * pz;
    yz += (lam * Azx + mu * Axz) * px + (lam * Azy + mu * Ayz) * py + ((lam + mu) * Azz + Lp) * pz;
  }
}

// y = K p at node (i,j,k) = index n (free rows only).
template <typename T>
__device__ __forceinline__ void node_apply(const MechGrid &M, int i, int j, int k, int64_t n, const T *const *pv,
                                           T &yx, T &yy, T &yz) {
  const DevGrid &g = M.g;
  yx = yy = yz = T(0);
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int ox = c & 1, oy = (c >> 1) & 1, oz = c >> 2;
    const int ci = i - 1 + ox, cj = j - 1 + oy, ck = k - 1 + oz;
    if (ci < 0 || ci >= g.nx || cj < 0 || cj >= g.ny || ck < 0 || ck >= g.nz) continue;
    const int64_t nb0 = n + (ox - 1) + (oy - 1) * g.sy + (oz - 1) * g.sz;
    cell_rows<T>(g, ci, cj, ck, 1 - ox, 1 - oy, 1 - oz, nb0, pv, yx, yy, yz);
  }
  const uint8_t f = M.fixed[n];
  if (f & 1) yx = T(0);
  if (f & 2) yy = T(0);
  if (f & 4) yz = T(0);
}

}  // namespace mech
}  // namespace etm
