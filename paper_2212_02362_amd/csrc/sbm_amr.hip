// sbm_amr.hip -- block-structured adaptive composite solve (BSAMR) on one GPU:
// refinement tags and block flags, node classes, coarse-fine ghost fill, the
// composite residual and the composite multilevel cycle, plus the sbm_amr_*
// C ABI.
//
// The paper (Sec. 2.2) runs the same operator on block-structured AMR levels
// that exchange data by averaging fine to coarse and by ghost cells coarse to
// fine, treats the refined levels as the upper part of the multigrid level
// sequence, and pads every level with one extra ghost layer so that the
// restriction stencil stays translation invariant and no special coarse-fine
// stencil is needed.  Reading used here (the details of the cited AMR
// framework are not in the paper):
//   * AMR level a has spacing h0 / 2^a and is stored densely over the box;
//     levels a >= 1 are active on cubic blocks of `block` cells.  Level-a
//     cells are tagged where |grad psi| h > threshold (central differences
//     clamped at the box, h the largest spacing; Sec. 3.3 uses 0.05).  A
//     level-(a+1) block is active when a tagged level-a cell lies in its
//     footprint grown by one cell; nesting activates the parent block and the
//     parent's neighbours on the sides the block touches.
//   * Node classes of a level a >= 1: 1 interior (unknown), 2 interface
//     (owned by level a-1), 3 and 4 the first and second node layers outside
//     the active region.  Classes 2-4 are ghosts, filled from level a-1 by
//     tensor-product quadratic interpolation.
//   * Covered coarse cells take the mean psi of their children; covered
//     coarse nodes take the injected fine values.
//   * Composite residual: padded fine residual on classes 1-3; coarse nodes
//     on or inside the finer region (fine class 1 or 2) take R of it; other
//     nodes keep their level residual.  Norm over the composite unknowns.
//   * Composite cycle: full-approximation multilevel cycle over the AMR levels
//     (smooth, restrict the padded residual, coarse load R w + K_c x_c on
//     covered and interface nodes, recurse, correct with P(x_c - inject x_f),
//     smooth) ending in one V-cycle of the base grid's uniform hierarchy; it
//     is applied in correction form inside an FP64 outer loop (mixed
//     precision: the cycle runs in FP32 on the residual scaled to unit norm).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/sbm.h"
#include "sbm_internal.h"

using namespace sbm;

namespace {

constexpr int kMaxAmrLevels = 4;  // base + up to 3 refined levels
// device ints of the set-up: [0] error flags, [12 + a] ghost nodes, [16 + a]
// tiles with unknowns, [20 + a] ghost nodes outside them, [24 + a] coarse
// nodes under the region, of level a
constexpr int kIflags = 28;
// Tile lists of sparsely refined levels: shallowest chunk depth, and the
// number of workgroups the listed tiles should give (a few per CU).
constexpr int kAmrKzMin = 6;
constexpr int64_t kAmrTiles = 2048;

#define AMR_LAUNCH(kern, grid, block, st, ...)                             \
  do {                                                                     \
    (void)hipGetLastError();                                               \
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, st, __VA_ARGS__); \
    return hipGetLastError();                                              \
  } while (0)

__device__ __forceinline__ int64_t fine_of_coarse(const Geom &gf, int I, int J, int K) {
  return 2 * I + (int64_t)gf.nx * (2 * J + (int64_t)gf.ny * (2 * K));
}

// Node iteration of the level kernels: one node per thread over the whole
// level, or (TILED) one workgroup per listed tile, looping over its nodes.
struct TileArg {
  TileGeom tg;
  const int *ids;
};

template <bool TILED, class F>
__device__ __forceinline__ void for_nodes(const Geom &g, const TileArg &ta, F &&fn) {
  if constexpr (!TILED) {
    const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (id < g.nn) fn(id);
  } else {
    // one workgroup per plane of a listed tile
    const int t = ta.ids[blockIdx.x / ta.tg.kz];
    const int tx = t % ta.tg.ntx, rest = t / ta.tg.ntx;
    const int ty = rest % ta.tg.nty, tz = rest / ta.tg.nty;
    const int x0 = tx * kTileX, y0 = ty * kTileY;
    const int k = tz * ta.tg.kz + (int)(blockIdx.x % ta.tg.kz);
    if (k >= g.nz) return;
    for (int e = threadIdx.x; e < kTileX * kTileY; e += kBlock) {
      const int x = x0 + e % kTileX, y = y0 + e / kTileX;
      if (x < g.nx && y < g.ny) fn((int64_t)x + (int64_t)g.nx * (y + (int64_t)g.ny * k));
    }
  }
}

// ------------------------------------------------------------- setup kernels

// Refinement tags of the cells of one level: |grad psi|^2 h^2 > threshold^2
// with central differences (neighbours clamped at the box).  Evaluated without
// contraction so that the integer decision does not depend on FMA formation.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_amr_tags(Geom g, double hx, double hy, double hz,
                                                     double hmax2, double thr2,
                                                     const double *__restrict__ psi,
                                                     uint8_t *__restrict__ tags) {
#pragma clang fp contract(off)
  const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (id >= g.nc) return;
  int i, j, k;
  cell_ijk(g, id, i, j, k);
  const int c[3] = {i, j, k};
  const int n[3] = {g.cx, g.cy, g.cz};
  const double h[3] = {hx, hy, hz};
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    int p[3] = {c[0], c[1], c[2]}, m[3] = {c[0], c[1], c[2]};
    p[a] = c[a] + 1 < n[a] ? c[a] + 1 : c[a];
    m[a] = c[a] > 0 ? c[a] - 1 : c[a];
    const double d = psi[p[0] + (int64_t)g.cx * (p[1] + (int64_t)g.cy * p[2])] -
                     psi[m[0] + (int64_t)g.cx * (m[1] + (int64_t)g.cy * m[2])];
    const double gr = d / (2.0 * h[a]);
    s = s + gr * gr;
  }
  tags[id] = (s * hmax2 > thr2) ? 1 : 0;
}

// Block flags of level a from the tags of level a-1: one workgroup per block,
// OR over the block's coarse footprint grown by one cell.
__global__ __launch_bounds__(kBlock) void k_amr_blocks(Geom gc, int dim, int nbx, int nby,
                                                       int half, const uint8_t *__restrict__ tags,
                                                       uint8_t *__restrict__ blk) {
  const int b = blockIdx.x;
  const int bi[3] = {b % nbx, (b / nbx) % nby, b / (nbx * nby)};
  const int n[3] = {gc.cx, gc.cy, gc.cz};
  int lo[3], len[3];
  for (int a = 0; a < 3; ++a) {
    if (a < dim) {
      const int l = max(bi[a] * half - 1, 0);
      const int h = min(bi[a] * half + half, n[a] - 1);
      lo[a] = l;
      len[a] = h - l + 1;
    } else {
      lo[a] = 0;
      len[a] = 1;
    }
  }
  const int count = len[0] * len[1] * len[2];
  int any = 0;
  for (int t = threadIdx.x; t < count; t += blockDim.x) {
    const int x = lo[0] + t % len[0];
    const int y = lo[1] + (t / len[0]) % len[1];
    const int z = lo[2] + t / (len[0] * len[1]);
    if (tags[x + (int64_t)gc.cx * (y + (int64_t)gc.cy * z)]) any = 1;
  }
  any = __syncthreads_or(any);
  if (threadIdx.x == 0) blk[b] = (uint8_t)(any ? 1 : 0);
}

// Nesting: every active block of level a activates its parent block and the
// parent's neighbours on the sides the block touches (flags of level a-1).
__global__ __launch_bounds__(kBlock) void k_amr_nest(int dim, int nbx, int nby, int nbz,
                                                     const uint8_t *__restrict__ blk, int pnx,
                                                     int pny, int pnz, uint8_t *pblk) {
  const int b = blockIdx.x * kBlock + threadIdx.x;
  if (b >= nbx * nby * nbz || !blk[b]) return;
  const int bi[3] = {b % nbx, (b / nbx) % nby, b / (nbx * nby)};
  const int pn[3] = {pnx, pny, pnz};
  int pb[3], sg[3];
  for (int a = 0; a < 3; ++a) {
    pb[a] = bi[a] / 2;
    sg[a] = a < dim ? ((bi[a] % 2) ? 1 : -1) : 0;
  }
  for (int o = 0; o < 8; ++o) {
    int q[3];
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
      const int bit = (o >> a) & 1;
      if (a >= dim && bit) ok = false;
      q[a] = pb[a] + (bit ? sg[a] : 0);
      if (a < dim && (q[a] < 0 || q[a] >= pn[a])) ok = false;
    }
    if (ok) pblk[q[0] + pnx * (q[1] + pny * q[2])] = 1;
  }
}

// Node classes, pass 1: closure of the active region (clo) and classes 1/2.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_amr_classify(Geom g, int bc, int nbx, int nby,
                                                         const uint8_t *__restrict__ blk,
                                                         uint8_t *__restrict__ clo,
                                                         uint8_t *__restrict__ cls) {
  const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (id >= g.nn) return;
  int i, j, k;
  node_ijk(g, id, i, j, k);
  bool any = false, all = true;
#pragma unroll
  for (int o = 0; o < (1 << DIM); ++o) {
    const int x = i - 1 + (o & 1), y = j - 1 + ((o >> 1) & 1);
    const int z = DIM == 3 ? k - 1 + ((o >> 2) & 1) : 0;
    if (x < 0 || x >= g.cx || y < 0 || y >= g.cy || z < 0 || z >= g.cz) continue;
    const bool act = blk[x / bc + nbx * (y / bc + nby * (z / bc))] != 0;
    any = any || act;
    all = all && act;
  }
  clo[id] = any ? 1 : 0;
  cls[id] = any ? (all ? 1 : 2) : 0;
}

// Node classes, pass 2: the first (3) and second (4) node layers around the
// closure (Chebyshev distance 1 and 2).
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_amr_layers(Geom g, const uint8_t *__restrict__ clo,
                                                       uint8_t *__restrict__ cls) {
  const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (id >= g.nn || cls[id] != 0) return;
  int i, j, k;
  node_ijk(g, id, i, j, k);
  int best = 3;
  const int zr = DIM == 3 ? 2 : 0;
  for (int dz = -zr; dz <= zr; ++dz)
    for (int dy = -2; dy <= 2; ++dy)
      for (int dx = -2; dx <= 2; ++dx) {
        const int x = i + dx, y = j + dy, z = k + dz;
        if (x < 0 || x >= g.nx || y < 0 || y >= g.ny || z < 0 || z >= g.nz) continue;
        if (!clo[x + (int64_t)g.nx * (y + (int64_t)g.ny * z)]) continue;
        const int d = max(max(abs(dx), abs(dy)), abs(dz));
        best = min(best, d);
      }
  if (best <= 2) cls[id] = (uint8_t)(2 + best);
}

// psi of covered coarse cells: mean of the 2^d children (children summed in
// x-fastest order), FP64 and its FP32 copy.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_amr_avgdown(Geom gc, Geom gf, int bc, int nbx,
                                                        int nby, const uint8_t *__restrict__ blkf,
                                                        const double *__restrict__ psif,
                                                        double *__restrict__ psic,
                                                        float *__restrict__ psic32) {
  const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (id >= gc.nc) return;
  int I, J, K;
  cell_ijk(gc, id, I, J, K);
  const int x = 2 * I, y = 2 * J, z = DIM == 3 ? 2 * K : 0;
  if (!blkf[x / bc + nbx * (y / bc + nby * (z / bc))]) return;
  double s = 0.0;
#pragma unroll
  for (int o = 0; o < (1 << DIM); ++o) {
    const int qx = x + (o & 1), qy = y + ((o >> 1) & 1), qz = DIM == 3 ? z + ((o >> 2) & 1) : 0;
    s += psif[qx + (int64_t)gf.cx * (qy + (int64_t)gf.cy * qz)];
  }
  const double v = s / (double)(1 << DIM);
  psic[id] = v;
  psic32[id] = (float)v;
}

// ------------------------------------------------------------ cycle kernels

// Quadratic interpolation along one axis for fine node index n: even n takes
// coarse node n/2; odd n = 2I+1 takes {I-1, I, I+1} with (-1/8, 3/4, 3/8), or
// {0, 1, 2} with (3/8, 3/4, -1/8) when I = 0.
template <typename T>
__device__ __forceinline__ int quad_axis(int n, int idx[3], T w[3]) {
  if ((n & 1) == 0) {
    idx[0] = n >> 1;
    w[0] = T(1);
    return 1;
  }
  const int I = (n - 1) >> 1;
  if (I >= 1) {
    idx[0] = I - 1; idx[1] = I; idx[2] = I + 1;
    w[0] = T(-0.125); w[1] = T(0.75); w[2] = T(0.375);
  } else {
    idx[0] = I; idx[1] = I + 1; idx[2] = I + 2;
    w[0] = T(0.375); w[1] = T(0.75); w[2] = T(-0.125);
  }
  return 3;
}

// Ghost nodes (classes 2-4) of the fine level from the coarse level; fixed
// displacement DOF keep their values.  Weight products are exact dyadic
// numbers; every term is rounded before it is added.
template <typename T, int DIM>
__device__ __forceinline__ void ghost_node(const Geom &gf, const Geom &gc,
                                           const T *__restrict__ xc, T *__restrict__ xf,
                                           int64_t id) {
#pragma clang fp contract(off)
  int i, j, k;
  node_ijk(gf, id, i, j, k);
  int ix[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  T w[3][3] = {{T(1), T(0), T(0)}, {T(1), T(0), T(0)}, {T(1), T(0), T(0)}};
  int cnt[3] = {1, 1, 1};
  cnt[0] = quad_axis<T>(i, ix[0], w[0]);
  cnt[1] = quad_axis<T>(j, ix[1], w[1]);
  if (DIM == 3) cnt[2] = quad_axis<T>(k, ix[2], w[2]);
  // the loads of all taken coarse nodes are issued together, then summed in
  // x-fastest order
  constexpr int NZ = DIM == 3 ? 3 : 1;
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    if (is_dirichlet(gf, i, j, k, c)) continue;
    T v[NZ][3][3];
#pragma unroll
    for (int t2 = 0; t2 < NZ; ++t2)
#pragma unroll
      for (int t1 = 0; t1 < 3; ++t1)
#pragma unroll
        for (int t0 = 0; t0 < 3; ++t0) {
          const int64_t q = ix[0][t0] + (int64_t)gc.nx * (ix[1][t1] + (int64_t)gc.ny * ix[2][t2]);
          v[t2][t1][t0] =
              (t0 < cnt[0] && t1 < cnt[1] && t2 < cnt[2]) ? xc[c * gc.nn + q] : T(0);
        }
    T s = T(0);
#pragma unroll
    for (int t2 = 0; t2 < NZ; ++t2)
#pragma unroll
      for (int t1 = 0; t1 < 3; ++t1)
#pragma unroll
        for (int t0 = 0; t0 < 3; ++t0)
          if (t0 < cnt[0] && t1 < cnt[1] && t2 < cnt[2])
            s += w[0][t0] * w[1][t1] * w[2][t2] * v[t2][t1][t0];
    xf[c * gf.nn + id] = s;
  }
}

// The same over a list of the level's ghost nodes (one per thread).
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_amr_ghost_list(Geom gf, Geom gc,
                                                           const int *__restrict__ ids, int n,
                                                           const T *__restrict__ xc,
                                                           T *__restrict__ xf) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  ghost_node<T, DIM>(gf, gc, xc, xf, ids[t]);
}

// x = 0 at the nodes of a level (of its listed tiles when TILED).
template <typename T, bool TILED>
__global__ __launch_bounds__(kBlock) void k_amr_zero(Geom g, T *__restrict__ x, TileArg ta) {
  for_nodes<TILED>(g, ta, [&](int64_t id) {
    for (int c = 0; c < g.dim; ++c) x[c * g.nn + id] = T(0);
  });
}

// dst = src (0 when src is null) on the listed nodes (all components).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_amr_ghost_copy(int64_t nn, int dim,
                                                           const int *__restrict__ ids, int n,
                                                           const T *__restrict__ src,
                                                           T *__restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  const int64_t id = ids[t];
  for (int c = 0; c < dim; ++c) dst[c * nn + id] = src ? src[c * nn + id] : T(0);
}

// r = f - K u at the listed nodes of a level with classes (a padded residual
// as k_residual with a class mask: classes 1-3 carry one, the others get 0).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_residual_list(Geom g, Coef<T> C,
                                                          const T *__restrict__ psi,
                                                          const T *__restrict__ u,
                                                          const T *__restrict__ f,
                                                          T *__restrict__ r,
                                                          const uint8_t *__restrict__ cls,
                                                          const int *__restrict__ ids, int n) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  const int64_t id = ids[t];
  if (cls[id] == 0 || cls[id] > 3) {
    for (int c = 0; c < 3; ++c) r[c * g.nn + id] = T(0);
    return;
  }
  int i, j, k;
  node_ijk(g, id, i, j, k);
  T fv[3], out[3], dg[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) fv[c] = f[c * g.nn + id];
  node_stencil<T, 3>(g, C, psi, u, i, j, k, out, dg);
  const uint32_t fb = face_bits(g, i, j, k);
#pragma unroll
  for (int c = 0; c < 3; ++c) r[c * g.nn + id] = ((g.dmask >> c) & fb) ? T(0) : fv[c] - out[c];
}

// Node lists of a level (ids of the nodes a predicate selects, increasing),
// by a three-pass compaction: per-block counts, one-workgroup scan of the
// counts, per-block writes in node order.  Ghost nodes: class >= 2.  Ghost
// nodes in no flagged tile of a fixed-depth tile geometry (tflags: the flags
// of a tile list).  Coarse nodes the composite restriction writes: fine class
// 1 or 2 at the coinciding fine node.
constexpr int kCompactNodes = 4 * kBlock;  // nodes per block (four per thread)

struct GhostPick {
  const uint8_t *cls;
  __device__ bool operator()(int64_t id) const { return cls[id] >= 2; }
};
struct OutsidePick {
  Geom g;
  TileGeom tg;
  const int *tflags;
  const uint8_t *cls;
  __device__ bool operator()(int64_t id) const {
    if (cls[id] < 2) return false;
    int i, j, k;
    node_ijk(g, id, i, j, k);
    return !tflags[i / kTileX + tg.ntx * (j / kTileY + tg.nty * (k / tg.kz))];
  }
};
struct CifPick {
  Geom gf, gc;
  const uint8_t *clsf;
  __device__ bool operator()(int64_t id) const {
    int I, J, K;
    node_ijk(gc, id, I, J, K);
    const uint8_t fc = clsf[fine_of_coarse(gf, I, J, K)];
    return fc == 1 || fc == 2;
  }
};

template <class P>
__global__ __launch_bounds__(kBlock) void k_list_count(int64_t nn, P pick,
                                                       int *__restrict__ bcnt) {
  __shared__ int red[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kCompactNodes + 4 * threadIdx.x;
  int c = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) c += (base + e < nn && pick(base + e)) ? 1 : 0;
  red[threadIdx.x] = c;
  __syncthreads();
  for (int d = kBlock / 2; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) bcnt[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(1024) void k_scan_counts(const int *__restrict__ cnt, int n,
                                                      int *__restrict__ off, int *__restrict__ total) {
  __shared__ int sh[1024];
  const int t = threadIdx.x;
  const int chunk = (n + 1023) / 1024;
  const int lo = min(n, t * chunk), hi = min(n, lo + chunk);
  int c = 0;
  for (int i = lo; i < hi; ++i) c += cnt[i];
  sh[t] = c;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {  // inclusive scan
    const int v = t >= d ? sh[t - d] : 0;
    __syncthreads();
    sh[t] += v;
    __syncthreads();
  }
  int w = sh[t] - c;
  for (int i = lo; i < hi; ++i) {
    off[i] = w;
    w += cnt[i];
  }
  if (t == 1023) *total = sh[1023];
}

template <class P>
__global__ __launch_bounds__(kBlock) void k_list_write(int64_t nn, P pick,
                                                       const int *__restrict__ boff,
                                                       int *__restrict__ ids) {
  __shared__ int sh[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kCompactNodes + 4 * threadIdx.x;
  bool g[4];
  int c = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    g[e] = base + e < nn && pick(base + e);
    c += g[e] ? 1 : 0;
  }
  sh[threadIdx.x] = c;
  __syncthreads();
  for (int d = 1; d < kBlock; d <<= 1) {  // inclusive scan
    const int v = (int)threadIdx.x >= d ? sh[threadIdx.x - d] : 0;
    __syncthreads();
    sh[threadIdx.x] += v;
    __syncthreads();
  }
  int w = boff[blockIdx.x] + sh[threadIdx.x] - c;
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (g[e]) ids[w++] = (int)(base + e);
}

// Coarse nodes on or inside the fine region (fine class 1 or 2 at the
// coinciding node), free DOF: out = R r_f (+ add) (+ add2), R the
// full-weighting transpose of multilinear P over 2^d.  With ONLY_GHOSTS only
// fine nodes of class 2 and 3 contribute.  Other nodes are left untouched.
// One thread per listed coarse node (ids: those nodes, from CifPick).
template <typename T, int DIM, bool ONLY_GHOSTS>
__global__ __launch_bounds__(kBlock) void k_amr_restrict_cif(Geom gf, Geom gc,
                                                             const uint8_t *__restrict__ clsf,
                                                             const int *__restrict__ ids, int n,
                                                             const T *__restrict__ rf,
                                                             const T *__restrict__ add,
                                                             const T *__restrict__ add2,
                                                             T *__restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  const int64_t id = ids[t];
  int I, J, K;
  node_ijk(gc, id, I, J, K);
  T acc[3] = {T(0), T(0), T(0)};
  const int zlo = (DIM == 3) ? -1 : 0, zhi = (DIM == 3) ? 1 : 0;
  for (int dz = zlo; dz <= zhi; ++dz) {
    const int fk = 2 * K + dz;
    if (fk < 0 || fk >= gf.nz) continue;
    const T wz = dz == 0 ? T(1) : T(0.5);
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int fj = 2 * J + dy;
      if (fj < 0 || fj >= gf.ny) continue;
      const T wy = dy == 0 ? T(1) : T(0.5);
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int fi = 2 * I + dx;
        if (fi < 0 || fi >= gf.nx) continue;
        const T wgt = wz * wy * (dx == 0 ? T(1) : T(0.5));
        const int64_t q = fi + (int64_t)gf.nx * (fj + (int64_t)gf.ny * fk);
        if (ONLY_GHOSTS && clsf[q] != 2 && clsf[q] != 3) continue;
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc[c] += wgt * rf[c * gf.nn + q];
      }
    }
  }
  const T scale = (DIM == 3) ? T(0.125) : T(0.25);
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    if (is_dirichlet(gc, I, J, K, c)) continue;
    T v = acc[c] * scale;
    if (add) v = v + add[c * gc.nn + id];
    if (add2) v = v + add2[c * gc.nn + id];
    out[c * gc.nn + id] = v;
  }
}

// r32 = r / sqrt(*ss) in FP32, 0 on the padded ghost rows (classes 2 and 3)
// of an adaptive level (every node when cls is NULL).
template <int DIM, bool TILED>
__global__ __launch_bounds__(kBlock) void k_amr_cast(Geom g, const uint8_t *__restrict__ cls,
                                                     const double *__restrict__ r,
                                                     float *__restrict__ r32,
                                                     const double *__restrict__ ss, TileArg ta) {
  const double sn = sqrt(*ss);
  for_nodes<TILED>(g, ta, [&](int64_t id) {
    const bool ghost = cls && (cls[id] == 2 || cls[id] == 3);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const int64_t q = c * g.nn + id;
      r32[q] = (ghost || !(sn > 0.0)) ? 0.0f : (float)(r[q] / sn);
    }
  });
}

// Coarse nodes strictly inside the fine region (fine class 1) take the fine
// values at the coinciding node.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_amr_inject(Geom gf, Geom gc,
                                                       const uint8_t *__restrict__ clsf,
                                                       const T *__restrict__ xf,
                                                       T *__restrict__ xc) {
  const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (id >= gc.nn) return;
  int I, J, K;
  node_ijk(gc, id, I, J, K);
  const int64_t fid = fine_of_coarse(gf, I, J, K);
  if (clsf[fid] != 1) return;
#pragma unroll
  for (int c = 0; c < DIM; ++c) xc[c * gc.nn + id] = xf[c * gf.nn + fid];
}

// x_f += P (x_c - xinj_c) on the unknowns (class 1, free DOF) of the fine level.
template <typename T, int DIM, bool TILED>
__global__ __launch_bounds__(kBlock) void k_amr_correct(Geom gf, Geom gc,
                                                        const uint8_t *__restrict__ clsf,
                                                        const T *__restrict__ xc,
                                                        const T *__restrict__ xinj,
                                                        T *__restrict__ xf, TileArg ta) {
  for_nodes<TILED>(gf, ta, [&](int64_t id) {
    if (clsf[id] != 1) return;
    int i, j, k;
    node_ijk(gf, id, i, j, k);
    const int lo[3] = {i >> 1, j >> 1, DIM == 3 ? k >> 1 : 0};
    const int hi[3] = {(i + 1) >> 1, (j + 1) >> 1, DIM == 3 ? (k + 1) >> 1 : 0};
    const T wx = lo[0] == hi[0] ? T(1) : T(0.5), wy = lo[1] == hi[1] ? T(1) : T(0.5);
    const T wz = lo[2] == hi[2] ? T(1) : T(0.5);
    // the 2^DIM corners (lo or hi on each axis, x fastest), their loads
    // issued together; a corner repeating lo on an axis where hi == lo is
    // neither loaded (FP64) nor summed, so the sum takes the distinct coarse
    // nodes in x-fastest order
    constexpr int NB = DIM == 3 ? 8 : 4;
    int64_t qb[NB];
    bool use[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int b0 = b & 1, b1 = (b >> 1) & 1, b2 = b >> 2;
      qb[b] = (b0 ? hi[0] : lo[0]) + (int64_t)gc.nx * ((b1 ? hi[1] : lo[1]) +
                                                       (int64_t)gc.ny * (b2 ? hi[2] : lo[2]));
      use[b] = (!b0 || hi[0] != lo[0]) && (!b1 || hi[1] != lo[1]) && (!b2 || hi[2] != lo[2]);
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      if (is_dirichlet(gf, i, j, k, c)) continue;
      T d[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b)
        d[b] = (sizeof(T) == 4 || use[b]) ? xc[c * gc.nn + qb[b]] - xinj[c * gc.nn + qb[b]] : T(0);
      T acc = T(0);
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (use[b]) acc += wx * wy * wz * d[b];
      xf[c * gf.nn + id] += acc;
    }
  });
}

// u += s e on the free DOF of the level's unknowns (all nodes when cls is
// NULL, class 1 otherwise); s = sqrt(*ss) when ss is given, else 1.
template <typename T, int DIM, bool TILED>
__global__ __launch_bounds__(kBlock) void k_amr_update(Geom g, const uint8_t *__restrict__ cls,
                                                       double *__restrict__ u,
                                                       const T *__restrict__ e,
                                                       const double *__restrict__ ss, TileArg ta) {
  const double s = ss ? sqrt(*ss) : 1.0;
  for_nodes<TILED>(g, ta, [&](int64_t id) {
    if (cls && cls[id] != 1) return;
    int i, j, k;
    node_ijk(g, id, i, j, k);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      if (is_dirichlet(g, i, j, k, c)) continue;
      if (ss) u[c * g.nn + id] += s * (double)e[c * g.nn + id];
      else u[c * g.nn + id] += (double)e[c * g.nn + id];
    }
  });
}

// Per-block partial sums over the composite unknowns of one level: free DOF
// of class-1 nodes (every node when cls is NULL) not covered by the finer
// level (fine class 1 at the coinciding node; no finer level when clsf is
// NULL).  Sums r^2, or counts the DOF when r is NULL.
template <int DIM, bool TILED>
__global__ __launch_bounds__(kBlock) void k_amr_sumsq(Geom g, const uint8_t *__restrict__ cls,
                                                      Geom gf, const uint8_t *__restrict__ clsf,
                                                      const double *__restrict__ r,
                                                      double *__restrict__ partials, TileArg ta) {
  __shared__ double lds[kBlock / 64 + 1];
  double v = 0.0;
  for_nodes<TILED>(g, ta, [&](int64_t id) {
    if (cls && cls[id] != 1) return;
    int i, j, k;
    node_ijk(g, id, i, j, k);
    if (clsf && clsf[fine_of_coarse(gf, i, j, k)] == 1) return;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      if (is_dirichlet(g, i, j, k, c)) continue;
      if (r) {
        const double x = r[c * g.nn + id];
        v += x * x;
      } else {
        v += 1.0;
      }
    }
  });
  const double s = block_sum(v, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// ---------------------------------------------------------------- launchers

hipError_t launch_tags(const Level &L, double thresh, const double *psi, uint8_t *tags,
                       hipStream_t st) {
  double hmax = 0.0;
  for (int a = 0; a < L.g.dim; ++a) hmax = std::max(hmax, L.h[a]);
  const double hmax2 = hmax * hmax, thr2 = thresh * thresh;
  if (L.g.dim == 3)
    AMR_LAUNCH((k_amr_tags<3>), num_blocks(L.g.nc), kBlock, st, L.g, L.h[0], L.h[1], L.h[2], hmax2,
               thr2, psi, tags);
  AMR_LAUNCH((k_amr_tags<2>), num_blocks(L.g.nc), kBlock, st, L.g, L.h[0], L.h[1], L.h[2], hmax2,
             thr2, psi, tags);
}

// Grid and tile argument of a level kernel: the listed tiles, or every node.
struct NodeGrid {
  int blocks;
  bool tiled;
  TileArg ta;
};

static NodeGrid node_grid(const Level &L, const TileList *tl) {
  if (tl) {
    const TileGeom tg = tile_geom_of(L, tl->kz);
    return NodeGrid{tl->count * tg.kz, true, TileArg{tg, tl->ids}};
  }
  return NodeGrid{num_blocks(L.g.nn), false, TileArg{TileGeom{1, 1, 1, 1}, nullptr}};
}

#define AMR_NODE_LAUNCH(KT, KD, ng, st, ...)                                     \
  do {                                                                          \
    if ((ng).blocks == 0) return hipSuccess;                                    \
    if ((ng).tiled) AMR_LAUNCH(KT, (ng).blocks, kBlock, st, __VA_ARGS__, (ng).ta); \
    AMR_LAUNCH(KD, (ng).blocks, kBlock, st, __VA_ARGS__, (ng).ta);              \
  } while (0)

// The ghost nodes of a level listed at set-up.
struct GhostList {
  const int *ids = nullptr;
  int count = 0;
};

template <typename T>
hipError_t launch_ghost_list(const Level &F, const Level &C, const GhostList &gl, const T *xc,
                             T *xf, hipStream_t st) {
  if (gl.count == 0) return hipSuccess;
  const int nb = (gl.count + kBlock - 1) / kBlock;
  if (F.g.dim == 3)
    AMR_LAUNCH((k_amr_ghost_list<T, 3>), nb, kBlock, st, F.g, C.g, gl.ids, gl.count, xc, xf);
  AMR_LAUNCH((k_amr_ghost_list<T, 2>), nb, kBlock, st, F.g, C.g, gl.ids, gl.count, xc, xf);
}

template <typename T>
hipError_t launch_zero_nodes(const Level &L, const TileList *tl, T *x, hipStream_t st) {
  const NodeGrid ng = node_grid(L, tl);
  AMR_NODE_LAUNCH((k_amr_zero<T, true>), (k_amr_zero<T, false>), ng, st, L.g, x);
}

template <typename T>
hipError_t launch_ghost_copy(const Level &L, const GhostList &gl, const T *src, T *dst,
                             hipStream_t st) {
  if (gl.count == 0) return hipSuccess;
  const int nb = (gl.count + kBlock - 1) / kBlock;
  AMR_LAUNCH((k_amr_ghost_copy<T>), nb, kBlock, st, L.g.nn, L.g.dim, gl.ids, gl.count, src, dst);
}

template <typename T>
hipError_t launch_residual_list(const Level &L, const T *psi, const Coef<T> &C, const T *u,
                                const T *f, T *r, const uint8_t *cls, const GhostList &nl,
                                hipStream_t st) {
  if (nl.count == 0) return hipSuccess;
  const int nb = (nl.count + kBlock - 1) / kBlock;
  AMR_LAUNCH((k_residual_list<T>), nb, kBlock, st, L.g, C, psi, u, f, r, cls, nl.ids, nl.count);
}

// ids (increasing) of the nodes 0 .. nn-1 that pick selects, their number in
// *total; bcnt and boff hold one int per kCompactNodes nodes.
template <class P>
hipError_t launch_listing(int64_t nn, const P &pick, int *bcnt, int *boff, int *ids, int *total,
                          hipStream_t st) {
  const int64_t nb = (nn + kCompactNodes - 1) / kCompactNodes;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_list_count<P>, dim3((unsigned)nb), dim3(kBlock), 0, st, nn, pick, bcnt);
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, (const int *)bcnt, (int)nb, boff,
                     total);
  hipLaunchKernelGGL(k_list_write<P>, dim3((unsigned)nb), dim3(kBlock), 0, st, nn, pick,
                     (const int *)boff, ids);
  return hipGetLastError();
}

// cl: the coarse nodes on or inside the fine region, listed at set-up.
template <typename T>
hipError_t launch_restrict_cif(const Level &F, const Level &C, const uint8_t *clsf,
                               const GhostList &cl, const T *rf, const T *add, const T *add2,
                               T *out, hipStream_t st, bool only_ghosts = false) {
  if (cl.count == 0) return hipSuccess;
  const int nb = (cl.count + kBlock - 1) / kBlock;
  if (only_ghosts) {
    if (F.g.dim == 3)
      AMR_LAUNCH((k_amr_restrict_cif<T, 3, true>), nb, kBlock, st, F.g, C.g, clsf, cl.ids,
                 cl.count, rf, add, add2, out);
    AMR_LAUNCH((k_amr_restrict_cif<T, 2, true>), nb, kBlock, st, F.g, C.g, clsf, cl.ids, cl.count,
               rf, add, add2, out);
  }
  if (F.g.dim == 3)
    AMR_LAUNCH((k_amr_restrict_cif<T, 3, false>), nb, kBlock, st, F.g, C.g, clsf, cl.ids,
               cl.count, rf, add, add2, out);
  AMR_LAUNCH((k_amr_restrict_cif<T, 2, false>), nb, kBlock, st, F.g, C.g, clsf, cl.ids, cl.count,
             rf, add, add2, out);
}

hipError_t launch_amr_cast(const Level &L, const uint8_t *cls, const double *r, float *r32,
                           const double *ss, hipStream_t st, const TileList *tl = nullptr) {
  const NodeGrid ng = node_grid(L, tl);
  if (L.g.dim == 3)
    AMR_NODE_LAUNCH((k_amr_cast<3, true>), (k_amr_cast<3, false>), ng, st, L.g, cls, r, r32, ss);
  AMR_NODE_LAUNCH((k_amr_cast<2, true>), (k_amr_cast<2, false>), ng, st, L.g, cls, r, r32, ss);
}

template <typename T>
hipError_t launch_inject(const Level &F, const Level &C, const uint8_t *clsf, const T *xf, T *xc,
                         hipStream_t st) {
  if (F.g.dim == 3) AMR_LAUNCH((k_amr_inject<T, 3>), num_blocks(C.g.nn), kBlock, st, F.g, C.g, clsf, xf, xc);
  AMR_LAUNCH((k_amr_inject<T, 2>), num_blocks(C.g.nn), kBlock, st, F.g, C.g, clsf, xf, xc);
}

template <typename T>
hipError_t launch_amr_correct(const Level &F, const Level &C, const uint8_t *clsf, const T *xc,
                              const T *xinj, T *xf, hipStream_t st, const TileList *tl = nullptr) {
  const NodeGrid ng = node_grid(F, tl);
  if (F.g.dim == 3)
    AMR_NODE_LAUNCH((k_amr_correct<T, 3, true>), (k_amr_correct<T, 3, false>), ng, st, F.g, C.g,
                    clsf, xc, xinj, xf);
  AMR_NODE_LAUNCH((k_amr_correct<T, 2, true>), (k_amr_correct<T, 2, false>), ng, st, F.g, C.g,
                  clsf, xc, xinj, xf);
}

template <typename T>
hipError_t launch_update(const Level &L, const uint8_t *cls, double *u, const T *e,
                         const double *ss, hipStream_t st, const TileList *tl = nullptr) {
  const NodeGrid ng = node_grid(L, tl);
  if (L.g.dim == 3)
    AMR_NODE_LAUNCH((k_amr_update<T, 3, true>), (k_amr_update<T, 3, false>), ng, st, L.g, cls, u,
                    e, ss);
  AMR_NODE_LAUNCH((k_amr_update<T, 2, true>), (k_amr_update<T, 2, false>), ng, st, L.g, cls, u, e,
                  ss);
}

// Partial sums land in partials[0 .. blocks); with a tile list the rest of
// the level's slots must hold zeros.
hipError_t launch_sumsq(const Level &L, const uint8_t *cls, const Level *F, const uint8_t *clsf,
                        const double *r, double *partials, hipStream_t st,
                        const TileList *tl = nullptr) {
  const Geom gf = F ? F->g : L.g;
  const NodeGrid ng = node_grid(L, tl);
  if (L.g.dim == 3)
    AMR_NODE_LAUNCH((k_amr_sumsq<3, true>), (k_amr_sumsq<3, false>), ng, st, L.g, cls, gf, clsf, r,
                    partials);
  AMR_NODE_LAUNCH((k_amr_sumsq<2, true>), (k_amr_sumsq<2, false>), ng, st, L.g, cls, gf, clsf, r,
                  partials);
}

struct Carver {
  char *base;
  size_t off = 0;
  template <typename T>
  T *take(int64_t n) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? (T *)(base + off) : nullptr;
    off += (size_t)std::max<int64_t>(n, 1) * sizeof(T);
    return p;
  }
};

}  // namespace

// ------------------------------------------------------------------ context

struct AmrLevel {
  Level L;                 // geometry, coefficients, psi (FP64 / FP32)
  int nb[3] = {1, 1, 1};   // blocks per axis (a >= 1)
  uint8_t *blk = nullptr;  // block flags (a >= 1)
  uint8_t *cls = nullptr;  // node classes (a >= 1)
  uint8_t *clo = nullptr;  // closure scratch (a >= 1)
  uint8_t *tags = nullptr; // cell tags (a < A)
  double *fP = nullptr, *r = nullptr, *e = nullptr, *w = nullptr, *xinj = nullptr, *tmp = nullptr;
  float *e32 = nullptr, *f32 = nullptr, *w32 = nullptr, *xinj32 = nullptr, *tmp32 = nullptr;
  float *g32 = nullptr;    // FP32 cycle: R of the finer level's ghost-row loads (a < A)
  int *tflags = nullptr;   // tile flags (listing scratch, tiled levels a >= 1)
  int *tids1 = nullptr;    // the column tiles that hold unknowns (class 1)
  int *goids = nullptr;    // ghost nodes outside those tiles
  int *cids = nullptr;     // level a-1 nodes on or inside this level's region
  int *gids = nullptr, *gcnt = nullptr, *goff = nullptr;  // ghost-node list and its scratch
  GhostList gl;            // the level's ghost nodes (a >= 1; count 0 until set_problem)
  TileList tl1;            // its tiles with unknowns (count 0 until set_problem)
  GhostList go;            // its ghost nodes in none of those tiles
  GhostList cl;            // the coarse nodes its composite restriction writes
  bool tiled = false;      // the level's passes run over tl1 (and the lists)
  // the tiles of every pass over the level: the smoothing, correction, update,
  // norm and zeroing touch class-1 nodes only; the residual and the FP32 loads
  // also reach the ghost nodes, by the list go for those outside the tiles
  const TileList *unknown_tiles() const { return tiled ? &tl1 : nullptr; }
  int part_off = 0;        // offset of this level's partial sums
  Traction tr{};
  int64_t nblocks() const { return (int64_t)nb[0] * nb[1] * nb[2]; }
  int64_t nv() const { return (int64_t)L.g.dim * L.g.nn; }
};

struct sbm_amr_ctx {
  int dim = 0, A = 0, bc = 0;
  sbm_grid base_grid{};
  sbm_options opt{};
  hipStream_t st = nullptr;
  std::vector<AmrLevel> lv;
  sbm_ctx *base = nullptr;
  size_t base_bytes = 0;
  double *partials = nullptr;
  int npart = 0;
  double *scal = nullptr;
  int *iflag = nullptr;
  double *host = nullptr;  // pinned host scalars
  sbm_material mat{};
  DispValues dv{};
  double fnorm = 0.0;
  int64_t comp_dof = 0;
  bool have_problem = false;
  double cluster_eff = 0.0;  // Berger-Rigoutsos efficiency of the block boxes (0: off)
  // live timing of finest-level launches
  bool prof_on = false;
  std::vector<hipEvent_t> prof_ev;  // pairs
  std::vector<int> prof_cls;        // class of each pair in use
  double prof_ms[SBM_PROF_N] = {0};
  int64_t prof_n[SBM_PROF_N] = {0};
};

// Berger-Rigoutsos point clustering of the block flags of one level (host):
// every flagged block ends inside an accepted box, a box being the bounding
// box of its flags, accepted when flags >= eff * volume.  A box that is not
// accepted is cut, and both parts are processed again, at
//   1. a hole: an interior slab without flags (first axis that has one; the
//      hole nearest the middle, the lower on a tie; the slab joins neither
//      part), else
//   2. the strongest inflection of the signature s (flags per slab): where
//      the discrete Laplacian s(i-1) - 2 s(i) + s(i+1) changes sign strictly
//      between slabs i and i+1, strength the jump of the Laplacian; strongest
//      over all axes, the first met (axis order, ascending i) on a tie, else
//   3. the middle of the longest axis (first longest; the lower part keeps
//      the middle slab).
// The blocks of the accepted boxes form the new flags.  Parts are processed
// from an explicit stack; the union of the boxes does not depend on order.
struct BrBox {
  int lo[3], hi[3];
};

static void br_cluster(int dim, const int nb[3], const uint8_t *in, double eff, uint8_t *out) {
  const int64_t nx = nb[0], nxy = (int64_t)nb[0] * nb[1];
  auto at = [&](int x, int y, int z) { return x + nx * y + nxy * z; };
  std::fill(out, out + nxy * nb[2], (uint8_t)0);
  std::vector<BrBox> todo;
  todo.push_back(BrBox{{0, 0, 0}, {nb[0] - 1, nb[1] - 1, nb[2] - 1}});
  std::vector<int> sig[3];
  while (!todo.empty()) {
    BrBox B = todo.back();
    todo.pop_back();
    int lo[3] = {B.hi[0] + 1, B.hi[1] + 1, B.hi[2] + 1};
    int hi[3] = {B.lo[0] - 1, B.lo[1] - 1, B.lo[2] - 1};
    int64_t cnt = 0;
    for (int z = B.lo[2]; z <= B.hi[2]; ++z)
      for (int y = B.lo[1]; y <= B.hi[1]; ++y)
        for (int x = B.lo[0]; x <= B.hi[0]; ++x)
          if (in[at(x, y, z)]) {
            ++cnt;
            const int q[3] = {x, y, z};
            for (int a = 0; a < 3; ++a) {
              lo[a] = std::min(lo[a], q[a]);
              hi[a] = std::max(hi[a], q[a]);
            }
          }
    if (cnt == 0) continue;
    double vol = 1.0;
    for (int a = 0; a < 3; ++a) vol *= (double)(hi[a] - lo[a] + 1);
    if ((double)cnt >= eff * vol) {
      for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
          for (int x = lo[0]; x <= hi[0]; ++x) out[at(x, y, z)] = 1;
      continue;
    }
    for (int a = 0; a < dim; ++a) sig[a].assign(hi[a] - lo[a] + 1, 0);
    for (int z = lo[2]; z <= hi[2]; ++z)
      for (int y = lo[1]; y <= hi[1]; ++y)
        for (int x = lo[0]; x <= hi[0]; ++x)
          if (in[at(x, y, z)]) {
            const int q[3] = {x, y, z};
            for (int a = 0; a < dim; ++a) ++sig[a][q[a] - lo[a]];
          }
    int axis = -1, end_lo = 0, start_hi = 0;
    for (int a = 0; a < dim && axis < 0; ++a) {  // 1. holes
      int best = -1, bestd = 0;
      for (int i = lo[a] + 1; i < hi[a]; ++i) {
        if (sig[a][i - lo[a]]) continue;
        const int dd = std::abs(2 * i - lo[a] - hi[a]);
        if (best < 0 || dd < bestd) {
          best = i;
          bestd = dd;
        }
      }
      if (best >= 0) {
        axis = a;
        end_lo = best - 1;
        start_hi = best + 1;
      }
    }
    if (axis < 0) {  // 2. inflections
      int64_t best = 0;
      for (int a = 0; a < dim; ++a) {
        const std::vector<int> &S = sig[a];
        const int n = hi[a] - lo[a] + 1;
        for (int i = 1; i + 2 < n; ++i) {  // slabs lo+i and lo+i+1, both interior
          const int64_t l0 = (int64_t)S[i - 1] - 2 * S[i] + S[i + 1];
          const int64_t l1 = (int64_t)S[i] - 2 * S[i + 1] + S[i + 2];
          if (!((l0 < 0 && l1 > 0) || (l0 > 0 && l1 < 0))) continue;
          const int64_t jump = l1 > l0 ? l1 - l0 : l0 - l1;
          if (jump > best) {
            best = jump;
            axis = a;
            end_lo = lo[a] + i;
            start_hi = lo[a] + i + 1;
          }
        }
      }
    }
    if (axis < 0) {  // 3. middle of the longest axis
      int len = 0;
      for (int a = 0; a < dim; ++a)
        if (hi[a] - lo[a] + 1 > len) {
          len = hi[a] - lo[a] + 1;
          axis = a;
        }
      end_lo = (lo[axis] + hi[axis]) / 2;
      start_hi = end_lo + 1;
    }
    BrBox P{{lo[0], lo[1], lo[2]}, {hi[0], hi[1], hi[2]}}, Q = P;
    P.hi[axis] = end_lo;
    Q.lo[axis] = start_hi;
    todo.push_back(Q);
    todo.push_back(P);
  }
}

// Brackets the launches of its scope with an event pair when profiling is on
// and the scope belongs to the finest level.
struct AmrProf {
  sbm_amr_ctx *c;
  bool on;
  size_t pair = 0;
  AmrProf(sbm_amr_ctx *c_, int cls, bool finest) : c(c_), on(c_->prof_on && finest) {
    if (!on) return;
    pair = c->prof_cls.size();
    while (c->prof_ev.size() < 2 * (pair + 1)) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) {
        on = false;
        return;
      }
      c->prof_ev.push_back(e);
    }
    c->prof_cls.push_back(cls);
    (void)hipEventRecord(c->prof_ev[2 * pair], c->st);
  }
  ~AmrProf() {
    if (on) (void)hipEventRecord(c->prof_ev[2 * pair + 1], c->st);
  }
};

// Accumulates the completed pairs (the stream is idle) and frees the pool.
static void amr_prof_harvest(sbm_amr_ctx *c) {
  for (size_t p = 0; p < c->prof_cls.size(); ++p) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, c->prof_ev[2 * p], c->prof_ev[2 * p + 1]) == hipSuccess) {
      c->prof_ms[c->prof_cls[p]] += ms;
      c->prof_n[c->prof_cls[p]] += 1;
    }
  }
  c->prof_cls.clear();
}

static sbm_status amr_fail(sbm_status s, const std::string &m) { return set_error(s, m); }

#define AMR_HIP(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return amr_fail(SBM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

#define AMR_TRY(expr)            \
  do {                           \
    sbm_status s_ = (expr);      \
    if (s_ != SBM_OK) return s_; \
  } while (0)

// Shapes of the AMR levels; false when the layout is not supported.
static bool amr_layout(const sbm_grid *g, int levels, int block, std::vector<AmrLevel> &lv,
                       std::string &why) {
  if (!g || (g->dim != 2 && g->dim != 3)) return why = "dim must be 2 or 3", false;
  if (levels < 1 || levels > kMaxAmrLevels) return why = "levels must be 1..4", false;
  if (block < 2 || block % 2) return why = "block must be even and >= 2", false;
  for (int a = 0; a < g->dim; ++a) {
    if (g->ncell[a] < 2 || !(g->h[a] > 0.0) || !isfinite(g->h[a]))
      return why = "base grid needs ncell >= 2 and h > 0", false;
    if (levels > 1 && (2 * g->ncell[a]) % block)
      return why = "block must divide twice the base cell count", false;
  }
  lv.assign(levels, AmrLevel());
  for (int a = 0; a < levels; ++a) {
    int64_t nc[3] = {1, 1, 1};
    double h[3] = {1.0, 1.0, 1.0};
    for (int x = 0; x < g->dim; ++x) {
      nc[x] = g->ncell[x] << a;
      h[x] = g->h[x] / (double)(1 << a);
    }
    int64_t nodes = 1;
    for (int x = 0; x < g->dim; ++x) nodes *= nc[x] + 1;
    if (nodes * g->dim >= ((int64_t)1 << 31)) return why = "finest level exceeds 2^31 DOF", false;
    make_level(g->dim, nc, h, lv[a].L);
    if (a >= 1)
      for (int x = 0; x < g->dim; ++x) lv[a].nb[x] = (int)(nc[x] / block);
  }
  return true;
}

static size_t amr_carve(sbm_amr_ctx *c, char *base) {
  Carver cv{base};
  const int A = c->A;
  int npart = 0;
  for (int a = 0; a <= A; ++a) {
    AmrLevel &l = c->lv[a];
    const int64_t nv = l.nv();
    l.L.psi64 = cv.take<double>(l.L.g.nc);
    l.L.psi32 = cv.take<float>(l.L.g.nc);
    if (a >= 1) {
      l.blk = cv.take<uint8_t>(l.nblocks());
      l.cls = cv.take<uint8_t>(l.L.g.nn);
      l.clo = cv.take<uint8_t>(l.L.g.nn);
      l.gids = cv.take<int>(l.L.g.nn);
      const int64_t ncb = (l.L.g.nn + 4 * kBlock - 1) / (4 * kBlock);
      l.gcnt = cv.take<int>(ncb);
      l.goff = cv.take<int>(ncb);
      l.cids = cv.take<int>(c->lv[a - 1].L.g.nn);
      l.tiled = tiled_ok(l.L) && tile_geom_of(l.L).ntiles <= num_blocks(l.L.g.nn);
      if (l.tiled) {
        // sized for the most tiles the set-up may list: the default chunks
        // or the shallowest ones it may choose
        const int nt = std::max(tile_geom_of(l.L).ntiles, tile_geom_of(l.L, kAmrKzMin).ntiles);
        l.tflags = cv.take<int>(nt);
        l.tids1 = cv.take<int>(nt);
        l.goids = cv.take<int>(l.L.g.nn);
      }
    }
    if (a < A) l.tags = cv.take<uint8_t>(l.L.g.nc);
    l.fP = cv.take<double>(nv);
    l.r = cv.take<double>(nv);
    l.e = cv.take<double>(nv);
    l.w = cv.take<double>(nv);
    l.tmp = cv.take<double>(nv);
    l.e32 = cv.take<float>(nv);
    l.f32 = cv.take<float>(nv);
    l.w32 = cv.take<float>(nv);
    l.tmp32 = cv.take<float>(nv);
    if (a < A) {
      l.xinj = cv.take<double>(nv);
      l.xinj32 = cv.take<float>(nv);
      l.g32 = cv.take<float>(nv);
    }
    l.part_off = npart;
    npart += num_blocks(l.L.g.nn);
  }
  c->npart = npart;
  c->partials = cv.take<double>(npart);
  c->scal = cv.take<double>(16);
  c->iflag = cv.take<int>(kIflags);
  cv.off = (cv.off + 255) & ~(size_t)255;
  return cv.off;
}

static sbm_options base_options(const sbm_options &o) {
  sbm_options b = o;
  b.krylov = 0;
  b.use_graphs = 0;
  return b;
}

// ------------------------------------------------------------- cycle (host)

template <typename T>
struct AV;
template <>
struct AV<double> {
  static double *x(AmrLevel &l) { return l.e; }
  static double *f(AmrLevel &l) { return l.r; }
  static double *w(AmrLevel &l) { return l.w; }
  static double *xinj(AmrLevel &l) { return l.xinj; }
  static double *tmp(AmrLevel &l) { return l.tmp; }
  static const double *psi(const AmrLevel &l) { return l.L.psi64; }
  static const Coef<double> &coef(const AmrLevel &l) { return l.L.c64; }
};
template <>
struct AV<float> {
  static float *x(AmrLevel &l) { return l.e32; }
  static float *f(AmrLevel &l) { return l.f32; }
  static float *w(AmrLevel &l) { return l.w32; }
  static float *xinj(AmrLevel &l) { return l.xinj32; }
  static float *tmp(AmrLevel &l) { return l.tmp32; }
  static const float *psi(const AmrLevel &l) { return l.L.psi32; }
  static const Coef<float> &coef(const AmrLevel &l) { return l.L.c32; }
};

static double amr_omega(const sbm_options &o) {
  if (o.omega > 0.0) return o.omega;
  return o.smoother == 1 ? 0.8 : 1.0;
}

// nu sweeps on the unknowns of level a >= 1 (class 1); other nodes keep x.
// The cycle's iterate from zero: a tiled level zeroes its tiles with
// unknowns and the ghost nodes outside them (the nodes any of its passes
// read), not the whole level.
template <typename T>
static hipError_t amr_zero(sbm_amr_ctx *c, const AmrLevel &l, T *x) {
  if (!l.tiled) return launch_fill<T>(x, l.nv(), T(0), c->st);
  hipError_t e = launch_zero_nodes<T>(l.L, l.unknown_tiles(), x, c->st);
  if (e != hipSuccess) return e;
  return launch_ghost_copy<T>(l.L, l.go, nullptr, x, c->st);
}

// Padded residual of level l (classes 1-3; 0 at the other nodes of its
// tiles): a tiled level evaluates it over its tiles with unknowns and the
// ghost nodes outside them, so that no pass sweeps the tiles that only hold
// ghost faces.
template <typename T>
static hipError_t amr_residual(sbm_amr_ctx *c, const AmrLevel &l, const T *psi, const Coef<T> &C,
                               const T *x, const T *f, T *r) {
  if (!l.tiled && tiled_sweep_ok(l.L))
    return launch_residual_tiled<T>(l.L, psi, C, x, f, r, nullptr, c->st, l.cls, nullptr);
  if (!l.tiled)
    return launch_residual<T>(l.L, psi, C, x, f, r, nullptr, c->st, l.cls, nullptr);
  hipError_t e = launch_residual<T>(l.L, psi, C, x, f, r, nullptr, c->st, l.cls, l.unknown_tiles());
  if (e != hipSuccess) return e;
  return launch_residual_list<T>(l.L, psi, C, x, f, r, l.cls, l.go, c->st);
}

template <typename T>
static hipError_t amr_smooth(sbm_amr_ctx *c, int a, T *x, const T *f, T *tmp, int nu) {
  AmrLevel &l = c->lv[a];
  const double om = amr_omega(c->opt);
  const bool fin = a == c->A;
  hipError_t e = hipSuccess;
  if (c->opt.smoother == 1) {
    T *src = x, *dst = tmp;
    for (int s = 0; s < nu; ++s) {
      AmrProf pr(c, SBM_PROF_SMOOTH, fin);
      if ((e = launch_jacobi<T>(l.L, AV<T>::psi(l), AV<T>::coef(l), src, f, dst, om, c->st,
                                l.cls)) != hipSuccess)
        return e;
      std::swap(src, dst);
    }
    if (src != x) e = launch_copy<T>(src, x, l.nv(), c->st);
    return e;
  }
  // levels with tile lists sweep their listed tiles; a smaller level whose
  // half-sweep still pays tiled (from 97 nodes) sweeps all its tiles, the
  // class mask applied, as the node-parallel kernel does
  const bool tiled = l.tiled;
  const bool whole = !tiled && tiled_sweep_ok(l.L);
  // The listed tiles cover the unknowns, not every ghost node their stencils
  // read: the second half-sweep reads those from tmp, so tmp gets x's ghosts.
  if (tiled && (e = launch_ghost_copy<T>(l.L, l.gl, x, tmp, c->st)) != hipSuccess) return e;
  auto half = [&](const T *src, T *dst, int colour) {
    if (tiled || whole)
      return launch_rb_tiled<T>(l.L, AV<T>::psi(l), AV<T>::coef(l), src, f, dst, om, colour, c->st,
                                l.cls, l.unknown_tiles());
    return launch_rb_half<T>(l.L, AV<T>::psi(l), AV<T>::coef(l), src, f, dst, om, colour, c->st,
                             l.cls);
  };
  for (int s = 0; s < nu; ++s) {
    {
      AmrProf pr(c, SBM_PROF_SMOOTH, fin);
      if ((e = half(x, tmp, 0)) != hipSuccess) return e;
    }
    AmrProf pr(c, SBM_PROF_SMOOTH, fin);
    if ((e = half(tmp, x, 1)) != hipSuccess) return e;
  }
  return e;
}

// Full-approximation cycle over AMR levels a..1 on the level vectors of
// precision T (x, f, w, xinj, tmp), ending in the base V-cycle.
template <typename T>
static hipError_t amr_fas(sbm_amr_ctx *c, int a) {
  if (a == 0) {
    AmrLevel &l0 = c->lv[0];
    AmrProf pr(c, SBM_PROF_BOTTOM, true);
    return base_vcycle(c->base, sizeof(T) == 8 ? 0 : 1, AV<T>::x(l0), AV<T>::f(l0));
  }
  AmrLevel &F = c->lv[a];
  AmrLevel &C = c->lv[a - 1];
  const bool fin = a == c->A;
  hipError_t e;
  T *xf = AV<T>::x(F), *ff = AV<T>::f(F), *wf = AV<T>::w(F), *tf = AV<T>::tmp(F);
  T *xc = AV<T>::x(C), *fc = AV<T>::f(C), *xi = AV<T>::xinj(C), *tc = AV<T>::tmp(C);
  // The cycle runs in correction form from zero on every level, and nothing
  // has touched level a-1 when level a is entered (injections write class-1
  // nodes only), so the ghosts of level a already hold their fill from x_c =
  // 0 (zero), and the smoother leaves ghosts unchanged: the ghost fills before
  // and after pre-smoothing would rewrite the same values and are skipped.
  if ((e = amr_smooth<T>(c, a, xf, ff, tf, c->opt.nu_pre)) != hipSuccess) return e;
  {
    AmrProf pr(c, SBM_PROF_RESIDUAL, fin);
    if ((e = amr_residual<T>(c, F, AV<T>::psi(F), AV<T>::coef(F), xf, ff, wf)) != hipSuccess)
      return e;
  }
  if ((e = launch_inject<T>(F.L, C.L, F.cls, xf, xc, c->st)) != hipSuccess) return e;
  if ((e = launch_copy<T>(xc, xi, C.nv(), c->st)) != hipSuccess) return e;
  // coarse load on covered and interface nodes: R w + K_c x_c
  if ((e = launch_apply<T>(C.L, AV<T>::psi(C), AV<T>::coef(C), xc, tc, c->st)) != hipSuccess)
    return e;
  const T *g = nullptr;
  if constexpr (sizeof(T) == 4) g = C.g32;
  {
    AmrProf pr(c, SBM_PROF_RESTRICT, fin);
    if ((e = launch_restrict_cif<T>(F.L, C.L, F.cls, F.cl, wf, tc, g, fc, c->st)) != hipSuccess)
      return e;
  }
  if ((e = amr_fas<T>(c, a - 1)) != hipSuccess) return e;
  {
    AmrProf pr(c, SBM_PROF_PROLONG, fin);
    if ((e = launch_amr_correct<T>(F.L, C.L, F.cls, xc, xi, xf, c->st, F.unknown_tiles())) !=
        hipSuccess)
      return e;
  }
  {
    AmrProf pr(c, SBM_PROF_GHOST, fin);
    if ((e = launch_ghost_list<T>(F.L, C.L, F.gl, xc, xf, c->st)) != hipSuccess) return e;
  }
  return amr_smooth<T>(c, a, xf, ff, tf, c->opt.nu_post);
}

// Composite residual of x (ghosts refilled in place) for the loads f into r;
// ||r||^2 over the composite unknowns lands in scal[0] and host[0].
static sbm_status amr_comp_residual(sbm_amr_ctx *c, double *const *x, double *const *f,
                                    double *const *r, bool sync) {
  const int A = c->A;
  for (int a = 1; a <= A; ++a)
    AMR_HIP(launch_ghost_list<double>(c->lv[a].L, c->lv[a - 1].L, c->lv[a].gl, x[a - 1], x[a],
                                      c->st));
  for (int a = A; a >= 0; --a) {
    AmrLevel &l = c->lv[a];
    AmrProf pr(c, SBM_PROF_NORM, a == A);
    if (a >= 1)
      AMR_HIP(amr_residual<double>(c, l, l.L.psi64, l.L.c64, x[a], f[a], r[a]));
    else
      AMR_HIP(launch_residual<double>(l.L, l.L.psi64, l.L.c64, x[a], f[a], r[a], nullptr, c->st,
                                      nullptr, nullptr));
    if (a < A)
      AMR_HIP(launch_restrict_cif<double>(c->lv[a + 1].L, l.L, c->lv[a + 1].cls, c->lv[a + 1].cl,
                                          r[a + 1], nullptr, nullptr, r[a], c->st));
  }
  for (int a = 0; a <= A; ++a) {
    AmrLevel &l = c->lv[a];
    AMR_HIP(launch_sumsq(l.L, a >= 1 ? l.cls : nullptr, a < A ? &c->lv[a + 1].L : nullptr,
                         a < A ? c->lv[a + 1].cls : nullptr, r[a], c->partials + l.part_off,
                         c->st, a >= 1 ? l.unknown_tiles() : nullptr));
  }
  AMR_HIP(launch_finalize_sum(c->partials, c->npart, c->scal, c->st));
  if (sync) {
    AMR_HIP(hipMemcpyAsync(c->host, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->st));
    AMR_HIP(hipStreamSynchronize(c->st));
    if (c->prof_on) amr_prof_harvest(c);
  }
  return SBM_OK;
}

static sbm_status amr_inject_all(sbm_amr_ctx *c, double *const *u) {
  for (int a = c->A; a >= 1; --a)
    AMR_HIP(launch_inject<double>(c->lv[a].L, c->lv[a - 1].L, c->lv[a].cls, u[a], u[a - 1], c->st));
  return SBM_OK;
}

// ---------------------------------------------------------------------- ABI

extern "C" {

size_t sbm_amr_workspace_bytes(const sbm_grid *base, int levels, int block,
                               const sbm_options *opts) {
  if (!opts) return 0;
  sbm_amr_ctx c;
  std::string why;
  if (!amr_layout(base, levels, block, c.lv, why)) return 0;
  c.dim = base->dim;
  c.A = levels - 1;
  const sbm_options bo = base_options(*opts);
  const size_t bb = sbm_workspace_bytes(base, &bo);
  if (bb == 0) return 0;
  return amr_carve(&c, nullptr) + ((bb + 255) & ~(size_t)255);
}

sbm_status sbm_amr_create(const sbm_grid *base, int levels, int block, const sbm_options *opts,
                          void *workspace, size_t workspace_bytes, void *hip_stream,
                          sbm_amr_ctx **out) {
  if (!out) return amr_fail(SBM_E_ARG, "out is NULL");
  *out = nullptr;
  if (!opts) return amr_fail(SBM_E_ARG, "opts is NULL");
  if (opts->krylov != 0)
    return amr_fail(SBM_E_ARG, "the composite solve runs stationary cycles only (krylov = 0)");
  if (!workspace || ((uintptr_t)workspace & 255))
    return amr_fail(SBM_E_WORKSPACE, "workspace NULL or not 256-byte aligned");
  sbm_amr_ctx *c = new sbm_amr_ctx();
  std::string why;
  if (!amr_layout(base, levels, block, c->lv, why)) {
    delete c;
    return amr_fail(SBM_E_SHAPE, "unsupported adaptive layout: " + why);
  }
  c->dim = base->dim;
  c->A = levels - 1;
  c->bc = block;
  c->base_grid = *base;
  c->opt = *opts;
  c->st = (hipStream_t)hip_stream;
  const size_t own = amr_carve(c, nullptr);
  const sbm_options bo = base_options(*opts);
  const size_t bb = sbm_workspace_bytes(base, &bo);
  if (bb == 0) {
    delete c;
    return amr_fail(SBM_E_ARG, "invalid options or base grid");
  }
  const size_t need = own + ((bb + 255) & ~(size_t)255);
  if (workspace_bytes < need) {
    delete c;
    return amr_fail(SBM_E_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  }
  amr_carve(c, (char *)workspace);
  sbm_status s = sbm_create(base, &bo, (char *)workspace + own, workspace_bytes - own, hip_stream,
                            &c->base);
  if (s != SBM_OK) {
    delete c;
    return s;
  }
  hipError_t e = hipHostMalloc((void **)&c->host, 64 * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) {
    sbm_destroy(c->base);
    delete c;
    return amr_fail(SBM_E_HIP, std::string("hipHostMalloc: ") + hipGetErrorString(e));
  }
  *out = c;
  return SBM_OK;
}

sbm_status sbm_amr_profile(sbm_amr_ctx *c, int enable) {
  if (!c) return amr_fail(SBM_E_ARG, "ctx is NULL");
  AMR_HIP(hipStreamSynchronize(c->st));
  c->prof_cls.clear();
  for (int k = 0; k < SBM_PROF_N; ++k) {
    c->prof_ms[k] = 0.0;
    c->prof_n[k] = 0;
  }
  c->prof_on = enable != 0;
  return SBM_OK;
}

sbm_status sbm_amr_profile_read(sbm_amr_ctx *c, double *ms, int64_t *cnt) {
  if (!c || !ms || !cnt) return amr_fail(SBM_E_ARG, "NULL argument");
  AMR_HIP(hipStreamSynchronize(c->st));
  amr_prof_harvest(c);
  for (int k = 0; k < SBM_PROF_N; ++k) {
    ms[k] = c->prof_ms[k];
    cnt[k] = c->prof_n[k];
  }
  return SBM_OK;
}

void sbm_amr_destroy(sbm_amr_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->st);
  for (hipEvent_t e : c->prof_ev) (void)hipEventDestroy(e);
  if (c->base) sbm_destroy(c->base);
  if (c->host) (void)hipHostFree(c->host);
  delete c;
}

sbm_status sbm_amr_set_options(sbm_amr_ctx *c, const sbm_options *opts) {
  if (!c || !opts) return amr_fail(SBM_E_ARG, "NULL argument");
  if (opts->krylov != 0)
    return amr_fail(SBM_E_ARG, "the composite solve runs stationary cycles only (krylov = 0)");
  const sbm_options bo = base_options(*opts);
  AMR_TRY(sbm_set_options(c->base, &bo));
  c->opt = *opts;
  return SBM_OK;
}

// Replaces the block flags of level a by the blocks of their Berger-Rigoutsos
// boxes (device flags, staged through the host; synchronises).
static sbm_status amr_cluster_level(sbm_amr_ctx *c, int a) {
  AmrLevel &l = c->lv[a];
  const size_t n = l.nblocks();
  std::vector<uint8_t> in(n), out(n);
  AMR_HIP(hipMemcpyAsync(in.data(), l.blk, n, hipMemcpyDeviceToHost, c->st));
  AMR_HIP(hipStreamSynchronize(c->st));
  const int nb[3] = {l.nb[0], l.nb[1], l.nb[2]};
  br_cluster(c->dim, nb, in.data(), c->cluster_eff, out.data());
  AMR_HIP(hipMemcpyAsync(l.blk, out.data(), n, hipMemcpyHostToDevice, c->st));
  AMR_HIP(hipStreamSynchronize(c->st));
  return SBM_OK;
}

sbm_status sbm_amr_cluster(int dim, const int64_t *nblocks, const uint8_t *flags_host,
                           double efficiency, uint8_t *out_host) {
  if (!nblocks || !flags_host || !out_host) return amr_fail(SBM_E_ARG, "NULL argument");
  if (flags_host == out_host) return amr_fail(SBM_E_ARG, "out_host must not alias flags_host");
  if (dim != 2 && dim != 3) return amr_fail(SBM_E_SHAPE, "dim must be 2 or 3");
  if (!(efficiency >= 0.0 && efficiency <= 1.0)) return amr_fail(SBM_E_ARG, "efficiency in [0, 1]");
  int nb[3] = {1, 1, 1};
  for (int a = 0; a < dim; ++a) {
    if (nblocks[a] < 1 || nblocks[a] > (1 << 20)) return amr_fail(SBM_E_SHAPE, "block counts");
    nb[a] = (int)nblocks[a];
  }
  if ((int64_t)nb[0] * nb[1] * nb[2] > ((int64_t)1 << 30)) return amr_fail(SBM_E_SHAPE, "too many blocks");
  br_cluster(dim, nb, flags_host, efficiency, out_host);
  return SBM_OK;
}

sbm_status sbm_amr_set_clustering(sbm_amr_ctx *c, double efficiency) {
  if (!c) return amr_fail(SBM_E_ARG, "ctx is NULL");
  if (!(efficiency >= 0.0 && efficiency <= 1.0)) return amr_fail(SBM_E_ARG, "efficiency in [0, 1]");
  c->cluster_eff = efficiency;
  return SBM_OK;
}

sbm_status sbm_amr_set_problem(sbm_amr_ctx *c, const double *const *psi_raw,
                               const sbm_material *mat, const sbm_bc *bc, double tag_threshold,
                               const uint8_t *const *blocks_host) {
  if (!c || !psi_raw || !mat || !bc) return amr_fail(SBM_E_ARG, "NULL argument");
  const int A = c->A, d = c->dim;
  for (int a = 0; a <= A; ++a)
    if (!psi_raw[a]) return amr_fail(SBM_E_ARG, "psi_raw of a level is NULL");
  if (!isfinite(mat->lambda) || !isfinite(mat->mu) || !(mat->mu > 0.0) ||
      !(mat->lambda + mat->mu > 0.0) || !(mat->psi_floor >= 0.0))
    return amr_fail(SBM_E_ARG, "material needs mu > 0, lambda + mu > 0, psi_floor >= 0");
  if (!blocks_host && !(tag_threshold >= 0.0 && isfinite(tag_threshold)))
    return amr_fail(SBM_E_ARG, "tag_threshold must be finite and >= 0");
  uint32_t dmask = 0;
  memset(&c->dv, 0, sizeof(c->dv));
  Traction tr{};
  for (int F = 0; F < 2 * d; ++F)
    for (int k = 0; k < d; ++k) {
      if (bc->kind[F][k] != SBM_TRACTION && bc->kind[F][k] != SBM_DISPLACEMENT)
        return amr_fail(SBM_E_ARG, "bc kind must be TRACTION or DISPLACEMENT");
      if (!isfinite(bc->value[F][k])) return amr_fail(SBM_E_NONFINITE, "non-finite bc value");
      if (bc->kind[F][k] == SBM_DISPLACEMENT) {
        dmask |= 1u << (3 * F + k);
        c->dv.v[F][k] = bc->value[F][k];
      } else {
        tr.t[F][k] = bc->value[F][k];
      }
    }
  c->have_problem = false;
  c->mat = *mat;
  AMR_HIP(launch_fill<int>(c->iflag, kIflags, 0, c->st));
  for (int a = 0; a <= A; ++a) {
    AmrLevel &l = c->lv[a];
    l.L.g.dmask = dmask;
    set_coefs(l.L, mat->lambda, mat->mu, d);
    l.tr = tr;
    for (int F = 0; F < 6; ++F) l.tr.inv_h[F] = F / 2 < d ? 1.0 / l.L.h[F / 2] : 0.0;
    AMR_HIP(launch_floor_psi(psi_raw[a], mat->psi_floor, l.L.psi64, l.L.psi32, l.L.g.nc, 0,
                             c->iflag, c->st));
  }
  // block flags: tags of levels 0..A-1 (floored psi), footprints, nesting
  if (blocks_host) {
    for (int a = 1; a <= A; ++a) {
      if (!blocks_host[a - 1]) return amr_fail(SBM_E_ARG, "block flags of a level are NULL");
      AMR_HIP(hipMemcpyAsync(c->lv[a].blk, blocks_host[a - 1], c->lv[a].nblocks(),
                             hipMemcpyHostToDevice, c->st));
    }
  } else {
    for (int a = 0; a < A; ++a)
      AMR_HIP(launch_tags(c->lv[a].L, tag_threshold, c->lv[a].L.psi64, c->lv[a].tags, c->st));
    for (int a = 1; a <= A; ++a) {
      AmrLevel &l = c->lv[a];
      (void)hipGetLastError();
      hipLaunchKernelGGL(k_amr_blocks, dim3((unsigned)l.nblocks()), dim3(kBlock), 0, c->st,
                         c->lv[a - 1].L.g, d, l.nb[0], l.nb[1], c->bc / 2, c->lv[a - 1].tags,
                         l.blk);
      AMR_HIP(hipGetLastError());
    }
    // finest first: cluster (when enabled), then nest into the next coarser level
    for (int a = A; a >= 2; --a) {
      AmrLevel &l = c->lv[a], &p = c->lv[a - 1];
      if (c->cluster_eff > 0.0) {
        const sbm_status s = amr_cluster_level(c, a);
        if (s != SBM_OK) return s;
      }
      (void)hipGetLastError();
      hipLaunchKernelGGL(k_amr_nest, dim3(num_blocks(l.nblocks())), dim3(kBlock), 0, c->st, d,
                         l.nb[0], l.nb[1], l.nb[2], l.blk, p.nb[0], p.nb[1], p.nb[2], p.blk);
      AMR_HIP(hipGetLastError());
    }
    if (c->cluster_eff > 0.0 && A >= 1) {
      const sbm_status s = amr_cluster_level(c, 1);
      if (s != SBM_OK) return s;
    }
  }
  // node classes
  for (int a = 1; a <= A; ++a) {
    AmrLevel &l = c->lv[a];
    const int nb = num_blocks(l.L.g.nn);
    (void)hipGetLastError();
    if (d == 3) {
      hipLaunchKernelGGL(k_amr_classify<3>, dim3(nb), dim3(kBlock), 0, c->st, l.L.g, c->bc,
                         l.nb[0], l.nb[1], l.blk, l.clo, l.cls);
      hipLaunchKernelGGL(k_amr_layers<3>, dim3(nb), dim3(kBlock), 0, c->st, l.L.g, l.clo, l.cls);
    } else {
      hipLaunchKernelGGL(k_amr_classify<2>, dim3(nb), dim3(kBlock), 0, c->st, l.L.g, c->bc,
                         l.nb[0], l.nb[1], l.blk, l.clo, l.cls);
      hipLaunchKernelGGL(k_amr_layers<2>, dim3(nb), dim3(kBlock), 0, c->st, l.L.g, l.clo, l.cls);
    }
    AMR_HIP(hipGetLastError());
  }
  for (int a = 1; a <= A; ++a) {
    AmrLevel &l = c->lv[a];
    // the ghost nodes (classes 2-4), filled from the coarser level by a list
    // of their ids rather than by a pass over the level or its tiles
    l.gl = GhostList{l.gids, 0};
    AMR_HIP(launch_listing(l.L.g.nn, GhostPick{l.cls}, l.gcnt, l.goff, l.gids, c->iflag + 12 + a,
                           c->st));
    // the level a-1 nodes that the composite restriction writes, so that it
    // runs a thread per such node rather than over the whole coarse level
    l.cl = GhostList{l.cids, 0};
    AMR_HIP(launch_listing(c->lv[a - 1].L.g.nn, CifPick{l.L.g, c->lv[a - 1].L.g, l.cls}, l.gcnt,
                           l.goff, l.cids, c->iflag + 24 + a, c->st));
  }
  // psi of covered coarse cells, finest first
  for (int a = A; a >= 1; --a) {
    AmrLevel &f = c->lv[a], &p = c->lv[a - 1];
    (void)hipGetLastError();
    if (d == 3)
      hipLaunchKernelGGL(k_amr_avgdown<3>, dim3(num_blocks(p.L.g.nc)), dim3(kBlock), 0, c->st,
                         p.L.g, f.L.g, c->bc, f.nb[0], f.nb[1], f.blk, f.L.psi64, p.L.psi64,
                         p.L.psi32);
    else
      hipLaunchKernelGGL(k_amr_avgdown<2>, dim3(num_blocks(p.L.g.nc)), dim3(kBlock), 0, c->st,
                         p.L.g, f.L.g, c->bc, f.nb[0], f.nb[1], f.blk, f.L.psi64, p.L.psi64,
                         p.L.psi32);
    AMR_HIP(hipGetLastError());
  }
  // loads per level and diagonal checks
  for (int a = 0; a <= A; ++a) {
    AmrLevel &l = c->lv[a];
    AMR_HIP(launch_rhs(l.L, l.tr, nullptr, l.fP, c->iflag, c->st));
    AMR_HIP(launch_check_diag(l.L, c->iflag, c->st));
  }
  AMR_HIP(hipMemcpyAsync(c->host, c->iflag, kIflags * sizeof(int), hipMemcpyDeviceToHost, c->st));
  AMR_HIP(hipStreamSynchronize(c->st));
  int flags = 0, iv[kIflags];
  memcpy(iv, c->host, sizeof(iv));
  flags = iv[0];
  for (int a = 1; a <= A; ++a) {
    c->lv[a].gl.count = iv[12 + a];
    c->lv[a].cl.count = iv[24 + a];
  }
  // The passes over a tiled level run over its column tiles that hold
  // unknowns: the smoother relaxes class-1 nodes only, and the tiles of every
  // active node would cover 2.4x the unknowns of the 64^3 x 3 voids workload
  // against 1.3x (a block's ghost faces lie in the next tile).  The residual
  // (classes 1-3) runs over the same tiles and, node by node, over the ghost
  // nodes they leave out.
  auto list_unknowns = [&](AmrLevel &l, int a, int kz) -> sbm_status {
    l.tl1 = TileList{l.tids1, 0, kz};
    AMR_HIP(launch_active_tiles(l.L, l.cls, l.tflags, l.tids1, c->iflag + 16 + a, c->st, kz, true));
    const OutsidePick outside{l.L.g, tile_geom_of(l.L, kz), l.tflags, l.cls};
    AMR_HIP(launch_listing(l.L.g.nn, outside, l.gcnt, l.goff, l.goids, c->iflag + 20 + a, c->st));
    return SBM_OK;
  };
  auto read_counts = [&]() -> sbm_status {
    AMR_HIP(hipMemcpyAsync(c->host, c->iflag, kIflags * sizeof(int), hipMemcpyDeviceToHost, c->st));
    AMR_HIP(hipStreamSynchronize(c->st));
    memcpy(iv, c->host, sizeof(iv));
    for (int a = 1; a <= A; ++a)
      if (c->lv[a].tiled) {
        c->lv[a].tl1.count = iv[16 + a];
        c->lv[a].go.count = iv[20 + a];
      }
    return SBM_OK;
  };
  bool listed = false;
  for (int a = 1; a <= A; ++a) {
    AmrLevel &l = c->lv[a];
    l.tl1 = TileList{l.tids1, 0, 0};
    l.go = GhostList{l.goids, 0};
    if (!l.tiled) continue;
    AMR_TRY(list_unknowns(l, a, 0));
    listed = true;
  }
  if (listed) AMR_TRY(read_counts());
  // A level whose tiles with unknowns are few for the GPU (a fraction of its
  // default tile count) lists them again in shallower chunks, so that the
  // tiled kernels run about kAmrTiles workgroups: each chunk then re-reads
  // two more planes per kz, but the CUs are no longer half idle.  Every
  // listed tile-plane writes one partial sum of the level's share.
  bool relisted = false;
  for (int a = 1; a <= A; ++a) {
    AmrLevel &l = c->lv[a];
    if (!l.tiled || l.tl1.count == 0) continue;
    const int kz0 = tile_geom_of(l.L).kz;
    const int kz = std::max(kAmrKzMin, std::min(kz0, (int)((int64_t)kz0 * l.tl1.count / kAmrTiles)));
    const TileGeom tn = tile_geom_of(l.L, kz);
    if (kz >= kz0 || (int64_t)tn.ntiles * tn.kz > num_blocks(l.L.g.nn)) continue;
    AMR_TRY(list_unknowns(l, a, kz));
    relisted = true;
  }
  if (relisted) AMR_TRY(read_counts());
  // tiled levels write partial sums for their listed tiles only
  AMR_HIP(launch_fill<double>(c->partials, c->npart, 0.0, c->st));
  if (flags & 1) return amr_fail(SBM_E_NONFINITE, "NaN/Inf in psi");
  if (flags & 2) return amr_fail(SBM_E_DIAG, "a free DOF has no solid cell around it");
  // uniform hierarchy of the base level on the averaged-down psi
  AMR_TRY(sbm_set_problem(c->base, c->lv[0].L.psi64, mat, bc, nullptr));
  // ||lifted load||: composite residual of the prescribed values
  double *x[kMaxAmrLevels], *f[kMaxAmrLevels], *r[kMaxAmrLevels];
  for (int a = 0; a <= A; ++a) {
    AmrLevel &l = c->lv[a];
    AMR_HIP(launch_fill<double>(l.e, l.nv(), 0.0, c->st));
    AMR_HIP(launch_set_dirichlet(l.L, l.e, c->dv, c->st));
    x[a] = l.e;
    f[a] = l.fP;
    r[a] = l.r;
  }
  AMR_TRY(amr_comp_residual(c, x, f, r, true));
  if (!isfinite(c->host[0])) return amr_fail(SBM_E_NONFINITE, "non-finite load");
  c->fnorm = sqrt(c->host[0]);
  // composite DOF count
  for (int a = 0; a <= A; ++a) {
    AmrLevel &l = c->lv[a];
    AMR_HIP(launch_sumsq(l.L, a >= 1 ? l.cls : nullptr, a < A ? &c->lv[a + 1].L : nullptr,
                         a < A ? c->lv[a + 1].cls : nullptr, nullptr, c->partials + l.part_off,
                         c->st, a >= 1 ? l.unknown_tiles() : nullptr));
  }
  AMR_HIP(launch_finalize_sum(c->partials, c->npart, c->scal, c->st));
  AMR_HIP(hipMemcpyAsync(c->host, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->st));
  AMR_HIP(hipStreamSynchronize(c->st));
  c->comp_dof = (int64_t)llround(c->host[0]);
  c->have_problem = true;
  return SBM_OK;
}

#define AMR_NEED(c)                                                              \
  do {                                                                           \
    if (!(c)) return amr_fail(SBM_E_ARG, "ctx is NULL");                          \
    if (!(c)->have_problem) return amr_fail(SBM_E_ARG, "sbm_amr_set_problem first"); \
  } while (0)

sbm_status sbm_amr_level_info(sbm_amr_ctx *c, int level, int64_t *ncell_host,
                              int64_t *nblocks_host, uint8_t *blocks_host, uint8_t *classes,
                              double *psi) {
  AMR_NEED(c);
  if (level < 0 || level > c->A) return amr_fail(SBM_E_ARG, "level out of range");
  AmrLevel &l = c->lv[level];
  if (ncell_host) {
    ncell_host[0] = l.L.g.cx;
    ncell_host[1] = l.L.g.cy;
    ncell_host[2] = c->dim > 2 ? l.L.g.cz : 0;
  }
  if (nblocks_host)
    for (int x = 0; x < 3; ++x) nblocks_host[x] = level >= 1 && x < c->dim ? l.nb[x] : 0;
  if (blocks_host && level >= 1)
    AMR_HIP(hipMemcpyAsync(blocks_host, l.blk, l.nblocks(), hipMemcpyDeviceToHost, c->st));
  if (classes && level >= 1)
    AMR_HIP(hipMemcpyAsync(classes, l.cls, l.L.g.nn, hipMemcpyDeviceToDevice, c->st));
  if (psi) AMR_HIP(hipMemcpyAsync(psi, l.L.psi64, sizeof(double) * l.L.g.nc,
                                  hipMemcpyDeviceToDevice, c->st));
  AMR_HIP(hipStreamSynchronize(c->st));
  return SBM_OK;
}

sbm_status sbm_amr_stats(sbm_amr_ctx *c, int64_t *composite_dof_host, double *fnorm_host) {
  AMR_NEED(c);
  if (composite_dof_host) *composite_dof_host = c->comp_dof;
  if (fnorm_host) *fnorm_host = c->fnorm;
  return SBM_OK;
}

sbm_status sbm_amr_ghost_fill(sbm_amr_ctx *c, int level, const double *xc, double *xf) {
  AMR_NEED(c);
  if (level < 1 || level > c->A) return amr_fail(SBM_E_ARG, "level must be 1..levels-1");
  if (!xc || !xf) return amr_fail(SBM_E_ARG, "NULL argument");
  if (xc == xf) return amr_fail(SBM_E_ARG, "xf must not alias xc");
  AMR_HIP(launch_ghost_list<double>(c->lv[level].L, c->lv[level - 1].L, c->lv[level].gl, xc, xf,
                                    c->st));
  return SBM_OK;
}

sbm_status sbm_amr_residual(sbm_amr_ctx *c, double *const *u, double *const *r,
                            double *norm_host) {
  AMR_NEED(c);
  if (!u) return amr_fail(SBM_E_ARG, "u is NULL");
  double *f[kMaxAmrLevels], *rr[kMaxAmrLevels];
  for (int a = 0; a <= c->A; ++a) {
    if (!u[a]) return amr_fail(SBM_E_ARG, "u of a level is NULL");
    if (r && r[a] == u[a]) return amr_fail(SBM_E_ARG, "r of a level must not alias its u");
    f[a] = c->lv[a].fP;
    rr[a] = (r && r[a]) ? r[a] : c->lv[a].r;
  }
  AMR_TRY(amr_comp_residual(c, u, f, rr, true));
  if (norm_host) *norm_host = sqrt(c->host[0]);
  return SBM_OK;
}

sbm_status sbm_amr_solve(sbm_amr_ctx *c, double *const *u, double *hist_host, int hist_cap,
                         int *n_cycles_host, double *final_rel_host) {
  AMR_NEED(c);
  if (!u) return amr_fail(SBM_E_ARG, "u is NULL");
  const int A = c->A;
  double *f[kMaxAmrLevels], *r[kMaxAmrLevels];
  for (int a = 0; a <= A; ++a) {
    if (!u[a]) return amr_fail(SBM_E_ARG, "u of a level is NULL");
    AMR_HIP(launch_set_dirichlet(c->lv[a].L, u[a], c->dv, c->st));
    f[a] = c->lv[a].fP;
    r[a] = c->lv[a].r;
  }
  AMR_TRY(amr_inject_all(c, u));
  double rho = 0.0, rho_min = INFINITY;
  sbm_status status = SBM_NOT_CONVERGED;
  int m = 0;
  for (m = 0;; ++m) {
    AMR_TRY(amr_comp_residual(c, u, f, r, true));
    const double ss = c->host[0];
    rho = c->fnorm > 0.0 ? sqrt(ss) / c->fnorm : (ss > 0.0 ? INFINITY : 0.0);
    if (hist_host && m < hist_cap) hist_host[m] = rho;
    if (!isfinite(rho)) {
      status = amr_fail(SBM_E_NONFINITE, "non-finite residual at cycle " + std::to_string(m));
      break;
    }
    if (rho <= c->opt.rtol) {
      status = SBM_OK;
      break;
    }
    if (rho > 1e3 * rho_min) {
      status = amr_fail(SBM_E_DIVERGED, "residual grew above 1e3 x its minimum at cycle " +
                                            std::to_string(m));
      break;
    }
    rho_min = std::min(rho_min, rho);
    if (m >= c->opt.max_cycles) {
      set_error(SBM_NOT_CONVERGED, "max_cycles reached");
      status = SBM_NOT_CONVERGED;
      break;
    }
    if (c->opt.precision == 1) {
      // The padded residual rows of the ghost nodes (classes 2 and 3) stay
      // O(1) while the composite residual converges; they reach the cycle
      // only through R at the coarse covered/interface nodes, where they
      // largely cancel.  That restriction is taken here in FP64 (g) and the
      // FP32 loads carry zeros on those rows, so no FP32 sum cancels.
      for (int a = 0; a <= A; ++a) {
        AmrLevel &l = c->lv[a];
        // a tiled level casts over its tiles with unknowns; the ghost nodes
        // outside them get the zero load the cast gives every ghost row
        AMR_HIP(launch_amr_cast(l.L, a >= 1 ? l.cls : nullptr, l.r, l.f32, c->scal, c->st,
                                a >= 1 ? l.unknown_tiles() : nullptr));
        if (a >= 1 && l.tiled) AMR_HIP(launch_ghost_copy<float>(l.L, l.go, nullptr, l.f32, c->st));
        AMR_HIP(amr_zero<float>(c, l, l.e32));
        if (a < A) {
          AMR_HIP(launch_fill<double>(l.w, l.nv(), 0.0, c->st));
          AMR_HIP(launch_restrict_cif<double>(c->lv[a + 1].L, l.L, c->lv[a + 1].cls,
                                              c->lv[a + 1].cl, c->lv[a + 1].r, nullptr, nullptr,
                                              l.w, c->st, true));
          AMR_HIP(launch_cast_scaled(l.w, l.g32, l.nv(), c->scal, c->st));
        }
      }
      AMR_HIP(amr_fas<float>(c, A));
      for (int a = 0; a <= A; ++a)
        AMR_HIP(launch_update<float>(c->lv[a].L, a >= 1 ? c->lv[a].cls : nullptr, u[a],
                                     c->lv[a].e32, c->scal, c->st,
                                     a >= 1 ? c->lv[a].unknown_tiles() : nullptr));
    } else {
      for (int a = 0; a <= A; ++a) AMR_HIP(amr_zero<double>(c, c->lv[a], c->lv[a].e));
      AMR_HIP(amr_fas<double>(c, A));
      for (int a = 0; a <= A; ++a)
        AMR_HIP(launch_update<double>(c->lv[a].L, a >= 1 ? c->lv[a].cls : nullptr, u[a],
                                      c->lv[a].e, nullptr, c->st,
                                      a >= 1 ? c->lv[a].unknown_tiles() : nullptr));
    }
    AMR_TRY(amr_inject_all(c, u));
  }
  for (int a = 1; a <= A; ++a)
    AMR_HIP(launch_ghost_list<double>(c->lv[a].L, c->lv[a - 1].L, c->lv[a].gl, u[a - 1], u[a],
                                      c->st));
  AMR_HIP(hipStreamSynchronize(c->st));
  if (n_cycles_host) *n_cycles_host = m;
  if (final_rel_host) *final_rel_host = rho;
  return status;
}

}  // extern "C"
