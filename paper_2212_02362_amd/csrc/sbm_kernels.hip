// sbm_kernels.hip -- gfx950 kernels of the SBM elasticity multigrid and their
// launchers.  Every kernel is a coalesced sweep over nodes or cells of one
// level (HBM-bound stencils); reductions are deterministic two-pass block
// sums; the bottom solve is a single-workgroup CG.
#include <math.h>

#include "sbm_bottom.h"
#include "sbm_internal.h"

namespace sbm {

int num_blocks(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

// Stencil kernels: workgroup b runs on XCD b mod 8, so the logical block order
// deals each XCD a contiguous range of rows; the neighbouring rows and planes
// a block reads then sit in its own L2.  Grids of 64 or more blocks are
// padded to a multiple of 8 (padding blocks find no node).
int grid_blocks(int64_t n) {
  const int nb = num_blocks(n);
  return nb >= 64 ? (nb + 7) / 8 * 8 : nb;
}

// Threads per block of the V-cycle stencil and transfer kernels on a level
// of n work items: small levels take blocks of 128 (twice as many blocks,
// spread over more CUs; their launches are bound by latency, not bytes).
constexpr int64_t kSmallLevel = 300000;
static int level_block(int64_t n) { return n < kSmallLevel ? 128 : kBlock; }
static int level_grid(int64_t n) {
  const int bs = level_block(n);
  const int nb = (int)((n + bs - 1) / bs);
  return nb >= 64 ? (nb + 7) / 8 * 8 : nb;
}


// ------------------------------------------------------------------ apply --

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_apply(Geom g, Coef<T> C, const T *__restrict__ psi,
                                                  const T *__restrict__ u, T *__restrict__ y) {
  const int64_t id = (int64_t)xcd_block() * kBlock + threadIdx.x;
  if (id >= g.nn) return;
  int i, j, k;
  node_ijk(g, id, i, j, k);
  T out[3], dg[3];
  node_stencil<T, DIM>(g, C, psi, u, i, j, k, out, dg);
#pragma unroll
  for (int c = 0; c < DIM; ++c) y[c * g.nn + id] = out[c];
}

// r = f - K u on free DOF (0 on displacement DOF); optional per-block sums of r^2.
// MASK: a class array is given and only classes 1-3 (interior, interface,
// first outer layer: the padded region of an adaptive level) carry a
// residual; elsewhere r = 0.
template <typename T, int DIM, bool MASK>
__global__ __launch_bounds__(kBlock) void k_residual(Geom g, Coef<T> C, const T *__restrict__ psi,
                                                     const T *__restrict__ u,
                                                     const T *__restrict__ f, T *__restrict__ r,
                                                     double *__restrict__ partials,
                                                     const uint8_t *__restrict__ cls) {
  __shared__ double lds[kBlock / 64 + 1];
  const int64_t id = (int64_t)xcd_block() * (int)blockDim.x + threadIdx.x;
  double ss = 0.0;
  if (id < g.nn && MASK && (cls[id] == 0 || cls[id] > 3)) {
    for (int c = 0; c < DIM; ++c) r[c * g.nn + id] = T(0);
  } else if (id < g.nn) {
    int i, j, k;
    node_ijk(g, id, i, j, k);
    // f is loaded with the stencil's values (one round trip per thread)
    T fv[3], out[3], dg[3];
#pragma unroll
    for (int c = 0; c < DIM; ++c) fv[c] = f[c * g.nn + id];
    node_stencil<T, DIM>(g, C, psi, u, i, j, k, out, dg);
    const uint32_t fb = face_bits(g, i, j, k);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const T v = ((g.dmask >> c) & fb) ? T(0) : fv[c] - out[c];
      if (r) r[c * g.nn + id] = v;
      ss += (double)v * (double)v;
    }
  }
  if (partials) {
    const double s = block_sum(ss, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
}

// Residual norm of u (partials of ||f - K u||^2 over free DOF, as
// k_residual) and, from the same stencil evaluations, the colour-`colour`
// half-sweep of u into u_out (the nodes of the other colour copied): the
// convergence test of one V-cycle and the first smoothing step of the next in
// one pass.  Each relaxed node takes the expression of k_rb_half on the same
// values, so u_out equals that half-sweep.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_residual_sweep(Geom g, Coef<double> C,
                                                           const double *__restrict__ psi,
                                                           const double *__restrict__ u,
                                                           const double *__restrict__ f,
                                                           double *__restrict__ u_out,
                                                           double omega, int colour,
                                                           double *__restrict__ partials) {
  __shared__ double lds[kBlock / 64 + 1];
  const int64_t id = (int64_t)xcd_block() * kBlock + threadIdx.x;
  double ss = 0.0;
  if (id < g.nn) {
    int i, j, k;
    node_ijk(g, id, i, j, k);
    double fv[3], out[3], dg[3], uc[3];
#pragma unroll
    for (int c = 0; c < DIM; ++c) fv[c] = f[c * g.nn + id];
    node_stencil<double, DIM>(g, C, psi, u, i, j, k, out, dg, uc);
    const uint32_t fb = face_bits(g, i, j, k);
    const bool relax = ((i + j + k) & 1) == colour;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const bool dir = ((g.dmask >> c) & fb) != 0u;
      const double v = dir ? 0.0 : fv[c] - out[c];
      ss += v * v;
      const double w = dir ? 0.0 : omega;
      u_out[c * g.nn + id] = relax ? uc[c] + w * (fv[c] - out[c]) / dg[c] : uc[c];
    }
  }
  const double s = block_sum(ss, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// r32 = fp32((f - K u) / s) on free DOF: the scaled residual handed to the
// FP32 cycle of the mixed-precision solve.  s = sqrt(*ss) is the residual
// norm the convergence test just computed (device-resident, so a captured
// cycle needs no host-side argument).
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_residual_cast(Geom g, Coef<double> C,
                                                          const double *__restrict__ psi,
                                                          const double *__restrict__ u,
                                                          const double *__restrict__ f,
                                                          float *__restrict__ r32,
                                                          const double *__restrict__ ss) {
  const int64_t id = (int64_t)xcd_block() * kBlock + threadIdx.x;
  if (id >= g.nn) return;
  const double sn = sqrt(*ss);
  const double inv_s = sn > 0.0 ? 1.0 / sn : 0.0;
  int i, j, k;
  node_ijk(g, id, i, j, k);
  double fv[3], out[3], dg[3];
#pragma unroll
  for (int c = 0; c < DIM; ++c) fv[c] = f[c * g.nn + id];
  node_stencil<double, DIM>(g, C, psi, u, i, j, k, out, dg);
  const uint32_t fb = face_bits(g, i, j, k);
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    const float v = (float)((fv[c] - out[c]) * inv_s);
    r32[c * g.nn + id] = ((g.dmask >> c) & fb) ? 0.0f : v;
  }
}

// ------------------------------------------------------------- smoothers --

// Damped Jacobi (Sec. 2.3): u_out = u + omega D^-1 (f - K u) on free DOF.
// MASK: a class array is given and only class-1 nodes (the unknowns of an
// adaptive level) are relaxed; every other node is copied.
template <typename T, int DIM, bool MASK>
__global__ __launch_bounds__(kBlock) void k_jacobi(Geom g, Coef<T> C, const T *__restrict__ psi,
                                                   const T *__restrict__ u,
                                                   const T *__restrict__ f,
                                                   T *__restrict__ u_out, T omega,
                                                   const uint8_t *__restrict__ cls) {
  const int64_t id = (int64_t)xcd_block() * (int)blockDim.x + threadIdx.x;
  if (id >= g.nn) return;
  if (MASK && cls[id] != 1) {
    for (int c = 0; c < DIM; ++c) u_out[c * g.nn + id] = u[c * g.nn + id];
    return;
  }
  int i, j, k;
  node_ijk(g, id, i, j, k);
  T fv[3], out[3], dg[3], uc[3];
#pragma unroll
  for (int c = 0; c < DIM; ++c) fv[c] = f[c * g.nn + id];
  node_stencil<T, DIM>(g, C, psi, u, i, j, k, out, dg, uc);
  const uint32_t fb = face_bits(g, i, j, k);
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    const T w = ((g.dmask >> c) & fb) ? T(0) : omega;
    u_out[c * g.nn + id] = uc[c] + w * (fv[c] - out[c]) / dg[c];
  }
}

// Colour-synchronous Gauss-Seidel half-sweep: every node of the given colour
// ((x+y+z) mod 2) is relaxed from the state at the start of the half-sweep,
// all components together; nodes of the other colour are copied.  One thread
// owns the x-pair (2p, 2p+1) of a row: one node of each colour.
// MASK: a class array is given and only class-1 nodes are relaxed (adaptive
// levels).
template <typename T, int DIM, bool MASK>
__global__ __launch_bounds__(kBlock) void k_rb_half(Geom g, Coef<T> C, const T *__restrict__ psi,
                                                    const T *__restrict__ u,
                                                    const T *__restrict__ f,
                                                    T *__restrict__ u_out, T omega, int colour,
                                                    const uint8_t *__restrict__ cls) {
  const int npx = (g.nx + 1) >> 1;
  const int64_t tid = (int64_t)xcd_block() * (int)blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)npx * g.ny * g.nz;
  if (tid >= total) return;
  const uint32_t rest = g.fpx.div((uint32_t)tid);
  const int p = (int)((uint32_t)tid - rest * (uint32_t)npx);
  const int k = (int)g.fny.div(rest);
  const int j = (int)(rest - (uint32_t)k * (uint32_t)g.ny);
  const int par = (colour + j + k) & 1;
  const int iu = 2 * p + par, ic = 2 * p + 1 - par;
  const int64_t row = (int64_t)g.nx * (j + (int64_t)g.ny * k);
  // In an odd row the last pair has one node; the missing one is replaced by
  // its partner in every load (in range) and is not stored.
  const bool oku = iu < g.nx, okc = ic < g.nx;
  const int iq = oku ? iu : ic;
  const int64_t qu = row + iq, qc = row + (okc ? ic : iu);
  // f and the copied node are loaded before the stencil so that every load of
  // the thread is in flight together
  T fv[3], cv[3];
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    fv[c] = f[c * g.nn + qu];
    cv[c] = u[c * g.nn + qc];
  }
  T nv[3] = {T(0), T(0), T(0)};
  if (MASK && cls[qu] != 1) {
#pragma unroll
    for (int c = 0; c < DIM; ++c) nv[c] = u[c * g.nn + qu];
  } else {
    T out[3], dg[3], uc[3];
    node_stencil<T, DIM>(g, C, psi, u, iq, j, k, out, dg, uc);
    // a zero weight on displacement DOF keeps the update free of branches
    const uint32_t fb = face_bits(g, iq, j, k);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const T w = ((g.dmask >> c) & fb) ? T(0) : omega;
      nv[c] = uc[c] + w * (fv[c] - out[c]) / dg[c];
    }
  }
  // Both nodes of the pair are stored back to back, so that every written
  // line is complete in L2 when it leaves.  The stores are unconditional (a
  // lone node is written twice with its own value), which keeps the whole
  // computation out of branches.
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    u_out[c * g.nn + qu] = oku ? nv[c] : cv[c];
    u_out[c * g.nn + qc] = okc ? cv[c] : nv[c];
  }
}

// -------------------------------------------------------------- transfers --

// f_coarse(I) = 2^-d sum_n P(n, I) r(n): full weighting [1/2, 1, 1/2] per axis
// around the coincident fine node 2I; fine nodes outside the box are absent.
// The coarse node (I, J, K) with linear index id.
template <typename T, int DIM>
__device__ __forceinline__ void restrict_node(const Geom &gf, const Geom &gc, const T *r, T *fc,
                                              T *ec, int64_t id, int I, int J, int K) {
  // Branch-free gather (all 27 loads in flight together): a neighbour outside
  // the box is read at the centre with weight 0, which adds an exact zero, so
  // the sum equals the one over the neighbours inside, in the same order.
  T acc[3] = {T(0), T(0), T(0)};
  constexpr int ZLO = (DIM == 3) ? -1 : 0, ZHI = (DIM == 3) ? 1 : 0;
#pragma unroll
  for (int dz = ZLO; dz <= ZHI; ++dz) {
    const int fk = 2 * K + dz;
    const bool okz = fk >= 0 && fk < gf.nz;
    const T wz = okz ? (dz == 0 ? T(1) : T(0.5)) : T(0);
    const int fkc = okz ? fk : 2 * K;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int fj = 2 * J + dy;
      const bool oky = fj >= 0 && fj < gf.ny;
      const T wy = oky ? (dy == 0 ? T(1) : T(0.5)) : T(0);
      const int fjc = oky ? fj : 2 * J;
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int fi = 2 * I + dx;
        const bool okx = fi >= 0 && fi < gf.nx;
        const T w = wz * wy * (okx ? (dx == 0 ? T(1) : T(0.5)) : T(0));
        const int64_t q = (okx ? fi : 2 * I) + (int64_t)gf.nx * (fjc + (int64_t)gf.ny * fkc);
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc[c] += w * r[c * gf.nn + q];
      }
    }
  }
  const T scale = (DIM == 3) ? T(0.125) : T(0.25);
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    fc[c * gc.nn + id] = is_dirichlet(gc, I, J, K, c) ? T(0) : acc[c] * scale;
    if (ec) ec[c * gc.nn + id] = T(0);  // the coarse correction starts from zero
  }
}

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_restrict(Geom gf, Geom gc, const T *__restrict__ r,
                                                     T *__restrict__ fc, T *__restrict__ ec) {
  const int64_t id = (int64_t)xcd_block() * (int)blockDim.x + threadIdx.x;
  if (id >= gc.nn) return;
  int I, J, K;
  node_ijk(gc, id, I, J, K);
  restrict_node<T, DIM>(gf, gc, r, fc, ec, id, I, J, K);
}

// Tiled full weighting for 3D levels.  A workgroup owns RCX x RCY coarse node
// columns and a chunk of coarse planes [K0, K1); the fine planes 2 K0 - 1 ..
// 2 K1 - 1 of the (2 RCX + 1) x (2 RCY + 1) fine window under it pass through
// LDS, the next one loaded into registers while the current one is summed.
// LDS rows hold the even local columns first, then the odd ones, so a coarse
// column's centre (odd) and its two x-neighbours (even) are consecutive
// across the threads.  Each coarse node adds its 27 weighted fine values in
// k_restrict's order (z, y, x; a value outside the box is 0), so both give
// the same numbers.  The tiles cover the coarse columns [0, cxn) x [0, cyn);
// the last column / row of a 2^n + 1 coarse level (when cxn or cyn stops one
// short) goes to k_restrict_rest.
constexpr int RCX = 64, RCY = 4, RNT = RCX * RCY;
constexpr int RHE = RCX + 1;                  // even local columns of the 2 RCX + 1 window
constexpr int RROW = 2 * RHE;                 // LDS row (the odd half has one pad entry)
constexpr int RWY = 2 * RCY + 1;              // fine rows of the window
constexpr int RPL = 3 * RWY * RROW;           // LDS entries per fine plane
constexpr int RPT = (RPL + RNT - 1) / RNT;

struct RTile {
  int cxn, cyn, ntx, nty, nzc, ntiles;
};

static RTile restrict_tiles(const Geom &gc) {
  RTile t;
  t.cxn = (gc.nx > RCX && gc.nx % RCX == 1) ? gc.nx - 1 : gc.nx;
  t.cyn = (gc.ny > RCY && gc.ny % RCY == 1) ? gc.ny - 1 : gc.ny;
  t.ntx = (t.cxn + RCX - 1) / RCX;
  t.nty = (t.cyn + RCY - 1) / RCY;
  // about 1024 workgroups (two rounds of two per CU), chunks of 2 or more
  // coarse planes
  const int cols = t.ntx * t.nty;
  int nzc = 1024 / cols;
  nzc = nzc > gc.nz / 2 ? gc.nz / 2 : nzc;
  t.nzc = nzc < 1 ? 1 : nzc;
  t.ntiles = cols * t.nzc;
  return t;
}

template <typename T>
__global__ __launch_bounds__(RNT) void k_restrict_tile(Geom gf, Geom gc, RTile rt,
                                                       const T *__restrict__ r,
                                                       T *__restrict__ fc, T *__restrict__ ec) {
  __shared__ T sw[2][RPT * RNT];  // padded: every thread stores all its slots
  const int n8 = gridDim.x;       // a multiple of 8
  const int b = blockIdx.x;
  const int li = (b & 7) * (n8 >> 3) + (b >> 3);
  if (li >= rt.ntiles) return;
  const int tx = li % rt.ntx, rest = li / rt.ntx;
  const int ty = rest % rt.nty, tz = rest / rt.nty;
  const int I0 = tx * RCX, J0 = ty * RCY;
  const int K0 = tz * gc.nz / rt.nzc, K1 = (tz + 1) * gc.nz / rt.nzc;
  const int t = threadIdx.x;
  const int64_t fnxy = (int64_t)gf.nx * gf.ny;
  // the thread's load slots: offset within a fine plane, or -1 (outside the
  // box, or padding)
  int off[RPT];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int e = t + j * RNT;
    off[j] = -1;
    if (e < RPL) {
      const int c = e / (RWY * RROW), rr = e - c * (RWY * RROW);
      const int y = rr / RROW, s = rr - y * RROW;
      const int lx = s < RHE ? 2 * s : 2 * (s - RHE) + 1;
      const int gx = 2 * I0 - 1 + lx, gy = 2 * J0 - 1 + y;
      if (lx <= 2 * RCX && gx >= 0 && gx < gf.nx && gy >= 0 && gy < gf.ny)
        off[j] = (int)(c * gf.nn + gx + (int64_t)gf.nx * gy);
    }
  }
  auto fetch = [&](int fz, T (&v)[RPT]) __attribute__((always_inline)) {
    const bool zin = fz >= 0 && fz < gf.nz;
    const T *pl = r + (zin ? fz : 0) * fnxy;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const bool ok = zin && off[j] >= 0;
      const T val = pl[ok ? off[j] : 0];
      v[j] = ok ? val : T(0);
    }
  };
  auto put = [&](int buf, const T (&v)[RPT]) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < RPT; ++j) sw[buf][t + j * RNT] = v[j];
  };
  const int cx = t % RCX, cy = t / RCX;
  const int I = I0 + cx, J = J0 + cy;
  const bool own = I < rt.cxn && J < rt.cyn;
  // 2 K + dz, dz = -1, 0, 1, over the chunk's fine planes; a plane past the
  // box reads 0
  const int fz0 = 2 * K0 - 1, fz1 = 2 * K1 - 1;
  T R[RPT];
  fetch(fz0, R);
  put(0, R);
  __syncthreads();
  T acc[3] = {T(0), T(0), T(0)};
  for (int fz = fz0; fz <= fz1; ++fz) {
    const int buf = (fz - fz0) & 1;
    if (fz < fz1) fetch(fz + 1, R);
    const T *W = sw[buf];
    const bool odd = (fz & 1) != 0;
    // the weighted values of this plane for the node (z weight 1/2 on odd
    // planes, 1 on even), in k_restrict's y, x order
    T pv[3][9];
    const T wz = odd ? T(0.5) : T(1);
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const T wy = dy == 0 ? T(1) : T(0.5);
      const int row = (2 * cy + 1 + dy) * RROW;
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const T w = wz * wy * (dx == 0 ? T(1) : T(0.5));
        const int col = dx == 0 ? RHE + cx : cx + (dx > 0 ? 1 : 0);
#pragma unroll
        for (int c = 0; c < 3; ++c) pv[c][(dy + 1) * 3 + dx + 1] = w * W[c * RWY * RROW + row + col];
      }
    }
    // an odd plane 2K + 1 closes coarse plane K (its dz = +1 terms) and opens
    // K + 1 (dz = -1); an even plane 2K is the dz = 0 term of K
    if (odd && fz > fz0) {
      const int K = (fz - 1) / 2;
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int q = 0; q < 9; ++q) acc[c] += pv[c][q];
      if (own) {
        const int64_t id = I + (int64_t)gc.nx * (J + (int64_t)gc.ny * K);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          fc[c * gc.nn + id] = is_dirichlet(gc, I, J, K, c) ? T(0) : acc[c] * T(0.125);
          if (ec) ec[c * gc.nn + id] = T(0);
        }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] = T(0);
    }
    if (fz < fz1 || !odd) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int q = 0; q < 9; ++q) acc[c] += pv[c][q];
    }
    if (fz < fz1) put(buf ^ 1, R);
    __syncthreads();
  }
}

// The coarse nodes the tiles leave (column cxn and row cyn of a 2^n + 1
// coarse level), node-parallel as k_restrict.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict_rest(Geom gf, Geom gc, RTile rt,
                                                          const T *__restrict__ r,
                                                          T *__restrict__ fc, T *__restrict__ ec,
                                                          int n) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  const int ncol = gc.nx - rt.cxn;                      // 0 or 1 columns (all rows)
  const int per = ncol * gc.ny + (gc.ny - rt.cyn) * rt.cxn;  // nodes per coarse plane
  const int K = e / per;
  const int q = e - K * per;
  int I, J;
  if (q < ncol * gc.ny) {
    I = rt.cxn;
    J = q;
  } else {
    I = q - ncol * gc.ny;
    J = rt.cyn;
  }
  const int64_t id = I + (int64_t)gc.nx * (J + (int64_t)gc.ny * K);
  restrict_node<T, 3>(gf, gc, r, fc, ec, id, I, J, K);
}

// u_fine += P e_coarse (multilinear, node-centred) on free fine DOF.  One
// thread per coarse node I owns the 2^d fine nodes 2I + delta (delta in
// {0,1}^d): fine node 2I + delta takes the mean of the coarse corners
// I + delta' with delta' <= delta, summed in z, y, x order (x fastest).
// Loads are clamped at the last coarse / fine node; a fine node that does not
// exist (2I + 1 past the end) is the clamped one and receives that node's own
// value, so every store is unconditional and every load is in flight at once.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_prolong_add(Geom gf, Geom gc, const T *__restrict__ e,
                                                        T *__restrict__ u) {
  constexpr int NZ = (DIM == 3) ? 2 : 1;
  const int64_t id = (int64_t)xcd_block() * (int)blockDim.x + threadIdx.x;
  if (id >= gc.nn) return;
  int I, J, K;
  node_ijk(gc, id, I, J, K);
  const int I1 = min(I + 1, gc.nx - 1), J1 = min(J + 1, gc.ny - 1);
  const int K1 = (DIM == 3) ? min(K + 1, gc.nz - 1) : K;
  T ev[NZ][2][2][3], uv[NZ][2][2][3];
  int64_t fq[NZ][2][2];
  // the odd fine node of an axis exists unless 2I + 1 is past the end
  const bool ex = 2 * I + 1 < gf.nx, ey = 2 * J + 1 < gf.ny, ez = DIM == 3 && 2 * K + 1 < gf.nz;
#pragma unroll
  for (int b = 0; b < NZ; ++b)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int o = 0; o < 2; ++o) {
        const int64_t q = (o ? I1 : I) + (int64_t)gc.nx * ((a ? J1 : J) + (int64_t)gc.ny * (b ? K1 : K));
        const int fi = 2 * I + (o && ex ? 1 : 0), fj = 2 * J + (a && ey ? 1 : 0);
        const int fk = (DIM == 3) ? 2 * K + (b && ez ? 1 : 0) : 0;
        fq[b][a][o] = fi + (int64_t)gf.nx * (fj + (int64_t)gf.ny * fk);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
          ev[b][a][o][c] = e[c * gc.nn + q];
          uv[b][a][o][c] = u[c * gf.nn + fq[b][a][o]];
        }
      }
#pragma unroll
  for (int dz = 0; dz < NZ; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        // a missing odd node stands in for its even neighbour (same address)
        const int sx = (dx && ex) ? 1 : 0, sy = (dy && ey) ? 1 : 0, sz = (dz && ez) ? 1 : 0;
        const T w = T(1) / T((dx ? 2 : 1) * (dy ? 2 : 1) * (dz ? 2 : 1));
        T acc[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int b = 0; b <= dz; ++b)
#pragma unroll
          for (int a = 0; a <= dy; ++a)
#pragma unroll
            for (int o = 0; o <= dx; ++o)
#pragma unroll
              for (int c = 0; c < DIM; ++c) acc[c] += ev[b][a][o][c];
        const uint32_t fb = face_bits(gf, 2 * I + sx, 2 * J + sy, 2 * K + sz);
        // value of the node actually addressed: the stand-in's own if missing
        const bool own = sx == dx && sy == dy && sz == dz;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
          const T add = ((gf.dmask >> c) & fb) ? T(0) : w * acc[c];
          const T nv = uv[dz][dy][dx][c] + add;
          if (own) u[c * gf.nn + fq[dz][dy][dx]] = nv;
        }
      }
}

// ----------------------------------------------------------------- vectors --

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T *__restrict__ p, int64_t n, T v) {
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * kBlock)
    p[q] = v;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy(const T *__restrict__ s, T *__restrict__ d,
                                                 int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * kBlock)
    d[q] = s[q];
}

template <typename S, typename D>
__global__ __launch_bounds__(kBlock) void k_convert(const S *__restrict__ s, D *__restrict__ d,
                                                    int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * kBlock)
    d[q] = (D)s[q];
}

// u += s * e32 on free DOF (FP64 correction of the mixed cycle), s = sqrt(*ss).
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_correct(Geom g, double *__restrict__ u,
                                                    const float *__restrict__ e32,
                                                    const double *__restrict__ ss) {
  const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (id >= g.nn) return;
  const double s = sqrt(*ss);
  int i, j, k;
  node_ijk(g, id, i, j, k);
#pragma unroll
  for (int c = 0; c < DIM; ++c)
    if (!is_dirichlet(g, i, j, k, c)) u[c * g.nn + id] += s * (double)e32[c * g.nn + id];
}

// Displacement DOF take the value of the last fixing face (x-,x+,y-,y+,z-,z+).
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_set_dirichlet(Geom g, double *__restrict__ u,
                                                          DispValues dv) {
  const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (id >= g.nn) return;
  int i, j, k;
  node_ijk(g, id, i, j, k);
  const int at[6] = {i == 0, i == g.nx - 1, j == 0, j == g.ny - 1,
                     DIM == 3 && k == 0, DIM == 3 && k == g.nz - 1};
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    bool set = false;
    double v = 0.0;
#pragma unroll
    for (int F = 0; F < 2 * DIM; ++F)
      if (at[F] && ((g.dmask >> (3 * F + c)) & 1u)) {
        set = true;
        v = dv.v[F][c];
      }
    if (set) u[c * g.nn + id] = v;
  }
}

// ------------------------------------------------------------------- setup --

// psi = max(raw, floor) (raw = rho^3 when cube is set), plus its FP32 copy.
// raw may alias p64.
__global__ __launch_bounds__(kBlock) void k_floor_psi(const double *raw, double fl, double *p64,
                                                      float *__restrict__ p32, int64_t n,
                                                      int cube, int *flag) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= n) return;
  double v = raw[q];
  if (cube) v = v * v * v;
  if (!isfinite(v)) atomicOr(flag, 1);
  const double p = v > fl ? v : fl;
  p64[q] = p;
  p32[q] = (float)p;
}

// Coarse psi = mean of the 2^d child cells (FP64), plus its FP32 copy.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_coarsen_psi(Geom gf, Geom gc,
                                                        const double *__restrict__ pf,
                                                        double *__restrict__ pc,
                                                        float *__restrict__ pc32) {
  const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (id >= gc.nc) return;
  int I, J, K;
  cell_ijk(gc, id, I, J, K);
  double s = 0.0;
  for (int o = 0; o < (1 << DIM); ++o) {
    const int fi = 2 * I + (o & 1), fj = 2 * J + ((o >> 1) & 1);
    const int fk = (DIM == 3) ? 2 * K + ((o >> 2) & 1) : 0;
    s += pf[fi + (int64_t)gf.cx * (fj + (int64_t)gf.cy * fk)];
  }
  const double m = s / (double)(1 << DIM);
  pc[id] = m;
  pc32[id] = (float)m;
}

// Load: f = b + sum over traction faces F containing the node of
// (t_F / h_perp) * (mean of the 2^(d-1) cells that contain the node and touch
// F); 0 on displacement DOF.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_rhs(Geom g, Traction tr, const double *__restrict__ psi,
                                                const double *__restrict__ b,
                                                double *__restrict__ fA, int *flag) {
  const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (id >= g.nn) return;
  int n[3];
  node_ijk(g, id, n[0], n[1], n[2]);
  const int nn_[3] = {g.nx, g.ny, g.nz};
  const int nc_[3] = {g.cx, g.cy, g.cz};
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    const int64_t q = c * g.nn + id;
    if (is_dirichlet(g, n[0], n[1], n[2], c)) {
      fA[q] = 0.0;
      continue;
    }
    double f = 0.0;
    if (b) {
      f = b[q];
      if (!isfinite(f)) atomicOr(flag, 1);
    }
    for (int a = 0; a < DIM; ++a)
      for (int side = 0; side < 2; ++side) {
        const int F = 2 * a + side;
        const double t = tr.t[F][c];
        if (t == 0.0) continue;
        if (n[a] != (side ? nn_[a] - 1 : 0)) continue;
        // the other axes' cells around the node
        const int o1 = (a == 0) ? 1 : 0;
        const int o2 = (a == 2) ? 1 : 2;
        const int ca = side ? nc_[a] - 1 : 0;
        double s = 0.0;
        const int nb = (DIM == 3) ? 4 : 2;
        for (int o = 0; o < nb; ++o) {
          int cc[3];
          cc[a] = ca;
          cc[o1] = n[o1] - 1 + (o & 1);
          if (DIM == 3) cc[o2] = n[o2] - 1 + ((o >> 1) & 1);
          else cc[2] = 0;
          bool in = cc[o1] >= 0 && cc[o1] < nc_[o1];
          if (DIM == 3) in = in && cc[o2] >= 0 && cc[o2] < nc_[o2];
          if (in) s += psi[cc[0] + (int64_t)g.cx * (cc[1] + (int64_t)g.cy * cc[2])];
        }
        f += t * tr.inv_h[F] * (s / nb);
      }
    fA[q] = f;
  }
}

// Flags a free DOF whose diagonal vanishes (no solid cell around it).
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_check_diag(Geom g, const double *__restrict__ psi,
                                                       int *flag) {
  const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (id >= g.nn) return;
  int i, j, k;
  node_ijk(g, id, i, j, k);
  double s = 0.0;
  for (int o = 0; o < (1 << DIM); ++o) {
    const int xi = i - 1 + (o & 1), yj = j - 1 + ((o >> 1) & 1);
    const int zk = (DIM == 3) ? k - 1 + ((o >> 2) & 1) : 0;
    const bool in = xi >= 0 && xi < g.cx && yj >= 0 && yj < g.cy && zk >= 0 && zk < g.cz;
    if (in) s += psi[xi + (int64_t)g.cx * (yj + (int64_t)g.cy * zk)];
  }
  if (s > 0.0) return;
  for (int c = 0; c < DIM; ++c)
    if (!is_dirichlet(g, i, j, k, c)) atomicOr(flag, 2);
}

// ------------------------------------------------------------ reductions --

// Deterministic sum of n partials by one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_finalize_sum(const double *__restrict__ partials, int n,
                                                       double *__restrict__ out) {
  __shared__ double lds[1024 / 64 + 1];
  double s = 0.0;
  int q = threadIdx.x;
  // eight loads in flight per thread; the additions keep the order q, q +
  // 1024, q + 2048, ... (the result does not depend on the unrolling)
  for (; q + 7 * 1024 < n; q += 8 * 1024) {
    double v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = partials[q + t * 1024];
#pragma unroll
    for (int t = 0; t < 8; ++t) s += v[t];
  }
  for (; q < n; q += 1024) s += partials[q];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += lds[w];
    *out = t;
  }
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_sumsq_free(Geom g, const double *__restrict__ v,
                                                       double *__restrict__ partials) {
  __shared__ double lds[kBlock / 64 + 1];
  const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double ss = 0.0;
  if (id < g.nn) {
    int i, j, k;
    node_ijk(g, id, i, j, k);
#pragma unroll
    for (int c = 0; c < DIM; ++c)
      if (!is_dirichlet(g, i, j, k, c)) {
        const double x = v[c * g.nn + id];
        ss += x * x;
      }
  }
  const double s = block_sum(ss, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// An entry of a Krylov vector given in memory or as s * e (s = sc here).
__device__ __forceinline__ double zload(const ZSrc &zs, double sc, int64_t q) {
  return zs.z ? zs.z[q] : sc * (double)zs.e[q];
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_dot_free(Geom g, const double *__restrict__ a,
                                                     ZSrc b, double *__restrict__ partials) {
  __shared__ double lds[kBlock / 64 + 1];
  const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double ss = 0.0;
  if (id < g.nn) {
    int i, j, k;
    node_ijk(g, id, i, j, k);
    // all loads first (one memory round trip), displacement DOF masked after
    const double sb = b.z ? 0.0 : *b.s;
    double av[3], bv[3];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      av[c] = a[c * g.nn + id];
      bv[c] = zload(b, sb, c * g.nn + id);
    }
    const uint32_t fb = face_bits(g, i, j, k);
#pragma unroll
    for (int c = 0; c < DIM; ++c)
      if (!((g.dmask >> c) & fb)) ss += av[c] * bv[c];
  }
  const double s = block_sum(ss, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// ------------------------------------------------------------- Krylov ops --
// Vectors of the flexible CG on the finest level; every reduction writes one
// deterministic partial per block.

// q = K p on free DOF (0 on displacement DOF); partials of p.q.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_apply_dot(Geom g, Coef<double> C,
                                                      const double *__restrict__ psi,
                                                      const double *__restrict__ p,
                                                      double *__restrict__ q,
                                                      double *__restrict__ partials) {
  __shared__ double lds[kBlock / 64 + 1];
  const int64_t id = (int64_t)xcd_block() * kBlock + threadIdx.x;
  double ss = 0.0;
  if (id < g.nn) {
    int i, j, k;
    node_ijk(g, id, i, j, k);
    double out[3], dg[3], pc[3];
    node_stencil<double, DIM>(g, C, psi, p, i, j, k, out, dg, pc);
    const uint32_t fb = face_bits(g, i, j, k);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const double v = ((g.dmask >> c) & fb) ? 0.0 : out[c];
      q[c * g.nn + id] = v;
      ss += pc[c] * v;
    }
  }
  const double s = block_sum(ss, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// The CG update without the iterate: alpha = rz / pq (also stored to
// *alpha_out by the first thread), r -= alpha q on free DOF, partials of r.r
// (pr) and r.z (pz, z = the previous preconditioned residual).  The update
// x += alpha p is left to the next direction update (k_xpby_x) or to
// k_axpy_free: the same products, one vector pass fewer.  With r32 the new
// residual is also cast for the mixed preconditioner: r32 = fp32(r / s) with
// s = sqrt(*ss) (0 on displacement DOF), as k_cast_scaled forms it.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_cg_update_r(Geom g, double *__restrict__ r,
                                                        const double *__restrict__ q, ZSrc z,
                                                        const double *__restrict__ rz,
                                                        const double *__restrict__ pq,
                                                        double *__restrict__ alpha_out,
                                                        double *__restrict__ pr,
                                                        double *__restrict__ pz,
                                                        float *__restrict__ r32,
                                                        const double *__restrict__ ss) {
  __shared__ double lds[kBlock / 64 + 1];
  const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const double alpha = *rz / *pq;
  if (blockIdx.x == 0 && threadIdx.x == 0) *alpha_out = alpha;
  double srr = 0.0, srz = 0.0;
  if (id < g.nn) {
    int i, j, k;
    node_ijk(g, id, i, j, k);
    const double sz = z.z ? 0.0 : *z.s;
    double rv[3], qv[3], zv[3];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const int64_t qi = c * g.nn + id;
      rv[c] = r[qi];
      qv[c] = q[qi];
      zv[c] = zload(z, sz, qi);
    }
    const uint32_t fb = face_bits(g, i, j, k);
    const double sn = r32 ? sqrt(*ss) : 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      if ((g.dmask >> c) & fb) {
        if (r32) r32[c * g.nn + id] = 0.0f;
        continue;
      }
      const double rn = rv[c] - alpha * qv[c];
      r[c * g.nn + id] = rn;
      if (r32) r32[c * g.nn + id] = sn > 0.0 ? (float)(rn / sn) : 0.0f;
      srr += rn * rn;
      srz += rn * zv[c];
    }
  }
  const double a = block_sum(srr, lds);
  __syncthreads();
  const double b = block_sum(srz, lds);
  if (threadIdx.x == 0) {
    pr[blockIdx.x] = a;
    pz[blockIdx.x] = b;
  }
}

// The deferred iterate update and the new direction in one pass: on free DOF
// x += (*alpha) p (when alpha is given), then p = z + beta p, beta = (rznew -
// rzold) / rz (beta = 0 when rz is NULL: restart); p = 0 on displacement DOF.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_xpby_x(Geom g, double *__restrict__ x,
                                                   double *__restrict__ p, ZSrc z,
                                                   const double *__restrict__ rznew,
                                                   const double *__restrict__ rzold,
                                                   const double *__restrict__ rz,
                                                   const double *__restrict__ alpha) {
  const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (id >= g.nn) return;
  const double beta = rz ? (*rznew - *rzold) / *rz : 0.0;
  const double al = alpha ? *alpha : 0.0;
  int i, j, k;
  node_ijk(g, id, i, j, k);
  const double sz = z.z ? 0.0 : *z.s;
  double zv[3], pv[3], xv[3];
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    zv[c] = zload(z, sz, c * g.nn + id);
    pv[c] = p[c * g.nn + id];
    xv[c] = alpha ? x[c * g.nn + id] : 0.0;
  }
  const uint32_t fb = face_bits(g, i, j, k);
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    const bool fixed = (g.dmask >> c) & fb;
    if (alpha && !fixed) x[c * g.nn + id] = xv[c] + al * pv[c];
    p[c * g.nn + id] = fixed ? 0.0 : zv[c] + (rz ? beta * pv[c] : 0.0);
  }
}

// x += (*alpha) p on free DOF (the deferred CG update, when the iteration ends).
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_axpy_free(Geom g, double *__restrict__ x,
                                                      const double *__restrict__ p,
                                                      const double *__restrict__ alpha) {
  const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (id >= g.nn) return;
  const double al = *alpha;
  int i, j, k;
  node_ijk(g, id, i, j, k);
  const uint32_t fb = face_bits(g, i, j, k);
#pragma unroll
  for (int c = 0; c < DIM; ++c)
    if (!((g.dmask >> c) & fb)) x[c * g.nn + id] += al * p[c * g.nn + id];
}

// r32 = fp32(r / s) (s = sqrt(*ss)): the FP32 preconditioner of the mixed
// flexible CG sees a unit-norm residual; its output e32 is used as s * e32
// (ZSrc) without being written out in FP64.
__global__ __launch_bounds__(kBlock) void k_cast_scaled(const double *__restrict__ r,
                                                        float *__restrict__ r32, int64_t n,
                                                        const double *__restrict__ ss) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= n) return;
  const double sn = sqrt(*ss);
  r32[q] = sn > 0.0 ? (float)(r[q] / sn) : 0.0f;
}

// r32 = fp32(r / s) as k_residual_cast forms it (times the reciprocal of
// s = sqrt(*ss)), for a residual r already in memory.
__global__ __launch_bounds__(kBlock) void k_scale_cast(const double *__restrict__ r,
                                                       float *__restrict__ r32, int64_t n,
                                                       const double *__restrict__ ss) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= n) return;
  const double sn = sqrt(*ss);
  const double inv_s = sn > 0.0 ? 1.0 / sn : 0.0;
  r32[q] = (float)(r[q] * inv_s);
}

// As k_scale_cast, and the first colour-`colour` half-sweep of the FP32
// correction cycle from e = 0 written into t32 (relaxed nodes omega r32 / D
// with D the FP32 diagonal, the others 0): the FP32 V-cycle then starts at its
// second half-sweep.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_scale_cast_sweep(Geom g, Coef<float> C,
                                                             const float *__restrict__ psi,
                                                             const double *__restrict__ r,
                                                             float *__restrict__ r32,
                                                             float *__restrict__ t32,
                                                             float omega, int colour,
                                                             const double *__restrict__ ss) {
  const int64_t id = (int64_t)xcd_block() * kBlock + threadIdx.x;
  if (id >= g.nn) return;
  int i, j, k;
  node_ijk(g, id, i, j, k);
  const double sn = sqrt(*ss);
  const double inv_s = sn > 0.0 ? 1.0 / sn : 0.0;
  float dg[3];
  node_diag<float, DIM>(g, C, psi, i, j, k, dg);
  const uint32_t fb = face_bits(g, i, j, k);
  const bool relax = ((i + j + k) & 1) == colour;
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    const float v = (float)(r[c * g.nn + id] * inv_s);
    r32[c * g.nn + id] = v;
    const float w = ((g.dmask >> c) & fb) ? 0.0f : omega;
    t32[c * g.nn + id] = relax ? 0.0f + w * (v - 0.0f) / dg[c] : 0.0f;
  }
}

__global__ void k_store_sqrt(const double *__restrict__ ss, double *__restrict__ s_out) {
  if (threadIdx.x == 0) *s_out = sqrt(*ss);
}

// ----------------------------------------------------------------- bottom --

constexpr int kBottomThreads = 256;  // keeps the per-thread state of the global-memory CG in registers

// Jacobi-preconditioned CG on the free DOF, one workgroup, vectors in global
// memory (the variant for bottom grids too large for LDS).  On entry r holds
// the initial residual (0 on displacement DOF) and x the initial iterate;
// stops when ||r|| <= rtol ||r0||; returns the iterations.  Dot products are
// accumulated in FP64 whatever T is.
template <typename T, int DIM>
__device__ int cg_core(const Geom &g, const Coef<T> &C, const T *__restrict__ psi, T *x, T *r,
                       T *p, T *Ap, double rtol, int maxit, double *lds) {
  const int64_t n = g.nn;
  double lrr = 0.0, lrz = 0.0;
  for (int64_t id = threadIdx.x; id < n; id += blockDim.x) {
    int i, j, k;
    node_ijk(g, id, i, j, k);
    T dg[3];
    node_diag<T, DIM>(g, C, psi, i, j, k, dg);
    for (int c = 0; c < DIM; ++c) {
      const T v = r[c * n + id];
      const T z = is_dirichlet(g, i, j, k, c) ? T(0) : v / dg[c];
      p[c * n + id] = z;
      lrr += (double)v * (double)v;
      lrz += (double)v * (double)z;
    }
  }
  double rr = block_allsum(lrr, lds);
  double rz = block_allsum(lrz, lds);
  const double r0 = sqrt(rr);
  int it = 0;
  while (r0 > 0.0 && sqrt(rr) > rtol * r0 && it < maxit) {
    __syncthreads();
    double pap = 0.0;
    for (int64_t id = threadIdx.x; id < n; id += blockDim.x) {
      int i, j, k;
      node_ijk(g, id, i, j, k);
      T out[3], dg[3];
      node_stencil<T, DIM>(g, C, psi, p, i, j, k, out, dg);
      for (int c = 0; c < DIM; ++c) {
        const T a = is_dirichlet(g, i, j, k, c) ? T(0) : out[c];
        Ap[c * n + id] = a;
        pap += (double)p[c * n + id] * (double)a;
      }
    }
    pap = block_allsum(pap, lds);
    if (!(pap > 0.0)) break;
    const double alpha = rz / pap;
    double nrr = 0.0, nrz = 0.0;
    for (int64_t id = threadIdx.x; id < n; id += blockDim.x) {
      int i, j, k;
      node_ijk(g, id, i, j, k);
      T dg[3];
      node_diag<T, DIM>(g, C, psi, i, j, k, dg);
      for (int c = 0; c < DIM; ++c) {
        if (is_dirichlet(g, i, j, k, c)) continue;
        const int64_t q = c * n + id;
        x[q] = (T)((double)x[q] + alpha * (double)p[q]);
        const T rv = (T)((double)r[q] - alpha * (double)Ap[q]);
        r[q] = rv;
        nrr += (double)rv * (double)rv;
        nrz += (double)rv * ((double)rv / (double)dg[c]);
      }
    }
    nrr = block_allsum(nrr, lds);
    nrz = block_allsum(nrz, lds);
    const double beta = nrz / rz;
    rr = nrr;
    rz = nrz;
    __syncthreads();
    for (int64_t id = threadIdx.x; id < n; id += blockDim.x) {
      int i, j, k;
      node_ijk(g, id, i, j, k);
      T dg[3];
      node_diag<T, DIM>(g, C, psi, i, j, k, dg);
      for (int c = 0; c < DIM; ++c) {
        const int64_t q = c * n + id;
        p[q] = is_dirichlet(g, i, j, k, c)
                   ? T(0)
                   : (T)((double)r[q] / (double)dg[c] + beta * (double)p[q]);
      }
    }
    ++it;
  }
  __syncthreads();
  return it;
}

template <typename T, int DIM>
__global__ __launch_bounds__(kBottomThreads) void k_bottom_cg(Geom g, Coef<T> C,
                                                              const T *__restrict__ psi,
                                                              const T *__restrict__ f, T *x, T *r,
                                                              T *p, T *Ap, double rtol, int maxit,
                                                              int *iters) {
  __shared__ double lds[kBottomThreads / 64 + 1];
  const int64_t n = g.nn;
  for (int64_t id = threadIdx.x; id < n; id += blockDim.x) {
    int i, j, k;
    node_ijk(g, id, i, j, k);
    T out[3], dg[3];
    node_stencil<T, DIM>(g, C, psi, x, i, j, k, out, dg);
    for (int c = 0; c < DIM; ++c) {
      const int64_t q = c * n + id;
      r[q] = is_dirichlet(g, i, j, k, c) ? T(0) : f[q] - out[c];
    }
  }
  __syncthreads();
  const int it = cg_core<T, DIM>(g, C, psi, x, r, p, Ap, rtol, maxit, lds);
  if (threadIdx.x == 0 && iters) *iters = it;
}


// ---------------------------------------------------- LDS-resident bottom --
// (CG core and reductions in sbm_bottom.h)

// FP64 bottom: x += CG solution of K_FF d = (f - K x)_F.  f and x are FP64,
// or FP32 in the mixed cycle (read into and written from the FP64 solve).
template <int DIM, int Q, typename IO>
__global__ __launch_bounds__(kBotThreads) void k_bottom_lds64(Geom g, Coef<double> C,
                                                       const double *__restrict__ psi,
                                                       const IO *__restrict__ f, IO *x,
                                                       double rtol, int maxit, int *iters) {
  extern __shared__ double smem[];
  __shared__ double red[64];
  BotRed R{red, 0};
  const int64_t n = g.nn;
  double *psi_l = smem;
  double *p_l = smem + ((g.nc + 1) & ~(int64_t)1);
  for (int64_t q = threadIdx.x; q < g.nc; q += blockDim.x) psi_l[q] = psi[q];
  bool dir[Q][3];
  int cijk[Q][3];
  double r[Q][3], dd[Q][3], xv[Q][3];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t id = threadIdx.x + (int64_t)q * blockDim.x;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      dir[q][c] = true;
      r[q][c] = dd[q][c] = xv[q][c] = 0.0;
      cijk[q][c] = 0;
    }
    if (id >= n) continue;
    node_ijk(g, id, cijk[q][0], cijk[q][1], cijk[q][2]);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      dir[q][c] = is_dirichlet(g, cijk[q][0], cijk[q][1], cijk[q][2], c);
      xv[q][c] = (double)x[c * n + id];
      p_l[c * n + id] = xv[q][c];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t id = threadIdx.x + (int64_t)q * blockDim.x;
    if (id >= n) continue;
    double out[3], dg[3];
    node_stencil<double, DIM>(g, C, psi_l, p_l, cijk[q][0], cijk[q][1], cijk[q][2], out, dg);
#pragma unroll
    for (int c = 0; c < DIM; ++c) r[q][c] = dir[q][c] ? 0.0 : (double)f[c * n + id] - out[c];
  }
  __syncthreads();
  const int it = bot_cg<double, DIM, Q>(g, C, psi_l, p_l, r, dd, dir, cijk, rtol, maxit, R);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t id = threadIdx.x + (int64_t)q * blockDim.x;
    if (id >= n) continue;
#pragma unroll
    for (int c = 0; c < DIM; ++c)
      if (!dir[q][c]) x[c * n + id] = (IO)(xv[q][c] + dd[q][c]);
  }
  if (threadIdx.x == 0 && iters) *iters = it;
}


// ------------------------------------------------------------ sensitivity --

// g_c = -lam_c^T K_c u_c + lam^T df/dpsi_c per cell, with K_c in energy form:
//   edges (1/2^(d-1) each): sum_i a_ij / h_j^2 (d lam_i)(d u_i), a_ij = mu + (lam+mu) delta_ij
//   faces of the cell (3D: 1/2 each; 2D: the cell itself), plane (a, b):
//     lame (da lam_a db u_b + db lam_b da u_a) + mu (db lam_a da u_b + da lam_b db u_a)
//   with face-centre derivatives averaged over the face's two edges.
// lam enters scaled by lam_scale.  chain 1: g masked where the raw psi
// (design) is at or below the floor; chain 2: dL/drho = 3 rho^2 g where
// rho^3 > floor, else 0 (design = rho).
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_sensitivity(Geom g, double lame, double mu,
                                                        double h0, double h1, double h2,
                                                        Traction tr, const double *__restrict__ u,
                                                        const double *__restrict__ adj,
                                                        double lam_scale,
                                                        const double *__restrict__ design,
                                                        int chain, double fl,
                                                        double *__restrict__ out) {
  const int64_t id = (int64_t)xcd_block() * kBlock + threadIdx.x;
  if (id >= g.nc) return;
  int ci, cj, ck;
  cell_ijk(g, id, ci, cj, ck);
  constexpr int NCO = 1 << DIM;
  double U[3][NCO], A[3][NCO];
#pragma unroll
  for (int o = 0; o < NCO; ++o) {
    const int64_t node = (ci + (o & 1)) + (int64_t)g.nx * ((cj + ((o >> 1) & 1)) +
                                                            (int64_t)g.ny * (ck + ((o >> 2) & 1)));
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      U[c][o] = u[c * g.nn + node];
      A[c][o] = adj[c * g.nn + node];
    }
  }
  const double h[3] = {h0, h1, h2};
  const double we = 1.0 / (double)(1 << (DIM - 1));
  double acc = 0.0;
  // direct (edge) part
#pragma unroll
  for (int jx = 0; jx < DIM; ++jx) {
    const double ih2 = 1.0 / (h[jx] * h[jx]);
#pragma unroll
    for (int o = 0; o < NCO; ++o) {
      if ((o >> jx) & 1) continue;
      const int o2 = o | (1 << jx);
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        const double a = mu + (lame + mu) * (c == jx ? 1.0 : 0.0);
        acc += we * a * ih2 * (A[c][o2] - A[c][o]) * (U[c][o2] - U[c][o]);
      }
    }
  }
  // cross (face) part
  const double wf = (DIM == 3) ? 0.5 : 1.0;
  const int nfaces = (DIM == 3) ? 6 : 1;
#pragma unroll
  for (int fidx = 0; fidx < nfaces; ++fidx) {
    int a, b, m = -1, sm = 0;
    if (DIM == 3) {
      m = fidx >> 1;
      sm = fidx & 1;
      a = (m == 0) ? 1 : 0;
      b = (m == 2) ? 1 : 2;
    } else {
      a = 0;
      b = 1;
    }
    // corner index of face point (alpha, beta)
    auto cidx = [&](int al, int be) {
      int o = (al << a) | (be << b);
      if (m >= 0) o |= (sm << m);
      return o;
    };
    const int o00 = cidx(0, 0), o10 = cidx(1, 0), o01 = cidx(0, 1), o11 = cidx(1, 1);
    auto da = [&](const double (*V)[NCO], int c) {
      return ((V[c][o10] - V[c][o00]) + (V[c][o11] - V[c][o01])) / (2.0 * h[a]);
    };
    auto db = [&](const double (*V)[NCO], int c) {
      return ((V[c][o01] - V[c][o00]) + (V[c][o11] - V[c][o10])) / (2.0 * h[b]);
    };
    const double e = lame * (da(A, a) * db(U, b) + db(A, b) * da(U, a)) +
                     mu * (db(A, a) * da(U, b) + da(A, b) * db(U, a));
    acc += wf * e;
  }
  double gval = -acc;
  // traction source: df_n/dpsi_c = t / h_perp / 2^(d-1) on the corners n of c
  // lying on a traction face that c touches
  const int cc[3] = {ci, cj, ck};
  const int ncx[3] = {g.cx, g.cy, g.cz};
#pragma unroll
  for (int ax = 0; ax < DIM; ++ax)
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      if (cc[ax] != (side ? ncx[ax] - 1 : 0)) continue;
      const int F = 2 * ax + side;
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        const double t = tr.t[F][c];
        if (t == 0.0) continue;
        double s = 0.0;
#pragma unroll
        for (int o = 0; o < NCO; ++o)
          if (((o >> ax) & 1) == side) s += A[c][o];
        gval += s * t * tr.inv_h[F] * we;
      }
    }
  gval *= lam_scale;
  if (chain == 1) {
    gval = design[id] > fl ? gval : 0.0;
  } else if (chain == 2) {
    const double rv = design[id];
    gval = (rv * rv * rv > fl) ? 3.0 * rv * rv * gval : 0.0;
  }
  out[id] = gval;
}

// ---------------------------------------------------------------- launchers --

// The runtime's last-error slot is shared with every other HIP user of the
// thread; it is cleared before the launch so that the status returned is the
// launch's own.
#define SBM_LAUNCH(kern, grid, block, st, ...)                             \
  do {                                                                     \
    (void)hipGetLastError();                                               \
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, st, __VA_ARGS__); \
    return hipGetLastError();                                              \
  } while (0)

// The tiled stencil kernels write one partial sum per tile; they are used
// where they pay and where their partials fit the per-node-block count.
static bool use_tiled(const Level &L) {
  return tiled_ok(L) && tiled_partials(L) <= num_blocks(L.g.nn);
}

int stencil_partials(const Level &L) {
  return use_tiled(L) ? tiled_partials(L) : grid_blocks(L.g.nn);
}

static int fill_blocks(int64_t n) {
  const int64_t b = (n + kBlock - 1) / kBlock;
  return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

template <typename T>
hipError_t launch_apply(const Level &L, const T *psi, const Coef<T> &C, const T *u, T *y,
                        hipStream_t st) {
  if (L.g.dim == 3) SBM_LAUNCH((k_apply<T, 3>), grid_blocks(L.g.nn), kBlock, st, L.g, C, psi, u, y);
  SBM_LAUNCH((k_apply<T, 2>), grid_blocks(L.g.nn), kBlock, st, L.g, C, psi, u, y);
}

template <typename T>
hipError_t launch_residual(const Level &L, const T *psi, const Coef<T> &C, const T *u,
                           const T *f, T *r, double *partials, hipStream_t st,
                           const uint8_t *cls, const TileList *tl) {
  if (use_tiled(L)) return launch_residual_tiled<T>(L, psi, C, u, f, r, partials, st, cls, tl);
  // partial sums are counted per block of kBlock threads
  const int bs = partials ? kBlock : level_block(L.g.nn);
  const int nb = partials ? grid_blocks(L.g.nn) : level_grid(L.g.nn);
  if (L.g.dim == 3) {
    if (cls) SBM_LAUNCH((k_residual<T, 3, true>), nb, bs, st, L.g, C, psi, u, f, r, partials, cls);
    SBM_LAUNCH((k_residual<T, 3, false>), nb, bs, st, L.g, C, psi, u, f, r, partials, cls);
  }
  if (cls) SBM_LAUNCH((k_residual<T, 2, true>), nb, bs, st, L.g, C, psi, u, f, r, partials, cls);
  SBM_LAUNCH((k_residual<T, 2, false>), nb, bs, st, L.g, C, psi, u, f, r, partials, cls);
}

hipError_t launch_residual_sweep(const Level &L, const double *u, const double *f,
                                 double *u_out, double omega, int colour, double *partials,
                                 hipStream_t st) {
  if (use_tiled(L)) return hipErrorInvalidValue;  // partials are counted per node block
  if (L.g.dim == 3)
    SBM_LAUNCH((k_residual_sweep<3>), grid_blocks(L.g.nn), kBlock, st, L.g, L.c64, L.psi64, u, f,
               u_out, omega, colour, partials);
  SBM_LAUNCH((k_residual_sweep<2>), grid_blocks(L.g.nn), kBlock, st, L.g, L.c64, L.psi64, u, f,
             u_out, omega, colour, partials);
}

bool residual_sweep_ok(const Level &L) { return !use_tiled(L); }

hipError_t launch_residual_cast(const Level &L, const double *u, const double *f, float *r32,
                                const double *ss, hipStream_t st) {
  if (L.g.dim == 3)
    SBM_LAUNCH((k_residual_cast<3>), grid_blocks(L.g.nn), kBlock, st, L.g, L.c64, L.psi64, u, f,
               r32, ss);
  SBM_LAUNCH((k_residual_cast<2>), grid_blocks(L.g.nn), kBlock, st, L.g, L.c64, L.psi64, u, f, r32,
             ss);
}

template <typename T>
hipError_t launch_jacobi(const Level &L, const T *psi, const Coef<T> &C, const T *u, const T *f,
                         T *u_out, double omega, hipStream_t st, const uint8_t *cls) {
  const int nb = level_grid(L.g.nn), bs = level_block(L.g.nn);
  if (L.g.dim == 3) {
    if (cls) SBM_LAUNCH((k_jacobi<T, 3, true>), nb, bs, st, L.g, C, psi, u, f, u_out, (T)omega, cls);
    SBM_LAUNCH((k_jacobi<T, 3, false>), nb, bs, st, L.g, C, psi, u, f, u_out, (T)omega, cls);
  }
  if (cls) SBM_LAUNCH((k_jacobi<T, 2, true>), nb, bs, st, L.g, C, psi, u, f, u_out, (T)omega, cls);
  SBM_LAUNCH((k_jacobi<T, 2, false>), nb, bs, st, L.g, C, psi, u, f, u_out, (T)omega, cls);
}

template <typename T>
hipError_t launch_rb_half(const Level &L, const T *psi, const Coef<T> &C, const T *u,
                          const T *f, T *u_out, double omega, int colour, hipStream_t st,
                          const uint8_t *cls) {
  const int64_t pairs = (int64_t)((L.g.nx + 1) / 2) * L.g.ny * L.g.nz;
  const int nb = level_grid(pairs), bs = level_block(pairs);
  if (L.g.dim == 3) {
    if (cls)
      SBM_LAUNCH((k_rb_half<T, 3, true>), nb, bs, st, L.g, C, psi, u, f, u_out, (T)omega,
                 colour, cls);
    SBM_LAUNCH((k_rb_half<T, 3, false>), nb, bs, st, L.g, C, psi, u, f, u_out, (T)omega,
               colour, cls);
  }
  if (cls)
    SBM_LAUNCH((k_rb_half<T, 2, true>), nb, bs, st, L.g, C, psi, u, f, u_out, (T)omega,
               colour, cls);
  SBM_LAUNCH((k_rb_half<T, 2, false>), nb, bs, st, L.g, C, psi, u, f, u_out, (T)omega, colour,
             cls);
}

template <typename T>
hipError_t launch_restrict(const Level &F, const Level &Cl, const T *r, T *fc, hipStream_t st,
                           T *ec) {
  if (F.g.dim == 3 && tiled_ok(F)) {
    // the tiles, then the last coarse column / row they leave
    const RTile rt = restrict_tiles(Cl.g);
    (void)hipGetLastError();
    hipLaunchKernelGGL((k_restrict_tile<T>), dim3((rt.ntiles + 7) / 8 * 8), dim3(RNT), 0, st,
                       F.g, Cl.g, rt, r, fc, ec);
    const int nrest = ((Cl.g.nx - rt.cxn) * Cl.g.ny + (Cl.g.ny - rt.cyn) * rt.cxn) * Cl.g.nz;
    if (nrest > 0)
      hipLaunchKernelGGL((k_restrict_rest<T>), dim3((nrest + kBlock - 1) / kBlock), dim3(kBlock),
                         0, st, F.g, Cl.g, rt, r, fc, ec, nrest);
    return hipGetLastError();
  }
  const int nb = level_grid(Cl.g.nn), bs = level_block(Cl.g.nn);
  if (F.g.dim == 3) SBM_LAUNCH((k_restrict<T, 3>), nb, bs, st, F.g, Cl.g, r, fc, ec);
  SBM_LAUNCH((k_restrict<T, 2>), nb, bs, st, F.g, Cl.g, r, fc, ec);
}

template <typename T>
hipError_t launch_prolong_add(const Level &F, const Level &Cl, const T *e, T *u, hipStream_t st) {
  const int nb = level_grid(Cl.g.nn), bs = level_block(Cl.g.nn);
  if (F.g.dim == 3) SBM_LAUNCH((k_prolong_add<T, 3>), nb, bs, st, F.g, Cl.g, e, u);
  SBM_LAUNCH((k_prolong_add<T, 2>), nb, bs, st, F.g, Cl.g, e, u);
}

template <typename T>
hipError_t launch_fill(T *p, int64_t n, T v, hipStream_t st) {
  SBM_LAUNCH((k_fill<T>), fill_blocks(n), kBlock, st, p, n, v);
}

// Bandwidth probe (not part of the method): a = b + s c with 16-byte loads
// and stores, two doubles per thread.
__global__ __launch_bounds__(kBlock) void k_triad(double *__restrict__ a,
                                                  const double *__restrict__ b,
                                                  const double *__restrict__ c, int64_t n,
                                                  double s) {
  const int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * 2;
  if (i + 1 < n) {
    const double2 bv = *reinterpret_cast<const double2 *>(b + i);
    const double2 cv = *reinterpret_cast<const double2 *>(c + i);
    *reinterpret_cast<double2 *>(a + i) = make_double2(bv.x + s * cv.x, bv.y + s * cv.y);
  } else if (i < n) {
    a[i] = b[i] + s * c[i];
  }
}

hipError_t launch_triad(double *a, const double *b, const double *c, int64_t n, double s,
                        hipStream_t st) {
  const int64_t blocks = (n + 2 * kBlock - 1) / (2 * kBlock);
  SBM_LAUNCH(k_triad, (unsigned)blocks, kBlock, st, a, b, c, n, s);
}

template <typename T>
hipError_t launch_copy(const T *src, T *dst, int64_t n, hipStream_t st) {
  SBM_LAUNCH((k_copy<T>), fill_blocks(n), kBlock, st, src, dst, n);
}

hipError_t launch_correct(const Level &L, double *u, const float *e32, const double *ss,
                          hipStream_t st) {
  if (L.g.dim == 3) SBM_LAUNCH((k_correct<3>), num_blocks(L.g.nn), kBlock, st, L.g, u, e32, ss);
  SBM_LAUNCH((k_correct<2>), num_blocks(L.g.nn), kBlock, st, L.g, u, e32, ss);
}

hipError_t launch_set_dirichlet(const Level &L, double *u, const DispValues &dv, hipStream_t st) {
  if (L.g.dim == 3) SBM_LAUNCH((k_set_dirichlet<3>), num_blocks(L.g.nn), kBlock, st, L.g, u, dv);
  SBM_LAUNCH((k_set_dirichlet<2>), num_blocks(L.g.nn), kBlock, st, L.g, u, dv);
}

hipError_t launch_floor_psi(const double *raw, double floor_, double *psi64, float *psi32,
                            int64_t n, int cube, int *flag, hipStream_t st) {
  SBM_LAUNCH(k_floor_psi, num_blocks(n), kBlock, st, raw, floor_, psi64, psi32, n, cube, flag);
}

hipError_t launch_coarsen_psi(const Level &F, const Level &Cl, hipStream_t st) {
  if (F.g.dim == 3)
    SBM_LAUNCH((k_coarsen_psi<3>), num_blocks(Cl.g.nc), kBlock, st, F.g, Cl.g, F.psi64, Cl.psi64,
               Cl.psi32);
  SBM_LAUNCH((k_coarsen_psi<2>), num_blocks(Cl.g.nc), kBlock, st, F.g, Cl.g, F.psi64, Cl.psi64,
             Cl.psi32);
}

hipError_t launch_rhs(const Level &L, const Traction &tr, const double *b, double *fA, int *flag,
                      hipStream_t st) {
  if (L.g.dim == 3) SBM_LAUNCH((k_rhs<3>), num_blocks(L.g.nn), kBlock, st, L.g, tr, L.psi64, b, fA, flag);
  SBM_LAUNCH((k_rhs<2>), num_blocks(L.g.nn), kBlock, st, L.g, tr, L.psi64, b, fA, flag);
}

hipError_t launch_check_diag(const Level &L, int *flag, hipStream_t st) {
  if (L.g.dim == 3) SBM_LAUNCH((k_check_diag<3>), num_blocks(L.g.nn), kBlock, st, L.g, L.psi64, flag);
  SBM_LAUNCH((k_check_diag<2>), num_blocks(L.g.nn), kBlock, st, L.g, L.psi64, flag);
}

hipError_t launch_finalize_sum(const double *partials, int n, double *out, hipStream_t st) {
  SBM_LAUNCH(k_finalize_sum, 1, 1024, st, partials, n, out);
}

hipError_t launch_dot_free(const Level &L, const double *a, const ZSrc &b, double *partials,
                           hipStream_t st) {
  if (L.g.dim == 3) SBM_LAUNCH((k_dot_free<3>), num_blocks(L.g.nn), kBlock, st, L.g, a, b, partials);
  SBM_LAUNCH((k_dot_free<2>), num_blocks(L.g.nn), kBlock, st, L.g, a, b, partials);
}

hipError_t launch_apply_dot(const Level &L, const double *p, double *q, double *partials,
                           hipStream_t st) {
  if (use_tiled(L)) return launch_apply_dot_tiled(L, p, q, partials, st);
  if (L.g.dim == 3)
    SBM_LAUNCH((k_apply_dot<3>), grid_blocks(L.g.nn), kBlock, st, L.g, L.c64, L.psi64, p, q, partials);
  SBM_LAUNCH((k_apply_dot<2>), grid_blocks(L.g.nn), kBlock, st, L.g, L.c64, L.psi64, p, q, partials);
}

hipError_t launch_cg_update_r(const Level &L, double *r, const double *q, const ZSrc &z,
                              const double *rz, const double *pq, double *alpha_out, double *pr,
                              double *pz, hipStream_t st, float *r32, const double *ss) {
  if (L.g.dim == 3)
    SBM_LAUNCH((k_cg_update_r<3>), num_blocks(L.g.nn), kBlock, st, L.g, r, q, z, rz, pq,
               alpha_out, pr, pz, r32, ss);
  SBM_LAUNCH((k_cg_update_r<2>), num_blocks(L.g.nn), kBlock, st, L.g, r, q, z, rz, pq, alpha_out,
             pr, pz, r32, ss);
}

hipError_t launch_xpby_x(const Level &L, double *x, double *p, const ZSrc &z,
                         const double *rznew, const double *rzold, const double *rz,
                         const double *alpha, hipStream_t st) {
  if (L.g.dim == 3)
    SBM_LAUNCH((k_xpby_x<3>), num_blocks(L.g.nn), kBlock, st, L.g, x, p, z, rznew, rzold, rz,
               alpha);
  SBM_LAUNCH((k_xpby_x<2>), num_blocks(L.g.nn), kBlock, st, L.g, x, p, z, rznew, rzold, rz, alpha);
}

hipError_t launch_axpy_free(const Level &L, double *x, const double *p, const double *alpha,
                            hipStream_t st) {
  if (L.g.dim == 3) SBM_LAUNCH((k_axpy_free<3>), num_blocks(L.g.nn), kBlock, st, L.g, x, p, alpha);
  SBM_LAUNCH((k_axpy_free<2>), num_blocks(L.g.nn), kBlock, st, L.g, x, p, alpha);
}


hipError_t launch_cast_scaled(const double *r, float *r32, int64_t n, const double *ss,
                              hipStream_t st) {
  SBM_LAUNCH(k_cast_scaled, num_blocks(n), kBlock, st, r, r32, n, ss);
}

hipError_t launch_scale_cast(const double *r, float *r32, int64_t n, const double *ss,
                             hipStream_t st) {
  SBM_LAUNCH(k_scale_cast, num_blocks(n), kBlock, st, r, r32, n, ss);
}

// The first colour-`colour` half-sweep from a zero iterate for the load f,
// into t: omega f / D on the relaxed colour (D the diagonal), 0 elsewhere.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_zero_sweep(Geom g, Coef<T> C, const T *__restrict__ psi,
                                                       const T *__restrict__ f, T *__restrict__ t,
                                                       T omega, int colour) {
  const int64_t id = (int64_t)xcd_block() * kBlock + threadIdx.x;
  if (id >= g.nn) return;
  int i, j, k;
  node_ijk(g, id, i, j, k);
  T dg[3];
  node_diag<T, DIM>(g, C, psi, i, j, k, dg);
  const uint32_t fb = face_bits(g, i, j, k);
  const bool relax = ((i + j + k) & 1) == colour;
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    const T w = ((g.dmask >> c) & fb) ? T(0) : omega;
    t[c * g.nn + id] = relax ? T(0) + w * (f[c * g.nn + id] - T(0)) / dg[c] : T(0);
  }
}

hipError_t launch_zero_sweep(const Level &L, const double *f, double *t, double omega, int colour,
                             hipStream_t st) {
  if (L.g.dim == 3)
    SBM_LAUNCH((k_zero_sweep<double, 3>), grid_blocks(L.g.nn), kBlock, st, L.g, L.c64, L.psi64, f,
               t, omega, colour);
  SBM_LAUNCH((k_zero_sweep<double, 2>), grid_blocks(L.g.nn), kBlock, st, L.g, L.c64, L.psi64, f, t,
             omega, colour);
}

hipError_t launch_scale_cast_sweep(const Level &L, const double *r, float *r32, float *t32,
                                   double omega, int colour, const double *ss, hipStream_t st) {
  if (L.g.dim == 3)
    SBM_LAUNCH((k_scale_cast_sweep<3>), grid_blocks(L.g.nn), kBlock, st, L.g, L.c32, L.psi32, r,
               r32, t32, (float)omega, colour, ss);
  SBM_LAUNCH((k_scale_cast_sweep<2>), grid_blocks(L.g.nn), kBlock, st, L.g, L.c32, L.psi32, r, r32,
             t32, (float)omega, colour, ss);
}

hipError_t launch_store_sqrt(const double *ss, double *s_out, hipStream_t st) {
  SBM_LAUNCH(k_store_sqrt, 1, 64, st, ss, s_out);
}

hipError_t launch_sumsq_free(const Level &L, const double *v, double *partials, hipStream_t st) {
  if (L.g.dim == 3) SBM_LAUNCH((k_sumsq_free<3>), num_blocks(L.g.nn), kBlock, st, L.g, v, partials);
  SBM_LAUNCH((k_sumsq_free<2>), num_blocks(L.g.nn), kBlock, st, L.g, v, partials);
}

// One node per thread up to kBotThreads threads, then up to kBotQ per thread.
static int bottom_threads(int64_t nn) {
  int64_t t = (nn + 63) / 64 * 64;
  return (int)(t < 64 ? 64 : (t > kBotThreads ? kBotThreads : t));
}

static bool bottom_fits_lds(const Geom &g, size_t bytes) {
  return g.nn <= (int64_t)kBotQ * kBotThreads && bytes <= 64 * 1024;
}

static size_t bottom_lds64_bytes(const Geom &g) {
  return sizeof(double) * (size_t)(((g.nc + 1) & ~(int64_t)1) + g.dim * g.nn);
}


template <typename T>
hipError_t launch_bottom_cg(const Level &L, const T *psi, const Coef<T> &C, const T *f, T *x,
                            T *r, T *p, T *Ap, double rtol, int maxit, int *iters,
                            hipStream_t st) {
  if constexpr (sizeof(T) == 8) {
    const size_t by = bottom_lds64_bytes(L.g);
    if (bottom_fits_lds(L.g, by)) {
      const int nt = bottom_threads(L.g.nn);
      const bool one = L.g.nn <= kBotThreads;  // one node per thread: fewer registers
      (void)hipGetLastError();
      if (L.g.dim == 3) {
        if (one)
          hipLaunchKernelGGL((k_bottom_lds64<3, 1, double>), dim3(1), dim3(nt), by, st, L.g, C, psi, f, x,
                             rtol, maxit, iters);
        else
          hipLaunchKernelGGL((k_bottom_lds64<3, kBotQ, double>), dim3(1), dim3(nt), by, st, L.g, C, psi, f,
                             x, rtol, maxit, iters);
      } else {
        if (one)
          hipLaunchKernelGGL((k_bottom_lds64<2, 1, double>), dim3(1), dim3(nt), by, st, L.g, C, psi, f, x,
                             rtol, maxit, iters);
        else
          hipLaunchKernelGGL((k_bottom_lds64<2, kBotQ, double>), dim3(1), dim3(nt), by, st, L.g, C, psi, f,
                             x, rtol, maxit, iters);
      }
      return hipGetLastError();
    }
  }
  if (L.g.dim == 3)
    SBM_LAUNCH((k_bottom_cg<T, 3>), 1, kBottomThreads, st, L.g, C, psi, f, x, r, p, Ap, rtol,
               maxit, iters);
  SBM_LAUNCH((k_bottom_cg<T, 2>), 1, kBottomThreads, st, L.g, C, psi, f, x, r, p, Ap, rtol, maxit,
             iters);
}

hipError_t launch_bottom_f32io(const Level &L, const float *f32, float *x32, double *f64,
                               double *x64, double *r, double *p, double *Ap, double rtol,
                               int maxit, int *iters, hipStream_t st) {
  const size_t by = bottom_lds64_bytes(L.g);
  if (bottom_fits_lds(L.g, by)) {
    const int nt = bottom_threads(L.g.nn);
    const bool one = L.g.nn <= kBotThreads;
    (void)hipGetLastError();
    if (L.g.dim == 3) {
      if (one)
        hipLaunchKernelGGL((k_bottom_lds64<3, 1, float>), dim3(1), dim3(nt), by, st, L.g, L.c64,
                           L.psi64, f32, x32, rtol, maxit, iters);
      else
        hipLaunchKernelGGL((k_bottom_lds64<3, kBotQ, float>), dim3(1), dim3(nt), by, st, L.g,
                           L.c64, L.psi64, f32, x32, rtol, maxit, iters);
    } else {
      if (one)
        hipLaunchKernelGGL((k_bottom_lds64<2, 1, float>), dim3(1), dim3(nt), by, st, L.g, L.c64,
                           L.psi64, f32, x32, rtol, maxit, iters);
      else
        hipLaunchKernelGGL((k_bottom_lds64<2, kBotQ, float>), dim3(1), dim3(nt), by, st, L.g,
                           L.c64, L.psi64, f32, x32, rtol, maxit, iters);
    }
    return hipGetLastError();
  }
  // larger bottoms: the global-memory FP64 CG on converted copies
  const int64_t nv = (int64_t)L.g.dim * L.g.nn;
  hipError_t e;
  (void)hipGetLastError();
  hipLaunchKernelGGL((k_convert<float, double>), dim3(fill_blocks(nv)), dim3(kBlock), 0, st, f32,
                     f64, nv);
  hipLaunchKernelGGL((k_convert<float, double>), dim3(fill_blocks(nv)), dim3(kBlock), 0, st, x32,
                     x64, nv);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_bottom_cg<double>(L, L.psi64, L.c64, f64, x64, r, p, Ap, rtol, maxit, iters,
                                    st)) != hipSuccess)
    return e;
  hipLaunchKernelGGL((k_convert<double, float>), dim3(fill_blocks(nv)), dim3(kBlock), 0, st, x64,
                     x32, nv);
  return hipGetLastError();
}

hipError_t launch_sensitivity(const Level &L, double lam, double mu, const Traction &tr,
                              const double *u, const double *adj, double lam_scale,
                              const double *design, int chain, double psi_floor, double *g,
                              hipStream_t st) {
  if (L.g.dim == 3)
    SBM_LAUNCH((k_sensitivity<3>), grid_blocks(L.g.nc), kBlock, st, L.g, lam, mu, L.h[0], L.h[1],
               L.h[2], tr, u, adj, lam_scale, design, chain, psi_floor, g);
  SBM_LAUNCH((k_sensitivity<2>), grid_blocks(L.g.nc), kBlock, st, L.g, lam, mu, L.h[0], L.h[1],
             L.h[2], tr, u, adj, lam_scale, design, chain, psi_floor, g);
}

#define SBM_INST(T)                                                                            \
  template hipError_t launch_apply<T>(const Level &, const T *, const Coef<T> &, const T *, T *, \
                                      hipStream_t);                                            \
  template hipError_t launch_residual<T>(const Level &, const T *, const Coef<T> &, const T *,  \
                                         const T *, T *, double *, hipStream_t,                \
                                         const uint8_t *, const TileList *);                   \
  template hipError_t launch_jacobi<T>(const Level &, const T *, const Coef<T> &, const T *,    \
                                       const T *, T *, double, hipStream_t, const uint8_t *);  \
  template hipError_t launch_rb_half<T>(const Level &, const T *, const Coef<T> &, const T *,   \
                                        const T *, T *, double, int, hipStream_t,              \
                                        const uint8_t *);                                      \
  template hipError_t launch_restrict<T>(const Level &, const Level &, const T *, T *,          \
                                         hipStream_t, T *);                                    \
  template hipError_t launch_prolong_add<T>(const Level &, const Level &, const T *, T *,       \
                                            hipStream_t);                                      \
  template hipError_t launch_fill<T>(T *, int64_t, T, hipStream_t);                             \
  template hipError_t launch_copy<T>(const T *, T *, int64_t, hipStream_t);                     \
  template hipError_t launch_bottom_cg<T>(const Level &, const T *, const Coef<T> &, const T *, \
                                          T *, T *, T *, T *, double, int, int *, hipStream_t);

SBM_INST(double)
SBM_INST(float)
template hipError_t launch_fill<int>(int *, int64_t, int, hipStream_t);

}  // namespace sbm
