// sbm_device.h -- device-side building blocks of the gfx950 SBM multigrid:
// level geometry, operator coefficients, the node stencil of K, Dirichlet
// masks and deterministic block reductions.
//
// Operator (Agrawal & Runnels, Sec. 2.1 eq. SBMLinearElasticity with the
// cell-based indicator of Sec. 2.3): K u = -div(psi C grad u), displacement on
// nodes, psi on cells, psi = 0 outside the box.  In 2D/3D the divergence is
// taken in split flux form:
//   * direct part (derivative and flux along the same axis j): a 3-point
//     flux difference whose edge coefficient is the mean psi of the 2^(d-1)
//     cells around the edge;
//   * cross part (flux along j of the l-derivative, j != l): evaluated on the
//     four quadrants p = n + (sa e_a + sb e_b)/2 of each coordinate plane with
//     the mean psi of the 2^(d-2) cells touching p.
// For isotropic C the cross part of the quadrant (sa, sb) in plane (a, b)
// reduces to
//   row a -= sa sb Fsum [ cp (u_b(n+sa e_a+sb e_b) - u_b(n)) + cm (u_b(n+sb e_b) - u_b(n+sa e_a)) ]
//   row b -= sa sb Fsum [ cp (u_a(n+sa e_a+sb e_b) - u_a(n)) + cm (u_a(n+sa e_a) - u_a(n+sb e_b)) ]
// with cp = (lambda+mu)/(4 h_a h_b 2^(d-2)), cm = (lambda-mu)/(4 h_a h_b 2^(d-2))
// and Fsum the plain sum of the touching cells; the direct part is
//   row i -= sum_j cd_ij [ Esum(+j)(u_i(n+e_j)-u_i(n)) + Esum(-j)(u_i(n-e_j)-u_i(n)) ]
// with cd_ij = (mu + (lambda+mu) delta_ij) / (h_j^2 2^(d-1)).  The diagonal
// (Sec. 2.3, the Jacobi D) comes from the direct part only:
//   D_i = sum_j cd_ij (Esum(+j) + Esum(-j)).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sbm_fastdiv.h"

namespace sbm {

constexpr int kBlock = 256;  // threads per block of the node-parallel kernels

struct Geom {
  int dim;
  int nx, ny, nz;   // nodes per axis (nz = 1 in 2D)
  int cx, cy, cz;   // cells per axis (cz = 1 in 2D)
  int64_t nn;       // nodes (< 2^31)
  int64_t nc;       // cells
  uint32_t dmask;   // bit 3*F + k: face F fixes component k (F = x-,x+,y-,y+,z-,z+)
  FastDiv fnx, fny; // division by nx and ny (node index decoding)
  FastDiv fcx, fcy; // division by cx and cy (cell index decoding)
  FastDiv fpx;      // division by (nx + 1) / 2 (x-pairs of the colour sweeps)
};

template <typename T>
struct Coef {
  T cd[3][3];  // direct coefficients
  T cp[3];     // cross (lambda+mu) part, planes xy, xz, yz
  T cm[3];     // cross (lambda-mu) part
};

// Logical block of a node-parallel launch: workgroup b runs on XCD b mod 8,
// so for grids padded to a multiple of 8 each XCD is dealt a contiguous range
// of logical blocks (rows and planes it shares with its neighbours stay in
// its own L2).
__device__ __forceinline__ int xcd_block() {
  const int nwg = gridDim.x;
  return (nwg & 7) == 0 ? (int)(blockIdx.x & 7) * (nwg >> 3) + (int)(blockIdx.x >> 3)
                        : (int)blockIdx.x;
}

// Bit 3F is set when node (i, j, k) lies on face F (x-,x+,y-,y+,z-,z+), so
// that (dmask >> comp) & face_bits tests every face at once (no branches).
__device__ __forceinline__ uint32_t face_bits(const Geom &g, int i, int j, int k) {
  uint32_t b = (i == 0 ? 1u : 0u) | (i == g.nx - 1 ? 8u : 0u) | (j == 0 ? 64u : 0u) |
               (j == g.ny - 1 ? 512u : 0u);
  if (g.dim == 3) b |= (k == 0 ? 4096u : 0u) | (k == g.nz - 1 ? 32768u : 0u);
  return b;
}

__device__ __forceinline__ bool is_dirichlet(const Geom &g, int i, int j, int k, int comp) {
  return ((g.dmask >> comp) & face_bits(g, i, j, k)) != 0u;
}

// Node coordinates of a linear node index.
__device__ __forceinline__ void node_ijk(const Geom &g, int64_t id, int &i, int &j, int &k) {
  const uint32_t n = (uint32_t)id;
  const uint32_t row = g.fnx.div(n);
  i = (int)(n - row * (uint32_t)g.nx);
  k = (int)g.fny.div(row);
  j = (int)(row - (uint32_t)k * (uint32_t)g.ny);
}

// Cell coordinates of a linear cell index.
__device__ __forceinline__ void cell_ijk(const Geom &g, int64_t id, int &i, int &j, int &k) {
  const uint32_t n = (uint32_t)id;
  const uint32_t row = g.fcx.div(n);
  i = (int)(n - row * (uint32_t)g.cx);
  k = (int)g.fcy.div(row);
  j = (int)(row - (uint32_t)k * (uint32_t)g.cy);
}

// Coefficients of a level with cubic cells (h equal on every axis): the
// direct coefficients take two values (diagonal i == j, off-diagonal) and the
// cross coefficients one per kind, so a kernel needs 4 scalars instead of 15.
template <typename T>
struct CoefCubic {
  T dd, od, p, m;
};
template <typename T>
__device__ __forceinline__ T coef_cd(const Coef<T> &C, int i, int j) { return C.cd[i][j]; }
template <typename T>
__device__ __forceinline__ T coef_cp(const Coef<T> &C, int pl) { return C.cp[pl]; }
template <typename T>
__device__ __forceinline__ T coef_cm(const Coef<T> &C, int pl) { return C.cm[pl]; }
template <typename T>
__device__ __forceinline__ T coef_cd(const CoefCubic<T> &C, int i, int j) { return i == j ? C.dd : C.od; }
template <typename T>
__device__ __forceinline__ T coef_cp(const CoefCubic<T> &C, int) { return C.p; }
template <typename T>
__device__ __forceinline__ T coef_cm(const CoefCubic<T> &C, int) { return C.m; }

// 3D eq. K at one node: P[c2][c1][c0] is the psi of cell (i-1+c0, j-1+c1,
// k-1+c2) (0 outside the box) and U(c, dx, dy, dz) the c-th displacement at the
// neighbour (i+dx, j+dy, k+dz).  Writes (K u)(n) and the diagonal of K.  C is a
// Coef<T> or a CoefCubic<T>.
template <typename T, typename CO, typename UF>
__device__ __forceinline__ void stencil3(const CO &C, const T (&P)[2][2][2], UF &&U,
                                         T out[3], T diag[3]) {
  T E[3][2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    E[0][s] = P[0][0][s] + P[0][1][s] + P[1][0][s] + P[1][1][s];
    E[1][s] = P[0][s][0] + P[0][s][1] + P[1][s][0] + P[1][s][1];
    E[2][s] = P[s][0][0] + P[s][0][1] + P[s][1][0] + P[s][1][1];
  }
  // direct part
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T uc = U(c, 0, 0, 0);
    const T xp = U(c, 1, 0, 0) - uc, xm = U(c, -1, 0, 0) - uc;
    const T yp = U(c, 0, 1, 0) - uc, ym = U(c, 0, -1, 0) - uc;
    const T zp = U(c, 0, 0, 1) - uc, zm = U(c, 0, 0, -1) - uc;
    out[c] = -(coef_cd(C, c, 0) * (E[0][1] * xp + E[0][0] * xm) +
               coef_cd(C, c, 1) * (E[1][1] * yp + E[1][0] * ym) +
               coef_cd(C, c, 2) * (E[2][1] * zp + E[2][0] * zm));
    diag[c] = coef_cd(C, c, 0) * (E[0][0] + E[0][1]) + coef_cd(C, c, 1) * (E[1][0] + E[1][1]) +
              coef_cd(C, c, 2) * (E[2][0] + E[2][1]);
  }
  // cross part, plane (a, b) with third axis m
#pragma unroll
  for (int pl = 0; pl < 3; ++pl) {
    const int a = (pl == 2) ? 1 : 0;
    const int b = (pl == 0) ? 1 : 2;
    const T cp = coef_cp(C, pl), cm = coef_cm(C, pl);
    const T ua0 = U(a, 0, 0, 0), ub0 = U(b, 0, 0, 0);
    T ra = T(0), rb = T(0);
#pragma unroll
    for (int qa = 0; qa < 2; ++qa)
#pragma unroll
      for (int qb = 0; qb < 2; ++qb) {
        const int sa = 2 * qa - 1, sb = 2 * qb - 1;
        int da[3] = {0, 0, 0}, db[3] = {0, 0, 0};
        da[a] = sa;
        db[b] = sb;
        T F;
        if (pl == 0) F = P[0][qb][qa] + P[1][qb][qa];       // (x, y), m = z
        else if (pl == 1) F = P[qb][0][qa] + P[qb][1][qa];  // (x, z), m = y
        else F = P[qb][qa][0] + P[qb][qa][1];               // (y, z), m = x
        const T w = (sa * sb > 0) ? F : -F;
        const T uaab = U(a, da[0] + db[0], da[1] + db[1], da[2] + db[2]);
        const T ubab = U(b, da[0] + db[0], da[1] + db[1], da[2] + db[2]);
        const T uaa = U(a, da[0], da[1], da[2]), uab = U(a, db[0], db[1], db[2]);
        const T uba = U(b, da[0], da[1], da[2]), ubb = U(b, db[0], db[1], db[2]);
        ra += w * (cp * (ubab - ub0) + cm * (ubb - uba));
        rb += w * (cp * (uaab - ua0) + cm * (uaa - uab));
      }
    out[a] -= ra;
    out[b] -= rb;
  }
}

// Evaluates (K u)(n) for all components and the diagonal at node (i, j, k).
// Neighbour offsets are clamped at the box boundary: every term that would
// reach outside carries a zero psi weight, so the clamped value never counts.
// ctr (optional) receives u at the node itself.  GATHER keeps every load
// ahead of the arithmetic (a scheduling barrier); without it the compiler may
// interleave them, which needs fewer registers.
template <typename T, int DIM, bool GATHER = true, typename G = Geom, typename CO = Coef<T>>
__device__ __forceinline__ void node_stencil(const G &g, const CO &C,
                                             const T *__restrict__ psi,
                                             const T *__restrict__ u, int i, int j, int k,
                                             T out[3], T diag[3], T *ctr = nullptr) {
  // every index fits in 32 bits (nodes x components < 2^31)
  const int sy = g.nx, sz = g.nx * g.ny;
  const int idx = i + sy * j + sz * k;
  const int ox[3] = {i > 0 ? -1 : 0, 0, i < g.nx - 1 ? 1 : 0};
  const int oy[3] = {j > 0 ? -sy : 0, 0, j < g.ny - 1 ? sy : 0};
  const int nn = (int)g.nn;
  if constexpr (DIM == 3) {
    const int oz[3] = {k > 0 ? -sz : 0, 0, k < g.nz - 1 ? sz : 0};
    // Gather: the 8 cells around the node and the 45 displacement values eq. K
    // reads (all components at the node and its 6 face neighbours, the two
    // in-plane components at the 12 edge neighbours) are loaded before any of
    // them is used, so that every load of the thread is in flight at once.
    // P[oz][oy][ox] is cell (i-1+ox, j-1+oy, k-1+oz), read from a clamped cell
    // and zeroed outside the box.
    T pv[2][2][2];
    bool pin[2][2][2];
#pragma unroll
    for (int c2 = 0; c2 < 2; ++c2)
#pragma unroll
      for (int c1 = 0; c1 < 2; ++c1)
#pragma unroll
        for (int c0 = 0; c0 < 2; ++c0) {
          const int xi = i - 1 + c0, yj = j - 1 + c1, zk = k - 1 + c2;
          pin[c2][c1][c0] = xi >= 0 && xi < g.cx && yj >= 0 && yj < g.cy && zk >= 0 && zk < g.cz;
          const int xc = min(max(xi, 0), g.cx - 1), yc = min(max(yj, 0), g.cy - 1);
          const int zc = min(max(zk, 0), g.cz - 1);
          pv[c2][c1][c0] = psi[xc + g.cx * (yc + g.cy * zc)];
        }
    T V[3][27];  // V[c][(dx+1) + 3 (dy+1) + 9 (dz+1)]
    auto ld = [&](int c, int dx, int dy, int dz) {
      V[c][(dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)] =
          u[c * nn + idx + ox[dx + 1] + oy[dy + 1] + oz[dz + 1]];
    };
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      ld(c, 0, 0, 0);
      ld(c, -1, 0, 0);
      ld(c, 1, 0, 0);
      ld(c, 0, -1, 0);
      ld(c, 0, 1, 0);
      ld(c, 0, 0, -1);
      ld(c, 0, 0, 1);
    }
#pragma unroll
    for (int pl = 0; pl < 3; ++pl) {
      const int a = (pl == 2) ? 1 : 0, b = (pl == 0) ? 1 : 2;
#pragma unroll
      for (int sa = -1; sa <= 1; sa += 2)
#pragma unroll
        for (int sb = -1; sb <= 1; sb += 2) {
          int d[3] = {0, 0, 0};
          d[a] = sa;
          d[b] = sb;
          ld(a, d[0], d[1], d[2]);
          ld(b, d[0], d[1], d[2]);
        }
    }
    if constexpr (GATHER) __builtin_amdgcn_sched_barrier(0);
    T P[2][2][2];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      P[q >> 2][(q >> 1) & 1][q & 1] = pin[q >> 2][(q >> 1) & 1][q & 1] ? pv[q >> 2][(q >> 1) & 1][q & 1] : T(0);
    auto U = [&](int c, int dx, int dy, int dz) -> T {
      return V[c][(dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)];
    };
    stencil3<T>(C, P, U, out, diag);
    if (ctr)
#pragma unroll
      for (int c = 0; c < 3; ++c) ctr[c] = U(c, 0, 0, 0);
  } else {
    // Gather as in 3D: the 4 cells and both components at the node and its 8
    // neighbours (every one of them enters eq. K in 2D) before any arithmetic.
    T pv[2][2];
    bool pin[2][2];
#pragma unroll
    for (int c1 = 0; c1 < 2; ++c1)
#pragma unroll
      for (int c0 = 0; c0 < 2; ++c0) {
        const int xi = i - 1 + c0, yj = j - 1 + c1;
        pin[c1][c0] = xi >= 0 && xi < g.cx && yj >= 0 && yj < g.cy;
        const int xc = min(max(xi, 0), g.cx - 1), yc = min(max(yj, 0), g.cy - 1);
        pv[c1][c0] = psi[xc + g.cx * yc];
      }
    T V[2][9];  // V[c][(dx+1) + 3 (dy+1)]
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx)
          V[c][(dx + 1) + 3 * (dy + 1)] = u[c * nn + idx + ox[dx + 1] + oy[dy + 1]];
    if constexpr (GATHER) __builtin_amdgcn_sched_barrier(0);
    T P[2][2];  // P[oy][ox]
#pragma unroll
    for (int q = 0; q < 4; ++q) P[q >> 1][q & 1] = pin[q >> 1][q & 1] ? pv[q >> 1][q & 1] : T(0);
    T E[2][2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      E[0][s] = P[0][s] + P[1][s];
      E[1][s] = P[s][0] + P[s][1];
    }
    auto U = [&](int c, int dx, int dy) -> T { return V[c][(dx + 1) + 3 * (dy + 1)]; };
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const T uc = U(c, 0, 0);
      const T xp = U(c, 1, 0) - uc, xm = U(c, -1, 0) - uc;
      const T yp = U(c, 0, 1) - uc, ym = U(c, 0, -1) - uc;
      out[c] = -(coef_cd(C, c, 0) * (E[0][1] * xp + E[0][0] * xm) +
                 coef_cd(C, c, 1) * (E[1][1] * yp + E[1][0] * ym));
      diag[c] = coef_cd(C, c, 0) * (E[0][0] + E[0][1]) + coef_cd(C, c, 1) * (E[1][0] + E[1][1]);
    }
    const T cp = coef_cp(C, 0), cm = coef_cm(C, 0);
    const T ux0 = U(0, 0, 0), uy0 = U(1, 0, 0);
    T rx = T(0), ry = T(0);
#pragma unroll
    for (int qa = 0; qa < 2; ++qa)
#pragma unroll
      for (int qb = 0; qb < 2; ++qb) {
        const int sa = 2 * qa - 1, sb = 2 * qb - 1;
        const T F = P[qb][qa];
        const T w = (sa * sb > 0) ? F : -F;
        const T uxab = U(0, sa, sb), uyab = U(1, sa, sb);
        const T uxa = U(0, sa, 0), uxb = U(0, 0, sb);
        const T uya = U(1, sa, 0), uyb = U(1, 0, sb);
        rx += w * (cp * (uyab - uy0) + cm * (uyb - uya));
        ry += w * (cp * (uxab - ux0) + cm * (uxa - uxb));
      }
    out[0] -= rx;
    out[1] -= ry;
    out[2] = T(0);
    diag[2] = T(0);
    if (ctr) {
      ctr[0] = ux0;
      ctr[1] = uy0;
      ctr[2] = T(0);
    }
  }
}

// Diagonal of K at node (i, j, k) (the Jacobi D of Sec. 2.3): the direct
// part's edge sums only.
template <typename T, int DIM>
__device__ __forceinline__ void node_diag(const Geom &g, const Coef<T> &C,
                                          const T *__restrict__ psi, int i, int j, int k,
                                          T diag[3]) {
  T E[3][2] = {{T(0), T(0)}, {T(0), T(0)}, {T(0), T(0)}};
#pragma unroll
  for (int o = 0; o < (1 << DIM); ++o) {
    const int b0 = o & 1, b1 = (o >> 1) & 1, b2 = (o >> 2) & 1;
    const int xi = i - 1 + b0, yj = j - 1 + b1, zk = (DIM == 3) ? k - 1 + b2 : 0;
    const bool in = xi >= 0 && xi < g.cx && yj >= 0 && yj < g.cy && zk >= 0 && zk < g.cz;
    const T v = in ? psi[xi + g.cx * (yj + g.cy * zk)] : T(0);
    E[0][b0] += v;
    E[1][b1] += v;
    if (DIM == 3) E[2][b2] += v;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    diag[c] = T(0);
    if (c >= DIM) continue;
#pragma unroll
    for (int a = 0; a < DIM; ++a) diag[c] += C.cd[c][a] * (E[a][0] + E[a][1]);
  }
}

// One 32-bit half of a double moved across lanes by a DPP control (lanes
// whose source lies outside the row read zero).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xf, true);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave, returned in every lane, without LDS
// traffic: prefix sums inside each 16-lane row (row shifts 1, 2, 4, 8), the
// row totals carried into rows 1 and 3 and then into rows 2 and 3 (row
// broadcasts of lanes 15 and 31), the total read from lane 63.  The latency
// of the bottom CG is dominated by these reductions.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0x111, 0xf>(v);  // row_shr:1
  v += dpp_move<0x112, 0xf>(v);  // row_shr:2
  v += dpp_move<0x114, 0xf>(v);  // row_shr:4
  v += dpp_move<0x118, 0xf>(v);  // row_shr:8
  v += dpp_move<0x142, 0xa>(v);  // row_bcast:15
  v += dpp_move<0x143, 0xc>(v);  // row_bcast:31
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Sum over a block of kBlock threads in a fixed order; the result is valid in
// thread 0.  lds must hold kBlock/64 doubles.
__device__ __forceinline__ double block_sum(double v, double *lds) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int q = 0; q < nw; ++q) s += lds[q];
  }
  return s;
}

// Sum over the whole block, broadcast to every thread.  lds must hold
// blockDim/64 + 1 doubles.
__device__ __forceinline__ double block_allsum(double v, double *lds) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    const int nw = blockDim.x >> 6;
    for (int q = 0; q < nw; ++q) s += lds[q];
    lds[nw] = s;
  }
  __syncthreads();
  return lds[blockDim.x >> 6];
}

}  // namespace sbm
