// sbm_plastic.hip -- plastic strain on the finest grid (Sec. 3.1, 3D): the
// load of a cell plastic strain and the J2 radial-return update of the cell
// state, the two pointwise kernels of the staggered elastic / plastic step.
//
// Stress sigma = C (grad u - eps_p) turns the equilibrium into
// K u = b - div(psi C eps_p).  The divergence is the flux form of eq. K: for
// node n, component i,
//   fp_i(n) = -(1/4) sum_j (1/h_j) sum_{b in {0,1}^3} (2 b_j - 1) S_ij(c_b),
// over the 8 cells c_b = n - 1 + b around the node, S = psi C eps_p (cells
// outside the box count 0): the half-edge stresses are the means of the four
// cells around each edge, as the edge psi of eq. K.
//
// Cell state arrays (cells, x fastest): eps_p and beta as 6 components (xx,
// yy, zz, yz, xz, xy) one array after another, alpha one array.
#include "sbm_internal.h"

namespace sbm {
namespace {

constexpr int kVi[6] = {0, 1, 2, 1, 0, 0}, kVj[6] = {0, 1, 2, 2, 2, 1};

// fp = -div(psi C eps_p) at every node.  One thread per node; the 8 cells'
// psi and strains are loaded (clamped, zeroed outside) before any arithmetic.
__global__ __launch_bounds__(kBlock) void k_plastic_source(Geom g, double lam, double mu,
                                                          double ihx, double ihy, double ihz,
                                                          const double *__restrict__ psi,
                                                          const double *__restrict__ ep,
                                                          double *__restrict__ fp) {
  const int64_t id = (int64_t)xcd_block() * kBlock + threadIdx.x;
  if (id >= g.nn) return;
  int i, j, k;
  node_ijk(g, id, i, j, k);
  const int64_t nc = g.nc;
  double pv[8], ev[8][6];
  bool in[8];
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const int x = i - 1 + (b & 1), y = j - 1 + ((b >> 1) & 1), z = k - 1 + (b >> 2);
    in[b] = x >= 0 && x < g.cx && y >= 0 && y < g.cy && z >= 0 && z < g.cz;
    const int xc = min(max(x, 0), g.cx - 1), yc = min(max(y, 0), g.cy - 1);
    const int zc = min(max(z, 0), g.cz - 1);
    const int64_t q = xc + (int64_t)g.cx * (yc + (int64_t)g.cy * zc);
    pv[b] = psi[q];
#pragma unroll
    for (int m = 0; m < 6; ++m) ev[b][m] = ep[m * nc + q];
  }
  __builtin_amdgcn_sched_barrier(0);
  const double ih[3] = {ihx, ihy, ihz};
  double acc[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};  // [i][j]
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const double w = in[b] ? pv[b] : 0.0;
    const double tr = ev[b][0] + ev[b][1] + ev[b][2];
    double S[3][3];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      const double s = w * (2.0 * mu * ev[b][m] + (m < 3 ? lam * tr : 0.0));
      S[kVi[m]][kVj[m]] = s;
      S[kVj[m]][kVi[m]] = s;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int side = (b >> a) & 1;  // the cell lies on the + side of the node along a
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c][a] += side ? S[c][a] : -S[c][a];
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
    fp[c * g.nn + id] = -0.25 * (acc[c][0] * ih[0] + acc[c][1] * ih[1] + acc[c][2] * ih[2]);
}

// Radial return (linear combined hardening) of every cell for the strain of
// u: one thread per cell; the state is rewritten only where the cell yields.
// Counts the yielding cells (integer sum per block, one atomic per block).
__global__ __launch_bounds__(kBlock) void k_return_map(Geom g, double mu, double sy, double hb,
                                                      double theta, double ihx, double ihy,
                                                      double ihz, const double *__restrict__ u,
                                                      double *__restrict__ ep,
                                                      double *__restrict__ alpha,
                                                      double *__restrict__ beta,
                                                      int *__restrict__ count) {
  __shared__ int wcount[kBlock / 64];
  const int64_t cid = (int64_t)xcd_block() * kBlock + threadIdx.x;
  bool yielded = false;
  if (cid < g.nc) {
    int cx, cy, cz;
    cell_ijk(g, cid, cx, cy, cz);
    const int64_t nc = g.nc;
    // corner nodes: un[b][c] at node (cx + b0, cy + b1, cz + b2)
    double un[8][3];
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int64_t q = (cx + (b & 1)) + (int64_t)g.nx * ((cy + ((b >> 1) & 1)) +
                                                         (int64_t)g.ny * (cz + (b >> 2)));
#pragma unroll
      for (int c = 0; c < 3; ++c) un[b][c] = u[c * g.nn + q];
    }
    double e0[6], b0[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      e0[m] = ep[m * nc + cid];
      b0[m] = beta[m * nc + cid];
    }
    const double a0 = alpha[cid];
    __builtin_amdgcn_sched_barrier(0);
    // cell gradient G[c][l]: mean over the four cell edges along l
    const double ih[3] = {ihx, ihy, ihz};
    double G[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < 8; ++b)
          if ((b >> l) & 1) s += un[b][c] - un[b ^ (1 << l)][c];
        G[c][l] = 0.25 * s * ih[l];
      }
    // eta_trial = 2 mu dev(eps - eps_p) - beta
    double ee[6];
#pragma unroll
    for (int m = 0; m < 6; ++m)
      ee[m] = 0.5 * (G[kVi[m]][kVj[m]] + G[kVj[m]][kVi[m]]) - e0[m];
    const double tr3 = (ee[0] + ee[1] + ee[2]) / 3.0;
    double eta[6], n2 = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      eta[m] = 2.0 * mu * (ee[m] - (m < 3 ? tr3 : 0.0)) - b0[m];
      n2 += (m < 3 ? 1.0 : 2.0) * eta[m] * eta[m];
    }
    const double nrm = sqrt(n2);
    const double r23 = sqrt(2.0 / 3.0);
    const double ftrial = nrm - r23 * (sy + theta * hb * a0);
    if (ftrial > 0.0) {
      yielded = true;
      const double dg = ftrial / (2.0 * mu + (2.0 / 3.0) * hb);
      const double kb = (2.0 / 3.0) * (1.0 - theta) * hb * dg;
#pragma unroll
      for (int m = 0; m < 6; ++m) {
        const double nm = eta[m] / nrm;
        ep[m * nc + cid] = e0[m] + dg * nm;
        beta[m * nc + cid] = b0[m] + kb * nm;
      }
      alpha[cid] = a0 + r23 * dg;
    }
  }
  if (count) {
    const uint64_t ball = __ballot(yielded);
    if ((threadIdx.x & 63) == 0) wcount[threadIdx.x >> 6] = __popcll(ball);
    __syncthreads();
    if (threadIdx.x == 0) {
      int s = 0;
      for (int w = 0; w < kBlock / 64; ++w) s += wcount[w];
      if (s) atomicAdd(count, s);
    }
  }
}

}  // namespace

hipError_t launch_plastic_source(const Level &L, double lam, double mu, const double *eps_p,
                                 double *fp, hipStream_t st) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_plastic_source, dim3(grid_blocks(L.g.nn)), dim3(kBlock), 0, st, L.g, lam,
                     mu, 1.0 / L.h[0], 1.0 / L.h[1], 1.0 / L.h[2], L.psi64, eps_p, fp);
  return hipGetLastError();
}

hipError_t launch_return_map(const Level &L, double mu, double sigma_y, double hbar, double theta,
                             const double *u, double *eps_p, double *alpha, double *beta,
                             int *count, hipStream_t st) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_return_map, dim3(grid_blocks(L.g.nc)), dim3(kBlock), 0, st, L.g, mu,
                     sigma_y, hbar, theta, 1.0 / L.h[0], 1.0 / L.h[1], 1.0 / L.h[2], u, eps_p,
                     alpha, beta, count);
  return hipGetLastError();
}

}  // namespace sbm
