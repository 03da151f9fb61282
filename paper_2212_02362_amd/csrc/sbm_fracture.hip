// sbm_fracture.hip -- hybrid phase-field fracture on the finest grid (Sec.
// 3.2, eqs. PFFracture and PFFractureGL): the crack driving force of every
// cell and the explicit Ginzburg-Landau step of the crack field.  The elastic
// equilibrium of the model is the SBM solve with psi = g(c) + eta.
//
// Per cell, from the strain eps = sym(G u) (G: the cell gradient of the
// corner nodes, the mean difference quotient over the cell's edges along each
// axis; plane strain in 2D):
//   principal strains e_i (2D: closed form of the in-plane pair; 3D: cyclic
//   Jacobi rotations), W0+- = lambda/2 (sum <e_i>+-)^2 + mu sum <e_i>+-^2,
//   H <- max(H, W0+), intact <- W0+ < W0-.
// The crack step, with g(c) = 4c^3 - 3c^4, w = 1 - g:
//   c <- c - dt M [ g'(c) H - Gc (2 xi lap(c) + w'(c) / (2 xi)) ], projected
//   onto [0, 1] (the range of the crack field), c = 1 where intact, lap the
//   2d+1-point cell Laplacian with zero flux across the box faces;
//   psi = g(c) + eta for the next solve.
#include "sbm_internal.h"

namespace sbm {
namespace {

// Principal values of a symmetric 3x3 matrix by cyclic Jacobi rotations
// (each rotation zeroes one off-diagonal pair; a few sweeps converge).
__device__ __forceinline__ void jacobi_eigs3(double a[3][3], double e[3]) {
  for (int sweep = 0; sweep < 12; ++sweep) {
    if (a[0][1] == 0.0 && a[0][2] == 0.0 && a[1][2] == 0.0) break;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = p + 1; q < 3; ++q) {
        if (a[p][q] == 0.0) continue;
        const double th = 0.5 * (a[q][q] - a[p][p]) / a[p][q];
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double x = a[k][p], y = a[k][q];
          a[k][p] = cs * x - sn * y;
          a[k][q] = sn * x + cs * y;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double x = a[p][k], y = a[q][k];
          a[p][k] = cs * x - sn * y;
          a[q][k] = sn * x + cs * y;
        }
      }
  }
  e[0] = a[0][0];
  e[1] = a[1][1];
  e[2] = a[2][2];
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_crack_drive(Geom g, double lam, double mu, double ihx,
                                                       double ihy, double ihz,
                                                       const double *__restrict__ u,
                                                       double *__restrict__ H,
                                                       uint8_t *__restrict__ intact) {
  const int64_t cid = (int64_t)xcd_block() * kBlock + threadIdx.x;
  if (cid >= g.nc) return;
  int cx, cy, cz;
  cell_ijk(g, cid, cx, cy, cz);
  if (DIM == 2) cz = 0;
  constexpr int NB = 1 << DIM;
  double un[NB][DIM];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int64_t q = (cx + (b & 1)) + (int64_t)g.nx * ((cy + ((b >> 1) & 1)) +
                                                       (int64_t)g.ny * (DIM == 3 ? cz + (b >> 2) : 0));
#pragma unroll
    for (int c = 0; c < DIM; ++c) un[b][c] = u[c * g.nn + q];
  }
  const double h0 = H[cid];
  const double ih[3] = {ihx, ihy, ihz};
  double eps[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  double G[3][3];
#pragma unroll
  for (int c = 0; c < DIM; ++c)
#pragma unroll
    for (int l = 0; l < DIM; ++l) {
      double s = 0.0;
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if ((b >> l) & 1) s += un[b][c] - un[b ^ (1 << l)][c];
      G[c][l] = s / (double)(NB / 2) * ih[l];
    }
#pragma unroll
  for (int k = 0; k < DIM; ++k)
#pragma unroll
    for (int l = 0; l < DIM; ++l) eps[k][l] = 0.5 * (G[k][l] + G[l][k]);
  double e[3] = {0.0, 0.0, 0.0};
  if (DIM == 2) {
    const double m = 0.5 * (eps[0][0] + eps[1][1]);
    const double d = 0.5 * (eps[0][0] - eps[1][1]);
    const double r = sqrt(d * d + eps[0][1] * eps[0][1]);
    e[0] = m + r;
    e[1] = m - r;
  } else {
    jacobi_eigs3(eps, e);
  }
  double tp = 0.0, tm = 0.0, sp = 0.0, sm = 0.0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    const double ep = e[i] > 0.0 ? e[i] : 0.0, em = e[i] < 0.0 ? e[i] : 0.0;
    tp += ep;
    tm += em;
    sp += ep * ep;
    sm += em * em;
  }
  const double wp = 0.5 * lam * tp * tp + mu * sp, wm = 0.5 * lam * tm * tm + mu * sm;
  if (wp > h0) H[cid] = wp;
  intact[cid] = wp < wm ? 1 : 0;
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_phase_step(Geom g, double ihx2, double ihy2,
                                                      double ihz2, const double *__restrict__ c0,
                                                      const double *__restrict__ H,
                                                      const uint8_t *__restrict__ intact,
                                                      double Gc, double xi, double M, double dt,
                                                      double eta, double *__restrict__ c1,
                                                      double *__restrict__ psi) {
  const int64_t cid = (int64_t)xcd_block() * kBlock + threadIdx.x;
  if (cid >= g.nc) return;
  int cx, cy, cz;
  cell_ijk(g, cid, cx, cy, cz);
  const int64_t sy = g.cx, sz = (int64_t)g.cx * g.cy;
  // neighbours clamped at the box faces: a missing neighbour is the cell
  // itself, i.e. zero flux across the face
  const double cc = c0[cid];
  const double xm = c0[cid - (cx > 0 ? 1 : 0)], xp = c0[cid + (cx < g.cx - 1 ? 1 : 0)];
  const double ym = c0[cid - (cy > 0 ? sy : 0)], yp = c0[cid + (cy < g.cy - 1 ? sy : 0)];
  double lap = (xp - 2.0 * cc + xm) * ihx2 + (yp - 2.0 * cc + ym) * ihy2;
  if (DIM == 3) {
    const double zm = c0[cid - (cz > 0 ? sz : 0)], zp = c0[cid + (cz < g.cz - 1 ? sz : 0)];
    lap += (zp - 2.0 * cc + zm) * ihz2;
  }
  const double hv = H[cid];
  const bool keep = intact[cid] != 0;
  const double gp = 12.0 * cc * cc - 12.0 * cc * cc * cc;
  const double wpr = -gp;
  double cn = cc - dt * M * (gp * hv - Gc * (2.0 * xi * lap + wpr / (2.0 * xi)));
  // the crack field lives in [0, 1]: project (comparisons keep a NaN)
  cn = cn < 0.0 ? 0.0 : cn;
  cn = cn > 1.0 ? 1.0 : cn;
  if (keep) cn = 1.0;
  c1[cid] = cn;
  psi[cid] = 4.0 * cn * cn * cn - 3.0 * cn * cn * cn * cn + eta;
}

}  // namespace

hipError_t launch_crack_drive(const Level &L, double lam, double mu, const double *u, double *H,
                              uint8_t *intact, hipStream_t st) {
  (void)hipGetLastError();
  const dim3 grid(grid_blocks(L.g.nc)), block(kBlock);
  const double ihz = L.g.dim == 3 ? 1.0 / L.h[2] : 0.0;
  if (L.g.dim == 3)
    hipLaunchKernelGGL(k_crack_drive<3>, grid, block, 0, st, L.g, lam, mu, 1.0 / L.h[0],
                       1.0 / L.h[1], ihz, u, H, intact);
  else
    hipLaunchKernelGGL(k_crack_drive<2>, grid, block, 0, st, L.g, lam, mu, 1.0 / L.h[0],
                       1.0 / L.h[1], ihz, u, H, intact);
  return hipGetLastError();
}

hipError_t launch_phase_step(const Level &L, const double *c0, const double *H,
                             const uint8_t *intact, double Gc, double xi, double M, double dt,
                             double eta, double *c1, double *psi, hipStream_t st) {
  (void)hipGetLastError();
  const dim3 grid(grid_blocks(L.g.nc)), block(kBlock);
  const double ihx2 = 1.0 / (L.h[0] * L.h[0]), ihy2 = 1.0 / (L.h[1] * L.h[1]);
  const double ihz2 = L.g.dim == 3 ? 1.0 / (L.h[2] * L.h[2]) : 0.0;
  if (L.g.dim == 3)
    hipLaunchKernelGGL(k_phase_step<3>, grid, block, 0, st, L.g, ihx2, ihy2, ihz2, c0, H, intact,
                       Gc, xi, M, dt, eta, c1, psi);
  else
    hipLaunchKernelGGL(k_phase_step<2>, grid, block, 0, st, L.g, ihx2, ihy2, ihz2, c0, H, intact,
                       Gc, xi, M, dt, eta, c1, psi);
  return hipGetLastError();
}

}  // namespace sbm
