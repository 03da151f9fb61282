// sbm_bottom.h -- the Jacobi-preconditioned CG of the bottom level in one
// workgroup (shared by the bottom kernel and the one-workgroup tail).
#pragma once

#include "sbm_device.h"

namespace sbm {

// The bottom grid is small (a few to a few hundred nodes), so the whole CG
// runs in one workgroup with the search direction and psi in LDS and each
// thread's share of x, r, A p in registers.  Reductions sum the per-wave
// partials in every thread in the same fixed order (one barrier each; the
// partial buffers alternate so a reduction never overwrites partials that a
// slower thread is still reading).

constexpr int kBotQ = 4;          // nodes per thread
constexpr int kBotThreads = 256;  // at most: the per-thread state stays in registers

struct BotRed {
  double *buf;  // 2 phases x 32 doubles of LDS
  int phase;
};

__device__ __forceinline__ double bot_allsum(double v, BotRed &R) {
  v = wave_sum(v);
  double *b = R.buf + 32 * R.phase;
  R.phase ^= 1;
  if ((threadIdx.x & 63) == 0) b[threadIdx.x >> 6] = v;
  __syncthreads();
  const int nw = blockDim.x >> 6;
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += b[w];
  return s;
}

// Two sums with one barrier.
__device__ __forceinline__ void bot_allsum2(double &v0, double &v1, BotRed &R) {
  v0 = wave_sum(v0);
  v1 = wave_sum(v1);
  double *b = R.buf + 32 * R.phase;
  R.phase ^= 1;
  if ((threadIdx.x & 63) == 0) {
    b[threadIdx.x >> 6] = v0;
    b[16 + (threadIdx.x >> 6)] = v1;
  }
  __syncthreads();
  const int nw = blockDim.x >> 6;
  double s0 = 0.0, s1 = 0.0;
  for (int w = 0; w < nw; ++w) {
    s0 += b[w];
    s1 += b[16 + w];
  }
  v0 = s0;
  v1 = s1;
}

// Jacobi-preconditioned CG on K_FF d = r (d from 0) with p and psi in LDS;
// r, d and the inverse diagonal in registers.  Stops when
// ||r|| <= rtol ||r0||.  Returns the iterations; d holds the increment.
template <typename T, int DIM, int Q, bool GATHER = true>
__device__ int bot_cg(const Geom &g, const Coef<T> &C, const T *psi_l, T *p_l, T (&r)[Q][3],
                      T (&d)[Q][3], const bool (&dir)[Q][3], const int (&cijk)[Q][3],
                      double rtol, int maxit, BotRed &R) {
  const int64_t n = g.nn;
  T dinv[Q][3];
  double lrr = 0.0, lrz = 0.0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t id = threadIdx.x + (int64_t)q * blockDim.x;
#pragma unroll
    for (int c = 0; c < 3; ++c) dinv[q][c] = T(0);
    if (id >= n) continue;
    T dg[3];
    node_diag<T, DIM>(g, C, psi_l, cijk[q][0], cijk[q][1], cijk[q][2], dg);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      dinv[q][c] = dir[q][c] ? T(0) : T(1) / dg[c];
      d[q][c] = T(0);
      const T z = r[q][c] * dinv[q][c];
      p_l[c * n + id] = z;
      lrr += (double)r[q][c] * (double)r[q][c];
      lrz += (double)r[q][c] * (double)z;
    }
  }
  bot_allsum2(lrr, lrz, R);
  double rr = lrr, rz = lrz;
  const double r0 = sqrt(rr);
  int it = 0;
  while (r0 > 0.0 && sqrt(rr) > rtol * r0 && it < maxit) {
    __syncthreads();  // p visible
    T ap[Q][3];
    double pap = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t id = threadIdx.x + (int64_t)q * blockDim.x;
      if (id >= n) continue;
      T out[3], dg[3];
      node_stencil<T, DIM, GATHER>(g, C, psi_l, p_l, cijk[q][0], cijk[q][1], cijk[q][2], out, dg);
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        ap[q][c] = dir[q][c] ? T(0) : out[c];
        pap += (double)p_l[c * n + id] * (double)ap[q][c];
      }
    }
    pap = bot_allsum(pap, R);  // its barrier also ends every read of p
    if (!(pap > 0.0)) break;
    const double alpha = rz / pap;
    double nrr = 0.0, nrz = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t id = threadIdx.x + (int64_t)q * blockDim.x;
      if (id >= n) continue;
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        d[q][c] = (T)((double)d[q][c] + alpha * (double)p_l[c * n + id]);
        r[q][c] = (T)((double)r[q][c] - alpha * (double)ap[q][c]);
        nrr += (double)r[q][c] * (double)r[q][c];
        nrz += (double)r[q][c] * (double)(r[q][c] * dinv[q][c]);
      }
    }
    bot_allsum2(nrr, nrz, R);
    const double beta = nrz / rz;
    rr = nrr;
    rz = nrz;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t id = threadIdx.x + (int64_t)q * blockDim.x;
      if (id >= n) continue;
#pragma unroll
      for (int c = 0; c < DIM; ++c)
        p_l[c * n + id] =
            dir[q][c] ? T(0) : (T)((double)(r[q][c] * dinv[q][c]) + beta * (double)p_l[c * n + id]);
    }
    ++it;
  }
  __syncthreads();
  return it;
}

}  // namespace sbm
