// sbm_tail.hip -- the coarsest levels of a V-cycle in one workgroup.
//
// Below a few hundred nodes per level every kernel of the V-cycle is bound
// by launch and memory latency (about 4 us each whatever its size).  The
// tail kernel runs the whole cycle from such a level down to the bottom and
// back in one workgroup with every vector of those levels in LDS: the same
// operations in the same order as the per-kernel path (pre-smoothing,
// residual, full-weighting restriction, the Jacobi-preconditioned CG bottom
// solve in FP64, multilinear prolongation, post-smoothing), with workgroup
// barriers between the steps.  A colour half-sweep computes its nodes from
// the state at its start (all new values are held in registers until every
// thread has read its neighbours), which is the frozen-copy rule of the
// per-kernel half-sweep without a second buffer.  The bottom CG runs in the
// first wave alone (reductions by DPP, no barriers).
#include <algorithm>

#include "sbm_bottom.h"
#include "sbm_internal.h"

namespace sbm {
namespace {

constexpr int kTailThreads = 512;  // threads of the tail workgroup
constexpr int kTailQ = 2;          // nodes per thread on a tail level (at most)
constexpr int kTailDenseMax = 32;  // free bottom DOF up to which the matrix rows sit in registers
constexpr int kTailDenseLds = 64;  // ... and up to which the matrix is assembled (LDS beyond 32)

// Level table of a tail, written to device memory once per problem (the
// kernel indexes it by a runtime level; as a kernel argument that would be
// copied to scratch memory).
template <typename T>
struct TailArgs {
  int nl;  // tail levels; level nl-1 is the bottom
  Geom g[kTailMaxLevels];
  Coef<T> C[kTailMaxLevels];
  Geom gb;                        // bottom level (a copy of g[nl-1])
  Coef<double> Cb;                // bottom operator in FP64
  const T *psi[kTailMaxLevels];   // psi of the levels above the bottom
  const double *psib;             // bottom psi, FP64
  int ox[kTailMaxLevels], of[kTailMaxLevels], op[kTailMaxLevels];  // LDS byte offsets
  int orr, opb, opp;  // residual scratch, bottom psi and search direction
  int ored;           // reduction buffer of the workgroup-wide bottom CG
  int oxb, ofb;       // bottom x and f (copies of ox[nl-1], of[nl-1])
  // Dense bottom (nf > 0): the bottom operator on its nf free DOF, assembled
  // once per problem; fidx[i] = c nn + node of the i-th free DOF.  nf <=
  // kTailDenseMax: rows in registers, A[i nf + j] = (K e_j)_i; otherwise the
  // matrix is copied into LDS at byte offset oA, A[j nf + i] = (K e_j)_i.
  int nf;
  int oA;
  const double *A;
  int fidx[kTailDenseLds];
};
static_assert(sizeof(TailArgs<double>) <= kTailArgBytes, "tail table too large");

// Wave-scope ordering of LDS accesses between lanes of one wave (the bottom
// CG runs in a single wave and needs no barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, int DIM, bool WIDE>
struct Tail {
  const TailArgs<T> &a;
  const TailOpts &o;
  char *sm;
  __device__ T *X(int l) const { return (T *)(sm + a.ox[l]); }
  __device__ T *F(int l) const { return (T *)(sm + a.of[l]); }
  __device__ T *P(int l) const { return (T *)(sm + a.op[l]); }
  __device__ T *R() const { return (T *)(sm + a.orr); }

  // nu sweeps of the level's smoother on X(l) with load F(l).  A Jacobi
  // sweep relaxes every node (thread items are nodes); a colour half-sweep
  // relaxes one node of each x-pair (thread items are x-pairs, as in the
  // half-sweep kernel), so every item has work.
  __device__ __forceinline__ void smooth(int l, int nu, bool reverse) const {
    // arguments are copied to registers once: every barrier below is also a
    // fence, after which values read through a pointer would be loaded again
    const Geom g = a.g[l];
    const Coef<T> C = a.C[l];
    const T *psi = P(l);
    const int jacobi = o.jacobi;
    const T omega = (T)o.omega;
    const int npx = (g.nx + 1) >> 1;
    const int nitems = jacobi ? (int)g.nn : npx * g.ny * g.nz;
    int pj[kTailQ][3];  // Jacobi: node (i, j, k); colour: (pair, j, k)
#pragma unroll
    for (int q = 0; q < kTailQ; ++q) {
      const int t = threadIdx.x + q * kTailThreads;
      pj[q][0] = pj[q][1] = pj[q][2] = 0;
      if (t >= nitems) continue;
      if (jacobi) {
        node_ijk(g, t, pj[q][0], pj[q][1], pj[q][2]);
      } else {
        const uint32_t rest = g.fpx.div((uint32_t)t);
        pj[q][0] = (int)((uint32_t)t - rest * (uint32_t)npx);
        pj[q][2] = (int)g.fny.div(rest);
        pj[q][1] = (int)(rest - (uint32_t)pj[q][2] * (uint32_t)g.ny);
      }
    }
    T *x = X(l);
    const T *f = F(l);
    for (int s = 0; s < nu; ++s) {
      for (int h = 0; h < (jacobi ? 1 : 2); ++h) {
        const int colour = reverse ? 1 - h : h;
        T nv[kTailQ][3];
        int nid[kTailQ];
#pragma unroll
        for (int q = 0; q < kTailQ; ++q) {
          const int t = threadIdx.x + q * kTailThreads;
          const int j = pj[q][1], k = pj[q][2];
          const int i = jacobi ? pj[q][0] : 2 * pj[q][0] + ((colour + j + k) & 1);
          nid[q] = (t < nitems && i < g.nx) ? i + g.nx * (j + g.ny * k) : -1;
          nv[q][0] = nv[q][1] = nv[q][2] = T(0);
          if (nid[q] >= 0) {
            T out[3], dg[3], uc[3];
            node_stencil<T, DIM, false>(g, C, psi, x, i, j, k, out, dg, uc);
            const uint32_t fb = face_bits(g, i, j, k);
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
              const T w = ((g.dmask >> c) & fb) ? T(0) : omega;
              nv[q][c] = uc[c] + w * (f[c * g.nn + nid[q]] - out[c]) / dg[c];
            }
          }
        }
        __syncthreads();  // every read of the old state is done
#pragma unroll
        for (int q = 0; q < kTailQ; ++q)
          if (nid[q] >= 0)
#pragma unroll
            for (int c = 0; c < DIM; ++c) x[c * g.nn + nid[q]] = nv[q][c];
        __syncthreads();
      }
    }
  }

  // R = F(l) - K X(l) on free DOF, 0 on displacement DOF.
  __device__ __forceinline__ void residual(int l) const {
    const Geom g = a.g[l];
    const Coef<T> C = a.C[l];
    for (int id = threadIdx.x; id < g.nn; id += kTailThreads) {
      int i, j, k;
      node_ijk(g, id, i, j, k);
      const uint32_t fb = face_bits(g, i, j, k);
      T out[3], dg[3];
      node_stencil<T, DIM, false>(g, C, P(l), X(l), i, j, k, out, dg);
#pragma unroll
      for (int c = 0; c < DIM; ++c)
        R()[c * g.nn + id] = ((g.dmask >> c) & fb) ? T(0) : F(l)[c * g.nn + id] - out[c];
    }
    __syncthreads();
  }

  // F(l+1) = R r (full weighting, as the restriction kernel), X(l+1) = 0.
  __device__ __forceinline__ void restrict_to(int l) const {
    const Geom gf = a.g[l], gc = a.g[l + 1];
    for (int id = threadIdx.x; id < gc.nn; id += kTailThreads) {
      int I, J, K;
      node_ijk(gc, id, I, J, K);
      T acc[3] = {T(0), T(0), T(0)};
      constexpr int ZLO = (DIM == 3) ? -1 : 0, ZHI = (DIM == 3) ? 1 : 0;
      const T *r = R();
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
            const int q = (okx ? fi : 2 * I) + gf.nx * (fjc + gf.ny * fkc);
#pragma unroll
            for (int c = 0; c < DIM; ++c) acc[c] += w * r[c * gf.nn + q];
          }
        }
      }
      const T scale = (DIM == 3) ? T(0.125) : T(0.25);
      const uint32_t fb = face_bits(gc, I, J, K);
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        F(l + 1)[c * gc.nn + id] = ((gc.dmask >> c) & fb) ? T(0) : acc[c] * scale;
        X(l + 1)[c * gc.nn + id] = T(0);
      }
    }
    __syncthreads();
  }

  // X(l) += P X(l+1) on free DOF (corners summed in z, y, x order).
  __device__ __forceinline__ void prolong_from(int l) const {
    const Geom gf = a.g[l], gc = a.g[l + 1];
    for (int id = threadIdx.x; id < gf.nn; id += kTailThreads) {
      int i, j, k;
      node_ijk(gf, id, i, j, k);
      const int i0 = i >> 1, j0 = j >> 1, k0 = k >> 1;
      const bool oi = (i & 1) != 0, oj = (j & 1) != 0, ok = DIM == 3 && (k & 1) != 0;
      const T w = T(1) / T((oi ? 2 : 1) * (oj ? 2 : 1) * (ok ? 2 : 1));
      const T *e = X(l + 1);
      T acc[3] = {T(0), T(0), T(0)};
#pragma unroll
      for (int b = 0; b < (DIM == 3 ? 2 : 1); ++b)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int o = 0; o < 2; ++o) {
            if ((b && !ok) || (q && !oj) || (o && !oi)) continue;
            const int n = (i0 + o) + gc.nx * ((j0 + q) + gc.ny * (k0 + b));
#pragma unroll
            for (int c = 0; c < DIM; ++c) acc[c] += e[c * gc.nn + n];
          }
      const uint32_t fb = face_bits(gf, i, j, k);
#pragma unroll
      for (int c = 0; c < DIM; ++c)
        if (!((gf.dmask >> c) & fb)) X(l)[c * gf.nn + id] += w * acc[c];
    }
    __syncthreads();
  }

  // Bottoms over one wave of nodes: the workgroup-wide CG of the bottom
  // kernel (node t on thread t, reductions through LDS and barriers).
  __device__ __forceinline__ void bottom_wide(int *iters) const {
    const Geom &g = a.gb;
    const int n = (int)g.nn, id = threadIdx.x;
    T *xb = (T *)(sm + a.oxb);
    const T *fb_ = (const T *)(sm + a.ofb);
    BotRed R{(double *)(sm + a.ored), 0};
    double r[1][3] = {{0.0, 0.0, 0.0}}, d[1][3] = {{0.0, 0.0, 0.0}};
    bool dir[1][3] = {{true, true, true}};
    int cijk[1][3] = {{0, 0, 0}};
    if (id < n) {
      node_ijk(g, id, cijk[0][0], cijk[0][1], cijk[0][2]);
      const uint32_t fb = face_bits(g, cijk[0][0], cijk[0][1], cijk[0][2]);
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        dir[0][c] = ((g.dmask >> c) & fb) != 0u;
        r[0][c] = dir[0][c] ? 0.0 : (double)fb_[c * n + id];
      }
    }
    const int it = bot_cg<double, DIM, 1, false>(g, a.Cb, (const double *)(sm + a.opb),
                                                 (double *)(sm + a.opp), r, d, dir, cijk, o.rtol,
                                                 o.maxit, R);
    if (id < n)
#pragma unroll
      for (int c = 0; c < DIM; ++c) xb[c * n + id] = (T)d[0][c];
    if (id == 0 && iters) *iters = it;
    __syncthreads();
  }

  // The same CG on the assembled bottom matrix: lane i of the first wave
  // holds row i (free DOF i) in registers and the search direction is a
  // dense LDS vector over the free DOF, so A p is nf fused multiply-adds per
  // lane instead of a stencil evaluation.
  __device__ __forceinline__ void bottom_dense(int *iters) const {
    const int nb = (int)a.gb.nn;
    T *xb = (T *)(sm + a.oxb);
    const T *fb_ = (const T *)(sm + a.ofb);
    if (threadIdx.x < 64) {
      const int lane = threadIdx.x, nf = a.nf;
      const double rtol = o.rtol;
      const int maxit = o.maxit;
      const bool on = lane < nf;
      double *p = (double *)(sm + a.opp);
      double row[kTailDenseMax];
#pragma unroll
      for (int j = 0; j < kTailDenseMax; ++j) row[j] = (on && j < nf) ? a.A[lane * nf + j] : 0.0;
      const int fi = on ? a.fidx[lane] : 0;
      const double r0v = on ? (double)fb_[fi] : 0.0;
      const double dinv = on ? 1.0 / a.A[lane * nf + lane] : 0.0;
      double r = r0v, d = 0.0;
      double z = r * dinv;
      // p is padded with zeros to kTailDenseMax entries (as the rows are), so
      // A p needs no bounds tests: all its LDS reads go out together
      if (lane < kTailDenseMax) p[lane] = on ? z : 0.0;
      double rr = wave_sum(r * r), rz = wave_sum(r * z);
      const double r0 = sqrt(rr);
      int it = 0;
      while (r0 > 0.0 && sqrt(rr) > rtol * r0 && it < maxit) {
        wave_sync();  // p visible to every lane
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
        for (int j = 0; j < kTailDenseMax; j += 4) {
          s0 += row[j] * p[j];
          s1 += row[j + 1] * p[j + 1];
          s2 += row[j + 2] * p[j + 2];
          s3 += row[j + 3] * p[j + 3];
        }
        const double ap = (s0 + s1) + (s2 + s3);
        const double pl = on ? p[lane] : 0.0;
        const double pap = wave_sum(pl * ap);
        if (!(pap > 0.0)) break;
        const double alpha = rz / pap;
        d += alpha * pl;
        r -= alpha * ap;
        z = r * dinv;
        const double nrr = wave_sum(r * r), nrz = wave_sum(r * z);
        const double beta = nrz / rz;
        rr = nrr;
        rz = nrz;
        wave_sync();  // every lane has read p
        if (on) p[lane] = z + beta * pl;
        ++it;
      }
      if (on) xb[fi] = (T)d;  // displacement DOF stay 0 (zeroed by the restriction)
      if (lane == 0 && iters) *iters = it;
    }
    (void)nb;
    __syncthreads();
  }

  // The dense CG for kTailDenseMax < nf <= kTailDenseLds: the matrix is
  // copied into LDS (column j at stride kTailDenseLds, rows past nf zero) and
  // lane i reads row i one column at a time; the search direction stays in
  // the lanes' registers and entry j is broadcast from lane j (readlane), so
  // A p is the same zero-padded sum of 64 products as in the register version.
  __device__ __forceinline__ void bottom_dense_lds(int *iters) const {
    T *xb = (T *)(sm + a.oxb);
    const T *fb_ = (const T *)(sm + a.ofb);
    double *As = (double *)(sm + a.oA);
    const int nf = a.nf;
    for (int q = threadIdx.x; q < kTailDenseLds * kTailDenseLds; q += kTailThreads) {
      const int j = q / kTailDenseLds, i = q - j * kTailDenseLds;
      As[q] = (i < nf && j < nf) ? a.A[j * nf + i] : 0.0;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      const int lane = threadIdx.x;
      const double rtol = o.rtol;
      const int maxit = o.maxit;
      const bool on = lane < nf;
      const int fi = on ? a.fidx[lane] : 0;
      const double r0v = on ? (double)fb_[fi] : 0.0;
      const double dinv = on ? 1.0 / As[lane * kTailDenseLds + lane] : 0.0;
      double r = r0v, d = 0.0;
      double z = r * dinv;
      double pl = on ? z : 0.0;  // this lane's entry of the search direction
      double rr = wave_sum(r * r), rz = wave_sum(r * z);
      const double r0 = sqrt(rr);
      int it = 0;
      auto bcast = [&](int j) {
        const int lo = __builtin_amdgcn_readlane(__double2loint(pl), j);
        const int hi = __builtin_amdgcn_readlane(__double2hiint(pl), j);
        return __hiloint2double(hi, lo);
      };
      while (r0 > 0.0 && sqrt(rr) > rtol * r0 && it < maxit) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
        for (int j = 0; j < kTailDenseLds; j += 4) {
          s0 += As[j * kTailDenseLds + lane] * bcast(j);
          s1 += As[(j + 1) * kTailDenseLds + lane] * bcast(j + 1);
          s2 += As[(j + 2) * kTailDenseLds + lane] * bcast(j + 2);
          s3 += As[(j + 3) * kTailDenseLds + lane] * bcast(j + 3);
        }
        const double ap = (s0 + s1) + (s2 + s3);
        const double pap = wave_sum(pl * ap);
        if (!(pap > 0.0)) break;
        const double alpha = rz / pap;
        d += alpha * pl;
        r -= alpha * ap;
        z = r * dinv;
        const double nrr = wave_sum(r * r), nrz = wave_sum(r * z);
        const double beta = nrz / rz;
        rr = nrr;
        rz = nrz;
        pl = on ? z + beta * pl : 0.0;
        ++it;
      }
      if (on) xb[fi] = (T)d;  // displacement DOF stay 0 (zeroed by the restriction)
      if (lane == 0 && iters) *iters = it;
    }
    __syncthreads();
  }

  // X(B) = CG(K_B, F(B)) from zero, in FP64 in the first wave: Jacobi
  // preconditioning, stop at ||r|| <= rtol ||r0|| or maxit iterations.
  __device__ __forceinline__ void bottom(int *iters) const {
    if constexpr (WIDE) {
      bottom_wide(iters);
      return;
    }
    if (a.nf > kTailDenseMax) {
      bottom_dense_lds(iters);
      return;
    }
    if (a.nf > 0) {
      bottom_dense(iters);
      return;
    }
    const Geom &g = a.gb;
    const Coef<double> &Cb = a.Cb;
    const double rtol = o.rtol;
    const int maxit = o.maxit;
    T *xb = (T *)(sm + a.oxb);
    const T *fb_ = (const T *)(sm + a.ofb);
    if (threadIdx.x < 64) {
      const int lane = threadIdx.x;
      const int n = (int)g.nn;
      const double *psi = (const double *)(sm + a.opb);
      double *p = (double *)(sm + a.opp);
      double r[1][3], d[1][3], dinv[1][3];
      bool dir[1][3];
      int cijk[1][3];
      double lrr = 0.0, lrz = 0.0;
#pragma unroll
      for (int q = 0; q < 1; ++q) {
        const int id = lane + 64 * q;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          r[q][c] = d[q][c] = dinv[q][c] = 0.0;
          dir[q][c] = true;
          cijk[q][c] = 0;
        }
        if (id >= n) continue;
        node_ijk(g, id, cijk[q][0], cijk[q][1], cijk[q][2]);
        double dg[3];
        node_diag<double, DIM>(g, Cb, psi, cijk[q][0], cijk[q][1], cijk[q][2], dg);
        const uint32_t fb = face_bits(g, cijk[q][0], cijk[q][1], cijk[q][2]);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
          dir[q][c] = ((g.dmask >> c) & fb) != 0u;
          r[q][c] = dir[q][c] ? 0.0 : (double)fb_[c * n + id];
          dinv[q][c] = dir[q][c] ? 0.0 : 1.0 / dg[c];
          const double z = r[q][c] * dinv[q][c];
          p[c * n + id] = z;
          lrr += r[q][c] * r[q][c];
          lrz += r[q][c] * z;
        }
      }
      double rr = wave_sum(lrr), rz = wave_sum(lrz);
      const double r0 = sqrt(rr);
      int it = 0;
      while (r0 > 0.0 && sqrt(rr) > rtol * r0 && it < maxit) {
        wave_sync();  // p visible to every lane
        double ap[1][3];
        double pap = 0.0;
#pragma unroll
        for (int q = 0; q < 1; ++q) {
          const int id = lane + 64 * q;
#pragma unroll
          for (int c = 0; c < 3; ++c) ap[q][c] = 0.0;
          if (id >= n) continue;
          double out[3], dg[3];
          node_stencil<double, DIM, false>(g, Cb, psi, p, cijk[q][0], cijk[q][1], cijk[q][2],
                                           out, dg);
#pragma unroll
          for (int c = 0; c < DIM; ++c) {
            ap[q][c] = dir[q][c] ? 0.0 : out[c];
            pap += p[c * n + id] * ap[q][c];
          }
        }
        pap = wave_sum(pap);
        if (!(pap > 0.0)) break;
        const double alpha = rz / pap;
        double nrr = 0.0, nrz = 0.0;
#pragma unroll
        for (int q = 0; q < 1; ++q) {
          const int id = lane + 64 * q;
          if (id >= n) continue;
#pragma unroll
          for (int c = 0; c < DIM; ++c) {
            d[q][c] += alpha * p[c * n + id];
            r[q][c] -= alpha * ap[q][c];
            nrr += r[q][c] * r[q][c];
            nrz += r[q][c] * (r[q][c] * dinv[q][c]);
          }
        }
        nrr = wave_sum(nrr);
        nrz = wave_sum(nrz);
        const double beta = nrz / rz;
        rr = nrr;
        rz = nrz;
        wave_sync();  // every lane has read p
#pragma unroll
        for (int q = 0; q < 1; ++q) {
          const int id = lane + 64 * q;
          if (id >= n) continue;
#pragma unroll
          for (int c = 0; c < DIM; ++c)
            p[c * n + id] = dir[q][c] ? 0.0 : r[q][c] * dinv[q][c] + beta * p[c * n + id];
        }
        ++it;
      }
#pragma unroll
      for (int q = 0; q < 1; ++q) {
        const int id = lane + 64 * q;
        if (id >= n) continue;
#pragma unroll
        for (int c = 0; c < DIM; ++c) xb[c * n + id] = (T)d[q][c];
      }
      if (lane == 0 && iters) *iters = it;
    }
    __syncthreads();
  }
};

template <typename T, int DIM, bool WIDE>
__global__ __launch_bounds__(kTailThreads) void k_tail(const TailArgs<T> *__restrict__ ap,
                                                       TailOpts o, T *x, const T *__restrict__ f,
                                                       int *iters) {
  const TailArgs<T> &a = *ap;
  extern __shared__ double smem[];
  const Tail<T, DIM, WIDE> t{a, o, (char *)smem};
  const int B = a.nl - 1;
  for (int l = 0; l < B; ++l)
    for (int q = threadIdx.x; q < a.g[l].nc; q += kTailThreads) t.P(l)[q] = a.psi[l][q];
  {
    double *pb = (double *)((char *)smem + a.opb);
    for (int q = threadIdx.x; q < a.gb.nc; q += kTailThreads) pb[q] = a.psib[q];
  }
  const int n0 = DIM * (int)a.g[0].nn;
  for (int q = threadIdx.x; q < n0; q += kTailThreads) {
    t.X(0)[q] = x[q];
    t.F(0)[q] = f[q];
  }
  __syncthreads();
  for (int l = 0; l < B; ++l) {
    t.smooth(l, o.nu_pre, false);
    t.residual(l);
    t.restrict_to(l);
  }
  t.bottom(iters);
  for (int l = B - 1; l >= 0; --l) {
    t.prolong_from(l);
    t.smooth(l, o.nu_post, o.reverse != 0);
  }
  for (int q = threadIdx.x; q < n0; q += kTailThreads) x[q] = t.X(0)[q];
}

// Assembles the dense bottom matrix: column j is K applied to the unit
// vector of free DOF j (the stencil of the bottom level, FP64), read at every
// free DOF.  One wave; once per problem.
template <typename T, int DIM>
__global__ __launch_bounds__(64) void k_tail_assemble(const TailArgs<T> *__restrict__ ap) {
  const TailArgs<T> &a = *ap;
  __shared__ double p[3 * kTailWaveBottom];
  const Geom g = a.gb;
  const Coef<double> Cb = a.Cb;
  const double *psib = a.psib;
  const int nb = (int)g.nn, nf = a.nf, lane = threadIdx.x;
  double *A = const_cast<double *>(a.A);
  for (int q = lane; q < 3 * kTailWaveBottom; q += 64) p[q] = 0.0;
  int i = 0, j = 0, k = 0, c = 0;
  if (lane < nf) {
    c = a.fidx[lane] / nb;
    node_ijk(g, a.fidx[lane] - c * nb, i, j, k);
  }
  wave_sync();
  for (int col = 0; col < nf; ++col) {
    if (lane == 0) p[a.fidx[col]] = 1.0;
    wave_sync();
    if (lane < nf) {
      double out[3], dg[3];
      node_stencil<double, DIM, false>(g, Cb, psib, p, i, j, k, out, dg);
      if (nf > kTailDenseMax) A[col * nf + lane] = out[c];  // column-major (LDS copy)
      else A[lane * nf + col] = out[c];
    }
    wave_sync();
    if (lane == 0) p[a.fidx[col]] = 0.0;
  }
}

template <typename T>
const T *tail_psi(const Level &L);
template <>
const double *tail_psi<double>(const Level &L) { return L.psi64; }
template <>
const float *tail_psi<float>(const Level &L) { return L.psi32; }
template <typename T>
const Coef<T> &tail_coef(const Level &L);
template <>
const Coef<double> &tail_coef<double>(const Level &L) { return L.c64; }
template <>
const Coef<float> &tail_coef<float>(const Level &L) { return L.c32; }

// LDS layout of the tail from level l0 (levels l0..nlev-1); 0 if it does not
// apply (a level above the bottom with more nodes than threads, a bottom of
// more nodes than threads, fewer than two levels, too many levels).
template <typename T>
size_t tail_layout(const std::vector<Level> &L, int l0, TailArgs<T> *a,
                   const double *dense_A = nullptr, size_t lds_max = 0) {
  const int nlev = (int)L.size();
  const int nl = nlev - l0;
  if (nl < 2 || nl > kTailMaxLevels) return 0;
  const int B = nlev - 1;
  if (L[B].g.nn > kTailThreads) return 0;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 15) & ~(size_t)15;
    return (int)o;
  };
  const int d = L[B].g.dim;
  TailArgs<T> t{};
  t.nl = nl;
  for (int q = 0; q < nl; ++q) {
    const Level &V = L[l0 + q];
    if (q < nl - 1 && V.g.nn > kTailThreads * kTailQ) return 0;
    t.g[q] = V.g;
    t.C[q] = tail_coef<T>(V);
    t.ox[q] = take(sizeof(T) * d * V.g.nn);
    t.of[q] = take(sizeof(T) * d * V.g.nn);
    if (q < nl - 1) {
      t.psi[q] = tail_psi<T>(V);
      t.op[q] = take(sizeof(T) * V.g.nc);
    }
  }
  t.orr = take(sizeof(T) * d * L[l0].g.nn);
  t.opb = take(sizeof(double) * L[B].g.nc);
  t.opp = take(sizeof(double) * std::max<int64_t>(d * L[B].g.nn, kTailDenseLds));
  t.ored = take(sizeof(double) * 64);
  t.gb = L[B].g;
  t.oxb = t.ox[nl - 1];
  t.ofb = t.of[nl - 1];
  t.Cb = L[B].c64;
  t.psib = L[B].psi64;
  // free DOF of the bottom (component-major), for the dense bottom matrix
  const Geom &gb = L[B].g;
  int nf = 0;
  for (int c = 0; c < d; ++c)
    for (int n = 0; n < (int)gb.nn; ++n) {
      const int i = n % gb.nx, j = (n / gb.nx) % gb.ny, k = n / (gb.nx * gb.ny);
      uint32_t fb = (i == 0 ? 1u : 0u) | (i == gb.nx - 1 ? 8u : 0u) | (j == 0 ? 64u : 0u) |
                    (j == gb.ny - 1 ? 512u : 0u);
      if (d == 3) fb |= (k == 0 ? 4096u : 0u) | (k == gb.nz - 1 ? 32768u : 0u);
      if ((gb.dmask >> c) & fb) continue;
      if (nf < kTailDenseLds) t.fidx[nf] = c * (int)gb.nn + n;
      ++nf;
    }
  t.nf = (dense_A && nf <= kTailDenseLds && gb.nn <= kTailWaveBottom) ? nf : 0;
  t.oA = -1;
  if (t.nf > kTailDenseMax) {
    if (off + sizeof(double) * kTailDenseLds * kTailDenseLds <= lds_max)
      t.oA = take(sizeof(double) * kTailDenseLds * kTailDenseLds);
    else
      t.nf = 0;  // no room in LDS: the stencil CG
  }
  t.A = dense_A;
  if (a) *a = t;
  return off;
}

}  // namespace

int tail_level(const std::vector<Level> &L, int precision, size_t lds_max) {
  // the highest level whose tail fits
  for (int l0 = 0; l0 + 1 < (int)L.size(); ++l0) {
    const size_t by = precision == 1 ? tail_layout<float>(L, l0, nullptr)
                                     : tail_layout<double>(L, l0, nullptr);
    if (by > 0 && by <= lds_max) return l0;
  }
  return -1;
}

hipError_t tail_upload(const std::vector<Level> &L, int precision, int l0, void *dev,
                       double *dense_A, size_t lds_max, size_t *lds_bytes, hipStream_t st) {
  hipError_t e;
  const int dim = L[0].g.dim;
  (void)hipGetLastError();
  if (precision == 1) {
    TailArgs<float> a{};
    *lds_bytes = tail_layout<float>(L, l0, &a, dense_A, lds_max);
    if (*lds_bytes == 0) return hipErrorInvalidValue;
    if ((e = hipMemcpyAsync(dev, &a, sizeof(a), hipMemcpyHostToDevice, st)) != hipSuccess) return e;
    if (a.nf > 0) {
      const TailArgs<float> *da = (const TailArgs<float> *)dev;
      if (dim == 3) hipLaunchKernelGGL((k_tail_assemble<float, 3>), dim3(1), dim3(64), 0, st, da);
      else hipLaunchKernelGGL((k_tail_assemble<float, 2>), dim3(1), dim3(64), 0, st, da);
    }
  } else {
    TailArgs<double> a{};
    *lds_bytes = tail_layout<double>(L, l0, &a, dense_A, lds_max);
    if (*lds_bytes == 0) return hipErrorInvalidValue;
    if ((e = hipMemcpyAsync(dev, &a, sizeof(a), hipMemcpyHostToDevice, st)) != hipSuccess) return e;
    if (a.nf > 0) {
      const TailArgs<double> *da = (const TailArgs<double> *)dev;
      if (dim == 3) hipLaunchKernelGGL((k_tail_assemble<double, 3>), dim3(1), dim3(64), 0, st, da);
      else hipLaunchKernelGGL((k_tail_assemble<double, 2>), dim3(1), dim3(64), 0, st, da);
    }
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return hipStreamSynchronize(st);  // the table lives on this stack frame
}

template <typename T>
hipError_t launch_tail(int dim, bool wide_bottom, const void *dev, size_t lds_bytes,
                       T *x, const T *f, const TailOpts &o, int *iters, hipStream_t st) {
  const TailArgs<T> *a = (const TailArgs<T> *)dev;
  const dim3 grid(1), block(kTailThreads);
  (void)hipGetLastError();
  if (dim == 3) {
    if (wide_bottom)
      hipLaunchKernelGGL((k_tail<T, 3, true>), grid, block, lds_bytes, st, a, o, x, f, iters);
    else
      hipLaunchKernelGGL((k_tail<T, 3, false>), grid, block, lds_bytes, st, a, o, x, f, iters);
  } else {
    if (wide_bottom)
      hipLaunchKernelGGL((k_tail<T, 2, true>), grid, block, lds_bytes, st, a, o, x, f, iters);
    else
      hipLaunchKernelGGL((k_tail<T, 2, false>), grid, block, lds_bytes, st, a, o, x, f, iters);
  }
  return hipGetLastError();
}

template hipError_t launch_tail<double>(int, bool, const void *, size_t, double *, const double *,
                                        const TailOpts &, int *, hipStream_t);
template hipError_t launch_tail<float>(int, bool, const void *, size_t, float *, const float *,
                                       const TailOpts &, int *, hipStream_t);

}  // namespace sbm
