// sbm_traction.hip -- the load of a traction on the diffuse boundary (Sec.
// 2.1, eq. SBMLinearElasticity): the sharp-boundary traction, extended along
// the normals across the diffuse band, enters the equilibrium as
// t^0 |grad psi|.  With the outward-normal sign of K u = f, node n gets
//   f(n) = t^0(n) |grad psi(n)| + p grad psi(n),
// where p is a pressure pushing on the solid from the empty side (its
// traction -p n_out with n_out = -grad psi / |grad psi| times |grad psi|).
// psi = max(psi_raw, floor); the node gradient along axis a is the mean of
// the difference quotients of the 2^(d-1) cell pairs facing each other across
// the node along a, cells outside the box taking the value of the nearest
// cell inside (the box faces carry their own traction sources).
#include "sbm_internal.h"

namespace sbm {
namespace {

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_diffuse_traction(Geom g, double ihx, double ihy,
                                                            double ihz,
                                                            const double *__restrict__ psi_raw,
                                                            double floor_,
                                                            const double *__restrict__ t_hat,
                                                            double p, double *__restrict__ f) {
  const int64_t id = (int64_t)xcd_block() * kBlock + threadIdx.x;
  if (id >= g.nn) return;
  int i, j, k;
  node_ijk(g, id, i, j, k);
  // the 2^d cells around the node, clamped into the box; v[b] is cell
  // (i - 1 + b0, j - 1 + b1, k - 1 + b2)
  constexpr int NB = 1 << DIM;
  double v[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int x = min(max(i - 1 + (b & 1), 0), g.cx - 1);
    const int y = min(max(j - 1 + ((b >> 1) & 1), 0), g.cy - 1);
    const int z = DIM == 3 ? min(max(k - 1 + (b >> 2), 0), g.cz - 1) : 0;
    const double r = psi_raw[x + (int64_t)g.cx * (y + (int64_t)g.cy * z)];
    v[b] = r > floor_ ? r : floor_;
  }
  double tv[DIM];
  if (t_hat) {
#pragma unroll
    for (int c = 0; c < DIM; ++c) tv[c] = t_hat[c * g.nn + id];
  }
  const double ih[3] = {ihx, ihy, ihz};
  double grad[DIM];
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < NB; ++b)
      if ((b >> a) & 1) s += v[b] - v[b ^ (1 << a)];
    grad[a] = s * (1.0 / (NB / 2)) * ih[a];
  }
  double mag = 0.0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) mag += grad[a] * grad[a];
  mag = sqrt(mag);
#pragma unroll
  for (int c = 0; c < DIM; ++c) f[c * g.nn + id] = (t_hat ? tv[c] * mag : 0.0) + p * grad[c];
}

}  // namespace

hipError_t launch_diffuse_traction(const Level &L, const double *psi_raw, double floor_,
                                   const double *t_hat, double p, double *f, hipStream_t st) {
  (void)hipGetLastError();
  const dim3 grid(grid_blocks(L.g.nn)), block(kBlock);
  const double ihz = L.g.dim == 3 ? 1.0 / L.h[2] : 0.0;
  if (L.g.dim == 3)
    hipLaunchKernelGGL(k_diffuse_traction<3>, grid, block, 0, st, L.g, 1.0 / L.h[0],
                       1.0 / L.h[1], ihz, psi_raw, floor_, t_hat, p, f);
  else
    hipLaunchKernelGGL(k_diffuse_traction<2>, grid, block, 0, st, L.g, 1.0 / L.h[0],
                       1.0 / L.h[1], ihz, psi_raw, floor_, t_hat, p, f);
  return hipGetLastError();
}

}  // namespace sbm
