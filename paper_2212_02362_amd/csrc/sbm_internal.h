// sbm_internal.h -- host-side declarations shared by the kernel launchers
// (sbm_kernels.hip) and the solver / C ABI (sbm_solver.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/sbm.h"
#include "sbm_device.h"

namespace sbm {

// Traction source table: t[F][k] (0 where the face/component is not a
// traction condition) and 1/h_perp per face.
struct Traction {
  double t[6][3];
  double inv_h[6];
};

// Displacement values per face/component (used where dmask is set).
struct DispValues {
  double v[6][3];
};

struct Level {
  Geom g;
  double h[3];
  Coef<double> c64;
  Coef<float> c32;
  double *psi64 = nullptr;
  float *psi32 = nullptr;
  // FP64 vectors: level 0 uses f (load), r (residual / ping-pong); coarse
  // levels use e (correction), f (restricted residual), t (ping-pong / residual)
  double *e = nullptr, *f = nullptr, *t = nullptr;
  // FP32 vectors of the mixed cycle
  float *e32 = nullptr, *f32 = nullptr, *t32 = nullptr;
};

// Column tiles of the tiled 3D kernels: kTileX x kTileY nodes in x, y over a
// chunk of kz planes; tile id = tx + ntx (ty + nty tz).  When a level has one
// node more than a whole number of tiles along x (or y) -- the 2^n + 1 node
// counts of the benchmark grids -- the full launches stop the tiles before the
// last node column (row) and give those face nodes to `nface` node-parallel
// blocks launched after the tiles (xface / yface say which); a tile holding that single
// column would cost a whole tile's stencil rounds for 1/64 of the work.
constexpr int kTileX = 64, kTileY = 8;
// Chunks along z: with nzc > 0 (launches over a whole level) chunk tz holds
// planes [tz nz / nzc, (tz + 1) nz / nzc), depths differing by at most one, so
// that every tile -- and every XCD's contiguous range of tiles -- carries the
// same work; with nzc == 0 (tile lists, per-plane block maps) chunk tz holds
// planes [tz kz, min((tz + 1) kz, nz)).  kz is the deepest chunk either way.
struct TileGeom {
  int ntx, nty, kz, ntiles;
  int xface, yface, nface;
  int nzc;
};
// Tiles of level L in chunks of kz planes (0: the default depth, chosen so
// that the whole level gives about 1536 tiles).
TileGeom tile_geom_of(const Level &L, int kz = 0);
// A subset of a level's tiles (device ids in increasing order) and the chunk
// depth they were listed with.
struct TileList {
  const int *ids = nullptr;
  int count = 0;
  int kz = 0;
};

// A node vector read by the Krylov kernels: given in memory (z), or as
// s * e with e the FP32 correction of the mixed preconditioner and s = *s
// (the scaled-back preconditioned residual, never written out in FP64).
struct ZSrc {
  const double *z = nullptr;
  const float *e = nullptr;
  const double *s = nullptr;
};

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `st` and return the launch status.
template <typename T>
hipError_t launch_apply(const Level &L, const T *psi, const Coef<T> &C, const T *u, T *y,
                        hipStream_t st);
template <typename T>
hipError_t launch_residual(const Level &L, const T *psi, const Coef<T> &C, const T *u,
                           const T *f, T *r, double *partials, hipStream_t st,
                           const uint8_t *cls = nullptr, const TileList *tl = nullptr);
hipError_t launch_residual_cast(const Level &L, const double *u, const double *f, float *r32,
                                const double *ss, hipStream_t st);
template <typename T>
hipError_t launch_jacobi(const Level &L, const T *psi, const Coef<T> &C, const T *u, const T *f,
                         T *u_out, double omega, hipStream_t st, const uint8_t *cls = nullptr);
template <typename T>
hipError_t launch_rb_half(const Level &L, const T *psi, const Coef<T> &C, const T *u,
                          const T *f, T *u_out, double omega, int colour, hipStream_t st,
                          const uint8_t *cls = nullptr);
// Tiles of level L holding a node of class >= 1 (unknowns: of class 1):
// flags[ntiles] scratch, ids[ntiles] and *count (device) out.
hipError_t launch_active_tiles(const Level &L, const uint8_t *cls, int *flags, int *ids,
                               int *count, hipStream_t st, int kz = 0, bool unknowns = false);

// Residual-norm partials of u (as launch_residual with partials, counted by
// stencil_partials) together with the colour half-sweep of u into u_out (same
// result as launch_rb_half, omega applied); residual_sweep_ok: the level is
// swept by the node-parallel kernels.
bool residual_sweep_ok(const Level &L);
hipError_t launch_residual_sweep(const Level &L, const double *u, const double *f,
                                 double *u_out, double omega, int colour, double *partials,
                                 hipStream_t st);
// LDS-tiled 3D half-sweep (same result as launch_rb_half); tiled_ok tells
// whether a level is large enough for the 64 x 8 node tiles to pay.  With a
// tile list only those tiles are swept (nodes outside them stay untouched).
// With partials (whole level, no classes) the launch also writes the partial
// sums of f . u_out over free DOF, rb_tiled_partials(L, fp32) of them; an
// FP32 launch then reads the FP64 residual r64 instead of f (its load is
// fp32(r64 / s), s = sqrt(*ss), as the mixed cast makes it) and sums
// r64 . (s u_out).
bool tiled_ok(const Level &L);
// Levels whose colour half-sweeps take the tiled kernel (a superset of
// tiled_ok: the half-sweep pays from smaller levels than the other passes).
bool tiled_sweep_ok(const Level &L);
template <typename T>
hipError_t launch_rb_tiled(const Level &L, const T *psi, const Coef<T> &C, const T *u, const T *f,
                           T *u_out, double omega, int colour, hipStream_t st,
                           const uint8_t *cls = nullptr, const TileList *tl = nullptr,
                           double *partials = nullptr, const double *r64 = nullptr,
                           const double *ss = nullptr);
int rb_tiled_partials(const Level &L, bool fp32);
// Levels whose first sweep from a zero iterate runs as one launch
// (launch_rb_fused with u == nullptr).
bool zero_sweep_ok(const Level &L);
// One complete two-colour Gauss-Seidel sweep on a tiled level in one launch
// (the same result as the half-sweep of first_colour from u followed by the
// half-sweep of the other colour): u_out must not be u.  u == nullptr means
// a zero iterate (nothing is read).
template <typename T>
hipError_t launch_rb_fused(const Level &L, const T *psi, const Coef<T> &C, const T *u, const T *f,
                           T *u_out, double omega, int first_colour, hipStream_t st);
// Tiled residual / Krylov Apply (same results as the node-parallel kernels);
// their partial sums number tiled_partials(L).
int tiled_partials(const Level &L);
template <typename T>
hipError_t launch_residual_tiled(const Level &L, const T *psi, const Coef<T> &C, const T *u,
                                 const T *f, T *r, double *partials, hipStream_t st,
                                 const uint8_t *cls, const TileList *tl = nullptr);
hipError_t launch_apply_dot_tiled(const Level &L, const double *p, double *q, double *partials,
                                  hipStream_t st);
// Number of partial sums launch_residual / launch_apply_dot write for level L.
int stencil_partials(const Level &L);
// fc = R r (full weighting); with ec the coarse correction is zeroed too.
template <typename T>
hipError_t launch_restrict(const Level &F, const Level &Cl, const T *r, T *fc, hipStream_t st,
                           T *ec = nullptr);
template <typename T>
hipError_t launch_prolong_add(const Level &F, const Level &Cl, const T *e, T *u, hipStream_t st);
template <typename T>
hipError_t launch_fill(T *p, int64_t n, T v, hipStream_t st);
template <typename T>
hipError_t launch_copy(const T *src, T *dst, int64_t n, hipStream_t st);
// a = b + s c over n doubles (16-byte aligned arrays; bandwidth probe).
hipError_t launch_triad(double *a, const double *b, const double *c, int64_t n, double s,
                        hipStream_t st);
hipError_t launch_correct(const Level &L, double *u, const float *e32, const double *ss,
                          hipStream_t st);
hipError_t launch_set_dirichlet(const Level &L, double *u, const DispValues &dv, hipStream_t st);
hipError_t launch_floor_psi(const double *raw, double floor_, double *psi64, float *psi32,
                            int64_t n, int cube, int *flag, hipStream_t st);
hipError_t launch_coarsen_psi(const Level &F, const Level &Cl, hipStream_t st);
hipError_t launch_rhs(const Level &L, const Traction &tr, const double *b, double *fA, int *flag,
                      hipStream_t st);
hipError_t launch_check_diag(const Level &L, int *flag, hipStream_t st);
hipError_t launch_finalize_sum(const double *partials, int n, double *out, hipStream_t st);
hipError_t launch_dot_free(const Level &L, const double *a, const ZSrc &b, double *partials,
                           hipStream_t st);
// *s_out = sqrt(*ss) (the scale of the mixed preconditioner's output).
hipError_t launch_store_sqrt(const double *ss, double *s_out, hipStream_t st);
hipError_t launch_sumsq_free(const Level &L, const double *v, double *partials, hipStream_t st);
hipError_t launch_apply_dot(const Level &L, const double *p, double *q, double *partials,
                           hipStream_t st);
// The flexible-CG vector updates with the iterate update deferred: r -= alpha q
// (alpha = rz / pq, stored to *alpha_out) with the r.r and r.z partials; then
// x += (*alpha) p (alpha may be NULL) and p = z + beta p in one pass; or
// x += (*alpha) p alone.
// With r32, also r32 = fp32(r / sqrt(*ss)) for the mixed preconditioner.
hipError_t launch_cg_update_r(const Level &L, double *r, const double *q, const ZSrc &z,
                              const double *rz, const double *pq, double *alpha_out, double *pr,
                              double *pz, hipStream_t st, float *r32 = nullptr,
                              const double *ss = nullptr);
hipError_t launch_xpby_x(const Level &L, double *x, double *p, const ZSrc &z,
                         const double *rznew, const double *rzold, const double *rz,
                         const double *alpha, hipStream_t st);
hipError_t launch_axpy_free(const Level &L, double *x, const double *p, const double *alpha,
                            hipStream_t st);
// r32 = fp32(r / sqrt(*ss)) for a residual r in memory (the expression of
// launch_residual_cast).
hipError_t launch_scale_cast(const double *r, float *r32, int64_t n, const double *ss,
                             hipStream_t st);
// The first colour half-sweep from a zero iterate for the load f into t
// (finest level, FP64 operator).
hipError_t launch_zero_sweep(const Level &L, const double *f, double *t, double omega, int colour,
                             hipStream_t st);
// ... and the first colour half-sweep of the FP32 correction from zero into
// t32 (finest level, FP32 operator).
hipError_t launch_scale_cast_sweep(const Level &L, const double *r, float *r32, float *t32,
                                   double omega, int colour, const double *ss, hipStream_t st);
hipError_t launch_cast_scaled(const double *r, float *r32, int64_t n, const double *ss,
                              hipStream_t st);
int num_blocks(int64_t n);
// Grid of the XCD-ordered stencil kernels over n items (>= num_blocks(n)).
int grid_blocks(int64_t n);
template <typename T>
hipError_t launch_bottom_cg(const Level &L, const T *psi, const Coef<T> &C, const T *f, T *x,
                            T *r, T *p, T *Ap, double rtol, int maxit, int *iters,
                            hipStream_t st);
// Bottom solve of the FP32 cycle: the FP64 CG on the FP32 load, the result
// returned in FP32 (f64 / x64 / r / p / Ap: FP64 scratch of the bottom size).
hipError_t launch_bottom_f32io(const Level &L, const float *f32, float *x32, double *f64,
                               double *x64, double *r, double *p, double *Ap, double rtol,
                               int maxit, int *iters, hipStream_t st);
// The V-cycle from level l0 down to the bottom and back in one workgroup
// with every vector of those levels in LDS (sbm_tail.hip).  tail_level gives
// the highest level whose tail fits lds_max bytes of LDS (-1: none);
// tail_upload writes the tail's level table (kTailArgBytes of device memory)
// once per problem, after the psi hierarchy is in place, assembles the dense
// bottom matrix into dense_A (kTailDenseBytes; nullptr: none) when the bottom
// has few free DOF, and returns the LDS bytes; launch_tail runs the cycle on
// x (in/out, level l0) for the load f (wide_bottom: a bottom of more than
// kTailWaveBottom nodes, solved by the whole workgroup).
constexpr int kTailMaxLevels = 6;
constexpr size_t kTailArgBytes = 4096;
constexpr size_t kTailDenseBytes = 64 * 64 * sizeof(double);
constexpr int kTailWaveBottom = 64;  // bottoms up to this many nodes are solved in one wave
struct TailOpts {
  int nu_pre, nu_post, jacobi, reverse;
  double omega, rtol;
  int maxit;
};
int tail_level(const std::vector<Level> &L, int precision, size_t lds_max);
hipError_t tail_upload(const std::vector<Level> &L, int precision, int l0, void *dev,
                       double *dense_A, size_t lds_max, size_t *lds_bytes, hipStream_t st);
template <typename T>
hipError_t launch_tail(int dim, bool wide_bottom, const void *dev, size_t lds_bytes,
                       T *x, const T *f, const TailOpts &o, int *iters, hipStream_t st);
// Plastic strain (sbm_plastic.hip, 3D): the load -div(psi C eps_p) at every
// node, and the J2 radial return of the cell state for the strain of u
// (count: device int incremented by the yielding cells, nullable).
hipError_t launch_plastic_source(const Level &L, double lam, double mu, const double *eps_p,
                                 double *fp, hipStream_t st);
hipError_t launch_return_map(const Level &L, double mu, double sigma_y, double hbar, double theta,
                             const double *u, double *eps_p, double *alpha, double *beta,
                             int *count, hipStream_t st);
// Diffuse traction (sbm_traction.hip): f = t_hat |grad psi| + p grad psi at
// every node of the finest grid, psi = max(psi_raw, floor); t_hat may be NULL.
hipError_t launch_diffuse_traction(const Level &L, const double *psi_raw, double floor_,
                                   const double *t_hat, double p, double *f, hipStream_t st);
// Phase-field fracture (sbm_fracture.hip): crack driving force of every cell
// (H <- max(H, W0+), intact <- W0+ < W0-) and one explicit Ginzburg-Landau
// step of the crack field c (writing c1 and psi = g(c1) + eta).
hipError_t launch_crack_drive(const Level &L, double lam, double mu, const double *u, double *H,
                              uint8_t *intact, hipStream_t st);
hipError_t launch_phase_step(const Level &L, const double *c0, const double *H,
                             const uint8_t *intact, double Gc, double xi, double M, double dt,
                             double eta, double *c1, double *psi, hipStream_t st);
hipError_t launch_sensitivity(const Level &L, double lam, double mu, const Traction &tr,
                              const double *u, const double *adj, double lam_scale,
                              const double *design, int chain, double psi_floor, double *g,
                              hipStream_t st);

// ------------------------------------------------- shared host helpers
// Records msg as the thread's last error and returns s.
sbm_status set_error(sbm_status s, const std::string &msg);
// Geometry of a grid with ncell cells of spacing h (entries >= dim ignored).
void make_level(int dim, const int64_t *ncell, const double *h, Level &L);
// Operator coefficients of level L for the Lame constants (FP64 and FP32).
void set_coefs(Level &L, double lam, double mu, int dim);
// One V-cycle of the uniform hierarchy of c from its finest level: x (in/out)
// and f are finest-level vectors in FP64 (precision 0) or FP32 (precision 1).
hipError_t base_vcycle(sbm_ctx *c, int precision, void *x, const void *f);

}  // namespace sbm
