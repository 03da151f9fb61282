/*
 * sbm.h -- C ABI of the MI355X (gfx950) smooth-boundary-method elasticity
 * multigrid library.
 *
 * The library solves the diffuse-boundary equilibrium of Agrawal & Runnels,
 * arXiv:2212.02362, Sec. 2.1 (eq. SBMLinearElasticity):
 *
 *     div(psi C : grad u) + b = 0,      written  K u = f,  K = -div(psi C grad .)
 *
 * on a box, with the displacement u on the nodes and the indicator psi in the
 * cells (Sec. 2.3), isotropic moduli given as Lame constants (Sec. 2.4),
 * traction boundary data entering as source terms (Sec. 2.1) and displacement
 * data eliminated at the nodes (Sec. 2.1: essential conditions are not
 * diffused).  The solver is geometric multigrid (Sec. 2.2) with Jacobi or
 * two-colour Gauss-Seidel smoothing (Sec. 2.3), full-weighting restriction,
 * multilinear prolongation, coarse operators re-discretised on averaged psi
 * and a CG bottom solve.
 *
 * Layouts (all arrays dense, row-major, x fastest):
 *   node vector  v[k][z][y][x]   k < dim components, (nx+1)(ny+1)(nz+1) nodes
 *                                (2D: v[k][y][x])
 *   cell scalar  s[z][y][x]      nx*ny*nz cells (2D: s[y][x])
 * where (nx, ny, nz) = grid.ncell.  Faces are numbered x-,x+,y-,y+,z-,z+.
 *
 * Pointers: every array argument is a DEVICE pointer unless its name ends in
 * _host.  The caller owns all memory.  The library never allocates device
 * memory: every device buffer it needs is carved from the caller's workspace
 * (sbm_workspace_bytes), which must stay alive until sbm_destroy.
 * An output array must not be one of the call's input arrays or another of
 * its outputs unless the call says so (solution vectors documented "in/out"
 * are one array by design); the same pointer passed twice is rejected with
 * SBM_E_ARG (partial overlaps of distinct pointers are not detected).
 *
 * Streams: all device work is enqueued on the HIP stream given to sbm_create.
 * Calls documented "async" return before the work completes; the others
 * return with the stream idle.
 *
 * Errors: no exception crosses the ABI.  A negative status means the outputs
 * are unspecified; sbm_last_error() (thread-local) describes the failure.
 * SBM_NOT_CONVERGED (> 0) means the outputs are valid.
 *
 * Threading: a context is not thread-safe; distinct contexts are independent.
 */
#ifndef SBM_H
#define SBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sbm_ctx sbm_ctx;

typedef enum {
  SBM_OK = 0,
  SBM_NOT_CONVERGED = 1, /* max_cycles reached; u and history valid */
  SBM_E_ARG = -1,        /* null pointer, aliased buffers or out-of-range argument */
  SBM_E_SHAPE = -2,      /* unsupported grid (dim, cell counts) */
  SBM_E_HIP = -3,        /* a HIP runtime call failed */
  SBM_E_NONFINITE = -4,  /* NaN/Inf in psi, b, u0 or a residual */
  SBM_E_DIVERGED = -5,   /* residual grew 1e3 x above its minimum */
  SBM_E_DIAG = -6,       /* a free DOF has a zero diagonal (psi = 0 around it) */
  SBM_E_WORKSPACE = -7   /* workspace too small or misaligned */
} sbm_status;

typedef enum { SBM_TRACTION = 0, SBM_DISPLACEMENT = 1 } sbm_bc_kind;

/* Grid: dim 2 or 3; ncell[a] >= 1 for a < dim (unused entries ignored);
 * h[a] > 0 is the spacing along axis a.  Nodes per axis are ncell[a] + 1. */
typedef struct {
  int dim;
  int64_t ncell[3];
  double h[3];
} sbm_grid;

/* Boundary data per face F (x-,x+,y-,y+,z-,z+) and component k:
 *   kind TRACTION:     value is the traction component t_k on F (outward
 *                      normal convention: sigma n = t).  It enters as the
 *                      source (t_k / h_perp) * (mean of the 2^(d-1) cells that
 *                      contain the node and touch F), Sec. 2.1.
 *   kind DISPLACEMENT: the k-th displacement of every node of F is fixed to
 *                      value.  Where several displacement faces meet, the last
 *                      face in the order above wins. Displacement beats
 *                      traction on shared edges. */
typedef struct {
  int kind[6][3];
  double value[6][3];
} sbm_bc;

/* Isotropic Lame constants (Sec. 2.4) and the floor applied cell-wise to psi:
 * psi = max(psi_raw, psi_floor). */
typedef struct {
  double lambda, mu, psi_floor;
} sbm_material;

/* Solver options (the paper leaves these open; defaults in brackets):
 *   smoother       0 two-colour Gauss-Seidel [0], 1 damped Jacobi
 *   omega          relaxation factor [1.0 for Gauss-Seidel, 0.8 for Jacobi]
 *   nu_pre/post    smoothing sweeps per V-cycle leg [2, 2]
 *   precision      0 FP64 cycles [0]; 1 FP32 cycles with FP64 residual,
 *                  correction and bottom refinement
 *   rtol           stop when ||f - K u||_2 <= rtol ||f||_2 over free DOF [1e-10]
 *   max_cycles     V-cycle cap [200]
 *   bottom_rtol    CG tolerance on the bottom grid, relative [1e-12]
 *   bottom_max_iter CG iteration cap; <= 0 means 4 x free bottom DOF [0]
 *   use_graphs     1: each V-cycle is captured once into a HIP graph and
 *                  replayed (same kernels, same order, fewer launches) [1];
 *                  0: kernels are launched one by one
 *   krylov         0: stationary V-cycle iteration [0]; 1: flexible conjugate
 *                  gradients (Polak-Ribiere) preconditioned by one V-cycle
 *                  from zero per iteration, post-smoothing colours reversed
 *                  (black, red); the history then has one entry per CG
 *                  iteration and max_cycles caps the iterations
 *   fused_sweep    1: on levels wider than 192 nodes every Gauss-Seidel sweep
 *                  is one launch that relaxes the second colour one plane
 *                  behind the first (the same iterates as two half-sweeps);
 *                  0: two half-sweep launches per sweep [0] */
typedef struct {
  int smoother;
  double omega;
  int nu_pre, nu_post;
  int precision;
  double rtol;
  int max_cycles;
  double bottom_rtol;
  int bottom_max_iter;
  int use_graphs;
  int krylov;
  int fused_sweep;
} sbm_options;

/* Fills *opts with the defaults above. */
void sbm_default_options(sbm_options *opts);

/* Number of multigrid levels for a grid: the grid is halved while every
 * active cell count is even and >= 4 (power-of-two grids, Sec. 3.3); the last
 * level is the bottom.  Returns <= 0 for an invalid grid. */
int sbm_num_levels(const sbm_grid *grid);

/* Device workspace bytes needed by sbm_create for this grid (FP64 and FP32
 * hierarchies, residual partial sums, bottom scratch).  0 on invalid input. */
size_t sbm_workspace_bytes(const sbm_grid *grid, const sbm_options *opts);

/* Creates a context.  workspace: device pointer, 256-byte aligned, at least
 * sbm_workspace_bytes bytes, owned by the caller.  hip_stream: a hipStream_t
 * (NULL = default stream).  The current HIP device must own the workspace. */
sbm_status sbm_create(const sbm_grid *grid, const sbm_options *opts, void *workspace,
                      size_t workspace_bytes, void *hip_stream, sbm_ctx **out);

/* Replaces the solver options (same grid and workspace). */
sbm_status sbm_set_options(sbm_ctx *ctx, const sbm_options *opts);

/* Sets the problem (Sec. 2.1): psi_raw (cells, device) is floored, averaged
 * down the hierarchy (coarse psi = mean of the 2^d children) and cast for the
 * FP32 cycle; the load f = b + traction source (zero on displacement DOF) is
 * assembled.  body_force (node vector, device) may be NULL.  The inputs are
 * copied; the caller may free them afterwards.  Fails with SBM_E_NONFINITE on
 * NaN/Inf in psi_raw or b, SBM_E_DIAG when a free DOF has no solid cell
 * around it. */
sbm_status sbm_set_problem(sbm_ctx *ctx, const double *psi_raw, const sbm_material *mat,
                           const sbm_bc *bc, const double *body_force);

/* Solves K u = f (Sec. 2.2, V-cycles until rtol).  u (node vector, device):
 * in = initial guess (warm start, Sec. 3.2), out = solution; its displacement
 * DOF are overwritten with the prescribed values.  res_hist_host receives the
 * relative residuals rho_0 .. rho_m (at most hist_cap values; may be NULL),
 * *n_cycles_host the number m of V-cycles run, *final_rel_res_host rho_m.
 * Returns SBM_OK, SBM_NOT_CONVERGED, SBM_E_DIVERGED or SBM_E_NONFINITE. */
sbm_status sbm_solve(sbm_ctx *ctx, double *u, double *res_hist_host, int hist_cap,
                     int *n_cycles_host, double *final_rel_res_host);

/* Solves K x = g on the free DOF with x = 0 on displacement DOF (the adjoint
 * problem: K is symmetric).  g (node vector, device; its displacement DOF are
 * ignored), x (device, in = guess, out = solution).  Same history outputs. */
sbm_status sbm_solve_rhs(sbm_ctx *ctx, const double *g, double *x, double *res_hist_host,
                         int hist_cap, int *n_cycles_host, double *final_rel_res_host);

/* Ku = K u on every node of the finest grid (no boundary masking).  Async. */
sbm_status sbm_apply(sbm_ctx *ctx, const double *u, double *Ku);

/* r = f - K u on free DOF, 0 on displacement DOF (f from sbm_set_problem).
 * If norm_host is non-NULL, *norm_host = ||r||_2 and the call synchronises;
 * otherwise it is async.  r may be NULL when only the norm is wanted. */
sbm_status sbm_residual(sbm_ctx *ctx, const double *u, double *r, double *norm_host);

/* The assembled load of sbm_set_problem: fA (body force + traction source,
 * 0 on displacement DOF) and, if fB is non-NULL, the lifted load
 * fB = fA - K uD on free DOF (uD = prescribed values), whose norm normalises
 * the residual.  Async. */
sbm_status sbm_rhs(sbm_ctx *ctx, double *fA, double *fB);

/* sbm_residual without a context or workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): r = f - K u on free DOF, 0 on
 * displacement DOF (r may be NULL), and *norm_host = ||r||_2 over the free
 * DOF.  K is eq. K on the grid with the material's Lame constants and the
 * displacement faces of bc (bc values are not used: u carries them); psi is
 * the floored cell indicator (cells, finite, >= 0; not checked), u and f
 * node vectors; all device arrays.  The residual partial sums live in a
 * file-scope device array of 2^17 doubles (1 MiB per device, held until the
 * process ends), so grids needing more than 2^17 - 1 partial sums (about
 * 33 M nodes) are rejected with SBM_E_SHAPE.  Nothing is allocated: no
 * hipMalloc, no workspace.  Calls that overlap on one device (other host
 * threads, other streams) share that array and race.  Synchronises
 * hip_stream (NULL: the null stream). */
sbm_status sbm_residual_static(const sbm_grid *grid, const sbm_material *mat, const sbm_bc *bc,
                               const double *psi, const double *u, const double *f, double *r,
                               double *norm_host, void *hip_stream);

/* Adjoint sensitivity per cell: g_c = -lam_c^T K_c u_c + lam^T df/dpsi_c,
 * where K = sum_c psi_c K_c and f depends on psi through the traction source.
 * This is dL/dpsi for L(u(psi)) with K lam = dL/du.  u: node vector carrying
 * its prescribed values; lam: node vector, must be 0 on displacement DOF; it
 * is used as lam_scale * lam (Sec. 3.3's compliance J = h^d f.u is
 * self-adjoint: lam = h^d u, i.e. lam = u and lam_scale = h^d).
 * chain selects what g is differentiated with respect to:
 *   SBM_CHAIN_PSI   (0): the floored psi; design may be NULL;
 *   SBM_CHAIN_FLOOR (1): psi_raw (design = psi_raw cells): g where
 *                        psi_raw > psi_floor, 0 elsewhere;
 *   SBM_CHAIN_RHO3  (2): rho (design = rho cells, psi_raw = rho^3):
 *                        3 rho^2 g where rho^3 > psi_floor, 0 elsewhere.
 * g: cells.  Async. */
typedef enum { SBM_CHAIN_PSI = 0, SBM_CHAIN_FLOOR = 1, SBM_CHAIN_RHO3 = 2 } sbm_chain;
sbm_status sbm_sensitivity(sbm_ctx *ctx, const double *u, const double *lam, double lam_scale,
                           const double *design, int chain, double *g);

/* sbm_set_problem with psi_raw = rho^3 computed on the device from the
 * density rho (cells): the stiffness interpolation of Sec. 3.3, whose
 * (eta + zeta)^2 C becomes rho^3 C with the floor playing zeta^2. */
sbm_status sbm_set_problem_density(sbm_ctx *ctx, const double *rho, const sbm_material *mat,
                                   const sbm_bc *bc, const double *body_force);

/* ------------------------------------------------ plastic strain (J2) ---
 * Sec. 3.1: sigma = C (grad u - eps_p), so the equilibrium becomes
 * K u = b - div(psi C eps_p); the plastic state evolves by J2 plasticity with
 * linear combined hardening (eq. J2Plasticity), integrated over a load step
 * by radial return.  3D grids only (SBM_E_SHAPE otherwise).  Cell state
 * arrays (device, cells, x fastest): eps_p and beta hold 6 components (xx,
 * yy, zz, yz, xz, xy) one array after another (6 x cells doubles), alpha one
 * array.  A staggered step passes f as the body force of sbm_set_problem,
 * solves, and calls sbm_return_map on the solution. */
typedef struct {
  double sigma_y; /* yield strength (flow stress) */
  double hbar;    /* hardening modulus */
  double theta;   /* isotropic share of the hardening, 0..1 */
} sbm_j2;

/* f = -div(psi C eps_p) at every node (3 x nodes, device): the flux form of
 * eq. K with half-edge stresses averaged over the four cells around each
 * edge and psi the floored psi of sbm_set_problem.  Async. */
sbm_status sbm_plastic_source(sbm_ctx *ctx, const double *eps_p, double *f);

/* Radial return of every cell for the strain of u (cell-centre sym grad:
 * mean over the cell's four edges along each axis): eta = 2 mu dev(eps -
 * eps_p) - beta, f = |eta| - sqrt(2/3)(sigma_y + theta hbar alpha); where
 * f > 0, dgamma = f / (2 mu + 2 hbar / 3), n = eta / |eta|, eps_p += dgamma n,
 * alpha += sqrt(2/3) dgamma, beta += (2/3)(1 - theta) hbar dgamma n.  The
 * state is updated in place.  If n_plastic_host is non-NULL it receives the
 * number of yielding cells and the call synchronises; otherwise async. */
sbm_status sbm_return_map(sbm_ctx *ctx, const double *u, const sbm_j2 *mat, double *eps_p,
                          double *alpha, double *beta, int64_t *n_plastic_host);

/* ----------------------------------------------- diffuse traction -------
 * Sec. 2.1, eq. SBMLinearElasticity: a traction t0 on the (diffuse) surface
 * of the solid, extended along the normals across the diffuse band (t_hat,
 * the value at the closest point of the sharp boundary), is the load
 * t_hat |grad psi|.  This call writes, at every node,
 *   f = t_hat |grad psi| + pressure * grad psi,
 * psi = max(psi_raw, psi_floor) (cells, device), t_hat a node field of d
 * components (device, may be NULL), f a node field of d components (device,
 * overwritten).  The pressure term is the load of a pressure acting on the
 * solid from the empty side.  The sign is that of the box-face tractions of
 * sbm_set_problem (a traction along the outward normal of the solid pulls).
 * The node gradient along axis a is the mean of the difference quotients of
 * the 2^(d-1) cell pairs facing each other across the node; cells outside the
 * box take the value of the nearest cell inside (the box faces carry their
 * own tractions).  Pass f as (part of) the body force b of sbm_set_problem.
 * f may be t_hat (each node reads its own t_hat before writing), not psi_raw.
 * Needs only the grid of ctx.  Async. */
sbm_status sbm_diffuse_traction(sbm_ctx *ctx, const double *psi_raw, double psi_floor,
                                const double *t_hat, double pressure, double *f);

/* ------------------------------------------- phase-field fracture -------
 * Sec. 3.2 (hybrid formulation, eqs. PFFracture and PFFractureGL): the
 * equilibrium is the SBM solve with psi = g(c) + eta, g(c) = 4c^3 - 3c^4; the
 * crack field c (cells, device) evolves by an explicit Ginzburg-Landau step
 * driven by the history field H of the tensile strain energy.  2D (plane
 * strain) and 3D. */
typedef struct {
  double Gc;  /* fracture energy */
  double xi;  /* regularisation length */
  double M;   /* crack mobility */
  double dt;  /* time step */
  double eta; /* residual stiffness (psi = g(c) + eta) */
} sbm_pf;

/* Crack driving force of every cell for the strain of u (cell-centre sym
 * grad, as sbm_return_map): principal strains e_i, W0+- = lambda/2
 * (sum <e_i>+-)^2 + mu sum <e_i>+-^2; H <- max(H, W0+) in place; intact[c] =
 * 1 where W0+ < W0- (the crack field is held at 1 there), else 0.  H and
 * intact: cells (double, uint8).  u, H and intact must not alias each other
 * (SBM_E_ARG).  Async. */
sbm_status sbm_crack_drive(sbm_ctx *ctx, const double *u, double *H, uint8_t *intact);

/* One explicit step c_out = c - dt M [g'(c) H - Gc (2 xi lap(c) + w'(c) /
 * (2 xi))], w = 1 - g, projected onto [0, 1] (the range of the crack field;
 * a NaN stays NaN), c_out = 1 where intact; lap is the cell Laplacian
 * (2d+1 points) with zero flux across the box faces.  Also writes psi_out =
 * g(c_out) + eta, the indicator of the next sbm_set_problem (pass floor
 * <= eta).  crack_out and psi_out must not alias each other or the inputs
 * (SBM_E_ARG).  Needs only the grid of ctx.
 * Async. */
sbm_status sbm_phase_step(sbm_ctx *ctx, const double *crack, const double *H,
                          const uint8_t *intact, const sbm_pf *p, double *crack_out,
                          double *psi_out);

/* Compliance J = h^d sum over free DOF of fA . u (Sec. 3.3, the work of the
 * load), written to *J_host; synchronises. */
sbm_status sbm_compliance(sbm_ctx *ctx, const double *u, double *J_host);

/* Live kernel timing.  While enabled, every finest-level launch of the
 * classes below is bracketed by HIP events on the context's stream; the
 * elapsed times are collected at the solve's per-cycle synchronisation.
 * Cycles then run launch by launch (use_graphs is ignored while enabled).
 * sbm_profile(ctx, 1) enables and clears, sbm_profile(ctx, 0) disables.
 * sbm_profile_read fills ms_host[SBM_PROF_N] (total milliseconds) and
 * count_host[SBM_PROF_N] (launches) per class. */
typedef enum {
  SBM_PROF_SMOOTH = 0,   /* smoother sweep / half-sweep on the finest level */
  SBM_PROF_RESIDUAL = 1, /* residual feeding the restriction, finest level */
  SBM_PROF_RESTRICT = 2, /* restriction from the finest level */
  SBM_PROF_PROLONG = 3,  /* prolongation-add into the finest level */
  SBM_PROF_NORM = 4,     /* convergence-test residual norm (+ FP32 cast) */
  SBM_PROF_BOTTOM = 5,   /* whole bottom solve */
  SBM_PROF_GHOST = 6,    /* coarse-fine ghost fill of the finest adaptive level */
  SBM_PROF_SWEEP0 = 7,   /* one-launch sweep from a zero iterate, finest level */
  SBM_PROF_SMOOTH_DOT = 8, /* finest-level half-sweep that also forms the CG product r.z */
  SBM_PROF_N = 9
} sbm_prof_class;
sbm_status sbm_profile(sbm_ctx *ctx, int enable);
sbm_status sbm_profile_read(sbm_ctx *ctx, double *ms_host, int64_t *count_host);

/* Captured V-cycle graphs: number of captures and of graph launches since
 * sbm_create (both 0 when use_graphs is 0 or capture was not possible; the
 * reason of a failed capture is then in sbm_last_error()). */
sbm_status sbm_graph_info(sbm_ctx *ctx, int64_t *captures_host, int64_t *launches_host);

/* Bandwidth probe, not part of the method: a[i] = b[i] + s c[i] for i < n
 * (device arrays of n doubles, 16-byte aligned, a distinct from b and c), one
 * pass of 16-byte loads and stores enqueued on hip_stream (NULL: the null
 * stream).  Benchmarks time it to measure the bandwidth a plain streaming
 * kernel reaches on the device (24 bytes per element).  Async; SBM_E_ARG on
 * NULL, misaligned or aliased arrays or n < 1. */
sbm_status sbm_stream_triad(double *a, const double *b, const double *c, int64_t n, double s,
                            void *hip_stream);

/* Releases host-side state; the workspace stays the caller's. */
void sbm_destroy(sbm_ctx *ctx);

/* Thread-local description of the last failure ("" if none). */
const char *sbm_last_error(void);

/* ------------------------------------------------------------------------
 * Component entry points: one multigrid step at a time, on level l of the
 * context's hierarchy (0 = finest), for parity checks of each kernel.  All
 * arrays are device arrays in the level's layout; all calls are async.
 * ---------------------------------------------------------------------- */

/* Cells per axis of level l (ncell_host[3]; inactive axes 0). */
sbm_status sbm_level_shape(sbm_ctx *ctx, int level, int64_t *ncell_host);

/* The floored (level 0) or averaged (l > 0) psi of level l (FP64 cells). */
sbm_status sbm_level_psi(sbm_ctx *ctx, int level, double *psi);

/* Ku on level l (FP64), and the same operator evaluated in FP32 on the FP32
 * psi copy. */
sbm_status sbm_level_apply(sbm_ctx *ctx, int level, const double *u, double *Ku);
sbm_status sbm_level_apply_f32(sbm_ctx *ctx, int level, const float *u, float *Ku);

/* One smoothing step on level l, out of place (u_out != u_in):
 * colour < 0: damped Jacobi sweep u_out = u + omega D^-1 (f - K u) (Sec. 2.3);
 * colour 0/1: colour-synchronous Gauss-Seidel half-sweep updating the nodes
 * with (x+y+z) mod 2 == colour from the state u_in, copying the others.
 * Displacement DOF are copied unchanged. */
sbm_status sbm_level_smooth(sbm_ctx *ctx, int level, int colour, double omega,
                            const double *u_in, const double *f, double *u_out);

/* One complete two-colour Gauss-Seidel sweep on level l (Sec. 2.3), out of
 * place: the half-sweep of first_colour (0 or 1) from u_in, then the
 * half-sweep of the other colour from that intermediate state, each
 * colour-synchronous as in sbm_level_smooth; displacement DOF keep their
 * values.  u_in == NULL stands for a zero iterate.  u_out must differ from
 * u_in and f.  Levels wider than 192 nodes run it as one fused launch (the
 * second colour one plane behind the first); other levels run two half-sweeps
 * through the level's internal scratch vector.  The _f32 variant uses the
 * FP32 operator (FP32 psi copy) on FP32 vectors.  Async. */
sbm_status sbm_level_sweep(sbm_ctx *ctx, int level, int first_colour, double omega,
                           const double *u_in, const double *f, double *u_out);
sbm_status sbm_level_sweep_f32(sbm_ctx *ctx, int level, int first_colour, double omega,
                               const float *u_in, const float *f, float *u_out);

/* r = f - K u on free DOF of level l, 0 on displacement DOF. */
sbm_status sbm_level_residual(sbm_ctx *ctx, int level, const double *u, const double *f,
                              double *r);

/* f_coarse = P^T r_fine / 2^d from level l to l+1 (full weighting), 0 on
 * coarse displacement DOF. */
sbm_status sbm_level_restrict(sbm_ctx *ctx, int level, const double *r_fine, double *f_coarse);

/* u_fine += P e_coarse from level l+1 to level l (multilinear), free DOF only. */
sbm_status sbm_level_prolong_add(sbm_ctx *ctx, int level, const double *e_coarse,
                                 double *u_fine);

/* Bottom solve: x += CG solution of K_FF d = (f - K x)_F on the bottom level,
 * with the context's bottom tolerance.  *iters_host (may be NULL) receives
 * the iteration count (this call synchronises). */
sbm_status sbm_bottom_solve(sbm_ctx *ctx, const double *f, double *x, int *iters_host);

/* ------------------------------------------------------------------------
 * Block-structured adaptive composite solve (Sec. 2.2: AMR levels of the
 * same operator exchanging data by averaging and ghost cells, the refined
 * levels forming the upper part of the multigrid level sequence, every level
 * padded by a ghost layer so that no special coarse-fine stencil is needed).
 *
 * Layout: AMR level a = 0..levels-1 has cells ncell0 * 2^a per axis and
 * spacing h0 / 2^a and is stored DENSELY over the box (node vectors and cell
 * arrays in the layouts above).  Levels a >= 1 are active on cubic blocks of
 * `block` cells; block flags are uint8 [nbz][nby][nbx] with nb = ncell / block.
 * Nodes of a level a >= 1 carry a class (uint8, node layout): 0 unused,
 * 1 unknown (interior of the active region), 2 interface (owned by level
 * a-1), 3 and 4 the first and second node layer outside.  Classes 2-4 are
 * ghosts filled from level a-1 by tensor-product quadratic interpolation:
 * along an axis an even fine index copies the coinciding coarse node, an odd
 * index 2I+1 takes nodes I-1, I, I+1 with weights -1/8, 3/4, 3/8 (I = 0:
 * nodes 0, 1, 2 with 3/8, 3/4, -1/8).
 *
 * Refinement (when no block flags are given): level-a cells (a < levels-1)
 * are tagged where |grad psi| h > tag_threshold (central differences on the
 * floored psi, neighbours clamped at the box, h the largest spacing;
 * Sec. 3.3 uses 0.05); a level-(a+1) block is active when a tagged level-a
 * cell lies in its footprint grown by one cell; each active block then
 * activates its parent block and the parent's neighbours on the sides it
 * touches.  Covered coarse cells take the mean psi of their 2^d children.
 *
 * Composite residual: on levels a >= 1 the level residual on classes 1-3
 * (0 elsewhere); coarse nodes whose coinciding fine node has class 1 or 2
 * take the full-weighting restriction of it; the norm runs over the
 * composite unknowns (class 1 at a >= 1, every node at a = 0, minus nodes
 * covered by a finer class-1 node, minus displacement DOF), relative to the
 * same norm of the lifted load.
 *
 * Composite cycle: full-approximation cycle over the AMR levels (smooth the
 * unknowns, restrict the padded residual, coarse load R w + K_c x_c on
 * covered and interface nodes, recurse, correct the unknowns by
 * P (x_c - inject x_f), smooth) ending in one V-cycle of the base grid's
 * uniform hierarchy; run in correction form on the composite residual inside
 * an FP64 outer loop (options.precision 1: the cycle in FP32 on the residual
 * scaled to unit norm).  options.krylov must be 0.
 *
 * Conventions as above: device pointers unless _host, the caller owns all
 * memory, the workspace is carved (sbm_amr_workspace_bytes), work is
 * enqueued on the given stream.  Arrays of per-level pointers are HOST
 * arrays with `levels` entries (block flags: levels-1 entries for a >= 1).
 * ---------------------------------------------------------------------- */
typedef struct sbm_amr_ctx sbm_amr_ctx;

/* Workspace bytes for a base grid, levels (1..4, base included), block size
 * (even, dividing 2 * ncell0 on every axis) and options; 0 if unsupported. */
size_t sbm_amr_workspace_bytes(const sbm_grid *base, int levels, int block,
                               const sbm_options *opts);

sbm_status sbm_amr_create(const sbm_grid *base, int levels, int block, const sbm_options *opts,
                          void *workspace, size_t workspace_bytes, void *hip_stream,
                          sbm_amr_ctx **out);

sbm_status sbm_amr_set_options(sbm_amr_ctx *ctx, const sbm_options *opts);

/* Regridding by Berger-Rigoutsos point clustering (Sec. 2.2), used by the
 * next sbm_amr_set_problem that tags (blocks_host == NULL): on each level
 * a >= 1, finest first, the tagged block flags are replaced by the blocks of
 * boxes that each hold flags >= efficiency * volume, before they nest into
 * level a-1.  A box is the bounding box of its flags; one that is too sparse
 * is cut at an interior slab without flags (first axis that has one, the
 * slab nearest the middle, the lower on a tie), else between slabs i, i+1
 * where the discrete Laplacian of the signature (flags per slab) changes
 * sign, at the largest jump (first in axis order, then ascending i, on a
 * tie), else in the middle of its longest axis (the lower part keeps the
 * middle slab).  efficiency in [0, 1]; 0 (the default) keeps the tagged
 * blocks as they are.  Host-side; set_problem synchronises per level. */
sbm_status sbm_amr_set_clustering(sbm_amr_ctx *ctx, double efficiency);

/* The same clustering of one flag array, on the host (no device, no
 * context): flags_host / out_host are uint8 [nb2][nb1][nb0] (2D: [nb1][nb0]),
 * nblocks[0..dim-1] the counts per axis; out_host gets the blocks of the
 * accepted boxes (it must not alias flags_host). */
sbm_status sbm_amr_cluster(int dim, const int64_t *nblocks, const uint8_t *flags_host,
                           double efficiency, uint8_t *out_host);

/* psi_raw[a]: raw indicator at the cell centres of level a (device, dense),
 * floored cell-wise by mat->psi_floor.  blocks_host: NULL (tag with
 * tag_threshold) or levels-1 host arrays of block flags of levels 1.. that
 * are used as given.  Synchronises. */
sbm_status sbm_amr_set_problem(sbm_amr_ctx *ctx, const double *const *psi_raw,
                               const sbm_material *mat, const sbm_bc *bc, double tag_threshold,
                               const uint8_t *const *blocks_host);

/* Level a: cells per axis, blocks per axis (0 at a = 0), block flags (host,
 * a >= 1), node classes (device, a >= 1) and the floored, averaged-down psi
 * (device); every output may be NULL.  Synchronises. */
sbm_status sbm_amr_level_info(sbm_amr_ctx *ctx, int level, int64_t *ncell_host,
                              int64_t *nblocks_host, uint8_t *blocks_host, uint8_t *classes,
                              double *psi);

/* Number of composite unknowns (free DOF) and the norm of the lifted load. */
sbm_status sbm_amr_stats(sbm_amr_ctx *ctx, int64_t *composite_dof_host, double *fnorm_host);

/* Ghost nodes (classes 2-4, free DOF) of level a >= 1 in xf from xc of level
 * a-1 (async). */
sbm_status sbm_amr_ghost_fill(sbm_amr_ctx *ctx, int level, const double *xc, double *xf);

/* Composite residual of u (ghosts of u are refilled in place) into r (per
 * level; r or any r[a] may be NULL, r[a] must not be u[a]) and its norm
 * (absolute).  Synchronises. */
sbm_status sbm_amr_residual(sbm_amr_ctx *ctx, double *const *u, double *const *r,
                            double *norm_host);

/* Composite solve: u[a] in = guess (displacement DOF set, covered coarse
 * nodes injected), out = solution with covered nodes injected and ghosts
 * filled; history of relative composite residuals as in sbm_solve. */
sbm_status sbm_amr_solve(sbm_amr_ctx *ctx, double *const *u, double *hist_host, int hist_cap,
                         int *n_cycles_host, double *final_rel_host);

/* Live kernel timing of the finest adaptive level, as sbm_profile /
 * sbm_profile_read (classes SMOOTH, RESIDUAL (cycle and convergence test),
 * RESTRICT (restriction to the covered/interface nodes), PROLONG (coarse
 * correction), GHOST; BOTTOM times the whole base V-cycle). */
sbm_status sbm_amr_profile(sbm_amr_ctx *ctx, int enable);
sbm_status sbm_amr_profile_read(sbm_amr_ctx *ctx, double *ms_host, int64_t *count_host);

void sbm_amr_destroy(sbm_amr_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* SBM_H */
