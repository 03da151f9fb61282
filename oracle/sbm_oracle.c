/*
 * sbm_oracle.c -- plain, slow FP64 CPU reference for the smooth-boundary (SBM)
 * strong-form elasticity multigrid solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the HIP library; the two meet only at the
 * seeded input generators.
 *
 * What is computed (Agrawal & Runnels, "Robust, strong form mechanics on an
 * adaptive structured grid", arXiv:2212.02362):
 *
 *   Equilibrium with a diffuse boundary (Sec. 2.1, eq. SBMLinearElasticity):
 *       div(psi C : grad u) + b = 0,
 *   written here as K u = f with K = -div(psi C grad .).  Displacement u lives
 *   on the nodes, the indicator psi in the cells (Sec. 2.3: a node-based psi
 *   makes the Jacobi diagonal vanish next to non-zero neighbours; a cell-based
 *   psi does not).  The paper prints the 1D operator only (Sec. 2.3, the
 *   cell-based Jacobi update) and states that 2D and 3D behave the same; the
 *   2D/3D discretisation used here is the split flux form below ("eq. K"),
 *   which reduces to the paper's 1D cell operator, is symmetric, and is exact
 *   for quadratic u with constant or linear psi.
 *
 *   (Ku)_i(n) = - sum_j (1/h_j^2) sum_k C_ijkj [ psiE(n,+j)(u_k(n+e_j)-u_k(n))
 *                                               - psiE(n,-j)(u_k(n)-u_k(n-e_j)) ]
 *               - sum_{j!=l} (1/(2 h_j)) sum_{sj,sl=+-1} sj psiF(p) sum_k C_ijkl (G_l u_k)(p)
 *     p       = n + sj e_j/2 + sl e_l/2
 *     psiE    = mean of the 2^(d-1) cells sharing the edge (cells outside the
 *               box count as 0: traction-free box faces are natural)
 *     psiF(p) = 2D: the cell centred at p; 3D: mean of the two cells p +- e_m/2
 *     G_l u(p)= sl [ (u(n+sl e_l)-u(n)) + (u(n+sj e_j+sl e_l)-u(n+sj e_j)) ] / (2 h_l)
 *     C_ijkl  = lambda d_ij d_kl + mu (d_ik d_jl + d_il d_jk)   (Lame constants,
 *               Sec. 2.4: the material model is stored as (lambda, mu))
 *
 *   Boundary data enter as source terms (Sec. 2.1): a traction t on box face F
 *   adds (t / h_perp) * mean of the 2^(d-1) cells containing the node and
 *   touching F.  Displacement boundary conditions are not diffused (Sec. 2.1);
 *   those degrees of freedom are fixed and eliminated.
 *
 *   Multigrid (Sec. 2.2, 2.3): Jacobi u <- u + w D^-1 (f - K u) (Sec. 2.3),
 *   two-colour Gauss-Seidel with colour-synchronous half-sweeps, full-weighting
 *   restriction R = P^T / 2^d, multilinear prolongation P, coarse operators
 *   re-discretised on averaged psi, CG on the bottom grid, V-cycles until
 *   ||f - K u|| <= rtol ||f||.
 *
 * Array layouts: node vectors are component-major, x fastest:
 *   u[k][z][y][x] -> u[k*NN + x + nx1*(y + ny1*z)]
 * cell scalars psi[z][y][x] -> psi[x + ncx*(y + ncy*z)].  2D drops z.
 * Boundary faces are ordered x-, x+, y-, y+, z-, z+; bc arrays are [face][3].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_TRACTION 0
#define ORC_DISPLACEMENT 1

typedef struct {
  int dim;
  long nc[3]; /* cells per axis (1 on inactive axes) */
  long nn[3]; /* nodes per axis (1 on inactive axes) */
  long NN;    /* nodes */
  long NC;    /* cells */
  double h[3];
  double C[3][3][3][3];
} grid_t;

static void grid_init(grid_t *g, int dim, const long *nc, const double *h,
                      double lam, double mu) {
  memset(g, 0, sizeof(*g));
  g->dim = dim;
  for (int a = 0; a < 3; ++a) {
    g->nc[a] = (a < dim) ? nc[a] : 1;
    g->nn[a] = (a < dim) ? nc[a] + 1 : 1;
    g->h[a] = (a < dim) ? h[a] : 1.0;
  }
  g->NN = g->nn[0] * g->nn[1] * g->nn[2];
  g->NC = g->nc[0] * g->nc[1] * g->nc[2];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l)
          g->C[i][j][k][l] = lam * (i == j) * (k == l) +
                             mu * ((i == k) * (j == l) + (i == l) * (j == k));
}

static long node_id(const grid_t *g, const long *n) {
  return n[0] + g->nn[0] * (n[1] + g->nn[1] * n[2]);
}

static int node_inside(const grid_t *g, const long *n) {
  for (int a = 0; a < g->dim; ++a)
    if (n[a] < 0 || n[a] >= g->nn[a]) return 0;
  return 1;
}

/* psi source: either an array of cell values or the indicator of one cell. */
typedef struct {
  const double *arr;
  long cell; /* used when arr == NULL */
} psi_src;

static double psi_cell(const grid_t *g, const psi_src *ps, const long *c) {
  for (int a = 0; a < g->dim; ++a)
    if (c[a] < 0 || c[a] >= g->nc[a]) return 0.0; /* psi = 0 outside the box */
  long id = c[0] + g->nc[0] * (c[1] + g->nc[1] * c[2]);
  if (ps->arr) return ps->arr[id];
  return id == ps->cell ? 1.0 : 0.0;
}

/* psiE(n, s e_j): mean of the 2^(d-1) cells sharing edge (n, n + s e_j). */
static double psi_edge(const grid_t *g, const psi_src *ps, const long *n, int j, int s) {
  double sum = 0.0;
  int cnt = 0;
  long c[3] = {0, 0, 0};
  for (int o = 0; o < 8; ++o) {
    int skip = 0;
    for (int a = 0; a < 3; ++a) {
      int bit = (o >> a) & 1;
      if (a >= g->dim) { if (bit) skip = 1; c[a] = 0; continue; }
      if (a == j) { if (bit) skip = 1; c[a] = (s > 0) ? n[a] : n[a] - 1; }
      else c[a] = n[a] - 1 + bit;
    }
    if (skip) continue;
    sum += psi_cell(g, ps, c);
    ++cnt;
  }
  return sum / cnt;
}

/* psiF(p), p = n + sj e_j/2 + sl e_l/2: 2D the cell at p, 3D mean of the two
 * cells p +- e_m/2. */
static double psi_face(const grid_t *g, const psi_src *ps, const long *n, int j, int sj,
                       int l, int sl) {
  long c[3] = {0, 0, 0};
  c[j] = (sj > 0) ? n[j] : n[j] - 1;
  c[l] = (sl > 0) ? n[l] : n[l] - 1;
  if (g->dim == 2) return psi_cell(g, ps, c);
  int m = 3 - j - l;
  double sum = 0.0;
  c[m] = n[m] - 1;
  sum += psi_cell(g, ps, c);
  c[m] = n[m];
  sum += psi_cell(g, ps, c);
  return 0.5 * sum;
}

static double u_at(const grid_t *g, const double *u, int k, const long *n) {
  if (!node_inside(g, n)) return 0.0; /* only ever multiplied by a zero weight */
  return u[(long)k * g->NN + node_id(g, n)];
}

/* (G_l u_k)(p) for p = n + sj e_j/2 + sl e_l/2 */
static double grad_at(const grid_t *g, const double *u, int k, const long *n, int j,
                      int sj, int l, int sl) {
  long nl[3] = {n[0], n[1], n[2]};
  long nj[3] = {n[0], n[1], n[2]};
  long njl[3] = {n[0], n[1], n[2]};
  nl[l] += sl;
  nj[j] += sj;
  njl[j] += sj;
  njl[l] += sl;
  return sl * ((u_at(g, u, k, nl) - u_at(g, u, k, n)) +
               (u_at(g, u, k, njl) - u_at(g, u, k, nj))) /
         (2.0 * g->h[l]);
}

/* All rows of eq. K at node n: out[i] = (Ku)_i(n), i < d.  The edge and face
 * means of psi are evaluated once per node and shared by the rows. */
static void K_node(const grid_t *g, const psi_src *ps, const double *u, const long *n,
                   double *out) {
  const int d = g->dim;
  double pe[3][2];       /* psiE(n, -e_j), psiE(n, +e_j) */
  double pf[3][3][2][2]; /* psiF for (j, l, sj, sl) */
  for (int j = 0; j < d; ++j) {
    pe[j][0] = psi_edge(g, ps, n, j, -1);
    pe[j][1] = psi_edge(g, ps, n, j, +1);
    for (int l = 0; l < d; ++l) {
      if (l == j) continue;
      for (int sj = 0; sj < 2; ++sj)
        for (int sl = 0; sl < 2; ++sl)
          pf[j][l][sj][sl] = psi_face(g, ps, n, j, 2 * sj - 1, l, 2 * sl - 1);
    }
  }
  for (int i = 0; i < d; ++i) {
    double acc = 0.0;
    /* direct terms, j = l */
    for (int j = 0; j < d; ++j) {
      long np[3] = {n[0], n[1], n[2]}, nm[3] = {n[0], n[1], n[2]};
      np[j] += 1;
      nm[j] -= 1;
      for (int k = 0; k < d; ++k) {
        double Cc = g->C[i][j][k][j];
        if (Cc == 0.0) continue;
        double uc = u_at(g, u, k, n);
        double flux = pe[j][1] * (u_at(g, u, k, np) - uc) - pe[j][0] * (uc - u_at(g, u, k, nm));
        acc -= Cc * flux / (g->h[j] * g->h[j]);
      }
    }
    /* cross terms, j != l */
    for (int j = 0; j < d; ++j)
      for (int l = 0; l < d; ++l) {
        if (j == l) continue;
        for (int sj = -1; sj <= 1; sj += 2)
          for (int sl = -1; sl <= 1; sl += 2) {
            double f = pf[j][l][(sj + 1) / 2][(sl + 1) / 2];
            if (f == 0.0) continue;
            double gsum = 0.0;
            for (int k = 0; k < d; ++k) {
              double Cc = g->C[i][j][k][l];
              if (Cc == 0.0) continue;
              gsum += Cc * grad_at(g, u, k, n, j, sj, l, sl);
            }
            acc -= sj * f * gsum / (2.0 * g->h[j]);
          }
      }
    out[i] = acc;
  }
}

static void node_of(const grid_t *g, long id, long *n) {
  n[0] = id % g->nn[0];
  n[1] = (id / g->nn[0]) % g->nn[1];
  n[2] = id / (g->nn[0] * g->nn[1]);
}

/* ---------------------------------------------------------------- masks -- */

/* Dirichlet DOF: node on a face whose kind for component k is DISPLACEMENT.
 * The value comes from the last such face in the order x-,x+,y-,y+,z-,z+. */
static int dirichlet(const grid_t *g, const int *kind, const double *val, const long *n,
                     int k, double *value) {
  int is = 0;
  for (int a = 0; a < g->dim; ++a)
    for (int side = 0; side < 2; ++side) {
      int F = 2 * a + side;
      long at = side ? g->nn[a] - 1 : 0;
      if (n[a] == at && kind[F * 3 + k] == ORC_DISPLACEMENT) {
        is = 1;
        if (value) *value = val[F * 3 + k];
      }
    }
  return is;
}

void orc_dirichlet_mask(int dim, const long *nc, const int *kind, const double *val,
                        uint8_t *mask, double *uD) {
  grid_t g;
  double h[3] = {1, 1, 1};
  grid_init(&g, dim, nc, h, 0, 0);
  for (long id = 0; id < g.NN; ++id) {
    long n[3];
    node_of(&g, id, n);
    for (int k = 0; k < dim; ++k) {
      double v = 0.0;
      int is = dirichlet(&g, kind, val, n, k, &v);
      if (mask) mask[(long)k * g.NN + id] = (uint8_t)is;
      if (uD) uD[(long)k * g.NN + id] = is ? v : 0.0;
    }
  }
}

/* ---------------------------------------------------------- operators -- */

void orc_apply(int dim, const long *nc, const double *h, double lam, double mu,
               const double *psi, const double *u, double *Ku) {
  grid_t g;
  grid_init(&g, dim, nc, h, lam, mu);
  psi_src ps = {psi, -1};
#pragma omp parallel for schedule(static)
  for (long id = 0; id < g.NN; ++id) {
    long n[3];
    double out[3];
    node_of(&g, id, n);
    K_node(&g, &ps, u, n, out);
    for (int i = 0; i < dim; ++i) Ku[(long)i * g.NN + id] = out[i];
  }
}

/* Diagonal of eq. K: coefficient of u_i(n) in row i.  Only the direct terms
 * carry it (C_ijil = 0 for j != l):  D_i = sum_j C_ijij (psiE+ + psiE-)/h_j^2. */
static double K_diag(const grid_t *g, const psi_src *ps, const long *n, int i) {
  double D = 0.0;
  for (int j = 0; j < g->dim; ++j)
    D += g->C[i][j][i][j] * (psi_edge(g, ps, n, j, +1) + psi_edge(g, ps, n, j, -1)) /
         (g->h[j] * g->h[j]);
  return D;
}

void orc_diag(int dim, const long *nc, const double *h, double lam, double mu,
              const double *psi, double *D) {
  grid_t g;
  grid_init(&g, dim, nc, h, lam, mu);
  psi_src ps = {psi, -1};
#pragma omp parallel for schedule(static)
  for (long id = 0; id < g.NN; ++id) {
    long n[3];
    node_of(&g, id, n);
    for (int i = 0; i < dim; ++i) D[(long)i * g.NN + id] = K_diag(&g, &ps, n, i);
  }
}

/* psi floor (the order parameter is bounded below so that void regions stay
 * near-singular rather than singular). */
void orc_floor(long ncell, const double *psi_raw, double floor_, double *psi) {
  for (long c = 0; c < ncell; ++c) psi[c] = psi_raw[c] > floor_ ? psi_raw[c] : floor_;
}

/* Right-hand side.  fA: body force plus traction source on free DOF, zero on
 * Dirichlet DOF.  uD: prescribed values (zero on free DOF).  fB = fA - K uD on
 * free DOF (the lifted load whose norm normalises the residual). */
void orc_rhs(int dim, const long *nc, const double *h, double lam, double mu,
             const double *psi, const int *kind, const double *val, const double *b,
             double *fA, double *fB, double *uD) {
  grid_t g;
  grid_init(&g, dim, nc, h, lam, mu);
  psi_src ps = {psi, -1};
  uint8_t *mask = (uint8_t *)malloc((size_t)dim * g.NN);
  orc_dirichlet_mask(dim, nc, kind, val, mask, uD);
  for (long id = 0; id < g.NN; ++id) {
    long n[3];
    node_of(&g, id, n);
    for (int k = 0; k < dim; ++k) {
      long q = (long)k * g.NN + id;
      if (mask[q]) { fA[q] = 0.0; continue; }
      double f = b ? b[q] : 0.0;
      for (int a = 0; a < dim; ++a)
        for (int side = 0; side < 2; ++side) {
          int F = 2 * a + side;
          long at = side ? g.nn[a] - 1 : 0;
          if (n[a] != at || kind[F * 3 + k] != ORC_TRACTION) continue;
          double t = val[F * 3 + k];
          if (t == 0.0) continue;
          /* mean of the 2^(d-1) cells containing n that touch face F */
          double sum = 0.0;
          int cnt = 0;
          long c[3] = {0, 0, 0};
          for (int o = 0; o < 4; ++o) {
            int oi = 0, skip = 0;
            for (int bax = 0; bax < 3; ++bax) {
              if (bax == a) { c[bax] = side ? g.nc[a] - 1 : 0; continue; }
              if (bax >= dim) { c[bax] = 0; continue; }
              int bit = (o >> oi) & 1;
              ++oi;
              c[bax] = n[bax] - 1 + bit;
            }
            if (o >= (1 << (dim - 1))) skip = 1;
            if (skip) continue;
            sum += psi_cell(&g, &ps, c);
            ++cnt;
          }
          f += t / g.h[a] * (sum / cnt);
        }
      fA[q] = f;
    }
  }
  if (fB) {
    double *KuD = (double *)malloc(sizeof(double) * dim * g.NN);
    orc_apply(dim, nc, h, lam, mu, psi, uD, KuD);
    for (long q = 0; q < (long)dim * g.NN; ++q) fB[q] = mask[q] ? 0.0 : fA[q] - KuD[q];
    free(KuD);
  }
  free(mask);
}

/* r = f - K u on free DOF, 0 on Dirichlet DOF. */
void orc_residual(int dim, const long *nc, const double *h, double lam, double mu,
                  const double *psi, const uint8_t *mask, const double *u,
                  const double *f, double *r) {
  grid_t g;
  grid_init(&g, dim, nc, h, lam, mu);
  orc_apply(dim, nc, h, lam, mu, psi, u, r);
  for (long q = 0; q < (long)dim * g.NN; ++q) r[q] = mask[q] ? 0.0 : f[q] - r[q];
}

static double norm2_free(long n, const double *r, const uint8_t *mask) {
  double s = 0.0;
  for (long q = 0; q < n; ++q)
    if (!mask[q]) s += r[q] * r[q];
  return sqrt(s);
}

/* Damped Jacobi (Sec. 2.3): u_out = u + omega D^-1 (f - K u) on free DOF. */
void orc_jacobi(int dim, const long *nc, const double *h, double lam, double mu,
                const double *psi, const uint8_t *mask, double omega, const double *u,
                const double *f, double *u_out) {
  grid_t g;
  grid_init(&g, dim, nc, h, lam, mu);
  long n3 = (long)dim * g.NN;
  double *r = (double *)malloc(sizeof(double) * n3);
  double *D = (double *)malloc(sizeof(double) * n3);
  orc_residual(dim, nc, h, lam, mu, psi, mask, u, f, r);
  orc_diag(dim, nc, h, lam, mu, psi, D);
  for (long q = 0; q < n3; ++q) u_out[q] = mask[q] ? u[q] : u[q] + omega * r[q] / D[q];
  free(r);
  free(D);
}

/* One colour-synchronous half-sweep of two-colour Gauss-Seidel: the residual
 * is taken from the state at the start of the half-sweep, and every component
 * of each node of colour (x+y+z) mod 2 == colour is updated with D^-1. */
void orc_rb_half(int dim, const long *nc, const double *h, double lam, double mu,
                 const double *psi, const uint8_t *mask, double omega, int colour,
                 const double *u, const double *f, double *u_out) {
  grid_t g;
  grid_init(&g, dim, nc, h, lam, mu);
  long n3 = (long)dim * g.NN;
  double *r = (double *)malloc(sizeof(double) * n3);
  double *D = (double *)malloc(sizeof(double) * n3);
  orc_residual(dim, nc, h, lam, mu, psi, mask, u, f, r);
  orc_diag(dim, nc, h, lam, mu, psi, D);
#pragma omp parallel for schedule(static)
  for (long id = 0; id < g.NN; ++id) {
    long n[3];
    node_of(&g, id, n);
    int c = (int)((n[0] + n[1] + n[2]) % 2);
    for (int k = 0; k < dim; ++k) {
      long q = (long)k * g.NN + id;
      u_out[q] = (mask[q] || c != colour) ? u[q] : u[q] + omega * r[q] / D[q];
    }
  }
  free(r);
  free(D);
}

/* ------------------------------------------------------------ transfers -- */

/* Multilinear prolongation weight of coarse node I for fine node n, per axis:
 * n even -> I = n/2 (1); n odd -> I = (n-1)/2 and (n+1)/2 (1/2 each). */
static double p_weight_axis(long n, long I) {
  if (n % 2 == 0) return (I * 2 == n) ? 1.0 : 0.0;
  if (I * 2 == n - 1 || I * 2 == n + 1) return 0.5;
  return 0.0;
}

/* u_fine += P e_coarse on free fine DOF. nc_coarse are coarse cell counts. */
void orc_prolong_add(int dim, const long *nc_coarse, const double *e,
                     const uint8_t *mask_fine, double *u_fine) {
  grid_t gc, gf;
  double h[3] = {1, 1, 1};
  long ncf[3] = {2 * nc_coarse[0], 2 * nc_coarse[1], dim > 2 ? 2 * nc_coarse[2] : 0};
  grid_init(&gc, dim, nc_coarse, h, 0, 0);
  grid_init(&gf, dim, ncf, h, 0, 0);
#pragma omp parallel for schedule(static)
  for (long id = 0; id < gf.NN; ++id) {
    long n[3];
    node_of(&gf, id, n);
    /* coarse candidates: I_a in { floor(n_a/2), ceil(n_a/2) } */
    long lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      if (a < dim) { lo[a] = n[a] / 2; hi[a] = (n[a] + 1) / 2; }
      else { lo[a] = hi[a] = 0; }
    }
    for (int k = 0; k < dim; ++k) {
      long q = (long)k * gf.NN + id;
      if (mask_fine[q]) continue;
      double acc = 0.0;
      for (long I2 = lo[2]; I2 <= hi[2]; ++I2)
        for (long I1 = lo[1]; I1 <= hi[1]; ++I1)
          for (long I0 = lo[0]; I0 <= hi[0]; ++I0) {
            long I[3] = {I0, I1, I2};
            double w = 1.0;
            for (int a = 0; a < dim; ++a) w *= p_weight_axis(n[a], I[a]);
            acc += w * e[(long)k * gc.NN + node_id(&gc, I)];
          }
      u_fine[q] += acc;
    }
  }
}

/* f_coarse = (P^T r_fine) / 2^d, zero on coarse Dirichlet DOF:
 * f_coarse(I) = 2^-d sum over fine nodes n of P(n, I) r(n). */
void orc_restrict(int dim, const long *nc_fine, const double *r, const uint8_t *mask_coarse,
                  double *f_coarse) {
  grid_t gc, gf;
  double h[3] = {1, 1, 1};
  long ncc[3] = {nc_fine[0] / 2, nc_fine[1] / 2, dim > 2 ? nc_fine[2] / 2 : 0};
  grid_init(&gc, dim, ncc, h, 0, 0);
  grid_init(&gf, dim, nc_fine, h, 0, 0);
  double scale = 1.0 / (double)(1 << dim);
#pragma omp parallel for schedule(static)
  for (long cid = 0; cid < gc.NN; ++cid) {
    long I[3];
    node_of(&gc, cid, I);
    /* the fine nodes with P(n, I) != 0 lie within one node of 2I */
    long lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      if (a < dim) { lo[a] = 2 * I[a] - 1; hi[a] = 2 * I[a] + 1; }
      else { lo[a] = hi[a] = 0; }
    }
    double acc[3] = {0, 0, 0};
    for (long n2 = lo[2]; n2 <= hi[2]; ++n2)
      for (long n1 = lo[1]; n1 <= hi[1]; ++n1)
        for (long n0 = lo[0]; n0 <= hi[0]; ++n0) {
          long n[3] = {n0, n1, n2};
          if (!node_inside(&gf, n)) continue;
          double w = 1.0;
          for (int a = 0; a < dim; ++a) w *= p_weight_axis(n[a], I[a]);
          long fid = node_id(&gf, n);
          for (int k = 0; k < dim; ++k) acc[k] += w * r[(long)k * gf.NN + fid];
        }
    for (int k = 0; k < dim; ++k) {
      long q = (long)k * gc.NN + cid;
      f_coarse[q] = mask_coarse[q] ? 0.0 : acc[k] * scale;
    }
  }
}

/* Coarse psi: mean of the 2^d child cells. */
void orc_coarsen_psi(int dim, const long *nc_fine, const double *psi_f, double *psi_c) {
  long ncc[3] = {nc_fine[0] / 2, nc_fine[1] / 2, dim > 2 ? nc_fine[2] / 2 : 1};
  long ncf2 = dim > 2 ? nc_fine[2] : 1;
  for (long k = 0; k < ncc[2]; ++k)
    for (long j = 0; j < ncc[1]; ++j)
      for (long i = 0; i < ncc[0]; ++i) {
        double s = 0.0;
        for (int o = 0; o < (1 << dim); ++o) {
          long fi = 2 * i + (o & 1), fj = 2 * j + ((o >> 1) & 1), fk = dim > 2 ? 2 * k + ((o >> 2) & 1) : 0;
          s += psi_f[fi + nc_fine[0] * (fj + nc_fine[1] * fk)];
        }
        (void)ncf2;
        psi_c[i + ncc[0] * (j + ncc[1] * k)] = s / (double)(1 << dim);
      }
}

/* -------------------------------------------------------------- bottom -- */

/* Conjugate gradients with diagonal (Jacobi) preconditioning on the free DOF:
 * solves K_FF d = (f - K x)_F and adds d to x.  Stops when ||r|| <= rtol ||r0||
 * (unpreconditioned residual) or after maxit iterations.  Returns the
 * iteration count. */
int orc_cg(int dim, const long *nc, const double *h, double lam, double mu,
           const double *psi, const uint8_t *mask, const double *f, double *x,
           double rtol, int maxit) {
  grid_t g;
  grid_init(&g, dim, nc, h, lam, mu);
  long n3 = (long)dim * g.NN;
  double *r = (double *)malloc(sizeof(double) * n3);
  double *z = (double *)malloc(sizeof(double) * n3);
  double *p = (double *)malloc(sizeof(double) * n3);
  double *Ap = (double *)malloc(sizeof(double) * n3);
  double *D = (double *)malloc(sizeof(double) * n3);
  orc_diag(dim, nc, h, lam, mu, psi, D);
  orc_residual(dim, nc, h, lam, mu, psi, mask, x, f, r);
  double rr = 0.0, rz = 0.0;
  for (long q = 0; q < n3; ++q) {
    z[q] = mask[q] ? 0.0 : r[q] / D[q];
    rr += r[q] * r[q];
    rz += r[q] * z[q];
  }
  double r0 = sqrt(rr);
  int it = 0;
  for (long q = 0; q < n3; ++q) p[q] = z[q];
  while (r0 > 0.0 && sqrt(rr) > rtol * r0 && it < maxit) {
    orc_apply(dim, nc, h, lam, mu, psi, p, Ap); /* p is zero on Dirichlet DOF */
    double pAp = 0.0;
    for (long q = 0; q < n3; ++q)
      if (!mask[q]) pAp += p[q] * Ap[q];
    if (!(pAp > 0.0)) break;
    double alpha = rz / pAp;
    double rr_new = 0.0, rz_new = 0.0;
    for (long q = 0; q < n3; ++q) {
      if (mask[q]) continue;
      x[q] += alpha * p[q];
      r[q] -= alpha * Ap[q];
      z[q] = r[q] / D[q];
      rr_new += r[q] * r[q];
      rz_new += r[q] * z[q];
    }
    double beta = rz_new / rz;
    rr = rr_new;
    rz = rz_new;
    for (long q = 0; q < n3; ++q) p[q] = mask[q] ? 0.0 : z[q] + beta * p[q];
    ++it;
  }
  free(r);
  free(z);
  free(p);
  free(Ap);
  free(D);
  return it;
}

/* ---------------------------------------------------------------- solve -- */

typedef struct {
  int smoother; /* 0 two-colour Gauss-Seidel, 1 damped Jacobi */
  double omega;
  int nu_pre, nu_post;
  double rtol;
  int max_cycles;
  double bottom_rtol;
  int bottom_max_iter; /* <= 0: 4 x (number of free DOF) */
  int krylov;          /* 1: V-cycle-preconditioned flexible CG (post-smoothing black first) */
} orc_opts;

typedef struct {
  long nc[3];
  double h[3];
  double *psi;
  uint8_t *mask;
  double *e, *f, *r, *tmp;
  long n3;
} level_t;

static int count_levels(int dim, const long *nc) {
  long c[3] = {nc[0], nc[1], dim > 2 ? nc[2] : 4};
  int L = 1;
  for (;;) {
    int ok = 1;
    for (int a = 0; a < dim; ++a)
      if (c[a] % 2 != 0 || c[a] < 4) ok = 0;
    if (!ok) break;
    for (int a = 0; a < dim; ++a) c[a] /= 2;
    ++L;
  }
  return L;
}

int orc_num_levels(int dim, const long *nc) { return count_levels(dim, nc); }

/* reverse: colours in the order black, red (the adjoint of red, black), used
 * for post-smoothing when the V-cycle preconditions CG. */
static void smooth(int dim, level_t *L, double lam, double mu, const orc_opts *o,
                   double *x, const double *f, int sweeps, int reverse) {
  for (int s = 0; s < sweeps; ++s) {
    if (o->smoother == 1) {
      orc_jacobi(dim, L->nc, L->h, lam, mu, L->psi, L->mask, o->omega, x, f, L->tmp);
      memcpy(x, L->tmp, sizeof(double) * L->n3);
    } else {
      for (int k = 0; k < 2; ++k) {
        int c = reverse ? 1 - k : k;
        orc_rb_half(dim, L->nc, L->h, lam, mu, L->psi, L->mask, o->omega, c, x, f, L->tmp);
        memcpy(x, L->tmp, sizeof(double) * L->n3);
      }
    }
  }
}

static long count_free(const level_t *L) {
  long c = 0;
  for (long q = 0; q < L->n3; ++q) c += !L->mask[q];
  return c;
}

static void vcycle(int dim, level_t *lev, int nlev, int l, double lam, double mu,
                   const orc_opts *o, double *x, const double *f) {
  level_t *L = &lev[l];
  if (l == nlev - 1) {
    int maxit = o->bottom_max_iter > 0 ? o->bottom_max_iter : (int)(4 * count_free(L));
    orc_cg(dim, L->nc, L->h, lam, mu, L->psi, L->mask, f, x, o->bottom_rtol, maxit);
    return;
  }
  level_t *C = &lev[l + 1];
  smooth(dim, L, lam, mu, o, x, f, o->nu_pre, 0);
  orc_residual(dim, L->nc, L->h, lam, mu, L->psi, L->mask, x, f, L->r);
  orc_restrict(dim, L->nc, L->r, C->mask, C->f);
  memset(C->e, 0, sizeof(double) * C->n3);
  vcycle(dim, lev, nlev, l + 1, lam, mu, o, C->e, C->f);
  orc_prolong_add(dim, C->nc, C->e, L->mask, x);
  smooth(dim, L, lam, mu, o, x, f, o->nu_post, o->krylov);
}

/* Full FP64 solve.  u: in = initial guess, out = solution (Dirichlet DOF set to
 * their values).  hist receives rho_0..rho_m (at most hist_cap entries).
 * Returns 0 converged, 1 not converged. */
int orc_solve(int dim, const long *nc, const double *h, double lam, double mu,
              const double *psi_raw, double psi_floor, const int *kind, const double *val,
              const double *b, int smoother, double omega, int nu_pre, int nu_post,
              double rtol, int max_cycles, double bottom_rtol, int bottom_max_iter,
              int krylov, double *u, double *hist, int hist_cap, int *n_cycles) {
  orc_opts o = {smoother, omega, nu_pre, nu_post, rtol, max_cycles, bottom_rtol, bottom_max_iter,
                krylov};
  int nlev = count_levels(dim, nc);
  level_t *lev = (level_t *)calloc(nlev, sizeof(level_t));
  for (int l = 0; l < nlev; ++l) {
    level_t *L = &lev[l];
    for (int a = 0; a < 3; ++a) {
      L->nc[a] = (a < dim) ? (l == 0 ? nc[a] : lev[l - 1].nc[a] / 2) : 0;
      L->h[a] = (a < dim) ? (l == 0 ? h[a] : 2.0 * lev[l - 1].h[a]) : 1.0;
    }
    long NC = 1, NN = 1;
    for (int a = 0; a < dim; ++a) { NC *= L->nc[a]; NN *= L->nc[a] + 1; }
    L->n3 = (long)dim * NN;
    L->psi = (double *)malloc(sizeof(double) * NC);
    L->mask = (uint8_t *)malloc(L->n3);
    L->e = (double *)calloc(L->n3, sizeof(double));
    L->f = (double *)calloc(L->n3, sizeof(double));
    L->r = (double *)calloc(L->n3, sizeof(double));
    L->tmp = (double *)calloc(L->n3, sizeof(double));
    if (l == 0) orc_floor(NC, psi_raw, psi_floor, L->psi);
    else orc_coarsen_psi(dim, lev[l - 1].nc, lev[l - 1].psi, L->psi);
    orc_dirichlet_mask(dim, L->nc, kind, val, L->mask, NULL);
  }
  level_t *T = &lev[0];
  double *fA = (double *)malloc(sizeof(double) * T->n3);
  double *fB = (double *)malloc(sizeof(double) * T->n3);
  double *uD = (double *)malloc(sizeof(double) * T->n3);
  orc_rhs(dim, T->nc, T->h, lam, mu, T->psi, kind, val, b, fA, fB, uD);
  for (long q = 0; q < T->n3; ++q)
    if (T->mask[q]) u[q] = uD[q];
  double fn = norm2_free(T->n3, fB, T->mask);
  int status = 1, m = 0;
  if (!krylov) {
    for (m = 0;; ++m) {
      orc_residual(dim, T->nc, T->h, lam, mu, T->psi, T->mask, u, fA, T->r);
      double rho = fn > 0.0 ? norm2_free(T->n3, T->r, T->mask) / fn : 0.0;
      if (m < hist_cap) hist[m] = rho;
      if (rho <= rtol) { status = 0; break; }
      if (m >= max_cycles) break;
      vcycle(dim, lev, nlev, 0, lam, mu, &o, u, fA);
    }
  } else {
    /* Flexible preconditioned CG (Polak-Ribiere beta), one V-cycle from zero
     * per iteration as the preconditioner z = M r. */
    long n3 = T->n3;
    double *r = (double *)malloc(sizeof(double) * n3), *z = (double *)malloc(sizeof(double) * n3);
    double *pv = (double *)malloc(sizeof(double) * n3), *q = (double *)malloc(sizeof(double) * n3);
    orc_residual(dim, T->nc, T->h, lam, mu, T->psi, T->mask, u, fA, r);
    double rho = fn > 0.0 ? norm2_free(n3, r, T->mask) / fn : 0.0;
    if (hist_cap > 0) hist[0] = rho;
    int restart = 1;
    double rz = 0.0;
    for (m = 0;;) {
      if (rho <= rtol) { status = 0; break; }
      if (m >= max_cycles) break;
      if (restart) {
        memset(z, 0, sizeof(double) * n3);
        vcycle(dim, lev, nlev, 0, lam, mu, &o, z, r);
        rz = 0.0;
        for (long i = 0; i < n3; ++i) if (!T->mask[i]) rz += r[i] * z[i];
        for (long i = 0; i < n3; ++i) pv[i] = T->mask[i] ? 0.0 : z[i];
        restart = 0;
      }
      orc_apply(dim, T->nc, T->h, lam, mu, T->psi, pv, q);
      double pq = 0.0;
      for (long i = 0; i < n3; ++i) if (!T->mask[i]) pq += pv[i] * q[i];
      if (!(pq > 0.0)) break;
      double alpha = rz / pq, rzold = 0.0;
      for (long i = 0; i < n3; ++i) {
        if (T->mask[i]) continue;
        u[i] += alpha * pv[i];
        r[i] -= alpha * q[i];
        rzold += r[i] * z[i];
      }
      ++m;
      rho = fn > 0.0 ? norm2_free(n3, r, T->mask) / fn : 0.0;
      if (rho <= rtol) {
        /* accept only if the true residual agrees; else restart from it */
        orc_residual(dim, T->nc, T->h, lam, mu, T->psi, T->mask, u, fA, r);
        rho = fn > 0.0 ? norm2_free(n3, r, T->mask) / fn : 0.0;
        if (m < hist_cap) hist[m] = rho;
        if (rho > rtol) restart = 1;
        continue;
      }
      if (m < hist_cap) hist[m] = rho;
      memset(z, 0, sizeof(double) * n3);
      vcycle(dim, lev, nlev, 0, lam, mu, &o, z, r);
      double rznew = 0.0;
      for (long i = 0; i < n3; ++i) if (!T->mask[i]) rznew += r[i] * z[i];
      double beta = (rznew - rzold) / rz;
      rz = rznew;
      for (long i = 0; i < n3; ++i) pv[i] = T->mask[i] ? 0.0 : z[i] + beta * pv[i];
    }
    free(r); free(z); free(pv); free(q);
  }
  *n_cycles = m;
  for (int l = 0; l < nlev; ++l) {
    free(lev[l].psi); free(lev[l].mask); free(lev[l].e);
    free(lev[l].f); free(lev[l].r); free(lev[l].tmp);
  }
  free(lev);
  free(fA); free(fB); free(uD);
  return status;
}

/* ----------------------------------------------------------- sensitivity -- */

/* dL/dpsi_c = -lam^T (dK/dpsi_c) u + lam^T (df/dpsi_c).
 * K is linear in psi, so dK/dpsi_c is eq. K evaluated with psi = indicator of
 * cell c; it touches only the 2^d corner nodes of c.  df/dpsi_c is the
 * traction source of the faces that c touches.  lam must be zero on Dirichlet
 * DOF; u carries its prescribed values there.  Optional rho: the cells hold
 * psi = max(rho^3, floor), and g is chained to dL/drho = 3 rho^2 dL/dpsi where
 * rho^3 > floor (0 elsewhere). */
void orc_sensitivity(int dim, const long *nc, const double *h, double lam_, double mu,
                     const int *kind, const double *val, const double *u,
                     const double *lam, const double *rho, double psi_floor, double *g) {
  grid_t gr;
  grid_init(&gr, dim, nc, h, lam_, mu);
#pragma omp parallel for schedule(static)
  for (long cid = 0; cid < gr.NC; ++cid) {
    psi_src ps = {NULL, cid};
    long c[3] = {cid % gr.nc[0], (cid / gr.nc[0]) % gr.nc[1], cid / (gr.nc[0] * gr.nc[1])};
    double acc = 0.0;
    for (int o = 0; o < (1 << dim); ++o) {
      long n[3] = {c[0] + (o & 1), c[1] + ((o >> 1) & 1), dim > 2 ? c[2] + ((o >> 2) & 1) : 0};
      long id = node_id(&gr, n);
      for (int i = 0; i < dim; ++i) {
        double li = lam[(long)i * gr.NN + id];
        if (li == 0.0) continue;
        double row[3];
        K_node(&gr, &ps, u, n, row);
        acc -= li * row[i];
        /* traction source: face F of the box touched by cell c and containing n */
        for (int a = 0; a < dim; ++a)
          for (int side = 0; side < 2; ++side) {
            int F = 2 * a + side;
            long cat = side ? gr.nc[a] - 1 : 0, nat = side ? gr.nn[a] - 1 : 0;
            if (c[a] != cat || n[a] != nat || kind[F * 3 + i] != ORC_TRACTION) continue;
            acc += li * val[F * 3 + i] / gr.h[a] / (double)(1 << (dim - 1));
          }
      }
    }
    if (rho) {
      double r3 = rho[cid] * rho[cid] * rho[cid];
      acc = (r3 > psi_floor) ? 3.0 * rho[cid] * rho[cid] * acc : 0.0;
    }
    g[cid] = acc;
  }
}
