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

/* ------------------------------------------------ plastic strain (J2) -- */

/* Stress with a plastic strain (Sec. 3.1): sigma = C (grad u - eps_p), so the
 * equilibrium div(psi sigma) + b = 0 reads K u = b - div(psi C eps_p).  The
 * plastic strain lives in the cells (3D; components xx, yy, zz, yz, xz, xy,
 * cell scalar arrays one after another).  The divergence is taken in the same
 * flux form as eq. K: component i at node n is
 *     sum_j ( S_ij(n, +j) - S_ij(n, -j) ) / h_j,
 * S_ij(n, s e_j) = mean over the 4 cells sharing the edge (n, n + s e_j) of
 * psi_c (C eps_p,c)_ij, cells outside the box counting 0.  For a uniform
 * eps_p this equals -K applied to the linear field eps_p x at every node (the
 * direct part of eq. K is the j = l term; the two quadrants of each cross term
 * sum to the edge mean), so a compatible uniform plastic strain in a free body
 * is stress-free.  fp = -div(psi C eps_p) is the load it adds. */
static void voigt_to_mat(const double *v, double e[3][3]) {
  e[0][0] = v[0]; e[1][1] = v[1]; e[2][2] = v[2];
  e[1][2] = e[2][1] = v[3];
  e[0][2] = e[2][0] = v[4];
  e[0][1] = e[1][0] = v[5];
}

static void cell_state(const double *a, long NC, long cid, int ncomp, double *out) {
  for (int q = 0; q < ncomp; ++q) out[q] = a[(long)q * NC + cid];
}

int orc_plastic_source(int dim, const long *nc, const double *h, double lam, double mu,
                       const double *psi, const double *eps_p, double *fp) {
  if (dim != 3) return -1;
  grid_t g;
  grid_init(&g, dim, nc, h, lam, mu);
#pragma omp parallel for schedule(static)
  for (long id = 0; id < g.NN; ++id) {
    long n[3];
    node_of(&g, id, n);
    double div[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < 3; ++j)
      for (int s = -1; s <= 1; s += 2) {
        /* S(n, s e_j): mean over the 4 cells around the edge */
        double S[3] = {0.0, 0.0, 0.0};
        for (int o = 0; o < 4; ++o) {
          long c[3];
          int b = 0;
          for (int a = 0; a < 3; ++a) {
            if (a == j) c[a] = (s > 0) ? n[a] : n[a] - 1;
            else c[a] = n[a] - 1 + ((o >> (b++)) & 1);
          }
          int inside = 1;
          for (int a = 0; a < 3; ++a)
            if (c[a] < 0 || c[a] >= g.nc[a]) inside = 0;
          if (!inside) continue;
          long cid = c[0] + g.nc[0] * (c[1] + g.nc[1] * c[2]);
          double v[6], e[3][3];
          cell_state(eps_p, g.NC, cid, 6, v);
          voigt_to_mat(v, e);
          for (int i = 0; i < 3; ++i) {
            double sij = 0.0;
            for (int k = 0; k < 3; ++k)
              for (int l = 0; l < 3; ++l) sij += g.C[i][j][k][l] * e[k][l];
            S[i] += psi[cid] * sij;
          }
        }
        for (int i = 0; i < 3; ++i) div[i] += s * (S[i] / 4.0) / g.h[j];
      }
    for (int i = 0; i < 3; ++i) fp[(long)i * g.NN + id] = -div[i];
  }
  return 0;
}

/* J2 plasticity with linear combined hardening (Sec. 3.1, eq. J2Plasticity):
 * eta = dev(sigma) - beta, f = |eta| - sqrt(2/3) K(alpha),
 * K(alpha) = sigma_Y + theta Hbar alpha; flow eps_p' = gamma eta/|eta|,
 * alpha' = sqrt(2/3) gamma, beta' = (2/3)(1 - theta) Hbar gamma eta/|eta|.
 * Integrated over one load step by the radial return of the cited scheme:
 *   eps      = sym(G u) at the cell centre (G: mean over the cell's four
 *              edges along l of the difference quotient of u_k),
 *   s_trial  = 2 mu dev(eps - eps_p),   eta_trial = s_trial - beta,
 *   f_trial  = |eta_trial| - sqrt(2/3) K(alpha);  elastic if f_trial <= 0,
 *   else dgamma solves the consistency condition of the updated state,
 *   |eta_trial| - (2 mu + (2/3)(1-theta) Hbar) dgamma
 *        = sqrt(2/3) K(alpha + sqrt(2/3) dgamma),
 *   i.e. dgamma = f_trial / (2 mu + (2/3) Hbar), and with n = eta_trial/|eta_trial|
 *   eps_p += dgamma n, alpha += sqrt(2/3) dgamma,
 *   beta += (2/3)(1 - theta) Hbar dgamma n.
 * State arrays per cell: eps_p and beta 6 components (xx, yy, zz, yz, xz,
 * xy), alpha one.  Returns the number of cells that yielded. */
int orc_return_map(int dim, const long *nc, const double *h, double lam, double mu,
                   double sigma_y, double hbar, double theta, const double *u, double *eps_p,
                   double *alpha, double *beta) {
  if (dim != 3) return -1;
  grid_t g;
  grid_init(&g, dim, nc, h, lam, mu);
  long nplastic = 0;
  const double r23 = sqrt(2.0 / 3.0);
#pragma omp parallel for schedule(static) reduction(+ : nplastic)
  for (long cid = 0; cid < g.NC; ++cid) {
    long c[3] = {cid % g.nc[0], (cid / g.nc[0]) % g.nc[1], cid / (g.nc[0] * g.nc[1])};
    /* cell gradient G[k][l] = d u_k / d x_l */
    double G[3][3];
    for (int k = 0; k < 3; ++k)
      for (int l = 0; l < 3; ++l) {
        double acc = 0.0;
        for (int o = 0; o < 4; ++o) {
          long n0[3], n1[3];
          int b = 0;
          for (int a = 0; a < 3; ++a) {
            if (a == l) { n0[a] = c[a]; n1[a] = c[a] + 1; }
            else { n0[a] = n1[a] = c[a] + ((o >> (b++)) & 1); }
          }
          acc += (u[(long)k * g.NN + node_id(&g, n1)] - u[(long)k * g.NN + node_id(&g, n0)]) /
                 g.h[l];
        }
        G[k][l] = acc / 4.0;
      }
    double eps[3][3], ep[3][3], bt[3][3], v[6];
    for (int k = 0; k < 3; ++k)
      for (int l = 0; l < 3; ++l) eps[k][l] = 0.5 * (G[k][l] + G[l][k]);
    cell_state(eps_p, g.NC, cid, 6, v);
    voigt_to_mat(v, ep);
    cell_state(beta, g.NC, cid, 6, v);
    voigt_to_mat(v, bt);
    const double a0 = alpha[cid];
    /* trial deviatoric stress and relative stress */
    double ee[3][3], tr = 0.0;
    for (int k = 0; k < 3; ++k)
      for (int l = 0; l < 3; ++l) ee[k][l] = eps[k][l] - ep[k][l];
    for (int k = 0; k < 3; ++k) tr += ee[k][k];
    double eta[3][3], nrm2 = 0.0;
    for (int k = 0; k < 3; ++k)
      for (int l = 0; l < 3; ++l) {
        const double s = 2.0 * mu * (ee[k][l] - (k == l ? tr / 3.0 : 0.0));
        eta[k][l] = s - bt[k][l];
        nrm2 += eta[k][l] * eta[k][l];
      }
    const double nrm = sqrt(nrm2);
    const double ftrial = nrm - r23 * (sigma_y + theta * hbar * a0);
    if (!(ftrial > 0.0)) continue;
    ++nplastic;
    const double dg = ftrial / (2.0 * mu + (2.0 / 3.0) * hbar);
    double nv[3][3];
    for (int k = 0; k < 3; ++k)
      for (int l = 0; l < 3; ++l) nv[k][l] = eta[k][l] / nrm;
    const int vi[6] = {0, 1, 2, 1, 0, 0}, vj[6] = {0, 1, 2, 2, 2, 1};
    for (int q = 0; q < 6; ++q) {
      eps_p[(long)q * g.NC + cid] += dg * nv[vi[q]][vj[q]];
      beta[(long)q * g.NC + cid] += (2.0 / 3.0) * (1.0 - theta) * hbar * dg * nv[vi[q]][vj[q]];
    }
    alpha[cid] = a0 + r23 * dg;
  }
  return (int)nplastic;
}

/* ------------------------------------------------ phase-field fracture -- */

/* Hybrid phase-field fracture (Sec. 3.2, eqs. PFFracture, PFFractureGL).  The
 * equilibrium is the SBM equation with psi = g(c) + eta (g(c) = 4c^3 - 3c^4,
 * eta = 1e-4): linear, the elastic solve of this library.  The crack field c
 * lives in the cells.  Per cell, from the strain eps = sym(G u) (the cell
 * gradient of the corner nodes, as for plasticity; plane strain in 2D):
 *   eigenvalues e_i of eps (2D: the in-plane pair, the zero out-of-plane
 *   strain contributes nothing to either part),
 *   W0+- = lambda/2 (sum_i <e_i>+-)^2 + mu sum_i <e_i>+-^2,
 *   H <- max(H, W0+) (the history field), and the cell is held intact
 *   (c = 1) where W0+ < W0-.
 * Eigenvalues by cyclic Jacobi rotations (3D) or the closed form (2D). */
static void sym_eigs(int d, double a[3][3], double *e) {
  if (d == 2) {
    const double m = 0.5 * (a[0][0] + a[1][1]);
    const double r = sqrt(0.25 * (a[0][0] - a[1][1]) * (a[0][0] - a[1][1]) + a[0][1] * a[0][1]);
    e[0] = m + r;
    e[1] = m - r;
    return;
  }
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = fabs(a[0][1]) + fabs(a[0][2]) + fabs(a[1][2]);
    if (off == 0.0) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (a[p][q] == 0.0) continue;
        const double th = 0.5 * (a[q][q] - a[p][p]) / a[p][q];
        const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
        /* A <- J^T A J with the rotation in the (p, q) plane */
        for (int k = 0; k < 3; ++k) {
          const double akp = a[k][p], akq = a[k][q];
          a[k][p] = cs * akp - sn * akq;
          a[k][q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < 3; ++k) {
          const double apk = a[p][k], aqk = a[q][k];
          a[p][k] = cs * apk - sn * aqk;
          a[q][k] = sn * apk + cs * aqk;
        }
      }
  }
  for (int i = 0; i < 3; ++i) e[i] = a[i][i];
}

static void cell_grad(const grid_t *g, const double *u, const long *c, double G[3][3]) {
  const int d = g->dim;
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) G[k][l] = 0.0;
  const int ne = 1 << (d - 1); /* edges per axis */
  for (int k = 0; k < d; ++k)
    for (int l = 0; l < d; ++l) {
      double acc = 0.0;
      for (int o = 0; o < ne; ++o) {
        long n0[3] = {0, 0, 0}, n1[3] = {0, 0, 0};
        int b = 0;
        for (int a = 0; a < d; ++a) {
          if (a == l) { n0[a] = c[a]; n1[a] = c[a] + 1; }
          else { n0[a] = n1[a] = c[a] + ((o >> (b++)) & 1); }
        }
        acc += (u[(long)k * g->NN + node_id(g, n1)] - u[(long)k * g->NN + node_id(g, n0)]) /
               g->h[l];
      }
      G[k][l] = acc / ne;
    }
}

void orc_crack_drive(int dim, const long *nc, const double *h, double lam, double mu,
                     const double *u, double *H, uint8_t *intact) {
  grid_t g;
  grid_init(&g, dim, nc, h, lam, mu);
#pragma omp parallel for schedule(static)
  for (long cid = 0; cid < g.NC; ++cid) {
    long c[3] = {cid % g.nc[0], (cid / g.nc[0]) % g.nc[1], dim > 2 ? cid / (g.nc[0] * g.nc[1]) : 0};
    double G[3][3], eps[3][3], e[3] = {0.0, 0.0, 0.0};
    cell_grad(&g, u, c, G);
    for (int k = 0; k < 3; ++k)
      for (int l = 0; l < 3; ++l) eps[k][l] = 0.5 * (G[k][l] + G[l][k]);
    sym_eigs(dim, eps, e);
    double tp = 0.0, tm = 0.0, sp = 0.0, sm = 0.0;
    for (int i = 0; i < dim; ++i) {
      const double ep = e[i] > 0.0 ? e[i] : 0.0, em = e[i] < 0.0 ? e[i] : 0.0;
      tp += ep; tm += em;
      sp += ep * ep; sm += em * em;
    }
    const double wp = 0.5 * lam * tp * tp + mu * sp, wm = 0.5 * lam * tm * tm + mu * sm;
    if (wp > H[cid]) H[cid] = wp;
    intact[cid] = wp < wm;
  }
}

/* One explicit Ginzburg-Landau step (eq. PFFractureGL) on the cells:
 *   c <- c - dt M [ g'(c) H - Gc (2 xi lap(c) + w'(c) / (2 xi)) ],
 * g' = 12 c^2 - 12 c^3, w = 1 - g so w' = -g'; lap(c) is the cell Laplacian
 * (3 or 5 / 7-point) with zero flux across the box faces.  The crack field
 * lives in [0, 1] (0 in the crack, 1 in intact material, Sec. 3.2), so the
 * step is projected onto that interval (a NaN stays NaN); intact cells are
 * set to 1 (eq. PFFracture, last line).  Also returns psi = g(c) + eta of the
 * new field (the SBM indicator of the next solve). */
void orc_phase_step(int dim, const long *nc, const double *h, const double *c0, const double *H,
                    const uint8_t *intact, double Gc, double xi, double M, double dt,
                    double eta, double *c1, double *psi) {
  long n[3] = {nc[0], nc[1], dim > 2 ? nc[2] : 1};
  const long NC = n[0] * n[1] * n[2];
#pragma omp parallel for schedule(static)
  for (long cid = 0; cid < NC; ++cid) {
    long ci[3] = {cid % n[0], (cid / n[0]) % n[1], cid / (n[0] * n[1])};
    const double cc = c0[cid];
    double lap = 0.0;
    long stride = 1;
    for (int a = 0; a < dim; ++a) {
      const double cm = ci[a] > 0 ? c0[cid - stride] : cc;
      const double cp = ci[a] < n[a] - 1 ? c0[cid + stride] : cc;
      lap += (cp - 2.0 * cc + cm) / (h[a] * h[a]);
      stride *= n[a];
    }
    const double gp = 12.0 * cc * cc - 12.0 * cc * cc * cc;
    const double wp = -gp;
    double cn = cc - dt * M * (gp * H[cid] - Gc * (2.0 * xi * lap + wp / (2.0 * xi)));
    if (cn < 0.0) cn = 0.0;
    if (cn > 1.0) cn = 1.0;
    if (intact[cid]) cn = 1.0;
    c1[cid] = cn;
    psi[cid] = 4.0 * cn * cn * cn - 3.0 * cn * cn * cn * cn + eta;
  }
}

/* Diffuse traction on the diffuse boundary (Sec. 2.1, eq. SBMLinearElasticity):
 * the traction t0 of the sharp boundary, extended along the normals as t^0
 * (constant across the diffuse band), enters the load as t^0 |grad psi|.  In
 * the sign convention of K u = f (f = b + t for a traction t with the
 * outward normal of the solid), the load of node n is
 *     f(n) = t^0(n) |grad psi(n)| + p grad psi(n),
 * the second term being a pressure p acting on the solid from the empty side
 * (t = -p n_out with n_out = -grad psi / |grad psi|, so t |grad psi| =
 * p grad psi: no normal has to be formed).  psi = max(psi_raw, floor).  The
 * node gradient along axis a is the mean, over the 2^(d-1) pairs of cells
 * that face each other across the node along a, of their difference quotient;
 * a cell outside the box takes the value of the nearest cell inside, so the
 * box faces (whose tractions are the box-face sources) add nothing here.
 * t_hat: node field, dim components (NULL: none). */
static double psi_clamped(const grid_t *g, const double *psi, const long *c) {
  long q[3];
  for (int a = 0; a < 3; ++a) {
    q[a] = a < g->dim ? c[a] : 0;
    if (q[a] < 0) q[a] = 0;
    if (q[a] > g->nc[a] - 1) q[a] = g->nc[a] - 1;
  }
  return psi[q[0] + g->nc[0] * (q[1] + g->nc[1] * q[2])];
}

void orc_diffuse_traction(int dim, const long *nc, const double *h, const double *psi_raw,
                          double floor_, const double *t_hat, double p, double *f) {
  grid_t g;
  grid_init(&g, dim, nc, h, 0.0, 0.0);
  double *psi = (double *)malloc(sizeof(double) * g.NC);
  orc_floor(g.NC, psi_raw, floor_, psi);
  const int npair = 1 << (dim - 1);
  for (long id = 0; id < g.NN; ++id) {
    long n[3];
    node_of(&g, id, n);
    double grad[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < dim; ++a) {
      double acc = 0.0;
      for (int o = 0; o < npair; ++o) {
        long lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        int bit = 0;
        for (int e = 0; e < dim; ++e) {
          if (e == a) {
            lo[e] = n[e] - 1;
            hi[e] = n[e];
          } else {
            lo[e] = hi[e] = n[e] - 1 + ((o >> bit) & 1);
            ++bit;
          }
        }
        acc += psi_clamped(&g, psi, hi) - psi_clamped(&g, psi, lo);
      }
      grad[a] = acc / npair / g.h[a];
    }
    double mag = 0.0;
    for (int a = 0; a < dim; ++a) mag += grad[a] * grad[a];
    mag = sqrt(mag);
    for (int k = 0; k < dim; ++k) {
      const long q = (long)k * g.NN + id;
      f[q] = (t_hat ? t_hat[q] * mag : 0.0) + p * grad[k];
    }
  }
  free(psi);
}

/* ======================================================================
 * Block-structured adaptive composite solve (BSAMR).
 *
 * The paper solves on block-structured AMR levels of equal cell size that
 * exchange data by averaging (fine to coarse) and ghost cells (coarse to
 * fine), treats the refined levels as an extension of the multigrid level
 * sequence (Sec. 2.2), and pads levels with an extra ghost layer so that
 * restriction keeps its translational symmetry and no special coarse-fine
 * stencil is needed (Sec. 2.2, reflux-free).  The details live in a cited
 * work; the reading implemented here:
 *
 *  - AMR level a (0..A) has spacing h0 / 2^a and is stored densely over the
 *    whole box; levels a >= 1 are active on a union of cubic blocks of bc
 *    cells.  Level-a cells are tagged where |grad psi| h > threshold
 *    (central differences, clamped at the box; Sec. 3.3 uses 0.05); a
 *    level-(a+1) block is active if a tagged level-a cell lies in its
 *    footprint grown by one cell; every active block has its parent active,
 *    and the parent's neighbours on the sides the block touches.
 *  - Node classes of level a >= 1: 1 interior (unknown), 2 interface (on
 *    the boundary of the active region inside the box: owned by level a-1),
 *    3 and 4 the first and second layer outside.  Classes 2-4 are ghosts
 *    filled by tensor-product quadratic interpolation from level a-1.
 *  - psi is sampled per level; covered coarse cells take the mean of their
 *    children.  Covered coarse nodes take the injected fine values.
 *  - Composite residual: fine residual on classes 1-3 (padded region);
 *    coarse nodes on or inside the fine region take R of it; other coarse
 *    nodes take their own residual.
 *  - Composite cycle: full-approximation (FAS) multilevel cycle over the AMR
 *    levels (smooth level a, restrict its padded residual, coarse FAS load
 *    R w + K_c x_c on covered/interface nodes, recurse, correct with
 *    P(x_c - inject(x_f)), smooth), ending in the uniform V-cycle of the
 *    base grid; applied in correction form inside an FP64 outer loop.
 * ====================================================================== */

#define AMR_MAXL 4

typedef struct {
  int dim, A, bc;
  double lam, mu;
  int kind[18];
  double val[18];
  grid_t g[AMR_MAXL];         /* dense grid of each AMR level */
  long nb[AMR_MAXL][3];       /* blocks per axis (a >= 1) */
  uint8_t *blk[AMR_MAXL];     /* block flags (a >= 1) */
  uint8_t *cls[AMR_MAXL];     /* node classes (a >= 1) */
  double *psi[AMR_MAXL];      /* floored, averaged-down psi */
  uint8_t *dm[AMR_MAXL];      /* Dirichlet masks */
  double *uD[AMR_MAXL];       /* prescribed values */
  double *fP[AMR_MAXL];       /* loads */
  orc_opts o;
  level_t *hier;              /* uniform hierarchy of the base level */
  int nlev;
  double fnorm;
} amr_t;


/* Cells tagged for refinement: |grad psi| h > thresh with central differences
 * (neighbour indices clamped to the box), h the largest spacing. */
void orc_amr_tags(int dim, const long *nc, const double *h, const double *psi, double thresh,
                  uint8_t *tags) {
  grid_t g;
  grid_init(&g, dim, nc, h, 0, 0);
  double hmax = 0.0;
  for (int a = 0; a < dim; ++a) hmax = h[a] > hmax ? h[a] : hmax;
  for (long c = 0; c < g.NC; ++c) {
    long ci[3] = {c % g.nc[0], (c / g.nc[0]) % g.nc[1], c / (g.nc[0] * g.nc[1])};
    double s = 0.0;
    for (int a = 0; a < dim; ++a) {
      long p[3] = {ci[0], ci[1], ci[2]}, m[3] = {ci[0], ci[1], ci[2]};
      p[a] = ci[a] + 1 < g.nc[a] ? ci[a] + 1 : ci[a];
      m[a] = ci[a] > 0 ? ci[a] - 1 : ci[a];
      double d = psi[p[0] + g.nc[0] * (p[1] + g.nc[1] * p[2])] -
                 psi[m[0] + g.nc[0] * (m[1] + g.nc[1] * m[2])];
      double gr = d / (2.0 * h[a]);
      s = s + gr * gr;
    }
    tags[c] = (s * (hmax * hmax) > thresh * thresh) ? 1 : 0;
  }
}

/* Point clustering of flagged blocks into boxes (the Berger-Rigoutsos
 * algorithm the paper's AMR uses for regridding, Sec. 2.2): a box is the
 * bounding box of the flags it holds; it is accepted when flags >= eff *
 * volume; otherwise it is cut in two and each part is clustered again:
 *   (1) at a hole: an interior slab with no flag (the signature, the flag
 *       count per slab, is 0 there); first axis that has one, the hole
 *       nearest the middle of the box, the lower one on a tie; the hole slab
 *       belongs to neither part;
 *   (2) else at the strongest inflection of the signature: Lap(i) =
 *       S(i-1) - 2 S(i) + S(i+1) for interior slabs, a cut between slabs i and
 *       i+1 where Lap(i) Lap(i+1) < 0, strength |Lap(i+1) - Lap(i)|; the
 *       strongest over all axes, the first found (axis order, then i
 *       ascending) on a tie;
 *   (3) else in the middle of the longest axis (first longest), the lower
 *       half taking the middle slab.
 * Every block inside an accepted box is flagged in out.  Boxes in block
 * units, [lo, hi] inclusive.  Returns the number of accepted boxes; when
 * boxes != NULL, writes 6 longs (lo[3], hi[3]) per box (at most max_boxes). */
typedef struct {
  int dim;
  long n[3];
  const uint8_t *in;
  uint8_t *out;
  double eff;
  long nbox, max_boxes;
  long *boxes;
} br_t;

static int br_flag(const br_t *b, long x, long y, long z) {
  return b->in[x + b->n[0] * (y + b->n[1] * z)] != 0;
}

static void br_box(br_t *b, const long *lo0, const long *hi0) {
  long lo[3] = {lo0[0], lo0[1], lo0[2]}, hi[3] = {hi0[0], hi0[1], hi0[2]};
  /* shrink to the bounding box of the flags inside */
  long blo[3] = {hi[0] + 1, hi[1] + 1, hi[2] + 1}, bhi[3] = {lo[0] - 1, lo[1] - 1, lo[2] - 1};
  long cnt = 0;
  for (long z = lo[2]; z <= hi[2]; ++z)
    for (long y = lo[1]; y <= hi[1]; ++y)
      for (long x = lo[0]; x <= hi[0]; ++x) {
        if (!br_flag(b, x, y, z)) continue;
        ++cnt;
        const long p[3] = {x, y, z};
        for (int a = 0; a < 3; ++a) {
          if (p[a] < blo[a]) blo[a] = p[a];
          if (p[a] > bhi[a]) bhi[a] = p[a];
        }
      }
  if (cnt == 0) return;
  for (int a = 0; a < 3; ++a) { lo[a] = blo[a]; hi[a] = bhi[a]; }
  double vol = 1.0;
  for (int a = 0; a < 3; ++a) vol *= (double)(hi[a] - lo[a] + 1);
  if ((double)cnt >= b->eff * vol) {
    for (long z = lo[2]; z <= hi[2]; ++z)
      for (long y = lo[1]; y <= hi[1]; ++y)
        for (long x = lo[0]; x <= hi[0]; ++x) b->out[x + b->n[0] * (y + b->n[1] * z)] = 1;
    if (b->boxes && b->nbox < b->max_boxes)
      for (int a = 0; a < 3; ++a) {
        b->boxes[6 * b->nbox + a] = lo[a];
        b->boxes[6 * b->nbox + 3 + a] = hi[a];
      }
    ++b->nbox;
    return;
  }
  /* signatures */
  long *sig[3] = {0, 0, 0};
  for (int a = 0; a < b->dim; ++a) sig[a] = (long *)calloc(hi[a] - lo[a] + 1, sizeof(long));
  for (long z = lo[2]; z <= hi[2]; ++z)
    for (long y = lo[1]; y <= hi[1]; ++y)
      for (long x = lo[0]; x <= hi[0]; ++x) {
        if (!br_flag(b, x, y, z)) continue;
        const long p[3] = {x, y, z};
        for (int a = 0; a < b->dim; ++a) ++sig[a][p[a] - lo[a]];
      }
  int cut_axis = -1;
  long cut_lo_end = 0, cut_hi_start = 0; /* lower part ends at, upper part starts at */
  /* (1) holes */
  for (int a = 0; a < b->dim && cut_axis < 0; ++a) {
    long best = -1, bestd = 0;
    for (long i = lo[a] + 1; i < hi[a]; ++i) {
      if (sig[a][i - lo[a]] != 0) continue;
      long dist = 2 * i - (lo[a] + hi[a]);
      if (dist < 0) dist = -dist;
      if (best < 0 || dist < bestd) { best = i; bestd = dist; }
    }
    if (best >= 0) { cut_axis = a; cut_lo_end = best - 1; cut_hi_start = best + 1; }
  }
  /* (2) inflections */
  if (cut_axis < 0) {
    long best_s = 0;
    for (int a = 0; a < b->dim; ++a) {
      for (long i = lo[a] + 1; i + 1 <= hi[a] - 1; ++i) {
        const long *S = sig[a];
        long l0 = S[i - 1 - lo[a]] - 2 * S[i - lo[a]] + S[i + 1 - lo[a]];
        long l1 = S[i - lo[a]] - 2 * S[i + 1 - lo[a]] + S[i + 2 - lo[a]];
        if (!((l0 < 0 && l1 > 0) || (l0 > 0 && l1 < 0))) continue;
        long st = l1 - l0;
        if (st < 0) st = -st;
        if (st > best_s) { best_s = st; cut_axis = a; cut_lo_end = i; cut_hi_start = i + 1; }
      }
    }
  }
  /* (3) middle of the longest axis */
  if (cut_axis < 0) {
    long len = 0;
    for (int a = 0; a < b->dim; ++a)
      if (hi[a] - lo[a] + 1 > len) { len = hi[a] - lo[a] + 1; cut_axis = a; }
    const long mid = (lo[cut_axis] + hi[cut_axis]) / 2;
    cut_lo_end = mid;
    cut_hi_start = mid + 1;
  }
  for (int a = 0; a < b->dim; ++a) free(sig[a]);
  long lo1[3] = {lo[0], lo[1], lo[2]}, hi1[3] = {hi[0], hi[1], hi[2]};
  long lo2[3] = {lo[0], lo[1], lo[2]}, hi2[3] = {hi[0], hi[1], hi[2]};
  hi1[cut_axis] = cut_lo_end;
  lo2[cut_axis] = cut_hi_start;
  br_box(b, lo1, hi1);
  br_box(b, lo2, hi2);
}

long orc_br_cluster(int dim, const long *nb, const uint8_t *in, double eff, uint8_t *out,
                    long *boxes, long max_boxes) {
  br_t b;
  memset(&b, 0, sizeof(b));
  b.dim = dim;
  for (int a = 0; a < 3; ++a) b.n[a] = a < dim ? nb[a] : 1;
  b.in = in;
  b.out = out;
  b.eff = eff;
  b.boxes = boxes;
  b.max_boxes = max_boxes;
  memset(out, 0, (size_t)(b.n[0] * b.n[1] * b.n[2]));
  const long lo[3] = {0, 0, 0}, hi[3] = {b.n[0] - 1, b.n[1] - 1, b.n[2] - 1};
  br_box(&b, lo, hi);
  return b.nbox;
}

/* Block flags of levels 1..A from the tags of levels 0..A-1; with eff > 0
 * the flags of each level, finest first, are replaced by the blocks of their
 * Berger-Rigoutsos boxes before they nest into the next coarser level. */
static void amr_cluster_level(amr_t *m, int a, double eff) {
  const long nbt = m->nb[a][0] * m->nb[a][1] * m->nb[a][2];
  uint8_t *tmp = (uint8_t *)malloc(nbt);
  orc_br_cluster(m->dim, m->nb[a], m->blk[a], eff, tmp, NULL, 0);
  memcpy(m->blk[a], tmp, nbt);
  free(tmp);
}

static void amr_blocks(amr_t *m, uint8_t *const *tags, double eff) {
  const int d = m->dim;
  for (int a = 1; a <= m->A; ++a) {
    grid_t *gc = &m->g[a - 1];
    long half = m->bc / 2; /* a block covers bc/2 coarse cells per axis */
    long nbt = m->nb[a][0] * m->nb[a][1] * m->nb[a][2];
    for (long b = 0; b < nbt; ++b) {
      long bi[3] = {b % m->nb[a][0], (b / m->nb[a][0]) % m->nb[a][1], b / (m->nb[a][0] * m->nb[a][1])};
      long lo[3], hi[3];
      for (int ax = 0; ax < 3; ++ax) {
        if (ax < d) {
          lo[ax] = bi[ax] * half - 1;
          hi[ax] = bi[ax] * half + half; /* inclusive: footprint grown by one cell */
          if (lo[ax] < 0) lo[ax] = 0;
          if (hi[ax] > gc->nc[ax] - 1) hi[ax] = gc->nc[ax] - 1;
        } else { lo[ax] = hi[ax] = 0; }
      }
      int on = 0;
      for (long k = lo[2]; k <= hi[2] && !on; ++k)
        for (long j = lo[1]; j <= hi[1] && !on; ++j)
          for (long i = lo[0]; i <= hi[0] && !on; ++i)
            if (tags[a - 1][i + gc->nc[0] * (j + gc->nc[1] * k)]) on = 1;
      m->blk[a][b] = (uint8_t)on;
    }
  }
  /* nesting, finest first: parent and the parent's neighbours on the sides
   * the block touches */
  for (int a = m->A; a >= 2; --a) {
    if (eff > 0.0) amr_cluster_level(m, a, eff);
    long nbt = m->nb[a][0] * m->nb[a][1] * m->nb[a][2];
    for (long b = 0; b < nbt; ++b) {
      if (!m->blk[a][b]) continue;
      long bi[3] = {b % m->nb[a][0], (b / m->nb[a][0]) % m->nb[a][1], b / (m->nb[a][0] * m->nb[a][1])};
      long pb[3], sgn[3];
      for (int ax = 0; ax < 3; ++ax) {
        pb[ax] = bi[ax] / 2;
        sgn[ax] = (ax < d) ? ((bi[ax] % 2) ? 1 : -1) : 0;
      }
      for (int o = 0; o < 8; ++o) {
        long q[3];
        int ok = 1;
        for (int ax = 0; ax < 3; ++ax) {
          int bit = (o >> ax) & 1;
          if (ax >= d && bit) ok = 0;
          q[ax] = pb[ax] + (bit ? sgn[ax] : 0);
          if (ax < d && (q[ax] < 0 || q[ax] >= m->nb[a - 1][ax])) ok = 0;
        }
        if (!ok) continue;
        m->blk[a - 1][q[0] + m->nb[a - 1][0] * (q[1] + m->nb[a - 1][1] * q[2])] = 1;
      }
    }
  }
  if (eff > 0.0 && m->A >= 1) amr_cluster_level(m, 1, eff);
}

static int amr_cell_active(const amr_t *m, int a, const long *c) {
  for (int ax = 0; ax < m->dim; ++ax)
    if (c[ax] < 0 || c[ax] >= m->g[a].nc[ax]) return -1; /* outside the box */
  long b[3] = {0, 0, 0};
  for (int ax = 0; ax < m->dim; ++ax) b[ax] = c[ax] / m->bc;
  return m->blk[a][b[0] + m->nb[a][0] * (b[1] + m->nb[a][1] * b[2])];
}

/* Node classes of level a >= 1 (0 none, 1 interior, 2 interface, 3/4 outer layers). */
static void amr_classify(amr_t *m, int a) {
  grid_t *g = &m->g[a];
  const int d = m->dim;
  uint8_t *clo = (uint8_t *)calloc(g->NN, 1); /* in the closure of the active region */
  for (long id = 0; id < g->NN; ++id) {
    long n[3];
    node_of(g, id, n);
    int any = 0, all = 1;
    for (int o = 0; o < (1 << d); ++o) {
      long c[3] = {0, 0, 0};
      for (int ax = 0; ax < d; ++ax) c[ax] = n[ax] - 1 + ((o >> ax) & 1);
      int act = amr_cell_active(m, a, c);
      if (act < 0) continue;
      if (act) any = 1; else all = 0;
    }
    clo[id] = (uint8_t)any;
    m->cls[a][id] = any ? (all ? 1 : 2) : 0;
  }
  for (int layer = 1; layer <= 2; ++layer)
    for (long id = 0; id < g->NN; ++id) {
      if (m->cls[a][id] != 0) continue;
      long n[3];
      node_of(g, id, n);
      int near = 0;
      for (long dk = (d > 2 ? -layer : 0); dk <= (d > 2 ? layer : 0) && !near; ++dk)
        for (long dj = -layer; dj <= layer && !near; ++dj)
          for (long di = -layer; di <= layer && !near; ++di) {
            long q[3] = {n[0] + di, n[1] + dj, n[2] + dk};
            if (!node_inside(g, q)) continue;
            if (clo[node_id(g, q)]) near = 1;
          }
      if (near) m->cls[a][id] = (uint8_t)(2 + layer);
    }
  free(clo);
}

/* Quadratic interpolation weights along one axis for fine index n:
 * even n -> coarse n/2 (weight 1); odd n = 2I+1 -> nodes {I-1, I, I+1}
 * with (-1/8, 3/4, 3/8), or {I, I+1, I+2} with (3/8, 3/4, -1/8) when I = 0. */
static int quad_axis(long n, long ncn, long *idx, double *w) {
  (void)ncn;
  if (n % 2 == 0) { idx[0] = n / 2; w[0] = 1.0; return 1; }
  long I = (n - 1) / 2;
  if (I >= 1) { idx[0] = I - 1; idx[1] = I; idx[2] = I + 1; w[0] = -0.125; w[1] = 0.75; w[2] = 0.375; }
  else { idx[0] = I; idx[1] = I + 1; idx[2] = I + 2; w[0] = 0.375; w[1] = 0.75; w[2] = -0.125; }
  return 3;
}

/* Ghost nodes (classes 2-4) of level a from level a-1; displacement DOF keep
 * their values. */
static void amr_ghost_fill(const amr_t *m, int a, const double *xc, double *xf) {
  const grid_t *gf = &m->g[a], *gc = &m->g[a - 1];
  const int d = m->dim;
  for (long id = 0; id < gf->NN; ++id) {
    uint8_t c = m->cls[a][id];
    if (c < 2) continue;
    long n[3];
    node_of(gf, id, n);
    long ix[3][3];
    double w[3][3];
    int cnt[3] = {1, 1, 1};
    for (int ax = 0; ax < 3; ++ax) {
      if (ax < d) cnt[ax] = quad_axis(n[ax], gc->nn[ax], ix[ax], w[ax]);
      else { ix[ax][0] = 0; w[ax][0] = 1.0; }
    }
    for (int k = 0; k < d; ++k) {
      long q = (long)k * gf->NN + id;
      if (m->dm[a][q]) continue;
      double s = 0.0;
      for (int t2 = 0; t2 < cnt[2]; ++t2)
        for (int t1 = 0; t1 < cnt[1]; ++t1)
          for (int t0 = 0; t0 < cnt[0]; ++t0) {
            long I[3] = {ix[0][t0], ix[1][t1], ix[2][t2]};
            s += w[0][t0] * w[1][t1] * w[2][t2] * xc[(long)k * gc->NN + node_id(gc, I)];
          }
      xf[q] = s;
    }
  }
}

void orc_amr_ghost_fill(void *ctx, int level, const double *xc, double *xf) {
  amr_ghost_fill((amr_t *)ctx, level, xc, xf);
}

/* fine class at the node coinciding with coarse node cid of level a-1 */
static uint8_t amr_fine_class_at(const amr_t *m, int a, long cid) {
  long n[3];
  node_of(&m->g[a - 1], cid, n);
  long f[3] = {2 * n[0], 2 * n[1], m->dim > 2 ? 2 * n[2] : 0};
  return m->cls[a][node_id(&m->g[a], f)];
}

/* padded residual r = f - K x on the rows of level a that carry one
 * (a = 0: all nodes; a >= 1: classes 1-3), 0 elsewhere and on fixed DOF. */
static void amr_level_residual(const amr_t *m, int a, const double *x, const double *f, double *r) {
  const grid_t *g = &m->g[a];
  orc_residual(m->dim, g->nc, g->h, m->lam, m->mu, m->psi[a], m->dm[a], x, f, r);
  if (a == 0) return;
  for (long id = 0; id < g->NN; ++id) {
    uint8_t c = m->cls[a][id];
    if (c >= 1 && c <= 3) continue;
    for (int k = 0; k < m->dim; ++k) r[(long)k * g->NN + id] = 0.0;
  }
}

/* (R w_f)(I) = 2^-d sum P(n, I) w_f(n) at coarse node cid of level a-1 */
static void amr_restrict_at(const amr_t *m, int a, long cid, const double *wf, double *out) {
  const grid_t *gc = &m->g[a - 1], *gf = &m->g[a];
  const int d = m->dim;
  long I[3];
  node_of(gc, cid, I);
  for (int k = 0; k < d; ++k) out[k] = 0.0;
  for (long dk = (d > 2 ? -1 : 0); dk <= (d > 2 ? 1 : 0); ++dk)
    for (long dj = -1; dj <= 1; ++dj)
      for (long di = -1; di <= 1; ++di) {
        long n[3] = {2 * I[0] + di, 2 * I[1] + dj, d > 2 ? 2 * I[2] + dk : 0};
        if (!node_inside(gf, n)) continue;
        double w = 1.0;
        for (int ax = 0; ax < d; ++ax) w *= p_weight_axis(n[ax], I[ax]);
        long fid = node_id(gf, n);
        for (int k = 0; k < d; ++k) out[k] += w * wf[(long)k * gf->NN + fid];
      }
  for (int k = 0; k < d; ++k) out[k] /= (double)(1 << d);
}

/* Composite residual of (x, f): padded level residuals, coarse nodes on or
 * inside the next finer region replaced by R of its padded residual.
 * Ghosts of x are filled first.  Returns ||r|| over composite unknowns. */
static double amr_comp_residual(const amr_t *m, double **x, double *const *f, double **r) {
  const int d = m->dim;
  for (int a = 1; a <= m->A; ++a) amr_ghost_fill(m, a, x[a - 1], x[a]);
  for (int a = m->A; a >= 0; --a) {
    amr_level_residual(m, a, x[a], f[a], r[a]);
    if (a == m->A) continue;
    const grid_t *g = &m->g[a];
    for (long id = 0; id < g->NN; ++id) {
      uint8_t fc = amr_fine_class_at(m, a + 1, id);
      if (fc != 1 && fc != 2) continue;
      double rr[3];
      amr_restrict_at(m, a + 1, id, r[a + 1], rr);
      for (int k = 0; k < d; ++k) {
        long q = (long)k * g->NN + id;
        r[a][q] = m->dm[a][q] ? 0.0 : rr[k];
      }
    }
  }
  double s = 0.0;
  for (int a = 0; a <= m->A; ++a) {
    const grid_t *g = &m->g[a];
    for (long id = 0; id < g->NN; ++id) {
      if (a >= 1 && m->cls[a][id] != 1) continue;
      if (a < m->A && amr_fine_class_at(m, a + 1, id) == 1) continue; /* covered */
      for (int k = 0; k < d; ++k) {
        long q = (long)k * g->NN + id;
        if (!m->dm[a][q]) s += r[a][q] * r[a][q];
      }
    }
  }
  return sqrt(s);
}

/* coarse nodes strictly inside level a's region take the injected fine values */
static void amr_inject(const amr_t *m, int a, const double *xf, double *xc) {
  const grid_t *gc = &m->g[a - 1], *gf = &m->g[a];
  for (long id = 0; id < gc->NN; ++id) {
    if (amr_fine_class_at(m, a, id) != 1) continue;
    long n[3];
    node_of(gc, id, n);
    long fn[3] = {2 * n[0], 2 * n[1], m->dim > 2 ? 2 * n[2] : 0};
    long fid = node_id(gf, fn);
    for (int k = 0; k < m->dim; ++k) xc[(long)k * gc->NN + id] = xf[(long)k * gf->NN + fid];
  }
}

/* Colour-synchronous Gauss-Seidel half-sweep on the unknowns of level a >= 1
 * (class 1, free DOF); every other node keeps its value. */
static void amr_smooth(const amr_t *m, int a, double *x, const double *f, int sweeps, int reverse,
                       double *tmp) {
  const grid_t *g = &m->g[a];
  long n3 = (long)m->dim * g->NN;
  for (int s = 0; s < sweeps; ++s)
    for (int h = 0; h < 2; ++h) {
      int colour = reverse ? 1 - h : h;
      if (m->o.smoother == 1) { if (h == 1) break; }
      if (m->o.smoother == 1)
        orc_jacobi(m->dim, g->nc, g->h, m->lam, m->mu, m->psi[a], m->dm[a], m->o.omega, x, f, tmp);
      else
        orc_rb_half(m->dim, g->nc, g->h, m->lam, m->mu, m->psi[a], m->dm[a], m->o.omega, colour, x,
                    f, tmp);
      for (long q = 0; q < n3; ++q) {
        long id = q % g->NN;
        if (m->cls[a][id] == 1) x[q] = tmp[q];
      }
    }
}

/* FAS multilevel cycle over levels a..1 (x, f per level; f may be modified
 * at covered/interface nodes of coarser levels), ending in the base
 * V-cycle. */
static void amr_fas(amr_t *m, int a, double **x, double **f, double **w, double **xinj,
                    double **tmp) {
  const int d = m->dim;
  if (a == 0) {
    vcycle(d, m->hier, m->nlev, 0, m->lam, m->mu, &m->o, x[0], f[0]);
    return;
  }
  const grid_t *gc = &m->g[a - 1], *gf = &m->g[a];
  amr_ghost_fill(m, a, x[a - 1], x[a]);
  amr_smooth(m, a, x[a], f[a], m->o.nu_pre, 0, tmp[a]);
  amr_ghost_fill(m, a, x[a - 1], x[a]);
  amr_level_residual(m, a, x[a], f[a], w[a]);
  amr_inject(m, a, x[a], x[a - 1]);
  memcpy(xinj[a - 1], x[a - 1], sizeof(double) * d * gc->NN);
  /* FAS load on covered and interface coarse nodes: R w + K_c x_c */
  double *Kx = tmp[a - 1];
  orc_apply(d, gc->nc, gc->h, m->lam, m->mu, m->psi[a - 1], x[a - 1], Kx);
  for (long id = 0; id < gc->NN; ++id) {
    uint8_t fc = amr_fine_class_at(m, a, id);
    if (fc != 1 && fc != 2) continue;
    double rr[3];
    amr_restrict_at(m, a, id, w[a], rr);
    for (int k = 0; k < d; ++k) {
      long q = (long)k * gc->NN + id;
      if (!m->dm[a - 1][q]) f[a - 1][q] = rr[k] + Kx[q];
    }
  }
  amr_fas(m, a - 1, x, f, w, xinj, tmp);
  /* x_f += P (x_c - inject(x_f)) on the unknowns of level a */
  double *dc = tmp[a - 1];
  for (long q = 0; q < (long)d * gc->NN; ++q) dc[q] = x[a - 1][q] - xinj[a - 1][q];
  double *pf = w[a];
  memset(pf, 0, sizeof(double) * d * gf->NN);
  orc_prolong_add(d, gc->nc, dc, m->dm[a], pf);
  for (long q = 0; q < (long)d * gf->NN; ++q)
    if (m->cls[a][q % gf->NN] == 1) x[a][q] += pf[q];
  amr_ghost_fill(m, a, x[a - 1], x[a]);
  amr_smooth(m, a, x[a], f[a], m->o.nu_post, 0, tmp[a]);
}

/* psi_raw[a]: raw indicator sampled at level a's cell centres (dense). */
void *orc_amr_new(int dim, int A, int bc, const long *nc0, const double *h0, double lam, double mu,
                  const double *const *psi_raw, double psi_floor, const int *kind, const double *val,
                  double thresh, int smoother, double omega, int nu_pre, int nu_post,
                  double bottom_rtol, int bottom_max_iter, const uint8_t *const *blk_in,
                  double cluster_eff) {
  amr_t *m = (amr_t *)calloc(1, sizeof(amr_t));
  m->dim = dim; m->A = A; m->bc = bc; m->lam = lam; m->mu = mu;
  memcpy(m->kind, kind, sizeof(int) * 18);
  memcpy(m->val, val, sizeof(double) * 18);
  orc_opts o = {smoother, omega, nu_pre, nu_post, 0.0, 0, bottom_rtol, bottom_max_iter, 0};
  m->o = o;
  for (int a = 0; a <= A; ++a) {
    long nc[3];
    double h[3];
    for (int ax = 0; ax < 3; ++ax) {
      nc[ax] = ax < dim ? nc0[ax] << a : 0;
      h[ax] = ax < dim ? h0[ax] / (double)(1 << a) : 1.0;
    }
    grid_init(&m->g[a], dim, nc, h, lam, mu);
    m->psi[a] = (double *)malloc(sizeof(double) * m->g[a].NC);
    orc_floor(m->g[a].NC, psi_raw[a], psi_floor, m->psi[a]);
    m->dm[a] = (uint8_t *)malloc((size_t)dim * m->g[a].NN);
    m->uD[a] = (double *)malloc(sizeof(double) * dim * m->g[a].NN);
    orc_dirichlet_mask(dim, nc, kind, val, m->dm[a], m->uD[a]);
    if (a >= 1) {
      for (int ax = 0; ax < 3; ++ax) m->nb[a][ax] = ax < dim ? m->g[a].nc[ax] / bc : 1;
      m->blk[a] = (uint8_t *)calloc(m->nb[a][0] * m->nb[a][1] * m->nb[a][2], 1);
      m->cls[a] = (uint8_t *)calloc(m->g[a].NN, 1);
    }
  }
  if (blk_in) { /* block flags given (levels 1..A) */
    for (int a = 1; a <= A; ++a)
      memcpy(m->blk[a], blk_in[a - 1], m->nb[a][0] * m->nb[a][1] * m->nb[a][2]);
  } else {
    uint8_t *tags[AMR_MAXL] = {0};
    for (int a = 0; a < A; ++a) {
      tags[a] = (uint8_t *)malloc(m->g[a].NC);
      orc_amr_tags(dim, m->g[a].nc, m->g[a].h, m->psi[a], thresh, tags[a]);
    }
    amr_blocks(m, tags, cluster_eff);
    for (int a = 0; a < A; ++a) free(tags[a]);
  }
  for (int a = 1; a <= A; ++a) amr_classify(m, a);
  /* psi of covered coarse cells: mean of the children, finest first */
  for (int a = A; a >= 1; --a) {
    grid_t *gc = &m->g[a - 1];
    for (long c = 0; c < gc->NC; ++c) {
      long ci[3] = {c % gc->nc[0], (c / gc->nc[0]) % gc->nc[1], c / (gc->nc[0] * gc->nc[1])};
      long fc[3] = {2 * ci[0], 2 * ci[1], dim > 2 ? 2 * ci[2] : 0};
      if (amr_cell_active(m, a, fc) != 1) continue;
      double s = 0.0;
      for (int o2 = 0; o2 < (1 << dim); ++o2) {
        long q[3] = {fc[0] + (o2 & 1), fc[1] + ((o2 >> 1) & 1), dim > 2 ? fc[2] + ((o2 >> 2) & 1) : 0};
        s += m->psi[a][q[0] + m->g[a].nc[0] * (q[1] + m->g[a].nc[1] * q[2])];
      }
      m->psi[a - 1][c] = s / (double)(1 << dim);
    }
  }
  for (int a = 0; a <= A; ++a) {
    m->fP[a] = (double *)malloc(sizeof(double) * dim * m->g[a].NN);
    orc_rhs(dim, m->g[a].nc, m->g[a].h, lam, mu, m->psi[a], kind, val, NULL, m->fP[a], NULL, NULL);
  }
  /* uniform hierarchy of the base level */
  m->nlev = count_levels(dim, nc0);
  m->hier = (level_t *)calloc(m->nlev, sizeof(level_t));
  for (int l = 0; l < m->nlev; ++l) {
    level_t *L = &m->hier[l];
    for (int ax = 0; ax < 3; ++ax) {
      L->nc[ax] = (ax < dim) ? (l == 0 ? nc0[ax] : m->hier[l - 1].nc[ax] / 2) : 0;
      L->h[ax] = (ax < dim) ? (l == 0 ? h0[ax] : 2.0 * m->hier[l - 1].h[ax]) : 1.0;
    }
    long NC = 1, NN = 1;
    for (int ax = 0; ax < dim; ++ax) { NC *= L->nc[ax]; NN *= L->nc[ax] + 1; }
    L->n3 = (long)dim * NN;
    L->psi = (double *)malloc(sizeof(double) * NC);
    L->mask = (uint8_t *)malloc(L->n3);
    L->e = (double *)calloc(L->n3, sizeof(double));
    L->f = (double *)calloc(L->n3, sizeof(double));
    L->r = (double *)calloc(L->n3, sizeof(double));
    L->tmp = (double *)calloc(L->n3, sizeof(double));
    if (l == 0) memcpy(L->psi, m->psi[0], sizeof(double) * NC);
    else orc_coarsen_psi(dim, m->hier[l - 1].nc, m->hier[l - 1].psi, L->psi);
    orc_dirichlet_mask(dim, L->nc, kind, val, L->mask, NULL);
  }
  /* ||lifted load||: composite residual of the prescribed values */
  double *x[AMR_MAXL], *r[AMR_MAXL];
  for (int a = 0; a <= A; ++a) {
    x[a] = m->uD[a];
    r[a] = (double *)malloc(sizeof(double) * dim * m->g[a].NN);
  }
  double *xs[AMR_MAXL];
  for (int a = 0; a <= A; ++a) {
    xs[a] = (double *)malloc(sizeof(double) * dim * m->g[a].NN);
    memcpy(xs[a], x[a], sizeof(double) * dim * m->g[a].NN);
  }
  m->fnorm = amr_comp_residual(m, xs, m->fP, r);
  for (int a = 0; a <= A; ++a) { free(r[a]); free(xs[a]); }
  return m;
}

void orc_amr_free(void *ctx) {
  amr_t *m = (amr_t *)ctx;
  if (!m) return;
  for (int a = 0; a <= m->A; ++a) {
    free(m->blk[a]); free(m->cls[a]); free(m->psi[a]); free(m->dm[a]); free(m->uD[a]); free(m->fP[a]);
  }
  for (int l = 0; l < m->nlev; ++l) {
    free(m->hier[l].psi); free(m->hier[l].mask); free(m->hier[l].e);
    free(m->hier[l].f); free(m->hier[l].r); free(m->hier[l].tmp);
  }
  free(m->hier);
  free(m);
}

/* Level info: block flags (a >= 1), node classes (a >= 1), psi (all). */
void orc_amr_info(void *ctx, int a, uint8_t *blk, uint8_t *cls, double *psi, long *nb) {
  amr_t *m = (amr_t *)ctx;
  if (nb) for (int ax = 0; ax < 3; ++ax) nb[ax] = a >= 1 ? m->nb[a][ax] : 0;
  if (blk && a >= 1) memcpy(blk, m->blk[a], m->nb[a][0] * m->nb[a][1] * m->nb[a][2]);
  if (cls && a >= 1) memcpy(cls, m->cls[a], m->g[a].NN);
  if (psi) memcpy(psi, m->psi[a], sizeof(double) * m->g[a].NC);
}

double orc_amr_fnorm(void *ctx) { return ((amr_t *)ctx)->fnorm; }

/* Composite residual of the levels' x (ghosts of x are refilled) for the
 * problem's loads, or for the loads f when f is not NULL. */
double orc_amr_residual(void *ctx, double **x, double **f, double **r) {
  amr_t *m = (amr_t *)ctx;
  return amr_comp_residual(m, x, f ? f : m->fP, r);
}

/* Composite solve: u[a] in = guess (displacement DOF overwritten), out =
 * solution with covered nodes injected and ghosts filled. */
int orc_amr_solve(void *ctx, double rtol, int max_cycles, double **u, double *hist, int hist_cap,
                  int *n_cycles) {
  amr_t *m = (amr_t *)ctx;
  const int d = m->dim, A = m->A;
  double *r[AMR_MAXL], *e[AMR_MAXL], *w[AMR_MAXL], *xinj[AMR_MAXL], *tmp[AMR_MAXL];
  for (int a = 0; a <= A; ++a) {
    long n3 = (long)d * m->g[a].NN;
    for (long q = 0; q < n3; ++q)
      if (m->dm[a][q]) u[a][q] = m->uD[a][q];
    r[a] = (double *)malloc(sizeof(double) * n3);
    e[a] = (double *)malloc(sizeof(double) * n3);
    w[a] = (double *)malloc(sizeof(double) * n3);
    xinj[a] = (double *)malloc(sizeof(double) * n3);
    tmp[a] = (double *)malloc(sizeof(double) * n3);
  }
  for (int a = A; a >= 1; --a) amr_inject(m, a, u[a], u[a - 1]);
  int status = 1, cyc;
  for (cyc = 0;; ++cyc) {
    double rn = amr_comp_residual(m, u, m->fP, r);
    double rho = m->fnorm > 0.0 ? rn / m->fnorm : 0.0;
    if (cyc < hist_cap) hist[cyc] = rho;
    if (rho <= rtol) { status = 0; break; }
    if (cyc >= max_cycles) break;
    /* correction cycle: loads = composite residual, x = 0 */
    for (int a = 0; a <= A; ++a) memset(e[a], 0, sizeof(double) * d * m->g[a].NN);
    amr_fas(m, A, e, r, w, xinj, tmp);
    for (int a = 0; a <= A; ++a) {
      long n3 = (long)d * m->g[a].NN;
      for (long q = 0; q < n3; ++q) {
        if (m->dm[a][q]) continue;
        if (a >= 1 && m->cls[a][q % m->g[a].NN] != 1) continue;
        u[a][q] += e[a][q];
      }
    }
    for (int a = A; a >= 1; --a) amr_inject(m, a, u[a], u[a - 1]);
  }
  for (int a = 1; a <= A; ++a) amr_ghost_fill(m, a, u[a - 1], u[a]);
  *n_cycles = cyc;
  for (int a = 0; a <= A; ++a) { free(r[a]); free(e[a]); free(w[a]); free(xinj[a]); free(tmp[a]); }
  return status;
}
