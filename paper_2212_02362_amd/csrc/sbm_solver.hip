// sbm_solver.hip -- host orchestration (hierarchy, V-cycle, mixed-precision
// refinement, adjoint solve) and the C ABI declared in include/sbm.h.
//
// Multigrid follows Sec. 2.2-2.3 of Agrawal & Runnels: smoothing with Jacobi or
// Gauss-Seidel, levels coarsened by 2 while every cell count is even and >= 4
// (power-of-two grids, Sec. 3.3), coarse operators re-discretised on averaged
// psi, V(nu_pre, nu_post) cycles until the relative residual meets rtol.  The
// mixed mode runs the whole V-cycle in FP32 on a residual scaled to unit norm
// and keeps the fine residual, the correction and the bottom refinement in
// FP64.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <initializer_list>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sbm.h"
#include "sbm_internal.h"

using namespace sbm;

static thread_local std::string g_last_error;

static sbm_status fail(sbm_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

sbm_status sbm::set_error(sbm_status s, const std::string &msg) { return fail(s, msg); }

// True when two of the non-NULL pointers are equal (an output passed as an
// input or as another output of the same call).
static bool aliased(std::initializer_list<const void *> p) {
  for (auto a = p.begin(); a != p.end(); ++a)
    for (auto b = a + 1; b != p.end(); ++b)
      if (*a && *a == *b) return true;
  return false;
}
#define NO_ALIAS(...)                                                                   \
  do {                                                                                  \
    if (aliased({__VA_ARGS__}))                                                         \
      return fail(SBM_E_ARG, "an output buffer aliases an input or another output");    \
  } while (0)

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(SBM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));            \
  } while (0)

struct sbm_ctx {
  int dim = 0;
  int nlev = 0;
  std::vector<Level> L;
  sbm_options opt;
  hipStream_t st = nullptr;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  double *partials = nullptr;
  int npart = 0;
  double *scal = nullptr;  // device scalars
  int *iflag = nullptr;    // device int flags / counters
  // bottom scratch
  double *b_r = nullptr, *b_p = nullptr, *b_Ap = nullptr, *b_x64 = nullptr, *b_r64 = nullptr;
  double *host = nullptr;  // pinned host scalars
  bool have_problem = false;
  sbm_material mat{};
  sbm_bc bc{};
  Traction tr{};
  DispValues dv{};
  DispValues zero_dv{};
  double fnorm = 0.0;
  int last_bottom_iters = 0;
  double *x0 = nullptr;  // finest-level iterate (fixed address for captured cycles)
  double *kr = nullptr, *kz = nullptr, *kp = nullptr, *kq = nullptr;  // flexible CG vectors
  // set while a CG preconditioner cycle is built: its last finest half-sweep
  // also writes the partials of r . z there (mixed: from the FP64 residual
  // rz_r64, its FP32 cast scaled by sqrt(*rz_ss))
  double *rz_partials = nullptr;
  const double *rz_r64 = nullptr, *rz_ss = nullptr;
  double *partials2 = nullptr;
  // live kernel timing (sbm_profile)
  bool prof_on = false;
  std::vector<hipEvent_t> prof_ev;  // pairs
  std::vector<int> prof_cls;        // class of each pair in use
  double prof_ms[SBM_PROF_N] = {0};
  int64_t prof_n[SBM_PROF_N] = {0};
  // captured V-cycles
  struct CycleGraph {
    int mode;  // 0: outer-loop cycle on x0, 1: preconditioner z = M r, 2: as 0 with work
               // done by the convergence test (FP64: the first finest half-sweep;
               // mixed: the finest residual), 3: mixed, also the FP32 cycle's first
               // half-sweep made by the cast
    int precision;
    const double *f;
    bool prof;
    bool failed = false;
    hipGraphExec_t exec = nullptr;
    std::vector<hipEvent_t> ev;  // timing pairs recorded inside the graph
    std::vector<int> cls;
  };
  std::vector<CycleGraph *> graphs;
  CycleGraph *capturing = nullptr;  // graph under capture
  CycleGraph *pending = nullptr;    // graph launched since the last harvest
  hipStream_t cap_st = nullptr;
  int64_t graph_captures = 0, graph_launches = 0;
  std::string graph_error;
  double g_lam = NAN, g_mu = NAN;
  uint32_t g_dmask = 0;
  // first level of the one-workgroup tail of the FP64 / FP32 cycle (-1: none),
  // its level tables (device) and LDS bytes
  int tail64 = -1, tail32 = -1;
  char *tail_args = nullptr;
  double *tail_A = nullptr;  // dense bottom matrix of the tails
  size_t tail_lds64 = 0, tail_lds32 = 0;
  size_t tail_lds_max = 64 * 1024;  // LDS bytes a workgroup may hold on this device
  // set while a cycle runs whose first finest-level half-sweep was already
  // done by the convergence test (its result is in the level's tmp vector)
  bool first_half_done = false;
  // set while a cycle runs whose finest-level correction starts from zero on a
  // level swept by the fused two-colour kernel (nothing is filled or read: the
  // first sweep relaxes from a zero iterate)
  bool zero_start = false;
};

// Brackets one launch sequence with an event pair when profiling is on.
struct ProfScope {
  sbm_ctx *c;
  int cls;
  bool on;
  size_t pair;
  std::vector<hipEvent_t> *ev;
  ProfScope(sbm_ctx *c_, int cls_, bool active) : c(c_), cls(cls_), on(c_->prof_on && active) {
    if (!on) return;
    // inside a capture the pair belongs to the graph and is recorded by every replay
    ev = c->capturing ? &c->capturing->ev : &c->prof_ev;
    std::vector<int> &cl = c->capturing ? c->capturing->cls : c->prof_cls;
    pair = cl.size();
    while (ev->size() < 2 * (pair + 1)) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) {
        on = false;
        return;
      }
      ev->push_back(e);
    }
    cl.push_back(cls);
    (void)hipEventRecord((*ev)[2 * pair], c->st);
  }
  ~ProfScope() {
    if (on) (void)hipEventRecord((*ev)[2 * pair + 1], c->st);
  }
};

// Collects the elapsed times of completed event pairs (stream is idle): the
// pairs recorded eagerly and those of the last replayed graph.
static void prof_harvest(sbm_ctx *c) {
  auto take = [c](const std::vector<hipEvent_t> &ev, const std::vector<int> &cls) {
    for (size_t p = 0; p < cls.size(); ++p) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, ev[2 * p], ev[2 * p + 1]) == hipSuccess) {
        c->prof_ms[cls[p]] += ms;
        c->prof_n[cls[p]] += 1;
      }
    }
  };
  take(c->prof_ev, c->prof_cls);
  c->prof_cls.clear();
  if (c->pending) take(c->pending->ev, c->pending->cls);
  c->pending = nullptr;
}

static void drop_graphs(sbm_ctx *c) {
  for (auto *g : c->graphs) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    for (hipEvent_t e : g->ev) (void)hipEventDestroy(e);
    delete g;
  }
  c->graphs.clear();
  c->pending = nullptr;
}

// ------------------------------------------------------------ grid helpers

static bool grid_ok(const sbm_grid *g) {
  if (!g || (g->dim != 2 && g->dim != 3)) return false;
  for (int a = 0; a < g->dim; ++a) {
    if (g->ncell[a] < 1 || g->ncell[a] > (1 << 20)) return false;
    if (!(g->h[a] > 0.0) || !isfinite(g->h[a])) return false;
  }
  int64_t nodes = 1;
  for (int a = 0; a < g->dim; ++a) nodes *= g->ncell[a] + 1;
  return nodes * g->dim < ((int64_t)1 << 31);  // 32-bit indexing of every vector
}

static int count_levels(const sbm_grid *g) {
  int64_t c[3] = {g->ncell[0], g->ncell[1], g->dim > 2 ? g->ncell[2] : 4};
  int n = 1;
  for (;;) {
    bool ok = true;
    for (int a = 0; a < g->dim; ++a)
      if (c[a] % 2 != 0 || c[a] < 4) ok = false;
    if (!ok) break;
    for (int a = 0; a < g->dim; ++a) c[a] /= 2;
    ++n;
  }
  return n;
}

void sbm::make_level(int dim, const int64_t *ncell, const double *h, Level &lv) {
  Geom &G = lv.g;
  G.dim = dim;
  int64_t c[3];
  for (int a = 0; a < 3; ++a) {
    if (a < dim) {
      c[a] = ncell[a];
      lv.h[a] = h[a];
    } else {
      c[a] = 1;
      lv.h[a] = 1.0;
    }
  }
  G.cx = (int)c[0];
  G.cy = (int)c[1];
  G.cz = (int)c[2];
  G.nx = G.cx + 1;
  G.ny = G.cy + 1;
  G.nz = dim > 2 ? G.cz + 1 : 1;
  G.nn = (int64_t)G.nx * G.ny * G.nz;
  G.nc = (int64_t)G.cx * G.cy * G.cz;
  G.dmask = 0;
  G.fnx = make_fastdiv((uint32_t)G.nx);
  G.fny = make_fastdiv((uint32_t)G.ny);
  G.fcx = make_fastdiv((uint32_t)G.cx);
  G.fcy = make_fastdiv((uint32_t)G.cy);
  G.fpx = make_fastdiv((uint32_t)((G.nx + 1) / 2));
}

static void level_shapes(const sbm_grid *g, int nlev, std::vector<Level> &L) {
  L.assign(nlev, Level());
  for (int l = 0; l < nlev; ++l) {
    int64_t c[3] = {1, 1, 1};
    double h[3] = {1.0, 1.0, 1.0};
    for (int a = 0; a < g->dim; ++a) {
      c[a] = g->ncell[a] >> l;
      h[a] = g->h[a] * (double)(1 << l);
    }
    make_level(g->dim, c, h, L[l]);
  }
}

// Workspace carving: the same walk sizes the workspace (base == nullptr) and
// assigns the pointers.
struct Carver {
  char *base;
  size_t off = 0;
  template <typename T>
  T *take(int64_t n) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? (T *)(base + off) : nullptr;
    off += (size_t)n * sizeof(T);
    return p;
  }
};

static size_t carve(sbm_ctx *c, char *base) {
  Carver cv{base};
  const int d = c->dim;
  int64_t maxblocks = 1;
  for (int l = 0; l < c->nlev; ++l) {
    Level &L = c->L[l];
    const int64_t nv = (int64_t)d * L.g.nn;
    L.psi64 = cv.take<double>(L.g.nc);
    L.psi32 = cv.take<float>(L.g.nc);
    L.e = cv.take<double>(nv);
    L.f = cv.take<double>(nv);
    L.t = cv.take<double>(nv);
    L.e32 = cv.take<float>(nv);
    L.f32 = cv.take<float>(nv);
    L.t32 = cv.take<float>(nv);
    maxblocks = std::max<int64_t>(maxblocks, grid_blocks(L.g.nn));
    maxblocks = std::max<int64_t>(maxblocks, num_blocks(L.g.nc));
  }
  c->x0 = cv.take<double>((int64_t)d * c->L[0].g.nn);
  c->kr = cv.take<double>((int64_t)d * c->L[0].g.nn);
  c->kz = cv.take<double>((int64_t)d * c->L[0].g.nn);
  c->kp = cv.take<double>((int64_t)d * c->L[0].g.nn);
  c->kq = cv.take<double>((int64_t)d * c->L[0].g.nn);
  c->npart = (int)maxblocks;
  c->partials = cv.take<double>(maxblocks);
  c->partials2 = cv.take<double>(maxblocks);
  c->scal = cv.take<double>(16);
  c->iflag = cv.take<int>(16);
  const Level &B = c->L[c->nlev - 1];
  const int64_t nb = (int64_t)d * B.g.nn;
  c->b_r = cv.take<double>(nb);
  c->b_p = cv.take<double>(nb);
  c->b_Ap = cv.take<double>(nb);
  c->b_x64 = cv.take<double>(nb);
  c->b_r64 = cv.take<double>(nb);
  c->tail_args = cv.take<char>(2 * (int64_t)kTailArgBytes);
  c->tail_A = cv.take<double>((int64_t)(kTailDenseBytes / sizeof(double)));
  return cv.off + 256;
}

void sbm::set_coefs(Level &L, double lam, double mu, int dim) {
  const double dfac = 1.0 / (double)(1 << (dim - 1));
  const double pfac = dim == 3 ? 0.5 : 1.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double v = 0.0;
      if (i < dim && j < dim) v = (mu + (lam + mu) * (i == j ? 1.0 : 0.0)) / (L.h[j] * L.h[j]) * dfac;
      L.c64.cd[i][j] = v;
      L.c32.cd[i][j] = (float)v;
    }
  const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
  for (int p = 0; p < 3; ++p) {
    double cp = 0.0, cm = 0.0;
    if (pb[p] < dim) {
      const double ih = 1.0 / (4.0 * L.h[pa[p]] * L.h[pb[p]]);
      cp = (lam + mu) * ih * pfac;
      cm = (lam - mu) * ih * pfac;
    }
    L.c64.cp[p] = cp;
    L.c64.cm[p] = cm;
    L.c32.cp[p] = (float)cp;
    L.c32.cm[p] = (float)cm;
  }
}

static double opt_omega(const sbm_options &o) {
  if (o.omega > 0.0) return o.omega;
  return o.smoother == 1 ? 0.8 : 1.0;
}

static int bottom_maxit(const sbm_ctx *c) {
  if (c->opt.bottom_max_iter > 0) return c->opt.bottom_max_iter;
  const Level &B = c->L[c->nlev - 1];
  return (int)std::min<int64_t>(4 * (int64_t)c->dim * B.g.nn, 1 << 30);
}

// ---------------------------------------------------------------- V-cycle

template <typename T>
struct Prec;
template <>
struct Prec<double> {
  static const double *psi(const Level &L) { return L.psi64; }
  static const Coef<double> &coef(const Level &L) { return L.c64; }
  static double *e(Level &L) { return L.e; }
  static double *f(Level &L) { return L.f; }
  static double *t(Level &L) { return L.t; }
};
template <>
struct Prec<float> {
  static const float *psi(const Level &L) { return L.psi32; }
  static const Coef<float> &coef(const Level &L) { return L.c32; }
  static float *e(Level &L) { return L.e32; }
  static float *f(Level &L) { return L.f32; }
  static float *t(Level &L) { return L.t32; }
};

// A colour half-sweep of level L (LDS-tiled on wide 3D levels).
template <typename T>
static hipError_t half_sweep(const Level &L, const T *psi, const Coef<T> &C, const T *src,
                             const T *f, T *dst, double om, int colour, hipStream_t st) {
  return tiled_sweep_ok(L) ? launch_rb_tiled<T>(L, psi, C, src, f, dst, om, colour, st)
                     : launch_rb_half<T>(L, psi, C, src, f, dst, om, colour, st);
}

// nu sweeps on level l for x with load f; tmp is the ping-pong buffer.
template <typename T>
static hipError_t smooth(sbm_ctx *c, int l, T *x, const T *f, T *tmp, int nu, bool reverse,
                         bool pre) {
  Level &L = c->L[l];
  const T *psi = Prec<T>::psi(L);
  const Coef<T> &C = Prec<T>::coef(L);
  const double om = opt_omega(c->opt);
  hipError_t e = hipSuccess;
  if (c->opt.smoother == 1) {
    T *src = x, *dst = tmp;
    for (int s = 0; s < nu; ++s) {
      ProfScope ps(c, SBM_PROF_SMOOTH, l == 0);
      if ((e = launch_jacobi<T>(L, psi, C, src, f, dst, om, c->st)) != hipSuccess) return e;
      std::swap(src, dst);
    }
    if (src != x) e = launch_copy<T>(src, x, (int64_t)c->dim * L.g.nn, c->st);
    return e;
  }
  const int c0 = reverse ? 1 : 0;
  // the finest level starts from zero when the caller says so (zero_start);
  // a coarser level always does on its pre-smoothing (its correction is the
  // zero the restriction wrote)
  const bool zero = ((l == 0 && c->zero_start) || (l > 0 && pre)) && zero_sweep_ok(L);
  if (l == 0) c->zero_start = false;
  if (zero || (tiled_ok(L) && c->opt.fused_sweep == 1)) {
    // A sweep from a zero iterate (the first sweep of a correction that starts
    // from zero) is one launch that reads no iterate; with fused_sweep every
    // other sweep of a tiled level is one fused launch too (out of place:
    // cur -> the other buffer), else two half-sweeps (cur -> tmp -> cur).
    // The first sweep's output buffer is chosen so that the last sweep lands
    // in x.
    const bool all = c->opt.fused_sweep == 1 && tiled_ok(L);
    T *cur = zero ? nullptr : x;
    for (int s = 0; s < nu; ++s) {
      if (!cur) {
        const int toggles = all ? nu - 1 - s : 0;
        T *dst = toggles % 2 == 0 ? x : tmp;
        ProfScope ps(c, SBM_PROF_SWEEP0, l == 0);
        if ((e = launch_rb_fused<T>(L, psi, C, nullptr, f, dst, om, c0, c->st)) != hipSuccess)
          return e;
        cur = dst;
      } else if (all) {
        T *dst = cur == x ? tmp : x;
        ProfScope ps(c, SBM_PROF_SMOOTH, l == 0);
        if ((e = launch_rb_fused<T>(L, psi, C, cur, f, dst, om, c0, c->st)) != hipSuccess)
          return e;
        cur = dst;
      } else {
        T *oth = cur == x ? tmp : x;
        {
          ProfScope ps(c, SBM_PROF_SMOOTH, l == 0);
          if ((e = half_sweep<T>(L, psi, C, cur, f, oth, om, c0, c->st)) != hipSuccess) return e;
        }
        ProfScope ps(c, SBM_PROF_SMOOTH, l == 0);
        if ((e = half_sweep<T>(L, psi, C, oth, f, cur, om, 1 - c0, c->st)) != hipSuccess) return e;
      }
    }
    if (!cur) return launch_fill<T>(x, (int64_t)c->dim * L.g.nn, T(0), c->st);
    if (cur != x) return launch_copy<T>(cur, x, (int64_t)c->dim * L.g.nn, c->st);
    return hipSuccess;
  }
  // the first half-sweep of the outer cycle's pre-smoothing may already be in
  // tmp (computed with the convergence test of the previous cycle)
  const bool first_done = l == 0 && c->first_half_done;
  c->first_half_done = false;
  const bool tiled = tiled_sweep_ok(L);
  auto half = [&](const T *src, T *dst, int colour) {
    return tiled ? launch_rb_tiled<T>(L, psi, C, src, f, dst, om, colour, c->st)
                 : launch_rb_half<T>(L, psi, C, src, f, dst, om, colour, c->st);
  };
  for (int s = 0; s < nu; ++s) {
    if (s > 0 || !first_done) {
      ProfScope ps(c, SBM_PROF_SMOOTH, l == 0);
      if ((e = half(x, tmp, c0)) != hipSuccess) return e;
    }
    // the last half-sweep of a CG preconditioner's cycle writes z (= x) and
    // forms the partials of r . z (r = f) on the way
    double *dot = (l == 0 && !pre && s == nu - 1 && tiled) ? c->rz_partials : nullptr;
    ProfScope ps(c, dot ? SBM_PROF_SMOOTH_DOT : SBM_PROF_SMOOTH, l == 0);
    if (dot) {
      if ((e = launch_rb_tiled<T>(L, psi, C, tmp, f, x, om, 1 - c0, c->st, nullptr, nullptr, dot,
                                  c->rz_r64, c->rz_ss)) != hipSuccess)
        return e;
      continue;
    }
    if ((e = half(tmp, x, 1 - c0)) != hipSuccess) return e;
  }
  return e;
}

// Whether the mixed CG update casts the new residual for the preconditioner
// itself (a tiled finest level whose cycle starts with the sweep from zero):
// the cycle then runs as mode 4.
static bool cast_fused(const sbm_ctx *c) {
  return c->opt.precision == 1 && c->opt.smoother == 0 && c->opt.nu_pre >= 1 && c->nlev > 1 &&
         c->tail32 != 0 && tiled_ok(c->L[0]);
}

// Whether the CG preconditioner's last finest half-sweep forms r . z
// (Gauss-Seidel post-smoothing of a tiled finest level outside the tail; in
// the mixed cycle the FP32 half-sweep reads the FP64 residual for it).
static bool rz_fused(const sbm_ctx *c) {
  const Level &L0 = c->L[0];
  const bool fp32 = c->opt.precision == 1;
  return c->opt.smoother == 0 && c->opt.nu_post >= 1 && c->nlev > 1 &&
         (fp32 ? c->tail32 : c->tail64) != 0 && c->opt.fused_sweep != 1 && tiled_ok(L0) &&
         rb_tiled_partials(L0, fp32) <= c->npart;
}

// Arms (ss: the mixed cast's squared scale; fp64: the FP64 cycle) or
// disarms the r . z partials of the next preconditioner cycle.
static void rz_set(sbm_ctx *c, const double *ss, bool fp64 = false) {
  const bool on = (ss || fp64) && rz_fused(c);
  c->rz_partials = on ? c->partials : nullptr;
  c->rz_r64 = on && ss ? c->kr : nullptr;
  c->rz_ss = on ? ss : nullptr;
}

static hipError_t bottom64(sbm_ctx *c, const double *f, double *x) {
  Level &B = c->L[c->nlev - 1];
  return launch_bottom_cg<double>(B, B.psi64, B.c64, f, x, c->b_r, c->b_p, c->b_Ap,
                                  c->opt.bottom_rtol, bottom_maxit(c), c->iflag + 4, c->st);
}

static hipError_t bottom32(sbm_ctx *c, const float *f, float *x) {
  // the near-singular bottom is solved in FP64 also inside the FP32 cycle
  Level &B = c->L[c->nlev - 1];
  return launch_bottom_f32io(B, f, x, c->b_r64, c->b_x64, c->b_r, c->b_p, c->b_Ap,
                             c->opt.bottom_rtol, bottom_maxit(c), c->iflag + 4, c->st);
}

// V-cycle on level l: x (in/out), f (load), tmp (scratch of level l).
template <typename T>
static hipError_t vcycle(sbm_ctx *c, int l, T *x, const T *f, T *tmp) {
  hipError_t e;
  if (l == (sizeof(T) == 8 ? c->tail64 : c->tail32)) {
    // the rest of the cycle in one workgroup (LDS-resident levels)
    ProfScope ps(c, SBM_PROF_BOTTOM, true);
    const TailOpts o{c->opt.nu_pre, c->opt.nu_post, c->opt.smoother == 1, c->opt.krylov == 1,
                     opt_omega(c->opt), c->opt.bottom_rtol, bottom_maxit(c)};
    const bool fp64 = sizeof(T) == 8;
    return launch_tail<T>(c->dim, c->L.back().g.nn > kTailWaveBottom,
                          c->tail_args + (fp64 ? 0 : kTailArgBytes),
                          fp64 ? c->tail_lds64 : c->tail_lds32, x, f, o, c->iflag + 4, c->st);
  }
  if (l == c->nlev - 1) {
    ProfScope ps(c, SBM_PROF_BOTTOM, true);
    if constexpr (sizeof(T) == 8) return bottom64(c, f, x);
    else return bottom32(c, f, x);
  }
  Level &L = c->L[l];
  Level &C = c->L[l + 1];
  if ((e = smooth<T>(c, l, x, f, tmp, c->opt.nu_pre, false, true)) != hipSuccess) return e;
  {
    ProfScope ps(c, SBM_PROF_RESIDUAL, l == 0);
    if ((e = launch_residual<T>(L, Prec<T>::psi(L), Prec<T>::coef(L), x, f, tmp, nullptr,
                                c->st)) != hipSuccess)
      return e;
  }
  {
    ProfScope ps(c, SBM_PROF_RESTRICT, l == 0);
    if ((e = launch_restrict<T>(L, C, tmp, Prec<T>::f(C), c->st, Prec<T>::e(C))) != hipSuccess)
      return e;
  }
  if ((e = vcycle<T>(c, l + 1, Prec<T>::e(C), Prec<T>::f(C), Prec<T>::t(C))) != hipSuccess) return e;
  {
    ProfScope ps(c, SBM_PROF_PROLONG, l == 0);
    if ((e = launch_prolong_add<T>(L, C, Prec<T>::e(C), x, c->st)) != hipSuccess) return e;
  }
  // as a CG preconditioner the cycle is made symmetric: post-smoothing runs
  // the colours in reverse order
  return smooth<T>(c, l, x, f, tmp, c->opt.nu_post, c->opt.krylov == 1, false);
}

hipError_t sbm::base_vcycle(sbm_ctx *c, int precision, void *x, const void *f) {
  Level &L0 = c->L[0];
  if (precision == 1) return vcycle<float>(c, 0, (float *)x, (const float *)f, L0.t32);
  return vcycle<double>(c, 0, (double *)x, (const double *)f, L0.t);
}

// ||r||_2^2 of the level-0 residual f - K u (free DOF), synchronising.
static sbm_status residual_norm2(sbm_ctx *c, const double *u, const double *f, double *out) {
  Level &L = c->L[0];
  {
    ProfScope ps(c, SBM_PROF_NORM, true);
    HIP_TRY((launch_residual<double>(L, L.psi64, L.c64, u, f, nullptr, c->partials, c->st)));
  }
  HIP_TRY(launch_finalize_sum(c->partials, stencil_partials(L), c->scal, c->st));
  HIP_TRY(hipMemcpyAsync(c->host, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIP_TRY(hipStreamSynchronize(c->st));
  if (c->prof_on) prof_harvest(c);
  *out = c->host[0];
  return SBM_OK;
}

// As residual_norm2, and the first pre-smoothing half-sweep of the next
// V-cycle from the same pass (into the finest level's tmp vector).
static sbm_status residual_norm2_sweep(sbm_ctx *c, const double *u, const double *f,
                                       double *out) {
  Level &L = c->L[0];
  {
    ProfScope ps(c, SBM_PROF_NORM, true);
    HIP_TRY(launch_residual_sweep(L, u, f, L.t, opt_omega(c->opt), 0, c->partials, c->st));
  }
  HIP_TRY(launch_finalize_sum(c->partials, stencil_partials(L), c->scal, c->st));
  HIP_TRY(hipMemcpyAsync(c->host, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIP_TRY(hipStreamSynchronize(c->st));
  if (c->prof_on) prof_harvest(c);
  *out = c->host[0];
  return SBM_OK;
}

// As residual_norm2, and f - K u written into the finest tmp vector (the
// residual the mixed cycle then casts).
static sbm_status residual_norm2_keep(sbm_ctx *c, const double *u, const double *f,
                                      double *out) {
  Level &L = c->L[0];
  {
    ProfScope ps(c, SBM_PROF_NORM, true);
    HIP_TRY((launch_residual<double>(L, L.psi64, L.c64, u, f, L.t, c->partials, c->st)));
  }
  HIP_TRY(launch_finalize_sum(c->partials, stencil_partials(L), c->scal, c->st));
  HIP_TRY(hipMemcpyAsync(c->host, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIP_TRY(hipStreamSynchronize(c->st));
  if (c->prof_on) prof_harvest(c);
  *out = c->host[0];
  return SBM_OK;
}

// One cycle of the outer loop on the finest iterate x0 for the load f: an
// FP64 V-cycle, or (mixed) r32 = (f - K x0)/s, an FP32 V-cycle for e32 from
// zero, x0 += s e32 with s the residual norm left in scal[0] by the
// convergence test.
static hipError_t cycle_body(sbm_ctx *c, const double *f, int mode) {
  Level &L0 = c->L[0];
  const int64_t nv = (int64_t)c->dim * L0.g.nn;
  hipError_t e;
  if (mode == 4) {
    // the mixed preconditioner on an FP32 load the CG update already cast
    // (kr / s, s^2 in scal[7]): the finest level starts from zero
    c->zero_start = true;
    rz_set(c, c->scal + 7);
    e = vcycle<float>(c, 0, L0.e32, L0.f32, L0.t32);
    rz_set(c, nullptr);
    c->zero_start = false;
    if (e != hipSuccess) return e;
    return launch_store_sqrt(c->scal + 7, c->scal + 6, c->st);
  }
  if (mode == 1) {
    // preconditioner: kz = M kr, one V-cycle from zero (mixed: on kr / ||kr||
    // in FP32, ||kr||^2 in scal[0]).  When the finest level smooths outside
    // the tail, its first half-sweep from zero is pointwise (omega kr / D on
    // one colour) and is made together with the cast or instead of the fill.
    const bool skip = c->opt.smoother == 0 && c->opt.nu_pre >= 1 && c->nlev > 1;
    // a finest level swept by the fused kernel starts that sweep from zero
    const bool zs = skip && tiled_ok(L0);
    if (c->opt.precision == 1) {
      if (zs && c->tail32 != 0) {
        if ((e = launch_cast_scaled(c->kr, L0.f32, nv, c->scal, c->st)) != hipSuccess) return e;
        c->zero_start = true;
      } else if (skip && c->tail32 != 0) {
        if ((e = launch_scale_cast_sweep(L0, c->kr, L0.f32, L0.t32, opt_omega(c->opt), 0, c->scal,
                                         c->st)) != hipSuccess)
          return e;
        c->first_half_done = true;
      } else {
        if ((e = launch_cast_scaled(c->kr, L0.f32, nv, c->scal, c->st)) != hipSuccess) return e;
        if ((e = launch_fill<float>(L0.e32, nv, 0.0f, c->st)) != hipSuccess) return e;
      }
      rz_set(c, c->scal);  // every branch above cast kr with s^2 = scal[0]
      e = vcycle<float>(c, 0, L0.e32, L0.f32, L0.t32);
      rz_set(c, nullptr);
      c->first_half_done = false;
      c->zero_start = false;
      if (e != hipSuccess) return e;
      // z = s e32 with s = ||kr|| kept in scal[6]: the Krylov kernels read e32
      // and scale it themselves (the FP64 z is never written)
      return launch_store_sqrt(c->scal, c->scal + 6, c->st);
    }
    if (zs && c->tail64 != 0) {
      c->zero_start = true;
    } else if (skip && c->tail64 != 0) {
      if ((e = launch_zero_sweep(L0, c->kr, L0.t, opt_omega(c->opt), 0, c->st)) != hipSuccess)
        return e;
      c->first_half_done = true;
    } else if ((e = launch_fill<double>(c->kz, nv, 0.0, c->st)) != hipSuccess) {
      return e;
    }
    rz_set(c, nullptr, true);
    e = vcycle<double>(c, 0, c->kz, c->kr, L0.t);
    rz_set(c, nullptr);
    c->first_half_done = false;
    c->zero_start = false;
    return e;
  }
  if (c->opt.precision == 1) {
    if (mode == 3) {
      // the convergence test left f - K x0 in the finest tmp vector; its cast
      // also makes the FP32 cycle's first half-sweep from zero (into t32)
      if ((e = launch_scale_cast_sweep(L0, L0.t, L0.f32, L0.t32, opt_omega(c->opt), 0, c->scal,
                                       c->st)) != hipSuccess)
        return e;
      c->first_half_done = true;
      e = vcycle<float>(c, 0, L0.e32, L0.f32, L0.t32);
      c->first_half_done = false;
      if (e != hipSuccess) return e;
      return launch_correct(L0, c->x0, L0.e32, c->scal, c->st);
    }
    // mode 2: the convergence test left f - K x0 in the finest tmp vector
    if ((e = mode == 2 ? launch_scale_cast(L0.t, L0.f32, nv, c->scal, c->st)
                       : launch_residual_cast(L0, c->x0, f, L0.f32, c->scal, c->st)) != hipSuccess)
      return e;
    if (tiled_ok(L0) && c->opt.smoother == 0 && c->opt.nu_pre >= 1 && c->nlev > 1 &&
        c->tail32 != 0)
      c->zero_start = true;
    else if ((e = launch_fill<float>(L0.e32, nv, 0.0f, c->st)) != hipSuccess)
      return e;
    e = vcycle<float>(c, 0, L0.e32, L0.f32, L0.t32);
    c->zero_start = false;
    if (e != hipSuccess) return e;
    return launch_correct(L0, c->x0, L0.e32, c->scal, c->st);
  }
  c->first_half_done = mode == 2;
  e = vcycle<double>(c, 0, c->x0, f, L0.t);
  c->first_half_done = false;
  return e;
}

// Finds or captures the graph of cycle_body for (precision, f, profiling).
// Returns nullptr when capture is not possible (the cycle then runs eagerly).
static sbm_ctx::CycleGraph *cycle_graph(sbm_ctx *c, const double *f, int mode) {
  for (auto *g : c->graphs)
    if (g->mode == mode && g->precision == c->opt.precision && g->f == f && g->prof == c->prof_on)
      return g->failed ? nullptr : g;
  auto *g = new sbm_ctx::CycleGraph();
  g->mode = mode;
  g->precision = c->opt.precision;
  g->f = f;
  g->prof = c->prof_on;
  c->graphs.push_back(g);
  if (!c->cap_st && hipStreamCreateWithFlags(&c->cap_st, hipStreamNonBlocking) != hipSuccess) {
    c->cap_st = nullptr;
    g->failed = true;
    return nullptr;
  }
  hipStream_t user = c->st;
  c->st = c->cap_st;
  c->capturing = g;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(c->cap_st, hipStreamCaptureModeRelaxed);
  hipError_t eb = hipSuccess;
  if (e == hipSuccess) {
    eb = cycle_body(c, f, mode);
    e = hipStreamEndCapture(c->cap_st, &graph);
  }
  c->capturing = nullptr;
  c->st = user;
  if (e == hipSuccess && eb == hipSuccess && graph)
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  else if (e == hipSuccess)
    e = eb != hipSuccess ? eb : hipErrorUnknown;
  if (graph) {
    hipError_t ed = hipGraphDestroy(graph);
    if (e == hipSuccess) e = ed;
  }
  if (e != hipSuccess) {
    c->graph_error = hipGetErrorString(e);
    (void)hipGetLastError();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    g->exec = nullptr;
    g->failed = true;
    return nullptr;
  }
  ++c->graph_captures;
  return g;
}

static sbm_status run_cycle(sbm_ctx *c, const double *f, int mode) {
  // Live timing brackets single launches with events, so it runs the cycle
  // launch by launch (event records inside a replayed graph give no timings
  // on this runtime).
  if (c->opt.use_graphs && !c->prof_on) {
    sbm_ctx::CycleGraph *g = cycle_graph(c, f, mode);
    if (g) {
      HIP_TRY(hipGraphLaunch(g->exec, c->st));
      ++c->graph_launches;
      c->pending = g;
      return SBM_OK;
    }
  }
  HIP_TRY(cycle_body(c, f, mode));
  return SBM_OK;
}

// Finalises `n` partials into scal[slot] and copies scal[slot] to host[slot].
static sbm_status fin_to_host(sbm_ctx *c, const double *partials, int n, int slot) {
  HIP_TRY(launch_finalize_sum(partials, n, c->scal + slot, c->st));
  HIP_TRY(hipMemcpyAsync(c->host + slot, c->scal + slot, sizeof(double), hipMemcpyDeviceToHost,
                         c->st));
  return SBM_OK;
}

#define SBM_TRY(expr)                      \
  do {                                     \
    sbm_status s_ = (expr);                \
    if (s_ != SBM_OK) return s_;           \
  } while (0)

// Flexible CG (Polak-Ribiere beta) on the finest level, preconditioned by one
// V-cycle from zero per iteration.  Device scalars: scal[0] = r.r,
// scal[1] = r.z (new), scal[2] = p.q, scal[3] = r.z (old z), scal[4] = r.z
// of the previous iteration, scal[5] = alpha of the last update; mixed:
// scal[6] = the scale s of z = s e32, scal[7] = s^2 of the cast the CG update
// makes.  The update
// x += alpha p is deferred to the pass that forms the next direction (which
// reads p anyway), or made on its own when the iteration ends: the iterates
// are the same numbers.
static sbm_status solve_krylov(sbm_ctx *c, const double *f, double fnorm, double *u, double *hist,
                               int cap, int *ncyc, double *final_rel) {
  Level &L0 = c->L[0];
  const int64_t nv = (int64_t)c->dim * L0.g.nn;
  const int nb = num_blocks(L0.g.nn);       // node-parallel kernels
  const int ns = stencil_partials(L0);      // residual / Apply kernels
  // r . z from the preconditioner's last half-sweep, else a pass of its own
  const bool rzf = rz_fused(c);
  const bool castf = cast_fused(c);
  const int nrz = rzf ? rb_tiled_partials(L0, c->opt.precision == 1) : 0;
  double rho_min = INFINITY, rho = 0.0;
  sbm_status status = SBM_NOT_CONVERGED;
  // the preconditioned residual: kz, or (mixed) scal[6] * the FP32 correction
  const ZSrc z = c->opt.precision == 1 ? ZSrc{nullptr, L0.e32, c->scal + 6}
                                       : ZSrc{c->kz, nullptr, nullptr};
  HIP_TRY(launch_copy<double>(u, c->x0, nv, c->st));
  {
    ProfScope ps(c, SBM_PROF_NORM, true);
    HIP_TRY((launch_residual<double>(L0, L0.psi64, L0.c64, c->x0, f, c->kr, c->partials, c->st)));
  }
  SBM_TRY(fin_to_host(c, c->partials, ns, 0));
  HIP_TRY(hipStreamSynchronize(c->st));
  rho = fnorm > 0.0 ? sqrt(c->host[0]) / fnorm : (c->host[0] > 0.0 ? INFINITY : 0.0);
  if (hist && cap > 0) hist[0] = rho;
  bool restart = true;
  int m = 0;
  for (;;) {
    if (!isfinite(rho)) {
      status = fail(SBM_E_NONFINITE, "non-finite residual at iteration " + std::to_string(m));
      break;
    }
    if (rho <= c->opt.rtol) {
      status = SBM_OK;
      break;
    }
    if (rho > 1e3 * rho_min) {
      status = fail(SBM_E_DIVERGED, "residual grew above 1e3 x its minimum at iteration " +
                                        std::to_string(m));
      break;
    }
    rho_min = std::min(rho_min, rho);
    if (m >= c->opt.max_cycles) {
      g_last_error = "max_cycles reached";
      break;
    }
    if (restart) {
      SBM_TRY(run_cycle(c, nullptr, 1));
      if (rzf) {
        HIP_TRY(launch_finalize_sum(c->partials, nrz, c->scal + 4, c->st));
      } else {
        HIP_TRY(launch_dot_free(L0, c->kr, z, c->partials, c->st));
        HIP_TRY(launch_finalize_sum(c->partials, nb, c->scal + 4, c->st));
      }
      HIP_TRY(launch_xpby_x(L0, c->x0, c->kp, z, nullptr, nullptr, nullptr, nullptr, c->st));
      restart = false;
    }
    HIP_TRY(launch_apply_dot(L0, c->kp, c->kq, c->partials, c->st));
    SBM_TRY(fin_to_host(c, c->partials, ns, 2));
    HIP_TRY(hipStreamSynchronize(c->st));
    if (c->prof_on) prof_harvest(c);
    if (!(c->host[2] > 0.0)) {
      status = fail(SBM_E_DIVERGED, "preconditioned CG lost positivity (p.Kp <= 0)");
      break;
    }
    // r -= alpha q; the iterate update x += alpha p (alpha kept in scal[5]) is
    // made by the next direction update, or below when the iteration ends.
    // Mixed: the same pass casts r / s for the next cycle, s = the norm of
    // the residual before the update (scal[0] -> scal[7]).
    if (castf) HIP_TRY(launch_copy<double>(c->scal, c->scal + 7, 1, c->st));
    HIP_TRY(launch_cg_update_r(L0, c->kr, c->kq, z, c->scal + 4, c->scal + 2, c->scal + 5,
                               c->partials, c->partials2, c->st, castf ? L0.f32 : nullptr,
                               castf ? c->scal + 7 : nullptr));
    SBM_TRY(fin_to_host(c, c->partials, nb, 0));
    SBM_TRY(fin_to_host(c, c->partials2, nb, 3));
    HIP_TRY(hipStreamSynchronize(c->st));
    ++m;
    rho = fnorm > 0.0 ? sqrt(c->host[0]) / fnorm : 0.0;
    if (rho <= c->opt.rtol) {
      // accept on the true residual only; otherwise restart from it
      HIP_TRY(launch_axpy_free(L0, c->x0, c->kp, c->scal + 5, c->st));
      {
        ProfScope ps(c, SBM_PROF_NORM, true);
        HIP_TRY((launch_residual<double>(L0, L0.psi64, L0.c64, c->x0, f, c->kr, c->partials,
                                         c->st)));
      }
      SBM_TRY(fin_to_host(c, c->partials, ns, 0));
      HIP_TRY(hipStreamSynchronize(c->st));
      rho = fnorm > 0.0 ? sqrt(c->host[0]) / fnorm : 0.0;
      if (hist && m < cap) hist[m] = rho;
      if (rho > c->opt.rtol) restart = true;
      continue;
    }
    if (hist && m < cap) hist[m] = rho;
    SBM_TRY(run_cycle(c, nullptr, castf ? 4 : 1));
    if (rzf) {
      HIP_TRY(launch_finalize_sum(c->partials, nrz, c->scal + 1, c->st));
    } else {
      HIP_TRY(launch_dot_free(L0, c->kr, z, c->partials, c->st));
      HIP_TRY(launch_finalize_sum(c->partials, nb, c->scal + 1, c->st));
    }
    HIP_TRY(launch_xpby_x(L0, c->x0, c->kp, z, c->scal + 1, c->scal + 3, c->scal + 4,
                          c->scal + 5, c->st));
    HIP_TRY(launch_copy<double>(c->scal + 1, c->scal + 4, 1, c->st));
  }
  if (ncyc) *ncyc = m;
  if (final_rel) *final_rel = rho;
  HIP_TRY(launch_copy<double>(c->x0, u, nv, c->st));
  HIP_TRY(hipStreamSynchronize(c->st));
  if (c->prof_on) prof_harvest(c);
  return status;
}

// Outer loop on the finest level for K u = f, u carrying its displacement
// values; fnorm normalises the residual.  The iterate lives in x0 during the
// solve.
static sbm_status solve_impl(sbm_ctx *c, const double *f, double fnorm, double *u, double *hist,
                             int cap, int *ncyc, double *final_rel) {
  if (c->opt.krylov == 1) return solve_krylov(c, f, fnorm, u, hist, cap, ncyc, final_rel);
  Level &L0 = c->L[0];
  const int64_t nv = (int64_t)c->dim * L0.g.nn;
  double rho_min = INFINITY, rho = 0.0;
  int m = 0;
  sbm_status status = SBM_NOT_CONVERGED;
  HIP_TRY(launch_copy<double>(u, c->x0, nv, c->st));
  // FP64 V-cycles with Gauss-Seidel pre-smoothing on a finest level swept by
  // the node-parallel kernels: the convergence test also makes the next
  // cycle's first half-sweep (the iterate itself is left as it is, so a
  // converged solve returns the tested iterate)
  const bool fused = c->opt.precision == 0 && c->opt.smoother == 0 && c->opt.nu_pre >= 1 &&
                     c->nlev > 1 && c->tail64 != 0 && residual_sweep_ok(L0);
  // mixed: the convergence test keeps f - K x0 for the cycle's cast, which
  // also makes the FP32 cycle's first half-sweep when the finest level
  // smooths outside the tail
  const bool keep = c->opt.precision == 1 && residual_sweep_ok(L0);
  const bool keep_sweep = keep && c->opt.smoother == 0 && c->opt.nu_pre >= 1 && c->nlev > 1 &&
                          c->tail32 != 0;
  for (m = 0;; ++m) {
    double ss = 0.0;
    sbm_status s = fused  ? residual_norm2_sweep(c, c->x0, f, &ss)
                   : keep ? residual_norm2_keep(c, c->x0, f, &ss)
                          : residual_norm2(c, c->x0, f, &ss);
    if (s != SBM_OK) return s;
    rho = fnorm > 0.0 ? sqrt(ss) / fnorm : (ss > 0.0 ? INFINITY : 0.0);
    if (hist && m < cap) hist[m] = rho;
    if (!isfinite(rho)) {
      status = fail(SBM_E_NONFINITE, "non-finite residual at cycle " + std::to_string(m));
      break;
    }
    if (rho <= c->opt.rtol) {
      status = SBM_OK;
      break;
    }
    if (rho > 1e3 * rho_min) {
      status = fail(SBM_E_DIVERGED, "residual grew above 1e3 x its minimum at cycle " +
                                        std::to_string(m));
      break;
    }
    rho_min = std::min(rho_min, rho);
    if (m >= c->opt.max_cycles) {
      g_last_error = "max_cycles reached";
      status = SBM_NOT_CONVERGED;
      break;
    }
    s = run_cycle(c, f, keep_sweep ? 3 : (fused || keep ? 2 : 0));
    if (s != SBM_OK) return s;
  }
  if (ncyc) *ncyc = m;
  if (final_rel) *final_rel = rho;
  HIP_TRY(launch_copy<double>(c->x0, u, nv, c->st));
  HIP_TRY(hipStreamSynchronize(c->st));
  if (c->prof_on) prof_harvest(c);
  return status;
}

// ------------------------------------------------------------------- ABI

extern "C" {

void sbm_default_options(sbm_options *o) {
  if (!o) return;
  o->smoother = 0;
  o->omega = 0.0;
  o->nu_pre = 2;
  o->nu_post = 2;
  o->precision = 0;
  o->rtol = 1e-10;
  o->max_cycles = 200;
  o->bottom_rtol = 1e-12;
  o->bottom_max_iter = 0;
  o->use_graphs = 1;
  o->krylov = 0;
  o->fused_sweep = 0;
}

const char *sbm_last_error(void) { return g_last_error.c_str(); }

int sbm_num_levels(const sbm_grid *grid) {
  if (!grid_ok(grid)) return 0;
  return count_levels(grid);
}

static bool opts_ok(const sbm_options *o) {
  return o && (o->smoother == 0 || o->smoother == 1) && o->nu_pre >= 0 && o->nu_post >= 0 &&
         (o->precision == 0 || o->precision == 1) && o->rtol >= 0.0 && o->max_cycles >= 0 &&
         o->bottom_rtol >= 0.0 && isfinite(o->omega) && o->omega >= 0.0 && o->omega < 2.0 &&
         (o->use_graphs == 0 || o->use_graphs == 1) && (o->krylov == 0 || o->krylov == 1) &&
         (o->fused_sweep == 0 || o->fused_sweep == 1);
}

size_t sbm_workspace_bytes(const sbm_grid *grid, const sbm_options *opts) {
  if (!grid_ok(grid) || !opts_ok(opts)) return 0;
  sbm_ctx c;
  c.dim = grid->dim;
  c.nlev = count_levels(grid);
  level_shapes(grid, c.nlev, c.L);
  return carve(&c, nullptr);
}

sbm_status sbm_create(const sbm_grid *grid, const sbm_options *opts, void *workspace,
                      size_t workspace_bytes, void *hip_stream, sbm_ctx **out) {
  if (!out) return fail(SBM_E_ARG, "out is NULL");
  *out = nullptr;
  if (!grid_ok(grid)) return fail(SBM_E_SHAPE, "invalid grid (dim 2/3, ncell >= 1, h > 0)");
  if (!opts_ok(opts)) return fail(SBM_E_ARG, "invalid options");
  if (!workspace || ((uintptr_t)workspace & 255))
    return fail(SBM_E_WORKSPACE, "workspace NULL or not 256-byte aligned");
  sbm_ctx *c = new sbm_ctx();
  c->dim = grid->dim;
  c->nlev = count_levels(grid);
  level_shapes(grid, c->nlev, c->L);
  const size_t need = carve(c, nullptr);
  if (workspace_bytes < need) {
    delete c;
    return fail(SBM_E_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  }
  c->ws = (char *)workspace;
  c->ws_bytes = workspace_bytes;
  carve(c, c->ws);
  c->opt = *opts;
  c->st = (hipStream_t)hip_stream;
  {
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        lds <= 0)
      lds = 64 * 1024;
    (void)hipGetLastError();
    c->tail_lds_max = (size_t)lds;
    c->tail64 = tail_level(c->L, 0, (size_t)lds);
    c->tail32 = tail_level(c->L, 1, (size_t)lds);
  }
  hipError_t e = hipHostMalloc((void **)&c->host, 64 * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) {
    delete c;
    return fail(SBM_E_HIP, std::string("hipHostMalloc: ") + hipGetErrorString(e));
  }
  *out = c;
  return SBM_OK;
}

sbm_status sbm_set_options(sbm_ctx *c, const sbm_options *opts) {
  if (!c) return fail(SBM_E_ARG, "ctx is NULL");
  if (!opts_ok(opts)) return fail(SBM_E_ARG, "invalid options");
  const sbm_options &o = c->opt;
  const bool same = o.smoother == opts->smoother && o.omega == opts->omega &&
                    o.nu_pre == opts->nu_pre && o.nu_post == opts->nu_post &&
                    o.bottom_rtol == opts->bottom_rtol && o.bottom_max_iter == opts->bottom_max_iter &&
                    o.krylov == opts->krylov && o.fused_sweep == opts->fused_sweep;
  if (!same) {
    HIP_TRY(hipStreamSynchronize(c->st));
    drop_graphs(c);
  }
  c->opt = *opts;
  return SBM_OK;
}

void sbm_destroy(sbm_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->st);
  drop_graphs(c);
  if (c->cap_st) (void)hipStreamDestroy(c->cap_st);
  if (c->host) (void)hipHostFree(c->host);
  for (hipEvent_t e : c->prof_ev) (void)hipEventDestroy(e);
  delete c;
}

sbm_status sbm_profile(sbm_ctx *c, int enable) {
  if (!c) return fail(SBM_E_ARG, "ctx is NULL");
  HIP_TRY(hipStreamSynchronize(c->st));
  c->prof_cls.clear();
  for (int k = 0; k < SBM_PROF_N; ++k) {
    c->prof_ms[k] = 0.0;
    c->prof_n[k] = 0;
  }
  c->prof_on = enable != 0;
  return SBM_OK;
}

// -------------------------------------------- allocation-free residual
//
// sbm_residual_static keeps its partial sums in this file-scope device array
// (one copy per device, for the life of the process) instead of a workspace.
// Host code never passes `scratch` itself to a kernel: its device address is
// looked up once per device with hipGetSymbolAddress and kept in
// g_scratch_dev.
constexpr int kScratchDoubles = 1 << 17;  // 1 MiB: partial sums + the total
__device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_dev[kMaxDevices] = {};

static sbm_status scratch_address(double **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(SBM_E_ARG, "device id out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(SBM_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_dev[dev] = (double *)p;
  }
  *out = g_scratch_dev[dev];
  return SBM_OK;
}

sbm_status sbm_residual_static(const sbm_grid *grid, const sbm_material *mat, const sbm_bc *bc,
                               const double *psi, const double *u, const double *f, double *r,
                               double *norm_host, void *hip_stream) {
  if (!grid_ok(grid)) return fail(SBM_E_SHAPE, "unsupported grid");
  if (!mat || !bc || !psi || !u || !f || !norm_host) return fail(SBM_E_ARG, "NULL argument");
  NO_ALIAS(u, r);
  NO_ALIAS(f, r);
  NO_ALIAS(psi, r);
  if (!isfinite(mat->lambda) || !isfinite(mat->mu) || !(mat->mu > 0.0) ||
      !(mat->lambda + mat->mu > 0.0))
    return fail(SBM_E_ARG, "material needs mu > 0, lambda + mu > 0");
  uint32_t dmask = 0;
  for (int F = 0; F < 2 * grid->dim; ++F)
    for (int k = 0; k < grid->dim; ++k) {
      if (bc->kind[F][k] != SBM_TRACTION && bc->kind[F][k] != SBM_DISPLACEMENT)
        return fail(SBM_E_ARG, "bc kind must be TRACTION or DISPLACEMENT");
      if (bc->kind[F][k] == SBM_DISPLACEMENT) dmask |= 1u << (3 * F + k);
    }
  Level L;
  make_level(grid->dim, grid->ncell, grid->h, L);
  L.g.dmask = dmask;
  set_coefs(L, mat->lambda, mat->mu, grid->dim);
  const int np = stencil_partials(L);
  if (np > kScratchDoubles - 1)
    return fail(SBM_E_SHAPE, "grid too large for the static scratch of sbm_residual_static (" +
                                 std::to_string(np) + " partial sums, at most " +
                                 std::to_string(kScratchDoubles - 1) + ")");
  double *sc = nullptr;
  sbm_status s = scratch_address(&sc);
  if (s != SBM_OK) return s;
  hipStream_t st = (hipStream_t)hip_stream;
  // every partial sum and the total are written before they are read: the
  // array needs no clearing between calls
  HIP_TRY((launch_residual<double>(L, psi, L.c64, u, f, r, sc, st)));
  HIP_TRY(launch_finalize_sum(sc, np, sc + kScratchDoubles - 1, st));
  double ss = 0.0;
  HIP_TRY(hipMemcpyAsync(&ss, sc + kScratchDoubles - 1, sizeof(double), hipMemcpyDeviceToHost,
                         st));
  HIP_TRY(hipStreamSynchronize(st));
  *norm_host = sqrt(ss);
  return SBM_OK;
}

sbm_status sbm_stream_triad(double *a, const double *b, const double *cc, int64_t n, double s,
                            void *hip_stream) {
  if (!a || !b || !cc || n < 1) return fail(SBM_E_ARG, "NULL argument or n < 1");
  if (((uintptr_t)a | (uintptr_t)b | (uintptr_t)cc) & 15)
    return fail(SBM_E_ARG, "triad arrays must be 16-byte aligned");
  if (n > ((int64_t)1 << 40)) return fail(SBM_E_ARG, "n too large");
  NO_ALIAS(a, b);
  NO_ALIAS(a, cc);
  HIP_TRY(launch_triad(a, b, cc, n, s, (hipStream_t)hip_stream));
  return SBM_OK;
}

sbm_status sbm_graph_info(sbm_ctx *c, int64_t *captures, int64_t *launches) {
  if (!c || !captures || !launches) return fail(SBM_E_ARG, "NULL argument");
  *captures = c->graph_captures;
  *launches = c->graph_launches;
  if (!c->graph_error.empty()) g_last_error = "last capture failed: " + c->graph_error;
  return SBM_OK;
}

sbm_status sbm_profile_read(sbm_ctx *c, double *ms, int64_t *cnt) {
  if (!c || !ms || !cnt) return fail(SBM_E_ARG, "NULL argument");
  HIP_TRY(hipStreamSynchronize(c->st));
  prof_harvest(c);
  for (int k = 0; k < SBM_PROF_N; ++k) {
    ms[k] = c->prof_ms[k];
    cnt[k] = c->prof_n[k];
  }
  return SBM_OK;
}

static sbm_status set_problem_impl(sbm_ctx *c, const double *psi_raw, int cube,
                                   const sbm_material *mat, const sbm_bc *bc, const double *b) {
  if (!c || !psi_raw || !mat || !bc) return fail(SBM_E_ARG, "NULL argument");
  if (!isfinite(mat->lambda) || !isfinite(mat->mu) || !(mat->mu > 0.0) ||
      !(mat->lambda + mat->mu > 0.0) || !(mat->psi_floor >= 0.0))
    return fail(SBM_E_ARG, "material needs mu > 0, lambda + mu > 0, psi_floor >= 0");
  uint32_t dmask = 0;
  for (int F = 0; F < 2 * c->dim; ++F)
    for (int k = 0; k < c->dim; ++k) {
      if (bc->kind[F][k] != SBM_TRACTION && bc->kind[F][k] != SBM_DISPLACEMENT)
        return fail(SBM_E_ARG, "bc kind must be TRACTION or DISPLACEMENT");
      if (!isfinite(bc->value[F][k])) return fail(SBM_E_NONFINITE, "non-finite bc value");
      if (bc->kind[F][k] == SBM_DISPLACEMENT) dmask |= 1u << (3 * F + k);
    }
  c->mat = *mat;
  c->bc = *bc;
  memset(&c->tr, 0, sizeof(c->tr));
  memset(&c->dv, 0, sizeof(c->dv));
  memset(&c->zero_dv, 0, sizeof(c->zero_dv));
  for (int F = 0; F < 6; ++F) {
    const int a = F / 2;
    c->tr.inv_h[F] = a < c->dim ? 1.0 / c->L[0].h[a] : 0.0;
    for (int k = 0; k < 3; ++k) {
      if (F < 2 * c->dim && k < c->dim) {
        if (bc->kind[F][k] == SBM_TRACTION) c->tr.t[F][k] = bc->value[F][k];
        else c->dv.v[F][k] = bc->value[F][k];
      }
    }
  }
  if (!(c->g_lam == mat->lambda && c->g_mu == mat->mu && c->g_dmask == dmask)) {
    // captured cycles hold the coefficients and masks as kernel arguments
    HIP_TRY(hipStreamSynchronize(c->st));
    drop_graphs(c);
    c->g_lam = mat->lambda;
    c->g_mu = mat->mu;
    c->g_dmask = dmask;
  }
  for (int l = 0; l < c->nlev; ++l) {
    c->L[l].g.dmask = dmask;
    set_coefs(c->L[l], mat->lambda, mat->mu, c->dim);
  }
  Level &L0 = c->L[0];
  HIP_TRY(launch_fill<int>(c->iflag, 16, 0, c->st));
  HIP_TRY(launch_floor_psi(psi_raw, mat->psi_floor, L0.psi64, L0.psi32, L0.g.nc, cube, c->iflag,
                           c->st));
  for (int l = 1; l < c->nlev; ++l) HIP_TRY(launch_coarsen_psi(c->L[l - 1], c->L[l], c->st));
  // tail level tables and the dense bottom matrix (needs the bottom psi)
  if (c->tail64 >= 0)
    HIP_TRY(tail_upload(c->L, 0, c->tail64, c->tail_args, c->tail_A, c->tail_lds_max,
                        &c->tail_lds64, c->st));
  if (c->tail32 >= 0)
    HIP_TRY(tail_upload(c->L, 1, c->tail32, c->tail_args + kTailArgBytes, c->tail_A,
                        c->tail_lds_max, &c->tail_lds32, c->st));
  HIP_TRY(launch_rhs(L0, c->tr, b, L0.f, c->iflag, c->st));
  HIP_TRY(launch_check_diag(L0, c->iflag, c->st));
  int flags = 0;
  HIP_TRY(hipMemcpyAsync(c->host, c->iflag, sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIP_TRY(hipStreamSynchronize(c->st));
  memcpy(&flags, c->host, sizeof(int));
  c->have_problem = false;
  if (flags & 1) return fail(SBM_E_NONFINITE, "NaN/Inf in psi or body force");
  if (flags & 2) return fail(SBM_E_DIAG, "a free DOF has no solid cell around it (zero diagonal)");
  // fnorm = ||fA - K uD|| over free DOF (uD: prescribed values, 0 elsewhere)
  const int64_t nv = (int64_t)c->dim * L0.g.nn;
  HIP_TRY(launch_fill<double>(L0.t, nv, 0.0, c->st));
  HIP_TRY(launch_set_dirichlet(L0, L0.t, c->dv, c->st));
  double ss = 0.0;
  sbm_status s = residual_norm2(c, L0.t, L0.f, &ss);
  if (s != SBM_OK) return s;
  if (!isfinite(ss)) return fail(SBM_E_NONFINITE, "non-finite load");
  c->fnorm = sqrt(ss);
  c->have_problem = true;
  return SBM_OK;
}

sbm_status sbm_set_problem(sbm_ctx *c, const double *psi_raw, const sbm_material *mat,
                           const sbm_bc *bc, const double *b) {
  return set_problem_impl(c, psi_raw, 0, mat, bc, b);
}

sbm_status sbm_set_problem_density(sbm_ctx *c, const double *rho, const sbm_material *mat,
                                   const sbm_bc *bc, const double *b) {
  return set_problem_impl(c, rho, 1, mat, bc, b);
}

#define NEED_PROBLEM(c)                                                     \
  do {                                                                      \
    if (!(c)) return fail(SBM_E_ARG, "ctx is NULL");                        \
    if (!(c)->have_problem) return fail(SBM_E_ARG, "sbm_set_problem first"); \
  } while (0)

sbm_status sbm_solve(sbm_ctx *c, double *u, double *hist, int cap, int *ncyc, double *final_rel) {
  NEED_PROBLEM(c);
  if (!u) return fail(SBM_E_ARG, "u is NULL");
  Level &L0 = c->L[0];
  HIP_TRY(launch_set_dirichlet(L0, u, c->dv, c->st));
  return solve_impl(c, L0.f, c->fnorm, u, hist, cap, ncyc, final_rel);
}

sbm_status sbm_solve_rhs(sbm_ctx *c, const double *g, double *x, double *hist, int cap, int *ncyc,
                         double *final_rel) {
  NEED_PROBLEM(c);
  if (!g || !x) return fail(SBM_E_ARG, "NULL argument");
  Level &L0 = c->L[0];
  const int64_t nv = (int64_t)c->dim * L0.g.nn;
  // masked copy of g: r = g - K*0 on free DOF via the residual kernel
  HIP_TRY(launch_fill<double>(L0.t, nv, 0.0, c->st));
  HIP_TRY((launch_residual<double>(L0, L0.psi64, L0.c64, L0.t, g, L0.e, c->partials, c->st)));
  HIP_TRY(launch_finalize_sum(c->partials, stencil_partials(L0), c->scal, c->st));
  HIP_TRY(hipMemcpyAsync(c->host, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIP_TRY(hipStreamSynchronize(c->st));
  const double gn = sqrt(c->host[0]);
  HIP_TRY(launch_set_dirichlet(L0, x, c->zero_dv, c->st));
  return solve_impl(c, L0.e, gn, x, hist, cap, ncyc, final_rel);
}

sbm_status sbm_apply(sbm_ctx *c, const double *u, double *Ku) {
  NEED_PROBLEM(c);
  if (!u || !Ku) return fail(SBM_E_ARG, "NULL argument");
  NO_ALIAS(u, Ku);
  Level &L0 = c->L[0];
  HIP_TRY(launch_apply<double>(L0, L0.psi64, L0.c64, u, Ku, c->st));
  return SBM_OK;
}

sbm_status sbm_residual(sbm_ctx *c, const double *u, double *r, double *norm_host) {
  NEED_PROBLEM(c);
  if (!u) return fail(SBM_E_ARG, "u is NULL");
  NO_ALIAS(u, r);
  Level &L0 = c->L[0];
  if (!norm_host) {
    if (!r) return fail(SBM_E_ARG, "r and norm_host both NULL");
    HIP_TRY((launch_residual<double>(L0, L0.psi64, L0.c64, u, L0.f, r, nullptr, c->st)));
    return SBM_OK;
  }
  HIP_TRY((launch_residual<double>(L0, L0.psi64, L0.c64, u, L0.f, r, c->partials, c->st)));
  HIP_TRY(launch_finalize_sum(c->partials, stencil_partials(L0), c->scal, c->st));
  HIP_TRY(hipMemcpyAsync(c->host, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIP_TRY(hipStreamSynchronize(c->st));
  *norm_host = sqrt(c->host[0]);
  return SBM_OK;
}

sbm_status sbm_rhs(sbm_ctx *c, double *fA, double *fB) {
  NEED_PROBLEM(c);
  if (!fA) return fail(SBM_E_ARG, "fA is NULL");
  NO_ALIAS(fA, fB);
  Level &L0 = c->L[0];
  const int64_t nv = (int64_t)c->dim * L0.g.nn;
  HIP_TRY(launch_copy<double>(L0.f, fA, nv, c->st));
  if (fB) {
    HIP_TRY(launch_fill<double>(L0.t, nv, 0.0, c->st));
    HIP_TRY(launch_set_dirichlet(L0, L0.t, c->dv, c->st));
    HIP_TRY((launch_residual<double>(L0, L0.psi64, L0.c64, L0.t, L0.f, fB, nullptr, c->st)));
  }
  return SBM_OK;
}

sbm_status sbm_sensitivity(sbm_ctx *c, const double *u, const double *lam, double lam_scale,
                           const double *design, int chain, double *g) {
  NEED_PROBLEM(c);
  if (!u || !lam || !g) return fail(SBM_E_ARG, "NULL argument");
  if (aliased({u, g}) || aliased({lam, g}) || aliased({design, g}))
    return fail(SBM_E_ARG, "g aliases an input");
  if (chain < 0 || chain > 2 || (chain > 0 && !design))
    return fail(SBM_E_ARG, "chain must be 0, 1 or 2 (1 and 2 need design)");
  if (!isfinite(lam_scale)) return fail(SBM_E_ARG, "lam_scale must be finite");
  Level &L0 = c->L[0];
  HIP_TRY(launch_sensitivity(L0, c->mat.lambda, c->mat.mu, c->tr, u, lam, lam_scale, design, chain,
                             c->mat.psi_floor, g, c->st));
  return SBM_OK;
}

sbm_status sbm_plastic_source(sbm_ctx *c, const double *eps_p, double *f) {
  NEED_PROBLEM(c);
  if (!eps_p || !f) return fail(SBM_E_ARG, "NULL argument");
  NO_ALIAS(eps_p, f);
  if (c->dim != 3) return fail(SBM_E_SHAPE, "plastic strain: 3D grids only");
  Level &L0 = c->L[0];
  HIP_TRY(launch_plastic_source(L0, c->mat.lambda, c->mat.mu, eps_p, f, c->st));
  return SBM_OK;
}

sbm_status sbm_return_map(sbm_ctx *c, const double *u, const sbm_j2 *mat, double *eps_p,
                          double *alpha, double *beta, int64_t *n_plastic) {
  NEED_PROBLEM(c);
  if (!u || !mat || !eps_p || !alpha || !beta) return fail(SBM_E_ARG, "NULL argument");
  NO_ALIAS(u, eps_p, alpha, beta, n_plastic);
  if (c->dim != 3) return fail(SBM_E_SHAPE, "plastic strain: 3D grids only");
  if (!(mat->sigma_y >= 0.0) || !(mat->hbar >= 0.0) || !(mat->theta >= 0.0 && mat->theta <= 1.0) ||
      !isfinite(mat->sigma_y) || !isfinite(mat->hbar))
    return fail(SBM_E_ARG, "J2 parameters: sigma_y >= 0, hbar >= 0, 0 <= theta <= 1");
  Level &L0 = c->L[0];
  int *cnt = n_plastic ? c->iflag + 12 : nullptr;
  if (cnt) HIP_TRY(launch_fill<int>(cnt, 1, 0, c->st));
  HIP_TRY(launch_return_map(L0, c->mat.mu, mat->sigma_y, mat->hbar, mat->theta, u, eps_p, alpha,
                            beta, cnt, c->st));
  if (n_plastic) {
    HIP_TRY(hipMemcpyAsync(c->host, cnt, sizeof(int), hipMemcpyDeviceToHost, c->st));
    HIP_TRY(hipStreamSynchronize(c->st));
    int n = 0;
    memcpy(&n, c->host, sizeof(int));
    *n_plastic = n;
  }
  return SBM_OK;
}

sbm_status sbm_diffuse_traction(sbm_ctx *c, const double *psi_raw, double psi_floor,
                                const double *t_hat, double pressure, double *f) {
  if (!c) return fail(SBM_E_ARG, "ctx is NULL");
  if (!psi_raw || !f) return fail(SBM_E_ARG, "NULL argument");
  if (f == psi_raw) return fail(SBM_E_ARG, "f must not alias psi_raw");
  if (!(psi_floor >= 0.0) || !isfinite(psi_floor) || !isfinite(pressure))
    return fail(SBM_E_ARG, "psi_floor >= 0 and pressure must be finite");
  HIP_TRY(launch_diffuse_traction(c->L[0], psi_raw, psi_floor, t_hat, pressure, f, c->st));
  return SBM_OK;
}

sbm_status sbm_crack_drive(sbm_ctx *c, const double *u, double *H, uint8_t *intact) {
  NEED_PROBLEM(c);
  if (!u || !H || !intact) return fail(SBM_E_ARG, "NULL argument");
  if ((const void *)u == (const void *)H || (const void *)u == (const void *)intact ||
      (const void *)H == (const void *)intact)
    return fail(SBM_E_ARG, "u, H and intact must not alias each other");
  Level &L0 = c->L[0];
  HIP_TRY(launch_crack_drive(L0, c->mat.lambda, c->mat.mu, u, H, intact, c->st));
  return SBM_OK;
}

sbm_status sbm_phase_step(sbm_ctx *c, const double *crack, const double *H, const uint8_t *intact,
                          const sbm_pf *p, double *crack_out, double *psi_out) {
  if (!c) return fail(SBM_E_ARG, "ctx is NULL");
  if (!crack || !H || !intact || !p || !crack_out || !psi_out)
    return fail(SBM_E_ARG, "NULL argument");
  if (crack_out == crack || crack_out == H || psi_out == crack || psi_out == H ||
      psi_out == crack_out || (const void *)crack_out == (const void *)intact ||
      (const void *)psi_out == (const void *)intact)
    return fail(SBM_E_ARG, "crack_out and psi_out must not alias each other or the inputs");
  if (!(p->Gc >= 0.0) || !(p->xi > 0.0) || !(p->M >= 0.0) || !(p->dt >= 0.0) || !(p->eta >= 0.0) ||
      !isfinite(p->Gc) || !isfinite(p->xi) || !isfinite(p->M) || !isfinite(p->dt) ||
      !isfinite(p->eta))
    return fail(SBM_E_ARG, "phase-field parameters: Gc, M, dt, eta >= 0, xi > 0, finite");
  Level &L0 = c->L[0];
  HIP_TRY(launch_phase_step(L0, crack, H, intact, p->Gc, p->xi, p->M, p->dt, p->eta, crack_out,
                            psi_out, c->st));
  return SBM_OK;
}

sbm_status sbm_compliance(sbm_ctx *c, const double *u, double *J) {
  NEED_PROBLEM(c);
  if (!u || !J) return fail(SBM_E_ARG, "NULL argument");
  Level &L0 = c->L[0];
  HIP_TRY(launch_dot_free(L0, L0.f, ZSrc{u, nullptr, nullptr}, c->partials, c->st));
  HIP_TRY(launch_finalize_sum(c->partials, num_blocks(L0.g.nn), c->scal, c->st));
  HIP_TRY(hipMemcpyAsync(c->host, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIP_TRY(hipStreamSynchronize(c->st));
  double hd = 1.0;
  for (int a = 0; a < c->dim; ++a) hd *= L0.h[a];
  *J = hd * c->host[0];
  return SBM_OK;
}

// ------------------------------------------------------- component entries

#define LEVEL_OK(c, l)                                                      \
  do {                                                                      \
    NEED_PROBLEM(c);                                                        \
    if ((l) < 0 || (l) >= (c)->nlev) return fail(SBM_E_ARG, "level out of range"); \
  } while (0)

sbm_status sbm_level_shape(sbm_ctx *c, int l, int64_t *nc) {
  if (!c || !nc) return fail(SBM_E_ARG, "NULL argument");
  if (l < 0 || l >= c->nlev) return fail(SBM_E_ARG, "level out of range");
  const Geom &G = c->L[l].g;
  nc[0] = G.cx;
  nc[1] = G.cy;
  nc[2] = c->dim > 2 ? G.cz : 0;
  return SBM_OK;
}

sbm_status sbm_level_psi(sbm_ctx *c, int l, double *psi) {
  LEVEL_OK(c, l);
  if (!psi) return fail(SBM_E_ARG, "psi is NULL");
  HIP_TRY(launch_copy<double>(c->L[l].psi64, psi, c->L[l].g.nc, c->st));
  return SBM_OK;
}

sbm_status sbm_level_apply(sbm_ctx *c, int l, const double *u, double *Ku) {
  LEVEL_OK(c, l);
  if (!u || !Ku) return fail(SBM_E_ARG, "NULL argument");
  NO_ALIAS(u, Ku);
  Level &L = c->L[l];
  HIP_TRY(launch_apply<double>(L, L.psi64, L.c64, u, Ku, c->st));
  return SBM_OK;
}

sbm_status sbm_level_apply_f32(sbm_ctx *c, int l, const float *u, float *Ku) {
  LEVEL_OK(c, l);
  if (!u || !Ku) return fail(SBM_E_ARG, "NULL argument");
  NO_ALIAS(u, Ku);
  Level &L = c->L[l];
  HIP_TRY(launch_apply<float>(L, L.psi32, L.c32, u, Ku, c->st));
  return SBM_OK;
}

sbm_status sbm_level_smooth(sbm_ctx *c, int l, int colour, double omega, const double *u_in,
                            const double *f, double *u_out) {
  LEVEL_OK(c, l);
  if (!u_in || !f || !u_out) return fail(SBM_E_ARG, "NULL argument");
  NO_ALIAS(u_in, u_out);
  NO_ALIAS(f, u_out);
  if (!(omega > 0.0 && omega < 2.0) || colour > 1) return fail(SBM_E_ARG, "bad omega/colour");
  Level &L = c->L[l];
  if (colour < 0) HIP_TRY(launch_jacobi<double>(L, L.psi64, L.c64, u_in, f, u_out, omega, c->st));
  else if (tiled_sweep_ok(L))
    HIP_TRY(launch_rb_tiled<double>(L, L.psi64, L.c64, u_in, f, u_out, omega, colour, c->st));
  else HIP_TRY(launch_rb_half<double>(L, L.psi64, L.c64, u_in, f, u_out, omega, colour, c->st));
  return SBM_OK;
}

}  // extern "C"

template <typename T>
static sbm_status level_sweep(sbm_ctx *c, int l, int first, double omega, const T *u_in,
                              const T *f, T *u_out) {
  LEVEL_OK(c, l);
  if (!f || !u_out) return fail(SBM_E_ARG, "NULL argument");
  NO_ALIAS(u_in, u_out);
  NO_ALIAS(f, u_out);
  if (!(omega > 0.0 && omega < 2.0) || first < 0 || first > 1)
    return fail(SBM_E_ARG, "bad omega/colour");
  Level &L = c->L[l];
  const T *psi = Prec<T>::psi(L);
  const Coef<T> &C = Prec<T>::coef(L);
  if (tiled_ok(L)) {
    HIP_TRY(launch_rb_fused<T>(L, psi, C, u_in, f, u_out, omega, first, c->st));
    return SBM_OK;
  }
  // two half-sweeps through the level's scratch vector
  T *mid = Prec<T>::t(L);
  const T *src = u_in;
  if (!src) {
    HIP_TRY(launch_fill<T>(u_out, (int64_t)c->dim * L.g.nn, T(0), c->st));
    src = u_out;
  }
  HIP_TRY(launch_rb_half<T>(L, psi, C, src, f, mid, omega, first, c->st));
  HIP_TRY(launch_rb_half<T>(L, psi, C, mid, f, u_out, omega, 1 - first, c->st));
  return SBM_OK;
}

extern "C" {

sbm_status sbm_level_sweep(sbm_ctx *c, int l, int first_colour, double omega, const double *u_in,
                           const double *f, double *u_out) {
  return level_sweep<double>(c, l, first_colour, omega, u_in, f, u_out);
}

sbm_status sbm_level_sweep_f32(sbm_ctx *c, int l, int first_colour, double omega,
                               const float *u_in, const float *f, float *u_out) {
  return level_sweep<float>(c, l, first_colour, omega, u_in, f, u_out);
}

sbm_status sbm_level_residual(sbm_ctx *c, int l, const double *u, const double *f, double *r) {
  LEVEL_OK(c, l);
  if (!u || !f || !r) return fail(SBM_E_ARG, "NULL argument");
  NO_ALIAS(u, r);
  NO_ALIAS(f, r);
  Level &L = c->L[l];
  HIP_TRY((launch_residual<double>(L, L.psi64, L.c64, u, f, r, nullptr, c->st)));
  return SBM_OK;
}

sbm_status sbm_level_restrict(sbm_ctx *c, int l, const double *r, double *fc) {
  LEVEL_OK(c, l);
  if (l + 1 >= c->nlev) return fail(SBM_E_ARG, "no coarser level");
  if (!r || !fc) return fail(SBM_E_ARG, "NULL argument");
  NO_ALIAS(r, fc);
  HIP_TRY(launch_restrict<double>(c->L[l], c->L[l + 1], r, fc, c->st));
  return SBM_OK;
}

sbm_status sbm_level_prolong_add(sbm_ctx *c, int l, const double *e, double *u) {
  LEVEL_OK(c, l);
  if (l + 1 >= c->nlev) return fail(SBM_E_ARG, "no coarser level");
  if (!e || !u) return fail(SBM_E_ARG, "NULL argument");
  NO_ALIAS(e, u);
  HIP_TRY(launch_prolong_add<double>(c->L[l], c->L[l + 1], e, u, c->st));
  return SBM_OK;
}

sbm_status sbm_bottom_solve(sbm_ctx *c, const double *f, double *x, int *iters) {
  NEED_PROBLEM(c);
  if (!f || !x) return fail(SBM_E_ARG, "NULL argument");
  NO_ALIAS(f, x);
  HIP_TRY(bottom64(c, f, x));
  HIP_TRY(hipMemcpyAsync(c->host, c->iflag + 4, sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIP_TRY(hipStreamSynchronize(c->st));
  if (iters) memcpy(iters, c->host, sizeof(int));
  return SBM_OK;
}

}  // extern "C"
