// sbm_tiled.hip -- LDS-tiled finest-level stencil sweeps for 3D levels.
//
// A workgroup owns a 64 x 8 node column tile and marches up a chunk of z
// planes.  Three planes of u (all components, with a one-node halo) and two
// planes of cell psi (with halo) live in an LDS ring; the plane two steps
// ahead is fetched into registers while the current plane is computed, so
// every u, psi and f value crosses HBM about once per sweep (plus the halo
// and the two extra planes of each chunk).  Tiles are ordered x, y, z-chunk
// and dealt to the eight XCDs in contiguous ranges (workgroup b runs on XCD
// b mod 8), so neighbouring tiles that share halo rows sit behind the same
// L2.  Outside the box the halo holds zeros: every term that reaches there
// carries a zero psi weight, as in the unclamped form of eq. K.
#include <type_traits>

#include "sbm_internal.h"

namespace sbm {
namespace {

constexpr int kTileWG = 1536;  // target number of workgroups (sets the z-chunk depth)
constexpr int kTileKzMax = 32;

constexpr int TX = kTileX, TY = kTileY;     // interior nodes of a tile
constexpr int LX = TX + 2, LY = TY + 2;     // with the node halo
constexpr int CXL = TX + 1, CYL = TY + 1;   // cells touching the tile's nodes
constexpr int NT = TX / 2 * TY;             // threads: one x-pair per thread
constexpr int PLANE = LY * LX;              // LDS entries per component and plane
constexpr int NU = 3 * PLANE;
constexpr int NUPT = (NU + NT - 1) / NT;

// The level geometry the tiled kernels need (3D only; fewer scalar registers
// than Geom).
struct TG {
  int nx, ny, nz, cx, cy, cz, nn;
  uint32_t dmask;
};

TG make_tg(const Geom &g) { return TG{g.nx, g.ny, g.nz, g.cx, g.cy, g.cz, (int)g.nn, g.dmask}; }

__device__ __forceinline__ bool tg_dirichlet(const TG &g, int i, int j, int k, int comp) {
  const uint32_t m = g.dmask >> comp;
  return ((i == 0) && (m & 1u)) || ((i == g.nx - 1) && ((m >> 3) & 1u)) ||
         ((j == 0) && ((m >> 6) & 1u)) || ((j == g.ny - 1) && ((m >> 9) & 1u)) ||
         ((k == 0) && ((m >> 12) & 1u)) || ((k == g.nz - 1) && ((m >> 15) & 1u));
}

// whole: a launch over the whole level -- the last node column / row of a
// 2^n + 1 level go to node-parallel face blocks, and the z chunks are
// balanced (tile lists and the fused sweep keep whole tiles and fixed-depth
// chunks).  target: the number of tiles a whole-level launch aims at.
TileGeom tile_geom(const TG &g, bool whole = false, int kz_set = 0, int target = kTileWG);

// Whole-level tile targets per kernel, measured at the 257^3 level (128 tile
// columns; isolated launches, balanced chunks of 10 to 24 planes):
//   FP64 half-sweep: 14 chunks (335 us; 12, 16 and 24 chunks 354-360 us --
//     the eight XCDs then start their tile ranges at the same place in a
//     layer of tiles);
//   FP64 sweep from zero (three workgroups per CU): 12 chunks, two full
//     rounds of resident workgroups (342 us; 14 chunks 363 us);
//   FP64 residual and Krylov Apply: 14 chunks (386 and 296 us, within 2 %
//     of the best count);
//   FP32 (half the LDS, more resident workgroups): 16 chunks for all three
//     (200, 228 and 206 us).
enum class TileKind { half, zero, full };
template <typename T>
constexpr int tile_target(TileKind k) {
  return sizeof(T) != 8 ? 2048 : (k == TileKind::zero ? 1536 : 1792);
}

// Planes [k0, k1) of chunk tz.
__device__ __forceinline__ void tile_chunk(const TileGeom &tg, int tz, int nz, int &k0, int &k1) {
  if (tg.nzc > 0) {
    k0 = tz * nz / tg.nzc;
    k1 = (tz + 1) * nz / tg.nzc;
  } else {
    k0 = tz * tg.kz;
    k1 = min(k0 + tg.kz, nz);
  }
}

// Face node f of a launch with face blocks: the last column x = nx-1 (all
// rows) first, then the last row y = ny-1 (the other columns), plane by plane.
__device__ __forceinline__ bool face_node(const TG &g, const TileGeom &tg, int f, int &x, int &y,
                                          int &z) {
  const int per = (tg.xface ? g.ny : 0) + (tg.yface ? g.nx - tg.xface : 0);
  if (f >= per * g.nz) return false;
  z = f / per;
  const int e = f - z * per;
  if (tg.xface && e < g.ny) {
    x = g.nx - 1;
    y = e;
  } else {
    x = e - (tg.xface ? g.ny : 0);
    y = g.ny - 1;
  }
  return true;
}

TileGeom tile_geom(const TG &g, bool whole, int kz_set, int target) {
  TileGeom t;
  t.xface = whole && g.nx > TX && g.nx % TX == 1;
  t.yface = whole && g.ny > TY && g.ny % TY == 1;
  t.ntx = t.xface ? g.nx / TX : (g.nx + TX - 1) / TX;
  t.nty = t.yface ? g.ny / TY : (g.ny + TY - 1) / TY;
  const int64_t per_plane = (t.xface ? g.ny : 0) + (t.yface ? g.nx - t.xface : 0);
  t.nface = (int)((per_plane * g.nz + NT - 1) / NT);
  const int cols = t.ntx * t.nty;
  t.nzc = 0;
  if (whole && kz_set == 0) {
    // about `target` tiles (at the 257^3 level a whole number of rounds of
    // the resident workgroups), each chunk 4 to kTileKzMax planes deep
    int nzc = target / cols;
    nzc = std::min(nzc, g.nz / 4);
    nzc = std::max(nzc, (g.nz + kTileKzMax - 1) / kTileKzMax);
    t.nzc = std::max(nzc, 1);
    t.kz = (g.nz + t.nzc - 1) / t.nzc;
    t.ntiles = cols * t.nzc;
    return t;
  }
  // enough workgroups to fill 256 CUs several times over; each chunk re-reads
  // two planes
  int kz = kz_set > 0 ? kz_set : (int)((int64_t)g.nz * cols / kTileWG);
  kz = kz < 4 ? 4 : (kz > kTileKzMax ? kTileKzMax : kz);
  t.kz = kz;
  t.ntiles = cols * ((g.nz + kz - 1) / kz);
  return t;
}

// ---------------------------------------------------------------- buffers
//
// The tiled kernels address u, f, psi and the outputs through raw buffer
// descriptors: the per-thread byte offset within a plane (a VGPR computed once)
// plus the plane's offset (an SGPR) is added by the memory unit, and an offset
// at or past the buffer's size reads 0 and drops a store.  Halo entries
// outside the box therefore load as the zeros eq. K needs there, with no
// select per value, and a thread without a node stores nothing.  Offsets stay
// below 2^31 (tiled_ok limits a level's vector to that many bytes).
constexpr int kOOB = 0x7ffffff8;    // byte offset past every buffer
constexpr int kRsrcW3 = 0x00020000; // descriptor word 3: 32-bit data format, raw access

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, bytes, kRsrcW3);
}
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
typedef unsigned int u32x2 __attribute__((__vector_size__(2 * sizeof(unsigned int))));
template <typename T>
__device__ __forceinline__ void bstore(T v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  if constexpr (sizeof(T) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}

// ---------------------------------------------------------------- LDS tile
//
// A plane of u holds 3 components x LY rows x LX columns (the tile and its
// one-node halo); a plane of psi CYL rows of the CXL cells under them.  Each
// row is split by parity: the even local columns first, then the odd ones, so
// that the nodes a wave relaxes in one colour (every other column) and their
// x-neighbours (the other parity) sit in consecutive LDS words (no bank
// conflicts).  Local column lx is global x0 - 1 + lx.  Slots are padded to a
// whole number of loads per thread, so every thread stores every load.
constexpr int HUX = LX / 2;                  // columns per parity half (u rows)
constexpr int HCX = (CXL + 1) / 2;           // the same for cell rows
constexpr int CROW = 2 * HCX;                // LDS cell row (one pad entry)
constexpr int NPC = CYL * CROW;             // cell entries per plane
constexpr int NPCT = (NPC + NT - 1) / NT;
constexpr int SLOT_U = NUPT * NT, SLOT_P = NPCT * NT;
static_assert(LX % 2 == 0, "u rows split into two equal halves");

__device__ __forceinline__ int lds_col(int lx, int half) { return (lx & 1) * half + (lx >> 1); }

// Byte offsets (within a plane) of a thread's u and psi load slots, in LDS
// order; kOOB for halo entries outside the box and for padding.
template <int W>
__device__ __forceinline__ void tile_slots(const TG &g, int x0, int y0, int (&vu)[NUPT],
                                           int (&vp)[NPCT]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < NUPT; ++j) {
    const int e = t + j * NT;
    vu[j] = kOOB;
    if (e < NU) {
      const int c = e / PLANE, r = e - c * PLANE;
      const int y = r / LX, xr = r - y * LX;
      const int hf = xr >= HUX ? 1 : 0;
      const int gx = x0 - 1 + 2 * (xr - hf * HUX) + hf, gy = y0 - 1 + y;
      if (gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny) vu[j] = (c * g.nn + gx + g.nx * gy) * W;
    }
  }
#pragma unroll
  for (int j = 0; j < NPCT; ++j) {
    const int e = t + j * NT;
    vp[j] = kOOB;
    if (e < NPC) {
      const int y = e / CROW, xr = e - y * CROW;
      const int hf = xr >= HCX ? 1 : 0;
      const int lx = 2 * (xr - hf * HCX) + hf;
      const int gx = x0 - 1 + lx, gy = y0 - 1 + y;
      if (lx < CXL && gx >= 0 && gx < g.cx && gy >= 0 && gy < g.cy) vp[j] = (gx + g.cx * gy) * W;
    }
  }
}

// The buffers a tiled kernel reads (rnull: an empty buffer, every load 0).
struct TileBufs {
  __amdgpu_buffer_rsrc_t u, f, psi, out, null;
};

template <typename T>
__device__ __forceinline__ void tile_put_u(T *slot, const T (&ru)[NUPT]) {
#pragma unroll
  for (int j = 0; j < NUPT; ++j) slot[threadIdx.x + j * NT] = ru[j];
}
template <typename T>
__device__ __forceinline__ void tile_put_p(T *slot, const T (&rp)[NPCT]) {
#pragma unroll
  for (int j = 0; j < NPCT; ++j) slot[threadIdx.x + j * NT] = rp[j];
}

// Loads of u plane z / cell plane zc into registers (zeros outside the box).
template <typename T>
__device__ __forceinline__ void tile_fetch_u(const TG &g, const TileBufs &B, const int (&vu)[NUPT],
                                             int z, T (&ru)[NUPT]) {
  const bool zin = z >= 0 && z < g.nz;
  const __amdgpu_buffer_rsrc_t r1 = zin ? B.u : B.null;
  const int so = zin ? z * g.nx * g.ny * (int)sizeof(T) : 0;
#pragma unroll
  for (int j = 0; j < NUPT; ++j) ru[j] = bload<T>(r1, vu[j], so);
}
template <typename T>
__device__ __forceinline__ void tile_fetch_p(const TG &g, const TileBufs &B, const int (&vp)[NPCT],
                                             int zc, T (&rp)[NPCT]) {
  const bool zin = zc >= 0 && zc < g.cz;
  const __amdgpu_buffer_rsrc_t r2 = zin ? B.psi : B.null;
  const int sq = zin ? zc * g.cx * g.cy * (int)sizeof(T) : 0;
#pragma unroll
  for (int j = 0; j < NPCT; ++j) rp[j] = bload<T>(r2, vp[j], sq);
}

// The first step's planes: u k0-1..k0+1 and cells k0-1, k0 into their slots.
template <typename T>
__device__ __forceinline__ void tile_prologue(const TG &g, const TileBufs &B,
                                              const int (&vu)[NUPT], const int (&vp)[NPCT],
                                              int k0, T (*su)[SLOT_U], T (*sp)[SLOT_P]) {
  T r0[NUPT], r1[NUPT], r2[NUPT], q0[NPCT], q1[NPCT];
  tile_fetch_u<T>(g, B, vu, k0 - 1, r0);
  tile_fetch_u<T>(g, B, vu, k0, r1);
  tile_fetch_u<T>(g, B, vu, k0 + 1, r2);
  tile_fetch_p<T>(g, B, vp, k0 - 1, q0);
  tile_fetch_p<T>(g, B, vp, k0, q1);
  tile_put_u<T>(su[(k0 + 2) % 3], r0);
  tile_put_u<T>(su[k0 % 3], r1);
  tile_put_u<T>(su[(k0 + 1) % 3], r2);
  tile_put_p<T>(sp[(k0 + 1) & 1], q0);
  tile_put_p<T>(sp[k0 & 1], q1);
}

// eq. K at the node of local column lx (1..TX) and row yl of the tile from the
// LDS planes Lm / L0 / L1 (below, at, above) and the cell planes Pm / P0.
template <typename T, typename CO>
__device__ __forceinline__ void tile_stencil(const CO &C, const T *Lm, const T *L0, const T *L1,
                                             const T *Pm, const T *P0, int lx, int yl, T out[3],
                                             T dg[3]) {
  const int row = (yl + 1) * LX;
  const int cu = row + lds_col(lx, HUX);       // the node
  const int cm = row + lds_col(lx - 1, HUX);   // x - 1
  const int cp = row + lds_col(lx + 1, HUX);   // x + 1
  const int pc0 = lds_col(lx - 1, HCX), pc1 = lds_col(lx, HCX);  // cells i-1, i
  T P[2][2][2];
#pragma unroll
  for (int c1 = 0; c1 < 2; ++c1) {
    P[0][c1][0] = Pm[(yl + c1) * CROW + pc0];
    P[0][c1][1] = Pm[(yl + c1) * CROW + pc1];
    P[1][c1][0] = P0[(yl + c1) * CROW + pc0];
    P[1][c1][1] = P0[(yl + c1) * CROW + pc1];
  }
  auto U = [&](int c, int dx, int dy, int dz) -> T {
    const T *L = dz < 0 ? Lm : (dz > 0 ? L1 : L0);
    return L[c * PLANE + (dx == 0 ? cu : (dx > 0 ? cp : cm)) + dy * LX];
  };
  stencil3<T>(C, P, U, out, dg);
}

// Hardware block b of a launch over n listed (or all) tiles: the tiles first,
// in the XCD-ordered numbering of the first n rounded up to 8 blocks (workgroup
// b runs on XCD b mod 8; each XCD gets a contiguous range of tiles); the face
// blocks of a whole-level launch last (short node-parallel blocks that fill
// the slots the last tiles leave idle).  Returns the logical tile, or -1 - fb
// for face block fb.
__device__ __forceinline__ int tile_or_face(int n) {
  const int n8 = (n + 7) / 8 * 8;
  const int b = blockIdx.x;
  if (b >= n8) return -1 - (b - n8);
  return (b & 7) * (n8 >> 3) + (b >> 3);
}

// The FP64 residual an FP32 half-sweep with DOT reads instead of its load:
// the load is r / s (s = sqrt(*ss)) formed as the mixed cast forms it, and the
// sum is r . (s u_out), the CG's r . z with z = s e.
struct DotSrc {
  const double *r, *ss;
};

// A face node (last column / row of a 2^n + 1 level) of a whole-level tiled
// half-sweep: one node per thread from global memory, the same update.  With
// DOT the block's sum of f . u_out over free DOF goes to partials[ntiles + fb]
// (FP32: r . (s u_out), see DotSrc).
template <typename T, typename CO, bool MASK, bool DOT>
__device__ __forceinline__ void rb_face_node(const TG &g, const CO &C, const T *psi,
                                             const T *u, const T *f, T *u_out, T omega,
                                             int colour, const TileGeom &tg,
                                             const uint8_t *cls, int fb, double *partials,
                                             double *red, const DotSrc &ds) {
  constexpr bool R64 = DOT && sizeof(T) == 4;
  const double sn = R64 ? sqrt(*ds.ss) : 0.0;
  auto fval = [&](int qq) -> T {
    if constexpr (R64) {
      const double r = ds.r[qq];
      return sn > 0.0 ? (T)(r / sn) : T(0);
    } else {
      return f[qq];
    }
  };
  int x, y, z;
  double acc = 0.0;
  if (face_node(g, tg, fb * NT + (int)threadIdx.x, x, y, z)) {
    const int nn = g.nn;
    const int q = x + g.nx * (y + g.ny * z);
    T nv[3];
    if (((x + y + z) & 1) == colour && !(MASK && cls[q] != 1)) {
      T out[3], dg[3], uc[3];
      node_stencil<T, 3, true, TG, CO>(g, C, psi, u, x, y, z, out, dg, uc);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T upd_c = uc[c] + omega * (fval(c * nn + q) - out[c]) / dg[c];
        nv[c] = tg_dirichlet(g, x, y, z, c) ? uc[c] : upd_c;
      }
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) nv[c] = u[c * nn + q];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      u_out[c * nn + q] = nv[c];
      if (DOT && !tg_dirichlet(g, x, y, z, c)) {
        if constexpr (R64) acc += ds.r[c * nn + q] * (sn * (double)nv[c]);
        else acc += (double)f[c * nn + q] * (double)nv[c];
      }
    }
  }
  if constexpr (DOT) {
    const double sum = block_sum(acc, red);
    if (threadIdx.x == 0) partials[tg.ntiles + fb] = sum;
  }
}

// Colour-synchronous Gauss-Seidel half-sweep (nodes with (x+y+z) mod 2 ==
// colour updated from u, the others copied to u_out), as k_rb_half, over the
// tiles and, in a whole-level launch, the face blocks.  With MASK only
// class-1 nodes are updated.  A thread owns an x-pair (one node of each
// colour) and stores both.  The u and psi planes of the next step and f of
// the next plane are loaded while the current plane is computed.  With DOT
// (a whole-level launch) each tile also sums f . u_out over its free DOF --
// r . z of a preconditioned CG whose V-cycle ends with this half-sweep; in
// FP32 r . (s u_out) from the FP64 residual, see DotSrc -- into
// partials[tile], the face blocks into partials[ntiles + face block].
template <typename T, typename CO, bool MASK, bool DOT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_rb_tile(
    TG g, CO C, const T *__restrict__ psi, const T *__restrict__ u, const T *__restrict__ f,
    T *__restrict__ u_out, T omega, int colour, TileGeom tg, const uint8_t *__restrict__ cls,
    const int *__restrict__ ids, int n, double *__restrict__ partials, DotSrc ds) {
  __shared__ T su[3][SLOT_U];
  __shared__ T sp[2][SLOT_P];
  __shared__ double red[DOT ? NT / 64 + 1 : 1];
  const int li = tile_or_face(n);
  if (li < 0) {
    rb_face_node<T, CO, MASK, DOT>(g, C, psi, u, f, u_out, omega, colour, tg, cls, -1 - li,
                                   partials, red, ds);
    return;
  }
  if (li >= n) return;
  const int lt = ids ? ids[li] : li;
  constexpr int W = sizeof(T);
  const int nn = g.nn, nxy = g.nx * g.ny;
  const int vbytes = 3 * nn * W;
  const TileBufs B{make_rsrc(u, vbytes), make_rsrc(f, vbytes), make_rsrc(psi, g.cx * g.cy * g.cz * W),
                   make_rsrc(u_out, vbytes), make_rsrc(u, 0)};
  const int tx = lt % tg.ntx, rest = lt / tg.ntx;
  const int ty = rest % tg.nty, tz = rest / tg.nty;
  const int x0 = tx * TX, y0 = ty * TY;
  int k0, k1;
  tile_chunk(tg, tz, g.nz, k0, k1);
  int vu[NUPT], vp[NPCT];
  tile_slots<W>(g, x0, y0, vu, vp);
  const int yl = threadIdx.x / (TX / 2), p = threadIdx.x % (TX / 2);
  const int gy = y0 + yl;
  // byte offsets (in a plane) of the thread's two nodes, columns x0+2p and x0+2p+1
  const int vn0 = (gy < g.ny && x0 + 2 * p < g.nx) ? (gy * g.nx + x0 + 2 * p) * W : kOOB;
  const int vn1 = (gy < g.ny && x0 + 2 * p + 1 < g.nx) ? (gy * g.nx + x0 + 2 * p + 1) * W : kOOB;
  const int pg = (colour + gy) & 1;  // the updated column of plane k is x0 + 2p + ((pg + k) & 1)
  // f at the updated node of plane k (zeros past the chunk; with DOT also at
  // the copied node; an FP32 DOT sweep loads the FP64 residual instead, see
  // DotSrc)
  constexpr bool R64 = DOT && sizeof(T) == 4;
  using FT = std::conditional_t<R64, double, T>;
  const __amdgpu_buffer_rsrc_t rr = make_rsrc(R64 ? (const void *)ds.r : (const void *)f,
                                              R64 ? 3 * nn * 8 : vbytes);
  const int fw = R64 ? 8 / W : 1;  // FP64 offsets from FP32 ones
  const double sn = R64 ? sqrt(*ds.ss) : 0.0;
  auto fetch_f = [&](int k, FT (&r)[3], FT (&rc)[3]) __attribute__((always_inline)) {
    const bool ok = k < k1;
    const __amdgpu_buffer_rsrc_t rf = ok ? (R64 ? rr : B.f) : B.null;
    const int vo = ((pg + k) & 1) ? vn1 : vn0;
    const int so = ok ? k * nxy * W * fw : 0;
    const int vof = vo == kOOB ? kOOB : vo * fw;
#pragma unroll
    for (int c = 0; c < 3; ++c) r[c] = bload<FT>(rf, vof, so + (ok ? c * nn * W * fw : 0));
    if constexpr (DOT) {
      const int vc = ((pg + k) & 1) ? vn0 : vn1;
      const int vcf = vc == kOOB ? kOOB : vc * fw;
#pragma unroll
      for (int c = 0; c < 3; ++c) rc[c] = bload<FT>(rf, vcf, so + (ok ? c * nn * W * fw : 0));
    }
  };
  // MASK: the class of the updated node of plane k, loaded a plane ahead too
  auto fetch_cls = [&](int k) __attribute__((always_inline)) -> int {
    if constexpr (MASK) {
      const int gx = x0 + 2 * p + ((pg + k) & 1);
      return (k < k1 && gy < g.ny && gx < g.nx) ? (int)cls[k * nxy + gy * g.nx + gx] : 0;
    } else {
      return 0;
    }
  };
  FT FN[3], FC[3];
  fetch_f(k0, FN, FC);
  int CLN = fetch_cls(k0);
  tile_prologue<T>(g, B, vu, vp, k0, su, sp);
  __syncthreads();
  double acc = 0.0;
  T RU[NUPT], RP[NPCT];
  for (int k = k0; k < k1; ++k) {
    const int clk = CLN;
    CLN = fetch_cls(k + 1);
    T fv[3];
    FT fc[3], fr[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if constexpr (R64) {
        fr[c] = FN[c];
        fv[c] = sn > 0.0 ? (T)(FN[c] / sn) : T(0);
      } else {
        fv[c] = FN[c];
      }
      if (DOT) fc[c] = FC[c];
    }
    fetch_f(k + 1, FN, FC);
    tile_fetch_u<T>(g, B, vu, k + 2, RU);
    tile_fetch_p<T>(g, B, vp, k + 1, RP);
    const T *Lm = su[(k + 2) % 3], *L0 = su[k % 3], *L1 = su[(k + 1) % 3];
    const T *Pm = sp[(k + 1) & 1], *P0 = sp[k & 1];
    const int par = (pg + k) & 1;
    const int xu = 2 * p + par, gxu = x0 + xu;  // updated node; the copied one is xu +- 1
    const int lx = xu + 1;
    const int cu = (yl + 1) * LX + lds_col(lx, HUX);
    const int cc = (yl + 1) * LX + lds_col(par ? lx - 1 : lx + 1, HUX);
    const int so = k * nxy * W;
    T nv[3];
    bool upd = gy < g.ny && gxu < g.nx;
    if (MASK && upd) upd = clk == 1;
    if (upd) {
      T out[3], dg[3];
      tile_stencil<T>(C, Lm, L0, L1, Pm, P0, lx, yl, out, dg);
      // displacement DOF only exist on the box faces
      const bool face = gxu == 0 || gxu == g.nx - 1 || gy == 0 || gy == g.ny - 1 || k == 0 ||
                        k == g.nz - 1;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T uc = L0[c * PLANE + cu];
        const T upd_c = uc + omega * (fv[c] - out[c]) / dg[c];
        nv[c] = (face && tg_dirichlet(g, gxu, gy, k, c)) ? uc : upd_c;
      }
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) nv[c] = L0[c * PLANE + cu];
    }
    const int vo_u = par ? vn1 : vn0, vo_c = par ? vn0 : vn1;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      bstore<T>(nv[c], B.out, vo_u, so + c * nn * W);
      bstore<T>(L0[c * PLANE + cc], B.out, vo_c, so + c * nn * W);
    }
    if constexpr (DOT) {
      // f . u_out at both nodes (f reads 0 at a node outside the box)
      const int gxc = par ? gxu - 1 : gxu + 1;
      const bool fy = gy == 0 || gy == g.ny - 1 || k == 0 || k == g.nz - 1;
      const bool fu = fy || gxu == 0 || gxu == g.nx - 1, fcn = fy || gxc == 0 || gxc == g.nx - 1;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if constexpr (R64) {
          if (!(fu && tg_dirichlet(g, gxu, gy, k, c))) acc += fr[c] * (sn * (double)nv[c]);
          if (!(fcn && tg_dirichlet(g, gxc, gy, k, c)))
            acc += fc[c] * (sn * (double)L0[c * PLANE + cc]);
        } else {
          if (!(fu && tg_dirichlet(g, gxu, gy, k, c))) acc += (double)fv[c] * (double)nv[c];
          if (!(fcn && tg_dirichlet(g, gxc, gy, k, c)))
            acc += (double)fc[c] * (double)L0[c * PLANE + cc];
        }
      }
    }
    __syncthreads();
    // the planes of the next step go to the slots of planes k - 1 (u, cells)
    tile_put_u<T>(su[(k + 2) % 3], RU);
    tile_put_p<T>(sp[(k + 1) & 1], RP);
    __syncthreads();
  }
  if constexpr (DOT) {
    const double sum = block_sum(acc, red);
    if (threadIdx.x == 0) partials[li] = sum;
  }
}

// A face block of a whole-level k_full_tile pass: one node per thread, the
// block's sum in partials[ntiles + fb].
template <typename T, typename CO, int MODE, bool MASK>
__device__ __forceinline__ void full_face_block(const TG &g, const CO &C, const T *psi, const T *u,
                                                const T *f, T *r, double *partials,
                                                const TileGeom &tg, const uint8_t *cls, int fb,
                                                double *red) {
  const int nn = g.nn;
  double acc = 0.0;
  int x, y, z;
  if (face_node(g, tg, fb * NT + (int)threadIdx.x, x, y, z)) {
    const int q = x + g.nx * (y + g.ny * z);
    T v[3] = {T(0), T(0), T(0)};
    if (!(MASK && (cls[q] == 0 || cls[q] > 3))) {
      T out[3], dg[3], uc[3];
      node_stencil<T, 3, true, TG, CO>(g, C, psi, u, x, y, z, out, dg, uc);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T val = MODE == 0 ? f[c * nn + q] - out[c] : out[c];
        v[c] = tg_dirichlet(g, x, y, z, c) ? T(0) : val;
        if (MODE == 0) acc += (double)v[c] * (double)v[c];
        else acc += (double)uc[c] * (double)v[c];
      }
    }
    if (r)
#pragma unroll
      for (int c = 0; c < 3; ++c) r[c * nn + q] = v[c];
  }
  if (partials) {
    const double sum = block_sum(acc, red);
    if (threadIdx.x == 0) partials[tg.ntiles + fb] = sum;
  }
}

// Full stencil pass over the tiles (every node computed), thread per x-pair:
//   MODE 0 (residual): v = f - K u on free DOF, 0 on displacement DOF (and,
//     with MASK, outside classes 1-3); r = v when r is given; partial sum of
//     v^2 per tile when partials is given;
//   MODE 1 (Krylov Apply): v = K u on free DOF, 0 on displacement DOF; r = v;
//     partial sum of u . v per tile.
// Partials land in partials[tile], tiles in their logical order, then one per
// face block (partials[ntiles + face block]).
template <typename T, typename CO, int MODE, bool MASK>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_full_tile(
    TG g, CO C, const T *__restrict__ psi, const T *__restrict__ u, const T *__restrict__ f,
    T *__restrict__ r, double *__restrict__ partials, TileGeom tg,
    const uint8_t *__restrict__ cls, const int *__restrict__ ids, int n) {
  __shared__ T su[3][SLOT_U];
  __shared__ T sp[2][SLOT_P];
  __shared__ double red[NT / 64 + 1];
  const int li = tile_or_face(n);
  if (li < 0) {
    full_face_block<T, CO, MODE, MASK>(g, C, psi, u, f, r, partials, tg, cls, -1 - li, red);
    return;
  }
  if (li >= n) return;
  const int lt = ids ? ids[li] : li;
  constexpr int W = sizeof(T);
  const int nn = g.nn, nxy = g.nx * g.ny;
  const int vbytes = 3 * nn * W;
  const TileBufs B{make_rsrc(u, vbytes), make_rsrc(f, MODE == 0 ? vbytes : 0),
                   make_rsrc(psi, g.cx * g.cy * g.cz * W), make_rsrc(r, r ? vbytes : 0),
                   make_rsrc(u, 0)};
  const int tx = lt % tg.ntx, rest = lt / tg.ntx;
  const int ty = rest % tg.nty, tz = rest / tg.nty;
  const int x0 = tx * TX, y0 = ty * TY;
  int k0, k1;
  tile_chunk(tg, tz, g.nz, k0, k1);
  int vu[NUPT], vp[NPCT];
  tile_slots<W>(g, x0, y0, vu, vp);
  const int yl = threadIdx.x / (TX / 2), p = threadIdx.x % (TX / 2);
  const int gy = y0 + yl;
  const int gx0 = x0 + 2 * p;  // the pair: gx0, gx0 + 1
  const int vn[2] = {(gy < g.ny && gx0 < g.nx) ? (gy * g.nx + gx0) * W : kOOB,
                     (gy < g.ny && gx0 + 1 < g.nx) ? (gy * g.nx + gx0 + 1) * W : kOOB};
  // f of both nodes, one plane ahead
  auto fetch_f = [&](int k, T (&fr)[2][3]) __attribute__((always_inline)) {
    const bool ok = MODE == 0 && k < k1;
    const __amdgpu_buffer_rsrc_t rf = ok ? B.f : B.null;
    const int so = ok ? k * nxy * W : 0;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c = 0; c < 3; ++c) fr[h][c] = bload<T>(rf, vn[h], so + (ok ? c * nn * W : 0));
  };
  // MASK: the classes of both nodes of plane k, loaded a plane ahead too
  auto fetch_cls = [&](int k, int (&cl)[2]) __attribute__((always_inline)) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      cl[h] = 0;
      if constexpr (MASK) {
        const int gx = gx0 + h;
        if (k < k1 && gy < g.ny && gx < g.nx) cl[h] = cls[k * nxy + gy * g.nx + gx];
      }
    }
  };
  T FN[2][3];
  fetch_f(k0, FN);
  int CLN[2];
  fetch_cls(k0, CLN);
  tile_prologue<T>(g, B, vu, vp, k0, su, sp);
  __syncthreads();
  double acc = 0.0;
  T RU[NUPT], RP[NPCT];
  for (int k = k0; k < k1; ++k) {
    T fv[2][3];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c = 0; c < 3; ++c) fv[h][c] = FN[h][c];
    fetch_f(k + 1, FN);
    const int clk[2] = {CLN[0], CLN[1]};
    fetch_cls(k + 1, CLN);
    tile_fetch_u<T>(g, B, vu, k + 2, RU);
    tile_fetch_p<T>(g, B, vp, k + 1, RP);
    const T *Lm = su[(k + 2) % 3], *L0 = su[k % 3], *L1 = su[(k + 1) % 3];
    const T *Pm = sp[(k + 1) & 1], *P0 = sp[k & 1];
    const int so = k * nxy * W;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int gx = gx0 + h, lx = 2 * p + h + 1;
      T v[3] = {T(0), T(0), T(0)};
      bool live = gy < g.ny && gx < g.nx;
      if (MASK && live) {
        const int cl = clk[h];
        live = cl != 0 && cl <= 3;
      }
      if (live) {
        T out[3], dg[3];
        tile_stencil<T>(C, Lm, L0, L1, Pm, P0, lx, yl, out, dg);
        const bool face = gx == 0 || gx == g.nx - 1 || gy == 0 || gy == g.ny - 1 || k == 0 ||
                          k == g.nz - 1;
        const int cu = (yl + 1) * LX + lds_col(lx, HUX);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const bool fixed = face && tg_dirichlet(g, gx, gy, k, c);
          const T val = MODE == 0 ? fv[h][c] - out[c] : out[c];
          v[c] = fixed ? T(0) : val;
          if (MODE == 0) acc += (double)v[c] * (double)v[c];
          else acc += (double)L0[c * PLANE + cu] * (double)v[c];
        }
      }
      if (r)
#pragma unroll
        for (int c = 0; c < 3; ++c) bstore<T>(v[c], B.out, vn[h], so + c * nn * W);
    }
    __syncthreads();
    tile_put_u<T>(su[(k + 2) % 3], RU);
    tile_put_p<T>(sp[(k + 1) & 1], RP);
    __syncthreads();
  }
  if (partials) {
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partials[li] = s;
  }
}

// Tiles holding any node of class 1 .. cmax (one workgroup per tile).
__global__ __launch_bounds__(256) void k_tile_flags(TG g, TileGeom tg,
                                                    const uint8_t *__restrict__ cls, int cmax,
                                                    int *__restrict__ flags) {
  const int t = blockIdx.x;
  const int tx = t % tg.ntx, rest = t / tg.ntx, ty = rest % tg.nty, tz = rest / tg.nty;
  const int x0 = tx * TX, y0 = ty * TY;
  int k0, k1;
  tile_chunk(tg, tz, g.nz, k0, k1);
  int any = 0;
  const int n = TX * TY * (k1 - k0);
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int x = x0 + e % TX, y = y0 + (e / TX) % TY, k = k0 + e / (TX * TY);
    if (x < g.nx && y < g.ny) {
      const int cl = cls[x + g.nx * (y + g.ny * k)];
      if (cl >= 1 && cl <= cmax) any = 1;
    }
  }
  any = __syncthreads_or(any);
  if (threadIdx.x == 0) flags[t] = any;
}

// Ids of the flagged tiles in increasing order and their number (one
// workgroup: per-thread chunk counts, an exclusive scan in LDS, then writes).
__global__ __launch_bounds__(1024) void k_tile_compact(const int *__restrict__ flags, int n,
                                                       int *__restrict__ ids,
                                                       int *__restrict__ count) {
  __shared__ int off[1024];
  const int t = threadIdx.x;
  const int chunk = (n + 1023) / 1024;
  const int lo = min(n, t * chunk), hi = min(n, lo + chunk);
  int c = 0;
  for (int i = lo; i < hi; ++i) c += flags[i] ? 1 : 0;
  off[t] = c;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {  // inclusive scan
    const int v = t >= d ? off[t - d] : 0;
    __syncthreads();
    off[t] += v;
    __syncthreads();
  }
  int w = off[t] - c;
  for (int i = lo; i < hi; ++i)
    if (flags[i]) ids[w++] = i;
  if (t == 1023) *count = off[1023];
}


// ------------------------------------------------- fused two-colour sweep
//
// One launch makes a whole Gauss-Seidel sweep (Sec. 2.3): the half-sweep of
// the first colour A from u, then the half-sweep of the second colour B from
// that intermediate state, each colour-synchronous (every node of a colour
// relaxed from the state at the start of its half-sweep), as two k_rb_tile
// launches would.  The tile marches up its chunk with B one plane behind A:
// at step k it relaxes A on plane k from the old planes k-1..k+1, then B on
// plane k-1 from the intermediate planes k-2..k.  B on the tile's edge nodes
// reads A values of the edge nodes of the neighbouring tiles, so A is also
// relaxed on the ring of nodes around the tile (the old state is held with a
// two-node halo for that); an A value depends on the old state alone, so the
// neighbour computes the same value bit for bit.  A chunk relaxes A on one
// plane below and one plane above its own for the same reason.
//
// LDS (FP64): three old planes with the two-node halo (58.8 KB), three
// intermediate planes with the one-node halo (47.5 KB) and four cell planes
// (23.6 KB): 130 KB, one workgroup per CU (FP32: half, two).  Each step
// fetches the old plane and the cell plane it stores one step later, and the
// loads of f two steps before their use, so that about two planes of loads
// are in flight per workgroup.  ZERO: u is zero on entry (the first sweep of
// a V-cycle from zero); no old state is read and A is omega f / D.
constexpr int FX = TX + 4, FY = TY + 4, FPL = FX * FY;  // old u, two-node halo
constexpr int HX = TX + 2, HY = TY + 2, HPL = HX * HY;  // intermediate state, one-node halo
constexpr int QX = TX + 3, QY = TY + 3, QPL = QX * QY;  // cells under the intermediate region
constexpr int NRING = 2 * HX + 2 * TY;                  // ring nodes of the intermediate region
constexpr int NRA = TX + TY;                            // of them colour A, corners excluded
constexpr int FU = (3 * FPL + NT - 1) / NT;             // old-u load slots per thread
constexpr int FQ = (QPL + NT - 1) / NT;                 // cell load slots per thread
static_assert(NRING <= NT && NRA <= NT, "ring work needs one thread per ring node");

struct FSlots {
  int u[FU];
  int q[FQ];
};

__device__ __forceinline__ void make_fslots(const TG &g, int x0, int y0, FSlots &s) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < FU; ++i) {
    const int e = t + i * NT;
    s.u[i] = -1;
    if (e < 3 * FPL) {
      const int c = e / FPL, r = e - c * FPL;
      const int y = r / FX, x = r - y * FX;
      const int gx = x0 - 2 + x, gy = y0 - 2 + y;
      if (gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny) s.u[i] = c * g.nn + gx + g.nx * gy;
    }
  }
#pragma unroll
  for (int i = 0; i < FQ; ++i) {
    const int e = t + i * NT;
    s.q[i] = -1;
    if (e < QPL) {
      const int y = e / QX, x = e - y * QX;
      const int gx = x0 - 2 + x, gy = y0 - 2 + y;
      if (gx >= 0 && gx < g.cx && gy >= 0 && gy < g.cy) s.q[i] = gx + g.cx * gy;
    }
  }
}

// A plane of old u and a plane of cells in registers (loads in flight).
template <typename T, bool ZERO>
struct PlaneRegs {
  T u[ZERO ? 1 : FU];
  T q[FQ];
};

// Loads of old-u plane ku and cell plane kq; out-of-box entries load
// element 0 (in range) and are replaced by zeros only when stored.
template <typename T, bool ZERO>
__device__ __forceinline__ void fetch_planes(const TG &g, const FSlots &s, const T *__restrict__ u,
                                             const T *__restrict__ psi, int ku, int kq,
                                             PlaneRegs<T, ZERO> &r) {
  if constexpr (!ZERO) {
    const int zo = (ku >= 0 && ku < g.nz) ? ku * g.nx * g.ny : 0;
#pragma unroll
    for (int i = 0; i < FU; ++i) r.u[i] = u[s.u[i] >= 0 ? s.u[i] + zo : 0];
  }
  const int zq = (kq >= 0 && kq < g.cz) ? kq * g.cx * g.cy : 0;
#pragma unroll
  for (int i = 0; i < FQ; ++i) r.q[i] = psi[s.q[i] >= 0 ? s.q[i] + zq : 0];
}

template <typename T, bool ZERO>
__device__ __forceinline__ void store_planes(const TG &g, const FSlots &s, int ku, int kq, T *so,
                                             T *sq, const PlaneRegs<T, ZERO> &r) {
  if constexpr (!ZERO) {
    const bool kin = ku >= 0 && ku < g.nz;
#pragma unroll
    for (int i = 0; i < FU; ++i) {
      const int e = threadIdx.x + i * NT;
      if (e < 3 * FPL) so[e] = (kin && s.u[i] >= 0) ? r.u[i] : T(0);
    }
  }
  const bool qin = kq >= 0 && kq < g.cz;
#pragma unroll
  for (int i = 0; i < FQ; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e < QPL) sq[e] = (qin && s.q[i] >= 0) ? r.q[i] : T(0);
  }
}

// The loads of f one step needs: a = f at the thread's A node of plane k,
// b = f at its B node of plane k-1 (the same column), r = f at the thread's
// ring A node of plane k (threads below NRA).
template <typename T>
struct FRegs {
  T a[3], b[3], r[3];
};

// Ring A node `r` (< NRA) of plane k: the ring rows first, then the ring
// columns; corners are never needed by B.  x0 and y0 are even.  (Written
// with selects only: branches that assign x in one arm and y in the other
// made the compiler keep the pair in scratch memory.)
struct XY {
  int x, y;
};
__device__ __forceinline__ XY ring_a_node(int r, int x0, int y0, int k, int c0) {
  const bool row = r < TX;
  const bool lo = row ? r < TX / 2 : r < TX + TY / 2;
  const int j = row ? (lo ? r : r - TX / 2) : (lo ? r - TX : r - TX - TY / 2);
  const int fixed = row ? (lo ? y0 - 1 : y0 + TY) : (lo ? x0 - 1 : x0 + TX);
  const int run = (row ? x0 : y0) + 2 * j + ((c0 + fixed + k) & 1);
  return XY{row ? run : fixed, row ? fixed : run};
}

template <typename T>
__device__ __forceinline__ void fetch_f(const TG &g, const T *__restrict__ f, int k, int x0, int y0,
                                        int p, int gy, int c0, FRegs<T> &F) {
  const int nxy = g.nx * g.ny;
  const int xa = x0 + 2 * p + ((c0 + gy + k) & 1);
  const bool col = gy < g.ny && xa < g.nx;
  const int qa = (col && k >= 0 && k < g.nz) ? gy * g.nx + k * nxy + xa : 0;
  const int qb = (col && k >= 1 && k <= g.nz) ? gy * g.nx + (k - 1) * nxy + xa : 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) F.a[c] = f[c * g.nn + qa];
#pragma unroll
  for (int c = 0; c < 3; ++c) F.b[c] = f[c * g.nn + qb];
  // every thread loads (threads past NRA load element 0): with loads under a
  // branch the compiler's wait counting must assume none were issued and
  // waits for every older load at the next use
  const XY n = ring_a_node(min((int)threadIdx.x, NRA - 1), x0, y0, k, c0);
  const bool in = (int)threadIdx.x < NRA && n.x >= 0 && n.x < g.nx && n.y >= 0 && n.y < g.ny &&
                  k >= 0 && k < g.nz;
  const int qr = in ? n.y * g.nx + k * nxy + n.x : 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) F.r[c] = f[c * g.nn + qr];
}

// eq. K and the diagonal at a node from LDS planes Lm / L0 / L1 (below, at,
// above; S entries per component, row pitch W, the node at index ci) and
// the cell planes Pm / P0 below and above it (row pitch QX, cell (i-1, j-1)
// at index qi).
template <typename T, int S, int W>
__device__ __forceinline__ void lds_stencil(const Coef<T> &C, const T *Lm, const T *L0,
                                            const T *L1, int ci, const T *Pm, const T *P0, int qi,
                                            T out[3], T dg[3]) {
  T P[2][2][2];
#pragma unroll
  for (int c1 = 0; c1 < 2; ++c1)
#pragma unroll
    for (int c0 = 0; c0 < 2; ++c0) {
      P[0][c1][c0] = Pm[qi + c1 * QX + c0];
      P[1][c1][c0] = P0[qi + c1 * QX + c0];
    }
  auto U = [&](int c, int dx, int dy, int dz) -> T {
    const T *L = dz < 0 ? Lm : (dz > 0 ? L1 : L0);
    return L[c * S + ci + dx + dy * W];
  };
  stencil3<T>(C, P, U, out, dg);
}

// The diagonal alone (the same sums as stencil3).
template <typename T>
__device__ __forceinline__ void lds_diag(const Coef<T> &C, const T *Pm, const T *P0, int qi,
                                         T dg[3]) {
  T P[2][2][2];
#pragma unroll
  for (int c1 = 0; c1 < 2; ++c1)
#pragma unroll
    for (int c0 = 0; c0 < 2; ++c0) {
      P[0][c1][c0] = Pm[qi + c1 * QX + c0];
      P[1][c1][c0] = P0[qi + c1 * QX + c0];
    }
  T E[3][2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    E[0][s] = P[0][0][s] + P[0][1][s] + P[1][0][s] + P[1][1][s];
    E[1][s] = P[0][s][0] + P[0][s][1] + P[1][s][0] + P[1][s][1];
    E[2][s] = P[s][0][0] + P[s][0][1] + P[s][1][0] + P[s][1][1];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
    dg[c] = C.cd[c][0] * (E[0][0] + E[0][1]) + C.cd[c][1] * (E[1][0] + E[1][1]) +
            C.cd[c][2] * (E[2][0] + E[2][1]);
}

template <typename T, bool ZERO>
__global__ __launch_bounds__(NT) void k_rb_fused(TG g, Coef<T> C, const T *__restrict__ psi,
                                                 const T *__restrict__ u, const T *__restrict__ f,
                                                 T *__restrict__ u_out, T omega, int c0,
                                                 TileGeom tg) {
  __shared__ T so[ZERO ? 1 : 3][ZERO ? 1 : 3 * FPL];  // old u, planes k-1, k, k+1
  __shared__ T sa[3][3 * HPL];                         // intermediate, planes k-2, k-1, k
  __shared__ T sq[4][QPL];                             // cells, planes k-2 .. k+1
  const int nwg = gridDim.x;  // a multiple of 8
  const int b = blockIdx.x;
  const int li = (b & 7) * (nwg >> 3) + (b >> 3);
  if (li >= tg.ntiles) return;
  const int tx = li % tg.ntx;
  const int rest = li / tg.ntx;
  const int ty = rest % tg.nty;
  const int tz = rest / tg.nty;
  const int x0 = tx * TX, y0 = ty * TY;
  int k0, k1;
  tile_chunk(tg, tz, g.nz, k0, k1);
  const int nn = g.nn, nxy = g.nx * g.ny;
  const int t = threadIdx.x;
  const int yl = t / (TX / 2), p = t % (TX / 2);
  const int gy = y0 + yl;
  const bool row_ok = gy < g.ny;
  // ring slots: the planes k-2..k+1 live at k mod 3 (u, intermediate) and
  // k mod 4 (cells); k >= -2 here
  auto s3 = [](int k) { return (k + 6) % 3; };
  auto s4 = [](int k) { return (k + 8) & 3; };

  FSlots sl;
  make_fslots(g, x0, y0, sl);

  // f of the first two steps, then the prologue planes: old u k0-2..k0 and
  // cells k0-2, k0-1 straight to LDS, old u k0+1 and cells k0 in registers
  // (stored during the first step)
  FRegs<T> FA, FB;
  fetch_f(g, f, k0 - 1, x0, y0, p, gy, c0, FA);
  fetch_f(g, f, k0, x0, y0, p, gy, c0, FB);
  PlaneRegs<T, ZERO> RA, RB;
  {
    PlaneRegs<T, ZERO> r0, r1, r2;
    fetch_planes<T, ZERO>(g, sl, u, psi, k0 - 2, k0 - 2, r0);
    fetch_planes<T, ZERO>(g, sl, u, psi, k0 - 1, k0 - 1, r1);
    fetch_planes<T, ZERO>(g, sl, u, psi, k0, k0, r2);
    fetch_planes<T, ZERO>(g, sl, u, psi, k0 + 1, k0, RB);
    store_planes<T, ZERO>(g, sl, k0 - 2, k0 - 2, so[ZERO ? 0 : s3(k0 - 2)], sq[s4(k0 - 2)], r0);
    store_planes<T, ZERO>(g, sl, k0 - 1, k0 - 1, so[ZERO ? 0 : s3(k0 - 1)], sq[s4(k0 - 1)], r1);
    store_planes<T, ZERO>(g, sl, k0, k0, so[ZERO ? 0 : s3(k0)], sq[s4(k0)], r2);
  }
  __syncthreads();

  // One step: A on plane k (interior and ring), then B on plane k-1 with the
  // store of the planes fetched a step earlier (`st`), while `is` receives the
  // next ones; `fr` holds this step's f and receives the f of step k+2.
  auto step = [&](int k, PlaneRegs<T, ZERO> &is, PlaneRegs<T, ZERO> &st,
                  FRegs<T> &fr) __attribute__((always_inline)) {
    T fa[3], fb[3], frr[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      fa[c] = fr.a[c];
      fb[c] = fr.b[c];
      frr[c] = fr.r[c];
    }
    // unconditional (planes past the chunk load in-range dummies): the loads
    // of a step are then always the same, and the waits for them exact
    fetch_f(g, f, k + 2, x0, y0, p, gy, c0, fr);
    fetch_planes<T, ZERO>(g, sl, u, psi, k + 3, k + 2, is);

    // ---- A on plane k -> sa[k]
    T *H = sa[s3(k)];
    const int par = (c0 + gy + k) & 1;
    const int xa = 2 * p + par, xb = 2 * p + 1 - par;  // tile-local columns
    if (k >= 0 && k < g.nz) {
      const T *Om = so[ZERO ? 0 : s3(k - 1)], *O0 = so[ZERO ? 0 : s3(k)],
              *O1 = so[ZERO ? 0 : s3(k + 1)];
      const T *Qm = sq[s4(k - 1)], *Q0 = sq[s4(k)];
      auto relax_a = [&](int gx, int gyy, const T *fv, T va[3]) __attribute__((always_inline)) {
        const int lx = gx - x0 + 2, ly = gyy - y0 + 2;
        const int qi = (ly - 1) * QX + lx - 1;
        const bool face = gx == 0 || gx == g.nx - 1 || gyy == 0 || gyy == g.ny - 1 || k == 0 ||
                          k == g.nz - 1;
        T out[3], dg[3];
        if constexpr (ZERO) {
          lds_diag<T>(C, Qm, Q0, qi, dg);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const T upd = T(0) + omega * (fv[c] - T(0)) / dg[c];
            va[c] = (face && tg_dirichlet(g, gx, gyy, k, c)) ? T(0) : upd;
          }
        } else {
          const int ci = ly * FX + lx;
          lds_stencil<T, FPL, FX>(C, Om, O0, O1, ci, Qm, Q0, qi, out, dg);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const T uc = O0[c * FPL + ci];
            const T upd = uc + omega * (fv[c] - out[c]) / dg[c];
            va[c] = (face && tg_dirichlet(g, gx, gyy, k, c)) ? uc : upd;
          }
        }
      };
      // interior pair: A relaxed, B copied (zeros outside the box)
      {
        const int gxa = x0 + xa, gxb = x0 + xb;
        T va[3] = {T(0), T(0), T(0)};
        if (row_ok && gxa < g.nx) relax_a(gxa, gy, fa, va);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          H[c * HPL + (yl + 1) * HX + xa + 1] = va[c];
          T vb = T(0);
          if constexpr (!ZERO) vb = O0[c * FPL + (yl + 2) * FX + xb + 2];
          H[c * HPL + (yl + 1) * HX + xb + 1] = (row_ok && gxb < g.nx) ? vb : T(0);
        }
      }
      // ring: B nodes and corners copied, nodes outside the box zeroed
      if (t < NRING) {
        const bool row = t < 2 * HX;
        const bool lo = row ? t < HX : t < 2 * HX + TY;
        const int j = row ? (lo ? t : t - HX) : (lo ? t - 2 * HX : t - 2 * HX - TY);
        const int fixed = row ? (lo ? y0 - 1 : y0 + TY) : (lo ? x0 - 1 : x0 + TX);
        const int run = row ? x0 - 1 + j : y0 + j;
        const int x = row ? run : fixed, y = row ? fixed : run;
        const bool in = x >= 0 && x < g.nx && y >= 0 && y < g.ny;
        const bool corner = t == 0 || t == HX - 1 || t == HX || t == 2 * HX - 1;
        const bool isa = ((x + y + k) & 1) == c0;
        const int hi = (y - y0 + 1) * HX + (x - x0 + 1);
        if (!in) {
#pragma unroll
          for (int c = 0; c < 3; ++c) H[c * HPL + hi] = T(0);
        } else if (!isa || corner) {
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            T v = T(0);
            if constexpr (!ZERO) v = O0[c * FPL + (y - y0 + 2) * FX + (x - x0 + 2)];
            H[c * HPL + hi] = v;
          }
        }
      }
      // ring A nodes inside the box
      if (t < NRA) {
        const XY n = ring_a_node(t, x0, y0, k, c0);
        const int x = n.x, y = n.y;
        if (x >= 0 && x < g.nx && y >= 0 && y < g.ny) {
          T va[3];
          relax_a(x, y, frr, va);
          const int hi = (y - y0 + 1) * HX + (x - x0 + 1);
#pragma unroll
          for (int c = 0; c < 3; ++c) H[c * HPL + hi] = va[c];
        }
      }
    } else {
      // a plane outside the box: zeros
      for (int e = t; e < 3 * HPL; e += NT) H[e] = T(0);
    }
    __syncthreads();

    // the planes fetched a step earlier (old u k+2, cells k+1) go to the slots
    // round A has just released, before any store to global memory (so that
    // waiting for them never waits for a store)
    store_planes<T, ZERO>(g, sl, k + 2, k + 1, so[ZERO ? 0 : s3(k + 2)], sq[s4(k + 1)], st);

    // ---- B on plane k-1 (this chunk's planes only) and the output of plane k-1
    if (k - 1 >= k0) {
      const int kb = k - 1;
      const T *Hm = sa[s3(k - 2)], *H0 = sa[s3(k - 1)], *H1 = sa[s3(k)];
      const T *Qm = sq[s4(k - 2)], *Q0 = sq[s4(k - 1)];
      if (row_ok) {
        const int gxb = x0 + xa;       // B node of plane k-1: the column of A on plane k
        const int gxo = x0 + xb;       // A node of plane k-1 (relaxed at the previous step)
        const int row = gy * g.nx + kb * nxy;
        T vb[3] = {T(0), T(0), T(0)};
        if (gxb < g.nx) {
          const int lx = xa + 1, ly = yl + 1;
          const int ci = ly * HX + lx;
          const int qi = ly * QX + lx;  // cell (i-1, j-1): rows/columns shifted by one
          T out[3], dg[3];
          lds_stencil<T, HPL, HX>(C, Hm, H0, H1, ci, Qm, Q0, qi, out, dg);
          const bool face = gxb == 0 || gxb == g.nx - 1 || gy == 0 || gy == g.ny - 1 ||
                            kb == 0 || kb == g.nz - 1;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const T uc = H0[c * HPL + ci];
            const T upd = uc + omega * (fb[c] - out[c]) / dg[c];
            vb[c] = (face && tg_dirichlet(g, gxb, gy, kb, c)) ? uc : upd;
          }
        }
        // both nodes of the pair back to back (complete lines)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T aval = H0[c * HPL + (yl + 1) * HX + xb + 1];
          if (gxb < g.nx) u_out[c * nn + row + gxb] = vb[c];
          if (gxo < g.nx) u_out[c * nn + row + gxo] = aval;
        }
      }
    }
    __syncthreads();
  };

  int k = k0 - 1;
  for (; k + 1 <= k1; k += 2) {
    step(k, RA, RB, FA);
    step(k + 1, RB, RA, FB);
  }
  if (k <= k1) step(k, RA, RB, FA);
}


// ------------------------------------------- first sweep from a zero iterate
//
// The first Gauss-Seidel sweep of a correction that starts from zero (Sec.
// 2.3), in one launch: colour A is relaxed from u = 0, which is pointwise
// (a = omega f / D), and colour B from u_mid = (a on A, 0 on B).  At a B node
// the centre and the edge neighbours of eq. K are B nodes, all 0 in u_mid, so
// K u_mid there needs only the A values of the six face neighbours: the terms
// of the other neighbours are exact zeros and are left out (the sums are the
// same numbers).  A workgroup owns a 64 x 8 node column and marches up its
// chunk; the A values of the plane two steps ahead (halo included) are made in
// LDS from f and the cells, one row half per row (LDS holds only A values),
// and B is relaxed on the current plane.  The node column / row past the last
// whole tile of a 2^n + 1 level (x = nx - 1, y = ny - 1) belongs to the last
// tile of its row / column.
constexpr int ZX = TX + 4, ZY = TY + 3;     // local columns x0-1..x0+66, rows y0-1..y0+9
constexpr int ZHX = ZX / 2;                 // A nodes per row (one parity half)
constexpr int ZPA = ZY * ZHX;               // A nodes per plane and component
constexpr int ZCX = TX + 4, ZCY = TY + 4;   // cells: columns x0-2..x0+65, rows y0-2..y0+9
constexpr int ZNC = ZCX * ZCY, ZHC = ZCX / 2;
constexpr int ZSN = (ZPA + NT - 1) / NT;    // A nodes made per thread and plane
constexpr int ZSC = (ZNC + NT - 1) / NT;    // cell loads per thread and plane
static_assert(ZX % 2 == 0 && ZCX % 2 == 0, "rows split into two equal halves");

// Cell-local index of cell column clx (cells from x0 - 2, parity split).
__device__ __forceinline__ int zcell(int clx, int cly) { return cly * ZCX + lds_col(clx, ZHC); }

// The psi of the 8 cells around the node whose cells are (clx + a, cly + b) of
// the planes below / above (P[c2][c1][c0] as in stencil3), their edge sums E
// and the diagonal D of K (stencil3's direct part).
template <typename T, typename CO>
__device__ __forceinline__ void zero_cells(const CO &C, const T *Pm, const T *P0, int clx, int cly,
                                           T (&P)[2][2][2], T (&E)[3][2], T dg[3]) {
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      P[0][b][a] = Pm[zcell(clx + a, cly + b)];
      P[1][b][a] = P0[zcell(clx + a, cly + b)];
    }
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    E[0][s] = P[0][0][s] + P[0][1][s] + P[1][0][s] + P[1][1][s];
    E[1][s] = P[0][s][0] + P[0][s][1] + P[1][s][0] + P[1][s][1];
    E[2][s] = P[s][0][0] + P[s][0][1] + P[s][1][0] + P[s][1][1];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
    dg[c] = coef_cd(C, c, 0) * (E[0][0] + E[0][1]) + coef_cd(C, c, 1) * (E[1][0] + E[1][1]) +
            coef_cd(C, c, 2) * (E[2][0] + E[2][1]);
}

// (K u)(n) at a node n whose centre and edge neighbours are 0: F[c][a][s] is
// component c at the face neighbour n + (2s - 1) e_a.  The expressions are
// stencil3's with the zero terms removed.
template <typename T, typename CO>
__device__ __forceinline__ void zero_face_stencil(const CO &C, const T (&P)[2][2][2],
                                                  const T (&E)[3][2], const T (&F)[3][3][2],
                                                  T out[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
    out[c] = -(coef_cd(C, c, 0) * (E[0][1] * F[c][0][1] + E[0][0] * F[c][0][0]) +
               coef_cd(C, c, 1) * (E[1][1] * F[c][1][1] + E[1][0] * F[c][1][0]) +
               coef_cd(C, c, 2) * (E[2][1] * F[c][2][1] + E[2][0] * F[c][2][0]));
#pragma unroll
  for (int pl = 0; pl < 3; ++pl) {
    const int a = (pl == 2) ? 1 : 0;
    const int b = (pl == 0) ? 1 : 2;
    const T cm = coef_cm(C, pl);
    T ra = T(0), rb = T(0);
#pragma unroll
    for (int qa = 0; qa < 2; ++qa)
#pragma unroll
      for (int qb = 0; qb < 2; ++qb) {
        const int sa = 2 * qa - 1, sb = 2 * qb - 1;
        T Fs;
        if (pl == 0) Fs = P[0][qb][qa] + P[1][qb][qa];
        else if (pl == 1) Fs = P[qb][0][qa] + P[qb][1][qa];
        else Fs = P[qb][qa][0] + P[qb][qa][1];
        const T w = (sa * sb > 0) ? Fs : -Fs;
        // u_b(n + sb e_b) - u_b(n + sa e_a) and u_a(n + sa e_a) - u_a(n + sb e_b)
        ra += w * (cm * (F[b][b][qb] - F[b][a][qa]));
        rb += w * (cm * (F[a][a][qa] - F[a][b][qb]));
      }
    out[a] -= ra;
    out[b] -= rb;
  }
}

template <typename T, typename CO>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_rb_zero(
    TG g, CO C, const T *__restrict__ psi, const T *__restrict__ f, T *__restrict__ u_out,
    T omega, int c0, TileGeom tg) {
  __shared__ T sm[3][3 * ZPA];   // A values of planes k-1, k, k+1 (slot z mod 3)
  __shared__ T sc[4][ZNC];       // cell planes k-1 .. k+2 (slot z mod 4)
  const int n = tg.ntiles;
  const int n8 = (n + 7) / 8 * 8;
  const int li = (int)(blockIdx.x & 7) * (n8 >> 3) + (int)(blockIdx.x >> 3);
  if (li >= n) return;
  constexpr int W = sizeof(T);
  const int nn = g.nn, nxy = g.nx * g.ny;
  const int vbytes = 3 * nn * W;
  const __amdgpu_buffer_rsrc_t rf = make_rsrc(f, vbytes), rp = make_rsrc(psi, g.cx * g.cy * g.cz * W),
                               ro = make_rsrc(u_out, vbytes);
  const int tx = li % tg.ntx, rest = li / tg.ntx;
  const int ty = rest % tg.nty, tz = rest / tg.nty;
  const int x0 = tx * TX, y0 = ty * TY;
  int k0, k1;
  tile_chunk(tg, tz, g.nz, k0, k1);
  const int xe = (tg.xface && tx == tg.ntx - 1) ? 1 : 0;  // the tile also owns x = x0 + 64
  const int ye = (tg.yface && ty == tg.nty - 1) ? 1 : 0;  // ... and y = y0 + 8
  const int t = threadIdx.x;
  // A-node slot j of this thread: entry e = t + j NT of (row ly, index hi); in
  // plane z its local column is lx = 2 hi + ((c0 + x0 - 1 + y0 - 1 + ly + z) & 1)
  auto a_node = [&](int j, int z, int &lx, int &ly, int &gx, int &gyy) __attribute__((always_inline)) {
    const int e = t + j * NT;
    ly = e / ZHX;
    const int hi = e - ly * ZHX;
    gyy = y0 - 1 + ly;
    lx = 2 * hi + ((c0 + x0 - 1 + gyy + z) & 1);
    gx = x0 - 1 + lx;
    return e < ZPA && gx >= 0 && gx < g.nx && gyy >= 0 && gyy < g.ny && lx <= TX + 1 + xe &&
           ly <= TY + 1 + ye;
  };
  int vc[ZSC];
#pragma unroll
  for (int j = 0; j < ZSC; ++j) {
    const int e = t + j * NT;
    vc[j] = kOOB;
    if (e < ZNC) {
      const int cly = e / ZCX, xr = e - cly * ZCX;
      const int hf = xr >= ZHC ? 1 : 0;
      const int clx = 2 * (xr - hf * ZHC) + hf;
      const int gx = x0 - 2 + clx, gy = y0 - 2 + cly;
      if (gx >= 0 && gx < g.cx && gy >= 0 && gy < g.cy) vc[j] = (gx + g.cx * gy) * W;
    }
  }
  auto fetch_cells = [&](int zc_, T (&r)[ZSC]) __attribute__((always_inline)) {
    const bool in = zc_ >= 0 && zc_ < g.cz;
    const int so = in ? zc_ * g.cx * g.cy * W : 0;
#pragma unroll
    for (int j = 0; j < ZSC; ++j) r[j] = bload<T>(rp, in ? vc[j] : kOOB, so);
  };
  auto put_cells = [&](int zc_, const T (&r)[ZSC]) __attribute__((always_inline)) {
    T *d = sc[(zc_ + 4) & 3];
#pragma unroll
    for (int j = 0; j < ZSC; ++j)
      if (j < ZSC - 1 || t + j * NT < ZNC) d[t + j * NT] = r[j];
  };
  // f of the A nodes of plane z
  auto fetch_zf = [&](int z, T (&r)[ZSN][3]) __attribute__((always_inline)) {
    const bool in = z >= 0 && z < g.nz;
    const int so = in ? z * nxy * W : 0;
#pragma unroll
    for (int j = 0; j < ZSN; ++j) {
      int lx, ly, gx, gyy;
      const bool ok = in && a_node(j, z, lx, ly, gx, gyy);
      const int vo = ok ? (gx + g.nx * gyy) * W : kOOB;
#pragma unroll
      for (int c = 0; c < 3; ++c) r[j][c] = bload<T>(rf, vo, so + c * nn * W);
    }
  };
  // A values of plane z: omega f / D (0 on displacement DOF and outside the box)
  auto make_a = [&](int z, const T (&fz)[ZSN][3]) __attribute__((always_inline)) {
    T *d = sm[(z + 3) % 3];
    const T *Pm = sc[(z + 3) & 3], *P0 = sc[(z + 4) & 3];
    const bool zin = z >= 0 && z < g.nz;
#pragma unroll
    for (int j = 0; j < ZSN; ++j) {
      int lx, ly, gx, gyy;
      const bool inb = a_node(j, z, lx, ly, gx, gyy);
      const int e = t + j * NT;
      if (j < ZSN - 1 || e < ZPA) {
        T v[3] = {T(0), T(0), T(0)};
        if (zin && inb) {
          T P[2][2][2], E[3][2], dg[3];
          zero_cells<T>(C, Pm, P0, lx, ly, P, E, dg);
          const bool face = gx == 0 || gx == g.nx - 1 || gyy == 0 || gyy == g.ny - 1 || z == 0 ||
                            z == g.nz - 1;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const T upd = T(0) + omega * (fz[j][c] - T(0)) / dg[c];
            v[c] = (face && tg_dirichlet(g, gx, gyy, z, c)) ? T(0) : upd;
          }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) d[c * ZPA + e] = v[c];
      }
    }
  };
  // B nodes of this thread: the x-pair (2p, 2p+1) of row yl; in an edge tile
  // of a 2^n + 1 level also row 8 (threads 0-31: columns 2t, 2t+1) or column 64
  // (threads 32-40: with the out-of-box column 65 as its pair)
  const int yl = t / (TX / 2), p = t % (TX / 2);
  const int gy = y0 + yl;
  const int vn0 = (gy < g.ny && x0 + 2 * p < g.nx) ? (gy * g.nx + x0 + 2 * p) * W : kOOB;
  const int vn1 = (gy < g.ny && x0 + 2 * p + 1 < g.nx) ? (gy * g.nx + x0 + 2 * p + 1) * W : kOOB;
  const bool xrow = ye && t < TX / 2;
  const bool xcol = xe && t >= 32 && t < 32 + TY + ye && y0 + t - 32 < g.ny;
  const int ex = xrow ? 2 * t : TX, ey = xrow ? TY : t - 32;
  const int gey = y0 + ey;
  const int ve0 = ((xrow || xcol) && x0 + ex < g.nx) ? (gey * g.nx + x0 + ex) * W : kOOB;
  const int ve1 = (xrow && x0 + ex + 1 < g.nx) ? (gey * g.nx + x0 + ex + 1) * W : kOOB;
  // f of the B node of the pair and of the extra pair, plane k
  auto fetch_fb = [&](int k, T (&r)[2][3]) __attribute__((always_inline)) {
    const bool in = k < k1;
    const int so = in ? k * nxy * W : 0;
    const int pb0 = ((1 - c0) + gy + x0 + 2 * p + k) & 1;
    const int pb1 = ((1 - c0) + gey + x0 + ex + k) & 1;
    const int vo = pb0 ? vn1 : vn0, ve = pb1 ? ve1 : ve0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r[0][c] = bload<T>(rf, in ? vo : kOOB, so + c * nn * W);
      r[1][c] = bload<T>(rf, in ? ve : kOOB, so + c * nn * W);
    }
  };

  // prologue: cells k0-2..k0+1, A values of planes k0-1..k0+1
  T CQ[ZSC], FZ[ZSN][3], FB[2][3];
  fetch_cells(k0 - 2, CQ);
  put_cells(k0 - 2, CQ);
  fetch_cells(k0 - 1, CQ);
  put_cells(k0 - 1, CQ);
  fetch_cells(k0, CQ);
  put_cells(k0, CQ);
  fetch_cells(k0 + 1, CQ);
  put_cells(k0 + 1, CQ);
  __syncthreads();
  for (int z = k0 - 1; z <= k0 + 1; ++z) {
    fetch_zf(z, FZ);
    make_a(z, FZ);
  }
  fetch_fb(k0, FB);
  fetch_cells(k0 + 2, CQ);
  __syncthreads();
  for (int k = k0; k < k1; ++k) {
    // cells k + 2 (fetched a step ago) go to the slot of k - 2, unused from here
    put_cells(k + 2, CQ);
    fetch_zf(k + 2, FZ);
    fetch_cells(k + 3, CQ);
    const T *Am = sm[(k + 2) % 3], *A0 = sm[k % 3], *A1 = sm[(k + 1) % 3];
    const T *Pm = sc[(k + 3) & 3], *P0 = sc[k & 3];
    const int so = k * nxy * W;
    const int npass = (xrow || xcol) ? 2 : 1;
    for (int pass = 0; pass < npass; ++pass) {
      const int px = pass ? ex : 2 * p, py = pass ? ey : yl;
      const int gpy = y0 + py;
      const int o0 = pass ? ve0 : vn0, o1 = pass ? ve1 : vn1;
      const int pb = ((1 - c0) + gpy + x0 + px + k) & 1;  // 1: the second column is B
      const int lx = px + pb + 1, lxa = px + 1 - pb + 1, ly = py + 1;
      T vb[3] = {T(0), T(0), T(0)};
      if (gpy < g.ny && x0 + lx - 1 < g.nx) {
        T P[2][2][2], E[3][2], dg[3], F[3][3][2];
        zero_cells<T>(C, Pm, P0, lx, ly, P, E, dg);
        const int hx = ly * ZHX, hm = hx + ((lx - 1) >> 1), hp = hx + ((lx + 1) >> 1);
        const int hc = lx >> 1;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          F[c][0][0] = A0[c * ZPA + hm];
          F[c][0][1] = A0[c * ZPA + hp];
          F[c][1][0] = A0[c * ZPA + hx - ZHX + hc];
          F[c][1][1] = A0[c * ZPA + hx + ZHX + hc];
          F[c][2][0] = Am[c * ZPA + hx + hc];
          F[c][2][1] = A1[c * ZPA + hx + hc];
        }
        T out[3];
        zero_face_stencil<T>(C, P, E, F, out);
        const int gx = x0 + lx - 1;
        const bool face = gx == 0 || gx == g.nx - 1 || gpy == 0 || gpy == g.ny - 1 || k == 0 ||
                          k == g.nz - 1;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T fv = pass ? FB[1][c] : FB[0][c];
          const T upd = T(0) + omega * (fv - out[c]) / dg[c];
          vb[c] = (face && tg_dirichlet(g, gx, gpy, k, c)) ? T(0) : upd;
        }
      }
      const int ca = ly * ZHX + (lxa >> 1);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        bstore<T>(vb[c], ro, pb ? o1 : o0, so + c * nn * W);
        bstore<T>(A0[c * ZPA + ca], ro, pb ? o0 : o1, so + c * nn * W);
      }
    }
    // f of the next plane's B nodes (used a step later)
    fetch_fb(k + 1, FB);
    __syncthreads();
    // A values of plane k + 2 into the slot of plane k - 1
    make_a(k + 2, FZ);
    __syncthreads();
  }
}
}  // namespace

hipError_t launch_active_tiles(const Level &L, const uint8_t *cls, int *flags, int *ids,
                               int *count, hipStream_t st, int kz, bool unknowns) {
  const TG gg = make_tg(L.g);
  const TileGeom tg = tile_geom(gg, false, kz);
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_tile_flags, dim3(tg.ntiles), dim3(256), 0, st, gg, tg, cls,
                     unknowns ? 1 : 255, flags);
  hipLaunchKernelGGL(k_tile_compact, dim3(1), dim3(1024), 0, st, (const int *)flags, tg.ntiles,
                     ids, count);
  return hipGetLastError();
}

bool tiled_ok(const Level &L) {
  // the residual, Krylov Apply and restriction passes (and the tile lists of
  // adaptive levels): levels wider than 192 nodes, where they outrun the
  // node-parallel kernels (the half-sweep 1.5x at 257^3).  The buffer offsets
  // of a vector must stay below kOOB.
  return L.g.dim == 3 && L.g.nx > 3 * TX && L.g.ny > 3 * TY &&
         3 * L.g.nn * (int64_t)sizeof(double) < (int64_t)kOOB;
}

bool tiled_sweep_ok(const Level &L) {
  // the half-sweep alone: also from 97 nodes (129^3, whose vectors sit in the
  // Infinity Cache: 41.2 us against 44.6 us for the node-parallel kernel in
  // FP64, 27.5 us against 36.2 us in FP32)
  return L.g.dim == 3 && L.g.nx > 96 && L.g.ny > 3 * TY &&
         3 * L.g.nn * (int64_t)sizeof(double) < (int64_t)kOOB;
}

// The level's coefficients as the 4 scalars of CoefCubic when its cells are
// cubic (the same numbers, so the results are those of Coef).
template <typename T>
static bool cubic_coef(const Coef<T> &C, CoefCubic<T> &cc) {
  cc = CoefCubic<T>{C.cd[0][0], C.cd[0][1], C.cp[0], C.cm[0]};
  for (int i = 0; i < 3; ++i) {
    if (C.cp[i] != cc.p || C.cm[i] != cc.m) return false;
    for (int j = 0; j < 3; ++j)
      if (C.cd[i][j] != (i == j ? cc.dd : cc.od)) return false;
  }
  return true;
}

TileGeom tile_geom_of(const Level &L, int kz) { return tile_geom(make_tg(L.g), false, kz); }

bool zero_sweep_ok(const Level &L) {
  // 3D levels wider than 96 nodes (measured: 129^3 70 us against 84 us for
  // the half-sweep pair; at 65^3 the 136 tiles leave most CUs idle and the
  // pair of node-parallel half-sweeps is faster)
  return L.g.dim == 3 && L.g.nx > 96 && L.g.ny >= 9 && L.g.nz >= 2 &&
         3 * L.g.nn * (int64_t)sizeof(double) < (int64_t)kOOB;
}

// Workgroups of a tiled launch over n tiles: the tiles rounded up to a
// multiple of 8 (XCD order), then the face blocks of a whole-level launch.
static int tiled_grid(int n, int nface) { return (n + 7) / 8 * 8 + nface; }

template <typename T>
hipError_t launch_rb_tiled(const Level &L, const T *psi, const Coef<T> &C, const T *u, const T *f,
                           T *u_out, double omega, int colour, hipStream_t st,
                           const uint8_t *cls, const TileList *tl, double *partials,
                           const double *r64, const double *ss) {
  const TG gg = make_tg(L.g);
  const TileGeom tg =
      tile_geom(gg, tl == nullptr, tl ? tl->kz : 0, tile_target<T>(TileKind::half));
  const int n = tl ? tl->count : tg.ntiles;
  const int *ids = tl ? tl->ids : nullptr;
  CoefCubic<T> cc;
  const bool cubic = cubic_coef(C, cc);
  (void)hipGetLastError();
  // the partials: whole-level launches; FP32 ones sum r . (s u_out) from the
  // FP64 residual r64 and s^2 = *ss
  if (partials && (cls || tl || (sizeof(T) != 8 && (!r64 || !ss)))) return hipErrorInvalidValue;
  const DotSrc ds{r64, ss};
  const int nface = tl ? 0 : tg.nface;
  if (n + nface > 0) {
    const dim3 grid(tiled_grid(n, nface)), block(NT);
    if (partials && cubic)
      hipLaunchKernelGGL((k_rb_tile<T, CoefCubic<T>, false, true>), grid, block, 0, st, gg, cc,
                         psi, u, f, u_out, (T)omega, colour, tg, cls, ids, n, partials, ds);
    else if (partials)
      hipLaunchKernelGGL((k_rb_tile<T, Coef<T>, false, true>), grid, block, 0, st, gg, C, psi,
                         u, f, u_out, (T)omega, colour, tg, cls, ids, n, partials, ds);
    else if (cls && cubic)
      hipLaunchKernelGGL((k_rb_tile<T, CoefCubic<T>, true, false>), grid, block, 0, st, gg, cc,
                         psi, u, f, u_out, (T)omega, colour, tg, cls, ids, n, partials, ds);
    else if (cls)
      hipLaunchKernelGGL((k_rb_tile<T, Coef<T>, true, false>), grid, block, 0, st, gg, C, psi,
                         u, f, u_out, (T)omega, colour, tg, cls, ids, n, partials, ds);
    else if (cubic)
      hipLaunchKernelGGL((k_rb_tile<T, CoefCubic<T>, false, false>), grid, block, 0, st, gg, cc,
                         psi, u, f, u_out, (T)omega, colour, tg, cls, ids, n, partials, ds);
    else
      hipLaunchKernelGGL((k_rb_tile<T, Coef<T>, false, false>), grid, block, 0, st, gg, C, psi,
                         u, f, u_out, (T)omega, colour, tg, cls, ids, n, partials, ds);
  }
  return hipGetLastError();
}

int rb_tiled_partials(const Level &L, bool fp32) {
  const TileGeom tg = tile_geom(make_tg(L.g), true, 0,
                                fp32 ? tile_target<float>(TileKind::half)
                                     : tile_target<double>(TileKind::half));
  return tg.ntiles + tg.nface;
}

template <typename T>
hipError_t launch_rb_fused(const Level &L, const T *psi, const Coef<T> &C, const T *u, const T *f,
                           T *u_out, double omega, int first_colour, hipStream_t st) {
  const TG gg = make_tg(L.g);
  const TileGeom tg = tile_geom(gg);
  const int grid = (tg.ntiles + 7) / 8 * 8;
  (void)hipGetLastError();
  if (u) {
    hipLaunchKernelGGL((k_rb_fused<T, false>), dim3(grid), dim3(NT), 0, st, gg, C, psi, u, f,
                       u_out, (T)omega, first_colour, tg);
  } else {
    // from zero: k_rb_zero over the tiles of the whole level (the last node
    // column / row of a 2^n + 1 level in the edge tiles)
    const TileGeom tz = tile_geom(gg, true, 0, tile_target<T>(TileKind::zero));
    TileGeom tf = tz;
    tf.nface = 0;
    const dim3 zgrid((tf.ntiles + 7) / 8 * 8);
    CoefCubic<T> cc;
    if (cubic_coef(C, cc))
      hipLaunchKernelGGL((k_rb_zero<T, CoefCubic<T>>), zgrid, dim3(NT), 0, st, gg, cc, psi, f,
                         u_out, (T)omega, first_colour, tf);
    else
      hipLaunchKernelGGL((k_rb_zero<T, Coef<T>>), zgrid, dim3(NT), 0, st, gg, C, psi, f, u_out,
                         (T)omega, first_colour, tf);
  }
  return hipGetLastError();
}

template hipError_t launch_rb_fused<double>(const Level &, const double *, const Coef<double> &,
                                            const double *, const double *, double *, double, int,
                                            hipStream_t);
template hipError_t launch_rb_fused<float>(const Level &, const float *, const Coef<float> &,
                                           const float *, const float *, float *, double, int,
                                           hipStream_t);

// (the FP64 launch geometry: only FP64 launches write partial sums)
int tiled_partials(const Level &L) {
  const TileGeom tg = tile_geom(make_tg(L.g), true, 0, tile_target<double>(TileKind::full));
  return tg.ntiles + tg.nface;
}

template <typename T, int MODE>
static void full_tiled(const Level &L, const T *psi, const Coef<T> &C, const T *u, const T *f,
                       T *r, double *partials, hipStream_t st, const uint8_t *cls,
                       const TileList *tl) {
  const TG gg = make_tg(L.g);
  const TileGeom tg =
      tile_geom(gg, tl == nullptr, tl ? tl->kz : 0, tile_target<T>(TileKind::full));
  const int n = tl ? tl->count : tg.ntiles;
  const int *ids = tl ? tl->ids : nullptr;
  CoefCubic<T> cc;
  const bool cubic = cubic_coef(C, cc);
  const int nface = tl ? 0 : tg.nface;
  if (n + nface > 0) {
    const dim3 grid(tiled_grid(n, nface)), block(NT);
    if (cls && cubic)
      hipLaunchKernelGGL((k_full_tile<T, CoefCubic<T>, MODE, true>), grid, block, 0, st, gg, cc,
                         psi, u, f, r, partials, tg, cls, ids, n);
    else if (cls)
      hipLaunchKernelGGL((k_full_tile<T, Coef<T>, MODE, true>), grid, block, 0, st, gg, C, psi,
                         u, f, r, partials, tg, cls, ids, n);
    else if (cubic)
      hipLaunchKernelGGL((k_full_tile<T, CoefCubic<T>, MODE, false>), grid, block, 0, st, gg, cc,
                         psi, u, f, r, partials, tg, cls, ids, n);
    else
      hipLaunchKernelGGL((k_full_tile<T, Coef<T>, MODE, false>), grid, block, 0, st, gg, C, psi,
                         u, f, r, partials, tg, cls, ids, n);
  }
}

template <typename T>
hipError_t launch_residual_tiled(const Level &L, const T *psi, const Coef<T> &C, const T *u,
                                 const T *f, T *r, double *partials, hipStream_t st,
                                 const uint8_t *cls, const TileList *tl) {
  if (partials && sizeof(T) != 8) return hipErrorInvalidValue;  // counted for FP64 tiles
  (void)hipGetLastError();
  full_tiled<T, 0>(L, psi, C, u, f, r, partials, st, cls, tl);
  return hipGetLastError();
}

hipError_t launch_apply_dot_tiled(const Level &L, const double *p, double *q, double *partials,
                                  hipStream_t st) {
  (void)hipGetLastError();
  full_tiled<double, 1>(L, L.psi64, L.c64, p, (const double *)nullptr, q, partials, st, nullptr,
                        nullptr);
  return hipGetLastError();
}

template hipError_t launch_residual_tiled<double>(const Level &, const double *,
                                                  const Coef<double> &, const double *,
                                                  const double *, double *, double *, hipStream_t,
                                                  const uint8_t *, const TileList *);
template hipError_t launch_residual_tiled<float>(const Level &, const float *, const Coef<float> &,
                                                 const float *, const float *, float *, double *,
                                                 hipStream_t, const uint8_t *, const TileList *);

template hipError_t launch_rb_tiled<double>(const Level &, const double *, const Coef<double> &,
                                            const double *, const double *, double *, double,
                                            int, hipStream_t, const uint8_t *, const TileList *,
                                            double *, const double *, const double *);
template hipError_t launch_rb_tiled<float>(const Level &, const float *, const Coef<float> &,
                                           const float *, const float *, float *, double, int,
                                           hipStream_t, const uint8_t *, const TileList *,
                                           double *, const double *, const double *);

}  // namespace sbm
