// host.cpp -- planner and C ABI of libgrmhd.so.
//
// The planner turns a grid descriptor into the integer and geometry tables the kernels
// read: the packed block layout, per-column metric tables (Sec. 2.2), and gather lists
// that fill every ghost cell and ghost face from its source (a neighbour block's
// interior, or the physical boundary rule).  Everything large lives in the caller's
// work buffer; this file allocates host memory only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdlib>
#include <cstddef>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/grmhd.h"
#include "device.h"
#include "internal.h"

using namespace grmhd;

static thread_local std::string g_err;

// An allocator whose resize leaves plain-data elements uninitialised, for the planner's
// large lists: they are filled right after (in parallel), and zeroing them first would
// touch every page once more on one thread.
template <class T>
struct NoInit : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInit<U>;
  };
  NoInit() = default;
  template <class U>
  NoInit(const NoInit<U>&) {}
  template <class U>
  void construct(U* ptr) noexcept {
    ::new ((void*)ptr) U;
  }
  template <class U, class... A>
  void construct(U* ptr, A&&... a) {
    ::new ((void*)ptr) U(std::forward<A>(a)...);
  }
};
template <class T>
using BigVec = std::vector<T, NoInit<T>>;

// Runs f(i) for i in [0, n) on up to 16 worker threads (the calling thread included);
// GRMHD_PLANNER_THREADS in the environment sets a lower count (1: the calling thread
// only).
template <class F>
static void parallel_for(int64_t n, F&& f) {
  std::atomic<int64_t> next{0};
  auto work = [&]() {
    for (int64_t i = next++; i < n; i = next++) f(i);
  };
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (const char* env = std::getenv("GRMHD_PLANNER_THREADS")) {
    const long v = std::strtol(env, nullptr, 10);
    if (v >= 1) nt = std::min<unsigned>(nt, (unsigned)v);
  }
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nt && (int64_t)t < n; t++) th.emplace_back(work);
  work();
  for (std::thread& t : th) t.join();
}

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int grmhd::set_error(int code, const char* msg) { return fail(code, msg); }

#define HIPCHK(x)                                                                  \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess)                                                          \
      return fail(GRMHD_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));     \
  } while (0)

// ------------------------------------------------------------------------ geometry

namespace {

template <typename T>
void ks_gcov(double a, T x1, T x2, T g[4][4]) {
  const T r = std::exp(x1);
  const T s = std::sin(x2), c = std::cos(x2);
  const T sig = r * r + a * a * c * c;
  const T q = 2.0 * r / sig;
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++) g[m][n] = T(0.0);
  g[0][0] = -(1.0 - q);
  g[0][1] = g[1][0] = q * r;
  g[0][3] = g[3][0] = -a * q * s * s;
  g[1][1] = (1.0 + q) * r * r;
  g[1][3] = g[3][1] = -a * s * s * (1.0 + q) * r;
  g[2][2] = sig;
  g[3][3] = s * s * (sig + a * a * s * s * (1.0 + q));
}

// closed-form inverse of the Kerr-Schild metric in internal coordinates
void ks_gcon(double a, double x1, double x2, double h[4][4]) {
  const double r = std::exp(x1), s = std::sin(x2), c = std::cos(x2);
  const double sig = r * r + a * a * c * c;
  const double delta = r * r - 2.0 * r + a * a;
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++) h[m][n] = 0.0;
  h[0][0] = -(1.0 + 2.0 * r / sig);
  h[0][1] = h[1][0] = 2.0 / sig;            // (2r/Sigma) / r
  h[1][1] = delta / (sig * r * r);
  h[1][3] = h[3][1] = a / (sig * r);
  h[2][2] = 1.0 / sig;
  h[3][3] = 1.0 / (sig * s * s);
}

// out[0..14] in Metric order; conn (optional) [40] = Gamma^l_{mn}, m <= n, l*10 + pair.
// Derivatives of the covariant metric by complex-step differentiation (exact to
// rounding, no subtractive cancellation).
void geometry_point(int coords, double a, double x1, double x2, double* out, double* conn) {
  double g[4][4], h[4][4];
  if (coords == GRMHD_MINK_CART) {
    for (int m = 0; m < 4; m++)
      for (int n = 0; n < 4; n++) g[m][n] = h[m][n] = (m == n) ? (m == 0 ? -1.0 : 1.0) : 0.0;
  } else {
    std::complex<double> gc[4][4];
    ks_gcov<std::complex<double>>(a, std::complex<double>(x1, 0.0), std::complex<double>(x2, 0.0), gc);
    for (int m = 0; m < 4; m++)
      for (int n = 0; n < 4; n++) g[m][n] = gc[m][n].real();
    ks_gcon(a, x1, x2, h);
  }
  out[G00] = g[0][0]; out[G01] = g[0][1]; out[G03] = g[0][3]; out[G11] = g[1][1];
  out[G13] = g[1][3]; out[G22] = g[2][2]; out[G33] = g[3][3];
  out[H00] = h[0][0]; out[H01] = h[0][1]; out[H11] = h[1][1]; out[H13] = h[1][3];
  out[H22] = h[2][2]; out[H33] = h[3][3];
  if (coords == GRMHD_MINK_CART) {
    out[GDET] = 1.0;
    out[ALPHA] = 1.0;
  } else {
    const double r = std::exp(x1), s = std::sin(x2), c = std::cos(x2);
    const double sig = r * r + a * a * c * c;
    out[GDET] = r * sig * std::fabs(s);
    out[ALPHA] = 1.0 / std::sqrt(1.0 + 2.0 * r / sig);
  }
  if (!conn) return;
  double dg[4][4][4] = {};
  if (coords == GRMHD_KS_LOGSPH) {
    const double hs = 1e-30;
    std::complex<double> gc[4][4];
    ks_gcov<std::complex<double>>(a, std::complex<double>(x1, hs), std::complex<double>(x2, 0.0), gc);
    for (int m = 0; m < 4; m++)
      for (int n = 0; n < 4; n++) dg[1][m][n] = gc[m][n].imag() / hs;
    ks_gcov<std::complex<double>>(a, std::complex<double>(x1, 0.0), std::complex<double>(x2, hs), gc);
    for (int m = 0; m < 4; m++)
      for (int n = 0; n < 4; n++) dg[2][m][n] = gc[m][n].imag() / hs;
  }
  for (int l = 0; l < 4; l++) {
    int p = 0;
    for (int m = 0; m < 4; m++)
      for (int n = m; n < 4; n++, p++) {
        double acc = 0.0;
        for (int k = 0; k < 4; k++) acc += h[l][k] * (dg[m][k][n] + dg[n][k][m] - dg[k][m][n]);
        conn[l * 10 + p] = 0.5 * acc;
      }
  }
}

int imod(int64_t a, int64_t n) {
  int64_t m = a % n;
  return (int)(m < 0 ? m + n : m);
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct GeoTable {
  int32_t l0, l1;            // x1, x2 refinement levels
  int32_t ti, tj;            // padded extents
  int64_t base;              // first column
};

struct Plan {
  grmhd_grid_desc d;
  std::vector<grmhd_block_desc> blocks;
  std::vector<BlockInfo> info;
  int64_t vtot = 0;          // total padded cells
  int64_t n_interior = 0;
  int32_t max_np[3] = {0, 0, 0}, max_n[3] = {0, 0, 0};
  int32_t lmax[3] = {0, 0, 0};  // finest refinement level per dimension
  bool refined = false;         // blocks at more than one refinement level
  std::vector<GeoTable> tables;
  int64_t ncol = 0;
  BigVec<int32_t> owner;   // block id per effective (finest-level) cell
  BigVec<GhostOp> ops[4];  // cells, x1 faces, x2 faces, x3 faces (by dst level, then block)
  BigVec<AmrOp> aops[4];   // ghost values across refinement levels (ordered likewise)
  BigVec<AmrSample> samples;   // in block order
  BigVec<uint8_t> samp_kind;   // the list (cells, x1/x2/x3 faces) of each sample
  // refinement faces between blocks of one time level (the coarse side takes the fine
  // side's fluxes in each stage), in the order the blocks are listed
  struct Link {
    int32_t c, f, d, side, e[3];
    int64_t lo[3], hi[3];   // shared patch, coarse global cells (transverse dimensions)
  };
  std::vector<Link> links;
  // Synchronisation tables, per block in block order (padded local indices):
  //   reflux: a boundary face of block b shared with a faster block D, and the elements
  //           of D covering it (its sub-faces where D is finer, the covering face where
  //           it is coarser);
  //   sync edges: a boundary edge of b whose dominant holder (fastest, then finest, then
  //           lowest index) D is faster, and D's elements covering it;
  //   stage edges: a boundary edge of b whose finest holder at b's time level is finer.
  struct Reflux {
    int32_t b, d, side, loc, D, n, sub[4];
  };
  struct EdgeRef {
    int32_t b, a, loc, D, n, sub[2];
  };
  std::vector<Reflux> reflux;
  std::vector<EdgeRef> sync_edges, stage_edges;
  // device lists built from them: per time level (offsets, +1 at the end)
  std::vector<MeanItem> fix;      // fluxes (kind 0) and EMFs (kind 1) of each stage
  std::vector<int64_t> fix_off;
  std::vector<MeanItem> bsync;    // coarse copies of refinement faces after each update
  std::vector<int64_t> bsync_off;
  std::vector<RegItem> regs;      // register elements of each level's corrector
  std::vector<int64_t> reg_off;
  int64_t nregF = 0, nregE = 0;
  std::vector<SyncCell> scells;   // by the slow block's level
  std::vector<int64_t> scell_off;
  std::vector<SyncFace> sfaces;
  std::vector<int64_t> sface_off;
  // work lists of the stage kernels for blocks of uneven sizes: per block list (each
  // time level, then all blocks) and region class, the (block, tile) items
  bool use_wl = false;
  std::vector<int2> wl;
  std::vector<int64_t> wl_off;   // [(list * WL_N + class)], one more at the end
  // local time stepping
  int32_t nlev = 1;
  std::vector<int32_t> lev_blocks;             // block ids sorted by level
  std::vector<int64_t> lev_boff;               // offsets into lev_blocks per level (+1)
  std::vector<int64_t> ops_off[4];             // offsets into ops[kind] per level (+1)
  std::vector<int64_t> aops_off[4];            // offsets into aops[kind] per level (+1)
  std::vector<int64_t> lev_cells;              // interior cells per level
  // per time level, the elements of its blocks that a faster neighbour reads as the old
  // state of a time-interpolated ghost: cells (element indices of the packed primitives)
  // and faces (of the packed face field), sorted, without repeats
  std::vector<uint32_t> slow_c, slow_f;
  std::vector<int64_t> slow_c_off, slow_f_off; // offsets per level (+1)
  // work-buffer offsets (bytes)
  size_t o_ps, o_balt, o_bc, o_f, o_e, o_gc, o_g1, o_g2, o_blk, o_ops[4], o_cnt, o_dtp, o_stp;
  int64_t slots;   // workgroups of a full-grid stage launch: Courant and statistics partials
  size_t o_aops[4], o_samp, o_fix, o_bsync, o_u9, o_wl;
  size_t o_pold, o_bold, o_slow, o_regs, o_regf, o_rege, o_scell, o_sface, o_ubuf, o_lev, total;
};

// cells of the grid at refinement levels lev along each dimension
void level_extent(const Plan& p, const int32_t* lev, int64_t N[3]) {
  for (int k = 0; k < 3; k++) N[k] = (int64_t)p.d.n_eff[k] >> (p.lmax[k] - lev[k]);
}

int validate(const grmhd_grid_desc* d) {
  if (!d) return fail(GRMHD_EINVAL, "desc is NULL");
  if (d->abi_version != GRMHD_ABI_VERSION) return fail(GRMHD_EINVAL, "abi_version mismatch");
  if (d->coords != GRMHD_MINK_CART && d->coords != GRMHD_KS_LOGSPH)
    return fail(GRMHD_EINVAL, "unknown coords");
  if (d->n_ghost < 2 || d->n_ghost > 4) return fail(GRMHD_EINVAL, "n_ghost must be 2..4");
  if ((d->recon == GRMHD_PPM || d->recon == GRMHD_PPM_FLAT) && d->n_ghost < 3)
    return fail(GRMHD_EINVAL, "PPM needs n_ghost >= 3");
  if (d->recon < GRMHD_PLM_MC || d->recon > GRMHD_PPM_FLAT) return fail(GRMHD_EINVAL, "unknown recon");
  if (d->riemann != GRMHD_LLF && d->riemann != GRMHD_HLLE) return fail(GRMHD_EINVAL, "unknown riemann");
  if (d->n_blocks < 1 || !d->blocks) return fail(GRMHD_EINVAL, "no blocks");
  if (d->n_lat_levels < 1 || d->n_lat_levels > 8) return fail(GRMHD_EINVAL, "n_lat_levels must be 1..8");
  for (int k = 0; k < 3; k++)
    if (d->n_eff[k] < 1 || !(d->xmax[k] > d->xmin[k])) return fail(GRMHD_EINVAL, "bad extent");
  if (!(d->bc[0] == GRMHD_BC_OUTFLOW || d->bc[0] == GRMHD_BC_PERIODIC) || !(d->bc[1] == d->bc[0]))
    return fail(GRMHD_EUNSUPPORTED, "x1 boundaries must be both outflow or both periodic");
  if (!(d->bc[2] == GRMHD_BC_POLAR || d->bc[2] == GRMHD_BC_PERIODIC) || !(d->bc[3] == d->bc[2]))
    return fail(GRMHD_EUNSUPPORTED, "x2 boundaries must be both polar or both periodic");
  if (d->bc[4] != GRMHD_BC_PERIODIC || d->bc[5] != GRMHD_BC_PERIODIC)
    return fail(GRMHD_EUNSUPPORTED, "x3 boundaries must be periodic");
  if (d->bc[2] == GRMHD_BC_POLAR && d->coords != GRMHD_KS_LOGSPH)
    return fail(GRMHD_EINVAL, "polar boundary needs spherical coordinates");
  if (d->c2p_maxit < 1 || d->c2p_maxit > 62) return fail(GRMHD_EINVAL, "c2p_maxit must be 1..62");
  if (!(d->c2p_tol > 0.0)) return fail(GRMHD_EINVAL, "c2p_tol must be positive");
  if (!(d->courant > 0.0)) return fail(GRMHD_EINVAL, "courant must be positive");
  if (d->c2p_guess != GRMHD_GUESS_PLAIN && d->c2p_guess != GRMHD_GUESS_MLP)
    return fail(GRMHD_EINVAL, "unknown c2p_guess");
  if (d->emf != GRMHD_EMF_AVERAGE && d->emf != GRMHD_EMF_UPWIND) return fail(GRMHD_EINVAL, "unknown emf");
  if (d->floor_frame != GRMHD_FLOOR_FIXED && d->floor_frame != GRMHD_FLOOR_DRIFT)
    return fail(GRMHD_EINVAL, "unknown floor_frame");
  if (d->c2p_guess == GRMHD_GUESS_MLP && !d->mlp_weights)
    return fail(GRMHD_EINVAL, "learned guess needs mlp_weights");
  int lmax[3] = {0, 0, 0};
  for (int b = 0; b < d->n_blocks; b++)
    for (int k = 0; k < 3; k++) {
      const int l = d->blocks[b].lev[k];
      if (l < 0 || l > 8) return fail(GRMHD_EINVAL, "block refinement level must be 0..8");
      lmax[k] = std::max(lmax[k], l);
    }
  for (int b = 0; b < d->n_blocks; b++) {
    const grmhd_block_desc& bd = d->blocks[b];
    for (int k = 0; k < 3; k++) {
      const int s = lmax[k] - bd.lev[k];
      const int64_t N = (int64_t)d->n_eff[k] >> s;
      if ((N << s) != d->n_eff[k] || N < 1)
        return fail(GRMHD_EINVAL, "effective grid not divisible by the refinement ratio");
      if (bd.n[k] < d->n_ghost && !(bd.n[k] == 1 && N == 1))
        return fail(GRMHD_EINVAL, "block smaller than the ghost width");
      if (bd.org[k] < 0 || bd.org[k] + bd.n[k] > N) return fail(GRMHD_EINVAL, "block outside the grid");
      if (k == 2 && d->bc[2] == GRMHD_BC_POLAR && N % 2 != 0 && N != 1)
        return fail(GRMHD_EINVAL, "polar boundary needs an even number of x3 cells at every level");
    }
    if (bd.lat < 0 || bd.lat >= d->n_lat_levels) return fail(GRMHD_EINVAL, "block lat out of range");
  }
  return GRMHD_OK;
}

// Composition of the physical boundary rules for a position outside the grid of extents
// N (one refinement level), applied x3 first, then x2, then x1 (the order in which ghost
// layers are filled, so that edge and corner ghosts take their values from
// already-filled layers).  kind 0 = cell, 1..3 = face of that component.  Returns false
// if the value is identically zero.
bool compose(const grmhd_grid_desc& d, const int64_t N[3], int kind, int64_t& i, int64_t& j,
             int64_t& k, int& flags) {
  const int64_t N1 = N[0], N2 = N[1], N3 = N[2];
  flags = 0;
  // x3: periodic
  if (kind == 3) {
    if (k < 0 || k > N3) k = imod(k, N3);
  } else if (k < 0 || k >= N3) {
    k = imod(k, N3);
  }
  // x2
  const bool polar = d.bc[2] == GRMHD_BC_POLAR;
  if (kind == 2) {
    if (polar && (j == 0 || j == N2)) return false;
    if (j < 0 || j > N2) {
      if (polar) {
        j = j < 0 ? -j : 2 * N2 - j;
        k = imod(k + N3 / 2, N3);
        flags |= GF_FLIP;
      } else {
        j = imod(j, N2);
      }
    }
  } else if (j < 0 || j >= N2) {
    if (polar) {
      j = j < 0 ? -1 - j : 2 * N2 - 1 - j;
      k = imod(k + N3 / 2, N3);
      if (kind == 0) flags |= GF_FLIP;
    } else {
      j = imod(j, N2);
    }
  }
  // x1
  const bool outflow = d.bc[0] == GRMHD_BC_OUTFLOW;
  if (kind == 1) {
    if (i < 0 || i > N1) {
      if (outflow) i = i < 0 ? 0 : N1;
      else i = imod(i, N1);
    }
  } else if (i < 0 || i >= N1) {
    if (outflow) {
      if (kind == 0) flags |= i < 0 ? GF_CLAMP_NEG : GF_CLAMP_POS;
      i = i < 0 ? 0 : N1 - 1;
    } else {
      i = imod(i, N1);
    }
  }
  return true;
}

// the block owning the cell (i, j, k) of the grid at refinement levels lev
int owner_at(const Plan& p, const int32_t* lev, int64_t i, int64_t j, int64_t k) {
  const int64_t N1 = p.d.n_eff[0], N2 = p.d.n_eff[1];
  i <<= (p.lmax[0] - lev[0]);
  j <<= (p.lmax[1] - lev[1]);
  k <<= (p.lmax[2] - lev[2]);
  return p.owner[(size_t)((k * N2 + j) * N1 + i)];
}

// Whether the stage kernels read padded cell x of a block: the face fluxes read cells
// along their normal across the whole ghost depth and one ghost layer sideways (the
// transverse fluxes of the boundary edges' EMFs).  So at most one index lies more than
// one layer outside the interior, and none in the last padding layer (which only
// completes the face layout).
bool cell_read(const BlockInfo& bi, int g, const int x[3]) {
  int far = 0;
  for (int d = 0; d < 3; d++) {
    if (x[d] < 0 || x[d] > 2 * g + bi.n[d] - 1) return false;
    if (x[d] < g - 1 || x[d] > g + bi.n[d]) far++;
  }
  return far <= 1;
}

// Whether a ghost element is read: a cell by the rule above (kind 0), or a face of
// component kind - 1 that bounds such a cell along its normal (the cell-centred field).
bool ghost_read(const BlockInfo& bi, int g, int kind, const int x[3]) {
  if (cell_read(bi, g, x)) return true;
  if (kind == 0) return false;
  const int y[3] = {x[0] - (kind == 1), x[1] - (kind == 2), x[2] - (kind == 3)};
  return cell_read(bi, g, y);
}

int32_t local_index(const BlockInfo& bi, int64_t li, int64_t lj, int64_t lk) {
  return (int32_t)((lk * bi.np[1] + lj) * bi.np[0] + li);
}

// Refinement of block o relative to levels lev: +1 finer, -1 coarser per dimension.
// Returns 0 same level, 1 finer by one level (in some dimensions), -1 coarser by one,
// 2 anything else (a jump of more than one level, or finer and coarser mixed).
int relation(const Plan& p, int o, const int32_t* lev, int r[3]) {
  int up = 0, down = 0;
  for (int k = 0; k < 3; k++) {
    r[k] = p.blocks[o].lev[k] - lev[k];
    if (r[k] > 1 || r[k] < -1) return 2;
    if (r[k] > 0) up = 1;
    if (r[k] < 0) down = 1;
  }
  if (up && down) return 2;
  return up ? 1 : (down ? -1 : 0);
}

int time_flags(const Plan& p, int src, int viewer) {
  if (p.blocks[src].lat > p.blocks[viewer].lat) return GF_SLOW;
  if (p.blocks[src].lat < p.blocks[viewer].lat) return GF_FAST;
  return 0;
}

// Of the blocks holding a copy of face (i, j, k) of component kind at levels lev (the
// cells on either side of it), the one a viewing block reads: itself, else one at the
// viewer's time level (blocks of one time level evolve such a face side by side and must
// read one copy of it), then the finest, then the one listed last.
int face_owner(const Plan& p, const int32_t* lev, const int64_t N[3], int kind, int64_t& i,
               int64_t& j, int64_t& k, int viewer) {
  const int d = kind - 1;
  // a face on a periodic seam (normal index 0 or N) lies between the first and the last
  // cell along its normal
  const bool per = d == 2 || p.d.bc[2 * d] == GRMHD_BC_PERIODIC;
  int cand[2];
  int nc = 0;
  int64_t q[3] = {i, j, k};
  if (q[d] < N[d] || per) {
    int64_t r[3] = {q[0], q[1], q[2]};
    r[d] = q[d] < N[d] ? q[d] : 0;
    cand[nc++] = owner_at(p, lev, r[0], r[1], r[2]);
  }
  if (q[d] - 1 >= 0 || per) {
    int64_t r[3] = {q[0], q[1], q[2]};
    r[d] = q[d] - 1 >= 0 ? q[d] - 1 : N[d] - 1;
    cand[nc++] = owner_at(p, lev, r[0], r[1], r[2]);
  }
  int best = cand[0];
  for (int c = 0; c < nc && best != viewer; c++) {
    const int o = cand[c];
    if (o == viewer) {
      best = viewer;
      break;
    }
    auto key = [&](int b) {
      const grmhd_block_desc& bd = p.blocks[b];
      return std::make_tuple(bd.lat == p.blocks[viewer].lat ? 1 : 0,
                             bd.lev[0] + bd.lev[1] + bd.lev[2], b);
    };
    if (key(o) > key(best)) best = o;
  }
  // the position in the chosen block's frame: the other representation of a seam face
  // where the block lies at the other end of the grid
  if (per && (q[d] == 0 || q[d] == N[d])) {
    const grmhd_block_desc& bd = p.blocks[best];
    const int s = lev[d] - bd.lev[d];
    const int64_t lo = s >= 0 ? bd.org[d] << s : bd.org[d] >> (-s);
    const int64_t hi = s >= 0 ? (bd.org[d] + bd.n[d]) << s : (bd.org[d] + bd.n[d]) >> (-s);
    if (q[d] < lo || q[d] > hi) q[d] = q[d] == 0 ? N[d] : 0;
  }
  i = q[0];
  j = q[1];
  k = q[2];
  return best;
}

struct Resolver {
  const Plan& p;
  int viewer;
  std::string err;

  // a cell value at position (i, j, k) of levels lev (inside the grid after the
  // boundary composition, with its flags): the owning block's own cell, or the
  // restriction of a finer owner; a coarser owner is an error
  bool cell_sample(const int32_t* lev, int64_t i, int64_t j, int64_t k, int flags, AmrSample& s) {
    const int o = owner_at(p, lev, i, j, k);
    int r[3];
    const int rel = relation(p, o, lev, r);
    const grmhd_block_desc& od = p.blocks[o];
    const BlockInfo& oi = p.info[o];
    const int g = p.d.n_ghost;
    s.blkf = o | ((flags | time_flags(p, o, viewer)) << 24);
    s.pad = 0;
    if (rel == 0) {
      s.loc = local_index(oi, i - od.org[0] + g, j - od.org[1] + g, k - od.org[2] + g);
      s.mask = 0;
      return true;
    }
    if (rel != 1) {
      err = "a refinement stencil reaches a block two levels away or a coarser block";
      return false;
    }
    const int64_t fi = i << r[0], fj = j << r[1], fk = k << r[2];
    const int64_t li = fi - od.org[0], lj = fj - od.org[1], lk = fk - od.org[2];
    if (li < 0 || lj < 0 || lk < 0 || li + r[0] >= od.n[0] || lj + r[1] >= od.n[1] ||
        lk + r[2] >= od.n[2]) {
      err = "refined blocks must start and end on coarse cell boundaries";
      return false;
    }
    s.loc = local_index(oi, li + g, lj + g, lk + g);
    s.mask = r[0] | (r[1] << 1) | (r[2] << 2);
    return true;
  }

  // a face value of component kind at position (i, j, k) of levels lev, after the
  // boundary composition (zero: a polar-axis face)
  bool face_sample(const int32_t* lev, const int64_t N[3], int kind, int64_t i, int64_t j,
                   int64_t k, bool zero, int flags, AmrSample& s) {
    s.pad = 0;
    if (zero) {
      s.blkf = viewer | (GF_ZERO << 24);
      s.loc = 0;
      s.mask = 0;
      return true;
    }
    const int d = kind - 1;
    const int o = face_owner(p, lev, N, kind, i, j, k, viewer);
    int r[3];
    const int rel = relation(p, o, lev, r);
    const grmhd_block_desc& od = p.blocks[o];
    const BlockInfo& oi = p.info[o];
    const int g = p.d.n_ghost;
    s.blkf = o | ((flags | time_flags(p, o, viewer)) << 24);
    if (rel == 0) {
      s.loc = local_index(oi, i - od.org[0] + g, j - od.org[1] + g, k - od.org[2] + g);
      s.mask = 0;
      return true;
    }
    if (rel != 1) {
      err = "a refinement stencil reaches a block two levels away or a coarser block";
      return false;
    }
    const int64_t li = (i << r[0]) - od.org[0], lj = (j << r[1]) - od.org[1],
                  lk = (k << r[2]) - od.org[2];
    const int64_t lq[3] = {li, lj, lk};
    for (int x = 0; x < 3; x++) {
      const bool bad = x == d ? (lq[x] < 0 || lq[x] > od.n[x]) : (lq[x] < 0 || lq[x] + r[x] >= od.n[x]);
      if (bad) {
        err = "refined blocks must start and end on coarse cell boundaries";
        return false;
      }
    }
    s.loc = local_index(oi, li + g, lj + g, lk + g);
    s.mask = (r[0] | (r[1] << 1) | (r[2] << 2)) & ~(1 << d);
    return true;
  }
};

// The ghost lists of one block (samples numbered from 0 within the block).
struct BlockOps {
  std::vector<GhostOp> ops[4];
  std::vector<AmrOp> aops[4];
  std::vector<AmrSample> samples;
  std::vector<uint8_t> samp_kind;
  int rc = GRMHD_OK;
  std::string err;
};

static int block_ops(const Plan& p, int b, BlockOps& out) {
  const int g = p.d.n_ghost;
  auto fail = [&](int code, const std::string& msg) {
    out.rc = code;
    out.err = msg;
    return code;
  };
  auto add_sample = [&](const AmrSample& s, int kind) {
    out.samples.push_back(s);
    out.samp_kind.push_back((uint8_t)kind);
  };
  const bool polar = p.d.bc[2] == GRMHD_BC_POLAR;
  {
    const BlockInfo& bi = p.info[b];
    const grmhd_block_desc& bd = p.blocks[b];
    Resolver R{p, b, std::string()};
    int64_t N[3];
    level_extent(p, bd.lev, N);
    for (int kind = 0; kind < 4; kind++) {
      for (int K = 0; K < bi.np[2]; K++)
        for (int J = 0; J < bi.np[1]; J++)
          for (int I = 0; I < bi.np[0]; I++) {
            const int L3[3] = {I, J, K};
            bool ghost = false;
            for (int dd = 0; dd < 3; dd++) {
              const int hi = (kind == dd + 1) ? g + bi.n[dd] : g + bi.n[dd] - 1;
              if (L3[dd] < g || L3[dd] > hi) ghost = true;
            }
            if (!ghost || !ghost_read(bi, g, kind, L3)) continue;
            int64_t gi = bd.org[0] + I - g, gj = bd.org[1] + J - g, gk = bd.org[2] + K - g;
            const bool across_pole = polar && (kind == 2 ? (gj < 0 || gj > N[1]) : (gj < 0 || gj >= N[1]));
            int flags = 0;
            const bool nz = compose(p.d, N, kind, gi, gj, gk, flags);
            const int32_t dst_loc = local_index(bi, I, J, K);
            if (!nz) {   // a polar-axis face: identically zero, no source
              GhostOp op{b, dst_loc, b | (GF_ZERO << 24), 0};
              out.ops[kind].push_back(op);
              continue;
            }
            // the block this value comes from at the block's own level
            const int src = kind == 0 ? owner_at(p, bd.lev, gi, gj, gk)
                                      : face_owner(p, bd.lev, N, kind, gi, gj, gk, b);
            int r[3];
            const int rel = relation(p, src, bd.lev, r);
            if (rel == 2) return fail(GRMHD_EINVAL, "neighbouring blocks differ by more than one refinement level");
            if (rel != 0 && across_pole)
              return fail(GRMHD_EUNSUPPORTED, "refinement jumps across the polar axis are not supported");
            if (rel == 0) {
              const grmhd_block_desc& sd = p.blocks[src];
              const BlockInfo& si = p.info[src];
              GhostOp op;
              op.dst_blk = b;
              op.dst_loc = dst_loc;
              op.src_blkf = src | ((flags | time_flags(p, src, b)) << 24);
              op.src_loc = local_index(si, gi - sd.org[0] + g, gj - sd.org[1] + g, gk - sd.org[2] + g);
              out.ops[kind].push_back(op);
              continue;
            }
            AmrOp op;
            op.dst_blk = b;
            op.dst_loc = dst_loc;
            op.samp = (int32_t)out.samples.size();
            op.mode = flags << AM_FLAGS_SHIFT;
            AmrSample s;
            if (rel == 1) {   // restriction of a finer neighbour
              const bool ok = kind == 0 ? R.cell_sample(bd.lev, gi, gj, gk, 0, s)
                                        : R.face_sample(bd.lev, N, kind, gi, gj, gk, false, 0, s);
              if (!ok) return fail(GRMHD_EINVAL, R.err);
              add_sample(s, kind);
              out.aops[kind].push_back(op);
              continue;
            }
            // prolongation from a coarser neighbour at levels mu
            const int32_t mu[3] = {bd.lev[0] + r[0], bd.lev[1] + r[1], bd.lev[2] + r[2]};
            int64_t M[3];
            level_extent(p, mu, M);
            const int pr[3] = {-r[0], -r[1], -r[2]};
            const int64_t q[3] = {gi, gj, gk};
            int64_t c[3];
            for (int x = 0; x < 3; x++) {
              c[x] = q[x] >> pr[x];
              if (pr[x]) op.mode |= 1 << x;
            }
            if (kind == 0) {
              for (int x = 0; x < 3; x++)
                if (pr[x] && (q[x] & 1)) op.mode |= 1 << (AM_UPPER_SHIFT + x);
              if (!R.cell_sample(mu, c[0], c[1], c[2], 0, s)) return fail(GRMHD_EINVAL, R.err);
              add_sample(s, kind);
              for (int x = 0; x < 3; x++) {
                if (!pr[x]) continue;
                for (int sg = -1; sg <= 1; sg += 2) {
                  int64_t t[3] = {c[0], c[1], c[2]};
                  t[x] += sg;
                  int fl = 0;
                  compose(p.d, M, 0, t[0], t[1], t[2], fl);
                  if (!R.cell_sample(mu, t[0], t[1], t[2], fl, s)) return fail(GRMHD_EINVAL, R.err);
                  add_sample(s, kind);
                }
              }
            } else {
              const int d = kind - 1;
              for (int x = 0; x < 3; x++)
                if (x != d && pr[x] && (q[x] & 1)) op.mode |= 1 << (AM_UPPER_SHIFT + x);
              const bool two = pr[d] && (q[d] & 1);
              if (two) op.mode |= AM_TWO;
              const int nst = two ? 2 : 1;
              for (int st = 0; st < nst; st++) {
                int64_t f0[3] = {c[0], c[1], c[2]};
                if (pr[d]) f0[d] = (q[d] >> 1) + st;   // the coarse faces bounding the cut cell
                else f0[d] = q[d];
                for (int m = -1; m < 6; m++) {
                  // m = -1: the coarse face; then (minus, plus) per prolonged transverse dim
                  int x = -1, sg = 0;
                  if (m >= 0) {
                    x = m / 2;
                    sg = (m & 1) ? 1 : -1;
                    if (x == d || !pr[x]) continue;
                  }
                  int64_t t[3] = {f0[0], f0[1], f0[2]};
                  if (x >= 0) t[x] += sg;
                  int fl = 0;
                  const bool fz = !compose(p.d, M, kind, t[0], t[1], t[2], fl);
                  if (!R.face_sample(mu, M, kind, t[0], t[1], t[2], fz, fl, s))
                    return fail(GRMHD_EINVAL, R.err);
                  add_sample(s, kind);
                }
              }
            }
            out.aops[kind].push_back(op);
          }
    }
  }
  return GRMHD_OK;
}

int build_ops(Plan& p) {
  const int nb = p.d.n_blocks;
  // blocks on worker threads; their lists are then laid out by the destination block's
  // time level and block order within a level (what the level launches take), with
  // the samples in block order (the lists do not depend on the threads)
  std::vector<BlockOps> per(nb);
  parallel_for(nb, [&](int64_t b) { block_ops(p, (int)b, per[b]); });
  for (const BlockOps& o : per)
    if (o.rc) return fail(o.rc, o.err);
  std::vector<int> order(nb);
  for (int b = 0; b < nb; b++) order[b] = b;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return p.blocks[x].lat < p.blocks[y].lat; });
  std::vector<size_t> at[4], aat[4], sat(nb);
  size_t stot = 0;
  for (int b = 0; b < nb; b++) {
    sat[b] = stot;
    stot += per[b].samples.size();
  }
  if (stot >= (size_t(1) << 31)) return fail(GRMHD_EINVAL, "too many refinement samples");
  for (int k = 0; k < 4; k++) {
    at[k].assign(nb, 0);
    aat[k].assign(nb, 0);
    size_t t = 0, u = 0;
    for (int b : order) {
      at[k][b] = t;
      aat[k][b] = u;
      t += per[b].ops[k].size();
      u += per[b].aops[k].size();
    }
    p.ops[k].clear();
    p.aops[k].clear();
    p.ops[k].resize(t);
    p.aops[k].resize(u);
  }
  p.samples.clear();
  p.samp_kind.clear();
  p.samples.resize(stot);
  p.samp_kind.resize(stot);
  parallel_for(nb, [&](int64_t b) {
    BlockOps& o = per[b];
    for (int k = 0; k < 4; k++) {
      std::copy(o.ops[k].begin(), o.ops[k].end(), p.ops[k].begin() + at[k][b]);
      AmrOp* dst = p.aops[k].data() + aat[k][b];
      for (AmrOp op : o.aops[k]) {
        op.samp += (int32_t)sat[b];
        *dst++ = op;
      }
    }
    std::copy(o.samples.begin(), o.samples.end(), p.samples.begin() + sat[b]);
    std::copy(o.samp_kind.begin(), o.samp_kind.end(), p.samp_kind.begin() + sat[b]);
    o = BlockOps();
  });
  return GRMHD_OK;
}

// The device form of the ghost copy lists: per time level, every ghost cell with the
// ghost faces at its local index that are plain copies from the same source element
// (same source block and local index, no flip, no zero, the same time relation), and
// the faces not carried that way.  Element indices are resolved against the block table.
struct DevGhosts {
  std::vector<GhostCF> cf;
  std::vector<GhostIdx> lf[4];      // lf[1..3]
  std::vector<int64_t> off[4];      // per level (+1): cf, lf[1..3]
};

static GhostIdx ghost_idx(const Plan& p, int kind, const GhostOp& op) {
  const BlockInfo& d = p.info[op.dst_blk];
  const BlockInfo& s = p.info[op.src_blkf & 0xFFFFFF];
  const int64_t nv = kind == 0 ? 5 : 3, cv = kind == 0 ? 0 : kind - 1;
  GhostIdx g;
  g.dst = (uint32_t)(nv * d.off + cv * d.vol + op.dst_loc);
  g.src = (uint32_t)(nv * s.off + cv * s.vol + op.src_loc);
  g.dvol = (uint32_t)d.vol;
  g.svol_fl = (uint32_t)s.vol | ((uint32_t)(op.src_blkf >> 24) & 0xFFu) << 24;
  return g;
}

static void device_ghosts(const Plan& p, DevGhosts& g) {
  const int L = std::max<int>(1, (int)p.ops_off[0].size() - 1);
  for (int k = 0; k < 4; k++) g.off[k].assign(1, 0);
  g.cf.reserve(p.ops[0].size());
  for (int l = 0; l < L; l++) {
    const int64_t c0 = p.ops_off[0].empty() ? 0 : p.ops_off[0][l];
    const int64_t c1 = p.ops_off[0].empty() ? (int64_t)p.ops[0].size() : p.ops_off[0][l + 1];
    int64_t j[4], je[4];
    for (int k = 1; k < 4; k++) {
      j[k] = p.ops_off[k].empty() ? 0 : p.ops_off[k][l];
      je[k] = p.ops_off[k].empty() ? (int64_t)p.ops[k].size() : p.ops_off[k][l + 1];
    }
    // within a level the lists run in block order and, per block, in increasing local
    // index: a merge by (block, local index)
    auto before = [](const GhostOp& a, const GhostOp& b) {
      return a.dst_blk != b.dst_blk ? a.dst_blk < b.dst_blk : a.dst_loc < b.dst_loc;
    };
    constexpr int kTime = GF_SLOW | GF_FAST;
    for (int64_t i = c0; i < c1; i++) {
      const GhostOp& c = p.ops[0][i];
      const int cfl = (c.src_blkf >> 24) & 0xFF;
      int fc = 0;
      for (int k = 1; k < 4; k++) {
        while (j[k] < je[k] && before(p.ops[k][j[k]], c)) g.lf[k].push_back(ghost_idx(p, k, p.ops[k][j[k]++]));
        if (j[k] < je[k]) {
          const GhostOp& f = p.ops[k][j[k]];
          const int ffl = (f.src_blkf >> 24) & 0xFF;
          if (f.dst_blk == c.dst_blk && f.dst_loc == c.dst_loc &&
              (f.src_blkf & 0xFFFFFF) == (c.src_blkf & 0xFFFFFF) && f.src_loc == c.src_loc &&
              (ffl & ~kTime) == 0 && (ffl & kTime) == (cfl & kTime)) {
            fc |= 1 << (k - 1);
            j[k]++;
          }
        }
      }
      const BlockInfo& d = p.info[c.dst_blk];
      const BlockInfo& s = p.info[c.src_blkf & 0xFFFFFF];
      GhostCF x;
      x.dp = (uint32_t)(5 * d.off + c.dst_loc);
      x.sp = (uint32_t)(5 * s.off + c.src_loc);
      x.db = (uint32_t)(3 * d.off + c.dst_loc);
      x.sb = (uint32_t)(3 * s.off + c.src_loc);
      x.dvol_fc = (uint32_t)d.vol | (uint32_t)fc << 24;
      x.svol_fl = (uint32_t)s.vol | (uint32_t)cfl << 24;
      g.cf.push_back(x);
    }
    for (int k = 1; k < 4; k++)
      while (j[k] < je[k]) g.lf[k].push_back(ghost_idx(p, k, p.ops[k][j[k]++]));
    g.off[0].push_back((int64_t)g.cf.size());
    for (int k = 1; k < 4; k++) g.off[k].push_back((int64_t)g.lf[k].size());
  }
}

// The old-state elements of each time level: every source of a ghost op or refinement
// sample read with GF_SLOW (for a restriction, each averaged sub-element), grouped by
// the source block's time level.
void build_slow(Plan& p) {
  const int L = p.nlev;
  std::vector<std::vector<uint32_t>> sc(L), sf(L);
  auto take = [&](int kind, int b, int64_t loc) {
    const BlockInfo& bi = p.info[b];
    if (kind == 0) {
      for (int v = 0; v < 5; v++) sc[bi.lat].push_back((uint32_t)(5 * bi.off + v * bi.vol + loc));
    } else {
      sf[bi.lat].push_back((uint32_t)(3 * bi.off + (kind - 1) * bi.vol + loc));
    }
  };
  for (int kind = 0; kind < 4; kind++)
    for (const GhostOp& op : p.ops[kind]) {
      const int fl = (op.src_blkf >> 24) & 0xFF;
      if ((fl & GF_SLOW) && !(fl & GF_ZERO)) take(kind, op.src_blkf & 0xFFFFFF, op.src_loc);
    }
  for (size_t i = 0; i < p.samples.size(); i++) {
    const AmrSample& s = p.samples[i];
    const int fl = (s.blkf >> 24) & 0xFF;
    if (!(fl & GF_SLOW) || (fl & GF_ZERO)) continue;
    const int b = s.blkf & 0xFFFFFF;
    const BlockInfo& bi = p.info[b];
    const int n0 = (s.mask & 1) ? 2 : 1, n1 = (s.mask & 2) ? 2 : 1, n2 = (s.mask & 4) ? 2 : 1;
    for (int ok = 0; ok < n2; ok++)
      for (int oj = 0; oj < n1; oj++)
        for (int oi = 0; oi < n0; oi++)
          take(p.samp_kind[i], b, s.loc + ((int64_t)ok * bi.np[1] + oj) * bi.np[0] + oi);
  }
  p.slow_c.clear();
  p.slow_f.clear();
  p.slow_c_off.assign(L + 1, 0);
  p.slow_f_off.assign(L + 1, 0);
  // the lists of each level and kind sorted side by side (independent of each other)
  parallel_for(2 * L, [&](int64_t t) {
    std::vector<uint32_t>& v = (t & 1) ? sf[t >> 1] : sc[t >> 1];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  });
  for (int l = 0; l < L; l++) {
    for (int w = 0; w < 2; w++) {
      const std::vector<uint32_t>& v = w ? sf[l] : sc[l];
      std::vector<uint32_t>& out = w ? p.slow_f : p.slow_c;
      out.insert(out.end(), v.begin(), v.end());
    }
    p.slow_c_off[l + 1] = (int64_t)p.slow_c.size();
    p.slow_f_off[l + 1] = (int64_t)p.slow_f.size();
  }
}

// ------------------------------------------------------------------ synchronisation

static bool periodic_dim(const Plan& p, int d) {
  return d == 2 || p.d.bc[2 * d] == GRMHD_BC_PERIODIC;
}

// The block holding cell x of the grid at levels lam; positions outside the grid wrap
// across periodic boundaries; -1 beyond an outflow or polar boundary.
static int holder(const Plan& p, const int32_t* lam, const int64_t x[3]) {
  int64_t N[3], y[3];
  level_extent(p, lam, N);
  for (int d = 0; d < 3; d++) {
    if (x[d] >= 0 && x[d] < N[d]) {
      y[d] = x[d];
      continue;
    }
    if (!periodic_dim(p, d)) return -1;
    y[d] = imod(x[d], N[d]);
  }
  return owner_at(p, lam, y[0], y[1], y[2]);
}

// The elements of block D covering the element at position pos of levels lam (kind 0 a
// cell, 1 a face with normal a, 2 an edge along a): one where D is as fine or coarser,
// two or four sub-elements where it is finer (z slowest, x fastest).  Returns their
// count, or -1 if one lies outside D or off D's lattice.
static int cover(const Plan& p, int D, const int32_t* lam, const int64_t pos[3], int kind, int a,
                 int32_t out[4]) {
  const grmhd_block_desc& bd = p.blocks[D];
  const BlockInfo& bi = p.info[D];
  const int g = p.d.n_ghost;
  int64_t N[3];
  level_extent(p, bd.lev, N);
  int64_t loc[3][2];
  int nv[3];
  for (int d = 0; d < 3; d++) {
    const int diff = bd.lev[d] - lam[d];
    const bool node = (kind == 1 && d == a) || (kind == 2 && d != a);
    int64_t v[2];
    if (node) {
      if (diff >= 0) {
        v[0] = pos[d] << diff;
      } else {
        if (pos[d] & 1) return -1;
        v[0] = pos[d] >> 1;
      }
      nv[d] = 1;
    } else if (diff > 0) {
      v[0] = pos[d] << 1;
      v[1] = v[0] + 1;
      nv[d] = 2;
    } else {
      v[0] = pos[d] >> (-diff);
      nv[d] = 1;
    }
    const int64_t hi = bd.org[d] + bd.n[d] + (node ? 1 : 0);
    for (int q = 0; q < nv[d]; q++) {
      const int64_t cand[3] = {v[q], v[q] - N[d], v[q] + N[d]};
      const int nc = periodic_dim(p, d) ? 3 : 1;
      int64_t got = -1;
      for (int c = 0; c < nc && got < 0; c++)
        if (cand[c] >= bd.org[d] && cand[c] < hi) got = cand[c];
      if (got < 0) return -1;
      loc[d][q] = got - bd.org[d] + g;
    }
  }
  int n = 0;
  for (int k = 0; k < nv[2]; k++)
    for (int j = 0; j < nv[1]; j++)
      for (int i = 0; i < nv[0]; i++) out[n++] = local_index(bi, loc[0][i], loc[1][j], loc[2][k]);
  return n;
}

// fastest, then finest, then lowest index
static bool dominates(const Plan& p, int x, int y) {
  const grmhd_block_desc &a = p.blocks[x], &b = p.blocks[y];
  const int la = a.lev[0] + a.lev[1] + a.lev[2], lb = b.lev[0] + b.lev[1] + b.lev[2];
  if (a.lat != b.lat) return a.lat < b.lat;
  if (la != lb) return la > lb;
  return x < y;
}

// Refinement faces between blocks of one time level: a block one level finer (in some
// dimensions, equal in the others) touching a coarse block across a face.
static void find_links(Plan& p) {
  const int nb = p.d.n_blocks;
  p.links.clear();
  if (!p.refined) return;
  for (int c = 0; c < nb; c++) {
    const grmhd_block_desc& bc = p.blocks[c];
    int64_t Nc[3];
    level_extent(p, bc.lev, Nc);
    for (int f = 0; f < nb; f++) {
      const grmhd_block_desc& bf = p.blocks[f];
      int e[3], any = 0, ok = 1;
      for (int x = 0; x < 3; x++) {
        e[x] = bf.lev[x] - bc.lev[x];
        if (e[x] < 0 || e[x] > 1) ok = 0;
        any |= e[x];
      }
      if (!ok || !any) continue;
      int64_t lo_f[3], hi_f[3], lo_c[3], hi_c[3];
      for (int x = 0; x < 3; x++) {
        lo_f[x] = bf.org[x] >> e[x];
        hi_f[x] = (bf.org[x] + bf.n[x]) >> e[x];
        lo_c[x] = bc.org[x];
        hi_c[x] = bc.org[x] + bc.n[x];
      }
      for (int d = 0; d < 3; d++) {
        bool overlap = true;
        for (int x = 0; x < 3; x++)
          if (x != d && std::max(lo_f[x], lo_c[x]) >= std::min(hi_f[x], hi_c[x])) overlap = false;
        if (!overlap) continue;
        const bool per = periodic_dim(p, d);
        const bool below = hi_f[d] == lo_c[d] || (per && lo_c[d] == 0 && hi_f[d] == Nc[d]);
        const bool above = hi_c[d] == lo_f[d] || (per && lo_f[d] == 0 && hi_c[d] == Nc[d]);
        for (int side = 0; side < 2; side++) {
          if (!(side == 0 ? below : above) || bc.lat != bf.lat) continue;
          Plan::Link L;
          L.c = c;
          L.f = f;
          L.d = d;
          L.side = side;
          for (int x = 0; x < 3; x++) {
            L.e[x] = e[x];
            L.lo[x] = std::max(lo_f[x], lo_c[x]);
            L.hi[x] = std::min(hi_f[x], hi_c[x]);
          }
          p.links.push_back(L);
        }
      }
    }
  }
}

// The reflux faces, sync edges and stage edges of every block (see Plan).
static int sync_tables(Plan& p) {
  const int nb = p.d.n_blocks;
  const bool polar = p.d.bc[2] == GRMHD_BC_POLAR;
  p.reflux.clear();
  p.sync_edges.clear();
  p.stage_edges.clear();
  if (!p.refined && p.nlev == 1) return GRMHD_OK;   // one level of each kind: nothing shared
  for (int b = 0; b < nb; b++) {
    const grmhd_block_desc& bb = p.blocks[b];
    const int32_t* lam = bb.lev;
    int64_t N[3];
    level_extent(p, lam, N);
    const int64_t* o = bb.org;
    const int32_t* n = bb.n;
    for (int d = 0; d < 3; d++) {
      const int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
      for (int side = 0; side < 2; side++) {
        const int64_t pl = o[d] + (side ? n[d] : 0);
        if (d == 1 && polar && (pl == 0 || pl == N[1])) continue;   // the axis carries no flux
        for (int64_t c1 = o[t1]; c1 < o[t1] + n[t1]; c1++)
          for (int64_t c0 = o[t0]; c0 < o[t0] + n[t0]; c0++) {
            int64_t cell[3];
            cell[d] = side ? pl : pl - 1;
            cell[t0] = c0;
            cell[t1] = c1;
            const int D = holder(p, lam, cell);
            if (D < 0 || p.blocks[D].lat >= bb.lat) continue;
            int64_t pos[3] = {cell[0], cell[1], cell[2]};
            pos[d] = pl;
            Plan::Reflux r;
            int32_t mine[4];
            if (cover(p, b, lam, pos, 1, d, mine) != 1) return fail(GRMHD_EINVAL, "planner: a block face outside its block");
            r.b = b;
            r.d = d;
            r.side = side;
            r.loc = mine[0];
            r.D = D;
            for (int q = 0; q < 4; q++) r.sub[q] = -1;
            r.n = cover(p, D, lam, pos, 1, d, r.sub);
            if (r.n < 1) return fail(GRMHD_EINVAL, "planner: a shared face off the faster block's lattice");
            p.reflux.push_back(r);
          }
      }
    }
    for (int a = 0; a < 3; a++) {
      const int t0 = a == 0 ? 1 : 0, t1 = a == 2 ? 1 : 2;
      for (int64_t x1 = o[t1]; x1 <= o[t1] + n[t1]; x1++)
        for (int64_t x0 = o[t0]; x0 <= o[t0] + n[t0]; x0++) {
          const bool on0 = x0 == o[t0] || x0 == o[t0] + n[t0];
          const bool on1 = x1 == o[t1] || x1 == o[t1] + n[t1];
          if (!on0 && !on1) continue;
          if (polar && (t0 == 1 || t1 == 1)) {
            const int64_t xt = t0 == 1 ? x0 : x1;
            if (xt == 0 || xt == N[1]) continue;   // on the axis E1 = E3 = 0
          }
          for (int64_t ca = o[a]; ca < o[a] + n[a]; ca++) {
            int hs[4], nh = 0;
            for (int64_t q0 = x0 - 1; q0 <= x0; q0++)
              for (int64_t q1 = x1 - 1; q1 <= x1; q1++) {
                int64_t cell[3];
                cell[a] = ca;
                cell[t0] = q0;
                cell[t1] = q1;
                const int h = holder(p, lam, cell);
                if (h < 0) continue;
                const int32_t* hl = p.blocks[h].lev;
                if ((hl[t0] < lam[t0] && (x0 & 1)) || (hl[t1] < lam[t1] && (x1 & 1))) continue;
                bool dup = false;
                for (int q = 0; q < nh; q++) dup |= hs[q] == h;
                if (!dup) hs[nh++] = h;
              }
            if (nh == 0) continue;
            int64_t pos[3];
            pos[a] = ca;
            pos[t0] = x0;
            pos[t1] = x1;
            int32_t mine[4];
            if (cover(p, b, lam, pos, 2, a, mine) != 1) return fail(GRMHD_EINVAL, "planner: a block edge outside its block");
            int Ds = -1, Da = -1;
            for (int q = 0; q < nh; q++) {
              if (p.blocks[hs[q]].lat == bb.lat && (Ds < 0 || dominates(p, hs[q], Ds))) Ds = hs[q];
              if (Da < 0 || dominates(p, hs[q], Da)) Da = hs[q];
            }
            auto add = [&](std::vector<Plan::EdgeRef>& v, int D) -> int {
              Plan::EdgeRef e;
              e.b = b;
              e.a = a;
              e.loc = mine[0];
              e.D = D;
              int32_t sub[4] = {-1, -1, -1, -1};
              e.n = cover(p, D, lam, pos, 2, a, sub);
              if (e.n < 1 || e.n > 2) return fail(GRMHD_EINVAL, "planner: a shared edge off the holder's lattice");
              e.sub[0] = sub[0];
              e.sub[1] = sub[1];
              v.push_back(e);
              return GRMHD_OK;
            };
            const int32_t* ld = p.blocks[Ds].lev;
            if (Ds != b && (ld[0] != lam[0] || ld[1] != lam[1] || ld[2] != lam[2]))
              if (int rc = add(p.stage_edges, Ds)) return rc;
            if (p.blocks[Da].lat < bb.lat)
              if (int rc = add(p.sync_edges, Da)) return rc;
          }
        }
    }
  }
  return GRMHD_OK;
}

static int x_range(const Plan::Link& lk, int d, int x) { return x == d ? 1 : 1 + lk.e[x]; }

// The device lists of the tables above.
static int sync_lists(Plan& p) {
  const int L = p.nlev;
  const int nb = p.d.n_blocks;
  const int g = p.d.n_ghost;
  auto lat = [&](int b) { return p.blocks[b].lat; };
  // stage corrections at one time level
  std::vector<std::vector<MeanItem>> fix(L), bs(L);
  for (const Plan::Link& lk : p.links) {
    const BlockInfo &ci = p.info[lk.c], &fi = p.info[lk.f];
    const grmhd_block_desc &cd = p.blocks[lk.c], &fd = p.blocks[lk.f];
    const int d = lk.d;
    int64_t lo[3], hi[3];
    for (int x = 0; x < 3; x++) {
      lo[x] = x == d ? 0 : lk.lo[x];
      hi[x] = x == d ? 1 : lk.hi[x];
    }
    for (int64_t ck = lo[2]; ck < hi[2]; ck++)
      for (int64_t cj = lo[1]; cj < hi[1]; cj++)
        for (int64_t ci_ = lo[0]; ci_ < hi[0]; ci_++) {
          const int64_t cg[3] = {ci_, cj, ck};
          int64_t pc[3];
          for (int x = 0; x < 3; x++) pc[x] = g + cg[x] - cd.org[x];
          pc[d] = g + (lk.side == 1 ? cd.n[d] : 0);
          MeanItem mf{}, mb{};
          mf.dst = 24 * ci.off + (int64_t)(d * 8) * ci.vol + local_index(ci, pc[0], pc[1], pc[2]);
          mb.dst = 3 * ci.off + (int64_t)d * ci.vol + local_index(ci, pc[0], pc[1], pc[2]);
          int n = 0;
          const int r0 = x_range(lk, d, 0), r1 = x_range(lk, d, 1), r2 = x_range(lk, d, 2);
          for (int ok = 0; ok < r2; ok++)
            for (int oj = 0; oj < r1; oj++)
              for (int oi = 0; oi < r0; oi++) {
                const int64_t off[3] = {oi, oj, ok};
                int64_t pf[3];
                for (int x = 0; x < 3; x++) pf[x] = g + (cg[x] << lk.e[x]) + off[x] - fd.org[x];
                pf[d] = g + (lk.side == 1 ? 0 : fd.n[d]);
                const int32_t lf = local_index(fi, pf[0], pf[1], pf[2]);
                mf.src[n] = 24 * fi.off + (int64_t)(d * 8) * fi.vol + lf;
                mb.src[n] = 3 * fi.off + (int64_t)d * fi.vol + lf;
                n++;
              }
          mf.n = mb.n = n;
          mf.ncomp = 8;
          mb.ncomp = 1;
          mf.dstride = ci.vol;
          mf.sstride = fi.vol;
          mb.dstride = mb.sstride = 0;
          mf.kind = 0;
          mb.kind = 2;
          fix[lat(lk.c)].push_back(mf);
          bs[lat(lk.c)].push_back(mb);
        }
  }
  for (const Plan::EdgeRef& e : p.stage_edges) {
    const BlockInfo &bi = p.info[e.b], &di = p.info[e.D];
    MeanItem m{};
    m.dst = 3 * bi.off + (int64_t)e.a * bi.vol + e.loc;
    for (int q = 0; q < e.n; q++) m.src[q] = 3 * di.off + (int64_t)e.a * di.vol + e.sub[q];
    m.n = e.n;
    m.ncomp = 1;
    m.kind = 1;
    fix[lat(e.b)].push_back(m);
  }
  auto flatten = [&](std::vector<std::vector<MeanItem>>& v, std::vector<MeanItem>& out,
                     std::vector<int64_t>& off) {
    out.clear();
    off.assign(L + 1, 0);
    for (int l = 0; l < L; l++) {
      out.insert(out.end(), v[l].begin(), v[l].end());
      off[l + 1] = (int64_t)out.size();
    }
  };
  flatten(fix, p.fix, p.fix_off);
  flatten(bs, p.bsync, p.bsync_off);
  // register slots: (block, component, local index) of every flux and EMF the
  // synchronisation reads, numbered by the block's time level
  auto key = [](int b, int c, int32_t loc) { return ((int64_t)b * 3 + c) << 24 | (int64_t)loc; };
  std::vector<int64_t> kf, ke;
  for (const Plan::Reflux& r : p.reflux) {
    kf.push_back(key(r.b, r.d, r.loc));
    for (int q = 0; q < r.n; q++) kf.push_back(key(r.D, r.d, r.sub[q]));
  }
  for (const Plan::EdgeRef& e : p.sync_edges) {
    ke.push_back(key(e.b, e.a, e.loc));
    for (int q = 0; q < e.n; q++) ke.push_back(key(e.D, e.a, e.sub[q]));
  }
  auto order = [&](std::vector<int64_t>& k) {
    std::sort(k.begin(), k.end(), [&](int64_t x, int64_t y) {
      const int bx = (int)((x >> 24) / 3), by = (int)((y >> 24) / 3);
      if (lat(bx) != lat(by)) return lat(bx) < lat(by);
      return x < y;
    });
    k.erase(std::unique(k.begin(), k.end()), k.end());
  };
  order(kf);
  order(ke);
  p.nregF = (int64_t)kf.size();
  p.nregE = (int64_t)ke.size();
  auto slot = [](const std::vector<int64_t>& k, int64_t x, auto&& less) -> int32_t {
    auto it = std::lower_bound(k.begin(), k.end(), x, less);
    return (int32_t)(it - k.begin());
  };
  auto lessF = [&](int64_t x, int64_t y) {
    const int bx = (int)((x >> 24) / 3), by = (int)((y >> 24) / 3);
    if (lat(bx) != lat(by)) return lat(bx) < lat(by);
    return x < y;
  };
  auto sF = [&](int b, int c, int32_t loc) { return slot(kf, key(b, c, loc), lessF); };
  auto sE = [&](int b, int c, int32_t loc) { return slot(ke, key(b, c, loc), lessF); };
  {
    std::vector<std::vector<RegItem>> rl(L);
    for (size_t i = 0; i < kf.size(); i++) {
      const int b = (int)((kf[i] >> 24) / 3), c = (int)((kf[i] >> 24) % 3);
      const int32_t loc = (int32_t)(kf[i] & 0xFFFFFF);
      const BlockInfo& bi = p.info[b];
      RegItem r{};
      r.src = 24 * bi.off + (int64_t)(c * 8) * bi.vol + loc;
      r.slot = (int32_t)i;
      r.kind = 0;
      r.stride = bi.vol;
      rl[lat(b)].push_back(r);
    }
    for (size_t i = 0; i < ke.size(); i++) {
      const int b = (int)((ke[i] >> 24) / 3), c = (int)((ke[i] >> 24) % 3);
      const int32_t loc = (int32_t)(ke[i] & 0xFFFFFF);
      const BlockInfo& bi = p.info[b];
      RegItem r{};
      r.src = 3 * bi.off + (int64_t)c * bi.vol + loc;
      r.slot = (int32_t)i;
      r.kind = 1;
      r.stride = 0;
      rl[lat(b)].push_back(r);
    }
    p.regs.clear();
    p.reg_off.assign(L + 1, 0);
    for (int l = 0; l < L; l++) {
      p.regs.insert(p.regs.end(), rl[l].begin(), rl[l].end());
      p.reg_off[l + 1] = (int64_t)p.regs.size();
    }
  }
  // the synchronisation of each slower block
  std::vector<std::vector<SyncCell>> cl(L);
  std::vector<std::vector<SyncFace>> fl(L);
  size_t ir = 0, ie = 0;
  for (int b = 0; b < nb; b++) {
    const BlockInfo& bi = p.info[b];
    const int32_t* n = bi.n;
    std::map<int32_t, std::vector<FluxTerm>> dU;   // per cell, terms in table order
    std::vector<int32_t> touched;
    std::vector<SyncFace> faces;
    std::unordered_map<int64_t, size_t> face_at;
    auto cell_terms = [&](int32_t loc) -> std::vector<FluxTerm>& { return dU[loc]; };
    auto face_of = [&](int comp, int32_t loc) -> SyncFace& {
      const int64_t k = (int64_t)comp << 32 | (uint32_t)loc;
      auto it = face_at.find(k);
      if (it != face_at.end()) return faces[it->second];
      SyncFace f{};
      f.blk = b;
      f.comp = comp;
      f.loc = loc;
      face_at[k] = faces.size();
      faces.push_back(f);
      return faces.back();
    };
    auto coords = [&](int32_t loc, int x[3]) {
      x[0] = loc % bi.np[0];
      x[1] = (loc / bi.np[0]) % bi.np[1];
      x[2] = loc / (bi.np[0] * bi.np[1]);
    };
    const size_t r0 = ir, e0 = ie;
    while (ir < p.reflux.size() && p.reflux[ir].b == b) {
      const Plan::Reflux& r = p.reflux[ir++];
      FluxTerm t{};
      t.mine = sF(b, r.d, r.loc);
      for (int q = 0; q < r.n; q++) t.th[q] = sF(r.D, r.d, r.sub[q]);
      t.nth = r.n;
      t.sgn = r.side == 1 ? 1 : -1;
      t.dx = bi.dx[r.d];
      int x[3];
      coords(r.loc, x);
      if (r.side == 1) x[r.d] -= 1;
      cell_terms(local_index(bi, x[0], x[1], x[2])).push_back(t);
    }
    auto owned = [&](int c, const int x[3]) {
      for (int e = 0; e < 3; e++)
        if (x[e] < g || x[e] > g + n[e] - (e == c ? 0 : 1)) return false;
      return true;
    };
    auto touch_face = [&](int c, const int x[3]) {
      for (int cp = x[c] - 1; cp <= x[c]; cp++)
        if (cp >= g && cp < g + n[c]) {
          int y[3] = {x[0], x[1], x[2]};
          y[c] = cp;
          touched.push_back(local_index(bi, y[0], y[1], y[2]));
        }
    };
    while (ie < p.sync_edges.size() && p.sync_edges[ie].b == b) {
      const Plan::EdgeRef& e = p.sync_edges[ie++];
      EdgeTerm t{};
      t.mine = sE(b, e.a, e.loc);
      for (int q = 0; q < e.n; q++) t.th[q] = sE(e.D, e.a, e.sub[q]);
      t.nth = e.n;
      int x[3];
      coords(e.loc, x);
      for (int pc = 0; pc < 3; pc++) {
        if (pc == e.a) continue;
        const int q = 3 - e.a - pc;
        const int sign = e.a == (pc + 1) % 3 ? 1 : -1;
        for (int w = 0; w < 2; w++) {
          int fx[3] = {x[0], x[1], x[2]};
          fx[q] = w == 0 ? x[q] - 1 : x[q];
          if (!owned(pc, fx)) continue;
          SyncFace& f = face_of(pc, local_index(bi, fx[0], fx[1], fx[2]));
          if (f.nt >= 4) return fail(GRMHD_EINVAL, "planner: more than four edges on a face");
          EdgeTerm tt = t;
          tt.sgn = sign * (w == 0 ? 1 : -1);
          tt.dx = bi.dx[q];
          f.t[f.nt++] = tt;
          touch_face(pc, fx);
        }
      }
    }
    for (size_t q = r0; q < ir; q++) {
      const Plan::Reflux& r = p.reflux[q];
      const int32_t* ld = p.blocks[r.D].lev;
      const int32_t* lb = p.blocks[b].lev;
      if (ld[0] < lb[0] || ld[1] < lb[1] || ld[2] < lb[2]) continue;   // the faster side is coarser
      SyncFace& f = face_of(r.d, r.loc);
      f.cblk = r.D;
      f.ncopy = r.n;
      for (int k = 0; k < 4; k++) f.csrc[k] = k < r.n ? r.sub[k] : 0;
      int x[3];
      coords(r.loc, x);
      touch_face(r.d, x);
    }
    if (ir == r0 && ie == e0) continue;
    std::vector<int32_t> all = touched;
    for (auto& c : dU) all.push_back(c.first);
    std::sort(all.begin(), all.end());
    all.erase(std::unique(all.begin(), all.end()), all.end());
    for (int32_t loc : all) {
      SyncCell c{};
      c.blk = b;
      c.loc = loc;
      auto d = dU.find(loc);
      if (d != dU.end()) {
        if (d->second.size() > 3) return fail(GRMHD_EINVAL, "planner: more than three reflux faces on a cell");
        c.nt = (int32_t)d->second.size();
        for (size_t k = 0; k < d->second.size(); k++) c.t[k] = d->second[k];
      }
      cl[lat(b)].push_back(c);
    }
    fl[lat(b)].insert(fl[lat(b)].end(), faces.begin(), faces.end());
  }
  p.scells.clear();
  p.sfaces.clear();
  p.scell_off.assign(L + 1, 0);
  p.sface_off.assign(L + 1, 0);
  for (int l = 0; l < L; l++) {
    p.scells.insert(p.scells.end(), cl[l].begin(), cl[l].end());
    p.sfaces.insert(p.sfaces.end(), fl[l].begin(), fl[l].end());
    p.scell_off[l + 1] = (int64_t)p.scells.size();
    p.sface_off[l + 1] = (int64_t)p.sfaces.size();
  }
  if (p.nregF >= (int64_t(1) << 31) || p.nregE >= (int64_t(1) << 31))
    return fail(GRMHD_EINVAL, "too many register elements");
  return GRMHD_OK;
}

int build_plan(const grmhd_grid_desc* desc, Plan& p, bool with_maps) {
  int rc = validate(desc);
  if (rc) return rc;
  p.d = *desc;
  p.blocks.assign(desc->blocks, desc->blocks + desc->n_blocks);
  p.d.blocks = nullptr;
  const int g = desc->n_ghost;
  const int nb = desc->n_blocks;
  for (int k = 0; k < 3; k++) p.lmax[k] = 0;
  for (int b = 0; b < nb; b++)
    for (int k = 0; k < 3; k++) p.lmax[k] = std::max(p.lmax[k], p.blocks[b].lev[k]);
  p.refined = false;
  for (int b = 0; b < nb; b++)
    for (int k = 0; k < 3; k++)
      if (p.blocks[b].lev[k] != p.lmax[k]) p.refined = true;
  // the list sizes of a refined grid, and the saved old-state elements of a grid with
  // several time levels, are only known once the lists are built
  if (p.refined || desc->n_lat_levels > 1) with_maps = true;
  // one geometry table per (x1, x2) level pair
  p.tables.clear();
  p.ncol = 0;
  p.info.resize(nb);
  int64_t off = 0;
  p.n_interior = 0;
  for (int b = 0; b < nb; b++) {
    BlockInfo& bi = p.info[b];
    const grmhd_block_desc& bd = p.blocks[b];
    int64_t N[3];
    level_extent(p, bd.lev, N);
    int t = -1;
    for (size_t q = 0; q < p.tables.size(); q++)
      if (p.tables[q].l0 == bd.lev[0] && p.tables[q].l1 == bd.lev[1]) t = (int)q;
    if (t < 0) {
      GeoTable T;
      T.l0 = bd.lev[0];
      T.l1 = bd.lev[1];
      T.ti = (int32_t)(N[0] + 2 * g + 1);
      T.tj = (int32_t)(N[1] + 2 * g + 1);
      T.base = p.ncol;
      p.ncol += (int64_t)T.ti * T.tj;
      p.tables.push_back(T);
      t = (int)p.tables.size() - 1;
    }
    bi.off = off;
    for (int k = 0; k < 3; k++) {
      bi.n[k] = bd.n[k];
      bi.np[k] = bd.n[k] + 2 * g + 1;
      p.max_np[k] = std::max(p.max_np[k], bi.np[k]);
      p.max_n[k] = std::max(p.max_n[k], bi.n[k]);
      bi.dx[k] = (desc->xmax[k] - desc->xmin[k]) / (double)N[k];
      bi.idx[k] = 1.0 / bi.dx[k];
    }
    bi.gorg[0] = (int32_t)bd.org[0];
    bi.gorg[1] = (int32_t)bd.org[1];
    bi.gorg[2] = (int32_t)bd.org[2];
    if ((int64_t)bi.np[0] * bi.np[1] * bi.np[2] >= (int64_t(1) << 24))
      return fail(GRMHD_EINVAL, "block too large (padded volume must stay below 2^24 cells)");
    bi.vol = bi.np[0] * bi.np[1] * bi.np[2];
    bi.lat = bd.lat;
    bi.gti = p.tables[t].ti;
    bi.gbase = p.tables[t].base;
    off += bi.vol;
    p.n_interior += (int64_t)bd.n[0] * bd.n[1] * bd.n[2];
  }
  p.vtot = off;
  if (p.vtot * 5 >= (int64_t(1) << 32))
    return fail(GRMHD_EINVAL, "grid too large (5 x padded cells must stay below 2^32)");
  // ownership of effective cells; every cell must be covered exactly once
  const int64_t N1 = desc->n_eff[0], N2 = desc->n_eff[1], N3 = desc->n_eff[2];
  if (N1 * N2 * N3 > (int64_t(1) << 31)) return fail(GRMHD_EINVAL, "effective grid too large");
  // The blocks' volumes must add up to the grid's; the blocks then fill the map in
  // parallel (rows of effective cells), and a cell left unfilled means that two blocks
  // overlap or that one is missing.
  int64_t vol = 0;
  for (int b = 0; b < nb; b++) {
    const grmhd_block_desc& bd = p.blocks[b];
    int64_t v = 1;
    for (int d = 0; d < 3; d++) v *= (int64_t)bd.n[d] << (p.lmax[d] - bd.lev[d]);
    vol += v;
  }
  if (vol != N1 * N2 * N3) return fail(GRMHD_EINVAL, "blocks do not tile the grid");
  p.owner.resize((size_t)(N1 * N2 * N3));
  parallel_for(N3, [&](int64_t k) {
    std::fill(p.owner.begin() + (size_t)(k * N2 * N1), p.owner.begin() + (size_t)((k + 1) * N2 * N1), -1);
  });
  parallel_for(nb, [&](int64_t b) {
    const grmhd_block_desc& bd = p.blocks[b];
    const int s0 = p.lmax[0] - bd.lev[0], s1 = p.lmax[1] - bd.lev[1], s2 = p.lmax[2] - bd.lev[2];
    const int64_t i0 = bd.org[0] << s0, i1 = (bd.org[0] + bd.n[0]) << s0;
    for (int64_t k = bd.org[2] << s2; k < (bd.org[2] + bd.n[2]) << s2; k++)
      for (int64_t j = bd.org[1] << s1; j < (bd.org[1] + bd.n[1]) << s1; j++) {
        const size_t row = (size_t)((k * N2 + j) * N1);
        std::fill(p.owner.begin() + row + i0, p.owner.begin() + row + i1, (int32_t)b);
      }
  });
  std::atomic<bool> hole{false};
  parallel_for(N3, [&](int64_t k) {
    const auto a = p.owner.begin() + (size_t)(k * N2 * N1);
    if (std::find(a, a + (size_t)(N2 * N1), -1) != a + (size_t)(N2 * N1)) hole = true;
  });
  if (hole) return fail(GRMHD_EINVAL, "blocks overlap");
  if (with_maps) {
    if ((rc = build_ops(p))) return rc;
  }
  find_links(p);
  // local time stepping tables
  p.nlev = desc->n_lat_levels;
  {
    const int L = p.nlev;
    p.lev_blocks.clear();
    p.lev_boff.assign(L + 1, 0);
    p.lev_cells.assign(L, 0);
    for (int l = 0; l < L; l++) {
      p.lev_boff[l] = (int64_t)p.lev_blocks.size();
      for (int b = 0; b < nb; b++)
        if (p.blocks[b].lat == l) {
          p.lev_blocks.push_back(b);
          p.lev_cells[l] += (int64_t)p.blocks[b].n[0] * p.blocks[b].n[1] * p.blocks[b].n[2];
        }
    }
    p.lev_boff[L] = (int64_t)p.lev_blocks.size();
    if (with_maps) {
      // the lists are ordered by the destination block's time level: offsets per level
      auto by_level = [&](const auto& v, std::vector<int64_t>& off) {
        off.assign(L + 1, 0);
        for (const auto& op : v) off[p.blocks[op.dst_blk].lat + 1]++;
        for (int l = 0; l < L; l++) off[l + 1] += off[l];
      };
      for (int kind = 0; kind < 4; kind++) {
        by_level(p.ops[kind], p.ops_off[kind]);
        by_level(p.aops[kind], p.aops_off[kind]);
      }
    }
    if (with_maps && L > 1) build_slow(p);
    // blocks that touch (across a face, an edge or a corner, and through the physical
    // boundaries) differ by at most one time level
    if (L > 1) {
      for (int b = 0; b < nb; b++) {
        const grmhd_block_desc& bd = p.blocks[b];
        int64_t N[3];
        level_extent(p, bd.lev, N);
        for (int64_t k = bd.org[2] - 1; k <= bd.org[2] + bd.n[2]; k++)
          for (int64_t j = bd.org[1] - 1; j <= bd.org[1] + bd.n[1]; j++)
            for (int64_t i = bd.org[0] - 1; i <= bd.org[0] + bd.n[0]; i++) {
              const bool in = i >= bd.org[0] && i < bd.org[0] + bd.n[0] && j >= bd.org[1] &&
                              j < bd.org[1] + bd.n[1] && k >= bd.org[2] && k < bd.org[2] + bd.n[2];
              if (in) continue;
              int64_t gi = i, gj = j, gk = k;
              int fl = 0;
              compose(p.d, N, 0, gi, gj, gk, fl);
              const int o = owner_at(p, bd.lev, gi, gj, gk);
              const int dl = p.blocks[o].lat - bd.lat;
              if (dl > 1 || dl < -1)
                return fail(GRMHD_EINVAL, "neighbouring time levels differ by more than one");
            }
      }
    }
    if ((rc = sync_tables(p))) return rc;
    if ((rc = sync_lists(p))) return rc;
    // work lists when block sizes differ (equal sizes leave no idle tiles in the grid)
    p.use_wl = false;
    for (int b = 1; b < nb; b++)
      for (int k = 0; k < 3; k++)
        if (p.blocks[b].n[k] != p.blocks[0].n[k]) p.use_wl = true;
    p.wl.clear();
    p.wl_off.clear();
    if (p.use_wl) {
      auto region = [&](int b, int cls) -> int64_t {
        const BlockInfo& bi = p.info[b];
        switch (cls) {
          case WL_BCELL: return (int64_t)(bi.np[0] - 1) * (bi.np[1] - 1) * (bi.np[2] - 1);
          case WL_EMF: return (int64_t)(bi.n[0] + 1) * (bi.n[1] + 1) * (bi.n[2] + 1);
          case WL_CELLS: return (int64_t)bi.n[0] * bi.n[1] * bi.n[2];
          case WL_EREF: return (int64_t)(bi.n[0] + 2) * (bi.n[1] + 2) * (bi.n[2] + 2);
          default: {   // faces along x^(d+1), or pairs of them
            const bool pair = cls >= WL_PAIR1;
            const int d = pair ? cls - WL_PAIR1 : cls - WL_FLUX1;
            int64_t r = 1;
            for (int e = 0; e < 3; e++)
              r *= e == d ? (pair ? (bi.n[e] + 2) / 2 : bi.n[e] + 1) : bi.n[e] + 2;
            return r;
          }
        }
      };
      for (int list = 0; list <= L; list++) {
        for (int cls = 0; cls < WL_N; cls++) {
          p.wl_off.push_back((int64_t)p.wl.size());
          const int64_t b0 = list < L ? p.lev_boff[list] : 0;
          const int64_t b1 = list < L ? p.lev_boff[list + 1] : nb;
          for (int64_t q = b0; q < b1; q++) {
            const int b = list < L ? p.lev_blocks[q] : (int)q;
            const int64_t nt = (region(b, cls) + STAGE_NT - 1) / STAGE_NT;
            for (int64_t t = 0; t < nt; t++) p.wl.push_back(make_int2(b, (int)t));
          }
        }
      }
      p.wl_off.push_back((int64_t)p.wl.size());
    }
  }
  // work-buffer layout
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
  const size_t V = (size_t)p.vtot;
  p.o_ps = take(5 * V * 8);
  p.o_balt = take(3 * V * 8);
  p.o_bc = take(3 * V * 8);
  p.o_f = take(24 * V * 8);
  p.o_e = take(3 * V * 8);
  p.o_u9 = take(9 * V * 8);
  p.o_gc = take((size_t)NGEO_C * p.ncol * 8);
  p.o_g1 = take((size_t)NGEO_F * p.ncol * 8);
  p.o_g2 = take((size_t)NGEO_F * p.ncol * 8);
  p.o_blk = take(nb * sizeof(BlockInfo));
  for (int kind = 0; kind < 4; kind++) {
    size_t count = with_maps ? p.ops[kind].size() : 0;
    if (!with_maps) {
      // the same count without building the lists: the read elements outside the
      // interior (cells, or faces on and inside the block's boundary)
      for (int b = 0; b < nb; b++) {
        const BlockInfo& bi = p.info[b];
        for (int K = 0; K < bi.np[2]; K++)
          for (int J = 0; J < bi.np[1]; J++)
            for (int I = 0; I < bi.np[0]; I++) {
              const int x[3] = {I, J, K};
              bool ghost = false;
              for (int dd = 0; dd < 3; dd++)
                if (x[dd] < g || x[dd] > g + bi.n[dd] - (kind == dd + 1 ? 0 : 1)) ghost = true;
              if (ghost && ghost_read(bi, g, kind, x)) count++;
            }
      }
    }
    // cells with their carried faces (GhostCF), or the faces left over (at most all)
    p.o_ops[kind] = take(count * (kind == 0 ? sizeof(GhostCF) : sizeof(GhostIdx)));
    p.o_aops[kind] = take(p.aops[kind].size() * sizeof(AmrOp));
  }
  p.o_samp = take(p.samples.size() * sizeof(AmrSample));
  p.o_fix = take(p.fix.size() * sizeof(MeanItem));
  p.o_bsync = take(p.bsync.size() * sizeof(MeanItem));
  p.o_wl = take(p.wl.size() * sizeof(int2));
  p.o_cnt = take(sizeof(Counters));
  const bool lat = p.nlev > 1;
  p.o_pold = take(lat ? 5 * V * 8 : 0);
  p.o_bold = take(lat ? 3 * V * 8 : 0);
  p.o_slow = take((p.slow_c.size() + p.slow_f.size()) * sizeof(uint32_t));
  p.o_regs = take(p.regs.size() * sizeof(RegItem));
  p.o_regf = take((size_t)p.nregF * 12 * 8);   // step and pair sets of six components
  p.o_rege = take((size_t)p.nregE * 2 * 8);
  p.o_scell = take(p.scells.size() * sizeof(SyncCell));
  p.o_sface = take(p.sfaces.size() * sizeof(SyncFace));
  p.o_ubuf = take(p.scells.size() * 9 * 8);
  p.o_lev = take((size_t)nb * sizeof(int32_t));
  {
    const int64_t r = (int64_t)p.max_n[0] * p.max_n[1] * p.max_n[2];
    p.slots = (r + 255) / 256 * nb;
    p.o_dtp = take((size_t)p.slots * 2 * 8);   // two per workgroup for the div B maxima
    p.o_stp = take((size_t)STAT_COPIES * NSTAT * 8);
  }
  p.total = o;
  return GRMHD_OK;
}

void build_geometry(const Plan& p, std::vector<double>& gc, std::vector<double>& g1,
                    std::vector<double>& g2) {
  const grmhd_grid_desc& d = p.d;
  const int g = d.n_ghost;
  const bool polar = d.bc[2] == GRMHD_BC_POLAR;
  gc.assign((size_t)NGEO_C * p.ncol, 0.0);
  g1.assign((size_t)NGEO_F * p.ncol, 0.0);
  g2.assign((size_t)NGEO_F * p.ncol, 0.0);
  auto mirror = [&](double x2) {
    if (polar && x2 < d.xmin[1]) return 2.0 * d.xmin[1] - x2;
    if (polar && x2 > d.xmax[1]) return 2.0 * d.xmax[1] - x2;
    return x2;
  };
  double tmp[NGEO_F], conn[40];
  for (const GeoTable& T : p.tables) {
    const int32_t lev[3] = {T.l0, T.l1, p.lmax[2]};
    int64_t N[3];
    level_extent(p, lev, N);
    const double dx1 = (d.xmax[0] - d.xmin[0]) / (double)N[0];
    const double dx2 = (d.xmax[1] - d.xmin[1]) / (double)N[1];
    for (int J = 0; J < T.tj; J++)
      for (int I = 0; I < T.ti; I++) {
        const int64_t col = T.base + (int64_t)J * T.ti + I;
        const double x1c = d.xmin[0] + (I - g + 0.5) * dx1, x1f = d.xmin[0] + (I - g) * dx1;
        const double x2c = d.xmin[1] + (J - g + 0.5) * dx2, x2f = d.xmin[1] + (J - g) * dx2;
        geometry_point(d.coords, d.spin_a, x1c, mirror(x2c), tmp, conn);
        for (int q = 0; q < NGEO_F; q++) gc[q * p.ncol + col] = tmp[q];
        for (int q = 0; q < 40; q++) gc[(CONN0 + q) * p.ncol + col] = conn[q];
        const double r = d.coords == GRMHD_KS_LOGSPH ? std::exp(x1c) : 1.0;
        gc[RHOFL * p.ncol + col] = d.rho_fl_c * std::pow(r, d.rho_fl_p);
        gc[UFL * p.ncol + col] = d.u_fl_c * std::pow(r, d.u_fl_p);
        geometry_point(d.coords, d.spin_a, x1f, mirror(x2c), tmp, nullptr);
        for (int q = 0; q < NGEO_F; q++) g1[q * p.ncol + col] = tmp[q];
        const bool axis = polar && (J == g || J == g + N[1]);
        if (axis) {
          for (int q = 0; q < NGEO_F; q++) g2[q * p.ncol + col] = 0.0;   // sqrt(-g) = 0 on the axis
          g2[ALPHA * p.ncol + col] = 1.0;
        } else {
          geometry_point(d.coords, d.spin_a, x1c, mirror(x2f), tmp, nullptr);
          for (int q = 0; q < NGEO_F; q++) g2[q * p.ncol + col] = tmp[q];
        }
      }
  }
}

}  // namespace

// ------------------------------------------------------------------------- context

enum { KC_GHOST, KC_BCELL, KC_FLUX1, KC_FLUX2, KC_FLUX3, KC_EMF, KC_UPDATE, KC_DT, KC_N };

struct grmhd_ctx {
  Plan plan;
  bool profile = false;
  std::vector<hipEvent_t> prof_ev;   // pairs (start, stop)
  std::vector<int> prof_cls;
  size_t prof_used = 0;
  Launch L;
  grmhd_buffers bufs;
  hipStream_t stream;
  double *ps, *balt, *bc, *f, *e, *dtp, *u9;
  GhostCF* cf;                 // cells with carried faces, by time level
  GhostIdx* ops[4];            // ops[1..3]: faces not carried by a cell, by time level
  std::vector<int64_t> gh_off[4];   // per time level (+1): cf for 0, ops[k] for k = 1..3
  AmrOp* aops[4];
  int64_t naops[4];
  AmrSample* samp = nullptr;
  const MeanItem *fix = nullptr, *bsync = nullptr;
  int2* wl = nullptr;
  bool b_in_alt = false;
  const void* mlp = nullptr;   // packed MLP blob when the learned guess is on
  // local time stepping
  double *pold = nullptr, *bold = nullptr, *regf = nullptr, *rege = nullptr, *ubuf = nullptr;
  const uint32_t *slow_c = nullptr, *slow_f = nullptr;
  int32_t* lev_list = nullptr;
  const RegItem* regs = nullptr;
  const SyncCell* scells = nullptr;
  const SyncFace* sfaces = nullptr;
  bool batched = false;     // LAT cycles captured as a graph
  bool per_block = false;   // one launch per block and kernel class (plain)
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipEvent_t ev0, ev1;
  // two side streams (default priority) for the x2 and x3 face fluxes, with the events
  // that fork them from the launch stream and join them back
  hipStream_t side[2] = {nullptr, nullptr};
  hipEvent_t fork_ev = nullptr, join_ev[2] = {nullptr, nullptr};
  int64_t* ext_off = nullptr;   // per-block output offsets of grmhd_extract_cells (uneven blocks)
};

// The plan of the last grmhd_sizes call, handed to grmhd_init_grid when it is called
// with the same grid structure (building the tables is the costly part of setting up a
// large refined grid).  Keyed by every descriptor field the tables depend on; the
// others are copied from the descriptor init receives.
static std::mutex g_plan_mu;
static std::vector<char> g_plan_key;
static std::unique_ptr<Plan> g_plan;

static std::vector<char> plan_key(const grmhd_grid_desc* d) {
  std::vector<char> k;
  auto put = [&](const void* x, size_t n) {
    const char* c = (const char*)x;
    k.insert(k.end(), c, c + n);
  };
  put(&d->abi_version, 4);
  put(&d->coords, 4);
  put(&d->spin_a, 8);
  put(d->xmin, 24);
  put(d->xmax, 24);
  put(d->n_eff, 12);
  put(&d->n_ghost, 4);
  put(&d->n_blocks, 4);
  put(&d->n_lat_levels, 4);
  put(&d->recon, 4);
  put(&d->riemann, 4);
  put(d->bc, 24);
  for (int b = 0; b < d->n_blocks; b++) {
    const grmhd_block_desc& bd = d->blocks[b];
    put(bd.lev, 12);
    put(&bd.lat, 4);
    put(bd.org, 24);
    put(bd.n, 12);
  }
  return k;
}

static void keep_plan(const grmhd_grid_desc* d, std::unique_ptr<Plan> p) {
  std::vector<char> k = plan_key(d);
  std::lock_guard<std::mutex> lock(g_plan_mu);
  g_plan_key.swap(k);
  g_plan = std::move(p);
}

static std::unique_ptr<Plan> take_plan(const grmhd_grid_desc* d) {
  std::vector<char> k = plan_key(d);
  std::lock_guard<std::mutex> lock(g_plan_mu);
  if (!g_plan || k != g_plan_key) return nullptr;
  g_plan_key.clear();
  return std::move(g_plan);
}

// the work lists of block list `list` (a time level, or nlev for all blocks) into L
static void set_work_lists(const grmhd_ctx* c, Launch& L, int list) {
  const Plan& p = c->plan;
  for (int cls = 0; cls < WL_N; cls++) {
    if (!p.use_wl) {
      L.wls[cls] = nullptr;
      L.nwls[cls] = 0;
      continue;
    }
    const int64_t o = p.wl_off[(size_t)list * WL_N + cls];
    L.wls[cls] = c->wl + o;
    L.nwls[cls] = (int32_t)(p.wl_off[(size_t)list * WL_N + cls + 1] - o);
  }
}

extern "C" {

int grmhd_sizes(const grmhd_grid_desc* desc, size_t* prim_elems, size_t* bface_elems,
                size_t* work_bytes) {
  std::unique_ptr<Plan> p(new Plan());
  int rc = build_plan(desc, *p, false);
  if (rc) return rc;
  if (prim_elems) *prim_elems = (size_t)p->vtot * 5;
  if (bface_elems) *bface_elems = (size_t)p->vtot * 3;
  if (work_bytes) *work_bytes = p->total;
  if (p->refined || p->nlev > 1) keep_plan(desc, std::move(p));   // built with its lists
  return GRMHD_OK;
}

int grmhd_block_layout(const grmhd_grid_desc* desc, int32_t b, int64_t* cell_offset,
                       int32_t np[3]) {
  int rc = validate(desc);
  if (rc) return rc;
  if (b < 0 || b >= desc->n_blocks) return fail(GRMHD_EINVAL, "block index out of range");
  int64_t off = 0;
  for (int q = 0; q < b; q++) {
    int64_t v = 1;
    for (int k = 0; k < 3; k++) v *= desc->blocks[q].n[k] + 2 * desc->n_ghost + 1;
    off += v;
  }
  if (cell_offset) *cell_offset = off;
  if (np)
    for (int k = 0; k < 3; k++) np[k] = desc->blocks[b].n[k] + 2 * desc->n_ghost + 1;
  return GRMHD_OK;
}

int grmhd_init_grid(const grmhd_grid_desc* desc, const grmhd_buffers* bufs, void* hip_stream,
                    grmhd_ctx** out) {
  if (!out || !bufs) return fail(GRMHD_EINVAL, "NULL argument");
  *out = nullptr;
  grmhd_ctx* c = new grmhd_ctx();
  int rc = validate(desc);
  if (!rc) {
    std::unique_ptr<Plan> kept = take_plan(desc);
    if (kept) {
      c->plan = std::move(*kept);
      c->plan.d = *desc;
      c->plan.d.blocks = nullptr;
    } else {
      rc = build_plan(desc, c->plan, true);
    }
  }
  if (rc) { delete c; return rc; }
  const Plan& p = c->plan;
  if (!bufs->prim || !bufs->bface || !bufs->work) { delete c; return fail(GRMHD_EINVAL, "NULL buffer"); }
  if (bufs->work_bytes < p.total) { delete c; return fail(GRMHD_EINVAL, "work buffer too small"); }
  if (((uintptr_t)bufs->work & 255) != 0) { delete c; return fail(GRMHD_EINVAL, "work buffer not 256-byte aligned"); }
  c->bufs = *bufs;
  c->stream = (hipStream_t)hip_stream;
  char* w = (char*)bufs->work;
  c->ps = (double*)(w + p.o_ps);
  c->balt = (double*)(w + p.o_balt);
  c->bc = (double*)(w + p.o_bc);
  c->f = (double*)(w + p.o_f);
  c->e = (double*)(w + p.o_e);
  c->dtp = (double*)(w + p.o_dtp);
  c->u9 = (double*)(w + p.o_u9);
  c->pold = (double*)(w + p.o_pold);
  c->slow_c = (const uint32_t*)(w + p.o_slow);
  c->slow_f = c->slow_c + p.slow_c.size();
  c->bold = (double*)(w + p.o_bold);
  c->regf = (double*)(w + p.o_regf);
  c->rege = (double*)(w + p.o_rege);
  c->ubuf = (double*)(w + p.o_ubuf);
  c->lev_list = (int32_t*)(w + p.o_lev);
  c->regs = (const RegItem*)(w + p.o_regs);
  c->scells = (const SyncCell*)(w + p.o_scell);
  c->sfaces = (const SyncFace*)(w + p.o_sface);
  if (desc->batched < 0 || desc->batched > 2) { delete c; return fail(GRMHD_EINVAL, "batched must be 0, 1 or 2"); }
  c->batched = desc->batched == 1;
  c->per_block = desc->batched == 0;
  std::vector<double> gc, g1, g2;
  build_geometry(p, gc, g1, g2);
  auto up = [&](size_t off, const void* src, size_t bytes) -> int {
    if (bytes == 0) return GRMHD_OK;
    HIPCHK(hipMemcpyAsync(w + off, src, bytes, hipMemcpyHostToDevice, c->stream));
    return GRMHD_OK;
  };
  if ((rc = up(p.o_gc, gc.data(), gc.size() * 8)) ||
      (rc = up(p.o_g1, g1.data(), g1.size() * 8)) ||
      (rc = up(p.o_g2, g2.data(), g2.size() * 8)) ||
      (rc = up(p.o_blk, p.info.data(), p.info.size() * sizeof(BlockInfo)))) {
    delete c;
    return rc;
  }
  // the ghost lists resolved against the block table (element indices of the packed
  // arrays); host staging kept until the stream synchronises below
  DevGhosts dg;
  device_ghosts(p, dg);
  c->cf = (GhostCF*)(w + p.o_ops[0]);
  c->ops[0] = nullptr;
  for (int k = 0; k < 4; k++) c->gh_off[k] = dg.off[k];
  if ((rc = up(p.o_ops[0], dg.cf.data(), dg.cf.size() * sizeof(GhostCF)))) {
    delete c;
    return rc;
  }
  for (int kind = 0; kind < 4; kind++) {
    if (kind) c->ops[kind] = (GhostIdx*)(w + p.o_ops[kind]);
    c->aops[kind] = (AmrOp*)(w + p.o_aops[kind]);
    c->naops[kind] = (int64_t)p.aops[kind].size();
    if ((kind && (rc = up(p.o_ops[kind], dg.lf[kind].data(), dg.lf[kind].size() * sizeof(GhostIdx)))) ||
        (rc = up(p.o_aops[kind], p.aops[kind].data(), p.aops[kind].size() * sizeof(AmrOp)))) {
      delete c;
      return rc;
    }
  }
  c->samp = (AmrSample*)(w + p.o_samp);
  c->fix = (const MeanItem*)(w + p.o_fix);
  c->bsync = (const MeanItem*)(w + p.o_bsync);
  c->wl = (int2*)(w + p.o_wl);
  if ((rc = up(p.o_wl, p.wl.data(), p.wl.size() * sizeof(int2)))) {
    delete c;
    return rc;
  }
  if ((rc = up(p.o_samp, p.samples.data(), p.samples.size() * sizeof(AmrSample))) ||
      (rc = up(p.o_fix, p.fix.data(), p.fix.size() * sizeof(MeanItem))) ||
      (rc = up(p.o_bsync, p.bsync.data(), p.bsync.size() * sizeof(MeanItem))) ||
      (rc = up(p.o_lev, p.lev_blocks.data(), p.lev_blocks.size() * sizeof(int32_t))) ||
      (rc = up(p.o_regs, p.regs.data(), p.regs.size() * sizeof(RegItem))) ||
      (rc = up(p.o_scell, p.scells.data(), p.scells.size() * sizeof(SyncCell))) ||
      (rc = up(p.o_sface, p.sfaces.data(), p.sfaces.size() * sizeof(SyncFace))) ||
      (rc = up(p.o_slow, p.slow_c.data(), p.slow_c.size() * sizeof(uint32_t))) ||
      (rc = up(p.o_slow + p.slow_c.size() * sizeof(uint32_t), p.slow_f.data(),
               p.slow_f.size() * sizeof(uint32_t)))) {
    delete c;
    return rc;
  }
  Launch& L = c->L;
  L.blk = (const BlockInfo*)(w + p.o_blk);
  L.blist = nullptr;
  L.nblk = desc->n_blocks;
  for (int k = 0; k < 3; k++) {
    L.max_np[k] = p.max_np[k];
    L.max_n[k] = p.max_n[k];
  }
  L.geo.c = (const double*)(w + p.o_gc);
  L.geo.f1 = (const double*)(w + p.o_g1);
  L.geo.f2 = (const double*)(w + p.o_g2);
  L.geo.ncol = p.ncol;
  L.ph.gam = desc->gamma_ad;
  L.ph.courant = desc->courant;
  L.ph.tol = desc->c2p_tol;
  L.ph.bsq_rho_max = desc->bsq_rho_max;
  L.ph.bsq_u_max = desc->bsq_u_max;
  L.ph.gamma_max = desc->gamma_max;
  L.ph.maxit = desc->c2p_maxit;
  L.ph.ng = desc->n_ghost;
  L.ph.floor_drift = desc->floor_frame == GRMHD_FLOOR_DRIFT;
  L.cnt = (Counters*)(w + p.o_cnt);
  L.stat_acc = (unsigned long long*)(w + p.o_stp);
  // the tallest update brick every block divides into (8 or 4 cells along x3), else none
  L.brick_upd = 0;
  for (int z : {8, 4}) {
    bool all = true;
    for (const BlockInfo& b : p.info) all = all && brick_x1(b.n, z) != 0;
    if (all) {
      L.brick_upd = z;
      break;
    }
  }
  L.stream = c->stream;
  for (int k = 0; k < 3; k++) L.var_flux[k] = 2;   // 4 waves per SIMD
  L.var_upd = 0;
  L.split_upd = 0;
  set_work_lists(c, L, p.nlev);   // the all-blocks lists
  L.wl = nullptr;
  c->profile = desc->profile != 0;
  c->mlp = desc->c2p_guess == GRMHD_GUESS_MLP ? desc->mlp_weights : nullptr;
  launch_counters_reset(L, true);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));   // host staging vectors go out of scope
  HIPCHK(hipEventCreate(&c->ev0));
  HIPCHK(hipEventCreate(&c->ev1));
  for (int k = 0; k < 2; k++) {
    HIPCHK(hipStreamCreateWithFlags(&c->side[k], hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&c->join_ev[k], hipEventDisableTiming));
  }
  HIPCHK(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
  *out = c;
  return GRMHD_OK;
}

// kernel-class timing with event pairs on the library stream (desc.profile)
static void prof_begin(grmhd_ctx* c, int cls) {
  if (!c->profile) return;
  if (c->prof_used + 2 > c->prof_ev.size()) {
    const size_t add = 512;
    for (size_t q = 0; q < add; q++) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      c->prof_ev.push_back(e);
    }
  }
  (void)hipEventRecord(c->prof_ev[c->prof_used], c->stream);
  c->prof_cls.push_back(cls);
}
static void prof_end(grmhd_ctx* c) {
  if (!c->profile || c->prof_cls.size() * 2 != c->prof_used + 2) return;
  (void)hipEventRecord(c->prof_ev[c->prof_used + 1], c->stream);
  c->prof_used += 2;
}

// the ghost lists of the blocks of one time level (lev >= 0) or of all blocks
static GhostLists ghost_lists(const grmhd_ctx* c, int lev) {
  GhostLists G;
  int64_t run = 0;
  G.ops[0] = nullptr;
  for (int k = 0; k < 4; k++) {
    const std::vector<int64_t>& off = c->gh_off[k];
    const int64_t o = lev < 0 ? 0 : off[lev];
    const int64_t n = lev < 0 ? off.back() : off[lev + 1] - o;
    if (k == 0)
      G.cf = c->cf + o;
    else
      G.ops[k] = c->ops[k] + o;
    run += n;
    G.end[k] = run;
  }
  return G;
}

// the refinement lists likewise
static AmrLists amr_lists(const grmhd_ctx* c, int lev) {
  AmrLists A;
  int64_t run = 0;
  for (int k = 0; k < 4; k++) {
    const int64_t o = lev < 0 ? 0 : c->plan.aops_off[k][lev];
    const int64_t n = lev < 0 ? c->naops[k] : c->plan.aops_off[k][lev + 1] - o;
    A.ops[k] = c->aops[k] + o;
    run += n;
    A.end[k] = run;
  }
  return A;
}

static void fill_ghosts(grmhd_ctx* c, double* P, double* B) {
  prof_begin(c, KC_GHOST);
  launch_ghosts(c->L, ghost_lists(c, -1), P, B);
  launch_amr_ghosts(c->L, amr_lists(c, -1), c->samp, P, nullptr, P, P, B, nullptr, B, B, 0.0);
  prof_end(c);
}

// The face fluxes of a stage.  The three directions read the same inputs and write
// disjoint parts of F: x1 runs on the launch stream and x2, x3 on the two side streams,
// forked and joined by events (inside a captured cycle these become parallel graph
// branches), so one direction's launch tail overlaps the others' work.  With per-class
// profiling on they run one after the other on the launch stream.
static void launch_fluxes(grmhd_ctx* c, const Launch& L, const double* Ps, const double* Bs) {
  const int recon = c->plan.d.recon, riem = c->plan.d.riemann;
  if (c->profile) {
    for (int dir = 1; dir <= 3; dir++) {
      prof_begin(c, KC_FLUX1 + dir - 1);
      launch_flux(L, dir, recon, riem, Ps, c->bc, Bs, c->f);
      prof_end(c);
    }
    return;
  }
  (void)hipEventRecord(c->fork_ev, L.stream);
  for (int k = 0; k < 2; k++) (void)hipStreamWaitEvent(c->side[k], c->fork_ev, 0);
  launch_flux(L, 1, recon, riem, Ps, c->bc, Bs, c->f);
  for (int k = 0; k < 2; k++) {
    Launch Ls = L;
    Ls.stream = c->side[k];
    launch_flux(Ls, k + 2, recon, riem, Ps, c->bc, Bs, c->f);
    (void)hipEventRecord(c->join_ev[k], c->side[k]);
    (void)hipStreamWaitEvent(L.stream, c->join_ev[k], 0);
  }
}

// Launches of the block-wise stage kernels over blocks hb[0..n) of a time level (their
// device ids at dev): batched, one launch per kernel class for all of them (work lists
// for uneven sizes); plain, one launch per block and kernel class (the paper's launch
// structure), each sized to its block.
}  // extern "C"

template <class Fn>
static void for_launches(grmhd_ctx* c, const Launch& L, const int32_t* hb, const int32_t* dev,
                         int64_t n, Fn&& fn) {
  if (!c->per_block) {
    fn(L, int64_t(-1));
    return;
  }
  for (int64_t q = 0; q < n; q++) {
    Launch Lb = L;
    Lb.blist = dev + q;
    Lb.nblk = 1;
    for (int cls = 0; cls < WL_N; cls++) {
      Lb.wls[cls] = nullptr;
      Lb.nwls[cls] = 0;
    }
    const BlockInfo& bi = c->plan.info[hb[q]];
    for (int k = 0; k < 3; k++) {
      Lb.max_n[k] = bi.n[k];
      Lb.max_np[k] = bi.np[k];
    }
    fn(Lb, q);
  }
}

extern "C" {

// The kernels of one stage over the blocks of a time level (lev, or all blocks for a
// grid without time levels): cell-centred field, face fluxes, EMFs, the same-level
// refinement corrections, the update, the coarse copies of refinement faces.  With
// dt_part the corrector also leaves the next Courant step's per-workgroup minima, a
// segment of dt_partials / blocks per block in the plain launch structure.
static void stage_kernels(grmhd_ctx* c, const Launch& L, int lev, const double* Pn,
                          const double* Bn, const double* Ps, const double* Bs, double factor,
                          double* Pout, double* Bout, double* dt_part) {
  const Plan& p = c->plan;
  const int lv = lev < 0 ? 0 : lev;
  const int32_t* hb = p.lev_blocks.data() + p.lev_boff[lv];
  const int32_t* dev = c->lev_list + p.lev_boff[lv];
  const int64_t nb = p.lev_boff[lv + 1] - p.lev_boff[lv];
  const int64_t fo = p.fix_off[lv], nfix = p.fix_off[lv + 1] - fo;
  const int64_t bo = p.bsync_off[lv], nbs = p.bsync_off[lv + 1] - bo;
  const int recon = p.d.recon, riem = p.d.riemann;
  prof_begin(c, KC_BCELL);
  for_launches(c, L, hb, dev, nb, [&](const Launch& Lb, int64_t) { launch_bcell(Lb, Bs, c->bc); });
  prof_end(c);
  if (c->per_block) {
    for_launches(c, L, hb, dev, nb, [&](const Launch& Lb, int64_t) {
      for (int dir = 1; dir <= 3; dir++) launch_flux(Lb, dir, recon, riem, Ps, c->bc, Bs, c->f);
    });
  } else {
    launch_fluxes(c, L, Ps, Bs);
  }
  prof_begin(c, KC_EMF);
  // upwinded EMFs read the cells' own-state EMFs and densities, kept in the split
  // update's buffer (9 V per block, not in use until the update) as 4 V per block
  const double* eref = p.d.emf == GRMHD_EMF_UPWIND ? c->u9 : nullptr;
  if (eref)
    for_launches(c, L, hb, dev, nb,
                 [&](const Launch& Lb, int64_t) { launch_emf_ref(Lb, Ps, c->bc, c->u9); });
  for_launches(c, L, hb, dev, nb,
               [&](const Launch& Lb, int64_t) { launch_emf(Lb, c->f, c->e, eref); });
  launch_means(L, c->fix + fo, nfix, c->f, c->e);
  prof_end(c);
  prof_begin(c, KC_UPDATE);
  if (dt_part && c->per_block) launch_fill(L, dt_part, dt_partials(L), INFINITY);
  const int64_t seg = dt_partials(L) / (L.nblk > 0 ? L.nblk : 1);
  for_launches(c, L, hb, dev, nb, [&](const Launch& Lb, int64_t q) {
    double* part = dt_part && q >= 0 ? dt_part + q * seg : dt_part;
    launch_update(Lb, Pn, Bn, Ps, c->bc, c->f, c->e, factor, Pout, Bout, part, c->mlp, c->u9);
  });
  prof_end(c);
  if (nbs > 0) {
    prof_begin(c, KC_GHOST);
    launch_means(L, c->bsync + bo, nbs, Bout, Bout);
    prof_end(c);
  }
}

static void stage(grmhd_ctx* c, const double* Pn, const double* Bn, const double* Ps,
                  const double* Bs, double factor, double* Pout, double* Bout, double* dt_part) {
  stage_kernels(c, c->L, -1, Pn, Bn, Ps, Bs, factor, Pout, Bout, dt_part);
}

// one block level of a substep: predictor and corrector with time-aware ghosts, then the
// flux/EMF registers and the face field copied back from the stage buffer
static void lat_level_step(grmhd_ctx* c, const Launch& base, int lev, int s) {
  const Plan& p = c->plan;
  Launch L = base;
  L.blist = c->lev_list + p.lev_boff[lev];
  L.nblk = (int32_t)(p.lev_boff[lev + 1] - p.lev_boff[lev]);
  set_work_lists(c, L, lev);
  if (L.nblk == 0) return;
  double* P = c->bufs.prim;
  double* B = c->bufs.bface;
  const double scale = std::ldexp(1.0, lev);
  const double period = std::ldexp(1.0, lev + 1);
  const double t0 = s - std::fmod((double)s, period);
  const double w_pred = (s - t0) / period;
  const double w_corr = (s + 0.5 * scale - t0) / period;
  {
    const int64_t oc = p.slow_c_off[lev], nc = p.slow_c_off[lev + 1] - oc;
    const int64_t of = p.slow_f_off[lev], nf = p.slow_f_off[lev + 1] - of;
    launch_copy_list(L, c->slow_c + oc, nc, P, c->pold, c->slow_f + of, nf, B, c->bold);
  }
  auto ghosts = [&](double* Pdst, double* Bdst, const double* Pcur, const double* Bcur, double w) {
    prof_begin(c, KC_GHOST);
    launch_ghosts_t(L, ghost_lists(c, lev), P, c->pold, Pcur, Pdst, B, c->bold, Bcur, Bdst, w);
    launch_amr_ghosts(L, amr_lists(c, lev), c->samp, P, c->pold, Pcur, Pdst, B, c->bold, Bcur,
                      Bdst, w);
    prof_end(c);
  };
  ghosts(P, B, P, B, w_pred);
  stage_kernels(c, L, lev, P, B, P, B, 0.5 * scale, c->ps, c->balt, nullptr);   // -> ps, balt
  ghosts(c->ps, c->balt, c->ps, c->balt, w_corr);
  stage_kernels(c, L, lev, P, B, c->ps, c->balt, scale, P, c->balt, nullptr);   // -> P, balt
  launch_registers(L, c->regs + p.reg_off[lev], p.reg_off[lev + 1] - p.reg_off[lev], c->f, c->e,
                   scale, (s % (2 << lev)) == 0 ? 1 : 0, c->regf, p.nregF, c->rege, p.nregE);
  launch_copy_blocks(L, c->balt, B, 3);
}

static void lat_cycle(grmhd_ctx* c) {
  const Plan& p = c->plan;
  const Launch& L = c->L;
  const int nsub = 1 << (p.nlev - 1);
  prof_begin(c, KC_DT);
  {
    const int64_t np = launch_dt(L, c->bufs.prim, c->bufs.bface, c->dtp, true);
    const int64_t r = (int64_t)L.max_n[0] * L.max_n[1] * L.max_n[2];
    const int gridx = (int)((r + 255) / 256);
    launch_dt_final_lat(L, c->dtp, np, gridx, L.wls[WL_CELLS]);
  }
  prof_end(c);
  for (int s = 0; s < nsub; s++) {
    for (int lev = p.nlev - 1; lev >= 0; lev--)
      if (s % (1 << lev) == 0) lat_level_step(c, L, lev, s);
    // the levels whose step ends here (1 .. m, independent of each other), one launch each
    // of cells, faces and re-inversion over their concatenated lists
    int m = 0;
    while (m + 1 < p.nlev && (s + 1) % (1 << (m + 1)) == 0) m++;
    if (m > 0) {
      const int64_t co = p.scell_off[1], nc = p.scell_off[m + 1] - co;
      const int64_t fo = p.sface_off[1], nf = p.sface_off[m + 1] - fo;
      launch_sync(L, c->scells + co, nc, c->sfaces + fo, nf, c->bufs.prim, c->bufs.bface, c->regf,
                  p.nregF, c->rege, p.nregE, c->ubuf);
    }
  }
  launch_tsim_cycle(L, (double)nsub);
}

int grmhd_step(grmhd_ctx* c, int32_t n_cycles, grmhd_step_stats* stats) {
  if (!c) return fail(GRMHD_EINVAL, "NULL context");
  if (n_cycles < 0) return fail(GRMHD_EINVAL, "negative step count");
  const Launch& L = c->L;
  HIPCHK(hipEventRecord(c->ev0, c->stream));
  launch_counters_reset(L, false);
  double* P = c->bufs.prim;
  if (c->plan.nlev > 1) {
    if (c->batched && !c->profile) {
      if (!c->graph_exec) {
        // capture one LAT cycle (every launch of it) into a graph on a private stream
        if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        HIPCHK(hipStreamSynchronize(c->stream));
        Launch saved = c->L;
        c->L.stream = c->cap_stream;
        HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        lat_cycle(c);
        hipError_t e = hipStreamEndCapture(c->cap_stream, &c->graph);
        c->L = saved;
        if (e != hipSuccess) return fail(GRMHD_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        HIPCHK(hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
      }
      for (int cyc = 0; cyc < n_cycles; cyc++) HIPCHK(hipGraphLaunch(c->graph_exec, c->stream));
    } else {
      for (int cyc = 0; cyc < n_cycles; cyc++) lat_cycle(c);
    }
    fill_ghosts(c, P, c->bufs.bface);
  }
  for (int s = 0; s < (c->plan.nlev > 1 ? 0 : n_cycles); s++) {
    double* Bcur = c->b_in_alt ? c->balt : c->bufs.bface;
    double* Both = c->b_in_alt ? c->bufs.bface : c->balt;
    fill_ghosts(c, P, Bcur);
    if (s == 0) {   // the Courant step of later steps comes out of the previous corrector
      prof_begin(c, KC_DT);
      launch_dt(L, P, Bcur, c->dtp);
      launch_dt_final(L, c->dtp);
      prof_end(c);
    }
    stage(c, P, Bcur, P, Bcur, 0.5, c->ps, Both, nullptr);   // predictor to t + dt/2
    fill_ghosts(c, c->ps, Both);
    stage(c, P, Bcur, c->ps, Both, 1.0, P, Both, c->dtp);    // corrector to t + dt
    launch_tsim(L);
    launch_dt_final(L, c->dtp);
    c->b_in_alt = !c->b_in_alt;
  }
  if (c->b_in_alt) {
    launch_copy(L, c->balt, c->bufs.bface, c->plan.vtot * 3);
    c->b_in_alt = false;
  }
  fill_ghosts(c, P, c->bufs.bface);
  launch_stats_fold(L);   // the update statistics of every stage of the call
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(c->ev1, c->stream));
  double cls_ms[KC_N] = {};
  int64_t cls_n[KC_N] = {};
  if (c->profile) {
    HIPCHK(hipStreamSynchronize(c->stream));
    for (size_t q = 0; q < c->prof_cls.size(); q++) {
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, c->prof_ev[2 * q], c->prof_ev[2 * q + 1]));
      cls_ms[c->prof_cls[q]] += ms;
      cls_n[c->prof_cls[q]] += 1;
    }
    c->prof_cls.clear();
    c->prof_used = 0;
  }
  if (stats) {
    Counters h;
    HIPCHK(hipMemcpyAsync(&h, L.cnt, sizeof(Counters), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    std::memset(stats, 0, sizeof(*stats));
    const Plan& p = c->plan;
    const int64_t cells = p.n_interior;
    const int64_t eff = (int64_t)p.d.n_eff[0] * p.d.n_eff[1] * p.d.n_eff[2];
    const int64_t nsub = (int64_t)1 << (p.nlev - 1);
    int64_t real = 0;
    for (int l = 0; l < p.nlev && l < 8; l++) {
      const int64_t steps = (nsub >> l) * n_cycles;
      stats->steps_per_level[l] = steps;
      real += p.lev_cells[l] * steps;
    }
    stats->real_zone_cycles = real;
    stats->lat_eff_zone_cycles = cells * nsub * n_cycles;
    stats->amr_lat_eff_zone_cycles = eff * nsub * n_cycles;
    for (int q = 0; q < 64; q++) stats->c2p_iter_hist[q] = (int64_t)h.hist[q];
    for (int q = 0; q < 5; q++) stats->c2p_tier[q] = (int64_t)h.tier[q];
    stats->floor_hits = (int64_t)h.floors;
    stats->mlp_guesses = (int64_t)h.mlp;
    stats->dt_min = h.dt_last;
    stats->t_sim = h.t_sim;
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    stats->kernel_ms = ms;
    for (int q = 0; q < KC_N; q++) {
      stats->class_ms[q] = cls_ms[q];
      stats->class_launches[q] = cls_n[q];
    }
    stats->bad_states = (int64_t)h.bad;
    if (h.bad)
      return fail(GRMHD_ESTATE, std::to_string(h.bad) +
                                    " cell updates left a non-finite state or rho <= 0 or u <= 0");
  }
  return GRMHD_OK;
}

int grmhd_set_variants(grmhd_ctx* c, const int32_t choice[5]) {
  if (!c || !choice) return fail(GRMHD_EINVAL, "NULL argument");
  for (int k = 0; k < 3; k++)
    if (choice[k] < 0 || choice[k] >= NVAR_FLUX) return fail(GRMHD_EINVAL, "flux variant out of range");
  if (choice[3] < 0 || choice[3] >= NVAR_UPD) return fail(GRMHD_EINVAL, "update variant out of range");
  if (choice[4] != 0 && choice[4] != 1) return fail(GRMHD_EINVAL, "update form must be 0 or 1");
  for (int k = 0; k < 3; k++) c->L.var_flux[k] = choice[k];
  c->L.var_upd = choice[3];
  c->L.split_upd = choice[4];
  if (c->graph_exec) {
    (void)hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
  }
  if (c->graph) {
    (void)hipGraphDestroy(c->graph);
    c->graph = nullptr;
  }
  return GRMHD_OK;
}

int grmhd_autotune(grmhd_ctx* c, int32_t choice[5], double* ms) {
  if (!c) return fail(GRMHD_EINVAL, "NULL context");
  if (c->b_in_alt) return fail(GRMHD_ESTATE, "state not in the caller's buffers");
  Launch& L = c->L;
  double* P = c->bufs.prim;
  double* B = c->bufs.bface;
  const bool prof = c->profile;
  c->profile = false;
  fill_ghosts(c, P, B);
  launch_counters_reset(L, false);
  launch_dt(L, P, B, c->dtp);
  launch_dt_final(L, c->dtp);
  launch_bcell(L, B, c->bc);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const int reps = 3;
  auto time_it = [&](auto fn, double& out) -> int {
    fn();   // warm-up (code object load, caches)
    HIPCHK(hipEventRecord(e0, c->stream));
    for (int r = 0; r < reps; r++) fn();
    HIPCHK(hipEventRecord(e1, c->stream));
    HIPCHK(hipEventSynchronize(e1));
    float t = 0.0f;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    out = t / reps;
    return GRMHD_OK;
  };
  int rc = GRMHD_OK;
  const int recon = c->plan.d.recon, riem = c->plan.d.riemann;
  for (int dir = 1; dir <= 3 && !rc; dir++) {
    double best = 1e300;
    int arg = L.var_flux[dir - 1];
    for (int v = 0; v < NVAR_FLUX && !rc; v++) {
      L.var_flux[dir - 1] = v;
      double t = 0.0;
      rc = time_it([&] { launch_flux(L, dir, recon, riem, P, c->bc, B, c->f); }, t);
      if (ms) ms[(dir - 1) * NVAR_FLUX + v] = t;
      if (t < best) { best = t; arg = v; }
    }
    L.var_flux[dir - 1] = arg;
  }
  if (!rc) {
    launch_emf(L, c->f, c->e);
    double best = 1e300;
    int arg = L.var_upd, arg_split = L.split_upd;
    for (int sp = 0; sp < 2 && !rc; sp++)
      for (int v = 0; v < NVAR_UPD && !rc; v++) {
        L.var_upd = v;
        L.split_upd = sp;
        double t = 0.0;
        rc = time_it([&] {
          launch_update(L, P, B, P, c->bc, c->f, c->e, 0.5, c->ps, c->balt, nullptr, c->mlp,
                        c->u9);
        }, t);
        if (ms) ms[3 * NVAR_FLUX + sp * NVAR_UPD + v] = t;
        if (t < best) {
          best = t;
          arg = v;
          arg_split = sp;
        }
      }
    L.var_upd = arg;
    L.split_upd = arg_split;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->profile = prof;
  if (rc) return rc;
  launch_counters_reset(L, false);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  // a captured cycle holds the previous choices: capture again on the next step
  if (c->graph_exec) {
    (void)hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
  }
  if (c->graph) {
    (void)hipGraphDestroy(c->graph);
    c->graph = nullptr;
  }
  if (choice) {
    for (int k = 0; k < 3; k++) choice[k] = L.var_flux[k];
    choice[3] = L.var_upd;
    choice[4] = L.split_upd;
  }
  return GRMHD_OK;
}

int grmhd_cons2prim(grmhd_ctx* c, const grmhd_c2p_batch* b, void* hip_stream) {
  (void)c;
  if (!b) return fail(GRMHD_EINVAL, "NULL batch");
  if (b->n < 0) return fail(GRMHD_EINVAL, "negative batch size");
  if (b->n > 0 && (!b->U || !b->geom || !(b->guess || b->mlp_weights) || !b->prev || !b->P ||
                   !b->iters || !b->tier))
    return fail(GRMHD_EINVAL, "NULL batch array");
  if (b->maxit < 1 || b->maxit > 62 || !(b->tol > 0.0)) return fail(GRMHD_EINVAL, "bad tol/maxit");
  launch_c2p_batch(b->n, b->U, b->geom, b->guess, b->prev, b->P, b->iters, b->tier, b->gamma_ad,
                   b->tol, b->maxit, b->mlp_weights, (hipStream_t)hip_stream);
  HIPCHK(hipGetLastError());
  return GRMHD_OK;
}

int grmhd_block_dt(grmhd_ctx* c, double* dt) {
  if (!c || !dt) return fail(GRMHD_EINVAL, "NULL argument");
  if (c->b_in_alt) return fail(GRMHD_ESTATE, "state not in the caller's buffers");
  const Plan& p = c->plan;
  const Launch& L = c->L;
  const int64_t np = launch_dt(L, c->bufs.prim, c->bufs.bface, c->dtp, true);
  HIPCHK(hipGetLastError());
  std::vector<double> part(np);
  HIPCHK(hipMemcpyAsync(part.data(), c->dtp, sizeof(double) * np, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  const size_t nb = p.blocks.size();
  std::vector<double> m(nb, INFINITY);
  if (L.wls[WL_CELLS]) {
    const int64_t o = p.wl_off[(size_t)p.nlev * WL_N + WL_CELLS];
    for (int64_t i = 0; i < np; i++) {
      const int b = p.wl[o + i].x;
      m[b] = std::min(m[b], part[i]);
    }
  } else {
    const int64_t gx = np / std::max<int64_t>((int64_t)nb, 1);
    for (int64_t i = 0; i < np; i++) {
      const size_t b = (size_t)(i / gx);
      if (b < nb) m[b] = std::min(m[b], part[i]);
    }
  }
  for (size_t b = 0; b < nb; b++) dt[b] = p.d.courant * m[b];
  return GRMHD_OK;
}

int grmhd_divb(grmhd_ctx* c, double* max_abs, double* max_rel, double* field) {
  if (!c) return fail(GRMHD_EINVAL, "NULL context");
  launch_counters_reset(c->L, false);
  launch_divb(c->L, c->bufs.bface, field, c->dtp);
  HIPCHK(hipGetLastError());
  Counters h;
  HIPCHK(hipMemcpyAsync(&h, c->L.cnt, sizeof(Counters), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  double a, r;
  std::memcpy(&a, &h.divb_abs, 8);
  std::memcpy(&r, &h.divb_rel, 8);
  if (max_abs) *max_abs = a;
  if (max_rel) *max_rel = r;
  return GRMHD_OK;
}

// The boxes of a regrid: every (new block, old block) overlap, in the new block's cells,
// with the level relation checked (one level apart at most per dimension, never finer
// in one dimension and coarser in another; where the new block is coarser, the old
// block's boundaries fall on its cell faces)
static int regrid_ops(const Plan& po, const Plan& pn, std::vector<RegridOp>& ops) {
  // positions in cells of the finer of the two finest levels per dimension (the new
  // layout may add or drop a finest level: its effective grid then doubles or halves)
  int ls[3];
  for (int d = 0; d < 3; d++) {
    if ((po.d.n_eff[d] >> po.lmax[d]) != (pn.d.n_eff[d] >> pn.lmax[d]) ||
        ((int64_t)(po.d.n_eff[d] >> po.lmax[d]) << po.lmax[d]) != po.d.n_eff[d] ||
        ((int64_t)(pn.d.n_eff[d] >> pn.lmax[d]) << pn.lmax[d]) != pn.d.n_eff[d] ||
        po.d.xmin[d] != pn.d.xmin[d] || po.d.xmax[d] != pn.d.xmax[d])
      return fail(GRMHD_EINVAL, "regrid: the layouts differ in domain or in their level-0 grid");
    ls[d] = std::max(po.lmax[d], pn.lmax[d]);
  }
  if (po.d.coords != pn.d.coords || po.d.spin_a != pn.d.spin_a)
    return fail(GRMHD_EINVAL, "regrid: the layouts differ in coordinates");
  if (po.d.n_ghost < 2) return fail(GRMHD_EINVAL, "regrid needs at least two ghost layers");
  for (size_t nb = 0; nb < pn.blocks.size(); nb++) {
    const grmhd_block_desc& bn = pn.blocks[nb];
    int64_t nlo[3], nhi[3];
    for (int d = 0; d < 3; d++) {
      const int sh = ls[d] - bn.lev[d];
      nlo[d] = bn.org[d] << sh;
      nhi[d] = (bn.org[d] + bn.n[d]) << sh;
    }
    int64_t covered = 0;
    for (size_t ob = 0; ob < po.blocks.size(); ob++) {
      const grmhd_block_desc& bo = po.blocks[ob];
      int64_t lo[3], hi[3];
      bool hit = true;
      for (int d = 0; d < 3; d++) {
        const int sh = ls[d] - bo.lev[d];
        lo[d] = std::max(nlo[d], bo.org[d] << sh);
        hi[d] = std::min(nhi[d], (bo.org[d] + bo.n[d]) << sh);
        hit = hit && lo[d] < hi[d];
      }
      if (!hit) continue;
      RegridOp op;
      op.nb = (int32_t)nb;
      op.ob = (int32_t)ob;
      int rmin = 0, rmax = 0;
      int64_t vol = 1;
      for (int d = 0; d < 3; d++) {
        op.r[d] = bn.lev[d] - bo.lev[d];
        rmin = std::min(rmin, op.r[d]);
        rmax = std::max(rmax, op.r[d]);
        const int sh = ls[d] - bn.lev[d];
        const int64_t w = (int64_t)1 << sh;
        if (lo[d] % w != 0 || hi[d] % w != 0)
          return fail(GRMHD_EINVAL, "regrid: an old block boundary cuts a cell of a new block");
        op.lo[d] = (int32_t)(lo[d] / w - bn.org[d]);
        op.ext[d] = (int32_t)((hi[d] - lo[d]) / w);
        op.top[d] = (op.lo[d] + op.ext[d] == bn.n[d]) ? 1 : 0;
        op.on[d] = (int32_t)bn.org[d];
        op.oo[d] = (int32_t)bo.org[d];
        vol *= op.ext[d];
      }
      if (rmin < -1 || rmax > 1 || (rmin < 0 && rmax > 0))
        return fail(GRMHD_EINVAL, "regrid: a new block is more than one level from an old block "
                                  "it overlaps, or finer in one dimension and coarser in another");
      covered += vol;
      ops.push_back(op);
    }
    if (covered != (int64_t)bn.n[0] * bn.n[1] * bn.n[2])
      return fail(GRMHD_EINVAL, "regrid: the old layout does not cover a new block");
  }
  return GRMHD_OK;
}

int grmhd_regrid(grmhd_ctx* from, grmhd_ctx* to, int32_t mode) {
  if (!from || !to || from == to) return fail(GRMHD_EINVAL, "regrid needs two distinct contexts");
  if (mode != GRMHD_REGRID_PRIMITIVE && mode != GRMHD_REGRID_CONSERVED)
    return fail(GRMHD_EINVAL, "unknown regrid mode");
  if (from->b_in_alt) return fail(GRMHD_ESTATE, "state not in the caller's buffers");
  std::vector<RegridOp> ops;
  if (int rc = regrid_ops(from->plan, to->plan, ops)) return rc;
  const int64_t nops = (int64_t)ops.size();
  std::vector<int64_t> start(4 * (nops + 1), 0);
  int64_t total[4] = {0, 0, 0, 0};
  for (int k = 0; k < 4; k++) {
    int64_t run = 0;
    for (int64_t q = 0; q < nops; q++) {
      start[k * (nops + 1) + q] = run;
      int64_t e[3] = {ops[q].ext[0], ops[q].ext[1], ops[q].ext[2]};
      if (k > 0) e[k - 1] += ops[q].top[k - 1];
      run += e[0] * e[1] * e[2];
    }
    start[k * (nops + 1) + nops] = run;
    total[k] = run;
  }
  RegridOp* dops = nullptr;
  int64_t* dstart = nullptr;
  HIPCHK(hipMalloc(&dops, sizeof(RegridOp) * std::max<int64_t>(nops, 1)));
  HIPCHK(hipMalloc(&dstart, sizeof(int64_t) * start.size()));
  hipStream_t st = from->stream;
  int rc = GRMHD_OK;
  hipError_t e = hipMemcpyAsync(dops, ops.data(), sizeof(RegridOp) * nops, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dstart, start.data(), sizeof(int64_t) * start.size(), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    // the new context's work must not overlap the copy: it starts on from's stream after
    // everything queued on to's stream, and to's stream waits for the regrid
    e = hipStreamSynchronize(to->stream);
  }
  if (e == hipSuccess) {
    fill_ghosts(from, from->bufs.prim, from->bufs.bface);
    launch_regrid(from->L, to->L, dops, nops, dstart, total, from->bufs.prim, from->bufs.bface,
                  to->bufs.prim, to->bufs.bface, mode == GRMHD_REGRID_CONSERVED);
    e = hipGetLastError();
  }
  if (e == hipSuccess)   // the simulation time carries over
    e = hipMemcpyAsync((char*)to->L.cnt + offsetof(Counters, t_sim),
                       (const char*)from->L.cnt + offsetof(Counters, t_sim), sizeof(double),
                       hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) rc = fail(GRMHD_EHIP, std::string("regrid: ") + hipGetErrorString(e));
  (void)hipFree(dops);
  (void)hipFree(dstart);
  to->b_in_alt = false;
  return rc;
}

int grmhd_plan_dump(const grmhd_grid_desc* desc, int32_t what, void* host_buf, size_t* bytes) {
  if (!bytes) return fail(GRMHD_EINVAL, "NULL argument");
  if (what < 0 || what > 23) return fail(GRMHD_EINVAL, "unknown table");
  Plan p;
  int rc = build_plan(desc, p, true);
  if (rc) return rc;
  const void* src;
  size_t need;
  std::vector<int32_t> sched;
  DevGhosts dg;
  if (what >= 20) {
    // the device ghost copy lists as uploaded: 20 cells with carried faces (GhostCF),
    // 21..23 the faces of components 1..3 not carried (GhostIdx), each in level order
    device_ghosts(p, dg);
    if (what == 20) {
      src = dg.cf.data();
      need = dg.cf.size() * sizeof(GhostCF);
    } else {
      src = dg.lf[what - 20].data();
      need = dg.lf[what - 20].size() * sizeof(GhostIdx);
    }
  } else if (what == 10) {
    // the order in which one cycle steps and synchronises blocks (as lat_cycle launches
    // them): per substep the due levels slowest first, then the sync points
    const int L = p.nlev, nsub = 1 << (L - 1);
    for (int s = 0; s < nsub; s++) {
      for (int lev = L - 1; lev >= 0; lev--)
        if (s % (1 << lev) == 0)
          for (int64_t q = p.lev_boff[lev]; q < p.lev_boff[lev + 1]; q++)
            sched.insert(sched.end(), {s, 0, lev, p.lev_blocks[q]});
      std::vector<char> syncs(p.blocks.size(), 0);
      for (const Plan::Reflux& r : p.reflux) syncs[r.b] = 1;
      for (const Plan::EdgeRef& e : p.sync_edges) syncs[e.b] = 1;
      for (size_t b = 0; b < p.blocks.size(); b++) {
        const int lev = p.blocks[b].lat;
        if (lev > 0 && syncs[b] && (s + 1) % (1 << lev) == 0)
          sched.insert(sched.end(), {s, 1, lev, (int32_t)b});
      }
    }
    src = sched.data();
    need = sched.size() * sizeof(int32_t);
  } else if (what == 11) {
    // the saved old-state elements per time level, as (level, list, block, element
    // offset within the block's part of the packed array)
    for (int w = 0; w < 2; w++) {
      const std::vector<uint32_t>& v = w ? p.slow_f : p.slow_c;
      const std::vector<int64_t>& o = w ? p.slow_f_off : p.slow_c_off;
      const int64_t nv = w ? 3 : 5;
      for (int l = 0; l + 1 < (int)o.size(); l++)
        for (int64_t q = o[l]; q < o[l + 1]; q++) {
          int b = 0;
          while (b + 1 < (int)p.info.size() && nv * p.info[b + 1].off <= (int64_t)v[q]) b++;
          sched.insert(sched.end(), {l, w, b, (int32_t)(v[q] - nv * p.info[b].off)});
        }
    }
    src = sched.data();
    need = sched.size() * sizeof(int32_t);
  } else if (what >= 15 && what <= 19) {
    // the device lists as uploaded (raw structures): 15 stage means, 16 face means,
    // 17 register items, 18 sync cells, 19 sync faces
    switch (what) {
      case 15: src = p.fix.data(); need = p.fix.size() * sizeof(MeanItem); break;
      case 16: src = p.bsync.data(); need = p.bsync.size() * sizeof(MeanItem); break;
      case 17: src = p.regs.data(); need = p.regs.size() * sizeof(RegItem); break;
      case 18: src = p.scells.data(); need = p.scells.size() * sizeof(SyncCell); break;
      default: src = p.sfaces.data(); need = p.sfaces.size() * sizeof(SyncFace); break;
    }
  } else if (what < 4) {
    src = p.ops[what].data();
    need = p.ops[what].size() * sizeof(GhostOp);
  } else if (what < 8) {
    src = p.aops[what - 4].data();
    need = p.aops[what - 4].size() * sizeof(AmrOp);
  } else if (what == 8) {
    src = p.samples.data();
    need = p.samples.size() * sizeof(AmrSample);
  } else if (what == 9) {
    // refinement faces at one time level: coarse, fine, d, side, e[3], lo[3], hi[3]
    for (const Plan::Link& lk : p.links)
      sched.insert(sched.end(), {lk.c, lk.f, lk.d, lk.side, lk.e[0], lk.e[1], lk.e[2],
                                 (int32_t)lk.lo[0], (int32_t)lk.lo[1], (int32_t)lk.lo[2],
                                 (int32_t)lk.hi[0], (int32_t)lk.hi[1], (int32_t)lk.hi[2]});
    src = sched.data();
    need = sched.size() * sizeof(int32_t);
  } else if (what == 12) {
    // reflux faces: block, d, side, local face, faster block, count, its elements[4]
    for (const Plan::Reflux& r : p.reflux)
      sched.insert(sched.end(), {r.b, r.d, r.side, r.loc, r.D, r.n, r.sub[0], r.sub[1], r.sub[2], r.sub[3]});
    src = sched.data();
    need = sched.size() * sizeof(int32_t);
  } else {
    // 13 sync edges, 14 stage edges: block, a, local edge, holder, count, its elements[2]
    for (const Plan::EdgeRef& e : what == 13 ? p.sync_edges : p.stage_edges)
      sched.insert(sched.end(), {e.b, e.a, e.loc, e.D, e.n, e.sub[0], e.sub[1]});
    src = sched.data();
    need = sched.size() * sizeof(int32_t);
  }
  if (!host_buf) {
    *bytes = need;
    return GRMHD_OK;
  }
  if (*bytes < need) return fail(GRMHD_EINVAL, "buffer too small");
  if (need) std::memcpy(host_buf, src, need);
  *bytes = need;
  return GRMHD_OK;
}

int grmhd_extract_cells(grmhd_ctx* c, double* P, double* B, double* geom) {
  if (!c || !P || !B || !geom) return fail(GRMHD_EINVAL, "NULL argument");
  if (c->b_in_alt) return fail(GRMHD_ESTATE, "state not in the caller's buffers");
  const auto& bl = c->plan.blocks;
  bool uneven = false;
  for (const auto& b : bl)
    for (int k = 0; k < 3; k++) uneven = uneven || b.n[k] != bl[0].n[k];
  if (uneven && !c->ext_off) {
    // first output index of each block, kept on the device for later calls
    std::vector<int64_t> off(bl.size());
    int64_t run = 0;
    for (size_t b = 0; b < bl.size(); b++) {
      off[b] = run;
      run += (int64_t)bl[b].n[0] * bl[b].n[1] * bl[b].n[2];
    }
    HIPCHK(hipMalloc(&c->ext_off, sizeof(int64_t) * off.size()));
    HIPCHK(hipMemcpy(c->ext_off, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice));
  }
  launch_extract(c->L, c->bufs.prim, c->bufs.bface, c->plan.n_interior, uneven ? c->ext_off : nullptr,
                 P, B, geom);
  HIPCHK(hipGetLastError());
  return GRMHD_OK;
}

int grmhd_destroy(grmhd_ctx* c) {
  if (!c) return GRMHD_OK;
  (void)hipEventDestroy(c->ev0);
  (void)hipEventDestroy(c->ev1);
  for (hipEvent_t e : c->prof_ev) (void)hipEventDestroy(e);
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (int k = 0; k < 2; k++) {
    if (c->side[k]) (void)hipStreamDestroy(c->side[k]);
    if (c->join_ev[k]) (void)hipEventDestroy(c->join_ev[k]);
  }
  if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
  if (c->ext_off) (void)hipFree(c->ext_off);
  delete c;
  return GRMHD_OK;
}

const char* grmhd_last_error(void) { return g_err.c_str(); }

// host-side geometry of the planner at one point (for CPU checks of the tables):
// out[15] metric entries in table order, conn[40] Christoffel symbols (nullable)
int grmhd_geometry_point(int32_t coords, double spin_a, double x1, double x2, double* out,
                         double* conn) {
  if (!out) return fail(GRMHD_EINVAL, "NULL output");
  if (coords != GRMHD_MINK_CART && coords != GRMHD_KS_LOGSPH) return fail(GRMHD_EINVAL, "coords");
  geometry_point(coords, spin_a, x1, x2, out, conn);
  return GRMHD_OK;
}

}  // extern "C"
