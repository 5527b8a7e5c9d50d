// kernels.hip -- HIP kernels of the GRMHD block update for gfx950 (CDNA4), FP64.
//
// One stage of the midpoint method (Sec. 2.1) runs as: ghost gather (cells, three face
// components) -> cell-centred field -> face fluxes along x1, x2, x3 -> edge EMFs ->
// cell update (constrained transport, conserved update with sources, inversion, floors).
// All state is structure-of-arrays per block with x1 fastest, so every kernel reads and
// writes consecutive doubles across the lanes of a wavefront.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.h"
#include "internal.h"
#include "mlp.h"
#include "wave.h"

namespace grmhd {

constexpr int NT = STAGE_NT;   // threads per workgroup (four wavefronts)

// The two heavy kernels come in occupancy variants: the minimum number of waves per
// SIMD the compiler must fit (trading registers for latency hiding).  Which variant a
// launch uses is the autotuner's choice (Launch::var_flux, Launch::var_upd).
// (variants asking for 6 or 8 waves spill and run 1.2-4x slower on MI355X; not built)
// flux variants: one face per thread at 1, 2, 4 waves per SIMD, then two faces per
// thread along the normal at 2 (it fits 3 waves; asked for 4 it spills)
constexpr int FLUX_OCC[NVAR_FLUX] = {1, 2, 4, 2};
constexpr bool FLUX_PAIR[NVAR_FLUX] = {false, false, false, true};
constexpr int UPD_OCC[NVAR_UPD] = {1, 2};

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.  Remap the
// dispatch order so that every XCD works on a contiguous range of (block, tile) indices:
// neighbouring tiles of a block then share one L2 for their stencil halos.
struct Tile {
  int x, y;
};
__device__ __forceinline__ Tile xcd_tile() {
  const int T = gridDim.x * gridDim.y;
  const int i = blockIdx.y * gridDim.x + blockIdx.x;
  const int x = i & 7, q = i >> 3;
  const int full = T >> 3, rem = T & 7;
  const int n = x < rem ? x * (full + 1) + q : rem * (full + 1) + (x - rem) * full + q;
  Tile t;
  t.x = n % gridDim.x;
  t.y = n / gridDim.x;
  return t;
}

// The block and tile of this workgroup: from the launch's work list when it has one
// (items of one block grouped on one XCD), else from the rectangular grid; slot is the
// workgroup's index for per-workgroup partials.
struct BlockTile {
  int blk, tile;
  int64_t slot;
};
__device__ __forceinline__ BlockTile block_tile(const Launch& L) {
  BlockTile r;
  if (L.wl) {
    const int T = gridDim.x, i = blockIdx.x;
    const int x = i & 7, q = i >> 3;
    const int full = T >> 3, rem = T & 7;
    const int n = x < rem ? x * (full + 1) + q : rem * (full + 1) + (x - rem) * full + q;
    const int2 w = L.wl[n];
    r.blk = w.x;
    r.tile = w.y;
    r.slot = n;
  } else {
    const Tile tl = xcd_tile();
    r.blk = L.blist ? L.blist[tl.y] : tl.y;
    r.tile = tl.x;
    r.slot = (int64_t)tl.y * gridDim.x + tl.x;
  }
  return r;
}

// decode a thread index of a box region (r0, r1, r2) starting at s into local coords
struct Cell {
  int I, J, K;
  int64_t loc;
};
__device__ __forceinline__ bool region_cell(const BlockInfo& bi, int t, int r0, int r1, int r2,
                                            int s0, int s1, int s2, Cell& c) {
  if (t >= r0 * r1 * r2) return false;
  const int i = t % r0;
  const int q = t / r0;
  const int j = q % r1;
  const int k = q / r1;
  c.I = s0 + i;
  c.J = s1 + j;
  c.K = s2 + k;
  c.loc = ((int64_t)c.K * bi.np[1] + c.J) * bi.np[0] + c.I;
  return true;
}


// ------------------------------------------------------------------ ghost gather

// One thread per entry of the concatenated lists: a ghost cell (five primitives, with
// the physical-boundary flip and clamps) or a ghost face (flip, or zero on the axis).
__global__ __launch_bounds__(NT) void k_ghosts(GhostLists G, double* __restrict__ P,
                                               double* __restrict__ B) {
  const int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (t >= G.end[3]) return;
  if (t < G.end[0]) {
    const GhostCF op = G.cf[t];
    const int fl = op.svol_fl >> 24, fc = op.dvol_fc >> 24;
    const int64_t svol = op.svol_fl & 0xFFFFFF, dvol = op.dvol_fc & 0xFFFFFF;
    const double* src = P + op.sp;
    double* dst = P + op.dp;
#pragma unroll
    for (int v = 0; v < 5; v++) {
      double x = src[v * svol];
      if (v == 3 && (fl & GF_FLIP)) x = -x;
      if (v == 2 && (fl & GF_CLAMP_NEG) && x > 0.0) x = 0.0;
      if (v == 2 && (fl & GF_CLAMP_POS) && x < 0.0) x = 0.0;
      dst[v * dvol] = x;
    }
#pragma unroll
    for (int c = 0; c < 3; c++)
      if ((fc >> c) & 1) B[op.db + c * dvol] = B[op.sb + c * svol];
    return;
  }
  const int k = t < G.end[1] ? 1 : (t < G.end[2] ? 2 : 3);
  const GhostIdx op = G.ops[k][t - G.end[k - 1]];
  const int fl = op.svol_fl >> 24;
  double x = B[op.src];
  if (fl & GF_ZERO) x = 0.0;
  else if (fl & GF_FLIP) x = -x;
  B[op.dst] = x;
}

// --------------------------------------------------------- cell-centred field

// B^i at cell centres = average of the two face fields / sqrt(-g) (Sec. 2.5), for every
// cell but the last padding layer (which no stencil reads; its upper faces lie outside
// the block's arrays)
__global__ __launch_bounds__(NT) void k_bcell(Launch L, const double* __restrict__ B,
                                              double* __restrict__ Bc) {
  const BlockTile bt = block_tile(L);
  const BlockInfo bi = L.blk[bt.blk];
  Cell c;
  if (!region_cell(bi, bt.tile * NT + threadIdx.x, bi.np[0] - 1, bi.np[1] - 1, bi.np[2] - 1, 0,
                   0, 0, c))
    return;
  const int64_t V = bi.vol;
  const double* b = B + 3 * bi.off;
  double* o = Bc + 3 * bi.off;
  const double gdet = L.geo.c[GDET * L.geo.ncol + geo_col(L.geo, bi, c.J, c.I)];
  const int64_t s2 = bi.np[0], s3 = (int64_t)bi.np[0] * bi.np[1];
  o[c.loc] = 0.5 * (b[c.loc] + b[c.loc + 1]) / gdet;
  o[V + c.loc] = 0.5 * (b[V + c.loc] + b[V + c.loc + s2]) / gdet;
  o[2 * V + c.loc] = 0.5 * (b[2 * V + c.loc] + b[2 * V + c.loc + s3]) / gdet;
}

// ------------------------------------------------------------------ face fluxes

// The flux of one face from its two reconstructed states: fluxes, conserved states and
// fast magnetosonic speeds of both sides, then HLLE (RIEMANN 1) or LLF (0); stored at
// out with stride V per component.
template <int DIR, int RIEMANN>
__device__ __forceinline__ void face_flux(const double PL[5], const double PR[5],
                                          const double BL[3], const double BR[3], const Metric& m,
                                          double gam, double* __restrict__ out, int64_t V) {
  constexpr int t1 = DIR == 1 ? 1 : 0;   // transverse field components (0-based)
  constexpr int t2 = DIR == 3 ? 1 : 2;
  double UL[9], UR[9], FL[8], FR[8];
  double vmaxL, vminL, vmaxR, vminR;
  {
    Fluid f;
    fluid_state<true>(PL, BL, m, f);
    const double kap = entropy_kappa<true>(PL, gam);
    flux_vector<0>(PL, f, m, gam, kap, UL);
    flux_vector<DIR>(PL, f, m, gam, kap, FL);
    wave_speeds<DIR, true>(PL, f, m, gam, vmaxL, vminL);
  }
  {
    Fluid f;
    fluid_state<true>(PR, BR, m, f);
    const double kap = entropy_kappa<true>(PR, gam);
    flux_vector<0>(PR, f, m, gam, kap, UR);
    flux_vector<DIR>(PR, f, m, gam, kap, FR);
    wave_speeds<DIR, true>(PR, f, m, gam, vmaxR, vminR);
  }
  // conserved components in flux order: mass, energy, momenta, transverse field, entropy
  constexpr int uidx[8] = {0, 1, 2, 3, 4, 5 + t1, 5 + t2, 8};
  const double cmax = fmax(0.0, fmax(vmaxL, vmaxR));
  const double cmin = -fmin(0.0, fmin(vminL, vminR));
  if (RIEMANN == 0) {
    const double cc = fmax(cmax, cmin);
#pragma unroll
    for (int q = 0; q < 8; q++) out[q * V] = 0.5 * (FL[q] + FR[q] - cc * (UR[uidx[q]] - UL[uidx[q]]));
  } else {
    if (cmax + cmin > 0.0) {
      const double ic = rcp_nr(cmax + cmin);
#pragma unroll
      for (int q = 0; q < 8; q++)
        out[q * V] = (cmin * FR[q] + cmax * FL[q] - cmax * cmin * (UR[uidx[q]] - UL[uidx[q]])) * ic;
    } else {
#pragma unroll
      for (int q = 0; q < 8; q++) out[q * V] = 0.5 * (FL[q] + FR[q]);
    }
  }
}

// One thread per face along x^DIR.  Normal range [ng, ng + n], transverse range widened
// by one ghost layer so the edge EMFs of every interior face have their four fluxes.
template <int DIR, int RECON, int RIEMANN, int OCC>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(OCC))) void k_flux(Launch L, const double* __restrict__ P,
                                             const double* __restrict__ Bc,
                                             const double* __restrict__ B,
                                             double* __restrict__ F) {
  const BlockTile bt = block_tile(L);
  const BlockInfo bi = L.blk[bt.blk];
  const int g = L.ph.ng;
  const int r0 = DIR == 1 ? bi.n[0] + 1 : bi.n[0] + 2;
  const int r1 = DIR == 2 ? bi.n[1] + 1 : bi.n[1] + 2;
  const int r2 = DIR == 3 ? bi.n[2] + 1 : bi.n[2] + 2;
  Cell c;
  if (!region_cell(bi, bt.tile * NT + threadIdx.x, r0, r1, r2, DIR == 1 ? g : g - 1,
                   DIR == 2 ? g : g - 1, DIR == 3 ? g : g - 1, c))
    return;
  const int64_t V = bi.vol;
  const int64_t st = DIR == 1 ? 1 : (DIR == 2 ? (int64_t)bi.np[0] : (int64_t)bi.np[0] * bi.np[1]);
  const int64_t col = geo_col(L.geo, bi, c.J, c.I);
  const double* tab = DIR == 1 ? L.geo.f1 : (DIR == 2 ? L.geo.f2 : L.geo.c);
  // All loads of the face (metric, the six-cell lines of the five primitives and of the
  // two transverse field components, the normal field) in one batch, closed by a
  // scheduling barrier: otherwise they are issued variable by variable between the
  // branches of the limiters, a memory round trip each.
  const Metric m = load_metric(tab, L.geo.ncol, col);
  double* out = F + 24 * bi.off + (int64_t)(DIR - 1) * 8 * V + c.loc;
  constexpr int t1 = DIR == 1 ? 1 : 0;   // transverse field components (0-based)
  constexpr int t2 = DIR == 3 ? 1 : 2;
  constexpr bool PLM = RECON == 0 || RECON == 2;
  constexpr int k0 = PLM ? 1 : 0, k1 = PLM ? 5 : 6;   // stencil used
  double sp[5][6], sb[2][6];
  const double* p = P + 5 * bi.off + c.loc;
  const double* bc = Bc + 3 * bi.off + c.loc;
#pragma unroll
  for (int k = 0; k < 6; k++) {
#pragma unroll
    for (int v = 0; v < 5; v++)
      sp[v][k] = (k < k0 || k >= k1) ? 0.0 : p[(int64_t)v * V + (k - 3) * st];
    sb[0][k] = (k < k0 || k >= k1) ? 0.0 : bc[(int64_t)t1 * V + (k - 3) * st];
    sb[1][k] = (k < k0 || k >= k1) ? 0.0 : bc[(int64_t)t2 * V + (k - 3) * st];
  }
  const double bface = B[3 * bi.off + (int64_t)(DIR - 1) * V + c.loc];
  __builtin_amdgcn_sched_barrier(0);
  if (DIR == 2 && m.gdet == 0.0) {   // the polar axis carries no flux
#pragma unroll
    for (int q = 0; q < 8; q++) out[q * V] = 0.0;
    return;
  }
  double PL[5], PR[5], BL[3], BR[3];
  double fl[2] = {0.0, 0.0};   // flattening of the two cells next to the face
  if (RECON == 3) {
    fl[0] = flatten_coef(sp[1], sp[1 + DIR], 2);
    fl[1] = flatten_coef(sp[1], sp[1 + DIR], 3);
  }
#pragma unroll
  for (int v = 0; v < 5; v++) recon_face<RECON>(sp[v], PL[v], PR[v], fl);
  recon_face<RECON>(sb[0], BL[t1], BR[t1], fl);
  recon_face<RECON>(sb[1], BL[t2], BR[t2], fl);
  const double bn = bface * rcp_nr(m.gdet);
  BL[DIR - 1] = bn;
  BR[DIR - 1] = bn;
  face_flux<DIR, RIEMANN>(PL, PR, BL, BR, m, L.ph.gam, out, V);
}

// Two faces per thread along x^DIR (the faces at normal index ng + 2i and ng + 2i + 1,
// the second only inside the normal range): the seven-cell line gives both faces' states
// with the slopes, interface values and limited parabola of the shared cells computed
// once.  Same arithmetic per face as k_flux.
template <int DIR, int RECON, int RIEMANN, int OCC>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(OCC))) void k_flux_pair(
    Launch L, const double* __restrict__ P, const double* __restrict__ Bc,
    const double* __restrict__ B, double* __restrict__ F) {
  const BlockTile bt = block_tile(L);
  const BlockInfo bi = L.blk[bt.blk];
  const int g = L.ph.ng;
  const int nn = bi.n[DIR - 1] + 1;   // faces along the normal
  const int r0 = DIR == 1 ? (nn + 1) / 2 : bi.n[0] + 2;
  const int r1 = DIR == 2 ? (nn + 1) / 2 : bi.n[1] + 2;
  const int r2 = DIR == 3 ? (nn + 1) / 2 : bi.n[2] + 2;
  const int t = bt.tile * NT + threadIdx.x;
  if (t >= r0 * r1 * r2) return;
  const int ti = t % r0, tq = t / r0, tj = tq % r1, tk = tq / r1;
  const int I = DIR == 1 ? g + 2 * ti : g - 1 + ti;
  const int J = DIR == 2 ? g + 2 * tj : g - 1 + tj;
  const int K = DIR == 3 ? g + 2 * tk : g - 1 + tk;
  const int64_t loc = ((int64_t)K * bi.np[1] + J) * bi.np[0] + I;
  const bool two = (DIR == 1 ? I : (DIR == 2 ? J : K)) + 1 <= g + bi.n[DIR - 1];
  const int64_t V = bi.vol;
  const int64_t st = DIR == 1 ? 1 : (DIR == 2 ? (int64_t)bi.np[0] : (int64_t)bi.np[0] * bi.np[1]);
  const double* tab = DIR == 1 ? L.geo.f1 : (DIR == 2 ? L.geo.f2 : L.geo.c);
  const Metric m0 = load_metric(tab, L.geo.ncol, geo_col(L.geo, bi, J, I));
  double* out = F + 24 * bi.off + (int64_t)(DIR - 1) * 8 * V + loc;
  constexpr int t1 = DIR == 1 ? 1 : 0;
  constexpr int t2 = DIR == 3 ? 1 : 2;
  constexpr bool PLM = RECON == 0 || RECON == 2;
  constexpr int k0 = PLM ? 1 : 0, k1 = PLM ? 6 : 7;   // stencil used
  double sp[5][7], sb[2][7];
  const double* p = P + 5 * bi.off + loc;
  const double* bc = Bc + 3 * bi.off + loc;
#pragma unroll
  for (int k = 0; k < 7; k++) {
#pragma unroll
    for (int v = 0; v < 5; v++)
      sp[v][k] = (k < k0 || k >= k1) ? 0.0 : p[(int64_t)v * V + (k - 3) * st];
    sb[0][k] = (k < k0 || k >= k1) ? 0.0 : bc[(int64_t)t1 * V + (k - 3) * st];
    sb[1][k] = (k < k0 || k >= k1) ? 0.0 : bc[(int64_t)t2 * V + (k - 3) * st];
  }
  const double* bf = B + 3 * bi.off + (int64_t)(DIR - 1) * V + loc;
  const double bface0 = bf[0], bface1 = bf[st];
  __builtin_amdgcn_sched_barrier(0);
  double PL0[5], PR0[5], PL1[5], PR1[5], BL0[3], BR0[3], BL1[3], BR1[3];
  double fl[3] = {0.0, 0.0, 0.0};   // flattening of the cells s[2], s[3], s[4]
  if (RECON == 3) {
#pragma unroll
    for (int q = 0; q < 3; q++) fl[q] = flatten_coef(sp[1], sp[1 + DIR], 2 + q);
  }
#pragma unroll
  for (int v = 0; v < 5; v++) recon_pair<RECON>(sp[v], PL0[v], PR0[v], PL1[v], PR1[v], fl);
  recon_pair<RECON>(sb[0], BL0[t1], BR0[t1], BL1[t1], BR1[t1], fl);
  recon_pair<RECON>(sb[1], BL0[t2], BR0[t2], BL1[t2], BR1[t2], fl);
  const double gam = L.ph.gam;
  // The second face's states wait in LDS while the first face's physics runs, so the
  // registers hold one face's physics at a time (the compiler barrier keeps it from
  // forwarding the stored values and holding them in registers after all).
  __shared__ double park[14][NT];
  {
    const int tx = threadIdx.x;
#pragma unroll
    for (int v = 0; v < 5; v++) {
      park[v][tx] = PL1[v];
      park[5 + v][tx] = PR1[v];
    }
    park[10][tx] = BL1[t1];
    park[11][tx] = BL1[t2];
    park[12][tx] = BR1[t1];
    park[13][tx] = BR1[t2];
  }
  asm volatile("" ::: "memory");
  if (DIR == 2 && m0.gdet == 0.0) {   // the polar axis carries no flux
#pragma unroll
    for (int q = 0; q < 8; q++) out[q * V] = 0.0;
  } else {
    const double bn = bface0 * rcp_nr(m0.gdet);
    BL0[DIR - 1] = bn;
    BR0[DIR - 1] = bn;
    face_flux<DIR, RIEMANN>(PL0, PR0, BL0, BR0, m0, gam, out, V);
  }
  if (!two) return;
  asm volatile("" ::: "memory");
  {
    const int tx = threadIdx.x;
#pragma unroll
    for (int v = 0; v < 5; v++) {
      PL1[v] = park[v][tx];
      PR1[v] = park[5 + v][tx];
    }
    BL1[t1] = park[10][tx];
    BL1[t2] = park[11][tx];
    BR1[t1] = park[12][tx];
    BR1[t2] = park[13][tx];
  }
  const Metric m1 =
      DIR == 3 ? m0 : load_metric(tab, L.geo.ncol, geo_col(L.geo, bi, J + (DIR == 2), I + (DIR == 1)));
  if (DIR == 2 && m1.gdet == 0.0) {
#pragma unroll
    for (int q = 0; q < 8; q++) out[st + q * V] = 0.0;
    return;
  }
  const double bn = bface1 * rcp_nr(m1.gdet);
  BL1[DIR - 1] = bn;
  BR1[DIR - 1] = bn;
  face_flux<DIR, RIEMANN>(PL1, PR1, BL1, BR1, m1, gam, out + st, V);
}

// ------------------------------------------------------------------ edge EMFs

// E^1 at (i, j-1/2, k-1/2), E^2 at (i-1/2, j, k-1/2), E^3 at (i-1/2, j-1/2, k): the
// average of the four face fluxes of B around the edge (Sec. 2.5); zero on the axis.
// With UPWIND, Gardiner & Stone's (2005) corrections are added (edge_upwind below).

// A mass flux at most this fraction of the largest conserved density sqrt(-g) rho u^t of
// the edge's four cells (a coordinate velocity through the face below it) counts as zero:
// such fluxes are rounding residuals of flows at rest through the face (symmetry planes,
// static atmospheres), whose sign no computation fixes.
constexpr double UPWIND_REST = 1e-12;

__device__ __forceinline__ double upwind_pick(double lo, double hi, double m, double rest) {
  return m > rest ? lo : (m < -rest ? hi : 0.5 * (lo + hi));
}

// The correction for the edge along x^(a+1) at local index l, (a, p, q) cyclic, with
// strides sp, sq of the cells along p and q.  Around the edge: two p-faces (rows qq = 0, 1
// at l - (1 - qq) sq) with face EMF -F_p(B^q) and mass flux F_p(rho), two q-faces
// (columns pp at l - (1 - pp) sp) with +F_q(B^p) and F_q(rho), and four cells with their
// own-state EMFs (er) and conserved densities (dd).  Each gradient toward a cell centre
// comes from the row (column) upstream of the mass flux through the face between the two
// candidates.
__device__ __forceinline__ double edge_upwind(const double* __restrict__ Fpb,
                                              const double* __restrict__ Fpr,
                                              const double* __restrict__ Fqb,
                                              const double* __restrict__ Fqr,
                                              const double* __restrict__ er,
                                              const double* __restrict__ dd, int64_t sp,
                                              int64_t sq) {
  const double Ep0 = -Fpb[-sq], Ep1 = -Fpb[0];
  const double Mp0 = Fpr[-sq], Mp1 = Fpr[0];
  const double Eq0 = Fqb[-sp], Eq1 = Fqb[0];
  const double Mq0 = Fqr[-sp], Mq1 = Fqr[0];
  const double r00 = er[-sp - sq], r01 = er[-sp], r10 = er[-sq], r11 = er[0];
  const double rest = UPWIND_REST * fmax(fmax(fabs(dd[-sp - sq]), fabs(dd[-sp])),
                                         fmax(fabs(dd[-sq]), fabs(dd[0])));
  const double dp_lo = upwind_pick(Ep0 - r00, Ep1 - r01, Mq0, rest);
  const double dp_hi = upwind_pick(r10 - Ep0, r11 - Ep1, Mq1, rest);
  const double dq_lo = upwind_pick(Eq0 - r00, Eq1 - r10, Mp0, rest);
  const double dq_hi = upwind_pick(r01 - Eq0, r11 - Eq1, Mp1, rest);
  return 0.25 * ((dp_lo - dp_hi) + (dq_lo - dq_hi));
}

template <bool UPWIND>
__global__ __launch_bounds__(NT) void k_emf(Launch L, const double* __restrict__ F,
                                            double* __restrict__ E,
                                            const double* __restrict__ eref) {
  const BlockTile bt = block_tile(L);
  const BlockInfo bi = L.blk[bt.blk];
  const int g = L.ph.ng;
  Cell c;
  if (!region_cell(bi, bt.tile * NT + threadIdx.x, bi.n[0] + 1, bi.n[1] + 1, bi.n[2] + 1, g, g,
                   g, c))
    return;
  const int64_t V = bi.vol;
  const int64_t s2 = bi.np[0], s3 = (int64_t)bi.np[0] * bi.np[1];
  const double* f = F + 24 * bi.off + c.loc;
  const double* F1B2 = f + 5 * V;    // x1 flux of B^2
  const double* F1B3 = f + 6 * V;    // x1 flux of B^3
  const double* F2B1 = f + 13 * V;   // x2 flux of B^1
  const double* F2B3 = f + 14 * V;   // x2 flux of B^3
  const double* F3B1 = f + 21 * V;   // x3 flux of B^1
  const double* F3B2 = f + 22 * V;   // x3 flux of B^2
  const bool pole = L.geo.f2[GDET * L.geo.ncol + geo_col(L.geo, bi, c.J, c.I)] == 0.0;
  double* e = E + 3 * bi.off + c.loc;
  const double* er = UPWIND ? eref + 4 * bi.off + c.loc : nullptr;   // [4][V] per block
  const double* dd = UPWIND ? er + 3 * V : nullptr;
  if (c.I < g + bi.n[0]) {
    double x = pole ? 0.0 : 0.25 * (F3B2[0] + F3B2[-s2] - F2B3[-s3] - F2B3[0]);
    // E^1: p = x2, q = x3
    if (UPWIND && !pole) x += edge_upwind(F2B3, f + 8 * V, F3B2, f + 16 * V, er, dd, s2, s3);
    e[0] = x;
  }
  if (c.J < g + bi.n[1]) {
    double x = 0.25 * (F1B3[-s3] + F1B3[0] - F3B1[0] - F3B1[-1]);
    // E^2: p = x3, q = x1
    if (UPWIND) x += edge_upwind(F3B1, f + 16 * V, F1B3, f, er + V, dd, s3, 1);
    e[V] = x;
  }
  if (c.K < g + bi.n[2]) {
    double x = pole ? 0.0 : 0.25 * (F2B1[-1] + F2B1[0] - F1B2[0] - F1B2[-s2]);
    // E^3: p = x1, q = x2
    if (UPWIND && !pole) x += edge_upwind(F1B2, f, F2B1, f + 8 * V, er + 2 * V, dd, 1, s2);
    e[2 * V] = x;
  }
}

// The EMF of each cell's own state, component a = the flux of B^(p+1) along x^(q+1),
// sqrt(-g) (b^p u^q - b^q u^p) with (a, p, q) cyclic, and as a fourth component the
// conserved density sqrt(-g) rho u^t, on the interior cells and one layer around them
// (the cells next to the block's edges); [4][V] per block
__global__ __launch_bounds__(NT) void k_emf_ref(Launch L, const double* __restrict__ P,
                                                const double* __restrict__ Bc,
                                                double* __restrict__ eref) {
  const BlockTile bt = block_tile(L);
  const BlockInfo bi = L.blk[bt.blk];
  const int g = L.ph.ng;
  Cell c;
  if (!region_cell(bi, bt.tile * NT + threadIdx.x, bi.n[0] + 2, bi.n[1] + 2, bi.n[2] + 2,
                   g - 1, g - 1, g - 1, c))
    return;
  const int64_t V = bi.vol;
  const Metric m = load_metric(L.geo.c, L.geo.ncol, geo_col(L.geo, bi, c.J, c.I));
  double p[5], b[3];
#pragma unroll
  for (int v = 0; v < 5; v++) p[v] = P[5 * bi.off + v * V + c.loc];
#pragma unroll
  for (int v = 0; v < 3; v++) b[v] = Bc[3 * bi.off + v * V + c.loc];
  Fluid fl;
  fluid_state(p, b, m, fl);
  double* o = eref + 4 * bi.off + c.loc;
  o[0] = m.gdet * (fl.bcon[2] * fl.ucon[3] - fl.bcon[3] * fl.ucon[2]);
  o[V] = m.gdet * (fl.bcon[3] * fl.ucon[1] - fl.bcon[1] * fl.ucon[3]);
  o[2 * V] = m.gdet * (fl.bcon[1] * fl.ucon[2] - fl.bcon[2] * fl.ucon[1]);
  o[3 * V] = m.gdet * p[0] * fl.ucon[0];
}

// ------------------------------------------------------------------ cell update

// minimum over the workgroup: wave minimum, then across the four waves through LDS;
// thread 0 returns the result
__device__ __forceinline__ double block_min(double v) {
  __shared__ double part[NT / 64];
  v = wave_min(v);
  if (lane_id() == 0) part[threadIdx.x / 64] = v;
  __syncthreads();
  double r = part[0];
#pragma unroll
  for (int w = 1; w < NT / 64; w++) r = fmin(r, part[w]);
  return r;
}

// per cell 1/dt = sum_d max(|v+|, |v-|)/dx_d from the cell-centred state (Sec. 2.1)
__device__ __forceinline__ double cell_dt(const double P[5], const double B[3], const Metric& m,
                                          const Phys& ph, const double idx[3]) {
  Fluid f;
  fluid_state(P, B, m, f);
  double vp, vm, inv = 0.0;
  wave_speeds<1>(P, f, m, ph.gam, vp, vm);
  inv += fmax(fabs(vp), fabs(vm)) * idx[0];
  wave_speeds<2>(P, f, m, ph.gam, vp, vm);
  inv += fmax(fabs(vp), fabs(vm)) * idx[1];
  wave_speeds<3>(P, f, m, ph.gam, vp, vm);
  inv += fmax(fabs(vp), fabs(vm)) * idx[2];
  return 1.0 / inv;
}

// Learned first guess for the cells of one workgroup: every thread passes the inversion
// input of its cell (or valid = false), every wavefront runs its 64 cells through the
// MLP with matrix cores, and each thread gets back (W0, v0) and whether to use it.
__device__ __forceinline__ bool mlp_guess_block(const MlpBlob* __restrict__ blob, const C2PIn& s,
                                                const Metric& m, bool valid, double& W0,
                                                double& v0) {
  __shared__ float feat[NT * 8];
  __shared__ float outv[NT * 2];
  const int t = threadIdx.x, w = t / 64;
  float x[8];
  bool ok = valid && mlp_features(s, m, x);
#pragma unroll
  for (int k = 0; k < 8; k++) feat[t * 8 + k] = ok ? (x[k] - blob->xmean[k]) / blob->xstd[k] : 0.0f;
  __syncthreads();
  mlp_wave(blob, feat + w * 64 * 8, outv + w * 64 * 2);
  __syncthreads();
  if (!ok) return false;
  const double lg = (double)(outv[t * 2] * blob->ystd[0] + blob->ymean[0]);
  const double lw = (double)(outv[t * 2 + 1] * blob->ystd[1] + blob->ymean[1]);
  const double G = exp(lg > 0.0 ? lg : 0.0);
  W0 = s.D * exp(lw);
  v0 = 1.0 - 1.0 / (G * G);
  return isfinite(W0) && W0 > 0.0 && v0 >= 0.0 && v0 < 1.0;
}

// The learned guess where it can pay: the network runs for a workgroup only if the plain
// guess (the stage primitives) of some cell in it leaves a residual misfit (c2p_misfit)
// above MLP_GATE.  The network's guesses are typically within about 10% of the root
// (Newton from them needs about 4.6 iterations to 1e-12 on the benchmark torus's cells);
// a plain guess with a smaller misfit is the better start, and the inference would cost
// more than it saves.  Large misfits come with cold starts, floors and strong jumps.
constexpr double MLP_GATE = 1e-1;
__device__ __forceinline__ bool learned_guess(const MlpBlob* __restrict__ blob, const C2PIn& s,
                                              const Metric& m, bool valid, const double PS[5],
                                              double& W0, double& v0) {
  bool need = false;
  if (valid) {
    double Wp, vp;
    guess_from_prims(s, m, PS, Wp, vp);
    need = !(c2p_misfit(s, Wp, vp) < MLP_GATE);
  }
  if (!__syncthreads_or(need)) return false;
  return mlp_guess_block(blob, s, m, valid, W0, v0);
}

// The conserved update of one interior cell (Sec. 2.5): constrained transport of its
// faces (written to Bout), U^n from P^n, the geometric source at the stage state, the
// flux divergence; leaves U (9 components, field from the new faces), the stage
// primitives PS and the cell's density and internal-energy floors fl.  U^n is
// recomputed from P^n in both stages: the kernel is bound by its memory traffic, and
// keeping U^n from the predictor for the corrector moved more bytes than it saved.
//
// The cell's ~120 global loads are issued in four batches (cell inputs, two halves of
// the connection coefficients, fluxes), each closed by a scheduling barrier: left to itself the
// compiler interleaves them with the arithmetic in small groups, and each group then
// costs a full memory round trip.
//
// BZ > 0: the workgroup is a brick of 256/BZ (x1, x2) columns of BZ cells along x3
// (brick_x1), so the cells of each column share the column's centre geometry (metric,
// connection coefficients, floors: NGEO_C values).  Each thread loads a 1/BZ share of its
// column's values with the cell inputs, the workgroup stages them in LDS (sgeo,
// [NGEO_C][256/BZ]), and the metric, the connection coefficients and the floors are read
// from there: 1/BZ of the geometry loads, and no memory round trip for the connection
// coefficients.  Every thread of the workgroup must call it.  With BZ = 0 the caller
// passes the metric in m.
template <int BZ>
__device__ __forceinline__ void conserve_cell(const Launch& L, const BlockInfo& bi, const Cell& c,
                                              Metric& m, double* sgeo, int64_t col,
                                              const double* __restrict__ Pn,
                                              const double* __restrict__ Bn,
                                              const double* __restrict__ Ps,
                                              const double* __restrict__ Bcs,
                                              const double* __restrict__ F,
                                              const double* __restrict__ E, double dt_factor,
                                              double* __restrict__ Bout, double U[9],
                                              double PS[5], double fl[2]) {
  const int g = L.ph.ng;
  const int64_t V = bi.vol;
  const int64_t s2 = bi.np[0], s3 = (int64_t)bi.np[0] * bi.np[1];
  const int64_t l = c.loc;
  const GeoTab& G = L.geo;
  const double dt = L.ph.courant * __longlong_as_double((long long)L.cnt->dt_bits);
  const double dts = dt_factor * dt;
  const double ix1 = bi.idx[0], ix2 = bi.idx[1], ix3 = bi.idx[2];
  const double* e1 = E + 3 * bi.off;
  const double* e2 = e1 + V;
  const double* e3 = e2 + V;
  const double* b1 = Bn + 3 * bi.off;
  const double* b2 = b1 + V;
  const double* b3 = b2 + V;
  constexpr int fq[6] = {0, 1, 2, 3, 4, 7};
  constexpr int uq[6] = {0, 1, 2, 3, 4, 8};

  // batch 1: faces and edges of the cell, polar flags, P^n, the stage
  // state, floors (every address is inside the block's arrays, also at the poles)
  const double glo = G.f2[GDET * G.ncol + col];
  const double ghi = G.f2[GDET * G.ncol + col + bi.gti];
  const double f1lo = b1[l], f1hi = b1[l + 1], f2lo = b2[l], f2hi = b2[l + s2];
  const double f3lo = b3[l], f3hi = b3[l + s3];
  const double e1a = e1[l], e1b = e1[l + s2], e1c = e1[l + s3], e1d = e1[l + s2 + s3];
  const double e2a = e2[l], e2b = e2[l + 1], e2c = e2[l + s3], e2d = e2[l + 1 + s3];
  const double e3a = e3[l], e3b = e3[l + 1], e3c = e3[l + s2], e3d = e3[l + 1 + s2];
  double P0[5], BS[3];
#pragma unroll
  for (int v = 0; v < 5; v++) P0[v] = Pn[5 * bi.off + (int64_t)v * V + l];
#pragma unroll
  for (int v = 0; v < 5; v++) PS[v] = Ps[5 * bi.off + (int64_t)v * V + l];
#pragma unroll
  for (int i = 0; i < 3; i++) BS[i] = Bcs[3 * bi.off + (int64_t)i * V + l];
  constexpr bool BRICK = BZ > 0;
  constexpr int Z = BRICK ? BZ : 1, COLS = 256 / Z;
  constexpr int NG = (NGEO_C + Z - 1) / Z;
  double gv[BRICK ? NG : 1];   // this thread's share of its column's geometry
  const int cidx = threadIdx.x & (COLS - 1), q0 = threadIdx.x / COLS;
  if (BRICK) {
#pragma unroll
    for (int k = 0; k < NG; k++) {
      const int q = q0 + Z * k;
      gv[k] = q < NGEO_C ? G.c[q * G.ncol + col] : 0.0;
    }
  } else {
    fl[0] = G.c[RHOFL * G.ncol + col];
    fl[1] = G.c[UFL * G.ncol + col];
  }
  __builtin_amdgcn_sched_barrier(0);
  if (BRICK) {
#pragma unroll
    for (int k = 0; k < NG; k++) {
      const int q = q0 + Z * k;
      if (q < NGEO_C) sgeo[q * COLS + cidx] = gv[k];
    }
    __syncthreads();
    m = load_metric(sgeo + cidx, COLS, 0);
    fl[0] = sgeo[RHOFL * COLS + cidx];
    fl[1] = sgeo[UFL * COLS + cidx];
  }

  // constrained transport of the six faces of this cell (Sec. 2.5)
  const double nb1lo = f1lo + dts * ((e2c - e2a) * ix3 - (e3c - e3a) * ix2);
  const double nb1hi = f1hi + dts * ((e2d - e2b) * ix3 - (e3d - e3b) * ix2);
  const double nb2lo = glo == 0.0 ? 0.0 : f2lo + dts * ((e3b - e3a) * ix1 - (e1c - e1a) * ix3);
  const double nb2hi = ghi == 0.0 ? 0.0 : f2hi + dts * ((e3d - e3c) * ix1 - (e1d - e1b) * ix3);
  const double nb3lo = f3lo + dts * ((e1b - e1a) * ix2 - (e2b - e2a) * ix1);
  const double nb3hi = f3hi + dts * ((e1d - e1c) * ix2 - (e2d - e2c) * ix1);
  double* o1 = Bout + 3 * bi.off;
  double* o2 = o1 + V;
  double* o3 = o2 + V;
  o1[l] = nb1lo;
  o2[l] = nb2lo;
  o3[l] = nb3lo;
  if (c.I == g + bi.n[0] - 1) o1[l + 1] = nb1hi;
  if (c.J == g + bi.n[1] - 1) o2[l + s2] = nb2hi;
  if (c.K == g + bi.n[2] - 1) o3[l + s3] = nb3hi;

  // U^n from P^n (Sec. 2.5)
  {
    double B0[3];
    const double hg = 0.5 / m.gdet;
    B0[0] = (f1lo + f1hi) * hg;
    B0[1] = (f2lo + f2hi) * hg;
    B0[2] = (f3lo + f3hi) * hg;
    Fluid f;
    fluid_state(P0, B0, m, f);
    flux_vector<0>(P0, f, m, L.ph.gam, entropy_kappa(P0, L.ph.gam), U);
  }

  // batches 2 and 3: the connection coefficients of the cell's column, Gamma^l_{nu k}
  // for l = 0, 1 and then for l = 2, 3 -> geometric source
  double Q[4];
  {
    double T[4][4];
    {
      Fluid f;
      fluid_state(PS, BS, m, f);
      stress_energy(PS, f, L.ph.gam, T);
    }
    double q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int h = 0; h < 2; h++) {
      double conn[20];
#pragma unroll
      for (int j = 0; j < 20; j++)
        conn[j] = BRICK ? sgeo[(CONN0 + 20 * h + j) * COLS + cidx]
                        : G.c[(CONN0 + 20 * h + j) * G.ncol + col];
      if (!BRICK) __builtin_amdgcn_sched_barrier(0);
      connection_contract(T, conn, 2 * h, q);
    }
#pragma unroll
    for (int nu = 0; nu < 4; nu++) Q[nu] = m.gdet * q[nu];
  }

  // batch 4: the fluxes on the six faces -> divergence
  const double* x1 = F + 24 * bi.off + l;
  const double* x2 = x1 + 8 * V;
  const double* x3 = x2 + 8 * V;
  double fx[6][6];
#pragma unroll
  for (int k = 0; k < 6; k++) {
    const int64_t o = (int64_t)fq[k] * V;
    fx[k][0] = x1[o + 1];
    fx[k][1] = x1[o];
    fx[k][2] = x2[o + s2];
    fx[k][3] = x2[o];
    fx[k][4] = x3[o + s3];
    fx[k][5] = x3[o];
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int k = 0; k < 6; k++) {
    const double div = (fx[k][0] - fx[k][1]) * ix1 + (fx[k][2] - fx[k][3]) * ix2 +
                       (fx[k][4] - fx[k][5]) * ix3;
    const double q = (k >= 1 && k <= 4) ? Q[k - 1] : 0.0;
    U[uq[k]] = U[uq[k]] - dts * div + dts * q;
  }
  U[5] = 0.5 * (nb1lo + nb1hi);
  U[6] = 0.5 * (nb2lo + nb2hi);
  U[7] = 0.5 * (nb3lo + nb3hi);
}

// The inversion of one cell and its floors (Sec. 2.6, 2.7; DRIFT: in the drift frame);
// writes the primitives and, with NEXT_DT, returns the cell's Courant step of the next
// step in dtc; bad = 1 when the result is not a physical state (a non-finite value,
// rho <= 0 or u <= 0)
template <bool NEXT_DT, bool DRIFT>
__device__ __forceinline__ void invert_cell(const Launch& L, const BlockInfo& bi, const Cell& c,
                                            const Metric& m, int64_t col, const C2PIn& cs,
                                            bool first, double W0, double v0, const double PS[5],
                                            const double fl[2], double* __restrict__ Pout,
                                            int& tier, int& iters, int& hits, int& bad,
                                            double& dtc) {
  double Pnew[5];
  tier = c2p_solve(cs, m, first, W0, v0, PS, L.ph.tol, L.ph.maxit, Pnew, iters);
  // B^i = Bbar^i / sqrt(-g) with Bbar^i the face average; c2p_setup holds alpha B^i
  const double ia = 1.0 / m.alpha;
  const double Bnew[3] = {cs.B1 * ia, cs.B2 * ia, cs.B3 * ia};
  if (DRIFT)
    hits = drift_floors(Pnew, Bnew, m, fl[0], fl[1], L.ph.bsq_rho_max, L.ph.bsq_u_max,
                        L.ph.gamma_max, L.ph.gam, L.ph.tol, L.ph.maxit);
  else
    hits = apply_floors(Pnew, Bnew, m, fl[0], fl[1], L.ph.bsq_rho_max, L.ph.bsq_u_max,
                        L.ph.gamma_max);
  bool ok = Pnew[0] > 0.0 && Pnew[1] > 0.0;
#pragma unroll
  for (int v = 0; v < 5; v++) ok = ok && isfinite(Pnew[v]);
#pragma unroll
  for (int v = 0; v < 3; v++) ok = ok && isfinite(Bnew[v]);
  bad = ok ? 0 : 1;
#pragma unroll
  for (int v = 0; v < 5; v++) Pout[5 * bi.off + (int64_t)v * bi.vol + c.loc] = Pnew[v];
  if (NEXT_DT) dtc = cell_dt(Pnew, Bnew, m, L.ph, bi.idx);
}

// Statistics of a workgroup (inversion tiers, Newton iteration numbers, floor limits):
// counted in LDS, then added per workgroup into one copy of the accumulators (atomics
// from every wave on the few counter addresses serialise and cost more than the update
// itself; spread over the copies, a few dozen workgroups meet on one address per launch)
template <bool STATS, bool NEXT_DT>
__device__ __forceinline__ void update_epilogue(const Launch& L, const BlockTile& bt, bool valid,
                                                int tier, int iters, int hits, int bad,
                                                bool learned, double dtc,
                                                double* __restrict__ dt_part) {
  if (NEXT_DT) {
    const double r = block_min(dtc);
    if (threadIdx.x == 0) dt_part[bt.slot] = r;
  }
  if (STATS) {
    __shared__ uint32_t cnt[NSTAT];
    for (int q = threadIdx.x; q < NSTAT; q += NT) cnt[q] = 0;
    __syncthreads();
    wave_count(cnt + ST_TIER, tier, valid);
    wave_count(cnt + ST_HIST, iters < 63 ? iters : 63, valid);
    const long long h = wave_sum(valid ? hits : 0);
    if (lane_id() == 0 && h) atomicAdd(&cnt[ST_FLOORS], (uint32_t)h);
    const unsigned long long lm = __ballot(valid && learned);
    if (lane_id() == 0 && lm) atomicAdd(&cnt[ST_MLP], (uint32_t)__popcll(lm));
    const unsigned long long bm = __ballot(valid && bad);
    if (lane_id() == 0 && bm) atomicAdd(&cnt[ST_BAD], (uint32_t)__popcll(bm));
    __syncthreads();
    unsigned long long* acc = L.stat_acc + (bt.slot & (STAT_COPIES - 1)) * NSTAT;
    for (int q = threadIdx.x; q < NSTAT; q += NT)
      if (cnt[q]) atomicAdd(&acc[q], (unsigned long long)cnt[q]);
  }
}

// the copies of the statistics accumulators added to the counters and cleared: one
// thread per statistic
__global__ __launch_bounds__(128) void k_stats_fold(Counters* __restrict__ cnt,
                                                    unsigned long long* __restrict__ acc) {
  const int q = threadIdx.x;
  if (q >= NSTAT) return;
  unsigned long long t = 0;
  for (int c = 0; c < STAT_COPIES; c++) {
    t += acc[c * NSTAT + q];
    acc[c * NSTAT + q] = 0;
  }
  unsigned long long* dst = q < ST_HIST     ? &cnt->tier[q - ST_TIER]
                            : q < ST_FLOORS ? &cnt->hist[q - ST_HIST]
                            : q == ST_FLOORS ? &cnt->floors
                            : q == ST_MLP    ? &cnt->mlp
                                             : &cnt->bad;
  *dst += t;
}

// fused update: conserved update, optional learned guess, inversion, floors, next dt
// BZ > 0: workgroups are bricks of 256/BZ columns x BZ cells (every block of the launch
// divides into them, brick_x1), with the geometry of their columns staged in LDS
// (conserve_cell).
template <bool STATS, bool NEXT_DT, bool MLP, int OCC, int BZ>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(OCC))) void k_update(
    Launch L, const double* __restrict__ Pn, const double* __restrict__ Bn,
    const double* __restrict__ Ps, const double* __restrict__ Bcs, const double* __restrict__ F,
    const double* __restrict__ E, double dt_factor, double* __restrict__ Pout,
    double* __restrict__ Bout, double* __restrict__ dt_part, const MlpBlob* __restrict__ mlp) {
  constexpr bool BRICK = BZ > 0;
  __shared__ double sgeo[BRICK ? NGEO_C * (256 / BZ) : 1];
  const BlockTile bt = block_tile(L);
  const BlockInfo bi = L.blk[bt.blk];
  const int g = L.ph.ng;
  Cell c;
  bool valid;
  if (BRICK) {
    // brick (b0, b1, b2) of the tile, x1 fastest, bx x by x BZ cells (bx by = 256/BZ,
    // so the thread's column in the brick is t % (256/BZ)); valid for the whole
    // workgroup or none
    constexpr int Z = BRICK ? BZ : 1, COLS = 256 / Z;
    const int bx = brick_x1(bi.n, Z), by = COLS / bx;
    const int nb0 = bi.n[0] / bx, nb1 = bi.n[1] / by, nb2 = bi.n[2] / Z;
    const int t = threadIdx.x;
    valid = bt.tile < nb0 * nb1 * nb2;
    const int b0 = bt.tile % nb0, r = bt.tile / nb0, b1 = r % nb1, b2 = r / nb1;
    c.I = g + b0 * bx + (t & (bx - 1));
    c.J = g + b1 * by + ((t & (COLS - 1)) / bx);
    c.K = g + b2 * Z + t / COLS;
    c.loc = ((int64_t)c.K * bi.np[1] + c.J) * bi.np[0] + c.I;
  } else {
    valid = region_cell(bi, bt.tile * NT + threadIdx.x, bi.n[0], bi.n[1], bi.n[2], g, g, g, c);
  }
  int tier = 0, iters = 0, hits = 0, bad = 0;
  double dtc = __longlong_as_double(0x7FF0000000000000LL);
  const int64_t col = valid ? geo_col(L.geo, bi, c.J, c.I) : 0;
  Metric m;
  C2PIn cs;
  double PS[5], fl[2];
  if (valid) {
    if (!BRICK) m = load_metric(L.geo.c, L.geo.ncol, col);
    double U[9];
    conserve_cell<BZ>(L, bi, c, m, sgeo, col, Pn, Bn, Ps, Bcs, F, E, dt_factor, Bout, U, PS,
                         fl);
    c2p_setup(U, m, L.ph.gam, cs);
  }
  bool first = false;
  double W0 = 0.0, v0 = 0.0;
  if (MLP) first = learned_guess(mlp, cs, m, valid, PS, W0, v0);
  if (valid)
    invert_cell<NEXT_DT, false>(L, bi, c, m, col, cs, first, W0, v0, PS, fl, Pout, tier, iters,
                                hits, bad, dtc);
  update_epilogue<STATS, NEXT_DT>(L, bt, valid, tier, iters, hits, bad, first, dtc, dt_part);
}

// split update, first half: the conserved state of every cell into ubuf [9][cell]
__global__ __launch_bounds__(NT) void k_conserve(Launch L, const double* __restrict__ Pn,
                                                 const double* __restrict__ Bn,
                                                 const double* __restrict__ Ps,
                                                 const double* __restrict__ Bcs,
                                                 const double* __restrict__ F,
                                                 const double* __restrict__ E, double dt_factor,
                                                 double* __restrict__ Bout,
                                                 double* __restrict__ ubuf) {
  const BlockTile bt = block_tile(L);
  const BlockInfo bi = L.blk[bt.blk];
  const int g = L.ph.ng;
  Cell c;
  if (!region_cell(bi, bt.tile * NT + threadIdx.x, bi.n[0], bi.n[1], bi.n[2], g, g, g, c)) return;
  const int64_t col = geo_col(L.geo, bi, c.J, c.I);
  const Metric m = load_metric(L.geo.c, L.geo.ncol, col);
  double U[9], PS[5], fl[2];
  Metric mc = m;
  conserve_cell<0>(L, bi, c, mc, nullptr, col, Pn, Bn, Ps, Bcs, F, E, dt_factor, Bout, U, PS,
                       fl);
  double* u = ubuf + 9 * bi.off + c.loc;
#pragma unroll
  for (int q = 0; q < 9; q++) u[(int64_t)q * bi.vol] = U[q];
}

// split update, second half: inversion, floors (DRIFT: in the drift frame; the fused
// update has fixed-utilde floors only), next dt from ubuf
template <bool STATS, bool NEXT_DT, bool MLP, int OCC, bool DRIFT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(OCC))) void k_invert(
    Launch L, const double* __restrict__ Ps, const double* __restrict__ ubuf,
    double* __restrict__ Pout, double* __restrict__ dt_part, const MlpBlob* __restrict__ mlp) {
  const BlockTile bt = block_tile(L);
  const BlockInfo bi = L.blk[bt.blk];
  const int g = L.ph.ng;
  Cell c;
  const bool valid = region_cell(bi, bt.tile * NT + threadIdx.x, bi.n[0], bi.n[1], bi.n[2], g,
                                 g, g, c);
  int tier = 0, iters = 0, hits = 0, bad = 0;
  double dtc = __longlong_as_double(0x7FF0000000000000LL);
  const int64_t col = valid ? geo_col(L.geo, bi, c.J, c.I) : 0;
  Metric m;
  C2PIn cs;
  double PS[5], fl[2];
  if (valid) {
    m = load_metric(L.geo.c, L.geo.ncol, col);
    double U[9];
    const double* u = ubuf + 9 * bi.off + c.loc;
#pragma unroll
    for (int q = 0; q < 9; q++) U[q] = u[(int64_t)q * bi.vol];
#pragma unroll
    for (int v = 0; v < 5; v++) PS[v] = Ps[5 * bi.off + (int64_t)v * bi.vol + c.loc];
    fl[0] = L.geo.c[RHOFL * L.geo.ncol + col];
    fl[1] = L.geo.c[UFL * L.geo.ncol + col];
    c2p_setup(U, m, L.ph.gam, cs);
  }
  bool first = false;
  double W0 = 0.0, v0 = 0.0;
  if (MLP) first = learned_guess(mlp, cs, m, valid, PS, W0, v0);
  if (valid)
    invert_cell<NEXT_DT, DRIFT>(L, bi, c, m, col, cs, first, W0, v0, PS, fl, Pout, tier, iters,
                                hits, bad, dtc);
  update_epilogue<STATS, NEXT_DT>(L, bt, valid, tier, iters, hits, bad, first, dtc, dt_part);
}

// ------------------------------------------------------------- Courant reduction

// the minimum cell time step over all interior cells, as per-workgroup partials
__global__ __launch_bounds__(NT) void k_dt(Launch L, const double* __restrict__ P,
                                           const double* __restrict__ B,
                                           double* __restrict__ dt_part) {
  const BlockTile bt = block_tile(L);
  const BlockInfo bi = L.blk[bt.blk];
  const int g = L.ph.ng;
  Cell c;
  const bool valid = region_cell(bi, bt.tile * NT + threadIdx.x, bi.n[0], bi.n[1], bi.n[2], g,
                                 g, g, c);
  double dtc = __longlong_as_double(0x7FF0000000000000LL);
  if (valid) {
    const int64_t V = bi.vol, l = c.loc;
    const int64_t s2 = bi.np[0], s3 = (int64_t)bi.np[0] * bi.np[1];
    const int64_t col = geo_col(L.geo, bi, c.J, c.I);
    const Metric m = load_metric(L.geo.c, L.geo.ncol, col);
    double Pc[5], Bc[3];
#pragma unroll
    for (int v = 0; v < 5; v++) Pc[v] = P[5 * bi.off + (int64_t)v * V + l];
    const double* b = B + 3 * bi.off;
    Bc[0] = 0.5 * (b[l] + b[l + 1]) / m.gdet;
    Bc[1] = 0.5 * (b[V + l] + b[V + l + s2]) / m.gdet;
    Bc[2] = 0.5 * (b[2 * V + l] + b[2 * V + l + s3]) / m.gdet;
    dtc = cell_dt(Pc, Bc, m, L.ph, bi.idx);
  }
  const double r = block_min(dtc);
  if (threadIdx.x == 0) dt_part[bt.slot] = r;
}

// one workgroup reduces the partials into the step's dt (order-free minimum)
__global__ __launch_bounds__(NT) void k_dt_final(Counters* cnt, const double* __restrict__ part,
                                                 int64_t n) {
  double v = __longlong_as_double(0x7FF0000000000000LL);
  for (int64_t i = threadIdx.x; i < n; i += NT) v = fmin(v, part[i]);
  const double r = block_min(v);
  if (threadIdx.x == 0) cnt->dt_bits = (unsigned long long)__double_as_longlong(r);
}

__global__ void k_reset(Counters* cnt, unsigned long long* acc, int all) {
  const int t = threadIdx.x;
  for (int q = t; q < STAT_COPIES * NSTAT; q += blockDim.x) acc[q] = 0;
  if (t < 5) cnt->tier[t] = 0;
  if (t < 64) cnt->hist[t] = 0;
  if (t == 0) {
    cnt->floors = 0;
    cnt->mlp = 0;
    cnt->bad = 0;
    cnt->divb_abs = 0;
    cnt->divb_rel = 0;
    cnt->dt_bits = 0x7FF0000000000000ULL;
    if (all) {
      cnt->t_sim = 0.0;
      cnt->dt_last = 0.0;
    }
  }
}

__global__ void k_tsim(Counters* cnt, double courant) {
  if (threadIdx.x == 0) {
    const double dt = courant * __longlong_as_double((long long)cnt->dt_bits);
    cnt->t_sim += dt;
    cnt->dt_last = dt;
  }
}

__global__ __launch_bounds__(NT) void k_copy(const double* __restrict__ s, double* __restrict__ d,
                                             int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    d[i] = s[i];
}

// ----------------------------------------------------------------- divergence

__global__ __launch_bounds__(NT) void k_divb(Launch L, const double* __restrict__ B,
                                             double* __restrict__ field,
                                             double* __restrict__ part) {
  const Tile tl = xcd_tile();
  const BlockInfo bi = L.blk[L.blist ? L.blist[tl.y] : tl.y];
  const int g = L.ph.ng;
  Cell c;
  const bool valid = region_cell(bi, tl.x * NT + threadIdx.x, bi.n[0], bi.n[1], bi.n[2], g,
                                 g, g, c);
  double a = 0.0, r = 0.0;
  if (valid) {
    const int64_t V = bi.vol, l = c.loc;
    const int64_t s2 = bi.np[0], s3 = (int64_t)bi.np[0] * bi.np[1];
    const double* b = B + 3 * bi.off;
    const double d1 = b[l + 1], d0 = b[l], e1 = b[V + l + s2], e0 = b[V + l];
    const double f1 = b[2 * V + l + s3], f0 = b[2 * V + l];
    const double dv = (d1 - d0) / bi.dx[0] + (e1 - e0) / bi.dx[1] + (f1 - f0) / bi.dx[2];
    const double den = (fabs(d1) + fabs(d0)) / bi.dx[0] + (fabs(e1) + fabs(e0)) / bi.dx[1] +
                       (fabs(f1) + fabs(f0)) / bi.dx[2];
    if (field) field[5 * bi.off + l] = dv;
    a = fabs(dv);
    // relative where the face values carry full precision (den >= 2^-969, 2^53 times the
    // smallest normal double); a field-free region's subnormal values carry none
    r = den >= 0x1p-969 ? a / den : 0.0;
  }
  // workgroup maxima as partials [2][slot] (reduced by k_divb_final)
  __shared__ double red[2][NT / 64];
  a = wave_max(a);
  r = wave_max(r);
  if (lane_id() == 0) {
    red[0][threadIdx.x / 64] = a;
    red[1][threadIdx.x / 64] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 1; w < NT / 64; w++) {
      a = fmax(a, red[0][w]);
      r = fmax(r, red[1][w]);
    }
    const int64_t n = (int64_t)gridDim.x * gridDim.y;
    const int64_t slot = (int64_t)tl.y * gridDim.x + tl.x;
    part[slot] = a;
    part[n + slot] = r;
  }
}

__global__ __launch_bounds__(NT) void k_divb_final(Counters* __restrict__ cnt,
                                                   const double* __restrict__ part, int64_t n) {
  __shared__ double red[2][NT / 64];
  double a = 0.0, r = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += NT) {
    a = fmax(a, part[i]);
    r = fmax(r, part[n + i]);
  }
  a = wave_max(a);
  r = wave_max(r);
  if (lane_id() == 0) {
    red[0][threadIdx.x / 64] = a;
    red[1][threadIdx.x / 64] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 1; w < NT / 64; w++) {
      a = fmax(a, red[0][w]);
      r = fmax(r, red[1][w]);
    }
    atomicMax(&cnt->divb_abs, (unsigned long long)__double_as_longlong(a));
    atomicMax(&cnt->divb_rel, (unsigned long long)__double_as_longlong(r));
  }
}

// -------------------------------------------------------------- cell extraction

// interior cells as flat batches: P[5][n], B[3][n] (coordinate field), geom[15][n]; the
// cells of block b start at b * (cells per block), order k, j, i (uniform block sizes)
// boff: first output index of each block (blocks of uneven sizes), or null for blocks of
// one size
__global__ __launch_bounds__(NT) void k_extract(Launch L, const double* __restrict__ Pin,
                                                const double* __restrict__ Bin, int64_t n,
                                                const int64_t* __restrict__ boff,
                                                double* __restrict__ P, double* __restrict__ B,
                                                double* __restrict__ geom) {
  const BlockInfo bi = L.blk[blockIdx.y];
  const int g = L.ph.ng;
  Cell c;
  const int t = blockIdx.x * NT + threadIdx.x;
  if (!region_cell(bi, t, bi.n[0], bi.n[1], bi.n[2], g, g, g, c)) return;
  const int64_t o = (boff ? boff[blockIdx.y] : (int64_t)blockIdx.y * bi.n[0] * bi.n[1] * bi.n[2]) + t;
  const int64_t V = bi.vol, l = c.loc;
  const int64_t s2 = bi.np[0], s3 = (int64_t)bi.np[0] * bi.np[1];
  const int64_t col = geo_col(L.geo, bi, c.J, c.I);
  for (int q = 0; q < NGEO_F; q++) geom[q * n + o] = L.geo.c[q * L.geo.ncol + col];
  const double gdet = L.geo.c[GDET * L.geo.ncol + col];
  for (int v = 0; v < 5; v++) P[v * n + o] = Pin[5 * bi.off + v * V + l];
  const double* b = Bin + 3 * bi.off;
  B[o] = 0.5 * (b[l] + b[l + 1]) / gdet;
  B[n + o] = 0.5 * (b[V + l] + b[V + l + s2]) / gdet;
  B[2 * n + o] = 0.5 * (b[2 * V + l] + b[2 * V + l + s3]) / gdet;
}

void launch_extract(const Launch& L, const double* Pin, const double* Bin, int64_t n,
                    const int64_t* boff, double* P, double* B, double* geom) {
  const int64_t r = (int64_t)L.max_n[0] * L.max_n[1] * L.max_n[2];
  hipLaunchKernelGGL(k_extract, dim3((unsigned)((r + NT - 1) / NT), L.nblk), dim3(NT), 0, L.stream,
                     L, Pin, Bin, n, boff, P, B, geom);
}

// ------------------------------------------------------------ batch inversion

__global__ __launch_bounds__(NT) void k_c2p_batch(int64_t n, const double* __restrict__ U,
                                                  const double* __restrict__ geom,
                                                  const double* __restrict__ guess,
                                                  const double* __restrict__ prev,
                                                  double* __restrict__ P, int32_t* __restrict__ iters,
                                                  int32_t* __restrict__ tier, double gam, double tol,
                                                  int32_t maxit) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const Metric m = load_metric(geom, n, i);
  double u[9], gs[5], pv[5], out[5];
#pragma unroll
  for (int q = 0; q < 9; q++) u[q] = U[q * n + i];
  bool distinct = false;
#pragma unroll
  for (int v = 0; v < 5; v++) {
    gs[v] = guess[v * n + i];
    pv[v] = prev[v * n + i];
    distinct |= gs[v] != pv[v];
  }
  int it = 0;
  const int t = cons2prim(u, m, gam, gs, pv, distinct, tol, maxit, out, it);
#pragma unroll
  for (int v = 0; v < 5; v++) P[v * n + i] = out[v];
  iters[i] = it;
  tier[i] = t;
}

// the same with the learned first guess: every lane of a workgroup takes part in the
// network's wavefront products, lanes past the end with a copy of the last cell
__global__ __launch_bounds__(NT) void k_c2p_batch_mlp(int64_t n, const double* __restrict__ U,
                                                      const double* __restrict__ geom,
                                                      const double* __restrict__ prev,
                                                      double* __restrict__ P,
                                                      int32_t* __restrict__ iters,
                                                      int32_t* __restrict__ tier, double gam,
                                                      double tol, int32_t maxit,
                                                      const MlpBlob* __restrict__ mlp) {
  const int64_t i0 = (int64_t)blockIdx.x * NT + threadIdx.x;
  const bool valid = i0 < n;
  const int64_t i = valid ? i0 : n - 1;
  const Metric m = load_metric(geom, n, i);
  double u[9];
#pragma unroll
  for (int q = 0; q < 9; q++) u[q] = U[q * n + i];
  C2PIn s;
  c2p_setup(u, m, gam, s);
  double W0 = 0.0, v0 = 0.0;
  const bool first = mlp_guess_block(mlp, s, m, valid, W0, v0);
  if (!valid) return;
  double pv[5], out[5];
#pragma unroll
  for (int v = 0; v < 5; v++) pv[v] = prev[v * n + i];
  int it = 0;
  const int t = c2p_solve(s, m, first, W0, v0, pv, tol, maxit, out, it);
#pragma unroll
  for (int v = 0; v < 5; v++) P[v * n + i] = out[v];
  iters[i] = it;
  tier[i] = t;
}

// ================================================================== launchers

static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

void launch_ghosts(const Launch& L, const GhostLists& G, double* P, double* B) {
  if (G.end[3] == 0) return;
  hipLaunchKernelGGL(k_ghosts, dim3(cdiv(G.end[3], NT)), dim3(NT), 0, L.stream, G, P, B);
}

// The grid of a stage kernel over region class cls (r: cells of the largest block's
// region): the launch's work list when it has one, else max tiles x blocks.  Lc is the
// launch's copy that carries the list to the kernel.
static dim3 stage_grid(const Launch& L, int cls, int64_t r, Launch& Lc) {
  Lc = L;
  Lc.wl = nullptr;
  if (cls >= 0 && L.wls[cls]) {
    Lc.wl = L.wls[cls];
    return dim3((unsigned)L.nwls[cls]);
  }
  return dim3(cdiv(r, NT), L.nblk);
}

void launch_bcell(const Launch& L, const double* B, double* Bc) {
  const int64_t r = (int64_t)(L.max_np[0] - 1) * (L.max_np[1] - 1) * (L.max_np[2] - 1);
  Launch Lc;
  const dim3 grid = stage_grid(L, WL_BCELL, r, Lc);
  hipLaunchKernelGGL(k_bcell, grid, dim3(NT), 0, L.stream, Lc, B, Bc);
}

template <int DIR>
static void flux_dir(const Launch& L, int recon, int riemann, const double* P, const double* Bc,
                     const double* B, double* F) {
  const int v = L.var_flux[DIR - 1];
  // faces (or face pairs) of the largest block's region
  int64_t r = 1;
  for (int d = 0; d < 3; d++)
    r *= (d == DIR - 1) ? (FLUX_PAIR[v] ? (L.max_n[d] + 2) / 2 : L.max_n[d] + 1) : L.max_n[d] + 2;
  Launch Lc;
  const dim3 grid = stage_grid(L, (FLUX_PAIR[v] ? WL_PAIR1 : WL_FLUX1) + DIR - 1, r, Lc);
#define GRMHD_FLUX(RC, RM, V)                                                                  \
  if constexpr (FLUX_PAIR[V])                                                                 \
    hipLaunchKernelGGL((k_flux_pair<DIR, RC, RM, FLUX_OCC[V]>), grid, dim3(NT), 0, L.stream, Lc, \
                       P, Bc, B, F);                                                          \
  else                                                                                        \
    hipLaunchKernelGGL((k_flux<DIR, RC, RM, FLUX_OCC[V]>), grid, dim3(NT), 0, L.stream, Lc, P, \
                       Bc, B, F)
#define GRMHD_FLUX_V(RC, RM)                                              \
  switch (v) {                                                            \
    case 0: GRMHD_FLUX(RC, RM, 0); break;                                 \
    case 1: GRMHD_FLUX(RC, RM, 1); break;                                 \
    case 2: GRMHD_FLUX(RC, RM, 2); break;                                 \
    default: GRMHD_FLUX(RC, RM, 3); break;                                \
  }
  if (recon == 0 && riemann == 0) {
    GRMHD_FLUX_V(0, 0);
  } else if (recon == 0) {
    GRMHD_FLUX_V(0, 1);
  } else if (recon == 2 && riemann == 0) {
    GRMHD_FLUX_V(2, 0);
  } else if (recon == 2) {
    GRMHD_FLUX_V(2, 1);
  } else if (recon == 3 && riemann == 0) {
    GRMHD_FLUX_V(3, 0);
  } else if (recon == 3) {
    GRMHD_FLUX_V(3, 1);
  } else if (riemann == 0) {
    GRMHD_FLUX_V(1, 0);
  } else {
    GRMHD_FLUX_V(1, 1);
  }
#undef GRMHD_FLUX_V
#undef GRMHD_FLUX
}

void launch_flux(const Launch& L, int dir, int recon, int riemann, const double* P,
                 const double* Bc, const double* B, double* F) {
  if (dir == 1) flux_dir<1>(L, recon, riemann, P, Bc, B, F);
  else if (dir == 2) flux_dir<2>(L, recon, riemann, P, Bc, B, F);
  else flux_dir<3>(L, recon, riemann, P, Bc, B, F);
}

void launch_emf(const Launch& L, const double* F, double* E, const double* eref) {
  const int64_t r = (int64_t)(L.max_n[0] + 1) * (L.max_n[1] + 1) * (L.max_n[2] + 1);
  Launch Lc;
  const dim3 grid = stage_grid(L, WL_EMF, r, Lc);
  if (eref)
    hipLaunchKernelGGL(k_emf<true>, grid, dim3(NT), 0, L.stream, Lc, F, E, eref);
  else
    hipLaunchKernelGGL(k_emf<false>, grid, dim3(NT), 0, L.stream, Lc, F, E, eref);
}

void launch_emf_ref(const Launch& L, const double* P, const double* Bc, double* eref) {
  const int64_t r = (int64_t)(L.max_n[0] + 2) * (L.max_n[1] + 2) * (L.max_n[2] + 2);
  Launch Lc;
  const dim3 grid = stage_grid(L, WL_EREF, r, Lc);
  hipLaunchKernelGGL(k_emf_ref, grid, dim3(NT), 0, L.stream, Lc, P, Bc, eref);
}

__global__ __launch_bounds__(NT) void k_fill(double* __restrict__ x, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i < n) x[i] = v;
}

void launch_fill(const Launch& L, double* x, int64_t n, double v) {
  if (n > 0) hipLaunchKernelGGL(k_fill, dim3(cdiv(n, NT)), dim3(NT), 0, L.stream, x, n, v);
}

int64_t dt_partials(const Launch& L) {
  const int64_t r = (int64_t)L.max_n[0] * L.max_n[1] * L.max_n[2];
  return (int64_t)cdiv(r, NT) * L.nblk;
}

void launch_stats_fold(const Launch& L) {
  hipLaunchKernelGGL(k_stats_fold, dim3(1), dim3(128), 0, L.stream, L.cnt, L.stat_acc);
}

int64_t launch_update(const Launch& L, const double* Pn, const double* Bn, const double* Ps,
                   const double* Bcs, const double* F, const double* E, double dt_factor,
                   double* Pout, double* Bout, double* dt_part, const void* mlp, double* ubuf) {
  const int64_t r = (int64_t)L.max_n[0] * L.max_n[1] * L.max_n[2];
  // with per-workgroup Courant partials the rectangular grid (the partials' layout)
  Launch Lc;
  const dim3 grid = stage_grid(L, dt_part ? -1 : WL_CELLS, r, Lc);
  const MlpBlob* blob = (const MlpBlob*)mlp;
  // floors in the drift frame run in the split form only
  if ((L.split_upd || L.ph.floor_drift) && ubuf) {
    hipLaunchKernelGGL(k_conserve, grid, dim3(NT), 0, L.stream, Lc, Pn, Bn, Ps, Bcs, F, E,
                       dt_factor, Bout, ubuf);
#define GRMHD_INV(ND, ML, V)                                                                   \
  if (L.ph.floor_drift)                                                                         \
    hipLaunchKernelGGL((k_invert<true, ND, ML, UPD_OCC[V], true>), grid, dim3(NT), 0, L.stream,   \
                       Lc, Ps, ubuf, Pout, dt_part, blob);                                      \
  else                                                                                          \
    hipLaunchKernelGGL((k_invert<true, ND, ML, UPD_OCC[V], false>), grid, dim3(NT), 0, L.stream,  \
                       Lc, Ps, ubuf, Pout, dt_part, blob)
#define GRMHD_INV_V(ND, ML) \
  if (L.var_upd == 0) { GRMHD_INV(ND, ML, 0); } else { GRMHD_INV(ND, ML, 1); }
    if (dt_part && blob) {
      GRMHD_INV_V(true, true);
    } else if (dt_part) {
      GRMHD_INV_V(true, false);
    } else if (blob) {
      GRMHD_INV_V(false, true);
    } else {
      GRMHD_INV_V(false, false);
    }
#undef GRMHD_INV_V
#undef GRMHD_INV
    return (int64_t)grid.x * grid.y;
  }
#define GRMHD_UPD(ND, ML, V)                                                                 \
  if (L.brick_upd == 8)                                                                     \
    hipLaunchKernelGGL((k_update<true, ND, ML, UPD_OCC[V], 8>), grid, dim3(NT), 0, L.stream,  \
                       Lc, Pn, Bn, Ps, Bcs, F, E, dt_factor, Pout, Bout, dt_part, blob);      \
  else if (L.brick_upd == 4)                                                                \
    hipLaunchKernelGGL((k_update<true, ND, ML, UPD_OCC[V], 4>), grid, dim3(NT), 0, L.stream,  \
                       Lc, Pn, Bn, Ps, Bcs, F, E, dt_factor, Pout, Bout, dt_part, blob);      \
  else                                                                                      \
    hipLaunchKernelGGL((k_update<true, ND, ML, UPD_OCC[V], 0>), grid, dim3(NT), 0,           \
                       L.stream, Lc, Pn, Bn, Ps, Bcs, F, E, dt_factor, Pout, Bout, dt_part, blob)
#define GRMHD_UPD_V(ND, ML)                                               \
  switch (L.var_upd) {                                                    \
    case 0: GRMHD_UPD(ND, ML, 0); break;                                  \
    default: GRMHD_UPD(ND, ML, 1); break;                                 \
  }
  if (dt_part && blob) {
    GRMHD_UPD_V(true, true);
  } else if (dt_part) {
    GRMHD_UPD_V(true, false);
  } else if (blob) {
    GRMHD_UPD_V(false, true);
  } else {
    GRMHD_UPD_V(false, false);
  }
#undef GRMHD_UPD_V
#undef GRMHD_UPD
  return (int64_t)grid.x * grid.y;
}

int64_t launch_dt(const Launch& L, const double* P, const double* B, double* dt_part,
                  bool work_list) {
  const int64_t r = (int64_t)L.max_n[0] * L.max_n[1] * L.max_n[2];
  Launch Lc;
  const dim3 grid = stage_grid(L, work_list ? WL_CELLS : -1, r, Lc);
  hipLaunchKernelGGL(k_dt, grid, dim3(NT), 0, L.stream, Lc, P, B, dt_part);
  return (int64_t)grid.x * grid.y;
}

void launch_dt_final(const Launch& L, const double* dt_part) {
  hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(NT), 0, L.stream, L.cnt, dt_part, dt_partials(L));
}

void launch_counters_reset(const Launch& L, bool all) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, L.stream, L.cnt, L.stat_acc, all ? 1 : 0);
}

void launch_tsim(const Launch& L) {
  hipLaunchKernelGGL(k_tsim, dim3(1), dim3(64), 0, L.stream, L.cnt, L.ph.courant);
}

void launch_copy(const Launch& L, const double* src, double* dst, int64_t n) {
  const unsigned nb = (unsigned)std::min<int64_t>(cdiv(n, NT), 4096);
  hipLaunchKernelGGL(k_copy, dim3(nb), dim3(NT), 0, L.stream, src, dst, n);
}

void launch_divb(const Launch& L, const double* B, double* field, double* part) {
  const int64_t r = (int64_t)L.max_n[0] * L.max_n[1] * L.max_n[2];
  const dim3 grid(cdiv(r, NT), L.nblk);
  hipLaunchKernelGGL(k_divb, grid, dim3(NT), 0, L.stream, L, B, field, part);
  hipLaunchKernelGGL(k_divb_final, dim3(1), dim3(NT), 0, L.stream, L.cnt, part,
                     (int64_t)grid.x * grid.y);
}

void launch_c2p_batch(int64_t n, const double* U, const double* geom, const double* guess,
                      const double* prev, double* P, int32_t* iters, int32_t* tier, double gam,
                      double tol, int32_t maxit, const void* mlp, hipStream_t stream) {
  if (n == 0) return;
  if (mlp)
    hipLaunchKernelGGL(k_c2p_batch_mlp, dim3(cdiv(n, NT)), dim3(NT), 0, stream, n, U, geom, prev,
                       P, iters, tier, gam, tol, maxit, (const MlpBlob*)mlp);
  else
    hipLaunchKernelGGL(k_c2p_batch, dim3(cdiv(n, NT)), dim3(NT), 0, stream, n, U, geom, guess,
                       prev, P, iters, tier, gam, tol, maxit);
}

}  // namespace grmhd
