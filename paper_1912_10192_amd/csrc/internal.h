// internal.h -- structures shared by the host planner and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "../../include/grmhd.h"

namespace grmhd {

// one block as the kernels see it
struct BlockInfo {
  int64_t off;      // cell offset of the block in the packed layout
  int32_t np[3];    // padded extents n + 2 ng + 1
  int32_t n[3];     // interior cells
  int32_t gorg[3];  // geometry-table index of local index 0 in x1, x2 (x3 unused)
  int32_t vol;      // np1 np2 np3
  int32_t lat;
  int32_t gti;      // row length of the block's geometry table
  int64_t gbase;    // first column of the block's geometry table (one table per x1-x2 level)
  double dx[3];     // cell spacing at the block's refinement level
  double idx[3];    // 1 / dx
};

// one ghost copy: destination (block, local), source (block | flags << 24, local)
struct GhostOp {
  int32_t dst_blk, dst_loc, src_blkf, src_loc;
};
enum { GF_FLIP = 1, GF_CLAMP_NEG = 2, GF_CLAMP_POS = 4, GF_ZERO = 8, GF_SLOW = 16, GF_FAST = 32 };

// A ghost copy as the kernels run it, resolved against the block table: element indices
// into the packed arrays (cells: variable 0 of P, then strides dvol / svol per variable;
// faces: the element of the list's component), svol_fl = source volume | flags << 24.
struct GhostIdx {
  uint32_t dst, src, dvol, svol_fl;
};

// A ghost cell copied together with the ghost faces at its local index that are plain
// copies of the faces at its source's local index (same source block, no flip, no
// zero, the same time relation): element indices of variable 0 of the primitives (dp,
// sp) and of component 0 of the face field (db, sb); dvol_fc = destination volume |
// carried face components (bits 0-2) << 24; svol_fl = source volume | the cell's flags
// << 24.  One index record serves up to eight copied values.
struct GhostCF {
  uint32_t dp, sp, db, sb, dvol_fc, svol_fl;
};

// The lists of one fill run as one launch: the cells with their carried faces, then the
// remaining faces of components 1..3 (ops[1..3]; ops[0] unused); thread t takes entry t
// of their concatenation (end: running totals).
struct GhostLists {
  const GhostCF* cf;
  const GhostIdx* ops[4];
  int64_t end[4];
};

// A ghost value that involves another refinement level: a restriction of a finer
// neighbour or a prolongation from a coarser one.  Samples are interior values of other
// blocks (or of the block itself) at the source's own level; the op combines them.
//   mode bits 0-2   prolonged dimensions (minmod slopes, or for a face component along
//                   its normal: the face cuts or lies on a coarse face)
//   mode bits 4-6   the child lies in the upper half of its parent along that dimension
//   mode bit 8      a face cutting a coarse cell: mean of the stencils on its two faces
//   mode bits 16-23 boundary flags applied to the result (GF_*)
// Samples: cells -- centre, then (minus, plus) per prolonged dimension in increasing
// order; faces -- per stencil, the coarse face then (minus, plus) per prolonged
// transverse dimension.  Without prolonged dimensions a single sample.
struct AmrOp {
  int32_t dst_blk, dst_loc, mode, samp;
};
// the four refinement lists of one fill as one launch (as GhostLists)
struct AmrLists {
  const AmrOp* ops[4];
  int64_t end[4];
};
// block | flags << 24 (time and boundary flags of this value), local index of the value
// (a cell, or a face of the op's component), and the dimensions averaged by a
// restriction (0: the value itself)
struct AmrSample {
  int32_t blkf, loc, mask, pad;
};

// One box of a regrid: the cells lo .. lo + ext - 1 (local, at the new block's levels)
// of new block nb, all covered by old block ob; r = new level - old level per dimension
// (-1: restricted, 0: copied, +1: prolonged); on, oo: the two blocks' origins, each at its
// own levels; top: the box reaches nb's upper face in that dimension, whose faces it then
// also fills
struct RegridOp {
  int32_t nb, ob;
  int32_t lo[3], ext[3], r[3], on[3], oo[3], top[3];
};
enum { AM_PDIMS = 7, AM_UPPER_SHIFT = 4, AM_TWO = 256, AM_FLAGS_SHIFT = 16 };

// A value that is the mean of n (1, 2 or 4) elements of one array, per component:
//   X[dst + q dstride] = (sum_i X[src_i + q sstride]) / n,  q < ncomp.
// Used where a block takes the values of a finer block of its own time level in each
// stage: kind 0 the face fluxes of a refinement face (8 components), kind 1 the EMF of
// an edge whose finest holder is finer (1 component), kind 2 the coarse copy of a
// refinement face (the face field, after the update).  Sources are never destinations
// of the same list, so the items of one list run in any order.
struct MeanItem {
  int64_t dst;
  int64_t src[4];
  int32_t n, ncomp, dstride, sstride;
  int32_t kind, pad;
};

// One element a block's corrector contributes to the time-integrated registers: kind 0
// the face flux at element src of F (the six conserved components 0-4 and 7, stride
// apart), kind 1 the EMF at element src of E.  Slot `slot` of the flux or EMF registers:
// step set = dt value, pair set = sum over the two steps a slower neighbour spans.
struct RegItem {
  int64_t src;
  int32_t slot, kind, stride, pad;
};

// End of a slower block's step, per cell whose conserved state or faces change:
// the cell (block, padded local index) and up to three flux corrections, one per
// boundary face of the cell shared with a faster block:
//   dU += (mine - mean(theirs)) / dx * sgn
// with mine the step register of the block's own face and theirs the pair registers of
// the faster block's sub-faces (nth of them).
struct FluxTerm {
  int32_t mine, th[4], nth, sgn, pad;
  double dx;
};
struct SyncCell {
  int32_t blk, loc, nt, pad;
  FluxTerm t[3];
};
// ... and per face of the slower block that changes: constrained-transport corrections
// from up to four edges whose dominant holder is faster,
//   B += sgn (mean(theirs) - mine) / dx
// or (ncopy > 0) the faster block's copy of a shared face: the mean of its ncopy faces
// at local indices csrc of block cblk (the same component), which takes precedence.
struct EdgeTerm {
  int32_t mine, th[2], nth, sgn, pad;
  double dx;
};
struct SyncFace {
  int32_t blk, comp, loc, nt;
  int32_t cblk, ncopy, csrc[4];
  EdgeTerm t[4];
};

static_assert(sizeof(MeanItem) == 64 && sizeof(RegItem) == 24 && sizeof(SyncCell) == 136 &&
                  sizeof(SyncFace) == 168,
              "list layouts as exported by grmhd_plan_dump");

// geometry tables: SoA [quantity][column]; one table per pair of x1/x2 refinement
// levels, column = gbase + j * gti + i of the block's table
struct GeoTab {
  const double* c;    // centre: NGEO_C quantities
  const double* f1;   // x1 faces: NGEO_F
  const double* f2;   // x2 faces: NGEO_F (sqrt(-g) = 0 marks the polar axis)
  int64_t ncol;       // columns of all tables together (stride between quantities)
};

struct Counters {   // device counters of one grmhd_step call
  unsigned long long tier[5];
  unsigned long long hist[64];
  unsigned long long floors;
  unsigned long long mlp;         // inversions started from the learned guess
  unsigned long long bad;         // cells left non-finite or with rho <= 0 or u <= 0
  unsigned long long dt_bits;     // min over cells of 1/sum_d(v_d/dx_d), as IEEE bits
  unsigned long long divb_abs;    // max |div B| bits
  unsigned long long divb_rel;
  double t_sim;
  double dt_last;
};

struct Phys {
  double gam, courant, tol;
  double bsq_rho_max, bsq_u_max, gamma_max;
  int32_t maxit;
  int32_t ng;
  int32_t floor_drift;   // floors in the drift frame (else at fixed utilde)
  int32_t pad;
};

__host__ __device__ inline int64_t geo_col(const GeoTab&, const BlockInfo& bi, int J, int I) {
  return bi.gbase + (int64_t)(bi.gorg[1] + J) * bi.gti + (bi.gorg[0] + I);
}

// region classes of the stage kernels' work lists: padded block, faces per direction,
// edges, interior cells
// (WL_EREF: the interior cells and one layer around them, whose own-state EMFs the
// upwinded edge EMFs read)
enum { WL_BCELL = 0, WL_FLUX1, WL_FLUX2, WL_FLUX3, WL_EMF, WL_CELLS, WL_PAIR1, WL_PAIR2, WL_PAIR3,
       WL_EREF, WL_N };
constexpr int STAGE_NT = 256;   // threads per workgroup of the stage kernels

// statistics of the update kernels: inversion tier counts, Newton iteration histogram,
// floor limits, inversions that used the learned guess.  Each workgroup adds its nonzero
// counts into one of STAT_COPIES copies of the accumulators (by workgroup index, so few
// workgroups meet on one address); launch_stats_fold adds the copies to the counters
// and clears them.
enum { ST_TIER = 0, ST_HIST = 5, ST_FLOORS = 69, ST_MLP = 70, ST_BAD = 71, NSTAT = 72 };
constexpr int STAT_COPIES = 64;

// occupancy variants of the flux and update kernels (see kernels.hip)
constexpr int NVAR_FLUX = GRMHD_NVAR_FLUX, NVAR_UPD = GRMHD_NVAR_UPD;

struct Launch {
  const BlockInfo* blk;   // device block table
  const int32_t* blist;   // device list of the blocks a launch covers (NULL = all)
  int32_t nblk;           // blocks covered
  int32_t max_np[3];      // largest padded extents
  int32_t max_n[3];       // largest interior extents
  GeoTab geo;
  Phys ph;
  Counters* cnt;
  hipStream_t stream;
  int32_t var_flux[3];    // variant of the flux kernel per direction
  int32_t var_upd;        // variant of the update kernel
  int32_t split_upd;      // 1: the update as two kernels (conserved state, then inversion)
  // Work lists of (block, tile) items for blocks of uneven sizes, one per region class
  // of the listed blocks (NULL: a rectangular grid of max tiles x blocks); wl is the
  // list of the launch in flight, set by the launcher on its own copy.
  const int2* wls[WL_N];
  int32_t nwls[WL_N];
  const int2* wl;
  // statistics accumulators of the update kernels, [STAT_COPIES][NSTAT]
  unsigned long long* stat_acc;
  // 8 or 4: every block divides into update bricks of that many cells along x3
  // (brick_x1): the fused update runs brick by brick with the column geometry staged in
  // LDS; 0: cell tiles
  int32_t brick_upd;
};

// Update bricks of 256 cells: 256/z (x1, x2) columns of z cells along x3 (z = 8, or 4
// where a block's x3 extent is not a multiple of 8), the columns as cols x 1, cols/2 x 2
// or cols/4 x 4 cells in x1 x x2.  brick_x1 is the brick's x1 width for a block of n
// interior cells (the widest that divides), 0 if the block divides into none; the brick
// count then equals the number of 256-cell tiles.
__host__ __device__ inline int brick_x1(const int32_t n[3], int z) {
  const int cols = 256 / z;
  if (n[2] % z != 0) return 0;
  for (int by = 1; by <= 4; by *= 2)
    if (n[0] % (cols / by) == 0 && n[1] % by == 0 && cols / by >= 16) return cols / by;
  return 0;
}

// records the message returned by grmhd_last_error() and returns code (host.cpp)
int set_error(int code, const char* msg);

// kernel launchers (kernels.hip)
void launch_ghosts(const Launch& L, const GhostLists& G, double* P, double* B);
void launch_bcell(const Launch& L, const double* B, double* Bc);
void launch_flux(const Launch& L, int dir, int recon, int riemann, const double* P,
                 const double* Bc, const double* B, double* F);
// edge EMFs from the face fluxes; with eref (the cells' own-state EMFs and conserved
// densities, [4][V] per block at 4 * off, from launch_emf_ref) the upwinded corrections
// are added
void launch_emf(const Launch& L, const double* F, double* E, const double* eref = nullptr);
void launch_emf_ref(const Launch& L, const double* P, const double* Bc, double* eref);
// update of one stage; with dt_part non-null the kernel also writes per-workgroup minima
// of the next Courant step (reduced by launch_dt_final)
// (mlp non-null: learned first guess of the inversion from the packed MLP blob)
// (returns the number of workgroups)
int64_t launch_update(const Launch& L, const double* Pn, const double* Bn, const double* Ps,
                   const double* Bcs, const double* F, const double* E, double dt_factor,
                   double* Pout, double* Bout, double* dt_part, const void* mlp, double* ubuf);
void launch_stats_fold(const Launch& L);
int64_t dt_partials(const Launch& L);
// per-workgroup minima of the Courant step of the listed blocks; over the work list of
// interior cells when work_list is set and the blocks have one (partials: one per item),
// else over the rectangular grid of tiles x blocks (dt_partials); returns the partials
int64_t launch_dt(const Launch& L, const double* P, const double* B, double* dt_part,
                  bool work_list = false);
void launch_dt_final(const Launch& L, const double* dt_part);
void launch_counters_reset(const Launch& L, bool all);
void launch_tsim(const Launch& L);
void launch_copy(const Launch& L, const double* src, double* dst, int64_t n);
void launch_fill(const Launch& L, double* x, int64_t n, double v);
// div B of the face field (field non-null: per cell), maxima through the per-workgroup
// partials part [2][workgroups]
void launch_divb(const Launch& L, const double* B, double* field, double* part);
// boff: first output index of each block, or null when all blocks have one size
void launch_extract(const Launch& L, const double* Pin, const double* Bin, int64_t n,
                    const int64_t* boff, double* P, double* B, double* geom);
// refinement levels (amr.hip)
void launch_amr_ghosts(const Launch& L, const AmrLists& A, const AmrSample* samp,
                       const double* Pmain, const double* Pold, const double* Pcur, double* Pdst,
                       const double* Bmain, const double* Bold, const double* Bcur, double* Bdst,
                       double w);
// a regrid: the new layout's interior faces and cells (conserved: restricted and
// prolonged cells from the conserved vector, then inverted; the boxes' cells, then faces of
// each direction: start[k][op], k = 0 cells, 1..3 faces, with total[k] = start[k][nops])
// from the old layout's padded state, whose ghosts are filled
void launch_regrid(const Launch& Lf, const Launch& Lt, const RegridOp* ops, int64_t nops,
                   const int64_t* start, const int64_t total[4], const double* Pf,
                   const double* Bf, double* Pt, double* Bt, bool conserved);
// the items of a mean list: kind 0 items on X0, the others on X1
void launch_means(const Launch& L, const MeanItem* items, int64_t n, double* X0, double* X1);
// local time stepping (lat.hip)
void launch_ghosts_t(const Launch& L, const GhostLists& G, const double* Pmain,
                     const double* Pold, const double* Pcur, double* Pdst, const double* Bmain,
                     const double* Bold, const double* Bcur, double* Bdst, double w);
void launch_copy_blocks(const Launch& L, const double* src, double* dst, int nvar);
void launch_copy_list(const Launch& L, const uint32_t* ic, int64_t nc, const double* P,
                      double* Pdst, const uint32_t* jf, int64_t nf, const double* B,
                      double* Bdst);
// registers of one level's corrector: regF [2][6][nf] (step, pair), regE [2][ne]
void launch_registers(const Launch& L, const RegItem* items, int64_t n, const double* F,
                      const double* E, double dt_factor, int first, double* regF, int64_t nf,
                      double* regE, int64_t ne);
// end-of-step synchronisation of slower blocks: cells and faces of the levels due
void launch_sync(const Launch& L, const SyncCell* cells, int64_t ncell, const SyncFace* faces,
                 int64_t nface, double* P, double* B, const double* regF, int64_t nf,
                 const double* regE, int64_t ne, double* Ubuf);
// dt of a cycle from n partials of launch_dt: min of partial / 2^lat of its block (the
// block of partial i: work-list item i, or i / gridx on the rectangular grid)
void launch_dt_final_lat(const Launch& L, const double* part, int64_t n, int gridx,
                         const int2* wl);
void launch_tsim_cycle(const Launch& L, double substeps);
void launch_c2p_batch(int64_t n, const double* U, const double* geom, const double* guess,
                      const double* prev, double* P, int32_t* iters, int32_t* tier, double gam,
                      double tol, int32_t maxit, const void* mlp, hipStream_t stream);

}  // namespace grmhd
