/*
 * grmhd.h -- C ABI of libgrmhd.so, the MI355X (gfx950) GRMHD block update.
 *
 * The library advances the ideal GRMHD equations in conservative form (paper
 * Sec. 2.4) on block-structured grids that are uniform in internal coordinates
 * x1 = ln r, x2 = theta, x3 = phi around a Kerr black hole in Kerr-Schild form
 * (Sec. 2.2), or on Cartesian Minkowski grids.  One step is the midpoint
 * predictor/corrector of Sec. 2.1: reconstruction (PPM or PLM-MC), HLLE or LLF
 * fluxes, edge EMFs as the four-flux average and constrained transport of the
 * staggered field (Sec. 2.5), the geometric source (Sec. 2.5), the 2D Newton
 * inversion with entropy backup (Sec. 2.6) and the floors of Sec. 2.7.  The
 * Courant step dt = C0 / (sum_i v_i / dx_i) is taken per cell and reduced on
 * the device (Sec. 2.1).
 *
 * Memory: every large buffer is device memory owned by the caller.  The library
 * allocates no device memory; it keeps host-side metadata only.  grmhd_sizes()
 * says how much the caller must provide.
 *
 * Layout of the state (per block b, blocks packed in table order):
 *   a block of n1 x n2 x n3 cells is stored padded by ng ghost layers below and
 *   ng + 1 above in every dimension, NPd = n_d + 2 ng + 1 cells, local index
 *   (K * NP2 + J) * NP1 + I (x1 fastest).  With V_b = NP1 NP2 NP3 and
 *   off_b = sum_{b' < b} V_b' (grmhd_block_layout):
 *     prim [5 off_b + v V_b + local]   v = rho, u_g, utilde^1, utilde^2, utilde^3
 *     bface[3 off_b + d V_b + local]   sqrt(-g) B^(d+1) on the LOWER d-face of the
 *                                      cell (x1 face at i - 1/2 for d = 0, ...)
 *
 * Errors: every call returns GRMHD_OK (0) or a negative code; the message is
 * available from grmhd_last_error() (thread-local).  Calls are ordered on the
 * HIP stream given at init; calls that return host values synchronise it.
 * A context is not thread-safe; distinct contexts are independent.
 */
#ifndef GRMHD_H
#define GRMHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GRMHD_ABI_VERSION 4

enum { GRMHD_OK = 0, GRMHD_EINVAL = -1, GRMHD_ENOMEM = -2, GRMHD_EHIP = -3,
       GRMHD_ESTATE = -4, GRMHD_EUNSUPPORTED = -5 };
enum { GRMHD_MINK_CART = 0, GRMHD_KS_LOGSPH = 1 };
/* reconstruction (Sec. 2.1): piecewise linear with the monotonised-central limiter, PPM
 * (Colella & Woodward), piecewise linear with the MINMOD limiter (Sec. 7.2's shock tubes
 * compare MINMOD and PPM), or PPM with the optional shock flattener (Colella & Woodward's
 * flattening coefficient from the pressure jump over a cell's neighbours where the flow
 * compresses, pulling the cell's interface values toward its mean) */
enum { GRMHD_PLM_MC = 0, GRMHD_PPM = 1, GRMHD_PLM_MINMOD = 2, GRMHD_PPM_FLAT = 3 };
enum { GRMHD_LLF = 0, GRMHD_HLLE = 1 };
enum { GRMHD_BC_OUTFLOW = 0, GRMHD_BC_POLAR = 1, GRMHD_BC_PERIODIC = 2 };
enum { GRMHD_GUESS_PLAIN = 0, GRMHD_GUESS_MLP = 1 };
/* edge EMFs (Sec. 2.5): the average of the four neighbouring face fluxes of B, or that
 * average with the upwinded corrections of Gardiner & Stone (2005) that the paper applies
 * by default (each corner takes the gradients of the EMF toward the neighbouring cell
 * centres, where the EMF of the cell's own state sits, from the side upstream of the mass
 * flux through the face between the candidates; a mass flux within 1e-12 of the largest
 * conserved density sqrt(-g) rho u^t of the edge's cells counts as zero and takes the
 * mean of both sides) */
enum { GRMHD_EMF_AVERAGE = 0, GRMHD_EMF_UPWIND = 1 };
/* floors (Sec. 2.7): after the Lorentz-factor ceiling, raise rho and u_g to their minima
 * at fixed utilde, or add the missing mass and internal energy as a parcel moving with
 * the drift frame of the field (Ressler et al. 2017; the paper's choice): u_D = g (u +
 * beta b), beta = -b^t / (b^2 u^t), the summed conserved state inverted from the cell's
 * primitives (cells whose inversion needs the entropy or keep-previous tier fall back to
 * the fixed-utilde floors, which also restore the minima after rounding) */
enum { GRMHD_FLOOR_FIXED = 0, GRMHD_FLOOR_DRIFT = 1 };

/* One block of the grid (Sec. 3.3 block structure; Sec. 3.4 coarsening toward the
 * poles is refinement in some dimensions only).  The effective grid n_eff is the grid
 * at the finest level of each dimension; a block at level l in dimension d has cells
 * 2^(lmax_d - l) effective cells wide (lmax_d = the largest level of any block in d),
 * and its origin and extent count cells of its own level.  The blocks must tile the
 * domain without overlap.  Blocks that touch (through faces, edges, corners and the
 * physical boundaries) differ by at most one level per dimension, never finer in one
 * dimension and coarser in another; refined blocks start and end on cells of the
 * coarser neighbour; no refinement jump lies across the polar axis.  Time levels are
 * independent of refinement levels and of the direction of a face; blocks that touch
 * differ by at most one time level. */
typedef struct {
  int32_t lev[3];   /* refinement level per dimension (0 = coarsest)            */
  int32_t lat;      /* local-time-stepping level (0 = fastest)                  */
  int64_t org[3];   /* origin in cells of the block's own level                 */
  int32_t n[3];     /* cells per dimension                                       */
} grmhd_block_desc;

typedef struct {
  int32_t abi_version;        /* GRMHD_ABI_VERSION */
  int32_t coords;             /* GRMHD_MINK_CART or GRMHD_KS_LOGSPH */
  double spin_a;              /* black-hole spin a/M (Kerr-Schild only) */
  double gamma_ad;            /* adiabatic index of p = (gamma - 1) u_g */
  double xmin[3], xmax[3];    /* internal-coordinate extent of the effective grid */
  int32_t n_eff[3];           /* effective cells per dimension */
  int32_t n_ghost;            /* 2 (PLM) or 3 (PPM) */
  int32_t n_blocks;
  int32_t n_lat_levels;       /* 1 = global time step */
  const grmhd_block_desc* blocks;  /* host array of n_blocks, copied at init */
  int32_t recon, riemann;
  int32_t bc[6];              /* x1lo, x1hi, x2lo, x2hi, x3lo, x3hi */
  double courant;             /* C0 */
  double rho_fl_c, rho_fl_p;  /* rho >= rho_fl_c r^rho_fl_p */
  double u_fl_c, u_fl_p;      /* u_g >= u_fl_c r^u_fl_p */
  double bsq_rho_max;         /* b^2/rho ceiling */
  double bsq_u_max;           /* b^2/u_g ceiling */
  double gamma_max;           /* Lorentz-factor ceiling */
  int32_t c2p_guess;          /* GRMHD_GUESS_PLAIN (Newton from the cell's previous
                                 primitives) or GRMHD_GUESS_MLP (the network's guess too:
                                 Newton from whichever of the two has the smaller residual
                                 misfit, then from the other).  Inside the update the
                                 network runs for a group of 256 cells only if the plain
                                 guess of one of them has a residual misfit above 1e-1;
                                 the other groups start from the plain guess */
  int32_t c2p_maxit;          /* Newton iteration cap (50) */
  double c2p_tol;             /* Newton tolerance (1e-12) */
  const void* mlp_weights;    /* device pointer to packed MLP weights, or NULL */
  int32_t batched;            /* 0 = plain: one launch per block and kernel class (the
                                 paper's per-block launches); 1 = batched: one launch per
                                 time level and kernel class over a work list of the
                                 level's blocks, LAT cycles captured as a hipGraph; 2 = the
                                 batched launches without the graph */
  int32_t profile;            /* 1 = time each kernel class with HIP events on the stream */
  int32_t emf;                /* GRMHD_EMF_AVERAGE or GRMHD_EMF_UPWIND */
  int32_t floor_frame;        /* GRMHD_FLOOR_FIXED or GRMHD_FLOOR_DRIFT */
} grmhd_grid_desc;

typedef struct {
  double* prim;               /* device, layout above, interior filled at init */
  double* bface;              /* device, layout above, interior faces filled at init */
  void* work;                 /* device scratch of work_bytes */
  size_t work_bytes;
} grmhd_buffers;

typedef struct {
  int64_t real_zone_cycles;         /* sum over blocks of cells x steps taken */
  int64_t lat_eff_zone_cycles;      /* cells x finest-level steps */
  int64_t amr_lat_eff_zone_cycles;  /* effective-grid cells x finest-level steps */
  int64_t steps_per_level[8];
  int64_t c2p_iter_hist[64];        /* Newton iterations of accepted solves; 63 = bracketing tiers */
  int64_t c2p_tier[5];              /* 0 first Newton start, 1 second start, 2 1D energy, 3 entropy, 4 failed */
  int64_t floor_hits;
  int64_t mlp_guesses;              /* inversions that started from the learned guess */
  double dt_min;                    /* last time step */
  double t_sim;                     /* simulated time since init */
  double kernel_ms;                 /* device time of this call (HIP events) */
  /* with desc.profile: device time and launch count per kernel class, in the order
   * ghost fill, cell field, x1 flux, x2 flux, x3 flux, EMF, cell update, Courant step and
   * statistics reductions */
  double class_ms[8];
  int64_t class_launches[8];
  int64_t bad_states;               /* cells an update left non-finite or with rho <= 0 or u <= 0 */
} grmhd_step_stats;

typedef struct grmhd_ctx grmhd_ctx;

/* Sizes the caller must allocate for desc: prim and bface element counts (doubles)
 * and the work buffer in bytes.  Returns GRMHD_EINVAL for an invalid desc, and for
 * grids whose packed arrays the ghost lists cannot index in 32 bits (a block's padded
 * volume (n + 2 n_ghost + 1)^3 of 2^24 cells or more, or 5 x all padded cells of 2^32
 * or more: about 8.6e8 padded cells, 34 GB per primitive array set). */
int grmhd_sizes(const grmhd_grid_desc* desc, size_t* prim_elems, size_t* bface_elems,
                size_t* work_bytes);

/* Offset (in cells) and padded extents of block b in the prim/bface layout. */
int grmhd_block_layout(const grmhd_grid_desc* desc, int32_t b, int64_t* cell_offset,
                       int32_t np[3]);

/* Build the context: block table, neighbour/ghost maps and geometry tables
 * (metric, inverse, sqrt(-g), lapse at centres and faces; Christoffel symbols at
 * centres, Sec. 2.2), all uploaded into bufs->work on hip_stream.  bufs must
 * outlive the context.  The interior of prim/bface holds the initial state. */
int grmhd_init_grid(const grmhd_grid_desc* desc, const grmhd_buffers* bufs, void* hip_stream,
                    grmhd_ctx** out);

/* Advance n_cycles steps (Sec. 2.1 midpoint method).  stats (host, nullable)
 * receives counters for this call; passing it synchronises the stream.  With stats,
 * the call also checks the state: if any update (the floors applied) left a cell with a
 * non-finite primitive or face-centred field, rho <= 0 or u <= 0, it returns
 * GRMHD_ESTATE (the counters are filled and the steps were taken; the state is not
 * usable).  Without stats nothing is checked. */
int grmhd_step(grmhd_ctx* ctx, int32_t n_cycles, grmhd_step_stats* stats);

/* Autotuner of the two heavy kernels.  The flux kernel (per direction) is built in
 * GRMHD_NVAR_FLUX variants: one face per thread at a minimum of 1, 2, 4 waves per SIMD
 * the compiler must fit, then two faces per thread along the normal (the shared cells'
 * reconstruction done once) at 2; the update kernel in GRMHD_NVAR_UPD occupancy
 * variants (1, 2 waves), and in
 * two forms: one fused kernel, or two (the conserved state of every cell through a
 * buffer, then the inversion).  This times every variant and form on the context's
 * current state (one predictor stage, three launches each after a warm-up) and keeps
 * the fastest for all later launches; without a call the flux kernel uses 4 waves and
 * the update is fused with 1.  choice (host, nullable, 5 ints) receives the chosen
 * flux variants (x1, x2, x3), the update variant and the update form (0 fused, 1
 * split); ms (host, nullable, 3 GRMHD_NVAR_FLUX + 2 GRMHD_NVAR_UPD doubles) the mean
 * milliseconds per variant (flux x1 variants, x2, x3, fused update variants, split
 * update variants).  The state is not modified; counters are reset; synchronises. */
#define GRMHD_NVAR_FLUX 4
#define GRMHD_NVAR_UPD 2
int grmhd_autotune(grmhd_ctx* ctx, int32_t choice[5], double* ms);
/* Sets the kernel variants directly (the layout of grmhd_autotune's choice), for
 * reproducible runs; EINVAL for an index out of range. */
int grmhd_set_variants(grmhd_ctx* ctx, const int32_t choice[5]);

/* Standalone inversion of a flat batch (Sec. 2.6), all pointers device memory:
 *   U[9][n]     conserved state incl. sqrt(-g): rho u^t, T^t_t + rho u^t, T^t_i, B^i, kappa rho u^t
 *   geom[15][n] g_tt g_t1 g_t3 g_11 g_13 g_22 g_33, g^tt g^t1 g^11 g^13 g^22 g^33,
 *               sqrt(-g), lapse  (metrics with the Kerr-Schild sparsity pattern)
 *   guess[5][n] first guess primitives; prev[5][n] plain guess and failure fallback
 *   P[5][n] out primitives; iters[n], tier[n] out (tier as in grmhd_step_stats)
 *   mlp_weights (nullable): a packed network blob (grmhd_mlp_pack); when set, the
 *               network's prediction replaces guess (which may then be NULL)
 * With a first guess distinct from prev, Newton starts from whichever of the two has
 * the smaller residual misfit and falls back to the other (tier 1).
 * No floors are applied.  ctx may be NULL. */
typedef struct {
  int64_t n;
  const double* U;
  const double* geom;
  const double* guess;
  const double* prev;
  double* P;
  int32_t* iters;
  int32_t* tier;
  double gamma_ad;
  double tol;
  int32_t maxit;
  const void* mlp_weights;
} grmhd_c2p_batch;
int grmhd_cons2prim(grmhd_ctx* ctx, const grmhd_c2p_batch* batch, void* hip_stream);

/* Each block's own Courant step (Sec. 2.1, Sec. 3.5: the local Courant condition that
 * sets a block's time level), C0 times the minimum over its interior cells of
 * 1/sum_d(v_d/dx_d), without the block's time-level factor; written to dt (host,
 * n_blocks doubles).  Synchronises.  GRMHD_ESTATE when the state is not in the caller's
 * buffers. */
int grmhd_block_dt(grmhd_ctx* ctx, double* dt);

/* Discrete divergence of the face field over all interior cells:
 * sum_d (Bbar^d_+ - Bbar^d_-)/dx^d.  Writes max |div| and max |div| / (sum_d
 * (|Bbar^d_+| + |Bbar^d_-|)/dx^d) to host scalars (synchronises), the relative form over
 * cells where that scale is at least 2^-969 (subnormal face values carry no relative
 * precision); field (device, nullable) receives the per-cell value in the prim layout
 * of variable 0. */
int grmhd_divb(grmhd_ctx* ctx, double* max_abs, double* max_rel, double* field);

/* Regrid (Sec. 3.3: blocks refined and derefined during a run).  Fills the interior
 * cells and faces of context `to` (a new block layout, created by grmhd_init_grid with
 * its own caller-owned buffers) from the state of context `from` at the end of its last
 * step; both contexts stay the caller's.
 * Layouts: both cover the same domain with the same level-0 grid (n_eff >> lmax per
 * dimension); the new one may add or drop a finest level, its n_eff then doubled or
 * halved.  Each new block is, in every dimension, at the level of each old block it
 * overlaps, one finer or one coarser (never finer in one dimension and coarser in
 * another), and where it is coarser the old block boundaries fall on its cell faces.
 * Cells (mode GRMHD_REGRID_PRIMITIVE): copied from the old block covering the cell,
 * restricted (sqrt(-g)-weighted mean of the covered primitives) or prolonged (the
 * parent's primitives plus +-1/4 of the minmod-limited slope per refined dimension).
 * Cells (mode GRMHD_REGRID_CONSERVED, the conservative form): where not copied, the
 * conserved vector U is restricted (mean of the covered cells' U) or prolonged (the
 * parent's U/sqrt(-g) plus +-1/4 of its minmod slopes, moved by one common amount in all
 * children so that their U, times each child's sqrt(-g), sum to the parent's); the cell
 * field comes from the new faces; then the inversion (from the primitive form's value)
 * and the floors of `to`.  Mass, energy and momenta summed over the grid are then kept
 * to the inversion's tolerance.
 * Faces: taken from the old block covering the cell above the face (below it for a
 * block's upper face): copied, restricted (mean of the fine sub-faces), or prolonged
 * divergence-free (Balsara 2001): a fine face on a parent face is the parent face plus
 * +-1/4 of its minmod slopes in the face's plane, a fine face inside a parent cell the
 * face average of the parent cell's divergence-free reconstruction, so every new cell
 * keeps div B = 0.
 * The old context's ghost values are refreshed first (its interior is not changed); the
 * simulated time carries over.  Synchronises both contexts' streams; allocates and frees
 * a small device table of boxes.  GRMHD_EINVAL for layouts that break the rules above or
 * an unknown mode, GRMHD_ESTATE when `from` holds its state outside the caller's
 * buffers. */
enum { GRMHD_REGRID_PRIMITIVE = 0, GRMHD_REGRID_CONSERVED = 1 };
int grmhd_regrid(grmhd_ctx* from, grmhd_ctx* to, int32_t mode);

/* Host-only planner introspection for bit-exact checks (no device needed): copies the
 * ghost gather list for what = 0 (cell variables) or 1..3 (face component 1..3) as
 * int32 quadruples (dst block, dst local index, src block | flags << 24, src local
 * index); flags 1 = negate utilde^2 / the face value, 2 = clamp utilde^1 <= 0,
 * 4 = clamp utilde^1 >= 0, 8 = zero (polar-axis face), 16 / 32 = the source runs
 * at a slower / faster time level.  what = 4..7: the ghost values that involve another
 * refinement level (cells, face components 1..3) as int32 quadruples (dst block, dst
 * local index, mode, first sample) -- mode bits 0-2 prolonged dimensions, bits 4-6
 * child in the upper half per dimension, bit 8 mean of two face stencils, bits 16-23
 * flags of the result; what = 8: their samples as int32 quadruples (block | flags <<
 * 24, local index, averaged dimensions of a restriction, 0); what = 9: the refinement
 * faces between blocks of one time level (Sec. 3.3) as 13 int32 each (coarse block,
 * fine block, normal dimension, side 0 = the coarse block's lower face / 1 = upper,
 * refined dimensions e[3], shared patch lo[3], hi[3] in the coarse block's global
 * cells); what = 10: the schedule of one local-time-stepping cycle (Sec. 3.5) as int32
 * quadruples (substep, 0 = the block steps / 1 = the slower block is synchronised
 * with faster neighbours, time level, block): steps in launch order, the
 * synchronisations of one substep (independent of each other) in block order;
 * what = 11: the old state a level step saves for faster neighbours (the sources of
 * time-interpolated ghosts, Sec. 3.5) as int32 quadruples (time level, 0 = primitives
 * / 1 = face field, block, element offset in the block's part of the packed array:
 * variable or component x padded volume + local index), per level and list sorted,
 * without repeats; what = 12: the faces each block refluxes at the end of its step
 * (Sec. 3.5, 3.3) as 10 int32 (block, normal dimension, side, padded local face index,
 * faster block, count n, that block's n covering faces, -1 padded to 4); what = 13:
 * the block edges whose dominant holder (fastest, then finest, then lowest index) is
 * faster, as 7 int32 (block, edge direction, local edge index, holder, count n, the
 * holder's n covering edges, -1 padded to 2); what = 14: likewise the edges whose
 * finest holder at the block's own time level is finer (EMF replaced in each stage);
 * what = 15..19: the device lists built from them as raw structures (internal layout,
 * for bounds checks); what = 20: the device ghost copy lists as uploaded, each ghost
 * cell with the ghost faces at its local index that copy the faces at its source's
 * local index unchanged, as 6 uint32 (destination and source element of primitive 0,
 * destination and source element of face component 0, destination padded volume |
 * carried face components (bits 0-2) << 24, source padded volume | cell flags << 24);
 * what = 21..23: the faces of components 1..3 not carried that way, as 4 uint32
 * (destination element, source element, destination padded volume, source padded
 * volume | flags << 24); both in time-level order.  Every table lists blocks in block order.  host_buf NULL queries
 * the size in bytes. */
int grmhd_plan_dump(const grmhd_grid_desc* desc, int32_t what, void* host_buf, size_t* bytes);

/* Planner geometry at one internal-coordinate point (host only, no device needed):
 * out[15] = g_tt g_t1 g_t3 g_11 g_13 g_22 g_33 g^tt g^t1 g^11 g^13 g^22 g^33 sqrt(-g)
 * lapse; conn[40] (nullable) = Gamma^l_{mn} for m <= n at index l*10 + pair(m, n), pairs
 * in the order (0,0) (0,1) (0,2) (0,3) (1,1) (1,2) (1,3) (2,2) (2,3) (3,3).  The
 * Kerr-Schild metric is the Kerr metric (Sec. 2.2) with x1 = ln r. */
int grmhd_geometry_point(int32_t coords, double spin_a, double x1, double x2, double* out,
                         double* conn);

/* ------------------------------------------------------------------------------
 * Learned first guess of the inversion (Sec. 2.6 solves the inversion iteratively;
 * its starting point is free).  An MLP 8 -> 64 -> 64 -> 64 -> 2 (tanh) maps normalised
 * features of a conserved state -- log D, asinh(tau/D), log1p(S^2/D^2), log1p(B^2/D),
 * log1p((S.B)^2/D^3), lapse, adiabatic index, sqrt(det gamma_ij) -- to normalised
 * log Gamma and log(W/D), W = (rho + u + p) Gamma^2.  Weights are FP32 masters
 * (n_params floats: W1[8][64] b1[64] W2[64][64] b2 W3[64][64] b3 W4[64][2] b4[2]);
 * products run on bfloat16 matrix cores with FP32 accumulation.  All pointers are
 * device memory and every call is ordered on hip_stream.
 * ------------------------------------------------------------------------------ */

/* Parameter count, bytes of the packed inference blob (desc.mlp_weights), and floats
 * of training scratch for a batch size. */
int grmhd_mlp_sizes(int32_t batch, size_t* n_params, size_t* blob_bytes, size_t* work_floats);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, step >= 1) on the mean squared error
 * of rows idx[batch] of X[n][8] (normalised features) against Y[n][2] (normalised
 * targets).  params, adam_m, adam_v: n_params floats each, updated in place; loss
 * (device float) receives the batch loss before the update. */
int grmhd_mlp_train_step(float* params, float* adam_m, float* adam_v, int32_t step,
                         const float* X, const float* Y, const int32_t* idx, int32_t batch,
                         float lr, float* work, float* loss, void* hip_stream);

/* The same training step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight training loops, harnesses that forbid hipMalloc): the
 * training scratch lives in a static device array of the library, sized for batches of
 * at most GRMHD_MLP_NOALLOC_MAX_BATCH rows (about 11 MB, one copy per device, held until
 * the process ends).  No allocation of any kind happens on this path.  Larger batches
 * return GRMHD_EINVAL.  All calls on one device share that array: calls that overlap on
 * one device (two streams, two threads) race and must be serialised by the caller.
 * Results are those of grmhd_mlp_train_step on the same inputs. */
#define GRMHD_MLP_NOALLOC_MAX_BATCH 8192
int grmhd_mlp_train_step_noalloc(float* params, float* adam_m, float* adam_v, int32_t step,
                                 const float* X, const float* Y, const int32_t* idx,
                                 int32_t batch, float lr, float* loss, void* hip_stream);

/* Gradients of the same loss without updating (grad_out: n_params floats). */
int grmhd_mlp_gradients(const float* params, const float* X, const float* Y,
                        const int32_t* idx, int32_t batch, float* work, float* grad_out,
                        float* loss, void* hip_stream);

/* Packs master parameters and norm[20] (feature means[8], stds[8], target means[2],
 * stds[2]) into the inference blob (16-byte aligned, blob_bytes). */
int grmhd_mlp_pack(const float* params, const float* norm, void* blob, void* hip_stream);

/* Normalised outputs Y[n][2] of normalised features X[n][8] through a packed blob. */
int grmhd_mlp_forward(const void* blob, const float* X, int64_t n, float* Y, void* hip_stream);

/* U[9][n] from primitives P[5][n], cell-centred field B[3][n] (coordinate B^i) and
 * geom[15][n] (layout of grmhd_c2p_batch), Sec. 2.3-2.5. */
int grmhd_prim2cons_batch(int64_t n, const double* P, const double* B, const double* geom,
                          double gamma_ad, double* U, void* hip_stream);

/* Raw features X[n][8] of U[9][n] and, if P is non-NULL, raw targets Y[n][2] of P;
 * ok[n] = 1 where every value is finite. */
int grmhd_mlp_dataset(int64_t n, const double* U, const double* P, const double* geom,
                      double gamma_ad, float* X, float* Y, int32_t* ok, void* hip_stream);

/* Column-wise normalisation of A[n][cols] in place: with compute = 1 the means and
 * standard deviations are computed first into mean/sd, else the given ones are used. */
int grmhd_mlp_normalize(float* A, int64_t n, int32_t cols, float* mean, float* sd,
                        int32_t compute, void* hip_stream);

/* Every interior cell of the grid as flat batches (block order, then k, j, i):
 * P[5][n] primitives, B[3][n] cell-centred coordinate field, geom[15][n] metric as in
 * grmhd_c2p_batch; n = number of interior cells.  Blocks may differ in size (the first
 * call then keeps a small device table of the blocks' output offsets until
 * grmhd_destroy). */
int grmhd_extract_cells(grmhd_ctx* ctx, double* P, double* B, double* geom);

int grmhd_destroy(grmhd_ctx* ctx);
const char* grmhd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
