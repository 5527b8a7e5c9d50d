/*
 * orc.h -- plain single-threaded FP64 CPU oracle for the GRMHD block update.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this code; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code with the HIP path.
 *
 * What it computes (paper: Liska et al., "H-AMR", arxiv 1912.10192):
 *   Sec. 2.1  midpoint predictor/corrector, HLLE (and LLF) fluxes, PPM / PLM-MC
 *             reconstruction, Courant time step dt = C0/(sum_i 1/dt^i)
 *   Sec. 2.2  Kerr metric in Kerr-Schild form in internal coords (log r, theta, phi),
 *             Christoffel symbols from derivatives of the internal-coordinate metric
 *   Sec. 2.3  primitives (rho, u_g, utilde^i, B^i), b^mu, T^mu_nu, entropy tracer
 *   Sec. 2.4  conservation laws, energy equation with the mass equation added
 *   Sec. 2.5  finite-volume update, geometric source, staggered CT, 4-flux EMF
 *             average, face-to-centre field average
 *   Sec. 2.6  2D Newton inversion, entropy backup inversion
 *   Sec. 2.7  density / internal-energy floors and magnetisation ceilings
 *
 * Array layout (host memory, all doubles):
 *   a grid of n1 x n2 x n3 interior cells padded by ng ghost layers below and
 *   ng+1 above in every dimension: NPd = n_d + 2*ng + 1, index (k*NP2 + j)*NP1 + i.
 *   P[5][NP3][NP2][NP1]   primitives rho, u_g, utilde^1..3 at cell centres
 *   B[3][NP3][NP2][NP1]   face field Bbar^d = sqrt(-g) B^d on the LOWER d-face of
 *                         each cell (index i holds the face at i-1/2 for d = 1)
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_MINK = 0, ORC_KS = 1 };
/* reconstruction (Sec. 2.1): piecewise linear with the monotonised-central limiter,
 * PPM, piecewise linear with the MINMOD limiter (the shock tubes of Sec. 7.2), or PPM
 * with the optional shock flattener (Sec. 2.1; Colella & Woodward 1984) */
enum { ORC_PLM = 0, ORC_PPM = 1, ORC_PLM_MINMOD = 2, ORC_PPM_FLAT = 3 };
enum { ORC_LLF = 0, ORC_HLLE = 1 };
/* edge EMFs: the average of the four neighbouring face fluxes of B (Sec. 2.5), or that
 * average corrected by the upwinded gradients of Gardiner & Stone (2005), which the
 * paper applies by default (Sec. 2.5, Fig. 1) */
enum { ORC_EMF_AVERAGE = 0, ORC_EMF_UPWIND = 1 };
enum { ORC_BC_OUTFLOW = 0, ORC_BC_POLAR = 1, ORC_BC_PERIODIC = 2 };
/* floors (Sec. 2.7): raise rho and u_g at fixed utilde, or inject the missing mass and
 * internal energy as a parcel moving with the drift frame of the field (Ressler et al.
 * 2017), which the paper uses, then invert the summed conserved state */
enum { ORC_FLOOR_FIXED = 0, ORC_FLOOR_DRIFT = 1 };

typedef struct {
  int32_t coords, n[3], ng, recon, riemann, bc[6], maxit, guess_mode;
  double a, gam;
  double xlo[3], xhi[3];
  double courant;
  double rho_fl_c, rho_fl_p, u_fl_c, u_fl_p, bsq_rho_max, bsq_u_max, gamma_max;
  double tol;
  int32_t emf;   /* ORC_EMF_AVERAGE or ORC_EMF_UPWIND */
  int32_t floor_frame;   /* ORC_FLOOR_FIXED or ORC_FLOOR_DRIFT */
} orc_desc;

typedef struct {
  int64_t tier[5];       /* con2prim outcome per tier (0 first guess .. 4 failed) */
  int64_t iter_hist[64]; /* Newton iterations of the accepted solve */
  int64_t floor_hits;
  int64_t cells;
} orc_stats;

typedef struct orc_ctx orc_ctx;

orc_ctx* orc_create(const orc_desc* d);
void     orc_free(orc_ctx* c);
int      orc_np(const orc_ctx* c, int dim);            /* padded extent */

/* geometry at one internal-coordinate point: gcov[16], gcon[16], gdet, alpha,
 * conn[64] = Gamma^l_{mn} at index (l*4+m)*4+n.  Returns 0. */
int orc_geom_point(const orc_desc* d, double x1, double x2,
                   double* gcov, double* gcon, double* gdet, double* alpha, double* conn);

/* point physics (geometry passed as gcov[16], gcon[16], gdet, alpha) */
void orc_prim_to_flux(const double* P, const double* Bcon, const double* gcov,
                      const double* gcon, double gdet, double alpha, double gam,
                      int dir, double* out9);
void orc_vchar(const double* P, const double* Bcon, const double* gcov,
               const double* gcon, double alpha, double gam, int dir,
               double* vmax, double* vmin);
void orc_source(const double* P, const double* Bcon, const double* gcov,
                const double* gcon, double gdet, double alpha, const double* conn,
                double gam, double* out9);
/* face states for one face from a 1D line of 6 cell values a[0..5], the face lying
 * between a[2] and a[3]. */
void orc_recon_face(int recon, const double* a6, double* left, double* right);
/* PPM face states with the cells next to the face flattened by f2 (cell a6[2]) and f3
 * (cell a6[3]); orc_flatten gives the coefficient of cell c of a line from the u_g and
 * normal-velocity lines (c - 2 .. c + 2 must lie in them) */
void orc_recon_face_flat(const double* a6, double f2, double f3, double* left, double* right);
double orc_flatten(const double* u, const double* v, int c);
/* floors of one cell's primitives P5 (in place) with the cell field Bcon3 and the floor
 * values rho_fl, u_fl, as the update applies them for floor_frame; returns the limits
 * applied */
int orc_floors(int floor_frame, double* P5, const double* Bcon3, const double* gcov,
               const double* gcon, double gdet, double alpha, double gam, double rho_fl,
               double u_fl, double bsq_rho_max, double bsq_u_max, double gamma_max, double tol,
               int maxit);

/* inversion of one cell.  U9 carries sqrt(-g); geometry as above.  guess5 is the
 * first guess, prev5 the plain guess (previous primitives).  Returns the tier. */
int orc_cons2prim(const double* U9, const double* gcov, const double* gcon, double gdet,
                  double alpha, double gam, const double* guess5, const double* prev5,
                  double tol, int maxit, double* P5, int* iters);
/* brute force: bisection of the one-variable energy equation to full precision. */
int orc_c2p_bisect(const double* U9, const double* gcov, const double* gcon, double gdet,
                   double alpha, double gam, double* P5);

/* grid operations */
void   orc_fill_bc(orc_ctx* c, double* P, double* B);
double orc_dt(orc_ctx* c, const double* P, const double* B);
/* one stage: Pout/Bout = update of (Pn,Bn) with fluxes/sources/EMFs evaluated
 * on (Ps,Bs) over dts; ghosts of Ps/Bs must be filled.  Pout/Bout ghosts untouched. */
void   orc_stage(orc_ctx* c, const double* Pn, const double* Bn, const double* Ps,
                 const double* Bs, double dts, double* Pout, double* Bout, orc_stats* st);
/* the same stage in two halves: orc_stage_flux evaluates the cell-centred field, the
 * face fluxes and the edge EMFs of (Ps,Bs) into the context; orc_stage_apply performs
 * the constrained transport and the cell update with whatever the context then holds
 * (a caller may correct fluxes and EMFs in between through the buffers below). */
void   orc_stage_flux(orc_ctx* c, const double* Ps, const double* Bs);
void   orc_stage_apply(orc_ctx* c, const double* Pn, const double* Bn, const double* Ps,
                       double dts, double* Pout, double* Bout, orc_stats* st);
/* writable views of the context's flux [3][9][NP3][NP2][NP1] and EMF [3][NP3][NP2][NP1]
 * buffers */
double* orc_flux_buffer(orc_ctx* c);
double* orc_emf_buffer(orc_ctx* c);
/* nsteps full midpoint steps (BC fill, Courant dt, predictor, corrector).
 * dt_fixed > 0 overrides the Courant step.  Returns the last dt. */
double orc_step(orc_ctx* c, double* P, double* B, int nsteps, double dt_fixed, orc_stats* st);
/* discrete div of the face field per interior cell (field may be NULL);
 * returns max |div| */
double orc_divb(orc_ctx* c, const double* B, double* field, double* max_rel);
/* copy of the oracle's face fluxes of the last stage: [3][9][NP3][NP2][NP1] */
const double* orc_last_flux(const orc_ctx* c);
/* edge EMFs of the last stage: [3][NP3][NP2][NP1] (E1 at (i, j-1/2, k-1/2), ...) */
const double* orc_last_emf(const orc_ctx* c);
/* Re-invert one interior cell after a correction of its conserved state (the flux
 * correction of local time stepping, Sec. 3.5): U = U(P, B_old) + dU for mass, energy,
 * momenta and entropy, field components from the corrected faces B_new; inversion from
 * the cell's P as guess, then floors.  Writes P of the cell; returns the tier. */
int orc_reinvert(orc_ctx* c, double* P, const double* Bold, const double* Bnew, int K, int J,
                 int I, const double* dU, orc_stats* st);

#ifdef __cplusplus
}
#endif
#endif
