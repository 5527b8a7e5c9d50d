/*
 * orc.c -- plain single-threaded FP64 CPU oracle for the GRMHD block update.
 *
 * TEST INFRASTRUCTURE ONLY (see orc.h).  Written for readability, not speed:
 * every quantity is computed the obvious way, in the paper's order and notation.
 * Built with -O2 -ffp-contract=off.  Shares no code with the HIP path.
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { RHO = 0, UU = 1, U1 = 2, U2 = 3, U3 = 4 };

struct orc_ctx {
  orc_desc d;
  int np[3];
  double dx[3];
  size_t ncell, ncol;
  /* per (J,I) column; kind 0 = cell centre, 1 = x1 face, 2 = x2 face.
   * x3 faces share the centre geometry (the metric does not depend on x3). */
  double* gcov[3];
  double* gcon[3];
  double* gdet[3];
  double* alpha[3];
  double* conn;           /* centre only, 64 per column */
  double* rho_fl;         /* centre only */
  double* u_fl;
  double* flux;           /* [3][9][ncell] */
  double* emf;            /* [3][ncell] */
  double* eref;           /* [4][ncell] cell-centred EMFs of the stage state and its
                             conserved density sqrt(-g) rho u^t (upwinding) */
  double* bcell;          /* [3][ncell] cell-centred B^i of the stage state */
  double *P1, *B1, *P2, *B2;
};

/* ------------------------------------------------------------------------- */
/* Geometry (Sec. 2.2)                                                        */
/* ------------------------------------------------------------------------- */

/* forward-mode dual numbers: exact first derivatives of the analytic metric.
 * The paper differentiates the internal-coordinate metric by finite differences;
 * this is the limit those differences approximate. */
typedef struct { double v, d; } dual;
static dual dd(double v, double d) { dual r = {v, d}; return r; }
static dual dadd(dual a, dual b) { return dd(a.v + b.v, a.d + b.d); }
static dual dmul(dual a, dual b) { return dd(a.v * b.v, a.d * b.v + a.v * b.d); }
static dual ddiv(dual a, dual b) { return dd(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)); }
static dual dscl(double s, dual a) { return dd(s * a.v, s * a.d); }
static dual dcst(double c) { return dd(c, 0.0); }
static dual dsin(dual a) { return dd(sin(a.v), cos(a.v) * a.d); }
static dual dcos(dual a) { return dd(cos(a.v), -sin(a.v) * a.d); }
static dual dexp(dual a) { double e = exp(a.v); return dd(e, e * a.d); }

/* Kerr metric in Kerr-Schild coordinates (t, r, theta, phi), M = 1, transformed to
 * the internal coordinates x1 = ln r, x2 = theta, x3 = phi with dr/dx1 = r. */
static void ks_gcov_dual(double a, dual x1, dual x2, dual g[4][4]) {
  dual r = dexp(x1);
  dual s = dsin(x2), c = dcos(x2);
  dual s2 = dmul(s, s), c2 = dmul(c, c);
  dual sig = dadd(dmul(r, r), dscl(a * a, c2));
  dual q = ddiv(dscl(2.0, r), sig);                  /* 2r/Sigma */
  dual one_q = dadd(dcst(1.0), q);
  dual ks[4][4];
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++) ks[m][n] = dcst(0.0);
  ks[0][0] = dadd(dcst(-1.0), q);                    /* -(1 - 2r/Sigma) */
  ks[0][1] = q;                                      /* 2r/Sigma */
  ks[0][3] = dscl(-a, dmul(q, s2));                  /* -2 a r sin^2/Sigma */
  ks[1][1] = one_q;                                  /* 1 + 2r/Sigma */
  ks[1][3] = dscl(-a, dmul(s2, one_q));              /* -a sin^2 (1 + 2r/Sigma) */
  ks[2][2] = sig;
  ks[3][3] = dmul(s2, dadd(sig, dscl(a * a, dmul(s2, one_q))));
  ks[1][0] = ks[0][1];
  ks[3][0] = ks[0][3];
  ks[3][1] = ks[1][3];
  dual jac[4] = {dcst(1.0), r, dcst(1.0), dcst(1.0)};
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++) g[m][n] = dmul(dmul(ks[m][n], jac[m]), jac[n]);
}

/* Gauss-Jordan inverse with partial pivoting; returns the determinant. */
static double inv4(const double a_in[16], double out[16]) {
  double a[4][8];
  for (int i = 0; i < 4; i++)
    for (int j = 0; j < 4; j++) {
      a[i][j] = a_in[i * 4 + j];
      a[i][j + 4] = (i == j) ? 1.0 : 0.0;
    }
  double det = 1.0;
  for (int col = 0; col < 4; col++) {
    int piv = col;
    for (int r = col + 1; r < 4; r++)
      if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
    if (piv != col) {
      for (int j = 0; j < 8; j++) { double t = a[col][j]; a[col][j] = a[piv][j]; a[piv][j] = t; }
      det = -det;
    }
    double p = a[col][col];
    det *= p;
    if (p == 0.0) return 0.0;
    for (int j = 0; j < 8; j++) a[col][j] /= p;
    for (int r = 0; r < 4; r++) {
      if (r == col) continue;
      double f = a[r][col];
      for (int j = 0; j < 8; j++) a[r][j] -= f * a[col][j];
    }
  }
  for (int i = 0; i < 4; i++)
    for (int j = 0; j < 4; j++) out[i * 4 + j] = a[i][j + 4];
  return det;
}

int orc_geom_point(const orc_desc* d, double x1, double x2, double* gcov, double* gcon,
                   double* gdet, double* alpha, double* conn) {
  if (d->coords == ORC_MINK) {
    for (int i = 0; i < 16; i++) gcov[i] = gcon[i] = 0.0;
    gcov[0] = gcon[0] = -1.0;
    for (int i = 1; i < 4; i++) gcov[i * 5] = gcon[i * 5] = 1.0;
    *gdet = 1.0;
    *alpha = 1.0;
    if (conn) for (int i = 0; i < 64; i++) conn[i] = 0.0;
    return 0;
  }
  dual g[4][4], g1[4][4], g2[4][4];
  ks_gcov_dual(d->a, dd(x1, 0.0), dd(x2, 0.0), g);
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++) gcov[m * 4 + n] = g[m][n].v;
  double det = inv4(gcov, gcon);
  *gdet = sqrt(fabs(det));
  *alpha = 1.0 / sqrt(-gcon[0]);
  if (conn) {
    /* dg[m][a][b] = d g_ab / d x^m; only x1 and x2 derivatives are non-zero */
    double dg[4][4][4];
    memset(dg, 0, sizeof(dg));
    ks_gcov_dual(d->a, dd(x1, 1.0), dd(x2, 0.0), g1);
    ks_gcov_dual(d->a, dd(x1, 0.0), dd(x2, 1.0), g2);
    for (int a = 0; a < 4; a++)
      for (int b = 0; b < 4; b++) {
        dg[1][a][b] = g1[a][b].d;
        dg[2][a][b] = g2[a][b].d;
      }
    /* Gamma^l_{mn} = 1/2 g^{lk} (d_m g_kn + d_n g_km - d_k g_mn) */
    for (int l = 0; l < 4; l++)
      for (int m = 0; m < 4; m++)
        for (int n = 0; n < 4; n++) {
          double s = 0.0;
          for (int k = 0; k < 4; k++)
            s += gcon[l * 4 + k] * (dg[m][k][n] + dg[n][k][m] - dg[k][m][n]);
          conn[(l * 4 + m) * 4 + n] = 0.5 * s;
        }
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Point physics (Sec. 2.3, 2.4, 2.5)                                         */
/* ------------------------------------------------------------------------- */

typedef struct { double ucon[4], ucov[4], bcon[4], bcov[4], bsq; } ostate;

static void lower(const double* gcov, const double* v, double* out) {
  for (int m = 0; m < 4; m++) {
    double s = 0.0;
    for (int n = 0; n < 4; n++) s += gcov[m * 4 + n] * v[n];
    out[m] = s;
  }
}

/* u^mu from utilde^i: Gamma = sqrt(1 + g_ij ut^i ut^j), u^t = Gamma/alpha,
 * u^i = ut^i - Gamma beta^i/alpha with beta^i = alpha^2 g^{ti};
 * b^t = B^i u_i, b^i = (B^i + b^t u^i)/u^t. */
static void get_state(const double* P, const double* B, const double* gcov,
                      const double* gcon, double alpha, ostate* s) {
  double qsq = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) qsq += gcov[(i + 1) * 4 + j + 1] * P[U1 + i] * P[U1 + j];
  double gamma = sqrt(1.0 + qsq);
  s->ucon[0] = gamma / alpha;
  for (int i = 0; i < 3; i++) {
    double beta = alpha * alpha * gcon[i + 1];
    s->ucon[i + 1] = P[U1 + i] - gamma * beta / alpha;
  }
  lower(gcov, s->ucon, s->ucov);
  double bt = 0.0;
  for (int i = 0; i < 3; i++) bt += B[i] * s->ucov[i + 1];
  s->bcon[0] = bt;
  for (int i = 0; i < 3; i++) s->bcon[i + 1] = (B[i] + bt * s->ucon[i + 1]) / s->ucon[0];
  lower(gcov, s->bcon, s->bcov);
  double bsq = 0.0;
  for (int m = 0; m < 4; m++) bsq += s->bcon[m] * s->bcov[m];
  s->bsq = bsq;
}

/* T^m_n = (rho + u + p + b^2) u^m u_n + delta^m_n (p + b^2/2) - b^m b_n */
static double tmunu(const ostate* s, double rho, double u, double p, int m, int n) {
  double w = rho + u + p;
  return (w + s->bsq) * s->ucon[m] * s->ucov[n] + (m == n ? p + 0.5 * s->bsq : 0.0)
         - s->bcon[m] * s->bcov[n];
}

/* dir = 0: conserved vector U; dir = 1..3: flux F^dir.  Both carry sqrt(-g).
 * components: rho u^d, T^d_t + rho u^d, T^d_i, b^i u^d - b^d u^i, kappa rho u^d */
void orc_prim_to_flux(const double* P, const double* Bcon, const double* gcov,
                      const double* gcon, double gdet, double alpha, double gam,
                      int dir, double* out) {
  ostate s;
  get_state(P, Bcon, gcov, gcon, alpha, &s);
  double rho = P[RHO], u = P[UU], p = (gam - 1.0) * u;
  double mass = rho * s.ucon[dir];
  out[0] = mass;
  out[1] = tmunu(&s, rho, u, p, dir, 0) + mass;
  for (int i = 0; i < 3; i++) out[2 + i] = tmunu(&s, rho, u, p, dir, i + 1);
  for (int i = 0; i < 3; i++)
    out[5 + i] = s.bcon[i + 1] * s.ucon[dir] - s.bcon[dir] * s.ucon[i + 1];
  double kappa = p / pow(rho, gam);
  out[8] = kappa * mass;
  for (int c = 0; c < 9; c++) out[c] *= gdet;
}

/* fast-speed estimate: roots of A v^2 - B v + C = 0 from the fluid-frame relation
 * (k.u)^2 = cms^2 (k.k + (k.u)^2), k = (-v, e_dir) */
void orc_vchar(const double* P, const double* Bcon, const double* gcov, const double* gcon,
               double alpha, double gam, int dir, double* vmax, double* vmin) {
  ostate s;
  get_state(P, Bcon, gcov, gcon, alpha, &s);
  double rho = P[RHO], u = P[UU], p = (gam - 1.0) * u;
  double w = rho + u + p;
  double cs2 = gam * p / w;
  double va2 = s.bsq / (s.bsq + w);
  double cms2 = va2 + cs2 * (1.0 - va2);
  double ut = s.ucon[0], ud = s.ucon[dir];
  double A = ut * ut * (1.0 - cms2) - cms2 * gcon[0];
  double B = 2.0 * (ut * ud * (1.0 - cms2) - cms2 * gcon[dir]);
  double C = ud * ud * (1.0 - cms2) - cms2 * gcon[dir * 4 + dir];
  double disc = B * B - 4.0 * A * C;
  if (disc < 0.0) disc = 0.0;
  double sq = sqrt(disc);
  double vp = (B + sq) / (2.0 * A), vm = (B - sq) / (2.0 * A);
  *vmax = vp > vm ? vp : vm;
  *vmin = vp > vm ? vm : vp;
}

/* geometric source Qbar_nu = sqrt(-g) T^k_l Gamma^l_{nu k} (Sec. 2.5) for the energy
 * and momentum equations; mass, induction and entropy have none. */
void orc_source(const double* P, const double* Bcon, const double* gcov, const double* gcon,
                double gdet, double alpha, const double* conn, double gam, double* out) {
  ostate s;
  get_state(P, Bcon, gcov, gcon, alpha, &s);
  double rho = P[RHO], u = P[UU], p = (gam - 1.0) * u;
  double T[4][4];
  for (int k = 0; k < 4; k++)
    for (int l = 0; l < 4; l++) T[k][l] = tmunu(&s, rho, u, p, k, l);
  for (int c = 0; c < 9; c++) out[c] = 0.0;
  for (int nu = 0; nu < 4; nu++) {
    double q = 0.0;
    for (int k = 0; k < 4; k++)
      for (int l = 0; l < 4; l++) q += T[k][l] * conn[(l * 4 + nu) * 4 + k];
    out[1 + nu] = gdet * q;
  }
}

/* ------------------------------------------------------------------------- */
/* Reconstruction (Sec. 2.1)                                                  */
/* ------------------------------------------------------------------------- */

/* monotonised-central limited slope; zero at extrema */
static double mc_slope(double dm, double dp) {
  if (dm * dp <= 0.0) return 0.0;
  double a = 2.0 * fabs(dm), b = 2.0 * fabs(dp), c = 0.5 * fabs(dm + dp);
  double m = a < b ? a : b;
  m = m < c ? m : c;
  return dm > 0.0 ? m : -m;
}

/* MINMOD limited slope: the smaller of the two one-sided differences, zero at extrema */
static double minmod_slope(double dm, double dp) {
  if (dm * dp <= 0.0) return 0.0;
  return fabs(dm) < fabs(dp) ? dm : dp;
}

/* PPM (Colella & Woodward 1984) limited parabola of cell with values am, a0, ap
 * and unlimited face values fl, fr; writes the monotonised face values. */
static void ppm_cell(double a0, double fl, double fr, double* ol, double* or_) {
  double l = fl, r = fr;
  if ((r - a0) * (a0 - l) <= 0.0) {
    l = a0;
    r = a0;
  } else {
    double dlr = r - l;
    double m6 = 6.0 * (a0 - 0.5 * (l + r));
    if (dlr * m6 > dlr * dlr) l = 3.0 * a0 - 2.0 * r;
    else if (-dlr * dlr > dlr * m6) r = 3.0 * a0 - 2.0 * l;
  }
  *ol = l;
  *or_ = r;
}

/* face value between cells c and c+1 from a[c-1..c+2] */
static double ppm_face(const double* a, int c) {
  double dc = mc_slope(a[c] - a[c - 1], a[c + 1] - a[c]);
  double dc1 = mc_slope(a[c + 1] - a[c], a[c + 2] - a[c + 1]);
  return 0.5 * (a[c] + a[c + 1]) - (dc1 - dc) / 6.0;
}

/* Shock flattening (Colella & Woodward 1984): a cell whose pressure jump over its two
 * neighbours is strong (relative jump above FLAT_EPS) where the flow compresses (the
 * normal velocity falls across it) gets the coefficient clip(FLAT_W2 (dp1/dp2 - FLAT_W1),
 * 0, 1), dp1 the jump over the neighbours and dp2 over the next ones (a steep jump:
 * dp1 close to dp2); 0 elsewhere and where dp2 vanishes.  The pressure of an ideal gas
 * is proportional to u_g, and the criteria are ratios, so the u_g line serves. */
#define FLAT_EPS 0.33
#define FLAT_W1 0.75
#define FLAT_W2 10.0
double orc_flatten(const double* u, const double* v, int c) {
  double dp1 = u[c + 1] - u[c - 1], dp2 = u[c + 2] - u[c - 2];
  double pmin = u[c + 1] < u[c - 1] ? u[c + 1] : u[c - 1];
  if (!(fabs(dp1) > FLAT_EPS * pmin) || !(v[c - 1] - v[c + 1] > 0.0) || dp2 == 0.0) return 0.0;
  double f = FLAT_W2 * (dp1 / dp2 - FLAT_W1);
  return f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
}

/* PPM with flattening: each cell's two interface values are pulled toward its mean by
 * its coefficient, a = f a0 + (1 - f) a, before the monotonisation */
void orc_recon_face_flat(const double* a, double f2, double f3, double* left, double* right) {
  double f15 = ppm_face(a, 1), f25 = ppm_face(a, 2), f35 = ppm_face(a, 3);
  double l2, r2, l3, r3;
  ppm_cell(a[2], f2 * a[2] + (1.0 - f2) * f15, f2 * a[2] + (1.0 - f2) * f25, &l2, &r2);
  ppm_cell(a[3], f3 * a[3] + (1.0 - f3) * f25, f3 * a[3] + (1.0 - f3) * f35, &l3, &r3);
  *left = r2;
  *right = l3;
}

void orc_recon_face(int recon, const double* a, double* left, double* right) {
  if (recon == ORC_PLM) {
    *left = a[2] + 0.5 * mc_slope(a[2] - a[1], a[3] - a[2]);
    *right = a[3] - 0.5 * mc_slope(a[3] - a[2], a[4] - a[3]);
    return;
  }
  if (recon == ORC_PLM_MINMOD) {
    *left = a[2] + 0.5 * minmod_slope(a[2] - a[1], a[3] - a[2]);
    *right = a[3] - 0.5 * minmod_slope(a[3] - a[2], a[4] - a[3]);
    return;
  }
  double f15 = ppm_face(a, 1), f25 = ppm_face(a, 2), f35 = ppm_face(a, 3);
  double l2, r2, l3, r3;
  ppm_cell(a[2], f15, f25, &l2, &r2);
  ppm_cell(a[3], f25, f35, &l3, &r3);
  *left = r2;
  *right = l3;
}

/* ------------------------------------------------------------------------- */
/* Con2prim (Sec. 2.6): 2D Newton in (W, v^2), 1D energy fallback, entropy     */
/* ------------------------------------------------------------------------- */

typedef struct {
  double D, Qdotn, Qtsq, Bsq, QdotB, QdotBsq, kappa, gam;
  double Qcov[3], Bc[3], gamcon[3][3];
} c2p_in;

static void c2p_setup(const double* U, const double* gcov, const double* gcon, double gdet,
                      double alpha, double gam, c2p_in* s) {
  double ig = 1.0 / gdet;
  s->gam = gam;
  s->D = alpha * U[0] * ig;
  double Qt = alpha * U[1] * ig - s->D;
  double beta[3];
  for (int i = 0; i < 3; i++) {
    s->Qcov[i] = alpha * U[2 + i] * ig;
    s->Bc[i] = alpha * U[5 + i] * ig;
    beta[i] = alpha * alpha * gcon[i + 1];
  }
  double bq = 0.0;
  for (int i = 0; i < 3; i++) bq += beta[i] * s->Qcov[i];
  s->Qdotn = (Qt - bq) / alpha;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      s->gamcon[i][j] = gcon[(i + 1) * 4 + j + 1] + beta[i] * beta[j] / (alpha * alpha);
  double qt = 0.0, bsq = 0.0, qb = 0.0;
  for (int i = 0; i < 3; i++) {
    for (int j = 0; j < 3; j++) {
      qt += s->gamcon[i][j] * s->Qcov[i] * s->Qcov[j];
      bsq += gcov[(i + 1) * 4 + j + 1] * s->Bc[i] * s->Bc[j];
    }
    qb += s->Qcov[i] * s->Bc[i];
  }
  s->Qtsq = qt;
  s->Bsq = bsq;
  s->QdotB = qb;
  s->QdotBsq = qb * qb;
  s->kappa = U[8] / U[0];
}

static double c2p_pres(const c2p_in* s, double W, double vsq) {
  return (s->gam - 1.0) / s->gam * (W * (1.0 - vsq) - s->D * sqrt(1.0 - vsq));
}

static void c2p_residual(const c2p_in* s, double W, double vsq, double* R1, double* R2) {
  double BW = s->Bsq + W;
  *R1 = vsq * BW * BW - s->QdotBsq * (s->Bsq + 2.0 * W) / (W * W) - s->Qtsq;
  *R2 = -0.5 * s->Bsq * (1.0 + vsq) + s->QdotBsq / (2.0 * W * W) - W + c2p_pres(s, W, vsq)
        - s->Qdotn;
}

static int c2p_recover(const c2p_in* s, double W, double vsq, double* P) {
  if (!(W > 0.0) || !(vsq >= 0.0) || !(vsq < 1.0)) return 1;
  double gamma = 1.0 / sqrt(1.0 - vsq);
  double rho = s->D / gamma;
  double w = W * (1.0 - vsq);
  double u = (w - rho) / s->gam;
  if (!(rho > 0.0) || !(u > 0.0)) return 1;
  P[RHO] = rho;
  P[UU] = u;
  double f = gamma / (W + s->Bsq);
  for (int i = 0; i < 3; i++) {
    double qc = 0.0;
    for (int j = 0; j < 3; j++) qc += s->gamcon[i][j] * s->Qcov[j];
    P[U1 + i] = f * (qc + s->QdotB * s->Bc[i] / W);
  }
  return 0;
}

/* Newton on (W, v^2) from a primitive guess.  Converged when the relative change in
 * W and the change in v^2 are below tol; one further iteration polishes the root. */
static int c2p_newton(const c2p_in* s, const double* gcov, const double* guess, double tol,
                      int maxit, double* P, int* iters) {
  double qsq = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) qsq += gcov[(i + 1) * 4 + j + 1] * guess[U1 + i] * guess[U1 + j];
  double gsq = 1.0 + qsq;
  double W = (guess[RHO] + s->gam * guess[UU]) * gsq;
  double vsq = qsq / gsq;
  if (!(W > 0.0)) return 1;
  double gm = (s->gam - 1.0) / s->gam;
  int converged = 0, it;
  for (it = 1; it <= maxit; it++) {
    double R1, R2;
    c2p_residual(s, W, vsq, &R1, &R2);
    double BW = s->Bsq + W;
    double sq = sqrt(1.0 - vsq);
    double J11 = 2.0 * vsq * BW + 2.0 * s->QdotBsq * BW / (W * W * W);
    double J12 = BW * BW;
    double J21 = -s->QdotBsq / (W * W * W) - 1.0 + gm * (1.0 - vsq);
    double J22 = -0.5 * s->Bsq + gm * (-W + s->D / (2.0 * sq));
    double det = J11 * J22 - J12 * J21;
    double dW = -(R1 * J22 - J12 * R2) / det;
    double dv = -(J11 * R2 - J21 * R1) / det;
    double Wn = W + dW, vn = vsq + dv;
    if (!(Wn > 0.0)) Wn = 0.5 * W;
    if (vn < 0.0) vn = 0.0;
    if (!(vn < 1.0)) vn = vsq + 0.5 * (1.0 - vsq);
    double chW = fabs(Wn - W), chv = fabs(vn - vsq);
    W = Wn;
    vsq = vn;
    if (converged) break;                    /* this was the polish iteration */
    if (chW <= tol * W && chv <= tol) converged = 1;
  }
  *iters = it > maxit ? maxit : it;
  if (!converged) return 1;
  return c2p_recover(s, W, vsq, P);
}

static double c2p_vsq_of_W(const c2p_in* s, double W) {
  double BW = s->Bsq + W;
  return (s->Qtsq + s->QdotBsq * (s->Bsq + 2.0 * W) / (W * W)) / (BW * BW);
}

/* one-variable energy equation f(W) = R2(W, v^2(W)) with v^2 eliminated through R1;
 * root by bisection after bracketing (deterministic, no tolerance parameter). */
static int c2p_energy_1d(const c2p_in* s, double* P) {
  double Wb = fabs(s->Qdotn) + s->D + s->Bsq;
  if (!(Wb > 0.0)) return 1;
  int k;
  for (k = 0; k < 200 && !(c2p_vsq_of_W(s, Wb) < 1.0); k++) Wb *= 2.0;
  if (k == 200) return 1;
  /* smallest W with v^2(W) < 1 */
  double lo = 0.0, hi = Wb;
  for (k = 0; k < 200; k++) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (c2p_vsq_of_W(s, mid) < 1.0) hi = mid; else lo = mid;
  }
  double Wlo = hi;
  double R1, R2;
  c2p_residual(s, Wlo, c2p_vsq_of_W(s, Wlo), &R1, &R2);
  if (!(R2 > 0.0)) return 1;
  double Whi = 2.0 * Wlo;
  for (k = 0; k < 200; k++) {
    c2p_residual(s, Whi, c2p_vsq_of_W(s, Whi), &R1, &R2);
    if (R2 < 0.0) break;
    Whi *= 2.0;
  }
  if (k == 200) return 1;
  lo = Wlo;
  hi = Whi;
  for (k = 0; k < 300; k++) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    c2p_residual(s, mid, c2p_vsq_of_W(s, mid), &R1, &R2);
    if (R2 > 0.0) lo = mid; else hi = mid;
  }
  double W = 0.5 * (lo + hi);
  return c2p_recover(s, W, c2p_vsq_of_W(s, W), P);
}

/* entropy backup (Sec. 2.6): p = kappa rho^gamma replaces the energy equation;
 * the momentum equation R1 is solved for v^2 by bisection. */
static double entropy_W(const c2p_in* s, double vsq) {
  double rho = s->D * sqrt(1.0 - vsq);
  double p = s->kappa * pow(rho, s->gam);
  double w = rho + s->gam / (s->gam - 1.0) * p;
  return w / (1.0 - vsq);
}

static int c2p_entropy(const c2p_in* s, double* P) {
  if (!(s->kappa > 0.0) || !(s->D > 0.0)) return 1;
  double lo = 0.0, hi = 1.0 - 0x1p-53;
  for (int k = 0; k < 300; k++) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    double W = entropy_W(s, mid);
    double BW = s->Bsq + W;
    double R1 = mid * BW * BW - s->QdotBsq * (s->Bsq + 2.0 * W) / (W * W) - s->Qtsq;
    if (R1 < 0.0) lo = mid; else hi = mid;
  }
  double vsq = 0.5 * (lo + hi);
  double W = entropy_W(s, vsq);
  if (!(W > 0.0)) return 1;
  double gamma = 1.0 / sqrt(1.0 - vsq);
  double rho = s->D / gamma;
  double p = s->kappa * pow(rho, s->gam);
  P[RHO] = rho;
  P[UU] = p / (s->gam - 1.0);
  if (!(rho > 0.0) || !(P[UU] > 0.0)) return 1;
  double f = gamma / (W + s->Bsq);
  for (int i = 0; i < 3; i++) {
    double qc = 0.0;
    for (int j = 0; j < 3; j++) qc += s->gamcon[i][j] * s->Qcov[j];
    P[U1 + i] = f * (qc + s->QdotB * s->Bc[i] / W);
  }
  return 0;
}

/* How far a start (the (W, v^2) of primitives G) is from solving the two equations:
 * |R1| / (B^2 + W)^2 + |R2| / W, each residual divided by the scale of its equation
 * (infinite outside W > 0, 0 <= v^2 < 1).  Of two distinct starts, Newton goes first from
 * the one with the smaller value. */
static double c2p_start_misfit(const c2p_in* s, const double* gcov, const double* G) {
  double qsq = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) qsq += gcov[(i + 1) * 4 + j + 1] * G[U1 + i] * G[U1 + j];
  double gsq = 1.0 + qsq;
  double W = (G[RHO] + s->gam * G[UU]) * gsq;
  double vsq = qsq / gsq;
  if (!(W > 0.0) || !(vsq >= 0.0) || !(vsq < 1.0)) return INFINITY;
  double R1, R2;
  c2p_residual(s, W, vsq, &R1, &R2);
  double BW = s->Bsq + W;
  return fabs(R1) / (BW * BW) + fabs(R2) / W;
}

int orc_cons2prim(const double* U, const double* gcov, const double* gcon, double gdet,
                  double alpha, double gam, const double* guess, const double* prev,
                  double tol, int maxit, double* P, int* iters) {
  c2p_in s;
  c2p_setup(U, gcov, gcon, gdet, alpha, gam, &s);
  double Pt[5];
  int it = 0;
  const int two = guess != prev && memcmp(guess, prev, 5 * sizeof(double)) != 0;
  const double* first = guess;
  const double* second = prev;
  if (two && c2p_start_misfit(&s, gcov, prev) < c2p_start_misfit(&s, gcov, guess)) {
    first = prev;
    second = guess;
  }
  if (c2p_newton(&s, gcov, first, tol, maxit, Pt, &it) == 0) {
    memcpy(P, Pt, sizeof(Pt));
    *iters = it;
    return 0;
  }
  if (two) {
    if (c2p_newton(&s, gcov, second, tol, maxit, Pt, &it) == 0) {
      memcpy(P, Pt, sizeof(Pt));
      *iters = it;
      return 1;
    }
  }
  *iters = 63;
  if (c2p_energy_1d(&s, Pt) == 0) {
    memcpy(P, Pt, sizeof(Pt));
    return 2;
  }
  if (c2p_entropy(&s, Pt) == 0) {
    memcpy(P, Pt, sizeof(Pt));
    return 3;
  }
  memcpy(P, prev, 5 * sizeof(double));
  return 4;
}

int orc_c2p_bisect(const double* U, const double* gcov, const double* gcon, double gdet,
                   double alpha, double gam, double* P) {
  c2p_in s;
  c2p_setup(U, gcov, gcon, gdet, alpha, gam, &s);
  return c2p_energy_1d(&s, P);
}

/* ------------------------------------------------------------------------- */
/* Grid context                                                               */
/* ------------------------------------------------------------------------- */

#define IDX(c, K, J, I) (((size_t)(K) * (c)->np[1] + (J)) * (c)->np[0] + (I))
#define COL(c, J, I) ((size_t)(J) * (c)->np[0] + (I))

static int is_pole_face(const orc_ctx* c, int J) {
  int g = c->d.ng;
  if (J == g && c->d.bc[2] == ORC_BC_POLAR) return 1;
  if (J == g + c->d.n[1] && c->d.bc[3] == ORC_BC_POLAR) return 1;
  return 0;
}

/* internal x2 of a column, mirrored across a polar boundary: ghost rows take the
 * geometry of the physical row they copy */
static double mirror_x2(const orc_ctx* c, double x2) {
  if (c->d.bc[2] == ORC_BC_POLAR && x2 < c->d.xlo[1]) x2 = 2.0 * c->d.xlo[1] - x2;
  if (c->d.bc[3] == ORC_BC_POLAR && x2 > c->d.xhi[1]) x2 = 2.0 * c->d.xhi[1] - x2;
  return x2;
}

orc_ctx* orc_create(const orc_desc* d) {
  orc_ctx* c = (orc_ctx*)calloc(1, sizeof(orc_ctx));
  c->d = *d;
  for (int k = 0; k < 3; k++) {
    c->np[k] = d->n[k] + 2 * d->ng + 1;
    c->dx[k] = (d->xhi[k] - d->xlo[k]) / d->n[k];
  }
  c->ncell = (size_t)c->np[0] * c->np[1] * c->np[2];
  c->ncol = (size_t)c->np[0] * c->np[1];
  for (int kind = 0; kind < 3; kind++) {
    c->gcov[kind] = (double*)calloc(c->ncol * 16, sizeof(double));
    c->gcon[kind] = (double*)calloc(c->ncol * 16, sizeof(double));
    c->gdet[kind] = (double*)calloc(c->ncol, sizeof(double));
    c->alpha[kind] = (double*)calloc(c->ncol, sizeof(double));
  }
  c->conn = (double*)calloc(c->ncol * 64, sizeof(double));
  c->rho_fl = (double*)calloc(c->ncol, sizeof(double));
  c->u_fl = (double*)calloc(c->ncol, sizeof(double));
  int g = d->ng;
  for (int J = 0; J < c->np[1]; J++)
    for (int I = 0; I < c->np[0]; I++) {
      size_t col = COL(c, J, I);
      for (int kind = 0; kind < 3; kind++) {
        double x1 = d->xlo[0] + (I - g + (kind == 1 ? 0.0 : 0.5)) * c->dx[0];
        double x2 = d->xlo[1] + (J - g + (kind == 2 ? 0.0 : 0.5)) * c->dx[1];
        if (kind == 2 && is_pole_face(c, J)) {
          /* the polar axis: sqrt(-g) = 0, no flux crosses it */
          c->gdet[kind][col] = 0.0;
          c->alpha[kind][col] = 1.0;
          continue;
        }
        x2 = mirror_x2(c, x2);
        orc_geom_point(d, x1, x2, c->gcov[kind] + col * 16, c->gcon[kind] + col * 16,
                       c->gdet[kind] + col, c->alpha[kind] + col,
                       kind == 0 ? c->conn + col * 64 : NULL);
        if (kind == 0) {
          double r = d->coords == ORC_KS ? exp(x1) : 1.0;
          c->rho_fl[col] = d->rho_fl_c * pow(r, d->rho_fl_p);
          c->u_fl[col] = d->u_fl_c * pow(r, d->u_fl_p);
        }
      }
    }
  c->flux = (double*)calloc(c->ncell * 27, sizeof(double));
  c->emf = (double*)calloc(c->ncell * 3, sizeof(double));
  c->eref = (double*)calloc(c->ncell * 4, sizeof(double));
  c->bcell = (double*)calloc(c->ncell * 3, sizeof(double));
  c->P1 = (double*)calloc(c->ncell * 5, sizeof(double));
  c->B1 = (double*)calloc(c->ncell * 3, sizeof(double));
  c->P2 = (double*)calloc(c->ncell * 5, sizeof(double));
  c->B2 = (double*)calloc(c->ncell * 3, sizeof(double));
  return c;
}

void orc_free(orc_ctx* c) {
  if (!c) return;
  for (int k = 0; k < 3; k++) {
    free(c->gcov[k]); free(c->gcon[k]); free(c->gdet[k]); free(c->alpha[k]);
  }
  free(c->conn); free(c->rho_fl); free(c->u_fl); free(c->flux); free(c->emf); free(c->eref);
  free(c->bcell); free(c->P1); free(c->B1); free(c->P2); free(c->B2);
  free(c);
}

int orc_np(const orc_ctx* c, int dim) { return c->np[dim]; }
const double* orc_last_flux(const orc_ctx* c) { return c->flux; }
const double* orc_last_emf(const orc_ctx* c) { return c->emf; }
double* orc_flux_buffer(orc_ctx* c) { return c->flux; }
double* orc_emf_buffer(orc_ctx* c) { return c->emf; }

/* ------------------------------------------------------------------------- */
/* Physical boundaries                                                        */
/* ------------------------------------------------------------------------- */

static int wrap(int I, int g, int n) {
  int m = (I - g) % n;
  if (m < 0) m += n;
  return g + m;
}

static void copy_cell(orc_ctx* c, double* P, double* B, size_t dst, size_t src,
                      int copyB1, int copyB2, int copyB3) {
  for (int v = 0; v < 5; v++) P[v * c->ncell + dst] = P[v * c->ncell + src];
  if (copyB1) B[0 * c->ncell + dst] = B[0 * c->ncell + src];
  if (copyB2) B[1 * c->ncell + dst] = B[1 * c->ncell + src];
  if (copyB3) B[2 * c->ncell + dst] = B[2 * c->ncell + src];
}

/* x1: outflow (zero gradient, no inflow) or periodic; x2: polar (transmissive
 * across the axis from phi + pi) or periodic; x3: periodic.  Filled x1, then x2
 * over all x1, then x3 over all x1, x2, so corners compose. */
void orc_fill_bc(orc_ctx* c, double* P, double* B) {
  const int g = c->d.ng, n1 = c->d.n[0], n2 = c->d.n[1], n3 = c->d.n[2];
  const int N1 = c->np[0], N2 = c->np[1], N3 = c->np[2];
  const size_t nc = c->ncell;
  /* x1 (the ranges in x2, x3 include the upper boundary-face index, so that the x2 and
   * x3 face fields of those faces are filled too; cell values there are overwritten by
   * the later passes) */
  for (int K = g; K <= g + n3; K++)
    for (int J = g; J <= g + n2; J++)
      for (int I = 0; I < N1; I++) {
        if (I >= g && I < g + n1) continue;
        size_t dst = IDX(c, K, J, I);
        int lo = I < g;
        int bc = c->d.bc[lo ? 0 : 1];
        if (bc == ORC_BC_PERIODIC) {
          size_t src = IDX(c, K, J, wrap(I, g, n1));
          copy_cell(c, P, B, dst, src, 0, 1, 1);
          if (I != g + n1) B[dst] = B[src];
        } else {
          int Is = lo ? g : g + n1 - 1;
          size_t src = IDX(c, K, J, Is);
          copy_cell(c, P, B, dst, src, 0, 1, 1);
          double* u1 = P + 2 * nc + dst;
          if (lo && *u1 > 0.0) *u1 = 0.0;
          if (!lo && *u1 < 0.0) *u1 = 0.0;
          /* normal face field: zero gradient from the boundary face */
          if (lo) B[dst] = B[IDX(c, K, J, g)];
          else if (I > g + n1) B[dst] = B[IDX(c, K, J, g + n1)];
        }
      }
  /* x2 */
  for (int K = g; K <= g + n3; K++)
    for (int J = 0; J < N2; J++) {
      if (J >= g && J < g + n2) continue;
      int lo = J < g;
      int bc = c->d.bc[lo ? 2 : 3];
      for (int I = 0; I < N1; I++) {
        size_t dst = IDX(c, K, J, I);
        if (bc == ORC_BC_POLAR) {
          int Js = lo ? 2 * g - 1 - J : 2 * (g + n2) - 1 - J;
          int Ks = wrap(K + n3 / 2, g, n3);
          size_t src = IDX(c, Ks, Js, I);
          copy_cell(c, P, B, dst, src, 1, 0, 1);
          P[3 * nc + dst] = -P[3 * nc + dst];
          /* x2 faces: face J mirrors face 2*edge - J with opposite sign */
          int edge = lo ? g : g + n2;
          if (J == edge) {
            B[nc + dst] = 0.0;
          } else {
            int Jf = 2 * edge - J;
            B[nc + dst] = -B[nc + IDX(c, Ks, Jf, I)];
          }
        } else {
          size_t src = IDX(c, K, wrap(J, g, n2), I);
          copy_cell(c, P, B, dst, src, 1, 0, 1);
          if (J != g + n2) B[nc + dst] = B[nc + src];
        }
      }
    }
  /* polar-axis faces inside the interior range carry no field */
  for (int K = 0; K < N3; K++)
    for (int I = 0; I < N1; I++) {
      if (c->d.bc[2] == ORC_BC_POLAR) B[nc + IDX(c, K, g, I)] = 0.0;
      if (c->d.bc[3] == ORC_BC_POLAR) B[nc + IDX(c, K, g + n2, I)] = 0.0;
    }
  /* x3 */
  for (int K = 0; K < N3; K++) {
    if (K >= g && K < g + n3) continue;
    for (int J = 0; J < N2; J++)
      for (int I = 0; I < N1; I++) {
        size_t dst = IDX(c, K, J, I);
        size_t src = IDX(c, wrap(K, g, n3), J, I);
        copy_cell(c, P, B, dst, src, 1, 1, 0);
        if (K != g + n3) B[2 * nc + dst] = B[2 * nc + src];
      }
  }
}

/* ------------------------------------------------------------------------- */
/* Stage (Sec. 2.5)                                                           */
/* ------------------------------------------------------------------------- */

static void geom_of(const orc_ctx* c, int kind, size_t col, const double** gcov,
                    const double** gcon, double* gdet, double* alpha) {
  *gcov = c->gcov[kind] + col * 16;
  *gcon = c->gcon[kind] + col * 16;
  *gdet = c->gdet[kind][col];
  *alpha = c->alpha[kind][col];
}

/* cell-centred B^i = average of the two face fields / sqrt(-g) at the centre */
static void cell_field(const orc_ctx* c, const double* B, double* bc) {
  const size_t nc = c->ncell;
  for (size_t q = 0; q < 3 * nc; q++) bc[q] = 0.0;
  for (int K = 0; K < c->np[2]; K++)
    for (int J = 0; J < c->np[1]; J++)
      for (int I = 0; I < c->np[0]; I++) {
        size_t id = IDX(c, K, J, I);
        double gdet = c->gdet[0][COL(c, J, I)];
        if (I + 1 < c->np[0]) bc[id] = 0.5 * (B[id] + B[IDX(c, K, J, I + 1)]) / gdet;
        if (J + 1 < c->np[1]) bc[nc + id] = 0.5 * (B[nc + id] + B[nc + IDX(c, K, J + 1, I)]) / gdet;
        if (K + 1 < c->np[2]) bc[2 * nc + id] = 0.5 * (B[2 * nc + id] + B[2 * nc + IDX(c, K + 1, J, I)]) / gdet;
      }
}

/* one face: reconstruct, evaluate U and F on both sides, Riemann flux */
static void face_flux(orc_ctx* c, const double* P, const double* bc, const double* B,
                      int d, int K, int J, int I, double* F) {
  const size_t nc = c->ncell;
  int st[3] = {0, 0, 0};
  st[d] = 1;
  size_t id = IDX(c, K, J, I);
  size_t col = COL(c, J, I);
  int kind = d == 0 ? 1 : (d == 1 ? 2 : 0);
  if (d == 1 && is_pole_face(c, J)) {
    for (int q = 0; q < 9; q++) F[q] = 0.0;
    return;
  }
  const double *gcov, *gcon;
  double gdet, alpha;
  geom_of(c, kind, col, &gcov, &gcon, &gdet, &alpha);
  int nmax = c->np[d] - 1;
  int pos = d == 0 ? I : (d == 1 ? J : K);
  double PL[5], PR[5], BL[3], BR[3];
  double line[8][6];
  for (int v = 0; v < 8; v++) {
    if (v >= 5 && v - 5 == d) continue;
    for (int s = 0; s < 6; s++) {
      int p = pos - 3 + s;
      if (p < 0) p = 0;
      if (p > nmax) p = nmax;
      size_t q = IDX(c, K + st[2] * (p - pos), J + st[1] * (p - pos), I + st[0] * (p - pos));
      line[v][s] = v < 5 ? P[v * nc + q] : bc[(v - 5) * nc + q];
    }
  }
  /* flattening of the two cells next to the face from u_g and the normal utilde */
  double f2 = 0.0, f3 = 0.0;
  if (c->d.recon == ORC_PPM_FLAT) {
    f2 = orc_flatten(line[1], line[2 + d], 2);
    f3 = orc_flatten(line[1], line[2 + d], 3);
  }
  for (int v = 0; v < 8; v++) {
    if (v >= 5 && v - 5 == d) continue;
    double l, r;
    if (c->d.recon == ORC_PPM_FLAT) orc_recon_face_flat(line[v], f2, f3, &l, &r);
    else orc_recon_face(c->d.recon, line[v], &l, &r);
    if (v < 5) { PL[v] = l; PR[v] = r; }
    else { BL[v - 5] = l; BR[v - 5] = r; }
  }
  BL[d] = BR[d] = B[d * nc + id] / gdet;
  double UL[9], UR[9], FL[9], FR[9];
  double gam = c->d.gam;
  orc_prim_to_flux(PL, BL, gcov, gcon, gdet, alpha, gam, 0, UL);
  orc_prim_to_flux(PR, BR, gcov, gcon, gdet, alpha, gam, 0, UR);
  orc_prim_to_flux(PL, BL, gcov, gcon, gdet, alpha, gam, d + 1, FL);
  orc_prim_to_flux(PR, BR, gcov, gcon, gdet, alpha, gam, d + 1, FR);
  double vmaxL, vminL, vmaxR, vminR;
  orc_vchar(PL, BL, gcov, gcon, alpha, gam, d + 1, &vmaxL, &vminL);
  orc_vchar(PR, BR, gcov, gcon, alpha, gam, d + 1, &vmaxR, &vminR);
  double cmax = fmax(0.0, fmax(vmaxL, vmaxR));
  double cmin = -fmin(0.0, fmin(vminL, vminR));
  if (c->d.riemann == ORC_LLF) {
    double cc = fmax(cmax, cmin);
    for (int q = 0; q < 9; q++) F[q] = 0.5 * (FL[q] + FR[q] - cc * (UR[q] - UL[q]));
  } else {
    if (cmax + cmin > 0.0) {
      for (int q = 0; q < 9; q++)
        F[q] = (cmin * FR[q] + cmax * FL[q] - cmax * cmin * (UR[q] - UL[q])) / (cmax + cmin);
    } else {
      for (int q = 0; q < 9; q++) F[q] = 0.5 * (FL[q] + FR[q]);
    }
  }
  F[5 + d] = 0.0;
}

/* Floors at fixed utilde (Sec. 2.7): Lorentz-factor ceiling, then rho >= max(rho_fl,
 * b^2/bsq_rho_max) and u >= max(u_fl, b^2/bsq_u_max) */
static int floors_fixed(double* P, const double* Bcon, const double* gcov, const double* gcon,
                        double alpha, double rho_fl, double u_fl, double bsq_rho_max,
                        double bsq_u_max, double gmax) {
  int hits = 0;
  double qsq = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) qsq += gcov[(i + 1) * 4 + j + 1] * P[U1 + i] * P[U1 + j];
  if (1.0 + qsq > gmax * gmax) {
    double f = sqrt((gmax * gmax - 1.0) / qsq);
    for (int i = 0; i < 3; i++) P[U1 + i] *= f;
    hits++;
  }
  ostate s;
  get_state(P, Bcon, gcov, gcon, alpha, &s);
  double rmin = fmax(rho_fl, s.bsq / bsq_rho_max);
  double umin = fmax(u_fl, s.bsq / bsq_u_max);
  if (P[RHO] < rmin) { P[RHO] = rmin; hits++; }
  if (P[UU] < umin) { P[UU] = umin; hits++; }
  return hits;
}

/* Floors in the drift frame (Sec. 2.7, Ressler et al. 2017).  After the Lorentz-factor
 * ceiling, the missing mass drho = rmin - rho and internal energy du = umin - u (where
 * positive) are added as a parcel of gas moving with the drift frame of the field,
 * u_D = g (u + beta b) with beta = -b^t / (b^2 u^t): the fluid four-velocity with its
 * motion along the field removed, so the field lines feel no drag and the gas no kick
 * along them.  (The parcel carries no field; g normalises u_D, with beta^2 b^2 capped at
 * 1 - 1/gamma_max^2.)  The summed conserved state U(P) + U(parcel) is inverted from the
 * previous primitives; the conserved entropy keeps the cell's specific value.  An
 * inversion that needs the entropy or keep-previous tier leaves the cell to the fixed-
 * utilde floors, which then apply in every case as the last guarantee of the minima. */
static int floors_drift(double* P, const double* Bcon, const double* gcov, const double* gcon,
                        double gdet, double alpha, double gam, double rho_fl, double u_fl,
                        double bsq_rho_max, double bsq_u_max, double gmax, double tol,
                        int maxit) {
  int hits = 0;
  double qsq = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) qsq += gcov[(i + 1) * 4 + j + 1] * P[U1 + i] * P[U1 + j];
  if (1.0 + qsq > gmax * gmax) {
    double f = sqrt((gmax * gmax - 1.0) / qsq);
    for (int i = 0; i < 3; i++) P[U1 + i] *= f;
    hits++;
  }
  ostate s;
  get_state(P, Bcon, gcov, gcon, alpha, &s);
  double rmin = fmax(rho_fl, s.bsq / bsq_rho_max);
  double umin = fmax(u_fl, s.bsq / bsq_u_max);
  double drho = fmax(rmin - P[RHO], 0.0), du = fmax(umin - P[UU], 0.0);
  if (drho > 0.0 || du > 0.0) {
    /* beta b does not change when the field is multiplied by a constant: it is formed
     * from the field divided by its largest component, so that a weak field (b^2 below
     * the smallest normal double) gives the same frame as a strong one of that direction;
     * without a field the drift frame is the fluid frame */
    double ud[4];
    for (int m = 0; m < 4; m++) ud[m] = s.ucon[m];
    double bmax = fmax(fmax(fabs(Bcon[0]), fabs(Bcon[1])), fabs(Bcon[2]));
    if (bmax > 0.0) {
      double Bs[3] = {Bcon[0] / bmax, Bcon[1] / bmax, Bcon[2] / bmax};
      ostate sb;
      get_state(P, Bs, gcov, gcon, alpha, &sb);
      if (sb.bsq > 0.0) {
        double bp = -sb.bcon[0] / (sb.bsq * sb.ucon[0]);
        double b2 = fmin(bp * bp * sb.bsq, 1.0 - 1.0 / (gmax * gmax));
        double g = 1.0 / sqrt(1.0 - b2);
        for (int m = 0; m < 4; m++) ud[m] = g * (s.ucon[m] + bp * sb.bcon[m]);
      }
    }
    /* the parcel's primitives: utilde^i = u^i + u^t beta^i, beta^i = alpha^2 g^{ti} */
    double Pp[5] = {drho, du, 0.0, 0.0, 0.0}, B0[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 3; i++) Pp[U1 + i] = ud[i + 1] + ud[0] * alpha * alpha * gcon[i + 1];
    double U[9], Up[9], Un[9];
    orc_prim_to_flux(P, Bcon, gcov, gcon, gdet, alpha, gam, 0, U);
    orc_prim_to_flux(Pp, B0, gcov, gcon, gdet, alpha, gam, 0, Up);
    for (int q = 0; q < 8; q++) Un[q] = U[q] + Up[q];
    Un[8] = U[8] / U[0] * Un[0];
    double Pn[5];
    int it = 0;
    int tier = orc_cons2prim(Un, gcov, gcon, gdet, alpha, gam, P, P, tol, maxit, Pn, &it);
    if (tier <= 2) {
      for (int v = 0; v < 5; v++) P[v] = Pn[v];
      /* the minima again at fixed utilde (rounding of the inversion), counted with the
       * injection */
      floors_fixed(P, Bcon, gcov, gcon, alpha, rho_fl, u_fl, bsq_rho_max, bsq_u_max, gmax);
      return hits + (drho > 0.0) + (du > 0.0);
    }
    /* an inversion that needs the entropy or keep-previous tier: fixed-utilde floors */
    return hits + floors_fixed(P, Bcon, gcov, gcon, alpha, rho_fl, u_fl, bsq_rho_max, bsq_u_max,
                               gmax);
  }
  return hits;
}

int orc_floors(int floor_frame, double* P, const double* Bcon, const double* gcov,
               const double* gcon, double gdet, double alpha, double gam, double rho_fl,
               double u_fl, double bsq_rho_max, double bsq_u_max, double gamma_max, double tol,
               int maxit) {
  if (floor_frame == ORC_FLOOR_DRIFT)
    return floors_drift(P, Bcon, gcov, gcon, gdet, alpha, gam, rho_fl, u_fl, bsq_rho_max,
                        bsq_u_max, gamma_max, tol, maxit);
  return floors_fixed(P, Bcon, gcov, gcon, alpha, rho_fl, u_fl, bsq_rho_max, bsq_u_max,
                      gamma_max);
}

static int apply_floors(const orc_ctx* c, double* P, const double* Bcon, const double* gcov,
                        const double* gcon, double gdet, double alpha, size_t col) {
  return orc_floors(c->d.floor_frame, P, Bcon, gcov, gcon, gdet, alpha, c->d.gam, c->rho_fl[col],
                    c->u_fl[col], c->d.bsq_rho_max, c->d.bsq_u_max, c->d.gamma_max, c->d.tol,
                    c->d.maxit);
}

#define FL(d, q, K, J, I) c->flux[((size_t)(d) * 9 + (q)) * nc + IDX(c, K, J, I)]

/* A mass flux counts as zero when it is at most this fraction of the largest conserved
 * density sqrt(-g) rho u^t of the cells around the edge, i.e. where the coordinate
 * velocity through the face is below it: such fluxes are rounding residuals of flows at
 * rest through the face (symmetry planes, static atmospheres), whose sign no computation
 * fixes. */
#define UPWIND_REST 1e-12

/* the value on the side the flow comes from: lo where the mass flux m is positive (flow
 * toward the upper side), hi where it is negative, their mean where it is zero within
 * rest (UPWIND_REST times the density scale) */
static double upwind(double lo, double hi, double m, double rest) {
  if (m > rest) return lo;
  if (m < -rest) return hi;
  return 0.5 * (lo + hi);
}

/* Gardiner & Stone's (2005) correction to the averaged EMF of the edge along x^(a+1) at
 * padded position x (I, J, K), with (a, p, q) cyclic.  Around the edge lie the cells
 * c[pp][qq] (pp, qq = 0 below, 1 above the edge in x^(p+1), x^(q+1)), two p-faces (normal
 * p, at qq = 0, 1) carrying the face EMF -F_p(B^q) and two q-faces (normal q, at pp) with
 * +F_q(B^p).  The gradients of the EMF between the edge and the cell centres, along p on
 * each row and along q on each column, are taken from the row (column) upstream of the
 * mass flux through the face between the two candidates; the correction is
 *   1/4 [(dp_low - dp_high) + (dq_low - dq_high)],
 * the dp at the lower/upper half of the edge in p (similarly q), which with the average
 * gives the face's Riemann EMF for flows that vary along one direction only. */
static double emf_upwind_correction(const orc_ctx* c, int a, const int x[3]) {
  const size_t nc = c->ncell;
  const int p = (a + 1) % 3, q = (a + 2) % 3;
  double Ep[2], Eq[2], Mp[2], Mq[2], Er[2][2], dmax = 0.0;
  for (int s = 0; s < 2; s++) {
    int y[3] = {x[0], x[1], x[2]};
    y[q] -= 1 - s;   /* p-face at row s */
    Ep[s] = -c->flux[((size_t)p * 9 + 5 + q) * nc + IDX(c, y[2], y[1], y[0])];
    Mp[s] = c->flux[((size_t)p * 9 + 0) * nc + IDX(c, y[2], y[1], y[0])];
    int z[3] = {x[0], x[1], x[2]};
    z[p] -= 1 - s;   /* q-face at column s */
    Eq[s] = c->flux[((size_t)q * 9 + 5 + p) * nc + IDX(c, z[2], z[1], z[0])];
    Mq[s] = c->flux[((size_t)q * 9 + 0) * nc + IDX(c, z[2], z[1], z[0])];
  }
  for (int sp = 0; sp < 2; sp++)
    for (int sq = 0; sq < 2; sq++) {
      int y[3] = {x[0], x[1], x[2]};
      y[p] -= 1 - sp;
      y[q] -= 1 - sq;
      Er[sp][sq] = c->eref[(size_t)a * nc + IDX(c, y[2], y[1], y[0])];
      dmax = fmax(dmax, fabs(c->eref[3 * nc + IDX(c, y[2], y[1], y[0])]));
    }
  const double rest = UPWIND_REST * dmax;
  /* along p: upstream in q through the q-face of each column */
  double dp_lo = upwind(Ep[0] - Er[0][0], Ep[1] - Er[0][1], Mq[0], rest);
  double dp_hi = upwind(Er[1][0] - Ep[0], Er[1][1] - Ep[1], Mq[1], rest);
  /* along q: upstream in p through the p-face of each row */
  double dq_lo = upwind(Eq[0] - Er[0][0], Eq[1] - Er[1][0], Mp[0], rest);
  double dq_hi = upwind(Er[0][1] - Eq[0], Er[1][1] - Eq[1], Mp[1], rest);
  return 0.25 * ((dp_lo - dp_hi) + (dq_lo - dq_hi));
}
#define EM(d, K, J, I) c->emf[(size_t)(d) * nc + IDX(c, K, J, I)]

/* Steps 1-2 of a stage: cell-centred field, face fluxes and edge EMFs of the stage
 * state, kept in the context until orc_stage_apply. */
void orc_stage_flux(orc_ctx* c, const double* Ps, const double* Bs) {
  const int g = c->d.ng, n1 = c->d.n[0], n2 = c->d.n[1], n3 = c->d.n[2];
  const size_t nc = c->ncell;
  double* bc = c->bcell;
  cell_field(c, Bs, bc);
  /* 1. face fluxes; transverse range extends one ghost layer for the EMFs */
  for (int d = 0; d < 3; d++) {
    int lo[3], hi[3];
    for (int e = 0; e < 3; e++) {
      lo[e] = e == d ? g : g - 1;
      hi[e] = e == d ? g + c->d.n[e] : g + c->d.n[e];
    }
    for (int K = lo[2]; K <= hi[2]; K++)
      for (int J = lo[1]; J <= hi[1]; J++)
        for (int I = lo[0]; I <= hi[0]; I++) {
          double F[9];
          face_flux(c, Ps, bc, Bs, d, K, J, I, F);
          size_t id = IDX(c, K, J, I);
          for (int q = 0; q < 9; q++) c->flux[((size_t)d * 9 + q) * nc + id] = F[q];
        }
  }
  /* for upwinding, the EMF of each cell's own state: component a (edge along x^(a+1))
   * is the flux of B^(p+1) along x^(q+1) with (a, p, q) cyclic, i.e. sqrt(-g) (b^p u^q -
   * b^q u^p), on every cell next to a block edge */
  if (c->d.emf == ORC_EMF_UPWIND) {
    for (int K = g - 1; K <= g + n3; K++)
      for (int J = g - 1; J <= g + n2; J++)
        for (int I = g - 1; I <= g + n1; I++) {
          size_t id = IDX(c, K, J, I);
          size_t col = COL(c, J, I);
          const double *gcov, *gcon;
          double gdet, alpha, Pc[5], Bc[3];
          geom_of(c, 0, col, &gcov, &gcon, &gdet, &alpha);
          for (int v = 0; v < 5; v++) Pc[v] = Ps[v * nc + id];
          for (int e = 0; e < 3; e++) Bc[e] = bc[e * nc + id];
          for (int a = 0; a < 3; a++) {
            int p = (a + 1) % 3, q = (a + 2) % 3;
            double F[9];
            orc_prim_to_flux(Pc, Bc, gcov, gcon, gdet, alpha, c->d.gam, q + 1, F);
            c->eref[(size_t)a * nc + id] = F[5 + p];
          }
          double U[9];
          orc_prim_to_flux(Pc, Bc, gcov, gcon, gdet, alpha, c->d.gam, 0, U);
          c->eref[3 * nc + id] = U[0];
        }
  }
  /* 2. edge EMFs as the average of the four neighbouring face fluxes of B */
  for (int K = g; K <= g + n3; K++)
    for (int J = g; J <= g + n2; J++)
      for (int I = g; I <= g + n1; I++) {
        int pole = is_pole_face(c, J);
        if (I < g + n1)
          EM(0, K, J, I) = pole ? 0.0
              : 0.25 * (FL(2, 6, K, J, I) + FL(2, 6, K, J - 1, I) - FL(1, 7, K - 1, J, I)
                        - FL(1, 7, K, J, I));
        if (J < g + n2)
          EM(1, K, J, I) = 0.25 * (FL(0, 7, K - 1, J, I) + FL(0, 7, K, J, I)
                                   - FL(2, 5, K, J, I) - FL(2, 5, K, J, I - 1));
        if (K < g + n3)
          EM(2, K, J, I) = pole ? 0.0
              : 0.25 * (FL(1, 5, K, J, I - 1) + FL(1, 5, K, J, I) - FL(0, 6, K, J, I)
                        - FL(0, 6, K, J - 1, I));
        if (c->d.emf == ORC_EMF_UPWIND) {
          int x[3] = {I, J, K};
          int lim[3] = {I < g + n1, J < g + n2, K < g + n3};
          for (int a = 0; a < 3; a++) {
            if (!lim[a] || (a != 1 && pole)) continue;
            EM(a, K, J, I) += emf_upwind_correction(c, a, x);
          }
        }
      }
}

/* Steps 3-4 of a stage from the fluxes and EMFs held in the context (as left by
 * orc_stage_flux, possibly corrected in between). */
void orc_stage_apply(orc_ctx* c, const double* Pn, const double* Bn, const double* Ps,
                     double dts, double* Pout, double* Bout, orc_stats* st) {
  const int g = c->d.ng, n1 = c->d.n[0], n2 = c->d.n[1], n3 = c->d.n[2];
  const size_t nc = c->ncell;
  const double *dx = c->dx;
  const double* bc = c->bcell;
  /* 3. constrained transport of the face field */
  for (int K = g; K <= g + n3; K++)
    for (int J = g; J <= g + n2; J++)
      for (int I = g; I <= g + n1; I++) {
        size_t id = IDX(c, K, J, I);
        if (J < g + n2 && K < g + n3)
          Bout[id] = Bn[id] + dts * ((EM(1, K + 1, J, I) - EM(1, K, J, I)) / dx[2]
                                     - (EM(2, K, J + 1, I) - EM(2, K, J, I)) / dx[1]);
        if (I < g + n1 && K < g + n3)
          Bout[nc + id] = is_pole_face(c, J) ? 0.0
              : Bn[nc + id] + dts * ((EM(2, K, J, I + 1) - EM(2, K, J, I)) / dx[0]
                                     - (EM(0, K + 1, J, I) - EM(0, K, J, I)) / dx[2]);
        if (I < g + n1 && J < g + n2)
          Bout[2 * nc + id] = Bn[2 * nc + id] + dts * ((EM(0, K, J + 1, I) - EM(0, K, J, I)) / dx[1]
                                                       - (EM(1, K, J, I + 1) - EM(1, K, J, I)) / dx[0]);
      }
  /* 4. cell update: U^n recomputed from P^n, flux divergence, source at the stage
   *    state, then inversion (guess: the stage state) and floors */
  for (int K = g; K < g + n3; K++)
    for (int J = g; J < g + n2; J++)
      for (int I = g; I < g + n1; I++) {
        size_t id = IDX(c, K, J, I);
        size_t col = COL(c, J, I);
        const double *gcov, *gcon;
        double gdet, alpha;
        geom_of(c, 0, col, &gcov, &gcon, &gdet, &alpha);
        double P0[5], PS[5], Bc0[3], BcS[3];
        for (int v = 0; v < 5; v++) { P0[v] = Pn[v * nc + id]; PS[v] = Ps[v * nc + id]; }
        Bc0[0] = 0.5 * (Bn[id] + Bn[IDX(c, K, J, I + 1)]) / gdet;
        Bc0[1] = 0.5 * (Bn[nc + id] + Bn[nc + IDX(c, K, J + 1, I)]) / gdet;
        Bc0[2] = 0.5 * (Bn[2 * nc + id] + Bn[2 * nc + IDX(c, K + 1, J, I)]) / gdet;
        for (int i = 0; i < 3; i++) BcS[i] = bc[i * nc + id];
        double U[9], Q[9];
        orc_prim_to_flux(P0, Bc0, gcov, gcon, gdet, alpha, c->d.gam, 0, U);
        orc_source(PS, BcS, gcov, gcon, gdet, alpha, c->conn + col * 64, c->d.gam, Q);
        static const int comps[6] = {0, 1, 2, 3, 4, 8};
        for (int cc = 0; cc < 6; cc++) {
          int q = comps[cc];
          double div = (FL(0, q, K, J, I + 1) - FL(0, q, K, J, I)) / dx[0]
                       + (FL(1, q, K, J + 1, I) - FL(1, q, K, J, I)) / dx[1]
                       + (FL(2, q, K + 1, J, I) - FL(2, q, K, J, I)) / dx[2];
          U[q] = U[q] - dts * div + dts * Q[q];
        }
        U[5] = 0.5 * (Bout[id] + Bout[IDX(c, K, J, I + 1)]);
        U[6] = 0.5 * (Bout[nc + id] + Bout[nc + IDX(c, K, J + 1, I)]);
        U[7] = 0.5 * (Bout[2 * nc + id] + Bout[2 * nc + IDX(c, K + 1, J, I)]);
        double Pnew[5], Bnew[3];
        int it = 0;
        int tier = orc_cons2prim(U, gcov, gcon, gdet, alpha, c->d.gam, PS, PS, c->d.tol,
                                 c->d.maxit, Pnew, &it);
        for (int i = 0; i < 3; i++) Bnew[i] = U[5 + i] / gdet;
        int hits = apply_floors(c, Pnew, Bnew, gcov, gcon, gdet, alpha, col);
        for (int v = 0; v < 5; v++) Pout[v * nc + id] = Pnew[v];
        if (st) {
          st->tier[tier]++;
          st->iter_hist[it < 63 ? it : 63]++;
          st->floor_hits += hits;
          st->cells++;
        }
      }
}
#undef FL
#undef EM

void orc_stage(orc_ctx* c, const double* Pn, const double* Bn, const double* Ps,
               const double* Bs, double dts, double* Pout, double* Bout, orc_stats* st) {
  orc_stage_flux(c, Ps, Bs);
  orc_stage_apply(c, Pn, Bn, Ps, dts, Pout, Bout, st);
}

double orc_dt(orc_ctx* c, const double* P, const double* B) {
  const int g = c->d.ng, n1 = c->d.n[0], n2 = c->d.n[1], n3 = c->d.n[2];
  const size_t nc = c->ncell;
  double best = 1e300;
  for (int K = g; K < g + n3; K++)
    for (int J = g; J < g + n2; J++)
      for (int I = g; I < g + n1; I++) {
        size_t id = IDX(c, K, J, I);
        size_t col = COL(c, J, I);
        const double *gcov, *gcon;
        double gdet, alpha;
        geom_of(c, 0, col, &gcov, &gcon, &gdet, &alpha);
        double Pc[5], Bc[3];
        for (int v = 0; v < 5; v++) Pc[v] = P[v * nc + id];
        Bc[0] = 0.5 * (B[id] + B[IDX(c, K, J, I + 1)]) / gdet;
        Bc[1] = 0.5 * (B[nc + id] + B[nc + IDX(c, K, J + 1, I)]) / gdet;
        Bc[2] = 0.5 * (B[2 * nc + id] + B[2 * nc + IDX(c, K + 1, J, I)]) / gdet;
        double inv = 0.0;
        for (int d = 0; d < 3; d++) {
          double vmax, vmin;
          orc_vchar(Pc, Bc, gcov, gcon, alpha, c->d.gam, d + 1, &vmax, &vmin);
          inv += fmax(fabs(vmax), fabs(vmin)) / c->dx[d];
        }
        double dtc = 1.0 / inv;
        if (dtc < best) best = dtc;
      }
  return c->d.courant * best;
}

double orc_step(orc_ctx* c, double* P, double* B, int nsteps, double dt_fixed, orc_stats* st) {
  const size_t nc = c->ncell;
  double dt = 0.0;
  for (int s = 0; s < nsteps; s++) {
    orc_fill_bc(c, P, B);
    dt = dt_fixed > 0.0 ? dt_fixed : orc_dt(c, P, B);
    memcpy(c->P1, P, 5 * nc * sizeof(double));
    memcpy(c->B1, B, 3 * nc * sizeof(double));
    orc_stage(c, P, B, P, B, 0.5 * dt, c->P1, c->B1, st);
    orc_fill_bc(c, c->P1, c->B1);
    memcpy(c->P2, P, 5 * nc * sizeof(double));
    memcpy(c->B2, B, 3 * nc * sizeof(double));
    orc_stage(c, P, B, c->P1, c->B1, dt, c->P2, c->B2, st);
    memcpy(P, c->P2, 5 * nc * sizeof(double));
    memcpy(B, c->B2, 3 * nc * sizeof(double));
  }
  orc_fill_bc(c, P, B);
  return dt;
}

double orc_divb(orc_ctx* c, const double* B, double* field, double* max_rel) {
  const int g = c->d.ng, n1 = c->d.n[0], n2 = c->d.n[1], n3 = c->d.n[2];
  const size_t nc = c->ncell;
  double mx = 0.0, mr = 0.0;
  for (int K = g; K < g + n3; K++)
    for (int J = g; J < g + n2; J++)
      for (int I = g; I < g + n1; I++) {
        size_t id = IDX(c, K, J, I);
        double b1p = B[IDX(c, K, J, I + 1)], b1m = B[id];
        double b2p = B[nc + IDX(c, K, J + 1, I)], b2m = B[nc + id];
        double b3p = B[2 * nc + IDX(c, K + 1, J, I)], b3m = B[2 * nc + id];
        double dv = (b1p - b1m) / c->dx[0] + (b2p - b2m) / c->dx[1] + (b3p - b3m) / c->dx[2];
        /* the same sum with every term taken by magnitude: the scale the differences
         * cancel against.  The relative form is taken where the scale is at least
         * 2^-969 (2^53 times the smallest normal double): below it the face values are
         * subnormal and carry no relative precision (a field-free region underflows). */
        double scale = (fabs(b1p) + fabs(b1m)) / c->dx[0] + (fabs(b2p) + fabs(b2m)) / c->dx[1]
                       + (fabs(b3p) + fabs(b3m)) / c->dx[2];
        if (field) field[id] = dv;
        if (fabs(dv) > mx) mx = fabs(dv);
        if (scale >= ldexp(1.0, -969) && fabs(dv) / scale > mr) mr = fabs(dv) / scale;
      }
  if (max_rel) *max_rel = mr;
  return mx;
}

int orc_reinvert(orc_ctx* c, double* P, const double* Bold, const double* Bnew, int K, int J,
                 int I, const double* dU, orc_stats* st) {
  const size_t nc = c->ncell;
  size_t id = IDX(c, K, J, I);
  size_t col = COL(c, J, I);
  const double *gcov, *gcon;
  double gdet, alpha;
  geom_of(c, 0, col, &gcov, &gcon, &gdet, &alpha);
  double P0[5], Bc[3], U[9];
  for (int v = 0; v < 5; v++) P0[v] = P[v * nc + id];
  Bc[0] = 0.5 * (Bold[id] + Bold[IDX(c, K, J, I + 1)]) / gdet;
  Bc[1] = 0.5 * (Bold[nc + id] + Bold[nc + IDX(c, K, J + 1, I)]) / gdet;
  Bc[2] = 0.5 * (Bold[2 * nc + id] + Bold[2 * nc + IDX(c, K + 1, J, I)]) / gdet;
  orc_prim_to_flux(P0, Bc, gcov, gcon, gdet, alpha, c->d.gam, 0, U);
  static const int comps[6] = {0, 1, 2, 3, 4, 8};
  for (int q = 0; q < 6; q++) U[comps[q]] += dU[comps[q]];
  U[5] = 0.5 * (Bnew[id] + Bnew[IDX(c, K, J, I + 1)]);
  U[6] = 0.5 * (Bnew[nc + id] + Bnew[nc + IDX(c, K, J + 1, I)]);
  U[7] = 0.5 * (Bnew[2 * nc + id] + Bnew[2 * nc + IDX(c, K + 1, J, I)]);
  double Pnew[5], Bn[3];
  int it = 0;
  int tier = orc_cons2prim(U, gcov, gcon, gdet, alpha, c->d.gam, P0, P0, c->d.tol, c->d.maxit,
                           Pnew, &it);
  for (int i = 0; i < 3; i++) Bn[i] = U[5 + i] / gdet;
  int hits = apply_floors(c, Pnew, Bn, gcov, gcon, gdet, alpha, col);
  for (int v = 0; v < 5; v++) P[v * nc + id] = Pnew[v];
  if (st) {
    st->tier[tier]++;
    st->iter_hist[it < 63 ? it : 63]++;
    st->floor_hits += hits;
  }
  return tier;
}
