// device.h -- per-cell GRMHD physics for gfx950, FP64.
//
// Metric storage follows the exact sparsity of Kerr-Schild in internal coordinates
// (x1 = ln r, x2 = theta, x3 = phi): g_tt g_t1 g_t3 g_11 g_13 g_22 g_33 and
// g^tt g^t1 g^11 g^13 g^22 g^33 are the only non-zero entries (Minkowski is a
// special case), so the contractions below skip the identically-zero terms.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace grmhd {

// geometry quantity indices in the per-column tables (structure of arrays)
enum {
  G00 = 0, G01, G03, G11, G13, G22, G33,   // covariant metric
  H00, H01, H11, H13, H22, H33,            // contravariant metric
  GDET, ALPHA,                              // sqrt(-g), lapse
  NGEO_F,                                   // entries of a face table
  CONN0 = NGEO_F,                           // 40 Christoffels Gamma^l_{mn}, m <= n, l*10 + pair
  RHOFL = CONN0 + 40, UFL,                  // density / internal-energy floors
  NGEO_C
};

// Reciprocal and square roots from the hardware estimates (v_rcp_f64, v_rsq_f64)
// refined by Newton-Raphson steps: r <- r + r (1 - b r) for 1/b, y <- y + y (1/2 - x y^2 / 2)
// for 1/sqrt(x), and one Heron correction s <- s + (x - s^2) / (2 s) for sqrt(x).  A few
// ulp from the correctly rounded values at about half the instructions of the IEEE
// sequences; used where the result only feeds arithmetic (the face fluxes), with
// arguments that are positive and finite there.
__device__ __forceinline__ double rcp_nr(double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(r, fma(-b, r, 1.0), r);
  return fma(r, fma(-b, r, 1.0), r);
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = fma(y, fma(-h * y, y, 0.5), y);
  return fma(y, fma(-h * y, y, 0.5), y);
}
// sqrt(x) for x >= 0; 0 below 2^-1000 (where the estimate's range ends), an absolute
// error under 1e-150
__device__ __forceinline__ double sqrt_nr(double x) {
  const double y = rsq_nr(x);
  double s = x * y;
  s = fma(0.5 * y, fma(-s, s, x), s);
  return x > 0x1p-1000 ? s : 0.0;
}

struct Metric {
  double g00, g01, g03, g11, g13, g22, g33;
  double h00, h01, h11, h13, h22, h33;
  double gdet, alpha;
};

__device__ __forceinline__ Metric load_metric(const double* __restrict__ tab, int64_t ncol,
                                              int64_t col) {
  Metric m;
  m.g00 = tab[G00 * ncol + col];
  m.g01 = tab[G01 * ncol + col];
  m.g03 = tab[G03 * ncol + col];
  m.g11 = tab[G11 * ncol + col];
  m.g13 = tab[G13 * ncol + col];
  m.g22 = tab[G22 * ncol + col];
  m.g33 = tab[G33 * ncol + col];
  m.h00 = tab[H00 * ncol + col];
  m.h01 = tab[H01 * ncol + col];
  m.h11 = tab[H11 * ncol + col];
  m.h13 = tab[H13 * ncol + col];
  m.h22 = tab[H22 * ncol + col];
  m.h33 = tab[H33 * ncol + col];
  m.gdet = tab[GDET * ncol + col];
  m.alpha = tab[ALPHA * ncol + col];
  return m;
}

// v_mu = g_mu nu v^nu
__device__ __forceinline__ void lower4(const Metric& m, const double v[4], double o[4]) {
  o[0] = m.g00 * v[0] + m.g01 * v[1] + m.g03 * v[3];
  o[1] = m.g01 * v[0] + m.g11 * v[1] + m.g13 * v[3];
  o[2] = m.g22 * v[2];
  o[3] = m.g03 * v[0] + m.g13 * v[1] + m.g33 * v[3];
}

struct Fluid {
  double ucon[4], ucov[4], bcon[4], bcov[4];
  double bsq;
};

// four-velocity from the relative velocity utilde^i (Gamma = sqrt(1 + g_ij ut^i ut^j),
// u^t = Gamma/alpha, u^i = ut^i - Gamma beta^i/alpha, beta^i = alpha^2 g^{ti}), and the
// fluid-frame field b^t = B^i u_i, b^i = (B^i + b^t u^i)/u^t.
// FAST: the square root and divisions through rsq_nr / rcp_nr.
template <bool FAST = false>
__device__ __forceinline__ void fluid_state(const double P[5], const double B[3], const Metric& m,
                                            Fluid& f) {
  const double u1 = P[2], u2 = P[3], u3 = P[4];
  const double qsq = m.g11 * u1 * u1 + 2.0 * m.g13 * u1 * u3 + m.g22 * u2 * u2 + m.g33 * u3 * u3;
  const double gamma = FAST ? sqrt_nr(1.0 + qsq) : sqrt(1.0 + qsq);
  f.ucon[0] = FAST ? gamma * rcp_nr(m.alpha) : gamma / m.alpha;
  f.ucon[1] = u1 - gamma * (m.alpha * m.h01);   // beta^1/alpha = alpha g^{t1}
  f.ucon[2] = u2;
  f.ucon[3] = u3;
  lower4(m, f.ucon, f.ucov);
  const double bt = B[0] * f.ucov[1] + B[1] * f.ucov[2] + B[2] * f.ucov[3];
  f.bcon[0] = bt;
  const double iut = FAST ? rcp_nr(f.ucon[0]) : 1.0 / f.ucon[0];
  f.bcon[1] = (B[0] + bt * f.ucon[1]) * iut;
  f.bcon[2] = (B[1] + bt * f.ucon[2]) * iut;
  f.bcon[3] = (B[2] + bt * f.ucon[3]) * iut;
  lower4(m, f.bcon, f.bcov);
  f.bsq = f.bcon[0] * f.bcov[0] + f.bcon[1] * f.bcov[1] + f.bcon[2] * f.bcov[2] +
          f.bcon[3] * f.bcov[3];
}

// entropy tracer kappa = p / rho^gamma of a state (one power per state; for the
// relativistic gamma = 4/3 the power is rho cbrt(rho), a cube root instead of a general
// log/exp power)
template <bool FAST = false>
__device__ __forceinline__ double entropy_kappa(const double P[5], double gam) {
  const double rg = gam == 4.0 / 3.0 ? P[0] * cbrt(P[0]) : pow(P[0], gam);
  return FAST ? (gam - 1.0) * P[1] * rcp_nr(rg) : (gam - 1.0) * P[1] / rg;
}

// Conserved vector (D = 0) or flux along x^D (D = 1..3), times sqrt(-g):
//   rho u^D, T^D_t + rho u^D, T^D_i, b^i u^D - b^D u^i, kappa rho u^D
// with T^m_n = (rho + u + p + b^2) u^m u_n + delta^m_n (p + b^2/2) - b^m b_n.
// The induction component along D itself (identically zero for D >= 1) is skipped:
// out[5..6] hold the two other field components in increasing order and out[7] the
// entropy; for D = 0 out[5..7] are the three field components and out[8] the entropy.

template <int D>
__device__ __forceinline__ void flux_vector(const double P[5], const Fluid& f, const Metric& m,
                                            double gam, double kappa, double* out) {
  const double rho = P[0], u = P[1];
  const double p = (gam - 1.0) * u;
  const double w = rho + u + p;
  const double wb = w + f.bsq;
  const double pb = p + 0.5 * f.bsq;
  const double ud = f.ucon[D], bd = f.bcon[D];
  const double mass = rho * ud;
  const double g = m.gdet;
  out[0] = g * mass;
  out[1] = g * (wb * ud * f.ucov[0] + (D == 0 ? pb : 0.0) - bd * f.bcov[0] + mass);
  out[2] = g * (wb * ud * f.ucov[1] + (D == 1 ? pb : 0.0) - bd * f.bcov[1]);
  out[3] = g * (wb * ud * f.ucov[2] + (D == 2 ? pb : 0.0) - bd * f.bcov[2]);
  out[4] = g * (wb * ud * f.ucov[3] + (D == 3 ? pb : 0.0) - bd * f.bcov[3]);
  if (D == 0) {
    out[5] = g * (f.bcon[1] * ud - bd * f.ucon[1]);
    out[6] = g * (f.bcon[2] * ud - bd * f.ucon[2]);
    out[7] = g * (f.bcon[3] * ud - bd * f.ucon[3]);
    out[8] = g * kappa * mass;
  } else {
    constexpr int t1 = D == 1 ? 2 : 1;
    constexpr int t2 = D == 3 ? 2 : 3;
    out[5] = g * (f.bcon[t1] * ud - bd * f.ucon[t1]);
    out[6] = g * (f.bcon[t2] * ud - bd * f.ucon[t2]);
    out[7] = g * kappa * mass;
  }
}

// Fast-speed estimate along x^D: roots of A v^2 - B v + C = 0 from
// (k.u)^2 = c_ms^2 (k.k + (k.u)^2), k = (-v, e_D), c_ms^2 = v_A^2 + c_s^2 (1 - v_A^2).
template <int D, bool FAST = false>
__device__ __forceinline__ void wave_speeds(const double P[5], const Fluid& f, const Metric& m,
                                            double gam, double& vmax, double& vmin) {
  const double p = (gam - 1.0) * P[1];
  const double w = P[0] + P[1] + p;
  const double wb = f.bsq + w;
  const double r = FAST ? rcp_nr(w * wb) : 1.0 / (w * wb);   // one division for both ratios
  const double cs2 = gam * p * wb * r;
  const double va2 = f.bsq * w * r;
  const double cms2 = va2 + cs2 * (1.0 - va2);
  const double ut = f.ucon[0], ud = f.ucon[D];
  const double h0d = D == 1 ? m.h01 : 0.0;
  const double hdd = D == 1 ? m.h11 : (D == 2 ? m.h22 : m.h33);
  const double A = ut * ut * (1.0 - cms2) - cms2 * m.h00;
  const double B = 2.0 * (ut * ud * (1.0 - cms2) - cms2 * h0d);
  const double C = ud * ud * (1.0 - cms2) - cms2 * hdd;
  double disc = B * B - 4.0 * A * C;
  disc = fmax(disc, 0.0);
  const double sq = FAST ? sqrt_nr(disc) : sqrt(disc);
  const double i2a = FAST ? 0.5 * rcp_nr(A) : 0.5 / A;
  const double vp = (B + sq) * i2a, vm = (B - sq) * i2a;
  vmax = fmax(vp, vm);
  vmin = fmin(vp, vm);
}

// ------------------------------------------------------------------ reconstruction

// min(2|dm|, 2|dp|, |dm + dp|/2) with the sign of dm, zero at an extremum; min and
// copysign map to single instructions (v_min_f64, a bit insert) where compare-and-select
// forms take three each
__device__ __forceinline__ double mc_lim(double dm, double dp) {
  if (dm * dp <= 0.0) return 0.0;
  const double s = fmin(2.0 * fmin(fabs(dm), fabs(dp)), 0.5 * fabs(dm + dp));
  return copysign(s, dm);
}

// the smaller one-sided difference (MINMOD), zero at an extremum
__device__ __forceinline__ double mm_lim(double dm, double dp) {
  if (dm * dp <= 0.0) return 0.0;
  return fabs(dm) < fabs(dp) ? dm : dp;
}

// the piecewise-linear limiter of RECON (0: monotonised central, 2: MINMOD)
template <int RECON>
__device__ __forceinline__ double plm_lim(double dm, double dp) {
  return RECON == 2 ? mm_lim(dm, dp) : mc_lim(dm, dp);
}

// monotonised parabola of one cell (Colella & Woodward 1984)
__device__ __forceinline__ void ppm_limit(double a0, double& l, double& r) {
  if ((r - a0) * (a0 - l) <= 0.0) {
    l = a0;
    r = a0;
  } else {
    const double d = r - l;
    const double m6 = 6.0 * (a0 - 0.5 * (l + r));
    if (d * m6 > d * d) l = 3.0 * a0 - 2.0 * r;
    else if (-d * d > d * m6) r = 3.0 * a0 - 2.0 * l;
  }
}

// Shock flattening (Colella & Woodward 1984) of the cell at line index c (c - 2 .. c + 2
// inside the lines): the u_g line u stands for the pressure (an ideal gas, ratios only),
// v is the normal velocity.  Where the jump over the neighbours exceeds 0.33 of the lower
// neighbour's value and the flow compresses, clip(10 (dp1/dp2 - 0.75), 0, 1) with dp1
// the jump over the neighbours and dp2 over the next ones; 0 elsewhere and where dp2
// vanishes
__device__ __forceinline__ double flatten_coef(const double* u, const double* v, int c) {
  const double dp1 = u[c + 1] - u[c - 1], dp2 = u[c + 2] - u[c - 2];
  const double pmin = fmin(u[c + 1], u[c - 1]);
  if (!(fabs(dp1) > 0.33 * pmin) || !(v[c - 1] - v[c + 1] > 0.0) || dp2 == 0.0) return 0.0;
  return fmin(1.0, fmax(0.0, 10.0 * (dp1 / dp2 - 0.75)));
}

// a cell's interface values pulled toward its mean by its flattening coefficient f
__device__ __forceinline__ void flatten_cell(double a0, double f, double& l, double& r) {
  l = f * a0 + (1.0 - f) * l;
  r = f * a0 + (1.0 - f) * r;
}

// face states of the face between s[2] and s[3] from the six-cell line s[0..5]; RECON 3
// (PPM with flattening) takes the flattening coefficients fl[0], fl[1] of s[2], s[3]
template <int RECON>
__device__ __forceinline__ void recon_face(const double s[6], double& left, double& right,
                                           const double* fl = nullptr) {
  if (RECON == 0 || RECON == 2) {
    left = s[2] + 0.5 * plm_lim<RECON>(s[2] - s[1], s[3] - s[2]);
    right = s[3] - 0.5 * plm_lim<RECON>(s[3] - s[2], s[4] - s[3]);
  } else {
    const double d1 = mc_lim(s[1] - s[0], s[2] - s[1]);
    const double d2 = mc_lim(s[2] - s[1], s[3] - s[2]);
    const double d3 = mc_lim(s[3] - s[2], s[4] - s[3]);
    const double d4 = mc_lim(s[4] - s[3], s[5] - s[4]);
    constexpr double sixth = 1.0 / 6.0;   // a multiply instead of three divisions
    const double f15 = 0.5 * (s[1] + s[2]) - (d2 - d1) * sixth;
    const double f25 = 0.5 * (s[2] + s[3]) - (d3 - d2) * sixth;
    const double f35 = 0.5 * (s[3] + s[4]) - (d4 - d3) * sixth;
    double l2 = f15, r2 = f25, l3 = f25, r3 = f35;
    if (RECON == 3) {
      flatten_cell(s[2], fl[0], l2, r2);
      flatten_cell(s[3], fl[1], l3, r3);
    }
    ppm_limit(s[2], l2, r2);
    ppm_limit(s[3], l3, r3);
    left = r2;
    right = l3;
  }
}

// face states of the faces between s[2], s[3] (l0, r0) and between s[3], s[4] (l1, r1)
// from the seven-cell line s[0..6]: the same values as recon_face on each face, with the
// slopes, interface values and limited parabola of the shared cells computed once
template <int RECON>
__device__ __forceinline__ void recon_pair(const double s[7], double& l0, double& r0, double& l1,
                                           double& r1, const double* fl = nullptr) {
  if (RECON == 0 || RECON == 2) {
    const double d2 = plm_lim<RECON>(s[2] - s[1], s[3] - s[2]);
    const double d3 = plm_lim<RECON>(s[3] - s[2], s[4] - s[3]);
    const double d4 = plm_lim<RECON>(s[4] - s[3], s[5] - s[4]);
    l0 = s[2] + 0.5 * d2;
    r0 = s[3] - 0.5 * d3;
    l1 = s[3] + 0.5 * d3;
    r1 = s[4] - 0.5 * d4;
  } else {
    const double d1 = mc_lim(s[1] - s[0], s[2] - s[1]);
    const double d2 = mc_lim(s[2] - s[1], s[3] - s[2]);
    const double d3 = mc_lim(s[3] - s[2], s[4] - s[3]);
    const double d4 = mc_lim(s[4] - s[3], s[5] - s[4]);
    const double d5 = mc_lim(s[5] - s[4], s[6] - s[5]);
    constexpr double sixth = 1.0 / 6.0;
    const double f15 = 0.5 * (s[1] + s[2]) - (d2 - d1) * sixth;
    const double f25 = 0.5 * (s[2] + s[3]) - (d3 - d2) * sixth;
    const double f35 = 0.5 * (s[3] + s[4]) - (d4 - d3) * sixth;
    const double f45 = 0.5 * (s[4] + s[5]) - (d5 - d4) * sixth;
    double l2 = f15, r2 = f25, l3 = f25, r3 = f35, l4 = f35, r4 = f45;
    if (RECON == 3) {
      flatten_cell(s[2], fl[0], l2, r2);
      flatten_cell(s[3], fl[1], l3, r3);
      flatten_cell(s[4], fl[2], l4, r4);
    }
    ppm_limit(s[2], l2, r2);
    ppm_limit(s[3], l3, r3);
    ppm_limit(s[4], l4, r4);
    l0 = r2;
    r0 = l3;
    l1 = r3;
    r1 = l4;
  }
}

// -------------------------------------------------------------- geometric source

// Qbar_nu = sqrt(-g) T^k_l Gamma^l_{nu k} for nu = t, 1, 2, 3 (energy and momentum)
__device__ __forceinline__ int sym_pair(int a, int b) {
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  return lo * 4 - (lo * (lo + 1)) / 2 + hi;   // (0,0)=0 .. (3,3)=9
}

// T^k_l of a state: (rho + u + p + b^2) u^k u_l + delta^k_l (p + b^2/2) - b^k b_l
__device__ __forceinline__ void stress_energy(const double P[5], const Fluid& f, double gam,
                                              double T[4][4]) {
  const double p = (gam - 1.0) * P[1];
  const double wb = P[0] + P[1] + p + f.bsq;
  const double pb = p + 0.5 * f.bsq;
#pragma unroll
  for (int k = 0; k < 4; k++)
#pragma unroll
    for (int l = 0; l < 4; l++)
      T[k][l] = wb * f.ucon[k] * f.ucov[l] + (k == l ? pb : 0.0) - f.bcon[k] * f.bcov[l];
}

// q_nu += T^k_l Gamma^l_{nu k} over l = l0, l0 + 1 (conn: the 20 coefficients
// Gamma^l_{mn}, m <= n, of those two l); summed over l, then k, so that successive calls
// for l0 = 0 and 2 add the terms in the order of the full contraction
__device__ __forceinline__ void connection_contract(const double T[4][4], const double conn[20],
                                                    int l0, double q[4]) {
#pragma unroll
  for (int nu = 0; nu < 4; nu++)
#pragma unroll
    for (int dl = 0; dl < 2; dl++)
#pragma unroll
      for (int k = 0; k < 4; k++) q[nu] += T[k][l0 + dl] * conn[dl * 10 + sym_pair(nu, k)];
}

// ---------------------------------------------------------------- inversion

struct C2PIn {
  double D, Qdotn, Qtsq, Bsq, QdotB, QdotBsq, kappa, gam;
  double Q1, Q2, Q3, B1, B2, B3;
  double y11, y13, y22, y33;   // spatial inverse metric gamma^{ij}
};

__device__ __forceinline__ void c2p_setup(const double U[9], const Metric& m, double gam,
                                          C2PIn& s) {
  const double ig = 1.0 / m.gdet;
  const double a = m.alpha;
  s.gam = gam;
  s.D = a * U[0] * ig;
  const double Qt = a * U[1] * ig - s.D;
  s.Q1 = a * U[2] * ig;
  s.Q2 = a * U[3] * ig;
  s.Q3 = a * U[4] * ig;
  s.B1 = a * U[5] * ig;
  s.B2 = a * U[6] * ig;
  s.B3 = a * U[7] * ig;
  const double beta1 = a * a * m.h01;
  s.Qdotn = (Qt - beta1 * s.Q1) / a;
  s.y11 = m.h11 + beta1 * beta1 / (a * a);
  s.y13 = m.h13;
  s.y22 = m.h22;
  s.y33 = m.h33;
  s.Qtsq = s.y11 * s.Q1 * s.Q1 + 2.0 * s.y13 * s.Q1 * s.Q3 + s.y22 * s.Q2 * s.Q2 +
           s.y33 * s.Q3 * s.Q3;
  s.Bsq = m.g11 * s.B1 * s.B1 + 2.0 * m.g13 * s.B1 * s.B3 + m.g22 * s.B2 * s.B2 +
          m.g33 * s.B3 * s.B3;
  s.QdotB = s.Q1 * s.B1 + s.Q2 * s.B2 + s.Q3 * s.B3;
  s.QdotBsq = s.QdotB * s.QdotB;
  s.kappa = U[8] / U[0];
}

__device__ __forceinline__ double c2p_R2(const C2PIn& s, double W, double vsq) {
  const double p = (s.gam - 1.0) / s.gam * (W * (1.0 - vsq) - s.D * sqrt(1.0 - vsq));
  return -0.5 * s.Bsq * (1.0 + vsq) + s.QdotBsq / (2.0 * W * W) - W + p - s.Qdotn;
}

__device__ __forceinline__ double c2p_vsq_of_W(const C2PIn& s, double W) {
  const double BW = s.Bsq + W;
  return (s.Qtsq + s.QdotBsq * (s.Bsq + 2.0 * W) / (W * W)) / (BW * BW);
}

__device__ __forceinline__ bool c2p_prims(const C2PIn& s, double W, double vsq, double rho,
                                          double u, double gamma, double P[5]) {
  if (!(rho > 0.0) || !(u > 0.0)) return false;
  P[0] = rho;
  P[1] = u;
  const double f = gamma / (W + s.Bsq);
  const double qb = s.QdotB / W;
  P[2] = f * (s.y11 * s.Q1 + s.y13 * s.Q3 + qb * s.B1);
  P[3] = f * (s.y22 * s.Q2 + qb * s.B2);
  P[4] = f * (s.y13 * s.Q1 + s.y33 * s.Q3 + qb * s.B3);
  return true;
}

__device__ __forceinline__ bool c2p_from_Wv(const C2PIn& s, double W, double vsq, double P[5]) {
  if (!(W > 0.0) || !(vsq >= 0.0) || !(vsq < 1.0)) return false;
  const double gamma = 1.0 / sqrt(1.0 - vsq);
  const double rho = s.D / gamma;
  const double u = (W * (1.0 - vsq) - rho) / s.gam;
  return c2p_prims(s, W, vsq, rho, u, gamma, P);
}

// 2D Newton in (W, v^2) (Noble et al. 2006) from a guess (W0, v0).  Converged when
// |dW| <= tol W and |dv^2| <= tol; one more iteration then polishes the root.
__device__ __forceinline__ bool c2p_newton_wv(const C2PIn& s, double W0, double v0, double tol,
                                              int maxit, double P[5], int& iters) {
  double W = W0, vsq = v0;
  iters = 0;
  if (!(W > 0.0) || !(vsq >= 0.0) || !(vsq < 1.0)) return false;
  const double gm = (s.gam - 1.0) / s.gam;
  bool conv = false;
  int it;
  for (it = 1; it <= maxit; it++) {
    const double BW = s.Bsq + W;
    const double sq = sqrt(1.0 - vsq);
    const double isq = 1.0 / sq;
    const double iW = 1.0 / W;            // one division for the powers of 1/W
    const double iW2 = iW * iW;
    const double R1 = vsq * BW * BW - s.QdotBsq * (s.Bsq + 2.0 * W) * iW2 - s.Qtsq;
    const double R2 = -0.5 * s.Bsq * (1.0 + vsq) + 0.5 * s.QdotBsq * iW2 - W +
                      gm * (W * (1.0 - vsq) - s.D * sq) - s.Qdotn;
    const double iW3 = iW2 * iW;
    const double J11 = 2.0 * vsq * BW + 2.0 * s.QdotBsq * BW * iW3;
    const double J12 = BW * BW;
    const double J21 = -s.QdotBsq * iW3 - 1.0 + gm * (1.0 - vsq);
    const double J22 = -0.5 * s.Bsq + gm * (-W + 0.5 * s.D * isq);
    const double idet = 1.0 / (J11 * J22 - J12 * J21);
    const double dW = -(R1 * J22 - J12 * R2) * idet;
    const double dv = -(J11 * R2 - J21 * R1) * idet;
    double Wn = W + dW, vn = vsq + dv;
    if (!(Wn > 0.0)) Wn = 0.5 * W;
    if (vn < 0.0) vn = 0.0;
    if (!(vn < 1.0)) vn = vsq + 0.5 * (1.0 - vsq);
    const double chW = fabs(Wn - W), chv = fabs(vn - vsq);
    W = Wn;
    vsq = vn;
    if (conv) break;
    if (chW <= tol * W && chv <= tol) conv = true;
  }
  iters = it > maxit ? maxit : it;
  if (!conv) return false;
  return c2p_from_Wv(s, W, vsq, P);
}

// the plain guess: W and v^2 of a primitive state under this metric
__device__ __forceinline__ void guess_from_prims(const C2PIn& s, const Metric& m, const double G[5],
                                                 double& W, double& vsq) {
  const double qsq = m.g11 * G[2] * G[2] + 2.0 * m.g13 * G[2] * G[4] + m.g22 * G[3] * G[3] +
                     m.g33 * G[4] * G[4];
  const double gsq = 1.0 + qsq;
  W = (G[0] + s.gam * G[1]) * gsq;
  vsq = qsq / gsq;
}

// one-variable energy equation in W (v^2 eliminated through the momentum equation),
// bracketed and bisected to the last bit
__device__ __forceinline__ bool c2p_energy_1d(const C2PIn& s, double P[5]) {
  double Wb = fabs(s.Qdotn) + s.D + s.Bsq;
  if (!(Wb > 0.0)) return false;
  int k;
  for (k = 0; k < 200 && !(c2p_vsq_of_W(s, Wb) < 1.0); k++) Wb *= 2.0;
  if (k == 200) return false;
  double lo = 0.0, hi = Wb;
  for (k = 0; k < 200; k++) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (c2p_vsq_of_W(s, mid) < 1.0) hi = mid;
    else lo = mid;
  }
  const double Wlo = hi;
  if (!(c2p_R2(s, Wlo, c2p_vsq_of_W(s, Wlo)) > 0.0)) return false;
  double Whi = 2.0 * Wlo;
  for (k = 0; k < 200; k++) {
    if (c2p_R2(s, Whi, c2p_vsq_of_W(s, Whi)) < 0.0) break;
    Whi *= 2.0;
  }
  if (k == 200) return false;
  lo = Wlo;
  hi = Whi;
  for (k = 0; k < 300; k++) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (c2p_R2(s, mid, c2p_vsq_of_W(s, mid)) > 0.0) lo = mid;
    else hi = mid;
  }
  const double W = 0.5 * (lo + hi);
  return c2p_from_Wv(s, W, c2p_vsq_of_W(s, W), P);
}

// entropy backup: p = kappa rho^gamma replaces the energy equation (Sec. 2.6)
__device__ __forceinline__ double entropy_W(const C2PIn& s, double vsq) {
  const double rho = s.D * sqrt(1.0 - vsq);
  const double p = s.kappa * pow(rho, s.gam);
  return (rho + s.gam / (s.gam - 1.0) * p) / (1.0 - vsq);
}

__device__ __forceinline__ bool c2p_entropy(const C2PIn& s, double P[5]) {
  if (!(s.kappa > 0.0) || !(s.D > 0.0)) return false;
  double lo = 0.0, hi = 1.0 - 0x1p-53;
  for (int k = 0; k < 300; k++) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    const double W = entropy_W(s, mid);
    const double BW = s.Bsq + W;
    const double R1 = mid * BW * BW - s.QdotBsq * (s.Bsq + 2.0 * W) / (W * W) - s.Qtsq;
    if (R1 < 0.0) lo = mid;
    else hi = mid;
  }
  const double vsq = 0.5 * (lo + hi);
  const double W = entropy_W(s, vsq);
  if (!(W > 0.0)) return false;
  const double gamma = 1.0 / sqrt(1.0 - vsq);
  const double rho = s.D / gamma;
  const double u = s.kappa * pow(rho, s.gam) / (s.gam - 1.0);
  return c2p_prims(s, W, vsq, rho, u, gamma, P);
}

// size of the two residuals at a guess, each in its natural scale (momentum: (B^2 +
// W)^2, energy: W); infinite for a guess outside W > 0, 0 <= v^2 < 1
__device__ __forceinline__ double c2p_misfit(const C2PIn& s, double W, double vsq) {
  if (!(W > 0.0) || !(vsq >= 0.0) || !(vsq < 1.0)) return __longlong_as_double(0x7FF0000000000000LL);
  const double BW = s.Bsq + W;
  const double iW = 1.0 / W;
  const double R1 = vsq * BW * BW - s.QdotBsq * (s.Bsq + 2.0 * W) * iW * iW - s.Qtsq;
  return fabs(R1) / (BW * BW) + fabs(c2p_R2(s, W, vsq)) * iW;
}

// Inversion with the fallback chain; returns the tier used (0..4).  With a second guess
// (W0, v0) (`first`: the learned guess), tier 0 is Newton from whichever of it and the
// plain guess prev has the smaller residual misfit, tier 1 Newton from the other;
// without, tier 0 starts from prev.  Tiers 2 and 3 are the bracketed energy and entropy
// solves; tier 4 keeps prev.
__device__ __forceinline__ int c2p_solve(const C2PIn& s, const Metric& m, bool first, double W0,
                                         double v0, const double prev[5], double tol, int maxit,
                                         double P[5], int& iters) {
  double Wp, vp;
  guess_from_prims(s, m, prev, Wp, vp);
  if (first) {
    if (c2p_misfit(s, Wp, vp) < c2p_misfit(s, W0, v0)) {
      const double tw = W0, tv = v0;
      W0 = Wp;
      v0 = vp;
      Wp = tw;
      vp = tv;
    }
    if (c2p_newton_wv(s, W0, v0, tol, maxit, P, iters)) return 0;
    if (c2p_newton_wv(s, Wp, vp, tol, maxit, P, iters)) return 1;
  } else {
    if (c2p_newton_wv(s, Wp, vp, tol, maxit, P, iters)) return 0;
  }
  iters = 63;
  if (c2p_energy_1d(s, P)) return 2;
  if (c2p_entropy(s, P)) return 3;
  for (int v = 0; v < 5; v++) P[v] = prev[v];
  return 4;
}

// inversion from primitive guesses: guess (tier 0) and prev (tier 1, fallback)
__device__ __forceinline__ int cons2prim(const double U[9], const Metric& m, double gam,
                                         const double guess[5], const double prev[5],
                                         bool distinct_guess, double tol, int maxit,
                                         double P[5], int& iters) {
  C2PIn s;
  c2p_setup(U, m, gam, s);
  if (!distinct_guess) return c2p_solve(s, m, false, 0.0, 0.0, prev, tol, maxit, P, iters);
  double W0, v0;
  guess_from_prims(s, m, guess, W0, v0);
  return c2p_solve(s, m, true, W0, v0, prev, tol, maxit, P, iters);
}

// raw MLP features of an inversion input (see mlp.h); false if any is not finite.  The
// ratios are formed in FP64 (their range can exceed FP32's), the logarithms in FP32:
// the features feed BF16 products, far coarser than FP32 rounding.
__device__ __forceinline__ bool mlp_features(const C2PIn& s, const Metric& m, float x[8]) {
  const double D = s.D;
  const double iD = 1.0 / D;
  const double tau = -s.Qdotn - D;
  x[0] = logf((float)D);
  x[1] = asinhf((float)(tau * iD));
  x[2] = log1pf((float)(s.Qtsq * iD * iD));
  x[3] = log1pf((float)(s.Bsq * iD));
  x[4] = log1pf((float)(s.QdotBsq * iD * iD * iD));
  x[5] = (float)m.alpha;
  x[6] = (float)s.gam;
  x[7] = (float)(m.gdet / m.alpha);
  bool ok = D > 0.0;
#pragma unroll
  for (int k = 0; k < 8; k++) ok = ok && isfinite(x[k]);
  return ok;
}

// floors (Sec. 2.7): Lorentz-factor ceiling, then rho >= max(rho_fl, b^2/bsq_rho_max)
// and u >= max(u_fl, b^2/bsq_u_max); returns the number of limits applied
__device__ __forceinline__ int apply_floors(double P[5], const double B[3], const Metric& m,
                                            double rho_fl, double u_fl, double bsq_rho_max,
                                            double bsq_u_max, double gamma_max) {
  int hits = 0;
  const double qsq = m.g11 * P[2] * P[2] + 2.0 * m.g13 * P[2] * P[4] + m.g22 * P[3] * P[3] +
                     m.g33 * P[4] * P[4];
  if (1.0 + qsq > gamma_max * gamma_max) {
    const double f = sqrt((gamma_max * gamma_max - 1.0) / qsq);
    P[2] *= f;
    P[3] *= f;
    P[4] *= f;
    hits++;
  }
  Fluid fl;
  fluid_state(P, B, m, fl);
  const double rmin = fmax(rho_fl, fl.bsq / bsq_rho_max);
  const double umin = fmax(u_fl, fl.bsq / bsq_u_max);
  if (P[0] < rmin) { P[0] = rmin; hits++; }
  if (P[1] < umin) { P[1] = umin; hits++; }
  return hits;
}

// Floors in the drift frame (Sec. 2.7, Ressler et al. 2017): after the Lorentz-factor
// ceiling, the missing mass and internal energy (drho = rmin - rho, du = umin - u where
// positive) are added as a parcel moving with the field's drift frame u_D = g (u + beta
// b), beta = -b^t / (b^2 u^t) (the fluid four-velocity with its motion along the field
// removed; beta^2 b^2 capped at 1 - 1/gamma_max^2), carrying no field.  The summed
// conserved state U(P) + U(parcel), with the cell's specific entropy, is inverted from P;
// the fixed-utilde floors then restore the minima after rounding (not counted), or act
// alone where that inversion needs the entropy or keep-previous tier.
__device__ __forceinline__ int drift_floors(double P[5], const double B[3], const Metric& m,
                                         double rho_fl, double u_fl, double bsq_rho_max,
                                         double bsq_u_max, double gamma_max, double gam,
                                         double tol, int maxit) {
  int hits = 0;
  const double qsq = m.g11 * P[2] * P[2] + 2.0 * m.g13 * P[2] * P[4] + m.g22 * P[3] * P[3] +
                     m.g33 * P[4] * P[4];
  if (1.0 + qsq > gamma_max * gamma_max) {
    const double f = sqrt((gamma_max * gamma_max - 1.0) / qsq);
    P[2] *= f;
    P[3] *= f;
    P[4] *= f;
    hits++;
  }
  Fluid fl;
  fluid_state(P, B, m, fl);
  const double rmin = fmax(rho_fl, fl.bsq / bsq_rho_max);
  const double umin = fmax(u_fl, fl.bsq / bsq_u_max);
  const double drho = fmax(rmin - P[0], 0.0), du = fmax(umin - P[1], 0.0);
  if (!(drho > 0.0 || du > 0.0)) return hits;
  // beta b is the same for every multiple of the field: it is formed from the field over
  // its largest component, which keeps weak fields (b^2 below the smallest normal double)
  // clear of underflow; no field at all leaves the fluid frame
  double ud[4];
#pragma unroll
  for (int q = 0; q < 4; q++) ud[q] = fl.ucon[q];
  const double bmax = fmax(fmax(fabs(B[0]), fabs(B[1])), fabs(B[2]));
  if (bmax > 0.0) {
    const double Bs[3] = {B[0] / bmax, B[1] / bmax, B[2] / bmax};
    double bc[4], bl[4];
    bc[0] = Bs[0] * fl.ucov[1] + Bs[1] * fl.ucov[2] + Bs[2] * fl.ucov[3];
    const double iut = 1.0 / fl.ucon[0];
#pragma unroll
    for (int i = 1; i < 4; i++) bc[i] = (Bs[i - 1] + bc[0] * fl.ucon[i]) * iut;
    lower4(m, bc, bl);
    const double bsq = bc[0] * bl[0] + bc[1] * bl[1] + bc[2] * bl[2] + bc[3] * bl[3];
    if (bsq > 0.0) {
      const double bp = -bc[0] * iut / bsq;
      const double b2 = fmin(bp * bp * bsq, 1.0 - 1.0 / (gamma_max * gamma_max));
      const double g = 1.0 / sqrt(1.0 - b2);
#pragma unroll
      for (int q = 0; q < 4; q++) ud[q] = g * (fl.ucon[q] + bp * bc[q]);
    }
  }
  // the parcel's primitives: utilde^i = u^i + u^t beta^i, beta^i = alpha^2 g^{ti}
  // (the shift of the Kerr-Schild metric has its x1 component only)
  const double Pp[5] = {drho, du, ud[1] + ud[0] * m.alpha * m.alpha * m.h01, ud[2], ud[3]};
  const double B0[3] = {0.0, 0.0, 0.0};
  double U[9], Up[9], Un[9];
  flux_vector<0>(P, fl, m, gam, entropy_kappa(P, gam), U);
  {
    Fluid fp;
    fluid_state(Pp, B0, m, fp);
    flux_vector<0>(Pp, fp, m, gam, 0.0, Up);
  }
#pragma unroll
  for (int q = 0; q < 8; q++) Un[q] = U[q] + Up[q];
  Un[8] = U[8] / U[0] * Un[0];
  C2PIn cs;
  c2p_setup(Un, m, gam, cs);
  double Pn[5];
  int it = 0;
  const int tier = c2p_solve(cs, m, false, 0.0, 0.0, P, tol, maxit, Pn, it);
  if (tier <= 2) {
#pragma unroll
    for (int v = 0; v < 5; v++) P[v] = Pn[v];
    apply_floors(P, B, m, rho_fl, u_fl, bsq_rho_max, bsq_u_max, gamma_max);
    return hits + (drho > 0.0) + (du > 0.0);
  }
  return hits + apply_floors(P, B, m, rho_fl, u_fl, bsq_rho_max, bsq_u_max, gamma_max);
}

}  // namespace grmhd
