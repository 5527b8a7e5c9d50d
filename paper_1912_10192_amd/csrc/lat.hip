// lat.hip -- kernels of local adaptive time-stepping (paper Sec. 3.5).
//
// Blocks carry a time level; a level-l block steps with dt_min 2^l.  The kernels here
// (1) fill ghosts whose sources run at another time level -- a slower neighbour is
//     interpolated linearly in time between its stored start state and its end state,
// (2) accumulate the time-integrated x1 fluxes and edge EMFs a block used on its x1
//     boundary planes, over its own step and over two of its steps,
// (3) at the end of a slower block's step, replace on each plane shared with a faster
//     neighbour the fluxes and EMFs it used by the faster side's integrals: conserved
//     update of the boundary cells, constrained-transport correction of the faces that
//     touch the shared edges, the faster side's copy of the shared faces, and a new
//     inversion of the corrected cells.
#include <hip/hip_runtime.h>

#include "device.h"
#include "internal.h"
#include "wave.h"

namespace grmhd {

constexpr int LT = 256;

__device__ __forceinline__ BlockInfo list_block(const Launch& L, int y) {
  return L.blk[L.blist ? L.blist[y] : y];
}

// ------------------------------------------------------------------ ghost gather

// The ghosts of one level's blocks from the concatenated lists (cells, then faces of
// components 1..3).  Source per op relation:
//   same level: `cur` (the main state for a predictor, the stage state for a corrector)
//   slower:     old + w (main - old)
//   faster:     main
// Physical-boundary flips, clamps and axis zeros apply afterwards.
__device__ __forceinline__ double timed_value(int fl, int64_t q, const double* __restrict__ main,
                                              const double* __restrict__ old,
                                              const double* __restrict__ cur, double w) {
  if (fl & GF_SLOW) return old[q] + w * (main[q] - old[q]);
  if (fl & GF_FAST) return main[q];
  return cur[q];
}

__global__ __launch_bounds__(LT) void k_ghosts_t(GhostLists G, const double* __restrict__ Pmain,
                                                 const double* __restrict__ Pold,
                                                 const double* __restrict__ Pcur,
                                                 double* __restrict__ Pdst,
                                                 const double* __restrict__ Bmain,
                                                 const double* __restrict__ Bold,
                                                 const double* __restrict__ Bcur,
                                                 double* __restrict__ Bdst, double w) {
  const int64_t t = (int64_t)blockIdx.x * LT + threadIdx.x;
  if (t >= G.end[3]) return;
  if (t < G.end[0]) {
    const GhostIdx op = G.ops[0][t];
    const int fl = op.svol_fl >> 24;
    const int64_t svol = op.svol_fl & 0xFFFFFF;
    double* out = Pdst + op.dst;
#pragma unroll
    for (int v = 0; v < 5; v++) {
      double x = timed_value(fl, op.src + v * svol, Pmain, Pold, Pcur, w);
      if (v == 3 && (fl & GF_FLIP)) x = -x;
      if (v == 2 && (fl & GF_CLAMP_NEG) && x > 0.0) x = 0.0;
      if (v == 2 && (fl & GF_CLAMP_POS) && x < 0.0) x = 0.0;
      out[v * (int64_t)op.dvol] = x;
    }
    return;
  }
  const int k = t < G.end[1] ? 1 : (t < G.end[2] ? 2 : 3);
  const GhostIdx op = G.ops[k][t - G.end[k - 1]];
  const int fl = op.svol_fl >> 24;
  double x = timed_value(fl, op.src, Bmain, Bold, Bcur, w);
  if (fl & GF_ZERO) x = 0.0;
  else if (fl & GF_FLIP) x = -x;
  Bdst[op.dst] = x;
}

// Copy the interior of every listed block: nvar = 5 primitives of the interior cells, or
// nvar = 3 face components, each on and inside the block's boundary (normal index ng to
// ng + n).  Ghost values are not copied: every reader of the copies (the ghost lists)
// takes interior values only, and every ghost is refilled before the stage that uses it.
__global__ __launch_bounds__(LT) void k_copy_blocks(Launch L, const double* __restrict__ src,
                                                    double* __restrict__ dst, int nvar) {
  const BlockInfo bi = list_block(L, blockIdx.y);
  const int g = L.ph.ng;
  const int64_t V = bi.vol;
  const int64_t base = (int64_t)nvar * bi.off;
  const bool faces = nvar == 3;
  for (int v = 0; v < nvar; v++) {
    const int r0 = bi.n[0] + (faces && v == 0 ? 1 : 0);
    const int r1 = bi.n[1] + (faces && v == 1 ? 1 : 0);
    const int r2 = bi.n[2] + (faces && v == 2 ? 1 : 0);
    const int64_t n = (int64_t)r0 * r1 * r2;
    for (int64_t t = (int64_t)blockIdx.x * LT + threadIdx.x; t < n; t += (int64_t)gridDim.x * LT) {
      const int i = (int)(t % r0);
      const int64_t q = t / r0;
      const int j = (int)(q % r1), k = (int)(q / r1);
      const int64_t l = ((int64_t)(k + g) * bi.np[1] + (j + g)) * bi.np[0] + (i + g);
      dst[base + v * V + l] = src[base + v * V + l];
    }
  }
}

// Copy the listed elements: nc cells of the primitives (element indices ic), then nf
// faces of the face field (indices jf).  The lists hold what faster neighbours read as
// the old state of time-interpolated ghosts, a few cell layers along shared faces.
__global__ __launch_bounds__(LT) void k_copy_list(const uint32_t* __restrict__ ic, int64_t nc,
                                                  const double* __restrict__ P,
                                                  double* __restrict__ Pdst,
                                                  const uint32_t* __restrict__ jf, int64_t nf,
                                                  const double* __restrict__ B,
                                                  double* __restrict__ Bdst) {
  const int64_t t = (int64_t)blockIdx.x * LT + threadIdx.x;
  if (t < nc) {
    const uint32_t q = ic[t];
    Pdst[q] = P[q];
  } else if (t < nc + nf) {
    const uint32_t q = jf[t - nc];
    Bdst[q] = B[q];
  }
}

// ------------------------------------------------------------------ registers

// per listed block and x1 side: dt-weighted corrector fluxes (8 components) on the x1
// boundary faces and EMFs E^2, E^3 on the x1 boundary edges; set 0 holds this step,
// set 1 the sum over a pair of steps (restarted when `first` is set)
__global__ __launch_bounds__(LT) void k_registers(Launch L, const double* __restrict__ F,
                                                  const double* __restrict__ E, double dt_factor,
                                                  int first, double* __restrict__ reg, int rs,
                                                  int rs2) {
  const int b = L.blist[blockIdx.y];
  const BlockInfo bi = L.blk[b];
  const int g = L.ph.ng;
  const int t = blockIdx.x * LT + threadIdx.x;
  const int n2 = bi.n[1], n3 = bi.n[2];
  if (t >= 2 * (n3 + 1) * (n2 + 1)) return;
  const int side = t / ((n3 + 1) * (n2 + 1));
  const int r = t % ((n3 + 1) * (n2 + 1));
  const int K = r / (n2 + 1), J = r % (n2 + 1);
  const double dt = dt_factor * L.ph.courant * __longlong_as_double((long long)L.cnt->dt_bits);
  const int I = side == 0 ? g : g + bi.n[0];
  const int64_t V = bi.vol;
  const int64_t loc = ((int64_t)(K + g) * bi.np[1] + (J + g)) * bi.np[0] + I;
  double* st = reg + (((int64_t)b * 2 + 0) * 2 + side) * 10 * rs;
  double* pr = reg + (((int64_t)b * 2 + 1) * 2 + side) * 10 * rs;
  const int o = K * rs2 + J;
  auto put = [&](int q, double v) {
    st[q * rs + o] = v;
    pr[q * rs + o] = first ? v : pr[q * rs + o] + v;
  };
  if (J < n2 && K < n3)
    for (int q = 0; q < 8; q++) put(q, dt * F[24 * bi.off + (int64_t)q * V + loc]);
  if (J < n2) put(8, dt * E[3 * bi.off + V + loc]);
  if (K < n3) put(9, dt * E[3 * bi.off + 2 * V + loc]);
}

// ------------------------------------------------------------------ reflux

// conserved state of the boundary-layer cells of each sync item, before the face
// corrections: U(P, B_old) plus the flux correction (mine - theirs)/dx1 * sign
__global__ __launch_bounds__(LT) void k_sync_u(Launch L, const SyncItem* __restrict__ items,
                                               const double* __restrict__ P,
                                               const double* __restrict__ B,
                                               const double* __restrict__ reg, int rs, int rs2,
                                               double* __restrict__ Ubuf, int layer) {
  const SyncItem it = items[blockIdx.y];
  const BlockInfo bi = L.blk[it.slow];
  const int g = L.ph.ng;
  const int t = blockIdx.x * LT + threadIdx.x;
  const int n2 = bi.n[1], n3 = bi.n[2];
  if (t >= n2 * n3) return;
  const int K = t / n2 + g, J = t % n2 + g;
  const int I = it.side == 0 ? g : g + bi.n[0] - 1;
  const int64_t V = bi.vol;
  const int64_t l = ((int64_t)K * bi.np[1] + J) * bi.np[0] + I;
  const int64_t s2 = bi.np[0], s3 = (int64_t)bi.np[0] * bi.np[1];
  const int64_t col = geo_col(L.geo, bi, J, I);
  const Metric m = load_metric(L.geo.c, L.geo.ncol, col);
  double p[5], bc[3], U[9];
  for (int v = 0; v < 5; v++) p[v] = P[5 * bi.off + v * V + l];
  const double* b = B + 3 * bi.off;
  bc[0] = 0.5 * (b[l] + b[l + 1]) / m.gdet;
  bc[1] = 0.5 * (b[V + l] + b[V + l + s2]) / m.gdet;
  bc[2] = 0.5 * (b[2 * V + l] + b[2 * V + l + s3]) / m.gdet;
  Fluid f;
  fluid_state(p, bc, m, f);
  flux_vector<0>(p, f, m, L.ph.gam, entropy_kappa(p, L.ph.gam), U);
  const double* mine = reg + (((int64_t)it.slow * 2 + 0) * 2 + it.side) * 10 * rs;
  const double* theirs = reg + (((int64_t)it.fast * 2 + 1) * 2 + (1 - it.side)) * 10 * rs;
  const int o = (K - g) * rs2 + (J - g);
  const double sgn = it.side == 1 ? 1.0 : -1.0;
  constexpr int fq[6] = {0, 1, 2, 3, 4, 7};
  constexpr int uq[6] = {0, 1, 2, 3, 4, 8};
  for (int k = 0; k < 6; k++)
    U[uq[k]] += (mine[fq[k] * rs + o] - theirs[fq[k] * rs + o]) / bi.dx[0] * sgn;
  double* u = Ubuf + ((int64_t)blockIdx.y * layer + t) * 9;
  for (int q = 0; q < 9; q++) u[q] = U[q];
}

// constrained-transport correction of the slow side's faces touching the shared edges,
// and the faster side's copy of the shared faces
__global__ __launch_bounds__(LT) void k_sync_faces(Launch L, const SyncItem* __restrict__ items,
                                                   double* __restrict__ B,
                                                   const double* __restrict__ reg, int rs,
                                                   int rs2) {
  const SyncItem it = items[blockIdx.y];
  const BlockInfo bi = L.blk[it.slow];
  const BlockInfo fi = L.blk[it.fast];
  const int g = L.ph.ng;
  const int t = blockIdx.x * LT + threadIdx.x;
  const int n2 = bi.n[1], n3 = bi.n[2];
  if (t >= (n2 + 1) * (n3 + 1)) return;
  const int kk = t / (n2 + 1), jj = t % (n2 + 1);
  const int K = kk + g, J = jj + g;
  const int Ic = it.side == 0 ? g : g + bi.n[0] - 1;
  const int If = it.side == 0 ? g : g + bi.n[0];
  const int Iff = it.side == 0 ? g + fi.n[0] : g;   // the same face in the faster block
  const int64_t V = bi.vol;
  const double sgn = it.side == 1 ? 1.0 : -1.0;
  const double* mine = reg + (((int64_t)it.slow * 2 + 0) * 2 + it.side) * 10 * rs;
  const double* theirs = reg + (((int64_t)it.fast * 2 + 1) * 2 + (1 - it.side)) * 10 * rs;
  const int o = kk * rs2 + jj;
  double* b = B + 3 * bi.off;
  const int64_t lc = ((int64_t)K * bi.np[1] + J) * bi.np[0] + Ic;
  if (kk < n3) {   // x2 faces of the layer, j in [g, g + n2]
    const double dE3 = theirs[9 * rs + o] - mine[9 * rs + o];
    b[V + lc] += sgn * dE3 / bi.dx[0];
  }
  if (jj < n2) {   // x3 faces of the layer, k in [g, g + n3]
    const double dE2 = theirs[8 * rs + o] - mine[8 * rs + o];
    b[2 * V + lc] -= sgn * dE2 / bi.dx[0];
  }
  if (kk < n3 && jj < n2) {
    const int64_t lf = ((int64_t)K * bi.np[1] + J) * bi.np[0] + If;
    const int64_t lff = ((int64_t)K * fi.np[1] + J) * fi.np[0] + Iff;
    b[lf] = B[3 * fi.off + lff];
  }
}

// new inversion of the corrected boundary-layer cells (guess: their primitives), floors
__global__ __launch_bounds__(LT) void k_sync_c2p(Launch L, const SyncItem* __restrict__ items,
                                                 double* __restrict__ P,
                                                 const double* __restrict__ B,
                                                 const double* __restrict__ Ubuf, int layer) {
  const SyncItem it = items[blockIdx.y];
  const BlockInfo bi = L.blk[it.slow];
  const int g = L.ph.ng;
  const int t = blockIdx.x * LT + threadIdx.x;
  const int n2 = bi.n[1], n3 = bi.n[2];
  const bool valid = t < n2 * n3;
  int tier = 0, hits = 0;
  if (valid) {
    const int K = t / n2 + g, J = t % n2 + g;
    const int I = it.side == 0 ? g : g + bi.n[0] - 1;
    const int64_t V = bi.vol;
    const int64_t l = ((int64_t)K * bi.np[1] + J) * bi.np[0] + I;
    const int64_t s2 = bi.np[0], s3 = (int64_t)bi.np[0] * bi.np[1];
    const int64_t col = geo_col(L.geo, bi, J, I);
    const Metric m = load_metric(L.geo.c, L.geo.ncol, col);
    double U[9], p[5];
    const double* u = Ubuf + ((int64_t)blockIdx.y * layer + t) * 9;
    for (int q = 0; q < 9; q++) U[q] = u[q];
    const double* b = B + 3 * bi.off;
    U[5] = 0.5 * (b[l] + b[l + 1]);
    U[6] = 0.5 * (b[V + l] + b[V + l + s2]);
    U[7] = 0.5 * (b[2 * V + l] + b[2 * V + l + s3]);
    for (int v = 0; v < 5; v++) p[v] = P[5 * bi.off + v * V + l];
    C2PIn cs;
    c2p_setup(U, m, L.ph.gam, cs);
    double Pn[5];
    int iters = 0;
    tier = c2p_solve(cs, m, false, 0.0, 0.0, p, L.ph.tol, L.ph.maxit, Pn, iters);
    const double Bn[3] = {U[5] / m.gdet, U[6] / m.gdet, U[7] / m.gdet};
    hits = apply_floors(Pn, Bn, m, L.geo.c[RHOFL * L.geo.ncol + col],
                        L.geo.c[UFL * L.geo.ncol + col], L.ph.bsq_rho_max, L.ph.bsq_u_max,
                        L.ph.gamma_max);
    for (int v = 0; v < 5; v++) P[5 * bi.off + v * V + l] = Pn[v];
  }
  // one counter add per distinct value per wave (every lane of the wave takes part)
  wave_count(L.cnt->tier, tier, valid);
  const long long h = wave_sum(valid ? hits : 0);
  if (lane_id() == 0 && h) atomicAdd(&L.cnt->floors, (unsigned long long)h);
}

// dt of a cycle: min over partials of the Courant step / 2^lat of the partial's block
__global__ __launch_bounds__(LT) void k_dt_final_lat(Counters* cnt, const double* __restrict__ part,
                                                     int64_t n, int gridx,
                                                     const BlockInfo* __restrict__ blk) {
  __shared__ double red[LT];
  double v = __longlong_as_double(0x7FF0000000000000LL);
  for (int64_t i = threadIdx.x; i < n; i += LT) {
    const int b = (int)(i / gridx);
    v = fmin(v, ldexp(part[i], -blk[b].lat));
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = LT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) cnt->dt_bits = (unsigned long long)__double_as_longlong(red[0]);
}

__global__ void k_tsim_cycle(Counters* cnt, double courant, double substeps) {
  if (threadIdx.x == 0) {
    const double dt = courant * __longlong_as_double((long long)cnt->dt_bits);
    cnt->t_sim += dt * substeps;
    cnt->dt_last = dt;
  }
}

// ================================================================== launchers

static inline unsigned cdv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

void launch_ghosts_t(const Launch& L, const GhostLists& G, const double* Pmain,
                     const double* Pold, const double* Pcur, double* Pdst, const double* Bmain,
                     const double* Bold, const double* Bcur, double* Bdst, double w) {
  if (G.end[3] == 0) return;
  hipLaunchKernelGGL(k_ghosts_t, dim3(cdv(G.end[3], LT)), dim3(LT), 0, L.stream, G, Pmain, Pold,
                     Pcur, Pdst, Bmain, Bold, Bcur, Bdst, w);
}

void launch_copy_blocks(const Launch& L, const double* src, double* dst, int nvar) {
  const int64_t r = (int64_t)(L.max_n[0] + 1) * (L.max_n[1] + 1) * (L.max_n[2] + 1);
  const unsigned gx = std::min<unsigned>(cdv(r, LT), 256);
  hipLaunchKernelGGL(k_copy_blocks, dim3(gx, L.nblk), dim3(LT), 0, L.stream, L, src, dst, nvar);
}

void launch_copy_list(const Launch& L, const uint32_t* ic, int64_t nc, const double* P,
                      double* Pdst, const uint32_t* jf, int64_t nf, const double* B,
                      double* Bdst) {
  if (nc + nf == 0) return;
  hipLaunchKernelGGL(k_copy_list, dim3(cdv(nc + nf, LT)), dim3(LT), 0, L.stream, ic, nc, P, Pdst,
                     jf, nf, B, Bdst);
}

void launch_registers(const Launch& L, const double* F, const double* E, double dt_factor,
                      int first, double* reg, int rs, int rs2) {
  const int64_t r = 2LL * (L.max_n[2] + 1) * (L.max_n[1] + 1);
  hipLaunchKernelGGL(k_registers, dim3(cdv(r, LT), L.nblk), dim3(LT), 0, L.stream, L, F, E,
                     dt_factor, first, reg, rs, rs2);
}

void launch_sync(const Launch& L, const SyncItem* items, int nitems, double* P, double* B,
                 const double* reg, int rs, int rs2, double* Ubuf) {
  if (nitems == 0) return;
  const int layer = L.max_n[1] * L.max_n[2];
  const int faces = (L.max_n[1] + 1) * (L.max_n[2] + 1);
  hipLaunchKernelGGL(k_sync_u, dim3(cdv(layer, LT), nitems), dim3(LT), 0, L.stream, L, items, P, B,
                     reg, rs, rs2, Ubuf, layer);
  hipLaunchKernelGGL(k_sync_faces, dim3(cdv(faces, LT), nitems), dim3(LT), 0, L.stream, L, items, B,
                     reg, rs, rs2);
  hipLaunchKernelGGL(k_sync_c2p, dim3(cdv(layer, LT), nitems), dim3(LT), 0, L.stream, L, items, P, B,
                     Ubuf, layer);
}

void launch_dt_final_lat(const Launch& L, const double* part, int64_t n, int gridx) {
  hipLaunchKernelGGL(k_dt_final_lat, dim3(1), dim3(LT), 0, L.stream, L.cnt, part, n, gridx, L.blk);
}

void launch_tsim_cycle(const Launch& L, double substeps) {
  hipLaunchKernelGGL(k_tsim_cycle, dim3(1), dim3(64), 0, L.stream, L.cnt, L.ph.courant, substeps);
}

}  // namespace grmhd
