// lat.hip -- kernels of local adaptive time-stepping (paper Sec. 3.5).
//
// Blocks carry a time level; a level-l block steps with dt_min 2^l.  The kernels here
// (1) fill ghosts whose sources run at another time level -- a slower neighbour is
//     interpolated linearly in time between its stored start state and its end state,
// (2) accumulate the time-integrated fluxes and edge EMFs that synchronisation reads
//     (listed elements on block boundaries), over a block's own step and over two of its
//     steps,
// (3) at the end of a slower block's step, replace the fluxes it used on faces shared
//     with a faster block by the faster side's time integrals (area means where the
//     faster side is finer), the EMFs of its edges whose dominant holder is faster by
//     that holder's integrals with constrained-transport correction of the faces around
//     them, give shared faces the faster copy, and invert every changed cell again.
// Time levels are independent of refinement levels and of the direction of a face.
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
    const GhostCF op = G.cf[t];
    const int fl = op.svol_fl >> 24, fc = op.dvol_fc >> 24;
    const int64_t svol = op.svol_fl & 0xFFFFFF, dvol = op.dvol_fc & 0xFFFFFF;
    double* out = Pdst + op.dp;
#pragma unroll
    for (int v = 0; v < 5; v++) {
      double x = timed_value(fl, op.sp + v * svol, Pmain, Pold, Pcur, w);
      if (v == 3 && (fl & GF_FLIP)) x = -x;
      if (v == 2 && (fl & GF_CLAMP_NEG) && x > 0.0) x = 0.0;
      if (v == 2 && (fl & GF_CLAMP_POS) && x < 0.0) x = 0.0;
      out[v * dvol] = x;
    }
#pragma unroll
    for (int c = 0; c < 3; c++)
      if ((fc >> c) & 1) Bdst[op.db + c * dvol] = timed_value(fl, op.sb + c * svol, Bmain, Bold, Bcur, w);
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

// One listed element per thread, from the corrector of a level's blocks: the dt-weighted
// face flux (six conserved components) or edge EMF, into the step set and the pair set
// (restarted when `first` is set, else summed).
__global__ __launch_bounds__(LT) void k_registers(const RegItem* __restrict__ items, int64_t n,
                                                  const double* __restrict__ F,
                                                  const double* __restrict__ E, double dt_factor,
                                                  double courant, const Counters* __restrict__ cnt,
                                                  int first, double* __restrict__ regF, int64_t nf,
                                                  double* __restrict__ regE, int64_t ne) {
  const int64_t t = (int64_t)blockIdx.x * LT + threadIdx.x;
  if (t >= n) return;
  const RegItem it = items[t];
  const double dt = dt_factor * courant * __longlong_as_double((long long)cnt->dt_bits);
  if (it.kind == 0) {
    constexpr int fq[6] = {0, 1, 2, 3, 4, 7};
#pragma unroll
    for (int q = 0; q < 6; q++) {
      const double v = dt * F[it.src + (int64_t)fq[q] * it.stride];
      const int64_t o = (int64_t)q * nf + it.slot;
      regF[o] = v;
      regF[6 * nf + o] = first ? v : regF[6 * nf + o] + v;
    }
  } else {
    const double v = dt * E[it.src];
    regE[it.slot] = v;
    regE[ne + it.slot] = first ? v : regE[ne + it.slot] + v;
  }
}

// ------------------------------------------------------------------ synchronisation

__device__ __forceinline__ int64_t cell_stride(const BlockInfo& bi, int d) {
  return d == 0 ? 1 : (d == 1 ? (int64_t)bi.np[0] : (int64_t)bi.np[0] * bi.np[1]);
}

// Conserved state of each listed cell before its faces change: U(P, B) plus the flux
// corrections (mine - mean(theirs)) / dx * sgn summed over the cell's terms.
__global__ __launch_bounds__(LT) void k_sync_u(Launch L, const SyncCell* __restrict__ cells,
                                               int64_t ncell, const double* __restrict__ P,
                                               const double* __restrict__ B,
                                               const double* __restrict__ regF, int64_t nf,
                                               double* __restrict__ Ubuf) {
  const int64_t t = (int64_t)blockIdx.x * LT + threadIdx.x;
  if (t >= ncell) return;
  const SyncCell sc = cells[t];
  const BlockInfo bi = L.blk[sc.blk];
  const int64_t V = bi.vol;
  const int64_t l = sc.loc;
  const int I = (int)(l % bi.np[0]);
  const int J = (int)((l / bi.np[0]) % bi.np[1]);
  const int64_t col = geo_col(L.geo, bi, J, I);
  const Metric m = load_metric(L.geo.c, L.geo.ncol, col);
  double p[5], bc[3], U[9];
  for (int v = 0; v < 5; v++) p[v] = P[5 * bi.off + v * V + l];
  const double* b = B + 3 * bi.off;
  bc[0] = 0.5 * (b[l] + b[l + 1]) / m.gdet;
  bc[1] = 0.5 * (b[V + l] + b[V + l + cell_stride(bi, 1)]) / m.gdet;
  bc[2] = 0.5 * (b[2 * V + l] + b[2 * V + l + cell_stride(bi, 2)]) / m.gdet;
  Fluid f;
  fluid_state(p, bc, m, f);
  flux_vector<0>(p, f, m, L.ph.gam, entropy_kappa(p, L.ph.gam), U);
  constexpr int uq[6] = {0, 1, 2, 3, 4, 8};
  double dU[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < sc.nt; k++) {
    const FluxTerm ft = sc.t[k];
    const double inv = 1.0 / ft.nth;
    const double sg = ft.sgn > 0 ? 1.0 : -1.0;
    for (int q = 0; q < 6; q++) {
      double th = 0.0;
      for (int i = 0; i < ft.nth; i++) th = th + regF[6 * nf + (int64_t)q * nf + ft.th[i]];
      th = th * inv;
      dU[q] = dU[q] + (regF[(int64_t)q * nf + ft.mine] - th) / ft.dx * sg;
    }
  }
  for (int q = 0; q < 6; q++) U[uq[q]] += dU[q];
  double* u = Ubuf + t * 9;
  for (int q = 0; q < 9; q++) u[q] = U[q];
}

// New values of the listed faces: the faster block's copy of a shared face, else the
// face plus the constrained-transport corrections sgn (mean(theirs) - mine) / dx of its
// edges.  Every face is listed once and no item reads a face another item writes.
__global__ __launch_bounds__(LT) void k_sync_faces(Launch L, const SyncFace* __restrict__ faces,
                                                   int64_t nface, double* __restrict__ B,
                                                   const double* __restrict__ regE, int64_t ne) {
  const int64_t t = (int64_t)blockIdx.x * LT + threadIdx.x;
  if (t >= nface) return;
  const SyncFace sf = faces[t];
  const BlockInfo bi = L.blk[sf.blk];
  double* dst = B + 3 * bi.off + (int64_t)sf.comp * bi.vol + sf.loc;
  if (sf.ncopy > 0) {
    const BlockInfo ci = L.blk[sf.cblk];
    const double* src = B + 3 * ci.off + (int64_t)sf.comp * ci.vol;
    double acc = 0.0;
    for (int i = 0; i < sf.ncopy; i++) acc = acc + src[sf.csrc[i]];
    *dst = acc * (1.0 / sf.ncopy);
    return;
  }
  double x = *dst;
  for (int k = 0; k < sf.nt; k++) {
    const EdgeTerm et = sf.t[k];
    double th = 0.0;
    for (int i = 0; i < et.nth; i++) th = th + regE[ne + et.th[i]];
    th = th * (1.0 / et.nth);
    const double dE = th - regE[et.mine];
    x += (et.sgn > 0 ? dE : -dE) / et.dx;
  }
  *dst = x;
}

// New inversion of the listed cells (guess: their primitives) from the corrected
// conserved state and the corrected faces, then floors.
template <bool DRIFT>
__global__ __launch_bounds__(LT) void k_sync_c2p(Launch L, const SyncCell* __restrict__ cells,
                                                 int64_t ncell, double* __restrict__ P,
                                                 const double* __restrict__ B,
                                                 const double* __restrict__ Ubuf) {
  const int64_t t = (int64_t)blockIdx.x * LT + threadIdx.x;
  const bool valid = t < ncell;
  int tier = 0, hits = 0;
  if (valid) {
    const SyncCell sc = cells[t];
    const BlockInfo bi = L.blk[sc.blk];
    const int64_t V = bi.vol;
    const int64_t l = sc.loc;
    const int I = (int)(l % bi.np[0]);
    const int J = (int)((l / bi.np[0]) % bi.np[1]);
    const int64_t col = geo_col(L.geo, bi, J, I);
    const Metric m = load_metric(L.geo.c, L.geo.ncol, col);
    double U[9], p[5];
    const double* u = Ubuf + t * 9;
    for (int q = 0; q < 9; q++) U[q] = u[q];
    const double* b = B + 3 * bi.off;
    U[5] = 0.5 * (b[l] + b[l + 1]);
    U[6] = 0.5 * (b[V + l] + b[V + l + cell_stride(bi, 1)]);
    U[7] = 0.5 * (b[2 * V + l] + b[2 * V + l + cell_stride(bi, 2)]);
    for (int v = 0; v < 5; v++) p[v] = P[5 * bi.off + v * V + l];
    C2PIn cs;
    c2p_setup(U, m, L.ph.gam, cs);
    double Pn[5];
    int iters = 0;
    tier = c2p_solve(cs, m, false, 0.0, 0.0, p, L.ph.tol, L.ph.maxit, Pn, iters);
    const double Bn[3] = {U[5] / m.gdet, U[6] / m.gdet, U[7] / m.gdet};
    const double rfl = L.geo.c[RHOFL * L.geo.ncol + col], ufl = L.geo.c[UFL * L.geo.ncol + col];
    hits = DRIFT ? drift_floors(Pn, Bn, m, rfl, ufl, L.ph.bsq_rho_max, L.ph.bsq_u_max,
                                L.ph.gamma_max, L.ph.gam, L.ph.tol, L.ph.maxit)
                 : apply_floors(Pn, Bn, m, rfl, ufl, L.ph.bsq_rho_max, L.ph.bsq_u_max,
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
                                                     const BlockInfo* __restrict__ blk,
                                                     const int2* __restrict__ wl) {
  __shared__ double red[LT];
  double v = __longlong_as_double(0x7FF0000000000000LL);
  for (int64_t i = threadIdx.x; i < n; i += LT) {
    const int b = wl ? wl[i].x : (int)(i / gridx);
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

void launch_registers(const Launch& L, const RegItem* items, int64_t n, const double* F,
                      const double* E, double dt_factor, int first, double* regF, int64_t nf,
                      double* regE, int64_t ne) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_registers, dim3(cdv(n, LT)), dim3(LT), 0, L.stream, items, n, F, E,
                     dt_factor, L.ph.courant, L.cnt, first, regF, nf, regE, ne);
}

void launch_sync(const Launch& L, const SyncCell* cells, int64_t ncell, const SyncFace* faces,
                 int64_t nface, double* P, double* B, const double* regF, int64_t nf,
                 const double* regE, int64_t ne, double* Ubuf) {
  if (ncell + nface == 0) return;
  if (ncell > 0)
    hipLaunchKernelGGL(k_sync_u, dim3(cdv(ncell, LT)), dim3(LT), 0, L.stream, L, cells, ncell, P,
                       B, regF, nf, Ubuf);
  if (nface > 0)
    hipLaunchKernelGGL(k_sync_faces, dim3(cdv(nface, LT)), dim3(LT), 0, L.stream, L, faces, nface,
                       B, regE, ne);
  if (ncell > 0) {
    if (L.ph.floor_drift)
      hipLaunchKernelGGL(k_sync_c2p<true>, dim3(cdv(ncell, LT)), dim3(LT), 0, L.stream, L, cells,
                         ncell, P, B, Ubuf);
    else
      hipLaunchKernelGGL(k_sync_c2p<false>, dim3(cdv(ncell, LT)), dim3(LT), 0, L.stream, L, cells,
                         ncell, P, B, Ubuf);
  }
}

void launch_dt_final_lat(const Launch& L, const double* part, int64_t n, int gridx,
                         const int2* wl) {
  hipLaunchKernelGGL(k_dt_final_lat, dim3(1), dim3(LT), 0, L.stream, L.cnt, part, n, gridx, L.blk,
                     wl);
}

void launch_tsim_cycle(const Launch& L, double substeps) {
  hipLaunchKernelGGL(k_tsim_cycle, dim3(1), dim3(64), 0, L.stream, L.cnt, L.ph.courant, substeps);
}

}  // namespace grmhd
