// amr.hip -- kernels of static mesh refinement (paper Sec. 3.3; the per-direction
// coarsening toward the poles of Sec. 3.4 is the same machinery with refinement in some
// dimensions only).
//
// Blocks carry a refinement level per dimension, and neighbours differ by at most one
// level.  The kernels here
// (1) fill ghost values that come from another level: a coarse ghost is the
//     restriction of the finer neighbour (sqrt(-g)-weighted mean of the primitives of
//     the covered fine cells; arithmetic mean of the fine sub-faces of a face), a fine
//     ghost the minmod-limited linear prolongation of the coarser neighbour's values
//     (slopes from the parent's neighbours at its own level, child = parent +-
//     slope/4 per refined dimension; a fine face that cuts a coarse cell in two takes
//     the mean of the prolonged values on the two coarse faces bounding that cell);
// (2) within a time level, make the coarse side of every refinement face use the fine
//     side's fluxes (area means) and every edge the EMF of its finest holder (edge
//     means), so both sides change the conserved totals and the face field by the same
//     amount;
// (3) after each update, give the coarse copy of every shared face the mean of the
//     fine faces, the finer side owning shared faces.
// Across time levels the same corrections happen at the end of the slower block's step
// from time-integrated registers (lat.hip).
// Each value is read from the source block's state as the viewing block sees it at its
// stage time (the time-level rules of local time stepping, as for plain copies).
#include <hip/hip_runtime.h>

#include "device.h"
#include "internal.h"

namespace grmhd {

constexpr int AT = 256;

__device__ __forceinline__ double minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return fmin(a, b);
  if (a < 0.0 && b < 0.0) return fmax(a, b);
  return 0.0;
}

// a value of the source state at index q, by the time relation of its block
__device__ __forceinline__ double timed(int fl, int64_t q, const double* __restrict__ main,
                                        const double* __restrict__ old,
                                        const double* __restrict__ cur, double w) {
  if (fl & GF_SLOW) return old[q] + w * (main[q] - old[q]);
  if (fl & GF_FAST) return main[q];
  return cur[q];
}

// The five primitives of one cell sample (a cell of the source block, or for a
// restriction the sqrt(-g)-weighted mean of the finer cells it covers), then the
// physical-boundary flip and clamps.  The sample's block record, indices and weights are
// decoded once for all five variables.
__device__ __forceinline__ void cell_values(const BlockInfo* __restrict__ blk, const GeoTab& G,
                            const AmrSample& s, const double* __restrict__ main,
                            const double* __restrict__ old, const double* __restrict__ cur,
                            double w, double x[5]) {
  const int sb = s.blkf & 0xFFFFFF, fl = (s.blkf >> 24) & 0xFF;
  const BlockInfo bi = blk[sb];
  const int64_t base = 5 * bi.off + s.loc;
  if (s.mask == 0) {
#pragma unroll
    for (int v = 0; v < 5; v++) x[v] = timed(fl, base + (int64_t)v * bi.vol, main, old, cur, w);
  } else {
    // the covered fine cells in (k, j, i) order (i fastest), their offsets and weights;
    // entry m = 4 ok + 2 oj + oi, present where the mask refines its dimensions
    int64_t off[8];
    double wg[8];
    double den = 0.0;
#pragma unroll
    for (int m = 0; m < 8; m++) {
      const int oi = m & 1, oj = (m >> 1) & 1, ok = m >> 2;
      const bool in = (!oi || (s.mask & 1)) && (!oj || (s.mask & 2)) && (!ok || (s.mask & 4));
      off[m] = ((int64_t)ok * bi.np[1] + oj) * bi.np[0] + oi;
      wg[m] = 0.0;
      if (in) {
        const int64_t l = s.loc + off[m];
        const int I = (int)(l % bi.np[0]), J = (int)((l / bi.np[0]) % bi.np[1]);
        wg[m] = G.c[GDET * G.ncol + geo_col(G, bi, J, I)];
        den = __dadd_rn(den, wg[m]);
      }
    }
#pragma unroll
    for (int v = 0; v < 5; v++) {
      const int64_t bv = base + (int64_t)v * bi.vol;
      double num = 0.0;
#pragma unroll
      for (int m = 0; m < 8; m++) {
        const int oi = m & 1, oj = (m >> 1) & 1, ok = m >> 2;
        const bool in = (!oi || (s.mask & 1)) && (!oj || (s.mask & 2)) && (!ok || (s.mask & 4));
        if (in) num = __dadd_rn(num, __dmul_rn(wg[m], timed(fl, bv + off[m], main, old, cur, w)));
      }
      x[v] = num / den;
    }
  }
  if (fl & GF_FLIP) x[3] = -x[3];
  if ((fl & GF_CLAMP_NEG) && x[2] > 0.0) x[2] = 0.0;
  if ((fl & GF_CLAMP_POS) && x[2] < 0.0) x[2] = 0.0;
}

__device__ double face_value(const BlockInfo* __restrict__ blk, const AmrSample& s, int comp,
                             const double* __restrict__ main, const double* __restrict__ old,
                             const double* __restrict__ cur, double w) {
  const int sb = s.blkf & 0xFFFFFF, fl = (s.blkf >> 24) & 0xFF;
  if (fl & GF_ZERO) return 0.0;
  const BlockInfo bi = blk[sb];
  const int64_t base = 3 * bi.off + (int64_t)comp * bi.vol;
  double x;
  if (s.mask == 0) {
    x = timed(fl, base + s.loc, main, old, cur, w);
  } else {
    const int n0 = (s.mask & 1) ? 2 : 1, n1 = (s.mask & 2) ? 2 : 1, n2 = (s.mask & 4) ? 2 : 1;
    double acc = 0.0;
    for (int ok = 0; ok < n2; ok++)
      for (int oj = 0; oj < n1; oj++)
        for (int oi = 0; oi < n0; oi++)
          acc += timed(fl, base + s.loc + ((int64_t)ok * bi.np[1] + oj) * bi.np[0] + oi, main,
                       old, cur, w);
    x = acc * (1.0 / (n0 * n1 * n2));
  }
  if (fl & GF_FLIP) x = -x;
  return x;
}

// a ghost cell from its refinement stencil (prolongation with minmod slopes, or a
// restriction sample), then the physical-boundary flip and clamps; per variable the
// same operations in the same order as one variable at a time
__device__ void amr_cell_op(const BlockInfo* __restrict__ blk, const GeoTab& G, const AmrOp op,
                            const AmrSample* __restrict__ samp, const double* __restrict__ main,
                            const double* __restrict__ old, const double* __restrict__ cur,
                            double w, double* __restrict__ dst) {
  const AmrSample* S = samp + op.samp;
  const int pd = op.mode & AM_PDIMS;
  const int ofl = (op.mode >> AM_FLAGS_SHIFT) & 0xFF;
  double c[5], x[5];
  cell_values(blk, G, S[0], main, old, cur, w, c);
#pragma unroll
  for (int v = 0; v < 5; v++) x[v] = c[v];
  int k = 1;
  for (int dd = 0; dd < 3; dd++) {
    if (!((pd >> dd) & 1)) continue;
    double sm[5], sp[5];
    cell_values(blk, G, S[k], main, old, cur, w, sm);
    cell_values(blk, G, S[k + 1], main, old, cur, w, sp);
    k += 2;
    const double sg = ((op.mode >> (AM_UPPER_SHIFT + dd)) & 1) ? 0.25 : -0.25;
#pragma unroll
    for (int v = 0; v < 5; v++) x[v] = x[v] + sg * minmod(c[v] - sm[v], sp[v] - c[v]);
  }
  if (ofl & GF_FLIP) x[3] = -x[3];
  if ((ofl & GF_CLAMP_NEG) && x[2] > 0.0) x[2] = 0.0;
  if ((ofl & GF_CLAMP_POS) && x[2] < 0.0) x[2] = 0.0;
  const BlockInfo d = blk[op.dst_blk];
  double* o = dst + 5 * d.off + op.dst_loc;
#pragma unroll
  for (int v = 0; v < 5; v++) o[(int64_t)v * d.vol] = x[v];
}

// a ghost face of component comp from its refinement stencil (the mean of two stencils
// for a face cutting a coarse cell), then the flip or the axis zero
__device__ void amr_face_op(const BlockInfo* __restrict__ blk, const AmrOp op,
                            const AmrSample* __restrict__ samp, const double* __restrict__ main,
                            const double* __restrict__ old, const double* __restrict__ cur,
                            double w, double* __restrict__ dst, int comp) {
  const BlockInfo d = blk[op.dst_blk];
  const AmrSample* S = samp + op.samp;
  const int t = op.mode & AM_PDIMS & ~(1 << comp);
  const int ofl = (op.mode >> AM_FLAGS_SHIFT) & 0xFF;
  const int nst = 1 + 2 * __popc(t);
  double st[2];
  const int ns = (op.mode & AM_TWO) ? 2 : 1;
  for (int q = 0; q < ns; q++) {
    const AmrSample* R = S + q * nst;
    const double c = face_value(blk, R[0], comp, main, old, cur, w);
    double x = c;
    int k = 1;
    for (int dd = 0; dd < 3; dd++) {
      if (!((t >> dd) & 1)) continue;
      const double sm = face_value(blk, R[k], comp, main, old, cur, w);
      const double sp = face_value(blk, R[k + 1], comp, main, old, cur, w);
      k += 2;
      const double sg = ((op.mode >> (AM_UPPER_SHIFT + dd)) & 1) ? 0.25 : -0.25;
      x = x + sg * minmod(c - sm, sp - c);
    }
    st[q] = x;
  }
  double x = ns == 2 ? 0.5 * (st[0] + st[1]) : st[0];
  if (ofl & GF_ZERO) x = 0.0;
  else if (ofl & GF_FLIP) x = -x;
  dst[3 * d.off + (int64_t)comp * d.vol + op.dst_loc] = x;
}

// One thread per entry of the concatenated refinement lists (cells, then faces of
// components 1..3).  With old == main and w = 0 slower sources read the main state.
__global__ __launch_bounds__(AT) void k_amr_ghosts(const BlockInfo* __restrict__ blk, GeoTab G,
                                                   AmrLists A, const AmrSample* __restrict__ samp,
                                                   const double* __restrict__ Pmain,
                                                   const double* __restrict__ Pold,
                                                   const double* __restrict__ Pcur,
                                                   double* __restrict__ Pdst,
                                                   const double* __restrict__ Bmain,
                                                   const double* __restrict__ Bold,
                                                   const double* __restrict__ Bcur,
                                                   double* __restrict__ Bdst, double w) {
  const int64_t t = (int64_t)blockIdx.x * AT + threadIdx.x;
  if (t >= A.end[3]) return;
  if (t < A.end[0]) {
    amr_cell_op(blk, G, A.ops[0][t], samp, Pmain, Pold, Pcur, w, Pdst);
    return;
  }
  const int k = t < A.end[1] ? 1 : (t < A.end[2] ? 2 : 3);
  amr_face_op(blk, A.ops[k][t - A.end[k - 1]], samp, Bmain, Bold, Bcur, w, Bdst, k - 1);
}

// ------------------------------------------------------------------ refinement faces

// One item per thread: the mean of the item's sources, per component.  Fluxes of a
// refinement face take the area mean of the finer block's fluxes, EMFs the finest
// holder's (the mean of its two sub-edges where it is finer along the edge), coarse
// copies of shared faces the mean of the fine faces.
__global__ __launch_bounds__(AT) void k_means(const MeanItem* __restrict__ items, int64_t n,
                                              double* __restrict__ X0, double* __restrict__ X1) {
  const int64_t t = (int64_t)blockIdx.x * AT + threadIdx.x;
  if (t >= n) return;
  const MeanItem it = items[t];
  double* X = it.kind == 0 ? X0 : X1;
  const double inv = 1.0 / it.n;
  for (int q = 0; q < it.ncomp; q++) {
    double acc = 0.0;
    for (int i = 0; i < it.n; i++) acc = acc + X[it.src[i] + (int64_t)q * it.sstride];
    X[it.dst + (int64_t)q * it.dstride] = acc * inv;
  }
}

// ------------------------------------------------------------------ launchers

// Without a stored start state (a gather outside a time-stepping cycle, where every
// block stands at the same time) samples flagged as slower read the main state too.
void launch_amr_ghosts(const Launch& L, const AmrLists& A, const AmrSample* samp,
                       const double* Pmain, const double* Pold, const double* Pcur, double* Pdst,
                       const double* Bmain, const double* Bold, const double* Bcur, double* Bdst,
                       double w) {
  if (A.end[3] <= 0) return;
  if (!Pold || !Bold) {
    Pold = Pmain;
    Bold = Bmain;
    w = 0.0;
  }
  k_amr_ghosts<<<dim3((unsigned)((A.end[3] + AT - 1) / AT)), dim3(AT), 0, L.stream>>>(
      L.blk, L.geo, A, samp, Pmain, Pold, Pcur, Pdst, Bmain, Bold, Bcur, Bdst, w);
}

void launch_means(const Launch& L, const MeanItem* items, int64_t n, double* X0, double* X1) {
  if (n <= 0) return;
  k_means<<<dim3((unsigned)((n + AT - 1) / AT)), dim3(AT), 0, L.stream>>>(items, n, X0, X1);
}

// ------------------------------------------------------------------ regrid
// A new block layout filled from an old one (Sec. 3.3 refinement and derefinement; the
// face field of new fine blocks by Balsara's 2001 divergence-free reconstruction).  Each
// thread writes one interior cell (five primitives) or one face of a new block, reading
// the old block that covers it in its padded arrays, ghosts included.

// the box holding item t of a list (start: nops + 1 ascending offsets)
__device__ __forceinline__ int regrid_box(const int64_t* __restrict__ start, int64_t nops,
                                          int64_t t) {
  int64_t lo = 0, hi = nops - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (start[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return (int)lo;
}

struct OldBlock {
  BlockInfo bi;
  int ng;
  int o[3];
  // element index in the padded arrays of global indices g (at the block's levels)
  __device__ __forceinline__ int64_t at(int g0, int g1, int g2) const {
    return ((int64_t)(g2 - o[2] + ng) * bi.np[1] + (g1 - o[1] + ng)) * bi.np[0] + (g0 - o[0] + ng);
  }
};

__device__ __forceinline__ OldBlock old_block(const BlockInfo* __restrict__ blk, const RegridOp& op) {
  OldBlock b;
  b.bi = blk[op.ob];
  b.ng = (b.bi.np[0] - b.bi.n[0] - 1) / 2;
  b.o[0] = op.oo[0];
  b.o[1] = op.oo[1];
  b.o[2] = op.oo[2];
  return b;
}

__global__ void __launch_bounds__(AT) k_regrid_cells(const BlockInfo* __restrict__ bf,
                                                     const BlockInfo* __restrict__ bt, GeoTab G,
                                                     const RegridOp* __restrict__ ops, int64_t nops,
                                                     const int64_t* __restrict__ start,
                                                     int64_t total, const double* __restrict__ Pf,
                                                     double* __restrict__ Pt) {
  const int64_t t = (int64_t)blockIdx.x * AT + threadIdx.x;
  if (t >= total) return;
  const int k = regrid_box(start, nops, t);
  const RegridOp op = ops[k];
  const int64_t q = t - start[k];
  int l[3];
  l[0] = op.lo[0] + (int)(q % op.ext[0]);
  l[1] = op.lo[1] + (int)((q / op.ext[0]) % op.ext[1]);
  l[2] = op.lo[2] + (int)(q / ((int64_t)op.ext[0] * op.ext[1]));
  const int gc[3] = {op.on[0] + l[0], op.on[1] + l[1], op.on[2] + l[2]};
  const BlockInfo bn = bt[op.nb];
  const int ngn = (bn.np[0] - bn.n[0] - 1) / 2;
  const int64_t dst = 5 * bn.off + ((int64_t)(l[2] + ngn) * bn.np[1] + (l[1] + ngn)) * bn.np[0] + (l[0] + ngn);
  const OldBlock ob = old_block(bf, op);
  const int64_t base = 5 * ob.bi.off;
  const int rmin = min(op.r[0], min(op.r[1], op.r[2]));
  const int rmax = max(op.r[0], max(op.r[1], op.r[2]));
  double val[5];
  if (rmin == 0 && rmax == 0) {
    const int64_t s = ob.at(gc[0], gc[1], gc[2]);
#pragma unroll
    for (int v = 0; v < 5; v++) val[v] = Pf[base + (int64_t)v * ob.bi.vol + s];
  } else if (rmax <= 0) {
    // sqrt(-g)-weighted mean of the covered fine cells, k outermost, i innermost
    double num[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, den = 0.0;
    const int n0 = op.r[0] < 0 ? 2 : 1, n1 = op.r[1] < 0 ? 2 : 1, n2 = op.r[2] < 0 ? 2 : 1;
    for (int ok = 0; ok < n2; ok++)
      for (int oj = 0; oj < n1; oj++)
        for (int oi = 0; oi < n0; oi++) {
          const int f0 = (gc[0] << (-op.r[0])) + oi, f1 = (gc[1] << (-op.r[1])) + oj,
                    f2 = (gc[2] << (-op.r[2])) + ok;
          const int64_t s = ob.at(f0, f1, f2);
          const double w = G.c[GDET * G.ncol + geo_col(G, ob.bi, f1 - ob.o[1] + ob.ng, f0 - ob.o[0] + ob.ng)];
#pragma unroll
          for (int v = 0; v < 5; v++)
            num[v] = __dadd_rn(num[v], __dmul_rn(w, Pf[base + (int64_t)v * ob.bi.vol + s]));
          den = __dadd_rn(den, w);
        }
#pragma unroll
    for (int v = 0; v < 5; v++) val[v] = num[v] / den;
  } else {
    // parent plus +-1/4 of the minmod slope per refined dimension
    const int pc[3] = {gc[0] >> op.r[0], gc[1] >> op.r[1], gc[2] >> op.r[2]};
    const int64_t s0 = ob.at(pc[0], pc[1], pc[2]);
    int64_t sm[3], sp[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
      int a[3] = {pc[0], pc[1], pc[2]};
      a[d] -= 1;
      sm[d] = ob.at(a[0], a[1], a[2]);
      a[d] += 2;
      sp[d] = ob.at(a[0], a[1], a[2]);
    }
#pragma unroll
    for (int v = 0; v < 5; v++) {
      const double* X = Pf + base + (int64_t)v * ob.bi.vol;
      const double c0 = X[s0];
      double x = c0;
#pragma unroll
      for (int d = 0; d < 3; d++) {
        if (!op.r[d]) continue;
        const double tw = (gc[d] & 1) ? 0.25 : -0.25;
        x = __dadd_rn(x, __dmul_rn(tw, minmod(__dsub_rn(c0, X[sm[d]]), __dsub_rn(X[sp[d]], c0))));
      }
      val[v] = x;
    }
  }
#pragma unroll
  for (int v = 0; v < 5; v++) Pt[dst + (int64_t)v * bn.vol] = val[v];
}

// Conserved form: U (the conserved vector of the update) of an old cell from its
// primitives and cell-centred field, with its sqrt(-g)
__device__ __forceinline__ double old_conserved(const OldBlock& ob, const GeoTab& G,
                                                const double* __restrict__ Pf,
                                                const double* __restrict__ Bf, const int g[3],
                                                double gam, double U[9]) {
  const int64_t s = ob.at(g[0], g[1], g[2]);
  const Metric m = load_metric(G.c, G.ncol, geo_col(G, ob.bi, g[1] - ob.o[1] + ob.ng, g[0] - ob.o[0] + ob.ng));
  double P[5], B[3];
#pragma unroll
  for (int v = 0; v < 5; v++) P[v] = Pf[5 * ob.bi.off + (int64_t)v * ob.bi.vol + s];
  const int64_t st[3] = {1, ob.bi.np[0], (int64_t)ob.bi.np[0] * ob.bi.np[1]};
#pragma unroll
  for (int d = 0; d < 3; d++) {
    const double* X = Bf + 3 * ob.bi.off + (int64_t)d * ob.bi.vol;
    B[d] = 0.5 * (X[s] + X[s + st[d]]) / m.gdet;
  }
  Fluid f;
  fluid_state(P, B, m, f);
  flux_vector<0>(P, f, m, gam, entropy_kappa(P, gam), U);
  return m.gdet;
}

// Restricted or prolonged cells of the conserved form: the mean of the covered cells' U,
// or the parent's densities U / sqrt(-g) plus +-1/4 of their minmod slopes, moved by one
// common amount in all children of the parent so that their U (densities times the
// child's sqrt(-g)) sum to the parent's U; the cell field from the new faces (already
// written); then the inversion,
// started from the primitive form's value, and the floors of the new grid.
__global__ void __launch_bounds__(AT) k_regrid_cells_cons(
    const BlockInfo* __restrict__ bf, const BlockInfo* __restrict__ bt, GeoTab Gf, GeoTab Gt,
    Phys ph, const RegridOp* __restrict__ ops, int64_t nops, const int64_t* __restrict__ start,
    int64_t total, const double* __restrict__ Pf, const double* __restrict__ Bf,
    double* __restrict__ Pt, const double* __restrict__ Bt) {
  const int64_t t = (int64_t)blockIdx.x * AT + threadIdx.x;
  if (t >= total) return;
  const int k = regrid_box(start, nops, t);
  const RegridOp op = ops[k];
  const int rmin = min(op.r[0], min(op.r[1], op.r[2]));
  const int rmax = max(op.r[0], max(op.r[1], op.r[2]));
  if (rmin == 0 && rmax == 0) return;   // copied cells: the primitive pass has them
  const int64_t q = t - start[k];
  int l[3];
  l[0] = op.lo[0] + (int)(q % op.ext[0]);
  l[1] = op.lo[1] + (int)((q / op.ext[0]) % op.ext[1]);
  l[2] = op.lo[2] + (int)(q / ((int64_t)op.ext[0] * op.ext[1]));
  const int gc[3] = {op.on[0] + l[0], op.on[1] + l[1], op.on[2] + l[2]};
  const BlockInfo bn = bt[op.nb];
  const int ngn = (bn.np[0] - bn.n[0] - 1) / 2;
  const int64_t loc = ((int64_t)(l[2] + ngn) * bn.np[1] + (l[1] + ngn)) * bn.np[0] + (l[0] + ngn);
  const OldBlock ob = old_block(bf, op);
  const double gam = ph.gam;
  double U[9];
  if (rmax <= 0) {
    double acc[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int n0 = op.r[0] < 0 ? 2 : 1, n1 = op.r[1] < 0 ? 2 : 1, n2 = op.r[2] < 0 ? 2 : 1;
    for (int ok = 0; ok < n2; ok++)
      for (int oj = 0; oj < n1; oj++)
        for (int oi = 0; oi < n0; oi++) {
          const int f[3] = {(gc[0] << (-op.r[0])) + oi, (gc[1] << (-op.r[1])) + oj,
                            (gc[2] << (-op.r[2])) + ok};
          double Us[9];
          old_conserved(ob, Gf, Pf, Bf, f, gam, Us);
#pragma unroll
          for (int v = 0; v < 9; v++) acc[v] = __dadd_rn(acc[v], Us[v]);
        }
    const double w = 1.0 / (n0 * n1 * n2);
#pragma unroll
    for (int v = 0; v < 9; v++) U[v] = __dmul_rn(acc[v], w);
  } else {
    const int pc[3] = {gc[0] >> op.r[0], gc[1] >> op.r[1], gc[2] >> op.r[2]};
    double U0[9], q0[9], sl[3][9];
    const double g0 = old_conserved(ob, Gf, Pf, Bf, pc, gam, U0);
#pragma unroll
    for (int v = 0; v < 9; v++) q0[v] = U0[v] / g0;
    for (int d = 0; d < 3; d++) {
#pragma unroll
      for (int v = 0; v < 9; v++) sl[d][v] = 0.0;
      if (!op.r[d]) continue;
      int a[3] = {pc[0], pc[1], pc[2]};
      a[d] -= 1;
      double Um[9], Up[9];
      const double gm = old_conserved(ob, Gf, Pf, Bf, a, gam, Um);
      a[d] += 2;
      const double gp = old_conserved(ob, Gf, Pf, Bf, a, gam, Up);
#pragma unroll
      for (int v = 0; v < 9; v++)
        sl[d][v] = minmod(__dsub_rn(q0[v], Um[v] / gm), __dsub_rn(Up[v] / gp, q0[v]));
    }
    // one child's U from its global cell index (its sqrt(-g) from the new grid's table)
    auto gdet_at = [&](const int c3[3]) {
      const int J = c3[1] - op.on[1] + ngn, I = c3[0] - op.on[0] + ngn;
      return Gt.c[GDET * Gt.ncol + geo_col(Gt, bn, J, I)];
    };
    auto child = [&](const int c3[3], double gd, double out[9]) {
#pragma unroll
      for (int v = 0; v < 9; v++) {
        double x = q0[v];
        for (int d = 0; d < 3; d++)
          if (op.r[d]) x = __dadd_rn(x, __dmul_rn((c3[d] & 1) ? 0.25 : -0.25, sl[d][v]));
        out[v] = __dmul_rn(gd, x);
      }
    };
    // the children's densities move by one common amount dq so that their U sum to the
    // parent's U times their number
    double acc[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, gsum = 0.0;
    const int n0 = op.r[0] ? 2 : 1, n1 = op.r[1] ? 2 : 1, n2 = op.r[2] ? 2 : 1;
    for (int ok = 0; ok < n2; ok++)
      for (int oj = 0; oj < n1; oj++)
        for (int oi = 0; oi < n0; oi++) {
          const int c3[3] = {(pc[0] << op.r[0]) + oi, (pc[1] << op.r[1]) + oj,
                             (pc[2] << op.r[2]) + ok};
          const double gd = gdet_at(c3);
          double Uc[9];
          child(c3, gd, Uc);
#pragma unroll
          for (int v = 0; v < 9; v++) acc[v] = __dadd_rn(acc[v], Uc[v]);
          gsum = __dadd_rn(gsum, gd);
        }
    const double cnt = (double)(n0 * n1 * n2);
    const double gme = gdet_at(gc);
    double Um[9];
    child(gc, gme, Um);
#pragma unroll
    for (int v = 0; v < 9; v++) {
      const double dq = __dsub_rn(__dmul_rn(cnt, U0[v]), acc[v]) / gsum;
      U[v] = __dadd_rn(Um[v], __dmul_rn(gme, dq));
    }
  }
  // the new cell: field from its new faces, the inversion, the floors
  const int64_t col = geo_col(Gt, bn, l[1] + ngn, l[0] + ngn);
  const Metric m = load_metric(Gt.c, Gt.ncol, col);
  const int64_t st[3] = {1, bn.np[0], (int64_t)bn.np[0] * bn.np[1]};
  double B[3];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    const double* X = Bt + 3 * bn.off + (int64_t)d * bn.vol;
    U[5 + d] = 0.5 * (X[loc] + X[loc + st[d]]);
    B[d] = U[5 + d] / m.gdet;
  }
  double guess[5], P[5];
#pragma unroll
  for (int v = 0; v < 5; v++) guess[v] = Pt[5 * bn.off + (int64_t)v * bn.vol + loc];
  C2PIn cs;
  c2p_setup(U, m, gam, cs);
  int iters = 0;
  c2p_solve(cs, m, false, 0.0, 0.0, guess, ph.tol, ph.maxit, P, iters);
  const double rfl = Gt.c[RHOFL * Gt.ncol + col], ufl = Gt.c[UFL * Gt.ncol + col];
  if (ph.floor_drift)
    drift_floors(P, B, m, rfl, ufl, ph.bsq_rho_max, ph.bsq_u_max, ph.gamma_max, gam, ph.tol, ph.maxit);
  else
    apply_floors(P, B, m, rfl, ufl, ph.bsq_rho_max, ph.bsq_u_max, ph.gamma_max);
#pragma unroll
  for (int v = 0; v < 5; v++) Pt[5 * bn.off + (int64_t)v * bn.vol + loc] = P[v];
}

// minmod slope along x_e (per parent cell) of the B^c faces at global face index g
__device__ __forceinline__ double face_slope(const OldBlock& ob, const double* __restrict__ X,
                                             const int g[3], int e) {
  int a[3] = {g[0], g[1], g[2]};
  const double c = X[ob.at(a[0], a[1], a[2])];
  a[e] -= 1;
  const double m = X[ob.at(a[0], a[1], a[2])];
  a[e] += 2;
  const double p = X[ob.at(a[0], a[1], a[2])];
  return minmod(__dsub_rn(c, m), __dsub_rn(p, c));
}

__global__ void __launch_bounds__(AT) k_regrid_faces(const BlockInfo* __restrict__ bf,
                                                     const BlockInfo* __restrict__ bt,
                                                     const RegridOp* __restrict__ ops, int64_t nops,
                                                     const int64_t* __restrict__ start,
                                                     int64_t t1, int64_t t2, int64_t t3,
                                                     const double* __restrict__ Bf,
                                                     double* __restrict__ Bt) {
  int64_t t = (int64_t)blockIdx.x * AT + threadIdx.x;
  int d;
  if (t < t1) {
    d = 0;
  } else if (t < t1 + t2) {
    d = 1;
    t -= t1;
  } else if (t < t1 + t2 + t3) {
    d = 2;
    t -= t1 + t2;
  } else {
    return;
  }
  const int64_t* st = start + (int64_t)(d + 1) * (nops + 1);
  const int k = regrid_box(st, nops, t);
  const RegridOp op = ops[k];
  const int64_t q = t - st[k];
  int ext[3] = {op.ext[0], op.ext[1], op.ext[2]};
  ext[d] += op.top[d];
  int l[3];
  l[0] = op.lo[0] + (int)(q % ext[0]);
  l[1] = op.lo[1] + (int)((q / ext[0]) % ext[1]);
  l[2] = op.lo[2] + (int)(q / ((int64_t)ext[0] * ext[1]));
  const int gf[3] = {op.on[0] + l[0], op.on[1] + l[1], op.on[2] + l[2]};
  const BlockInfo bn = bt[op.nb];
  const int ngn = (bn.np[0] - bn.n[0] - 1) / 2;
  const int64_t dst = 3 * bn.off + (int64_t)d * bn.vol +
                      ((int64_t)(l[2] + ngn) * bn.np[1] + (l[1] + ngn)) * bn.np[0] + (l[0] + ngn);
  const OldBlock ob = old_block(bf, op);
  const double* X = Bf + 3 * ob.bi.off + (int64_t)d * ob.bi.vol;
  const int rmin = min(op.r[0], min(op.r[1], op.r[2]));
  const int rmax = max(op.r[0], max(op.r[1], op.r[2]));
  double val;
  if (rmin == 0 && rmax == 0) {
    val = X[ob.at(gf[0], gf[1], gf[2])];
  } else if (rmax <= 0) {
    // mean of the fine sub-faces, k outermost, i innermost
    const int n0 = (d != 0 && op.r[0] < 0) ? 2 : 1, n1 = (d != 1 && op.r[1] < 0) ? 2 : 1,
              n2 = (d != 2 && op.r[2] < 0) ? 2 : 1;
    double acc = 0.0;
    for (int ok = 0; ok < n2; ok++)
      for (int oj = 0; oj < n1; oj++)
        for (int oi = 0; oi < n0; oi++)
          acc = __dadd_rn(acc, X[ob.at((gf[0] << (-op.r[0])) + oi, (gf[1] << (-op.r[1])) + oj,
                                       (gf[2] << (-op.r[2])) + ok)]);
    val = __dmul_rn(acc, 1.0 / (n0 * n1 * n2));
  } else {
    int pc[3] = {gf[0] >> op.r[0], gf[1] >> op.r[1], gf[2] >> op.r[2]};
    double tw[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int x = 0; x < 3; x++)
      if (x != d && op.r[x]) tw[x] = (gf[x] & 1) ? 0.25 : -0.25;
    if (op.r[d] == 0 || (gf[d] & 1) == 0) {
      // on a face of the parent cell: the parent face plus +-1/4 of its slopes
      val = X[ob.at(pc[0], pc[1], pc[2])];
#pragma unroll
      for (int e = 0; e < 3; e++)
        if (e != d && op.r[e]) val = __dadd_rn(val, __dmul_rn(tw[e], face_slope(ob, X, pc, e)));
    } else {
      // inside the parent cell: the face average of the divergence-free reconstruction
      int hi[3] = {pc[0], pc[1], pc[2]};
      hi[d] += 1;
      const double bm = X[ob.at(pc[0], pc[1], pc[2])], bp = X[ob.at(hi[0], hi[1], hi[2])];
      val = __dmul_rn(0.5, __dadd_rn(bm, bp));
#pragma unroll
      for (int e = 0; e < 3; e++) {
        if (e == d) continue;
        const double* Y = Bf + 3 * ob.bi.off + (int64_t)e * ob.bi.vol;
        int ep[3] = {pc[0], pc[1], pc[2]};
        ep[e] += 1;
        const double s_lo = face_slope(ob, Y, pc, d), s_hi = face_slope(ob, Y, ep, d);
        const double f = ob.bi.dx[d] / (8.0 * ob.bi.dx[e]);
        val = __dadd_rn(val, __dmul_rn(f, __dsub_rn(s_hi, s_lo)));
      }
#pragma unroll
      for (int e = 0; e < 3; e++) {
        if (e == d || !op.r[e]) continue;
        const double sl = __dadd_rn(face_slope(ob, X, pc, e), face_slope(ob, X, hi, e));
        val = __dadd_rn(val, __dmul_rn(__dmul_rn(tw[e], 0.5), sl));
      }
    }
  }
  Bt[dst] = val;
}

void launch_regrid(const Launch& Lf, const Launch& Lt, const RegridOp* ops, int64_t nops,
                   const int64_t* start, const int64_t total[4], const double* Pf,
                   const double* Bf, double* Pt, double* Bt, bool conserved) {
  if (nops <= 0) return;
  const int64_t nf = total[1] + total[2] + total[3];
  if (nf > 0)
    k_regrid_faces<<<dim3((unsigned)((nf + AT - 1) / AT)), dim3(AT), 0, Lf.stream>>>(
        Lf.blk, Lt.blk, ops, nops, start, total[1], total[2], total[3], Bf, Bt);
  if (total[0] > 0) {
    const dim3 grid((unsigned)((total[0] + AT - 1) / AT));
    k_regrid_cells<<<grid, dim3(AT), 0, Lf.stream>>>(Lf.blk, Lt.blk, Lf.geo, ops, nops, start,
                                                     total[0], Pf, Pt);
    if (conserved)
      k_regrid_cells_cons<<<grid, dim3(AT), 0, Lf.stream>>>(Lf.blk, Lt.blk, Lf.geo, Lt.geo, Lt.ph,
                                                            ops, nops, start, total[0], Pf, Bf,
                                                            Pt, Bt);
  }
}

}  // namespace grmhd
