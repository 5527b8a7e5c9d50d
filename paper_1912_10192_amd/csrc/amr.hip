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

}  // namespace grmhd
