// internal.h -- structures shared by the host planner and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace grmhd {

// one block as the kernels see it
struct BlockInfo {
  int64_t off;      // cell offset of the block in the packed layout
  int32_t np[3];    // padded extents n + 2 ng + 1
  int32_t n[3];     // interior cells
  int32_t gorg[3];  // geometry-table index of local index 0 in x1, x2 (x3 unused)
  int32_t vol;      // np1 np2 np3
  int32_t lat;
  int32_t pad;
};

// one ghost copy: destination (block, local), source (block | flags << 24, local)
struct GhostOp {
  int32_t dst_blk, dst_loc, src_blkf, src_loc;
};
enum { GF_FLIP = 1, GF_CLAMP_NEG = 2, GF_CLAMP_POS = 4, GF_ZERO = 8 };

// geometry tables: SoA [quantity][column], column = j * ti + i
struct GeoTab {
  const double* c;    // centre: NGEO_C quantities
  const double* f1;   // x1 faces: NGEO_F
  const double* f2;   // x2 faces: NGEO_F (sqrt(-g) = 0 marks the polar axis)
  int64_t ncol;
  int32_t ti;
};

struct Counters {   // device counters of one grmhd_step call
  unsigned long long tier[5];
  unsigned long long hist[64];
  unsigned long long floors;
  unsigned long long dt_bits;     // min over cells of 1/sum_d(v_d/dx_d), as IEEE bits
  unsigned long long divb_abs;    // max |div B| bits
  unsigned long long divb_rel;
  double t_sim;
  double dt_last;
};

struct Phys {
  double dx[3];
  double gam, courant, tol;
  double bsq_rho_max, bsq_u_max, gamma_max;
  int32_t maxit;
  int32_t ng;
};

struct Launch {
  const BlockInfo* blk;   // device block table
  int32_t nblk;
  int32_t max_np[3];      // largest padded extents
  int32_t max_n[3];       // largest interior extents
  GeoTab geo;
  Phys ph;
  Counters* cnt;
  hipStream_t stream;
};

// records the message returned by grmhd_last_error() and returns code (host.cpp)
int set_error(int code, const char* msg);

// kernel launchers (kernels.hip)
void launch_ghost_cells(const Launch& L, const GhostOp* ops, int64_t nops, double* P);
void launch_ghost_faces(const Launch& L, const GhostOp* ops, int64_t nops, double* B, int comp);
void launch_bcell(const Launch& L, const double* B, double* Bc);
void launch_flux(const Launch& L, int dir, int recon, int riemann, const double* P,
                 const double* Bc, const double* B, double* F);
void launch_emf(const Launch& L, const double* F, double* E);
// update of one stage; with dt_part non-null the kernel also writes per-workgroup minima
// of the next Courant step (reduced by launch_dt_final)
// (mlp non-null: learned first guess of the inversion from the packed MLP blob)
void launch_update(const Launch& L, const double* Pn, const double* Bn, const double* Ps,
                   const double* Bcs, const double* F, const double* E, double dt_factor,
                   double* Pout, double* Bout, double* dt_part, const void* mlp);
int64_t dt_partials(const Launch& L);
void launch_dt(const Launch& L, const double* P, const double* B, double* dt_part);
void launch_dt_final(const Launch& L, const double* dt_part);
void launch_counters_reset(const Launch& L, bool all);
void launch_tsim(const Launch& L);
void launch_copy(const Launch& L, const double* src, double* dst, int64_t n);
void launch_divb(const Launch& L, const double* B, double* field);
void launch_extract(const Launch& L, const double* Pin, const double* Bin, int64_t n, double* P,
                    double* B, double* geom);
void launch_c2p_batch(int64_t n, const double* U, const double* geom, const double* guess,
                      const double* prev, double* P, int32_t* iters, int32_t* tier, double gam,
                      double tol, int32_t maxit, hipStream_t stream);

}  // namespace grmhd
