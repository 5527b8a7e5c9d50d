// mlp.h -- learned first guess for the Newton inversion: an 8 -> 64 -> 64 -> 64 -> 2 MLP
// evaluated with bfloat16 matrix cores (v_mfma_f32_16x16x16_bf16, FP32 accumulation).
//
// Inference runs per wavefront on 64 cells in the transposed form D = W^T X^T: cells are
// the N dimension of the 16x16x16 tiles, so the accumulator layout of one layer (lane l
// holds rows 4*(l/16)..+3 of column l%16) is exactly the B-operand layout of the next
// layer and activations never leave registers.  Weights are pre-packed as A-operand
// fragments: lane l of fragment (layer, m-tile, k-step) holds W[in = 16 ks + 4 (l/16) + j]
// [out = 16 mt + l%16], j = 0..3, as bfloat16.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace grmhd {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int MLP_IN = 8, MLP_H = 64, MLP_OUT = 2;
constexpr int MLP_NPARAM = MLP_IN * MLP_H + MLP_H + 2 * (MLP_H * MLP_H + MLP_H) + MLP_H * MLP_OUT + MLP_OUT;
// fragment counts per layer: (m-tiles, k-steps)
constexpr int MLP_FRAGS = 4 * 1 + 4 * 4 + 4 * 4 + 1 * 4;

// packed inference blob (device memory)
struct MlpBlob {
  float xmean[8], xstd[8], ymean[2], ystd[2], pad[4];
  float b1[64], b2[64], b3[64], b4[16];
  bf16x4 frag[MLP_FRAGS * 64];
};

// offsets of the master (FP32) parameters: W1[8][64] b1 W2[64][64] b2 W3[64][64] b3 W4[64][2] b4
constexpr int P_W1 = 0, P_B1 = P_W1 + 8 * 64, P_W2 = P_B1 + 64, P_B2 = P_W2 + 64 * 64,
              P_W3 = P_B2 + 64, P_B3 = P_W3 + 64 * 64, P_W4 = P_B3 + 64, P_B4 = P_W4 + 64 * 2;

__device__ __forceinline__ short f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (short)0x7fc0;   // NaN
  u += 0x7fffu + ((u >> 16) & 1u);                               // round to nearest even
  return (short)(u >> 16);
}

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Forward pass of one wavefront's 64 cells.  feat: LDS [64][8] normalised features of
// this wave's cells; out: LDS [64][2] normalised outputs.  Every lane must call it.
// tanh x = 1 - 2 / (exp 2x + 1) from the hardware exp2 and reciprocal (absolute error
// ~1e-7, far below the BF16 rounding of the activations it feeds)
__device__ __forceinline__ float tanh_fast(float x) {
  const float xc = fminf(fmaxf(x, -15.0f), 15.0f);
  const float e = __builtin_amdgcn_exp2f(xc * 2.8853900817779268f);   // 2 log2(e)
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

__device__ __forceinline__ void mlp_wave(const MlpBlob* __restrict__ blob, const float* feat,
                                         float* out) {
  const int l = __lane_id();
  const int row = l & 15, grp = l >> 4;
#pragma unroll 1
  for (int t = 0; t < 4; t++) {
    // The weights and biases are re-read (from cache) for every tile of 16 cells: an
    // opaque copy of the blob pointer keeps the compiler from hoisting all 40 fragments
    // and the biases out of the loop, which would hold ~130 registers for the whole
    // pass (and, inlined into the update kernel, cost it a wavefront per SIMD).
    const MlpBlob* bp = blob;
    asm volatile("" : "+s"(bp));
    const bf16x4* F = bp->frag;
    const int cell = t * 16 + row;
    bf16x4 b[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int k = 4 * grp + j;
      b[0][j] = k < 8 ? f2bf(feat[cell * 8 + k]) : (short)0;
    }
    f32x4 h[4];
    // layer 1: 8 -> 64
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = mfma16(F[(0 + mt) * 64 + l], b[0], acc);
#pragma unroll
      for (int j = 0; j < 4; j++) acc[j] = tanh_fast(acc[j] + bp->b1[mt * 16 + 4 * grp + j]);
      h[mt] = acc;
    }
    // layers 2 and 3: 64 -> 64
#pragma unroll
    for (int layer = 0; layer < 2; layer++) {
      const int base = 4 + layer * 16;
      const float* bias = layer == 0 ? bp->b2 : bp->b3;
#pragma unroll
      for (int ks = 0; ks < 4; ks++)
#pragma unroll
        for (int j = 0; j < 4; j++) b[ks][j] = f2bf(h[ks][j]);
#pragma unroll
      for (int mt = 0; mt < 4; mt++) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ks++) acc = mfma16(F[(base + mt * 4 + ks) * 64 + l], b[ks], acc);
#pragma unroll
        for (int j = 0; j < 4; j++) acc[j] = tanh_fast(acc[j] + bias[mt * 16 + 4 * grp + j]);
        h[mt] = acc;
      }
    }
    // layer 4: 64 -> 2 (one padded m-tile)
#pragma unroll
    for (int ks = 0; ks < 4; ks++)
#pragma unroll
      for (int j = 0; j < 4; j++) b[ks][j] = f2bf(h[ks][j]);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 4; ks++) acc = mfma16(F[(36 + ks) * 64 + l], b[ks], acc);
    if (grp == 0) {
      out[cell * 2 + 0] = acc[0] + bp->b4[0];
      out[cell * 2 + 1] = acc[1] + bp->b4[1];
    }
  }
}

// raw features of a conserved state (see the oracle's definition: log D, asinh(tau/D),
// log1p(S^2/D^2), log1p(B^2/D), log1p((S.B)^2/D^3), lapse, gamma, sqrt(det gamma_ij))
struct MlpFeat {
  float x[8];
  bool ok;
};

}  // namespace grmhd
