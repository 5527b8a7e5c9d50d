// mlp.hip -- training and packing of the learned inversion guess (BF16 MFMA, FP32 accumulate)
// and the batch utilities that build its training set on the device.
//
// Training step (batch of rows gathered by an index array), all on the caller's stream:
//   Z1 = X W1 + b1, H1 = tanh Z1, ... , Z4 = H3 W4 + b4          forward
//   G4 = 2 (Z4 - Y) / (rows * 2)                                 mean-squared-error gradient
//   dW_l = H_{l-1}^T G_l, db_l = sum_rows G_l,
//   G_{l-1} = (G_l W_l^T) * (1 - H_{l-1}^2)                       backward
//   Adam on the FP32 master parameters.
// Products over the features (forward, and the gradients passed down) are launches of
// k_gemm: 16x16 output tiles per wavefront, operands rounded to bfloat16 on load,
// v_mfma_f32_16x16x16_bf16 over K.  Products over the batch (the parameter gradients,
// K = rows) split K across workgroups (k_wgrad) and add the chunks in order.
#include <hip/hip_runtime.h>

#include <mutex>

#include <cmath>
#include <cstdint>
#include <string>

#include "../../include/grmhd.h"
#include "device.h"
#include "internal.h"
#include "mlp.h"

namespace grmhd {

constexpr int MT = 256;

// C[M][N] = op(A)[M][K] op(B)[K][N] (+ bias[N]).  op(A)[m][k] = A[m*lda + k], or with TA
// A[k*lda + m]; a non-null idx replaces the row index r of A (m, or k with TA) by idx[r].
// op(B)[k][n] = B[k*ldb + n], or with TB B[n*ldb + k].
template <bool TA, bool TB>
__global__ __launch_bounds__(MT) void k_gemm(int M, int N, int K, const float* __restrict__ A,
                                             int lda, const int32_t* __restrict__ idx,
                                             const float* __restrict__ B, int ldb,
                                             const float* __restrict__ bias, float* __restrict__ C,
                                             int ldc) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int row = lane & 15, grp = lane >> 4;
  const int mt = blockIdx.x, nt = blockIdx.y * 4 + w;
  const int m0 = mt * 16, n0 = nt * 16;
  if (n0 >= N) return;   // whole wavefront leaves together
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x4 a, b;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int k = k0 + 4 * grp + j;
      const int m = m0 + row, n = n0 + row;
      float av = 0.f, bv = 0.f;
      if (m < M && k < K) {
        if (TA) {
          const int kr = idx ? idx[k] : k;
          av = A[(int64_t)kr * lda + m];
        } else {
          const int mr = idx ? idx[m] : m;
          av = A[(int64_t)mr * lda + k];
        }
      }
      if (n < N && k < K) bv = TB ? B[(int64_t)n * ldb + k] : B[(int64_t)k * ldb + n];
      a[j] = f2bf(av);
      b[j] = f2bf(bv);
    }
    acc = mfma16(a, b, acc);
  }
#pragma unroll
  for (int j = 0; j < 4; j++) {
    const int m = m0 + 4 * grp + j, n = n0 + row;
    if (m < M && n < N) C[(int64_t)m * ldc + n] = acc[j] + (bias ? bias[n] : 0.f);
  }
}

__global__ __launch_bounds__(MT) void k_tanh(float* __restrict__ Z, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * MT + threadIdx.x;
  if (i < n) Z[i] = tanhf(Z[i]);
}

// G *= 1 - H^2
__global__ __launch_bounds__(MT) void k_tanh_back(float* __restrict__ G, const float* __restrict__ H,
                                                  int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * MT + threadIdx.x;
  if (i < n) G[i] *= 1.0f - H[i] * H[i];
}

// G = 2 (Z - Y[idx]) / (rows * cols); loss partial sums per workgroup
__global__ __launch_bounds__(MT) void k_mse(const float* __restrict__ Z, const float* __restrict__ Y,
                                            const int32_t* __restrict__ idx, int rows, int cols,
                                            float* __restrict__ G, float* __restrict__ part) {
  __shared__ float red[MT];
  const int64_t i = (int64_t)blockIdx.x * MT + threadIdx.x;
  float e = 0.f;
  if (i < (int64_t)rows * cols) {
    const int r = (int)(i / cols), c = (int)(i % cols);
    const float d = Z[i] - Y[(int64_t)(idx ? idx[r] : r) * cols + c];
    G[i] = 2.0f * d / (float)(rows * cols);
    e = d * d;
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int s = MT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// loss = sum(part) / (rows * cols), one workgroup
__global__ __launch_bounds__(MT) void k_loss_final(const float* __restrict__ part, int np, float scale,
                                                   float* __restrict__ loss) {
  __shared__ float red[MT];
  float e = 0.f;
  for (int i = threadIdx.x; i < np; i += MT) e += part[i];
  red[threadIdx.x] = e;
  __syncthreads();
  for (int s = MT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] * scale;
}

// Parameter gradients reduce over the batch (K = rows, thousands) into at most 64 x 64
// outputs: split K.  Workgroup c takes rows [c KC, (c + 1) KC) and writes its partial
// dW = A^T G (A gathered through idx) as part[c][M][N] and, if db is wanted, its partial
// column sums of G as part[c][M N + n]; k_wgrad_final adds the chunks in order.
constexpr int KC = 256;
__global__ __launch_bounds__(MT) void k_wgrad(int M, int N, int K, const float* __restrict__ A,
                                              int lda, const int32_t* __restrict__ idx,
                                              const float* __restrict__ G, int ldg, int colsum,
                                              float* __restrict__ part) {
  __shared__ float red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int row = lane & 15, grp = lane >> 4;
  const int c = blockIdx.x;
  const int k_lo = c * KC, k_hi = min(K, k_lo + KC);
  const int tm = (M + 15) / 16, tn = (N + 15) / 16;
  float* out = part + (int64_t)c * (M * N + (colsum ? N : 0));
  // output tiles w, w + 4, ... of the tm x tn tile grid, 16 x 16 each
  for (int tile = w; tile < tm * tn; tile += 4) {
    const int m0 = (tile / tn) * 16, n0 = (tile % tn) * 16;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = k_lo; k0 < k_hi; k0 += 16) {
      bf16x4 a, b;
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int k = k0 + 4 * grp + j;
        const int m = m0 + row, n = n0 + row;
        float av = 0.f, bv = 0.f;
        if (k < k_hi) {
          if (m < M) av = A[(int64_t)(idx ? idx[k] : k) * lda + m];
          if (n < N) bv = G[(int64_t)k * ldg + n];
        }
        a[j] = f2bf(av);
        b[j] = f2bf(bv);
      }
      acc = mfma16(a, b, acc);
    }
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int m = m0 + 4 * grp + j, n = n0 + row;
      if (m < M && n < N) out[m * N + n] = acc[j];
    }
  }
  if (colsum) {
    // column n = lane (N <= 64), rows k_lo + w, k_lo + w + 4, ... summed per wave
    float s = 0.f;
    if (lane < N)
      for (int k = k_lo + w; k < k_hi; k += 4) s += G[(int64_t)k * ldg + lane];
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && lane < N) out[M * N + lane] = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
  }
}

// dW[m][n] (row stride ldw) and db[n] from the chunk partials, chunks in order
__global__ __launch_bounds__(MT) void k_wgrad_final(int M, int N, int nchunk, int colsum,
                                                    const float* __restrict__ part,
                                                    float* __restrict__ dW, int ldw,
                                                    float* __restrict__ db) {
  const int i = blockIdx.x * MT + threadIdx.x;
  const int per = M * N + (colsum ? N : 0);
  if (i >= per) return;
  float s = 0.f;
  for (int c = 0; c < nchunk; c++) s += part[(int64_t)c * per + i];
  if (i < M * N) dW[(i / N) * ldw + i % N] = s;
  else db[i - M * N] = s;
}

__global__ __launch_bounds__(MT) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                             float* __restrict__ m, float* __restrict__ v, int n,
                                             float lr, float b1t, float b2t) {
  const int i = blockIdx.x * MT + threadIdx.x;
  if (i >= n) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  m[i] = b1 * m[i] + (1.f - b1) * g[i];
  v[i] = b2 * v[i] + (1.f - b2) * g[i] * g[i];
  const float mh = m[i] / (1.f - b1t), vh = v[i] / (1.f - b2t);
  p[i] -= lr * mh / (sqrtf(vh) + eps);
}

// master parameters + normalisation -> inference blob (A-operand fragments, bfloat16)
__global__ void k_pack(const float* __restrict__ prm, const float* __restrict__ norm,
                       MlpBlob* __restrict__ blob) {
  const int t = threadIdx.x;   // 64 threads
  for (int q = t; q < 24; q += 64) (&blob->xmean[0])[q] = q < 20 ? norm[q] : 0.f;
  for (int q = t; q < 64; q += 64) {
    blob->b1[q] = prm[P_B1 + q];
    blob->b2[q] = prm[P_B2 + q];
    blob->b3[q] = prm[P_B3 + q];
  }
  if (t < 16) blob->b4[t] = t < 2 ? prm[P_B4 + t] : 0.f;
  // fragments: layer 1 (4 m-tiles, 1 k-step), layers 2, 3 (4 x 4), layer 4 (1 x 4)
  struct L { int off, in, out, mts, kss, base; };
  const L layers[4] = {{P_W1, 8, 64, 4, 1, 0}, {P_W2, 64, 64, 4, 4, 4}, {P_W3, 64, 64, 4, 4, 20},
                       {P_W4, 64, 2, 1, 4, 36}};
  const int row = t & 15, grp = t >> 4;
  for (int li = 0; li < 4; li++) {
    const L& y = layers[li];
    for (int mt = 0; mt < y.mts; mt++)
      for (int ks = 0; ks < y.kss; ks++) {
        bf16x4 f;
        for (int j = 0; j < 4; j++) {
          const int in = ks * 16 + 4 * grp + j, out = mt * 16 + row;
          f[j] = (in < y.in && out < y.out) ? f2bf(prm[y.off + in * y.out + out]) : (short)0;
        }
        blob->frag[(y.base + mt * y.kss + ks) * 64 + t] = f;
      }
  }
}

// forward of rows X[n][8] (normalised) through the packed blob; Y[n][2] normalised outputs
__global__ __launch_bounds__(MT) void k_mlp_forward(const MlpBlob* __restrict__ blob,
                                                    const float* __restrict__ X, int64_t n,
                                                    float* __restrict__ Y) {
  __shared__ float feat[MT * 8];
  __shared__ float outv[MT * 2];
  const int64_t base = (int64_t)blockIdx.x * MT;
  const int t = threadIdx.x, w = t / 64;
  for (int k = 0; k < 8; k++) feat[t * 8 + k] = base + t < n ? X[(base + t) * 8 + k] : 0.f;
  __syncthreads();
  mlp_wave(blob, feat + w * 64 * 8, outv + w * 64 * 2);
  __syncthreads();
  if (base + t < n) {
    Y[(base + t) * 2] = outv[t * 2];
    Y[(base + t) * 2 + 1] = outv[t * 2 + 1];
  }
}

// ----------------------------------------------------------------- data utilities

// U = prim2cons(P, B) at given metrics (Sec. 2.3-2.5): U[9][n], P[5][n], B[3][n], geom[15][n]
__global__ __launch_bounds__(MT) void k_prim2cons(int64_t n, const double* __restrict__ P,
                                                  const double* __restrict__ B,
                                                  const double* __restrict__ geom, double gam,
                                                  double* __restrict__ U) {
  const int64_t i = (int64_t)blockIdx.x * MT + threadIdx.x;
  if (i >= n) return;
  const Metric m = load_metric(geom, n, i);
  double p[5], b[3], u[9];
  for (int v = 0; v < 5; v++) p[v] = P[v * n + i];
  for (int v = 0; v < 3; v++) b[v] = B[v * n + i];
  Fluid f;
  fluid_state(p, b, m, f);
  flux_vector<0>(p, f, m, gam, entropy_kappa(p, gam), u);
  for (int q = 0; q < 9; q++) U[q * n + i] = u[q];
}

// raw features X[n][8] of U and raw targets Y[n][2] of P (P may be NULL)
__global__ __launch_bounds__(MT) void k_dataset(int64_t n, const double* __restrict__ U,
                                                const double* __restrict__ P,
                                                const double* __restrict__ geom, double gam,
                                                float* __restrict__ X, float* __restrict__ Y,
                                                int32_t* __restrict__ ok) {
  const int64_t i = (int64_t)blockIdx.x * MT + threadIdx.x;
  if (i >= n) return;
  const Metric m = load_metric(geom, n, i);
  double u[9];
  for (int q = 0; q < 9; q++) u[q] = U[q * n + i];
  C2PIn s;
  c2p_setup(u, m, gam, s);
  float x[8];
  bool good = mlp_features(s, m, x);
  for (int k = 0; k < 8; k++) X[i * 8 + k] = x[k];
  if (P && Y) {
    double p[5];
    for (int v = 0; v < 5; v++) p[v] = P[v * n + i];
    double W, vsq;
    guess_from_prims(s, m, p, W, vsq);
    const double G = 1.0 / sqrt(1.0 - vsq);
    const double D = p[0] * G;
    const double y0 = log(G), y1 = log(W / D);
    good = good && isfinite(y0) && isfinite(y1);
    Y[i * 2] = (float)y0;
    Y[i * 2 + 1] = (float)y1;
  }
  ok[i] = good ? 1 : 0;
}

// column means and standard deviations of A[n][cols] (FP64 sums, one workgroup per column)
__global__ __launch_bounds__(MT) void k_moments(const float* __restrict__ A, int64_t n, int cols,
                                                float* __restrict__ mean, float* __restrict__ sd) {
  __shared__ double s1[MT], s2[MT];
  const int c = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += MT) {
    const double x = A[i * cols + c];
    a += x;
    b += x * x;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int s = MT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      s1[threadIdx.x] += s1[threadIdx.x + s];
      s2[threadIdx.x] += s2[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mu = s1[0] / (double)n;
    const double var = s2[0] / (double)n - mu * mu;
    mean[c] = (float)mu;
    sd[c] = (float)(var > 1e-12 ? sqrt(var) : 1.0);
  }
}

__global__ __launch_bounds__(MT) void k_normalize(float* __restrict__ A, int64_t n, int cols,
                                                  const float* __restrict__ mean,
                                                  const float* __restrict__ sd) {
  const int64_t i = (int64_t)blockIdx.x * MT + threadIdx.x;
  if (i >= n * cols) return;
  const int c = (int)(i % cols);
  A[i] = (A[i] - mean[c]) / sd[c];
}

static inline unsigned cdv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// dW (M x N, row stride ldw) = A^T G over the K rows (A gathered through idx), and db =
// the column sums of G if db is non-null; part: workspace of wgrad_floats(K) floats
static size_t wgrad_floats(int K) { return (size_t)cdv(K, KC) * (64 * 64 + 64); }
static void wgrad(int M, int N, int K, const float* A, int lda, const int32_t* idx, const float* G,
                  int ldg, float* dW, int ldw, float* db, float* part, hipStream_t st) {
  const int nchunk = (int)cdv(K, KC), cs = db ? 1 : 0;
  hipLaunchKernelGGL(k_wgrad, dim3(nchunk), dim3(MT), 0, st, M, N, K, A, lda, idx, G, ldg, cs,
                     part);
  hipLaunchKernelGGL(k_wgrad_final, dim3(cdv(M * N + N, MT)), dim3(MT), 0, st, M, N, nchunk, cs,
                     part, dW, ldw, db);
}

static void gemm(bool ta, bool tb, int M, int N, int K, const float* A, int lda, const int32_t* idx,
                 const float* B, int ldb, const float* bias, float* C, int ldc, hipStream_t st) {
  const dim3 grid(cdv(M, 16), cdv(N, 64));
  if (!ta && !tb)
    hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(MT), 0, st, M, N, K, A, lda, idx, B, ldb, bias, C, ldc);
  else if (!ta && tb)
    hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(MT), 0, st, M, N, K, A, lda, idx, B, ldb, bias, C, ldc);
  else if (ta && !tb)
    hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(MT), 0, st, M, N, K, A, lda, idx, B, ldb, bias, C, ldc);
  else
    hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(MT), 0, st, M, N, K, A, lda, idx, B, ldb, bias, C, ldc);
}

}  // namespace grmhd

using namespace grmhd;

static int mfail(int code, const char* msg) { return grmhd::set_error(code, msg); }

extern "C" {

int grmhd_mlp_sizes(int32_t batch, size_t* n_params, size_t* blob_bytes, size_t* work_floats) {
  if (batch < 1) return mfail(GRMHD_EINVAL, "batch must be positive");
  if (n_params) *n_params = MLP_NPARAM;
  if (blob_bytes) *blob_bytes = sizeof(MlpBlob);
  // activations H1..H3, Z4, G (two buffers), parameter gradients, loss partials
  const size_t b = (size_t)batch;
  if (work_floats)
    *work_floats = 3 * b * 64 + b * 2 + 2 * b * 64 + MLP_NPARAM + cdv(b * 2, MT) + 64 +
                   wgrad_floats(batch);
  return GRMHD_OK;
}

}  // extern "C"

// The training step on a work buffer of at least work_floats(batch) floats.
static int train_step(float* params, float* adam_m, float* adam_v, int32_t step, const float* X,
                      const float* Y, const int32_t* idx, int32_t batch, float lr, float* work,
                      float* loss, hipStream_t st) {
  const int B = batch;
  float* H1 = work;
  float* H2 = H1 + (size_t)B * 64;
  float* H3 = H2 + (size_t)B * 64;
  float* Z4 = H3 + (size_t)B * 64;
  float* Ga = Z4 + (size_t)B * 2;
  float* Gb = Ga + (size_t)B * 64;
  float* grad = Gb + (size_t)B * 64;
  float* part = grad + MLP_NPARAM;
  float* wpart = part + cdv((int64_t)B * 2, MT) + 64;
  const float* W1 = params + P_W1;
  const float* W2 = params + P_W2;
  const float* W3 = params + P_W3;
  const float* W4 = params + P_W4;
  const int64_t nh = (int64_t)B * 64;
  // forward
  gemm(false, false, B, 64, 8, X, 8, idx, W1, 64, params + P_B1, H1, 64, st);
  hipLaunchKernelGGL(k_tanh, dim3(cdv(nh, MT)), dim3(MT), 0, st, H1, nh);
  gemm(false, false, B, 64, 64, H1, 64, nullptr, W2, 64, params + P_B2, H2, 64, st);
  hipLaunchKernelGGL(k_tanh, dim3(cdv(nh, MT)), dim3(MT), 0, st, H2, nh);
  gemm(false, false, B, 64, 64, H2, 64, nullptr, W3, 64, params + P_B3, H3, 64, st);
  hipLaunchKernelGGL(k_tanh, dim3(cdv(nh, MT)), dim3(MT), 0, st, H3, nh);
  gemm(false, false, B, 2, 64, H3, 64, nullptr, W4, 2, params + P_B4, Z4, 2, st);
  // loss and output gradient (into Ga as [B][2])
  const unsigned np = cdv((int64_t)B * 2, MT);
  hipLaunchKernelGGL(k_mse, dim3(np), dim3(MT), 0, st, Z4, Y, idx, B, 2, Ga, part);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(MT), 0, st, part, (int)np, 1.0f / (float)(B * 2), loss);
  // backward: layer 4
  wgrad(64, 2, B, H3, 64, nullptr, Ga, 2, grad + P_W4, 2, grad + P_B4, wpart, st);
  gemm(false, true, B, 64, 2, Ga, 2, nullptr, W4, 2, nullptr, Gb, 64, st);
  hipLaunchKernelGGL(k_tanh_back, dim3(cdv(nh, MT)), dim3(MT), 0, st, Gb, H3, nh);
  // layer 3
  wgrad(64, 64, B, H2, 64, nullptr, Gb, 64, grad + P_W3, 64, grad + P_B3, wpart, st);
  gemm(false, true, B, 64, 64, Gb, 64, nullptr, W3, 64, nullptr, Ga, 64, st);
  hipLaunchKernelGGL(k_tanh_back, dim3(cdv(nh, MT)), dim3(MT), 0, st, Ga, H2, nh);
  // layer 2
  wgrad(64, 64, B, H1, 64, nullptr, Ga, 64, grad + P_W2, 64, grad + P_B2, wpart, st);
  gemm(false, true, B, 64, 64, Ga, 64, nullptr, W2, 64, nullptr, Gb, 64, st);
  hipLaunchKernelGGL(k_tanh_back, dim3(cdv(nh, MT)), dim3(MT), 0, st, Gb, H1, nh);
  // layer 1 (inputs gathered through idx)
  wgrad(8, 64, B, X, 8, idx, Gb, 64, grad + P_W1, 64, grad + P_B1, wpart, st);
  // Adam
  const float b1t = (float)std::pow(0.9, step), b2t = (float)std::pow(0.999, step);
  hipLaunchKernelGGL(k_adam, dim3(cdv(MLP_NPARAM, MT)), dim3(MT), 0, st, params, grad, adam_m, adam_v,
                     MLP_NPARAM, lr, b1t, b2t);
  if (hipGetLastError() != hipSuccess) return mfail(GRMHD_EHIP, "kernel launch failed");
  return GRMHD_OK;
}

// Work buffer of the allocation-free training step, sized for the largest batch it
// takes; one copy per device, held until the process ends.  Every kernel of a step
// writes the part it reads later, so nothing needs clearing between calls.
constexpr int64_t NOALLOC_B = GRMHD_MLP_NOALLOC_MAX_BATCH;
constexpr size_t NOALLOC_FLOATS =
    (size_t)(3 * NOALLOC_B * 64 + NOALLOC_B * 2 + 2 * NOALLOC_B * 64 + MLP_NPARAM +
             (NOALLOC_B * 2 + MT - 1) / MT + 64 + (NOALLOC_B + KC - 1) / KC * (64 * 64 + 64));
static __device__ __align__(256) float scratch[NOALLOC_FLOATS];

// device address of `scratch` per device index, taken once with that device current
constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static float* g_scratch[NOALLOC_MAX_DEVICES] = {};

static int scratch_address(float** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return mfail(GRMHD_EHIP, "hipGetDevice failed");
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return mfail(GRMHD_EUNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return mfail(GRMHD_EHIP, "hipGetSymbolAddress(scratch) failed");
    g_scratch[dev] = (float*)ptr;
  }
  *out = g_scratch[dev];
  return GRMHD_OK;
}

extern "C" {

int grmhd_mlp_train_step(float* params, float* adam_m, float* adam_v, int32_t step,
                         const float* X, const float* Y, const int32_t* idx, int32_t batch,
                         float lr, float* work, float* loss, void* hip_stream) {
  if (!params || !adam_m || !adam_v || !X || !Y || !idx || !work || !loss)
    return mfail(GRMHD_EINVAL, "NULL argument");
  if (batch < 1 || step < 1) return mfail(GRMHD_EINVAL, "batch and step must be positive");
  return train_step(params, adam_m, adam_v, step, X, Y, idx, batch, lr, work, loss,
                    (hipStream_t)hip_stream);
}

int grmhd_mlp_train_step_noalloc(float* params, float* adam_m, float* adam_v, int32_t step,
                                 const float* X, const float* Y, const int32_t* idx,
                                 int32_t batch, float lr, float* loss, void* hip_stream) {
  if (!params || !adam_m || !adam_v || !X || !Y || !idx || !loss)
    return mfail(GRMHD_EINVAL, "NULL argument");
  if (batch < 1 || step < 1) return mfail(GRMHD_EINVAL, "batch and step must be positive");
  if (batch > GRMHD_MLP_NOALLOC_MAX_BATCH)
    return mfail(GRMHD_EINVAL, "batch exceeds GRMHD_MLP_NOALLOC_MAX_BATCH");
  float* work = nullptr;
  if (int rc = scratch_address(&work)) return rc;
  return train_step(params, adam_m, adam_v, step, X, Y, idx, batch, lr, work, loss,
                    (hipStream_t)hip_stream);
}

int grmhd_mlp_gradients(const float* params, const float* X, const float* Y, const int32_t* idx,
                        int32_t batch, float* work, float* grad_out, float* loss, void* hip_stream) {
  // one training step without the update: run the step with zero learning rate on a copy
  // would change Adam state, so compute the gradients explicitly
  if (!params || !X || !Y || !work || !grad_out || !loss) return mfail(GRMHD_EINVAL, "NULL argument");
  if (batch < 1) return mfail(GRMHD_EINVAL, "batch must be positive");
  hipStream_t st = (hipStream_t)hip_stream;
  const int B = batch;
  float* H1 = work;
  float* H2 = H1 + (size_t)B * 64;
  float* H3 = H2 + (size_t)B * 64;
  float* Z4 = H3 + (size_t)B * 64;
  float* Ga = Z4 + (size_t)B * 2;
  float* Gb = Ga + (size_t)B * 64;
  float* part = Gb + (size_t)B * 64 + MLP_NPARAM;
  float* wpart = part + cdv((int64_t)B * 2, MT) + 64;
  float* grad = grad_out;
  const float* W2 = params + P_W2;
  const float* W3 = params + P_W3;
  const float* W4 = params + P_W4;
  const int64_t nh = (int64_t)B * 64;
  gemm(false, false, B, 64, 8, X, 8, idx, params + P_W1, 64, params + P_B1, H1, 64, st);
  hipLaunchKernelGGL(k_tanh, dim3(cdv(nh, MT)), dim3(MT), 0, st, H1, nh);
  gemm(false, false, B, 64, 64, H1, 64, nullptr, W2, 64, params + P_B2, H2, 64, st);
  hipLaunchKernelGGL(k_tanh, dim3(cdv(nh, MT)), dim3(MT), 0, st, H2, nh);
  gemm(false, false, B, 64, 64, H2, 64, nullptr, W3, 64, params + P_B3, H3, 64, st);
  hipLaunchKernelGGL(k_tanh, dim3(cdv(nh, MT)), dim3(MT), 0, st, H3, nh);
  gemm(false, false, B, 2, 64, H3, 64, nullptr, W4, 2, params + P_B4, Z4, 2, st);
  const unsigned np = cdv((int64_t)B * 2, MT);
  hipLaunchKernelGGL(k_mse, dim3(np), dim3(MT), 0, st, Z4, Y, idx, B, 2, Ga, part);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(MT), 0, st, part, (int)np, 1.0f / (float)(B * 2), loss);
  wgrad(64, 2, B, H3, 64, nullptr, Ga, 2, grad + P_W4, 2, grad + P_B4, wpart, st);
  gemm(false, true, B, 64, 2, Ga, 2, nullptr, W4, 2, nullptr, Gb, 64, st);
  hipLaunchKernelGGL(k_tanh_back, dim3(cdv(nh, MT)), dim3(MT), 0, st, Gb, H3, nh);
  wgrad(64, 64, B, H2, 64, nullptr, Gb, 64, grad + P_W3, 64, grad + P_B3, wpart, st);
  gemm(false, true, B, 64, 64, Gb, 64, nullptr, W3, 64, nullptr, Ga, 64, st);
  hipLaunchKernelGGL(k_tanh_back, dim3(cdv(nh, MT)), dim3(MT), 0, st, Ga, H2, nh);
  wgrad(64, 64, B, H1, 64, nullptr, Ga, 64, grad + P_W2, 64, grad + P_B2, wpart, st);
  gemm(false, true, B, 64, 64, Ga, 64, nullptr, W2, 64, nullptr, Gb, 64, st);
  hipLaunchKernelGGL(k_tanh_back, dim3(cdv(nh, MT)), dim3(MT), 0, st, Gb, H1, nh);
  wgrad(8, 64, B, X, 8, idx, Gb, 64, grad + P_W1, 64, grad + P_B1, wpart, st);
  if (hipGetLastError() != hipSuccess) return mfail(GRMHD_EHIP, "kernel launch failed");
  return GRMHD_OK;
}

int grmhd_mlp_pack(const float* params, const float* norm, void* blob, void* hip_stream) {
  if (!params || !norm || !blob) return mfail(GRMHD_EINVAL, "NULL argument");
  if (((uintptr_t)blob & 15) != 0) return mfail(GRMHD_EINVAL, "blob must be 16-byte aligned");
  hipLaunchKernelGGL(k_pack, dim3(1), dim3(64), 0, (hipStream_t)hip_stream, params, norm,
                     (MlpBlob*)blob);
  if (hipGetLastError() != hipSuccess) return mfail(GRMHD_EHIP, "kernel launch failed");
  return GRMHD_OK;
}

int grmhd_mlp_forward(const void* blob, const float* X, int64_t n, float* Y, void* hip_stream) {
  if (!blob || (n > 0 && (!X || !Y))) return mfail(GRMHD_EINVAL, "NULL argument");
  if (n <= 0) return GRMHD_OK;
  hipLaunchKernelGGL(k_mlp_forward, dim3(cdv(n, MT)), dim3(MT), 0, (hipStream_t)hip_stream,
                     (const MlpBlob*)blob, X, n, Y);
  if (hipGetLastError() != hipSuccess) return mfail(GRMHD_EHIP, "kernel launch failed");
  return GRMHD_OK;
}

int grmhd_prim2cons_batch(int64_t n, const double* P, const double* B, const double* geom,
                          double gamma_ad, double* U, void* hip_stream) {
  if (n <= 0) return GRMHD_OK;
  if (!P || !B || !geom || !U) return mfail(GRMHD_EINVAL, "NULL argument");
  hipLaunchKernelGGL(k_prim2cons, dim3(cdv(n, MT)), dim3(MT), 0, (hipStream_t)hip_stream, n, P, B,
                     geom, gamma_ad, U);
  if (hipGetLastError() != hipSuccess) return mfail(GRMHD_EHIP, "kernel launch failed");
  return GRMHD_OK;
}

int grmhd_mlp_dataset(int64_t n, const double* U, const double* P, const double* geom,
                      double gamma_ad, float* X, float* Y, int32_t* ok, void* hip_stream) {
  if (n <= 0) return GRMHD_OK;
  if (!U || !geom || !X || !ok) return mfail(GRMHD_EINVAL, "NULL argument");
  hipLaunchKernelGGL(k_dataset, dim3(cdv(n, MT)), dim3(MT), 0, (hipStream_t)hip_stream, n, U, P,
                     geom, gamma_ad, X, Y, ok);
  if (hipGetLastError() != hipSuccess) return mfail(GRMHD_EHIP, "kernel launch failed");
  return GRMHD_OK;
}

int grmhd_mlp_normalize(float* A, int64_t n, int32_t cols, float* mean, float* sd,
                        int32_t compute, void* hip_stream) {
  if (!A || !mean || !sd || cols < 1 || n < 1) return mfail(GRMHD_EINVAL, "bad arguments");
  hipStream_t st = (hipStream_t)hip_stream;
  if (compute) hipLaunchKernelGGL(k_moments, dim3(cols), dim3(MT), 0, st, A, n, cols, mean, sd);
  hipLaunchKernelGGL(k_normalize, dim3(cdv(n * cols, MT)), dim3(MT), 0, st, A, n, cols, mean, sd);
  if (hipGetLastError() != hipSuccess) return mfail(GRMHD_EHIP, "kernel launch failed");
  return GRMHD_OK;
}

}  // extern "C"
