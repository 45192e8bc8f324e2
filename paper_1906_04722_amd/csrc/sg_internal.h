// sg_internal.h -- kernels of the learned entry-pressure surrogate (internal;
// the public interface is lbm_surrogate.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sg {

typedef uint16_t bf16;  // bfloat16 bit pattern (round to nearest even from FP32)

constexpr int kFeat = 80;
constexpr int kHidden = 256;
constexpr int kOut = 17;
constexpr int kLayers = 4;
// widths of the layer inputs/outputs: 80 -> 256 -> 256 -> 256 -> 17
constexpr int kWidth[kLayers + 1] = {kFeat, kHidden, kHidden, kHidden, kOut};
// offsets of W_l ([out][in]) and b_l inside one member's flat parameters
constexpr long long w_off(int l) {
  long long o = 0;
  for (int i = 0; i < l; ++i) o += (long long)kWidth[i + 1] * kWidth[i] + kWidth[i + 1];
  return o;
}
constexpr long long b_off(int l) { return w_off(l) + (long long)kWidth[l + 1] * kWidth[l]; }
constexpr long long kParams = w_off(kLayers);
static_assert(kParams == 156689, "parameter count");

constexpr int kOcc = 32;   // occupancy samples per axis
constexpr int kPool = 8;   // samples per pooled cell and axis

// epilogues of the contraction C[m][n] = sum_k A(m,k) B(k,n)
enum Epi : int {
  kEpiF32 = 0,       // C = acc
  kEpiBiasF32 = 1,   // C = acc + bias[n]
  kEpiBiasSilu = 2,  // C = z = acc + bias[n], Cb = bf16(silu(z))
  kEpiDsilu = 3,     // C = d = acc * silu'(Zin[m][n]), Cb = bf16(d)
};

// A(m,k) = A[z*saz + m*sam + k*sak]; B(k,n) = B[z*sbz + k*sbk + n*sbn];
// outputs are row-major [M][N] per member z (member stride scz / sbzc)
struct Gemm {
  const bf16 *A;
  long long sam, sak, saz;
  const bf16 *B;
  long long sbk, sbn, sbz;
  int M, N, K, members;
  int epi;
  const float *bias;  // [z*bstride + n]
  long long bstride;
  float *C;           // f32 out
  long long scz;
  bf16 *Cb;           // bf16 out (epilogues 2, 3)
  long long sbzc;
  const float *Zin;   // pre-activation (epilogue 3), same layout as C
  long long szz;
};

hipError_t launch_gemm(const Gemm &g, hipStream_t st);

// per-column mean and population std (FP64) of X [n][cols], std < 1e-12 -> 1
hipError_t launch_col_stats(const double *X, int n, int cols, double *mu, double *sd,
                            hipStream_t st);
// Y[i][j] = (float)((X[i][j] - mu[j]) / sd[j])
hipError_t launch_standardise(const double *X, int n, int cols, const double *mu,
                              const double *sd, float *Y, hipStream_t st);
// Per-member work buffers are [member][cap][width] with cap the batch
// capacity.  A0[z][b][k] = bf16(X[idx[z*idx_stride + b]][k]) (k < 80),
// T0[z][b][j] = T[idx[...]][j] (T may be null); idx null means row b
hipError_t launch_gather(const float *X, const float *T, const int *idx, long long idx_stride,
                         int members, int bsz, long long cap, bf16 *A0, float *T0,
                         hipStream_t st);
// dY = 2 (Y - T) / (bsz * 17) in f32 and bf16; loss[z] = mean (Y - T)^2 (FP64)
hipError_t launch_loss_grad(const float *Y, const float *T, int members, int bsz, long long cap,
                            float *dY, bf16 *dYb, double *loss, hipStream_t st);
// db[z*pstride + n] = sum_b D[z][b][n]
hipError_t launch_bias_grad(const float *D, int members, int bsz, int N, long long cap, float *db,
                            long long pstride, hipStream_t st);
// Adam on all members' flat parameters, then the bf16 copy
hipError_t launch_adam(float *w, const float *g, float *m, float *v, bf16 *wb, long long count,
                       float lr, float b1, float b2, float eps, float bc1, float bc2,
                       hipStream_t st);
hipError_t launch_to_bf16(const float *w, bf16 *wb, long long count, hipStream_t st);
// ensemble mean / population std of the de-standardised outputs
hipError_t launch_ensemble(const float *Y, int members, int n, long long cap, const double *mu,
                           const double *sd, double *mean, double *std, hipStream_t st);
// descriptor of n four-sphere throats: geo[n][19] = 4 spheres (cx, cy, cz, r;
// throat spheres first) and nx, ny, nz; feat [n][80]
hipError_t launch_describe(const double *geo, int n, double *feat, hipStream_t st);

}  // namespace sg
