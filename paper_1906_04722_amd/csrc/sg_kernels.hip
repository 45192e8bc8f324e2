// sg_kernels.hip -- kernels of the learned entry-pressure surrogate on gfx950:
// a BF16 matrix-core contraction with fused bias / SiLU / SiLU-derivative
// epilogues (FP32 accumulation), the loss gradient, bias gradients, Adam on
// FP32 master weights, standardisation, ensemble statistics and the
// geometry + occupancy descriptor of a throat.
#include <hip/hip_runtime.h>

#include "geom.h"
#include "sg_internal.h"

namespace sg {

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16 to_bf16(float f) {
  // round to nearest, ties to even (inputs are finite)
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16)(u >> 16);
}

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }

__device__ __forceinline__ float dsilu(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// ---- contraction ----------------------------------------------------------
// Block tile 64 x 64 of C, four waves of 32 x 32, K staged through LDS 64 at a
// time.  Each wave issues 2 x 2 v_mfma_f32_16x16x32_bf16 (gfx950) per 32 of
// K.  Operand layout of that instruction (64 lanes, 8 values each): lane l
// holds A[l % 16][8 (l / 16) + i] and B[8 (l / 16) + i][l % 16]; the result
// C[4 (l / 16) + i][l % 16].  Both tiles sit in LDS k-contiguous ([row][k],
// rows padded to 72 bf16 = 144 bytes), so every operand is one 16-byte LDS
// read.  Staging moves 16 bytes (8 bf16) per load where the operand allows:
// along k when it is k-contiguous (X W^T, D W), along the rows when it is
// row-contiguous (the weight gradients D^T A), scattering the 8 values into
// their k-contiguous LDS rows; other shapes fall back to one value per load.
constexpr int BM = 64, BN = 64, BK = 64, LDK = BK + 8;
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// stage rows r0 .. r0+63 and k0 .. k0+63 of X(row, k) = X[row*srow + k*sk]
// (nrow rows, K columns) into S[row - r0][k - k0], zero outside
__device__ __forceinline__ void stage(bf16 (&S)[64][LDK], const bf16 *X, long long srow,
                                      long long sk, int nrow, int K, int r0, int k0, int tid) {
  const bool aligned = ((uintptr_t)X & 15u) == 0;
  if (sk == 1 && aligned && (srow & 7) == 0 && (K & 7) == 0) {
    // k-contiguous: 8 consecutive k of one row per load (K % 8 == 0: a group
    // of 8 lies wholly inside or outside the matrix)
#pragma unroll
    for (int t = 0; t < (64 * BK / 8) / 256; ++t) {
      const int v = tid + 256 * t, r = v / (BK / 8), c = (v % (BK / 8)) * 8;
      const int row = r0 + r, k = k0 + c;
      uint4 q = make_uint4(0u, 0u, 0u, 0u);
      if (row < nrow && k < K) q = *(const uint4 *)(X + (long long)row * srow + k);
      *(uint4 *)&S[r][c] = q;
    }
  } else if (srow == 1 && aligned && (sk & 7) == 0 && (nrow & 7) == 0) {
    // row-contiguous: 8 consecutive rows of one k per load, scattered into
    // the k-contiguous tile (nrow % 8 == 0: a group lies wholly inside or out)
#pragma unroll
    for (int t = 0; t < (64 * BK / 8) / 256; ++t) {
      const int v = tid + 256 * t, c = v / (64 / 8), r = (v % (64 / 8)) * 8;
      const int row = r0 + r, k = k0 + c;
      uint4 q = make_uint4(0u, 0u, 0u, 0u);
      if (row < nrow && k < K) q = *(const uint4 *)(X + (long long)k * sk + row);
      const bf16 *e = (const bf16 *)&q;
#pragma unroll
      for (int i = 0; i < 8; ++i) S[r + i][c] = e[i];
    }
  } else {
    // one value per load; consecutive threads walk the contiguous index
    const bool kc = sk == 1;
#pragma unroll 4
    for (int t = 0; t < (64 * BK) / 256; ++t) {
      const int idx = tid + 256 * t;
      const int r = kc ? idx / BK : idx % 64;
      const int c = kc ? idx % BK : idx / 64;
      const int row = r0 + r, k = k0 + c;
      S[r][c] = (row < nrow && k < K) ? X[(long long)row * srow + (long long)k * sk] : (bf16)0;
    }
  }
}

__global__ __launch_bounds__(256) void k_gemm(Gemm g) {
  __shared__ __attribute__((aligned(16))) bf16 As[BM][LDK];
  __shared__ __attribute__((aligned(16))) bf16 Bs[BN][LDK];
  const int z = blockIdx.z;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  const bf16 *A = g.A + (long long)z * g.saz;
  const bf16 *B = g.B + (long long)z * g.sbz;
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < g.K; k0 += BK) {
    // A(m, k) rows m; B(k, n) staged as rows n
    stage(As, A, g.sam, g.sak, g.M, g.K, m0, k0, tid);
    stage(Bs, B, g.sbn, g.sbk, g.N, g.K, n0, k0, tid);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      v8bf a[2], b[2];
      const int q = kk + 8 * (lane >> 4);
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = *(const v8bf *)&As[wm + 16 * i + (lane & 15)][q];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = *(const v8bf *)&Bs[wn + 16 * j + (lane & 15)][q];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int n = n0 + wn + 16 * j + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        const long long o = (long long)m * g.N + n;
        float s = acc[i][j][r];
        switch (g.epi) {
          case kEpiF32:
            g.C[(long long)z * g.scz + o] = s;
            break;
          case kEpiBiasF32:
            g.C[(long long)z * g.scz + o] = s + g.bias[(long long)z * g.bstride + n];
            break;
          case kEpiBiasSilu: {
            const float zz = s + g.bias[(long long)z * g.bstride + n];
            g.C[(long long)z * g.scz + o] = zz;
            g.Cb[(long long)z * g.sbzc + o] = to_bf16(silu(zz));
            break;
          }
          default: {  // kEpiDsilu
            const float d = s * dsilu(g.Zin[(long long)z * g.szz + o]);
            g.C[(long long)z * g.scz + o] = d;
            g.Cb[(long long)z * g.sbzc + o] = to_bf16(d);
            break;
          }
        }
      }
}

hipError_t launch_gemm(const Gemm &g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0 || g.members <= 0) return hipSuccess;
  dim3 grid((unsigned)((g.N + BN - 1) / BN), (unsigned)((g.M + BM - 1) / BM), (unsigned)g.members);
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

// ---- fixed-order block reduction (FP64) -------------------------------------
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_col_stats(const double *X, int n, int cols, double *mu,
                                                   double *sd) {
  __shared__ double sh[256];
  const int c = blockIdx.x;
  double s = 0;
  for (int i = threadIdx.x; i < n; i += 256) s += X[(long long)i * cols + c];
  const double mean = block_sum<256>(s, sh) / n;
  double q = 0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double d = X[(long long)i * cols + c] - mean;
    q += d * d;
  }
  const double var = block_sum<256>(q, sh) / n;
  if (threadIdx.x == 0) {
    mu[c] = mean;
    const double s2 = sqrt(var);
    sd[c] = s2 < 1e-12 ? 1.0 : s2;
  }
}

hipError_t launch_col_stats(const double *X, int n, int cols, double *mu, double *sd,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_col_stats, dim3((unsigned)cols), dim3(256), 0, st, X, n, cols, mu, sd);
  return hipGetLastError();
}

__global__ void k_standardise(const double *X, long long total, int cols, const double *mu,
                              const double *sd, float *Y) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int c = (int)(i % cols);
  Y[i] = (float)((X[i] - mu[c]) / sd[c]);
}

hipError_t launch_standardise(const double *X, int n, int cols, const double *mu,
                              const double *sd, float *Y, hipStream_t st) {
  const long long total = (long long)n * cols;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_standardise, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, X,
                     total, cols, mu, sd, Y);
  return hipGetLastError();
}

__global__ void k_gather(const float *X, const float *T, const int *idx, long long idx_stride,
                         int members, int bsz, long long cap, bf16 *A0, float *T0) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long per = (long long)bsz * (kFeat + kOut);
  if (i >= per * members) return;
  const int z = (int)(i / per);
  const long long r = i % per;
  const int b = (int)(r / (kFeat + kOut)), c = (int)(r % (kFeat + kOut));
  const long long src = idx ? idx[z * idx_stride + b] : b;
  if (c < kFeat)
    A0[(long long)z * cap * kFeat + (long long)b * kFeat + c] = to_bf16(X[src * kFeat + c]);
  else if (T)
    T0[(long long)z * cap * kOut + (long long)b * kOut + (c - kFeat)] = T[src * kOut + (c - kFeat)];
}

hipError_t launch_gather(const float *X, const float *T, const int *idx, long long idx_stride,
                         int members, int bsz, long long cap, bf16 *A0, float *T0,
                         hipStream_t st) {
  const long long total = (long long)members * bsz * (kFeat + kOut);
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, X, T, idx,
                     idx_stride, members, bsz, cap, A0, T0);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_loss_grad(const float *Y, const float *T, int bsz,
                                                   long long cap, float *dY, bf16 *dYb,
                                                   double *loss) {
  __shared__ double sh[256];
  const int z = blockIdx.x;
  const long long base = (long long)z * cap * kOut;
  const int cnt = bsz * kOut;
  const float sc = 2.0f / (float)cnt;
  double s = 0;
  for (int i = threadIdx.x; i < cnt; i += 256) {
    const float d = Y[base + i] - T[base + i];
    const float gd = sc * d;
    dY[base + i] = gd;
    dYb[base + i] = to_bf16(gd);
    s += (double)d * (double)d;
  }
  const double tot = block_sum<256>(s, sh);
  if (threadIdx.x == 0) loss[z] = tot / cnt;
}

hipError_t launch_loss_grad(const float *Y, const float *T, int members, int bsz, long long cap,
                            float *dY, bf16 *dYb, double *loss, hipStream_t st) {
  hipLaunchKernelGGL(k_loss_grad, dim3((unsigned)members), dim3(256), 0, st, Y, T, bsz, cap, dY,
                     dYb, loss);
  return hipGetLastError();
}

__global__ void k_bias_grad(const float *D, int bsz, int N, long long cap, float *db,
                            long long pstride) {
  const int z = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const float *d = D + (long long)z * cap * N + n;
  float s = 0.f;
  for (int b = 0; b < bsz; ++b) s += d[(long long)b * N];
  db[(long long)z * pstride + n] = s;
}

hipError_t launch_bias_grad(const float *D, int members, int bsz, int N, long long cap, float *db,
                            long long pstride, hipStream_t st) {
  hipLaunchKernelGGL(k_bias_grad, dim3((unsigned)((N + 255) / 256), (unsigned)members), dim3(256),
                     0, st, D, bsz, N, cap, db, pstride);
  return hipGetLastError();
}

__global__ void k_adam(float *w, const float *g, float *m, float *v, bf16 *wb, long long count,
                       float lr, float b1, float b2, float eps, float bc1, float bc2) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  w[i] = wi;
  wb[i] = to_bf16(wi);
}

hipError_t launch_adam(float *w, const float *g, float *m, float *v, bf16 *wb, long long count,
                       float lr, float b1, float b2, float eps, float bc1, float bc2,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, w, g, m, v,
                     wb, count, lr, b1, b2, eps, bc1, bc2);
  return hipGetLastError();
}

__global__ void k_to_bf16(const float *w, bf16 *wb, long long count) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < count) wb[i] = to_bf16(w[i]);
}

hipError_t launch_to_bf16(const float *w, bf16 *wb, long long count, hipStream_t st) {
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, w, wb,
                     count);
  return hipGetLastError();
}

__global__ void k_ensemble(const float *Y, int members, int n, long long cap, const double *mu,
                           const double *sd, double *mean, double *std) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= (long long)n * kOut) return;
  const int j = (int)(i % kOut);
  double s = 0;
  for (int z = 0; z < members; ++z) s += (double)Y[(long long)z * cap * kOut + i] * sd[j] + mu[j];
  const double mn = s / members;
  double q = 0;
  for (int z = 0; z < members; ++z) {
    const double d = (double)Y[(long long)z * cap * kOut + i] * sd[j] + mu[j] - mn;
    q += d * d;
  }
  mean[i] = mn;
  std[i] = sqrt(q / members);
}

hipError_t launch_ensemble(const float *Y, int members, int n, long long cap, const double *mu,
                           const double *sd, double *mean, double *std, hipStream_t st) {
  const long long total = (long long)n * kOut;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ensemble, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, Y,
                     members, n, cap, mu, sd, mean, std);
  return hipGetLastError();
}

// ---- descriptor -------------------------------------------------------------
// One workgroup per pooled cell (8^3 samples) and throat.  Sample i of an axis
// of length n sits at (i + 0.5) n / 32 - 0.5 lattice units; the point is solid
// if it is in a sphere or outside the prism over the throat spheres 0..2.
__global__ __launch_bounds__(512) void k_describe(const double *geo, double *feat) {
  const int cell = blockIdx.x, t = blockIdx.y;
  const double *G = geo + (long long)t * 19;
  const double *S = G;  // 4 spheres (cx, cy, cz, r), throat spheres first
  const double nx = G[16], ny = G[17], nz = G[18];
  const int k = kOcc / kPool;
  const int cx = cell % k, cy = (cell / k) % k, cz = cell / (k * k);
  const int tid = threadIdx.x;
  const int ix = cx * kPool + tid % kPool, iy = cy * kPool + (tid / kPool) % kPool,
            iz = cz * kPool + tid / (kPool * kPool);
  const double px = __dsub_rn(__dmul_rn(__dmul_rn((double)ix + 0.5, nx), 1.0 / kOcc), 0.5);
  const double py = __dsub_rn(__dmul_rn(__dmul_rn((double)iy + 0.5, ny), 1.0 / kOcc), 0.5);
  const double pz = __dsub_rn(__dmul_rn(__dmul_rn((double)iz + 0.5, nz), 1.0 / kOcc), 0.5);
  bool solid = !geom::in_prism(S, S + 4, S + 8, px, py);
  for (int i = 0; i < 4 && !solid; ++i) solid = geom::in_sphere(px, py, pz, S + 4 * i);
  const int cnt = __syncthreads_count(solid);
  double *f = feat + (long long)t * kFeat;
  if (tid == 0) f[16 + cell] = (double)cnt / (double)(kPool * kPool * kPool);
  if (cell == 0 && tid < 16) {
    const double rbar = __ddiv_rn(__dadd_rn(__dadd_rn(S[3], S[7]), S[11]), 3.0);
    if (tid < 4) {
      f[tid] = __ddiv_rn(S[4 * tid + 3], rbar);
    } else {
      const int s = (tid - 4) / 3, a = (tid - 4) % 3;
      const double c = __ddiv_rn(__dadd_rn(__dadd_rn(S[a], S[4 + a]), S[8 + a]), 3.0);
      f[tid] = __ddiv_rn(__dsub_rn(S[4 * s + a], c), rbar);
    }
  }
}

hipError_t launch_describe(const double *geo, int n, double *feat, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int k = kOcc / kPool;
  hipLaunchKernelGGL(k_describe, dim3((unsigned)(k * k * k), (unsigned)n), dim3(512), 0, st, geo,
                     feat);
  return hipGetLastError();
}

}  // namespace sg
