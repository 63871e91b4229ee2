// Workgroup-level FP64 GEMM on the matrix cores (v_mfma_f64_16x16x4f64).
//
//   C (M x N) = beta C + alpha op(A) op(B),   op(A) is M x K, op(B) is K x N,
//
// all row-major in device memory; op(A)(i,k) = ta ? A[k*lda + i] : A[i*lda + k]
// and op(B)(k,j) = tb ? B[j*ldb + k] : B[k*ldb + j].  One workgroup of 256
// threads (4 waves, 2 x 2) computes 64 x 64 tiles of C one after another;
// operand tiles of depth 16 are staged through LDS.  Operand layout of the
// 16x16x4 FP64 instruction (wave64): A(i,k) in lane i + 16k, B(k,j) in lane
// j + 16k, result D(i,j) in lane j + 16 (i % 4), element i / 4.
#pragma once

#include "common.h"

namespace hif {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int kGemmTile = 64;
constexpr int kGemmK = 16;
// LDS doubles needed by wg_gemm: A tile [64][17] and B tile [16][65].
constexpr int kGemmLds = kGemmTile * (kGemmK + 1) + kGemmK * (kGemmTile + 1);

__device__ __forceinline__ double4_t mfma_f64(double a, double b, double4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Requires blockDim.x == 256.  Every thread of the workgroup must call it.
// C must not overlap A or B (unless beta == 0 and alpha == 0).
__device__ inline void wg_gemm(int M, int N, int K, double alpha, const double* __restrict__ A, int lda, bool ta,
                               const double* __restrict__ B, int ldb, bool tb, double beta, double* C, int ldc,
                               double* lds) {
  if (M <= 0 || N <= 0) return;
  double* sA = lds;                               // [64][17]
  double* sB = lds + kGemmTile * (kGemmK + 1);    // [16][65]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int wr = wv >> 1, wc = wv & 1;            // wave position in the 2 x 2 arrangement
  const int li = lane & 15, lk = lane >> 4;
  for (int tm = 0; tm < M; tm += kGemmTile) {
    for (int tn = 0; tn < N; tn += kGemmTile) {
      double4_t acc[2][2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = double4_t{0.0, 0.0, 0.0, 0.0};
      // Software pipeline: the next depth-16 slice is fetched into registers
      // while the matrix cores work on the current one.
      double ra[4], rb[4];
      auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + q * 256;
          int i, k;
          if (ta) { k = e >> 6; i = e & 63; } else { i = e >> 4; k = e & 15; }
          const int gi = tm + i, gk = k0 + k;
          ra[q] = (gi < M && gk < K) ? (ta ? A[int64_t(gk) * lda + gi] : A[int64_t(gi) * lda + gk]) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + q * 256;
          int k, j;
          if (tb) { j = e >> 4; k = e & 15; } else { k = e >> 6; j = e & 63; }
          const int gk = k0 + k, gj = tn + j;
          rb[q] = (gk < K && gj < N) ? (tb ? B[int64_t(gj) * ldb + gk] : B[int64_t(gk) * ldb + gj]) : 0.0;
        }
      };
      fetch(0);
      for (int k0 = 0; k0 < K; k0 += kGemmK) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + q * 256;
          int i, k;
          if (ta) { k = e >> 6; i = e & 63; } else { i = e >> 4; k = e & 15; }
          sA[i * (kGemmK + 1) + k] = ra[q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + q * 256;
          int k, j;
          if (tb) { j = e >> 4; k = e & 15; } else { k = e >> 6; j = e & 63; }
          sB[k * (kGemmTile + 1) + j] = rb[q];
        }
        __syncthreads();
        if (k0 + kGemmK < K) fetch(k0 + kGemmK);
#pragma unroll
        for (int kk = 0; kk < kGemmK; kk += 4) {
          double af[2], bf[2];
#pragma unroll
          for (int a = 0; a < 2; ++a) af[a] = sA[(wr * 32 + a * 16 + li) * (kGemmK + 1) + kk + lk];
#pragma unroll
          for (int b = 0; b < 2; ++b) bf[b] = sB[(kk + lk) * (kGemmTile + 1) + wc * 32 + b * 16 + li];
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = mfma_f64(af[a], bf[b], acc[a][b]);
        }
      }
      // write back
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int gi = tm + wr * 32 + a * 16 + 4 * v + lk;
            const int gj = tn + wc * 32 + b * 16 + li;
            if (gi < M && gj < N) {
              double* cp = C + int64_t(gi) * ldc + gj;
              const double r = alpha * acc[a][b][v];
              *cp = (beta == 0.0) ? r : beta * (*cp) + r;
            }
          }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// FP32 variant for the mixed-precision mode: same interface and tiling, the
// operands rounded to float as they are staged, v_mfma_f32_16x16x4f32 with
// FP32 accumulation, alpha / beta applied in FP64 on write-back.  Operand
// layout as above; result D(i,j) in lane j + 16 (i / 4), element i % 4.
// ---------------------------------------------------------------------------
typedef float float4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4_t mfma_f32(float a, float b, float4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Requires blockDim.x == 256 and kGemmLds doubles of LDS (uses half).
__device__ inline void wg_gemm_f32(int M, int N, int K, double alpha, const double* __restrict__ A, int lda, bool ta,
                                   const double* __restrict__ B, int ldb, bool tb, double beta, double* C, int ldc,
                                   double* lds) {
  if (M <= 0 || N <= 0) return;
  float* sA = reinterpret_cast<float*>(lds);      // [64][17]
  float* sB = sA + kGemmTile * (kGemmK + 1);      // [16][65]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int wr = wv >> 1, wc = wv & 1;
  const int li = lane & 15, lk = lane >> 4;
  for (int tm = 0; tm < M; tm += kGemmTile) {
    for (int tn = 0; tn < N; tn += kGemmTile) {
      float4_t acc[2][2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = float4_t{0.f, 0.f, 0.f, 0.f};
      float ra[4], rb[4];
      auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + q * 256;
          int i, k;
          if (ta) { k = e >> 6; i = e & 63; } else { i = e >> 4; k = e & 15; }
          const int gi = tm + i, gk = k0 + k;
          ra[q] = (gi < M && gk < K) ? float(ta ? A[int64_t(gk) * lda + gi] : A[int64_t(gi) * lda + gk]) : 0.f;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + q * 256;
          int k, j;
          if (tb) { j = e >> 4; k = e & 15; } else { k = e >> 6; j = e & 63; }
          const int gk = k0 + k, gj = tn + j;
          rb[q] = (gk < K && gj < N) ? float(tb ? B[int64_t(gj) * ldb + gk] : B[int64_t(gk) * ldb + gj]) : 0.f;
        }
      };
      fetch(0);
      for (int k0 = 0; k0 < K; k0 += kGemmK) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + q * 256;
          int i, k;
          if (ta) { k = e >> 6; i = e & 63; } else { i = e >> 4; k = e & 15; }
          sA[i * (kGemmK + 1) + k] = ra[q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + q * 256;
          int k, j;
          if (tb) { j = e >> 4; k = e & 15; } else { k = e >> 6; j = e & 63; }
          sB[k * (kGemmTile + 1) + j] = rb[q];
        }
        __syncthreads();
        if (k0 + kGemmK < K) fetch(k0 + kGemmK);
#pragma unroll
        for (int kk = 0; kk < kGemmK; kk += 4) {
          float af[2], bf[2];
#pragma unroll
          for (int a = 0; a < 2; ++a) af[a] = sA[(wr * 32 + a * 16 + li) * (kGemmK + 1) + kk + lk];
#pragma unroll
          for (int b = 0; b < 2; ++b) bf[b] = sB[(kk + lk) * (kGemmTile + 1) + wc * 32 + b * 16 + li];
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = mfma_f32(af[a], bf[b], acc[a][b]);
        }
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int gi = tm + wr * 32 + a * 16 + 4 * lk + v;
            const int gj = tn + wc * 32 + b * 16 + li;
            if (gi < M && gj < N) {
              double* cp = C + int64_t(gi) * ldc + gj;
              const double r = alpha * double(acc[a][b][v]);
              *cp = (beta == 0.0) ? r : beta * (*cp) + r;
            }
          }
    }
  }
  __syncthreads();
}

}  // namespace hif
