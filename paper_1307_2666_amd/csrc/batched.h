// Per-panel batched kernels (batched.hip) for sub-levels with few large
// problems.  Internal, not part of the ABI.
#pragma once

#include <vector>

#include "kernels.h"

namespace hif {

// Row compression problems (same fields as RowQrArgs).
using QrBatch = RowQrArgs;
// Few large problems: max_rows/max_cols bound rows/cols over the batch.
void launch_qr_batched(const QrBatch& A, int max_rows, int max_cols, hipStream_t s);

// Row compression of problems taller than one TSQR stack holds (more than
// kTsqrSplitRows rows), from host copies of the problems' offsets (from
// base), leading dimensions, rows and columns: each is cut into row blocks
// factored as problems of their own, whose R factors are stacked and factored
// again.  Leaves R0 in the leading n x n block of every problem with m > n,
// as launch_qr_batched does.
// Blocks have at least half kTsqrSplitRows rows, and at least twice the
// columns for up to 16384 columns, so each round shrinks the stack.
constexpr int kTsqrSplitRows = 32768;
inline bool rowqr_split_fits(int max_rows, int max_cols) {
  return max_rows > kTsqrSplitRows && max_cols <= kTsqrSplitRows / 2;
}
void launch_rowqr_split(double* base, const std::vector<int64_t>& moff, const std::vector<int32_t>& ld,
                        const std::vector<int32_t>& rows, const std::vector<int32_t>& cols, MemTracker* mt,
                        hipStream_t s);

// Communication-avoiding panels of the row compression: panel width, rows per
// chunk (one per thread) and the largest stack of chunk R factors.
constexpr int kTsqrNb = 32;
constexpr int kTsqrRows = 256;
constexpr int kTsqrStack = 1024;
__host__ __device__ inline int tsqr_chunks(int mp) { return (mp + kTsqrRows - 1) / kTsqrRows; }
// Scratch of one problem with m rows (doubles): V (m x nb) | T per chunk |
// stacked R | stacked V | stack T.
struct TsqrLayout {
  int64_t V, Tc, S, Vs, Ts, total;
};
__host__ __device__ inline TsqrLayout tsqr_layout(int m) {
  const int64_t nm = tsqr_chunks(m), b2 = int64_t(kTsqrNb) * kTsqrNb;
  TsqrLayout L;
  L.V = 0;
  L.Tc = int64_t(m) * kTsqrNb;
  L.S = L.Tc + nm * b2;
  L.Vs = L.S + nm * b2;
  L.Ts = L.Vs + nm * b2;
  L.total = L.Ts + b2;
  return L;
}
// Scratch doubles every row-compression path needs for an m x n problem
// (m > n); the TSQR panels alternate between two copies of the layout.
inline int64_t rowqr_scratch(int64_t m, int64_t n) {
  const int64_t fused = m * 16 + 16 * n + 256;
  const int64_t tsqr = 2 * tsqr_layout(int(m)).total;
  return fused > tsqr ? fused : tsqr;
}

// Partial LU problems: n x n row-major blocks (leading dimension n) factored
// over their first r columns with pivots among rows < r.
struct LuBatch {
  double* base;
  const int64_t* moff;
  const int32_t* n;
  const int32_t* r;
  int32_t* piv;           // pivots of problem q at piv + poff[q]
  const int64_t* poff;
  int32_t* status;
  int nprob = 0;
  int fp32 = 0;  // mixed precision: trailing tiles inside the skeleton block on FP32 matrix cores
};
void launch_lu_batched(const LuBatch& A, int max_r, int max_n, hipStream_t s);

// One entry of a batched GEMM: C = beta C + alpha op(A) op(B).
struct GemmDesc {
  int M, N, K;
  int ta, tb;
  int lda, ldb, ldc;
  double alpha, beta;
  const double* A;
  const double* B;
  double* C;
  int fp32 = 0;  // mixed precision: FP32 matrix cores, FP32 accumulation
};
void launch_gemm_tiles(const GemmDesc* D, int nd, int max_m, int max_n, hipStream_t s);

}  // namespace hif
