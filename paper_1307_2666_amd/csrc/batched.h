// Per-panel batched kernels (batched.hip) for sub-levels with few large
// problems.  Internal, not part of the ABI.
#pragma once

#include "kernels.h"

namespace hif {

// Row compression problems (same fields as RowQrArgs); scratch per problem:
// V (m x 16) followed by T (16 x 16).
using QrBatch = RowQrArgs;
void launch_qr_batched(const QrBatch& A, int max_cols, hipStream_t s);

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
};
void launch_gemm_tiles(const GemmDesc* D, int nd, int max_m, int max_n, hipStream_t s);

}  // namespace hif
