// Factored apply / solve sweeps: F = U_0^{-T} ... D ... V_0^{-1} and
// F^{-1} = V_0 ... D^{-1} ... U_0^T (eqns rskelf, hifie2, hifie3) and their
// transposes.  A group record holds T, the row-pivoted LU of B_rr
// (P B_rr = L U), L_sr = B_sr U^{-1} and U_rs = L^{-1} P B_rs (the operators
// R_p, S_p of Lemma 2.1 with Q = [I 0; -T I] of Lemma 2.4, (redundant,
// skeleton) order).  Per group:
//   solve   up:   u_r -= T^T u_s;  u_r = L^{-1} P u_r;     u_s -= L_sr u_r
//           down: u_r -= U_rs u_s; u_r = U^{-1} u_r;       u_s -= T u_r
//   solve_T up:   u_r -= T^T u_s;  u_r = U^{-T} u_r;       u_s -= U_rs^T u_r
//           down: u_r -= L_sr^T u_s; u_r = P^T L^{-T} u_r; u_s -= T u_r
//   apply   up:   x_s += T x_r;    x_r = U x_r + U_rs x_s
//           down: y_s += L_sr y_r; y_r = P^T L y_r;        y_r += T^T y_s
//   apply_T up:   x_s += T x_r;    x_r = L^T P x_r + L_sr^T x_s
//           down: y_s += U_rs^T y_r; y_r = U^T y_r;        y_r += T^T y_s
// with the top block A_L (LU with pivoting) solved or applied in between.
// "up" visits sub-levels finest first, "down" in reverse; the groups of one
// sub-level touch disjoint DOFs and run as one launch, one workgroup each.
// Vectors are [nrhs][N] in the caller's order; every product works in place
// through the records' global DOF indices.
#include <mutex>
#include <string>
#include <type_traits>

#include "common.h"
#include "wave.h"

namespace hif {

namespace {

constexpr int kBlock = 256;

struct SwArgs {
  const GroupRec* recs;
  const int32_t* iarena;
  const double* darena;
  double* u;
  double* work;
  int64_t N;
  int nrhs;
  int op;
};

// u[yi[i]] += sgn * sum_j M[i*ld + j] u[xi[j]]   (one wave per row)
__device__ void gemv_rows(const double* M, int nrow, int ncol, int ld, const int32_t* yi, const int32_t* xi,
                          double* u, int64_t N, int nrhs, double sgn) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int i = wv; i < nrow; i += nw) {
    const double* mr = M + int64_t(i) * ld;
    for (int v = 0; v < nrhs; ++v) {
      const double* uv = u + v * N;
      double s = 0.0;
      for (int j = lane; j < ncol; j += 64) s += mr[j] * uv[xi[j]];
      s = wave_sum(s);
      if (lane == 0) u[v * N + yi[i]] += sgn * s;
    }
  }
}

// u[yi[j]] += sgn * sum_i M[i*ld + j] u[xi[i]]   (one thread per column and RHS)
__device__ void gemv_cols(const double* M, int nrow, int ncol, int ld, const int32_t* yi, const int32_t* xi,
                          double* u, int64_t N, int nrhs, double sgn) {
  for (int e = threadIdx.x; e < ncol * nrhs; e += blockDim.x) {
    const int j = e % ncol, v = e / ncol;
    const double* uv = u + v * N;
    double s = 0.0;
    for (int i = 0; i < nrow; ++i) s += M[int64_t(i) * ld + j] * uv[xi[i]];
    u[v * N + yi[j]] += sgn * s;
  }
}

// Triangular pieces on u_r = u[v*N + idx[i]], i < n, all RHS; LU is n x n
// row-major holding unit-lower L and upper U; piv the row interchanges.
__device__ void swaps_fwd(const int32_t* piv, int n, const int32_t* idx, double* u, int64_t N, int nrhs) {
  for (int v = threadIdx.x; v < nrhs; v += blockDim.x)
    for (int j = 0; j < n; ++j)
      if (piv[j] != j) {
        double* a = u + v * N + idx[j];
        double* b = u + v * N + idx[piv[j]];
        const double t = *a; *a = *b; *b = t;
      }
  __syncthreads();
}
__device__ void swaps_rev(const int32_t* piv, int n, const int32_t* idx, double* u, int64_t N, int nrhs) {
  for (int v = threadIdx.x; v < nrhs; v += blockDim.x)
    for (int j = n - 1; j >= 0; --j)
      if (piv[j] != j) {
        double* a = u + v * N + idx[j];
        double* b = u + v * N + idx[piv[j]];
        const double t = *a; *a = *b; *b = t;
      }
  __syncthreads();
}
// x = L^{-1} x (unit lower), column oriented
__device__ void solve_L(const double* LU, int n, const int32_t* idx, double* u, int64_t N, int nrhs) {
  for (int j = 0; j < n - 1; ++j) {
    const int w = n - 1 - j;
    for (int e = threadIdx.x; e < w * nrhs; e += blockDim.x) {
      const int i = j + 1 + e % w, v = e / w;
      u[v * N + idx[i]] -= LU[int64_t(i) * n + j] * u[v * N + idx[j]];
    }
    __syncthreads();
  }
  __syncthreads();
}
// x = U^{-1} x
__device__ void solve_U(const double* LU, int n, const int32_t* idx, double* u, int64_t N, int nrhs) {
  for (int j = n - 1; j >= 0; --j) {
    const double inv = 1.0 / LU[int64_t(j) * n + j];
    for (int e = threadIdx.x; e < j * nrhs; e += blockDim.x) {
      const int i = e % j, v = e / j;
      u[v * N + idx[i]] -= LU[int64_t(i) * n + j] * (u[v * N + idx[j]] * inv);
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < n * nrhs; e += blockDim.x) {
    const int i = e % n, v = e / n;
    u[v * N + idx[i]] /= LU[int64_t(i) * n + i];
  }
  __syncthreads();
}
// x = U^{-T} x (U^T lower)
__device__ void solve_UT(const double* LU, int n, const int32_t* idx, double* u, int64_t N, int nrhs) {
  for (int j = 0; j < n; ++j) {
    const double inv = 1.0 / LU[int64_t(j) * n + j];
    const int w = n - 1 - j;
    for (int e = threadIdx.x; e < w * nrhs; e += blockDim.x) {
      const int i = j + 1 + e % w, v = e / w;
      u[v * N + idx[i]] -= LU[int64_t(j) * n + i] * (u[v * N + idx[j]] * inv);
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < n * nrhs; e += blockDim.x) {
    const int i = e % n, v = e / n;
    u[v * N + idx[i]] /= LU[int64_t(i) * n + i];
  }
  __syncthreads();
}
// x = L^{-T} x (L^T unit upper)
__device__ void solve_LT(const double* LU, int n, const int32_t* idx, double* u, int64_t N, int nrhs) {
  for (int j = n - 1; j > 0; --j) {
    for (int e = threadIdx.x; e < j * nrhs; e += blockDim.x) {
      const int i = e % j, v = e / j;
      u[v * N + idx[i]] -= LU[int64_t(j) * n + i] * u[v * N + idx[j]];
    }
    __syncthreads();
  }
  __syncthreads();
}
// x = op(x) through the work buffer: mode 0: U x, 1: L x, 2: L^T x, 3: U^T x
__device__ void tri_mul(const double* LU, int n, const int32_t* idx, double* u, double* work, int64_t N, int nrhs,
                        int mode) {
  for (int e = threadIdx.x; e < n * nrhs; e += blockDim.x) {
    const int i = e % n, v = e / n;
    const double* uv = u + v * N;
    double s = 0.0;
    if (mode == 0) {
      for (int j = i; j < n; ++j) s += LU[int64_t(i) * n + j] * uv[idx[j]];
    } else if (mode == 1) {
      s = uv[idx[i]];
      for (int j = 0; j < i; ++j) s += LU[int64_t(i) * n + j] * uv[idx[j]];
    } else if (mode == 2) {
      s = uv[idx[i]];
      for (int j = i + 1; j < n; ++j) s += LU[int64_t(j) * n + i] * uv[idx[j]];
    } else {
      for (int j = 0; j <= i; ++j) s += LU[int64_t(j) * n + i] * uv[idx[j]];
    }
    work[v * N + idx[i]] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * nrhs; e += blockDim.x) {
    const int i = e % n, v = e / n;
    u[v * N + idx[i]] = work[v * N + idx[i]];
  }
  __syncthreads();
}

__global__ void k_up(SwArgs A) {
  const GroupRec R = A.recs[blockIdx.x];
  const int r = R.r, k = R.k;
  const int32_t* rd = A.iarena + R.idx;
  const int32_t* sk = rd + r;
  const int32_t* piv = sk + k;
  const double* T = A.darena + R.off;
  const double* Lsr = T + int64_t(k) * r;
  const double* Urs = Lsr + int64_t(k) * r;
  const double* LU = Urs + int64_t(r) * k;
  double* u = A.u;
  const int64_t N = A.N;
  const int nr = A.nrhs;
  if (A.op <= 1) {
    if (k > 0) gemv_cols(T, k, r, r, rd, sk, u, N, nr, -1.0);  // u_r -= T^T u_s
    __syncthreads();
    if (A.op == 0) {
      swaps_fwd(piv, r, rd, u, N, nr);
      solve_L(LU, r, rd, u, N, nr);
      if (k > 0) gemv_rows(Lsr, k, r, r, sk, rd, u, N, nr, -1.0);  // u_s -= L_sr u_r
    } else {
      solve_UT(LU, r, rd, u, N, nr);
      if (k > 0) gemv_cols(Urs, r, k, k, sk, rd, u, N, nr, -1.0);  // u_s -= U_rs^T u_r
    }
  } else {
    if (k > 0) gemv_rows(T, k, r, r, sk, rd, u, N, nr, 1.0);  // x_s += T x_r
    __syncthreads();
    if (A.op == 2) {
      tri_mul(LU, r, rd, u, A.work, N, nr, 0);                     // x_r = U x_r
      if (k > 0) gemv_rows(Urs, r, k, k, rd, sk, u, N, nr, 1.0);   //      + U_rs x_s
    } else {
      swaps_fwd(piv, r, rd, u, N, nr);
      tri_mul(LU, r, rd, u, A.work, N, nr, 2);                     // x_r = L^T P x_r
      if (k > 0) gemv_cols(Lsr, k, r, r, rd, sk, u, N, nr, 1.0);   //      + L_sr^T x_s
    }
  }
}

__global__ void k_down(SwArgs A) {
  const GroupRec R = A.recs[blockIdx.x];
  const int r = R.r, k = R.k;
  const int32_t* rd = A.iarena + R.idx;
  const int32_t* sk = rd + r;
  const int32_t* piv = sk + k;
  const double* T = A.darena + R.off;
  const double* Lsr = T + int64_t(k) * r;
  const double* Urs = Lsr + int64_t(k) * r;
  const double* LU = Urs + int64_t(r) * k;
  double* u = A.u;
  const int64_t N = A.N;
  const int nr = A.nrhs;
  if (A.op <= 1) {
    if (A.op == 0) {
      if (k > 0) gemv_rows(Urs, r, k, k, rd, sk, u, N, nr, -1.0);  // u_r -= U_rs u_s
      __syncthreads();
      solve_U(LU, r, rd, u, N, nr);
    } else {
      if (k > 0) gemv_cols(Lsr, k, r, r, rd, sk, u, N, nr, -1.0);  // u_r -= L_sr^T u_s
      __syncthreads();
      solve_LT(LU, r, rd, u, N, nr);
      swaps_rev(piv, r, rd, u, N, nr);
    }
    if (k > 0) gemv_rows(T, k, r, r, sk, rd, u, N, nr, -1.0);  // u_s -= T u_r
  } else {
    if (A.op == 2) {
      if (k > 0) gemv_rows(Lsr, k, r, r, sk, rd, u, N, nr, 1.0);  // y_s += L_sr y_r
      __syncthreads();
      tri_mul(LU, r, rd, u, A.work, N, nr, 1);                    // y_r = P^T L y_r
      swaps_rev(piv, r, rd, u, N, nr);
    } else {
      if (k > 0) gemv_cols(Urs, r, k, k, sk, rd, u, N, nr, 1.0);  // y_s += U_rs^T y_r
      __syncthreads();
      tri_mul(LU, r, rd, u, A.work, N, nr, 3);                    // y_r = U^T y_r
    }
    if (k > 0) gemv_cols(T, k, r, r, rd, sk, u, N, nr, 1.0);  // y_r += T^T y_s
  }
}

// Block solve / multiply with an LU factorization P B = L U (row interchanges
// j <-> piv[j] applied in order j = 0..n-1), on the entries u[v*N + idx[i]].
__device__ void lu_op(const double* LU, const int32_t* piv, int n, const int32_t* idx, double* u, double* work,
                      int64_t N, int nrhs, int op) {
  const int tid = threadIdx.x, B = blockDim.x;
  auto X = [&](int i, int v) -> double& { return u[v * N + idx[i]]; };
  auto W = [&](int i, int v) -> double& { return work[v * N + idx[i]]; };
  if (op == 0) {  // x = B^{-1} x = U^{-1} L^{-1} P x
    for (int v = tid; v < nrhs; v += B)
      for (int j = 0; j < n; ++j)
        if (piv[j] != j) { double t = X(j, v); X(j, v) = X(piv[j], v); X(piv[j], v) = t; }
    __syncthreads();
    for (int j = 0; j < n - 1; ++j) {
      const int w = n - 1 - j;
      for (int e = tid; e < w * nrhs; e += B) {
        const int i = j + 1 + e % w, v = e / w;
        X(i, v) -= LU[int64_t(i) * n + j] * X(j, v);
      }
      __syncthreads();
    }
    for (int j = n - 1; j >= 0; --j) {
      const double inv = 1.0 / LU[int64_t(j) * n + j];
      for (int e = tid; e < j * nrhs; e += B) {
        const int i = e % j, v = e / j;
        X(i, v) -= LU[int64_t(i) * n + j] * (X(j, v) * inv);
      }
      __syncthreads();
    }
    for (int e = tid; e < n * nrhs; e += B) {
      const int i = e % n, v = e / n;
      X(i, v) /= LU[int64_t(i) * n + i];
    }
  } else if (op == 1) {  // x = B^{-T} x = P^T L^{-T} U^{-T} x
    for (int j = 0; j < n; ++j) {
      const double inv = 1.0 / LU[int64_t(j) * n + j];
      const int w = n - 1 - j;
      for (int e = tid; e < w * nrhs; e += B) {
        const int i = j + 1 + e % w, v = e / w;
        X(i, v) -= LU[int64_t(j) * n + i] * (X(j, v) * inv);
      }
      __syncthreads();
    }
    for (int e = tid; e < n * nrhs; e += B) {
      const int i = e % n, v = e / n;
      X(i, v) /= LU[int64_t(i) * n + i];
    }
    __syncthreads();
    for (int j = n - 1; j > 0; --j) {
      for (int e = tid; e < j * nrhs; e += B) {
        const int i = e % j, v = e / j;
        X(i, v) -= LU[int64_t(j) * n + i] * X(j, v);
      }
      __syncthreads();
    }
    for (int v = tid; v < nrhs; v += B)
      for (int j = n - 1; j >= 0; --j)
        if (piv[j] != j) { double t = X(j, v); X(j, v) = X(piv[j], v); X(piv[j], v) = t; }
  } else if (op == 2) {  // x = B x = P^T L U x
    for (int e = tid; e < n * nrhs; e += B) {
      const int i = e % n, v = e / n;
      double s = 0.0;
      for (int j = i; j < n; ++j) s += LU[int64_t(i) * n + j] * X(j, v);
      W(i, v) = s;
    }
    __syncthreads();
    for (int e = tid; e < n * nrhs; e += B) {
      const int i = e % n, v = e / n;
      double s = W(i, v);
      for (int j = 0; j < i; ++j) s += LU[int64_t(i) * n + j] * W(j, v);
      X(i, v) = s;
    }
    __syncthreads();
    for (int v = tid; v < nrhs; v += B)
      for (int j = n - 1; j >= 0; --j)
        if (piv[j] != j) { double t = X(j, v); X(j, v) = X(piv[j], v); X(piv[j], v) = t; }
  } else {  // x = B^T x = U^T L^T P x
    for (int v = tid; v < nrhs; v += B)
      for (int j = 0; j < n; ++j)
        if (piv[j] != j) { double t = X(j, v); X(j, v) = X(piv[j], v); X(piv[j], v) = t; }
    __syncthreads();
    for (int e = tid; e < n * nrhs; e += B) {
      const int i = e % n, v = e / n;
      double s = X(i, v);
      for (int j = i + 1; j < n; ++j) s += LU[int64_t(j) * n + i] * X(j, v);
      W(i, v) = s;
    }
    __syncthreads();
    for (int e = tid; e < n * nrhs; e += B) {
      const int i = e % n, v = e / n;
      double s = 0.0;
      for (int j = 0; j <= i; ++j) s += LU[int64_t(j) * n + i] * W(j, v);
      X(i, v) = s;
    }
  }
}

__global__ void k_top(const double* LU, const int32_t* piv, int n, const int32_t* idx, double* u, double* work,
                      int64_t N, int nrhs, int op) {
  lu_op(LU, piv, n, idx, u, work, N, nrhs, op);
}

// ---------------------------------------------------------------------------
// LDS-staged solve / solve_T.  The entries u_r, u_s of a group (or the top
// block's entries) are gathered into LDS once; the products and the blocked
// triangular solves (64-column diagonal blocks solved by one wave with
// shuffles, then one update of the remaining rows) run there, and the results
// are scattered back.  The row interchanges use the gather index perm,
// (P x)[i] = x[perm[i]].
// ---------------------------------------------------------------------------
constexpr int kNbT = 64;
constexpr int kMaxV = 8;       // right-hand sides per pass
static_assert(kMaxV == 8, "the row products reduce their kMaxV sums with wave_rs8, 4 rows with wave_rs32");
constexpr int kCapL = 16384;   // LDS doubles, largest records and the top block
// Sub-levels with at least this many records run 64, 128 or 256 threads per
// record (launch-shape table), fewer records 1024 threads each.
constexpr int kManyRecords = 1024;
// Top blocks of at least this many unknowns are solved by the many-workgroup
// blocked triangular solves (one workgroup is latency-bound there).
constexpr int64_t kTopSplitMin = 512;

// The helpers below issue their global loads eight at a time before using
// them, so that a single workgroup (one per large group) keeps many requests
// in flight.  Indices past a block are guarded on both factors.
constexpr int kU = 8;

// y[v*ys + i] += sgn * sum_j M[i*ld + j] x[v*xs + j]   (one wave per row)
__device__ __forceinline__ void l_gemv_n(const double* __restrict__ M, int nrow, int ncol, int ld, const double* x, int xs, double* y,
                         int ys, int nv, double sgn) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (ncol <= 64) {
    // rows of at most one element per lane: x in registers, four rows of the
    // wave at a time with their loads issued together
    double xv[kMaxV];
#pragma unroll
    for (int v = 0; v < kMaxV; ++v) xv[v] = (v < nv && lane < ncol) ? x[v * xs + lane] : 0.0;
    for (int i0 = wv; i0 < nrow; i0 += 4 * nw) {
      double m[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + q * nw;
        m[q] = (i < nrow && lane < ncol) ? M[int64_t(i) * ld + lane] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + q * nw;
        if (i < nrow) {
          double acc[kMaxV];
#pragma unroll
          for (int v = 0; v < kMaxV; ++v) acc[v] = m[q] * xv[v];
          const double t = wave_rs8(acc);
          const int v = lane >> 3;
          if ((lane & 7) == 0 && v < nv) y[v * ys + i] += sgn * t;
        }
      }
    }
    return;
  }
  if (ncol <= 128) {
    // rows of at most two entries per lane: four rows of the wave at a time,
    // their eight loads issued together, x read from LDS (no more registers
    // than one row at a time); each sum in the order of the general path
    for (int i0 = wv; i0 < nrow; i0 += 4 * nw) {
      double m[4][2];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + q * nw;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int j = 64 * h + lane;
          m[q][h] = (i < nrow && j < ncol) ? M[int64_t(i) * ld + j] : 0.0;
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + q * nw;
        if (i < nrow) {
          double acc[kMaxV];
#pragma unroll
          for (int v = 0; v < kMaxV; ++v) acc[v] = 0.0;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int j = 64 * h + lane;
            if (j < ncol) {
#pragma unroll
              for (int v = 0; v < kMaxV; ++v)
                if (v < nv) acc[v] += m[q][h] * x[v * xs + j];
            }
          }
          const double t = wave_rs8(acc);
          const int v = lane >> 3;
          if ((lane & 7) == 0 && v < nv) y[v * ys + i] += sgn * t;
        }
      }
    }
    return;
  }
  for (int i = wv; i < nrow; i += nw) {
    const double* mr = M + int64_t(i) * ld;
    double acc[kMaxV];
#pragma unroll
    for (int v = 0; v < kMaxV; ++v) acc[v] = 0.0;
    for (int j0 = 0; j0 < ncol; j0 += 64 * kU) {
      double mv[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int j = j0 + u * 64 + lane;
        mv[u] = j < ncol ? mr[j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int j = j0 + u * 64 + lane;
        if (j < ncol) {
#pragma unroll
          for (int v = 0; v < kMaxV; ++v)
            if (v < nv) acc[v] += mv[u] * x[v * xs + j];
        }
      }
    }
    // the 8 right-hand sides' sums at once: lane l holds that of l >> 3
    const double t = wave_rs8(acc);
    const int v = lane >> 3;
    if ((lane & 7) == 0 && v < nv) y[v * ys + i] += sgn * t;
  }
}

// y[v*ys + j] += sgn * sum_i M[i*ld + j] x[v*xs + i]   (one thread per column).
// With few columns the waves split the rows: wave w takes column group
// w % ncg (64 columns) and row slice w / ncg (at most 4 slices), and the
// slices add their partial sums in slice order (deterministic).  Every
// thread of the workgroup calls it; it ends synchronized.
__device__ __forceinline__ void l_gemv_t(const double* __restrict__ M, int nrow, int ncol, int ld, const double* x, int xs, double* y,
                         int ys, int nv, double sgn) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (ncol <= 0 || nrow <= 0) {
    __syncthreads();
    return;
  }
  const int ncg = (ncol + 63) / 64;
  const int nrs = ncg <= nw ? min(4, nw / ncg) : 1;
  const bool split = ncg <= nw;
  const int cg = split ? wv % ncg : 0, rs = split ? wv / ncg : 0;
  const bool active = !split || wv < ncg * nrs;
  const int ib = split ? (nrow * rs) / nrs : 0, ie = split ? (nrow * (rs + 1)) / nrs : nrow;
  double acc[kMaxV];
  for (int j = split ? cg * 64 + lane : threadIdx.x; active && j < ncol; j += split ? ncol : blockDim.x) {
#pragma unroll
    for (int v = 0; v < kMaxV; ++v) acc[v] = 0.0;
    for (int i0 = ib; i0 < ie; i0 += kU) {
      double mv[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) mv[u] = i0 + u < ie ? M[int64_t(i0 + u) * ld + j] : 0.0;
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (i0 + u < ie) {
#pragma unroll
          for (int v = 0; v < kMaxV; ++v)
            if (v < nv) acc[v] += mv[u] * x[v * xs + i0 + u];
        }
    }
    if (!split)
#pragma unroll
      for (int v = 0; v < kMaxV; ++v)
        if (v < nv) y[v * ys + j] += sgn * acc[v];
  }
  if (split) {
    const int j = cg * 64 + lane;
    for (int p = 0; p < nrs; ++p) {
      __syncthreads();
      if (active && rs == p && j < ncol)
#pragma unroll
        for (int v = 0; v < kMaxV; ++v)
          if (v < nv) y[v * ys + j] += sgn * acc[v];
    }
  }
  __syncthreads();
}

// x = L^{-1} x, L the unit lower triangle of the row-major n x n LU.
__device__ __forceinline__ void l_solve_L(const double* __restrict__ LU, int n, double* x, int xs, int nv) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
  for (int j0 = 0; j0 < n; j0 += kNbT) {
    const int nb = min(kNbT, n - j0);
    const double* Lr = LU + int64_t(j0 + min(lane, nb - 1)) * n + j0;
    // a wave takes right-hand sides v and v + nw together: one load of each
    // entry of L for both
    for (int v = wv; v < nv; v += 2 * nw) {
      auto pass = [&](auto two_c) {
        constexpr bool TWO = decltype(two_c)::value;
        double xi = lane < nb ? x[v * xs + j0 + lane] : 0.0;
        double xj = TWO && lane < nb ? x[(v + nw) * xs + j0 + lane] : 0.0;
        for (int c0 = 0; c0 < nb - 1; c0 += kU) {
          double lr[kU];
#pragma unroll
          for (int u = 0; u < kU; ++u) lr[u] = c0 + u < nb ? Lr[c0 + u] : 0.0;
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            const int c = c0 + u;
            if (c < nb - 1) {
              const double xc = __shfl(xi, c, 64);
              if (lane > c && lane < nb) xi -= lr[u] * xc;
              if constexpr (TWO) {
                const double xd = __shfl(xj, c, 64);
                if (lane > c && lane < nb) xj -= lr[u] * xd;
              }
            }
          }
        }
        if (lane < nb) {
          x[v * xs + j0 + lane] = xi;
          if constexpr (TWO) x[(v + nw) * xs + j0 + lane] = xj;
        }
      };
      if (v + nw < nv)
        pass(std::true_type{});
      else
        pass(std::false_type{});
    }
    __syncthreads();
    // the rows below: x_i -= L(i, block) x_block, four rows of a wave at a time
    if (j0 + nb < n) l_gemv_n(LU + int64_t(j0 + nb) * n + j0, n - j0 - nb, nb, n, x + j0, xs, x + j0 + nb, xs, nv, -1.0);
    __syncthreads();
  }
}

// x = U^{-1} x, U the upper triangle of the LU.
__device__ __forceinline__ void l_solve_U(const double* __restrict__ LU, int n, double* x, int xs, int nv) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
  if (n <= 0) return;
  for (int j0 = ((n - 1) / kNbT) * kNbT; j0 >= 0; j0 -= kNbT) {
    const int nb = min(kNbT, n - j0);
    const double* Ur = LU + int64_t(j0 + min(lane, nb - 1)) * n + j0;
    for (int v = wv; v < nv; v += 2 * nw) {  // two right-hand sides per pass, as in l_solve_L
      auto pass = [&](auto two_c) {
        constexpr bool TWO = decltype(two_c)::value;
        double xi = lane < nb ? x[v * xs + j0 + lane] : 0.0;
        double xj = TWO && lane < nb ? x[(v + nw) * xs + j0 + lane] : 0.0;
        for (int cb = ((nb - 1) / kU) * kU; cb >= 0; cb -= kU) {
          double ur[kU];
#pragma unroll
          for (int u = 0; u < kU; ++u) ur[u] = cb + u < nb ? Ur[cb + u] : 1.0;
#pragma unroll
          for (int u = kU - 1; u >= 0; --u) {
            const int c = cb + u;
            if (c < nb) {
              if (lane == c) xi = xi / ur[u];
              const double xc = __shfl(xi, c, 64);
              if (lane < c) xi -= ur[u] * xc;
              if constexpr (TWO) {
                if (lane == c) xj = xj / ur[u];
                const double xd = __shfl(xj, c, 64);
                if (lane < c) xj -= ur[u] * xd;
              }
            }
          }
        }
        if (lane < nb) {
          x[v * xs + j0 + lane] = xi;
          if constexpr (TWO) x[(v + nw) * xs + j0 + lane] = xj;
        }
      };
      if (v + nw < nv)
        pass(std::true_type{});
      else
        pass(std::false_type{});
    }
    __syncthreads();
    // the rows above: x_i -= U(i, block) x_block
    if (j0 > 0) l_gemv_n(LU + j0, j0, nb, n, x + j0, xs, x, xs, nv, -1.0);
    __syncthreads();
  }
}

// x = U^{-T} x (U^T lower with diagonal U_jj), forward over column blocks.
__device__ __forceinline__ void l_solve_UT(const double* __restrict__ LU, int n, double* x, int xs, int nv) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
  for (int j0 = 0; j0 < n; j0 += kNbT) {
    const int nb = min(kNbT, n - j0);
    const int cl = j0 + min(lane, nb - 1);
    for (int v = wv; v < nv; v += 2 * nw) {  // two right-hand sides per pass, as in l_solve_L
      auto pass = [&](auto two_c) {
        constexpr bool TWO = decltype(two_c)::value;
        double xi = lane < nb ? x[v * xs + j0 + lane] : 0.0;
        double xj = TWO && lane < nb ? x[(v + nw) * xs + j0 + lane] : 0.0;
        for (int c0 = 0; c0 < nb; c0 += kU) {
          double uc[kU], ud[kU];
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            const int c = c0 + u < nb ? c0 + u : nb - 1;
            uc[u] = LU[int64_t(j0 + c) * n + cl];
            ud[u] = LU[int64_t(j0 + c) * n + j0 + c];
          }
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            const int c = c0 + u;
            if (c < nb) {
              if (lane == c) xi = xi / ud[u];
              const double xc = __shfl(xi, c, 64);
              if (lane > c && lane < nb) xi -= uc[u] * xc;
              if constexpr (TWO) {
                if (lane == c) xj = xj / ud[u];
                const double xd = __shfl(xj, c, 64);
                if (lane > c && lane < nb) xj -= uc[u] * xd;
              }
            }
          }
        }
        if (lane < nb) {
          x[v * xs + j0 + lane] = xi;
          if constexpr (TWO) x[(v + nw) * xs + j0 + lane] = xj;
        }
      };
      if (v + nw < nv)
        pass(std::true_type{});
      else
        pass(std::false_type{});
    }
    __syncthreads();
    // the entries below: x_i -= sum_c U(j0 + c, i) x_{j0 + c} (rows of the block, read by columns)
    if (j0 + nb < n) l_gemv_t(LU + int64_t(j0) * n + j0 + nb, nb, n - j0 - nb, n, x + j0, xs, x + j0 + nb, xs, nv, -1.0);
    __syncthreads();
  }
}

// x = L^{-T} x (L^T unit upper), backward over column blocks.
__device__ __forceinline__ void l_solve_LT(const double* __restrict__ LU, int n, double* x, int xs, int nv) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
  if (n <= 0) return;
  for (int j0 = ((n - 1) / kNbT) * kNbT; j0 >= 0; j0 -= kNbT) {
    const int nb = min(kNbT, n - j0);
    const int cl = j0 + min(lane, nb - 1);
    for (int v = wv; v < nv; v += 2 * nw) {  // two right-hand sides per pass, as in l_solve_L
      auto pass = [&](auto two_c) {
        constexpr bool TWO = decltype(two_c)::value;
        double xi = lane < nb ? x[v * xs + j0 + lane] : 0.0;
        double xj = TWO && lane < nb ? x[(v + nw) * xs + j0 + lane] : 0.0;
        for (int cb = ((nb - 1) / kU) * kU; cb >= 0; cb -= kU) {
          double lc[kU];
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            const int c = cb + u < nb ? cb + u : nb - 1;
            lc[u] = LU[int64_t(j0 + c) * n + cl];
          }
#pragma unroll
          for (int u = kU - 1; u >= 0; --u) {
            const int c = cb + u;
            if (c < nb && c > 0) {
              const double xc = __shfl(xi, c, 64);
              if (lane < c) xi -= lc[u] * xc;
              if constexpr (TWO) {
                const double xd = __shfl(xj, c, 64);
                if (lane < c) xj -= lc[u] * xd;
              }
            }
          }
        }
        if (lane < nb) {
          x[v * xs + j0 + lane] = xi;
          if constexpr (TWO) x[(v + nw) * xs + j0 + lane] = xj;
        }
      };
      if (v + nw < nv)
        pass(std::true_type{});
      else
        pass(std::false_type{});
    }
    __syncthreads();
    // the entries above: x_i -= sum_c L(j0 + c, i) x_{j0 + c}
    if (j0 > 0) l_gemv_t(LU + int64_t(j0) * n, nb, j0, n, x + j0, xs, x, xs, nv, -1.0);
    __syncthreads();
  }
}

// x = M x through the scratch tp (both [nv][n] in LDS), M a triangle of the
// row-major n x n LU: mode 0 U (columns j >= i), 1 the unit lower L (x_i plus
// columns j < i), both one wave per row; mode 2 the unit upper L^T (x_i plus
// rows j > i of L), 3 U^T (rows j <= i of U), both one thread per column.
__device__ __forceinline__ void l_trmv(const double* __restrict__ LU, int n, double* x, double* tp, int nv, int mode) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
  if (mode <= 1) {
    for (int i = wv; i < n; i += nw) {
      const double* mr = LU + int64_t(i) * n;
      const int jb = mode == 0 ? i : 0, je = mode == 0 ? n : i;
      double acc[kMaxV];
#pragma unroll
      for (int v = 0; v < kMaxV; ++v) acc[v] = 0.0;
      for (int j0 = jb; j0 < je; j0 += 64 * kU) {
        double mv[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int j = j0 + u * 64 + lane;
          mv[u] = j < je ? mr[j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int j = j0 + u * 64 + lane;
          if (j < je) {
#pragma unroll
            for (int v = 0; v < kMaxV; ++v)
              if (v < nv) acc[v] += mv[u] * x[v * n + j];
          }
        }
      }
      const double t = wave_rs8(acc);
      const int v = lane >> 3;
      if ((lane & 7) == 0 && v < nv) tp[v * n + i] = t + (mode == 1 ? x[v * n + i] : 0.0);
    }
  } else {
    for (int i = tid; i < n; i += blockDim.x) {
      const int jb = mode == 2 ? i + 1 : 0, je = mode == 2 ? n : i + 1;
      double acc[kMaxV];
#pragma unroll
      for (int v = 0; v < kMaxV; ++v) acc[v] = 0.0;
      for (int j0 = jb; j0 < je; j0 += kU) {
        double mv[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) mv[u] = j0 + u < je ? LU[int64_t(j0 + u) * n + i] : 0.0;
#pragma unroll
        for (int u = 0; u < kU; ++u)
          if (j0 + u < je) {
#pragma unroll
            for (int v = 0; v < kMaxV; ++v)
              if (v < nv) acc[v] += mv[u] * x[v * n + j0 + u];
          }
      }
#pragma unroll
      for (int v = 0; v < kMaxV; ++v)
        if (v < nv) tp[v * n + i] = acc[v] + (mode == 2 ? x[v * n + i] : 0.0);
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nv * n; e += blockDim.x) x[e] = tp[e];
  __syncthreads();
}

// x = P x (fwd) or P^T x through the scratch tp, both [nv][n] in LDS.
__device__ __forceinline__ void l_permute(const int32_t* perm, int n, double* x, double* tp, int nv, bool fwd) {
  for (int e = threadIdx.x; e < nv * n; e += blockDim.x) {
    const int v = e / n, i = e % n;
    if (fwd)
      tp[e] = x[v * n + perm[i]];
    else
      tp[v * n + perm[i]] = x[e];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nv * n; e += blockDim.x) x[e] = tp[e];
  __syncthreads();
}

// One group per workgroup of BS threads; op 0 solve, 1 solve_T, 2 apply,
// 3 apply_T (the per-group steps in the header of this file); down = 0 for
// the upward sweep (finest sub-level first), 1 for the downward one.  The LDS
// holds cap doubles (sized by the launch to the sub-level's largest record);
// the caller guarantees 2r + k <= cap.
// Registers are capped for 4 waves per SIMD (only the 64-thread shape
// spills, a few bytes): the 1024 records of a 512^2 level-1 sub-level then
// all run at once, 4 per CU.
template <int BS>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(4))) void k_sweep_lds(SwArgs A, int down, int cap) {
  extern __shared__ double sm[];
  const GroupRec R = A.recs[blockIdx.x];
  const int r = R.r, k = R.k;
  const int32_t* rd = A.iarena + R.idx;
  const int32_t* sk = rd + r;
  const int32_t* perm = sk + k + r;
  const double* T = A.darena + R.off;
  const double* Lsr = T + int64_t(k) * r;
  const double* Urs = Lsr + int64_t(k) * r;
  const double* LU = Urs + int64_t(r) * k;
  const int64_t N = A.N;
  const int tid = threadIdx.x;
  const int nvb = max(1, min(A.nrhs, cap / (2 * r + k)));
  for (int v0 = 0; v0 < A.nrhs; v0 += nvb) {
    const int nv = min(nvb, A.nrhs - v0);
    double* xr = sm;           // [nv][r]
    double* xs = sm + nv * r;  // [nv][k]
    double* tp = xs + nv * k;  // [nv][r]
    double* u = A.u + v0 * N;
    for (int e = tid; e < nv * r; e += BS) xr[e] = u[(e / r) * N + rd[e % r]];
    for (int e = tid; e < nv * k; e += BS) xs[e] = u[(e / k) * N + sk[e % k]];
    __syncthreads();
    if (A.op == 0 && !down) {
      if (k > 0) l_gemv_t(T, k, r, r, xs, k, xr, r, nv, -1.0);  // u_r -= T^T u_s
      __syncthreads();
      l_permute(perm, r, xr, tp, nv, true);                     // u_r = P u_r
      l_solve_L(LU, r, xr, r, nv);                              // u_r = L^{-1} u_r
      if (k > 0) l_gemv_n(Lsr, k, r, r, xr, r, xs, k, nv, -1.0);  // u_s -= L_sr u_r
    } else if (A.op == 0) {
      if (k > 0) l_gemv_n(Urs, r, k, k, xs, k, xr, r, nv, -1.0);  // u_r -= U_rs u_s
      __syncthreads();
      l_solve_U(LU, r, xr, r, nv);                                 // u_r = U^{-1} u_r
      if (k > 0) l_gemv_n(T, k, r, r, xr, r, xs, k, nv, -1.0);    // u_s -= T u_r
    } else if (A.op == 1 && !down) {
      if (k > 0) l_gemv_t(T, k, r, r, xs, k, xr, r, nv, -1.0);    // u_r -= T^T u_s
      __syncthreads();
      l_solve_UT(LU, r, xr, r, nv);                                // u_r = U^{-T} u_r
      if (k > 0) l_gemv_t(Urs, r, k, k, xr, r, xs, k, nv, -1.0);  // u_s -= U_rs^T u_r
    } else if (A.op == 1) {
      if (k > 0) l_gemv_t(Lsr, k, r, r, xs, k, xr, r, nv, -1.0);  // u_r -= L_sr^T u_s
      __syncthreads();
      l_solve_LT(LU, r, xr, r, nv);                                // u_r = L^{-T} u_r
      l_permute(perm, r, xr, tp, nv, false);                       // u_r = P^T u_r
      if (k > 0) l_gemv_n(T, k, r, r, xr, r, xs, k, nv, -1.0);    // u_s -= T u_r
    } else if (A.op == 2 && !down) {
      if (k > 0) l_gemv_n(T, k, r, r, xr, r, xs, k, nv, 1.0);     // x_s += T x_r
      __syncthreads();
      l_trmv(LU, r, xr, tp, nv, 0);                                // x_r = U x_r
      if (k > 0) l_gemv_n(Urs, r, k, k, xs, k, xr, r, nv, 1.0);   //     + U_rs x_s
    } else if (A.op == 2) {
      if (k > 0) l_gemv_n(Lsr, k, r, r, xr, r, xs, k, nv, 1.0);   // y_s += L_sr y_r
      __syncthreads();
      l_trmv(LU, r, xr, tp, nv, 1);                                // y_r = L y_r
      l_permute(perm, r, xr, tp, nv, false);                       // y_r = P^T y_r
      if (k > 0) l_gemv_t(T, k, r, r, xs, k, xr, r, nv, 1.0);     // y_r += T^T y_s
    } else if (!down) {
      if (k > 0) l_gemv_n(T, k, r, r, xr, r, xs, k, nv, 1.0);     // x_s += T x_r
      __syncthreads();
      l_permute(perm, r, xr, tp, nv, true);                        // x_r = P x_r
      l_trmv(LU, r, xr, tp, nv, 2);                                // x_r = L^T x_r
      if (k > 0) l_gemv_t(Lsr, k, r, r, xs, k, xr, r, nv, 1.0);   //     + L_sr^T x_s
    } else {
      if (k > 0) l_gemv_t(Urs, r, k, k, xr, r, xs, k, nv, 1.0);   // y_s += U_rs^T y_r
      __syncthreads();
      l_trmv(LU, r, xr, tp, nv, 3);                                // y_r = U^T y_r
      if (k > 0) l_gemv_t(T, k, r, r, xs, k, xr, r, nv, 1.0);     // y_r += T^T y_s
    }
    __syncthreads();
    for (int e = tid; e < nv * r; e += BS) u[(e / r) * N + rd[e % r]] = xr[e];
    for (int e = tid; e < nv * k; e += BS) u[(e / k) * N + sk[e % k]] = xs[e];
    __syncthreads();
  }
}

// Top block: x = A_L^{-1} x (op 0), A_L^{-T} x (op 1), A_L x (op 2) or
// A_L^T x (op 3) with A_L = P^T L U; requires 2n <= kCapL.
__global__ __launch_bounds__(1024) void k_top_lds(const double* LU, const int32_t* perm, int n, const int32_t* idx,
                                                  double* u, int64_t N, int nrhs, int op) {
  __shared__ double sm[kCapL];
  const int tid = threadIdx.x, B = blockDim.x;
  const int nvb = max(1, min(nrhs, kCapL / (2 * n)));
  for (int v0 = 0; v0 < nrhs; v0 += nvb) {
    const int nv = min(nvb, nrhs - v0);
    double* x = sm;
    double* tp = sm + nv * n;
    double* uu = u + v0 * N;
    for (int e = tid; e < nv * n; e += B) x[e] = uu[(e / n) * N + idx[e % n]];
    __syncthreads();
    if (op == 0) {
      l_permute(perm, n, x, tp, nv, true);
      l_solve_L(LU, n, x, n, nv);
      l_solve_U(LU, n, x, n, nv);
    } else if (op == 1) {
      l_solve_UT(LU, n, x, n, nv);
      l_solve_LT(LU, n, x, n, nv);
      l_permute(perm, n, x, tp, nv, false);
    } else if (op == 2) {
      l_trmv(LU, n, x, tp, nv, 0);
      l_trmv(LU, n, x, tp, nv, 1);
      l_permute(perm, n, x, tp, nv, false);
    } else {
      l_permute(perm, n, x, tp, nv, true);
      l_trmv(LU, n, x, tp, nv, 2);
      l_trmv(LU, n, x, tp, nv, 3);
    }
    for (int e = tid; e < nv * n; e += B) uu[(e / n) * N + idx[e % n]] = x[e];
    __syncthreads();
  }
}

// Gather form of the row interchanges j <-> piv[j], j = 0..n-1 (in order).
constexpr int kPermLds = 8192;
__device__ void make_perm(const int32_t* piv, int32_t* perm, int n) {
  __shared__ int32_t sp[kPermLds];
  __shared__ int32_t spv[kPermLds];
  if (n <= kPermLds) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      sp[i] = i;
      spv[i] = piv[i];
    }
    __syncthreads();
    if (threadIdx.x == 0)
      for (int j = 0; j < n; ++j) {
        const int p = spv[j];
        const int t = sp[j];
        sp[j] = sp[p];
        sp[p] = t;
      }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) perm[i] = sp[i];
  } else {
    for (int i = threadIdx.x; i < n; i += blockDim.x) perm[i] = i;
    __syncthreads();
    if (threadIdx.x == 0)
      for (int j = 0; j < n; ++j) {
        const int p = piv[j];
        const int t = perm[j];
        perm[j] = perm[p];
        perm[p] = t;
      }
  }
}

__global__ __launch_bounds__(64) void k_make_perm(const GroupRec* recs, int32_t* iarena) {
  const GroupRec R = recs[blockIdx.x];
  int32_t* piv = iarena + R.idx + R.r + R.k;
  make_perm(piv, piv + R.r, R.r);
}

__global__ __launch_bounds__(64) void k_make_perm_top(const int32_t* piv, int32_t* perm, int n) {
  make_perm(piv, perm, n);
}

__global__ void k_copy(const double* x, double* y, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    y[i] = x[i];
}

// ---------------------------------------------------------------------------
// Solve and transposed solve (op 0, 1) for sub-levels with few, large
// records: each record is spread over many workgroups and all right-hand
// sides go through its factors in one pass (the LDS kernel above holds
// 2r + k entries per right-hand side and so rereads large factors once per
// right-hand side).  Per record, B holds the right-hand sides of the
// triangular solve and X its solution, both [nv][r] at nv * woff in the work
// buffer.  The products with T, L_sr and U_rs are spread over many
// workgroups per record; the triangular solve of every record of the pass is
// one launch of workgroups that hand 64-row blocks of X to each other
// (k_sp_chain).
// ---------------------------------------------------------------------------
struct SpArgs {
  const GroupRec* recs;
  const int32_t* iarena;
  const double* darena;
  const int64_t* woff;
  double* u;  // [nv][N]
  double* B;
  double* X;
  int64_t N;
  int nv;
  const double* dinv;  // diagonal-block inverses (SubLevel::dinv layout)
  int dnb;             // blocks per record in dinv
  // Ticket counter of the chained triangular solve.
  uint32_t* sync = nullptr;
  int nbm = 0;  // blocks of the largest record
  long long wait_ticks = 0;  // bound on each wait, in ticks of the 100 MHz constant clock
};

struct SpRec {
  int r, k;
  const int32_t *rd, *sk, *perm;
  const double *T, *Lsr, *Urs, *LU;
  double *B, *X;
};

__device__ __forceinline__ SpRec sp_rec(const SpArgs& A, int i) {
  const GroupRec R = A.recs[i];
  SpRec v;
  v.r = R.r;
  v.k = R.k;
  v.rd = A.iarena + R.idx;
  v.sk = v.rd + R.r;
  v.perm = v.sk + R.k + R.r;
  v.T = A.darena + R.off;
  v.Lsr = v.T + int64_t(R.k) * R.r;
  v.Urs = v.Lsr + int64_t(R.k) * R.r;
  v.LU = v.Urs + int64_t(R.r) * R.k;
  v.B = A.B + A.nv * A.woff[i];
  v.X = A.X + A.nv * A.woff[i];
  return v;
}

// The first kernel of a pass readies the chained solve that follows it:
// workgroup (0, 0) clears the ticket counter, and every workgroup marks its
// rows of X pending (rows i0 .. i0 + nrow - 1 of each right-hand side).  The
// next launch on the stream sees both.
constexpr uint64_t kXPending = 0x7FF4A3B2C1D0E0F1ull;  // a signaling NaN: no arithmetic result
__device__ __forceinline__ void sp_ready_chain(const SpArgs& A, const SpRec& R, int i0, int nrow) {
  if (!A.sync) return;
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) A.sync[0] = 0u;
  const int n = min(nrow, R.r - i0);
  uint64_t* X = reinterpret_cast<uint64_t*>(R.X);
  for (int e = threadIdx.x; e < A.nv * n; e += blockDim.x) X[(e / n) * R.r + i0 + e % n] = kXPending;
}

constexpr int kSpChunk = 512;  // skeleton entries staged in LDS per pass
constexpr int kUc = 16;         // loads in flight per lane in the column-form products

// The sums over the wave of acc[q][v] (4 rows q of the wave, kMaxV
// right-hand sides) in one reduce-scatter: returns the total of row q =
// lane >> 4, right-hand side v = (lane >> 1) & 7, held by lanes 2c and
// 2c + 1 (c = 8q + v).
__device__ __forceinline__ double sp_rows_sum(const double (&acc)[4][kMaxV]) {
  double p[kRs];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int v = 0; v < kMaxV; ++v) p[q * kMaxV + v] = acc[q][v];
  return wave_rs32(p);
}

// dst[v][e] = src(v, e) for e < n, v < nv, with src(v, e) = base[v ld + idx[e]]
// (idx given) or base[v ld + e]: an entry per thread and step, its index
// loaded once and its right-hand sides' loads issued together before any is
// stored (the caller synchronizes before the block is read).
__device__ __forceinline__ void sp_stage(const double* base, int64_t ld, const int32_t* idx, int n, int nv,
                                         double (*dst)[kSpChunk]) {
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int64_t g = idx ? int64_t(idx[e]) : int64_t(e);
    double t[kMaxV];
#pragma unroll
    for (int v = 0; v < kMaxV; ++v) t[v] = v < nv ? base[v * ld + g] : 0.0;
#pragma unroll
    for (int v = 0; v < kMaxV; ++v)
      if (v < nv) dst[v][e] = t[v];
  }
}

// acc[q][v] += sum_{c < nc} mr[q][c] s[v][c] for a wave's 4 rows q (mr[q] null
// past the record; its sums are then never used), lane c = lane, lane + 64, ...
// The loads of the 4 rows and of two column steps are issued together before
// any is used; each acc[q][v] still adds its terms in increasing c.  TRI >= 0
// keeps one triangle of rows iq[q] (column c0 + c): 0 the upper one with the
// diagonal, 1 the strictly lower one; the other entries count as zero.
template <int TRI = -1>
__device__ __forceinline__ void sp_rows4_acc(const double* const (&mr)[4], int nc, const double (*s)[kSpChunk], int nv,
                                             double (&acc)[4][kMaxV], int c0 = 0, const int* iq = nullptr) {
  const int lane = threadIdx.x & 63;
  for (int c = lane; c < nc; c += 128) {
    double m[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int cc = c + 64 * u;
        bool keep = mr[q] && cc < nc;
        if constexpr (TRI == 0) keep = keep && c0 + cc >= iq[q];
        if constexpr (TRI == 1) keep = keep && c0 + cc < iq[q];
        m[u][q] = keep ? mr[q][cc] : 0.0;
      }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int cc = c + 64 * u;
      if (cc < nc)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int v = 0; v < kMaxV; ++v)
            if (v < nv) acc[q][v] += m[u][q] * s[v][cc];
    }
  }
}

// First step of an up pass (and of the transposed solve's down pass), column
// form: B(v, i) = u_r(v, c) - (M^T u_s)(v, c) with c = perm[i] (PERM: the
// row interchanges of the solve, B = P(u_r - T^T u_s)) or c = i, and
// M = T (k x r), or L_sr with LSR.  With ADD instead u_r(v, i) += (M^T u_s)(v, i)
// in place (the last step of the apply sweeps' down pass).  64 rows i per
// workgroup, lane per row, the sum over the skeleton split between the 4
// waves and added through LDS.
template <bool LSR, bool PERM, bool ADD = false>
__global__ __launch_bounds__(256) void k_sp_first_cols(SpArgs A) {
  const SpRec R = sp_rec(A, blockIdx.y);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;  // 64 rows per workgroup
  if (!ADD) sp_ready_chain(A, R, blockIdx.x * 64, 64);
  if (blockIdx.x * 64 >= R.r) return;
  const int nv = A.nv;
  const double* M = LSR ? R.Lsr : R.T;
  __shared__ double sus[kMaxV][kSpChunk];
  __shared__ double sred[4][kMaxV][64];
  const int c = i < R.r ? (PERM ? R.perm[i] : i) : 0;
  double acc[kMaxV];
#pragma unroll
  for (int v = 0; v < kMaxV; ++v) acc[v] = 0.0;
  for (int j0 = 0; j0 < R.k; j0 += kSpChunk) {
    const int nj = min(kSpChunk, R.k - j0);
    __syncthreads();
    sp_stage(A.u, A.N, R.sk + j0, nj, nv, sus);
    __syncthreads();
    // wave wv takes the quarter [jb, je) of the chunk
    const int jb = (nj * wv) / 4, je = (nj * (wv + 1)) / 4;
    if (i < R.r) {
      const double* tc = M + int64_t(j0) * R.r + c;
      for (int j = jb; j < je; j += kUc) {
        double t[kUc];
#pragma unroll
        for (int u = 0; u < kUc; ++u) t[u] = j + u < je ? tc[int64_t(j + u) * R.r] : 0.0;
#pragma unroll
        for (int u = 0; u < kUc; ++u)
          if (j + u < je)
#pragma unroll
            for (int v = 0; v < kMaxV; ++v)
              if (v < nv) acc[v] += t[u] * sus[v][j + u];
      }
    }
  }
#pragma unroll
  for (int v = 0; v < kMaxV; ++v) sred[wv][v][lane] = acc[v];
  __syncthreads();
  if (wv == 0 && i < R.r)
#pragma unroll
    for (int v = 0; v < kMaxV; ++v)
      if (v < nv) {
        const double t = (sred[0][v][lane] + sred[1][v][lane]) + (sred[2][v][lane] + sred[3][v][lane]);
        if (ADD)
          A.u[v * A.N + R.rd[c]] += t;
        else
          R.B[v * R.r + i] = A.u[v * A.N + R.rd[c]] - t;
      }
}

// Down, first step of the solve: B(v, i) = (u_r - U_rs u_s)(v, i), one wave
// per row i.
__global__ __launch_bounds__(256) void k_sp_down_first(SpArgs A) {
  const SpRec R = sp_rec(A, blockIdx.y);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i0 = blockIdx.x * 16;  // 16 rows per workgroup, 4 per wave
  sp_ready_chain(A, R, i0, 16);
  if (i0 >= R.r) return;
  const int nv = A.nv;
  __shared__ double sus[kMaxV][kSpChunk];
  double acc[4][kMaxV];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int v = 0; v < kMaxV; ++v) acc[q][v] = 0.0;
  for (int j0 = 0; j0 < R.k; j0 += kSpChunk) {
    const int nj = min(kSpChunk, R.k - j0);
    __syncthreads();
    sp_stage(A.u, A.N, R.sk + j0, nj, nv, sus);
    __syncthreads();
    const double* mr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + wv * 4 + q;
      mr[q] = i < R.r ? R.Urs + int64_t(i) * R.k + j0 : nullptr;
    }
    sp_rows4_acc(mr, nj, sus, nv, acc);
  }
  {
    const double t = sp_rows_sum(acc);
    const int i = i0 + wv * 4 + (lane >> 4), v = (lane >> 1) & 7;
    if ((lane & 1) == 0 && i < R.r && v < nv) R.B[v * R.r + i] = A.u[v * A.N + R.rd[i]] - t;
  }
}

// u_s += sgn M x (M = L_sr or T, k x r), one wave per skeleton row; x is X,
// or with GATHER the record's u_r read through its indices; staged in LDS by
// chunks of columns.
template <bool GATHER>
__global__ __launch_bounds__(256) void k_sp_skel_update(SpArgs A, int which, double sgn) {
  const SpRec R = sp_rec(A, blockIdx.y);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j0 = blockIdx.x * 16;
  if (j0 >= R.k) return;
  const int nv = A.nv;
  const double* M = which ? R.T : R.Lsr;
  __shared__ double sx[kMaxV][kSpChunk];
  double acc[4][kMaxV];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int v = 0; v < kMaxV; ++v) acc[q][v] = 0.0;
  for (int c0 = 0; c0 < R.r; c0 += kSpChunk) {
    const int nc = min(kSpChunk, R.r - c0);
    __syncthreads();
    if (GATHER)
      sp_stage(A.u, A.N, R.rd + c0, nc, nv, sx);
    else
      sp_stage(R.X + c0, R.r, nullptr, nc, nv, sx);
    __syncthreads();
    const double* mr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + wv * 4 + q;
      mr[q] = j < R.k ? M + int64_t(j) * R.r + c0 : nullptr;
    }
    sp_rows4_acc(mr, nc, sx, nv, acc);
  }
  {
    const double t = sp_rows_sum(acc);
    const int j = j0 + wv * 4 + (lane >> 4), v = (lane >> 1) & 7;
    if ((lane & 1) == 0 && j < R.k && v < nv) A.u[v * A.N + R.sk[j]] += sgn * t;
  }
}

// u_s += sgn U_rs^T x (U_rs r x k), x = X or with GATHER the record's u_r
// read through its indices: lane per skeleton entry j, 64 per workgroup, the
// sum over the rows of U_rs split between the 4 waves and added through LDS;
// x staged in LDS by chunks.
template <bool GATHER>
__global__ __launch_bounds__(256) void k_sp_skel_update_T(SpArgs A, double sgn) {
  const SpRec R = sp_rec(A, blockIdx.y);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  if (blockIdx.x * 64 >= R.k) return;
  const int nv = A.nv;
  __shared__ double sx[kMaxV][kSpChunk];
  __shared__ double sred[4][kMaxV][64];
  double acc[kMaxV];
#pragma unroll
  for (int v = 0; v < kMaxV; ++v) acc[v] = 0.0;
  for (int i0 = 0; i0 < R.r; i0 += kSpChunk) {
    const int ni = min(kSpChunk, R.r - i0);
    __syncthreads();
    if (GATHER)
      sp_stage(A.u, A.N, R.rd + i0, ni, nv, sx);
    else
      sp_stage(R.X + i0, R.r, nullptr, ni, nv, sx);
    __syncthreads();
    const int ib = (ni * wv) / 4, ie = (ni * (wv + 1)) / 4;
    if (j < R.k) {
      const double* mc = R.Urs + int64_t(i0) * R.k + j;
      for (int i = ib; i < ie; i += kUc) {
        double m[kUc];
#pragma unroll
        for (int u = 0; u < kUc; ++u) m[u] = i + u < ie ? mc[int64_t(i + u) * R.k] : 0.0;
#pragma unroll
        for (int u = 0; u < kUc; ++u)
          if (i + u < ie)
#pragma unroll
            for (int v = 0; v < kMaxV; ++v)
              if (v < nv) acc[v] += m[u] * sx[v][i + u];
      }
    }
  }
#pragma unroll
  for (int v = 0; v < kMaxV; ++v) sred[wv][v][lane] = acc[v];
  __syncthreads();
  if (wv == 0 && j < R.k)
#pragma unroll
    for (int v = 0; v < kMaxV; ++v)
      if (v < nv)
        A.u[v * A.N + R.sk[j]] += sgn * ((sred[0][v][lane] + sred[1][v][lane]) + (sred[2][v][lane] + sred[3][v][lane]));
}

// u_r = x, or with PERM u_r = P^T x (u_r[perm[i]] = x[i]); x = X (src 0) or
// B (src 1).
template <bool PERM>
__global__ __launch_bounds__(256) void k_sp_scatter(SpArgs A, int src) {
  const SpRec R = sp_rec(A, blockIdx.y);
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= R.r) return;
  const double* x = src ? R.B : R.X;
  const int d = R.rd[PERM ? R.perm[i] : i];
  for (int v = 0; v < A.nv; ++v) A.u[v * A.N + d] = x[v * R.r + i];
}

// B = u_r, or with PERM B = P u_r (B[i] = u_r[perm[i]]).
template <bool PERM>
__global__ __launch_bounds__(256) void k_sp_gather(SpArgs A) {
  const SpRec R = sp_rec(A, blockIdx.y);
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= R.r) return;
  const int d = R.rd[PERM ? R.perm[i] : i];
  for (int v = 0; v < A.nv; ++v) R.B[v * R.r + i] = A.u[v * A.N + d];
}

// The triangular products of the apply sweeps (and the rectangular ones
// beside them), for few large records: x = B, out = X (io 0) or x = X,
// out = B (io 1).  Row form: out(v, i) = (M x)(v, i) [+ (U_rs u_s)(v, i)]
// with M the upper U of the record's LU (TRI 0, columns j >= i) or its unit
// lower L (TRI 1, x_i plus the columns j < i); one wave per row i, 16 rows
// per workgroup, x and u_s staged in LDS by chunks.
template <int TRI, bool RECT>
__global__ __launch_bounds__(256) void k_sp_rowmv(SpArgs A, int io) {
  const SpRec R = sp_rec(A, blockIdx.y);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i0 = blockIdx.x * 16;
  if (i0 >= R.r) return;
  const int nv = A.nv, r = R.r;
  const double* x = io ? R.X : R.B;
  double* out = io ? R.B : R.X;
  __shared__ double sx[kMaxV][kSpChunk];
  double acc[4][kMaxV];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int v = 0; v < kMaxV; ++v) acc[q][v] = 0.0;
  // the columns the workgroup's rows reach
  const int cb = TRI == 0 ? i0 : 0, ce = TRI == 0 ? r : min(r, i0 + 16);
  for (int c0 = cb; c0 < ce; c0 += kSpChunk) {
    const int nc = min(kSpChunk, ce - c0);
    __syncthreads();
    sp_stage(x + c0, r, nullptr, nc, nv, sx);
    __syncthreads();
    const double* mr[4];
    int iq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      iq[q] = i0 + wv * 4 + q;
      mr[q] = iq[q] < r ? R.LU + int64_t(iq[q]) * r + c0 : nullptr;
    }
    sp_rows4_acc<TRI == 0 ? 0 : 1>(mr, nc, sx, nv, acc, c0, iq);
  }
  if (RECT)
    for (int j0 = 0; j0 < R.k; j0 += kSpChunk) {
      const int nj = min(kSpChunk, R.k - j0);
      __syncthreads();
      sp_stage(A.u, A.N, R.sk + j0, nj, nv, sx);
      __syncthreads();
      const double* mr[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + wv * 4 + q;
        mr[q] = i < r ? R.Urs + int64_t(i) * R.k + j0 : nullptr;
      }
      sp_rows4_acc(mr, nj, sx, nv, acc);
    }
  {
    const double t = sp_rows_sum(acc);
    const int i = i0 + wv * 4 + (lane >> 4), v = (lane >> 1) & 7;
    if ((lane & 1) == 0 && i < r && v < nv) out[v * r + i] = t + (TRI == 1 ? x[v * r + i] : 0.0);
  }
}

// Column form: out(v, i) = (M^T x)(v, i) [+ (L_sr^T u_s)(v, i)] with M^T the
// unit upper L^T (TRI 2: x_i plus the rows j > i of L) or the lower U^T
// (TRI 3: the rows j <= i of U); lane per i, 64 per workgroup, the sum over
// j split between the 4 waves and added through LDS.
template <int TRI, bool RECT>
__global__ __launch_bounds__(256) void k_sp_colmv(SpArgs A, int io) {
  const SpRec R = sp_rec(A, blockIdx.y);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int ib = blockIdx.x * 64, i = ib + lane;
  if (ib >= R.r) return;
  const int nv = A.nv, r = R.r;
  const double* x = io ? R.X : R.B;
  double* out = io ? R.B : R.X;
  __shared__ double sx[kMaxV][kSpChunk];
  __shared__ double sred[4][kMaxV][64];
  double acc[kMaxV];
#pragma unroll
  for (int v = 0; v < kMaxV; ++v) acc[v] = 0.0;
  // the rows the workgroup's columns reach
  const int jb = TRI == 2 ? ib : 0, je = TRI == 2 ? r : min(r, ib + 64);
  for (int j0 = jb; j0 < je; j0 += kSpChunk) {
    const int nj = min(kSpChunk, je - j0);
    __syncthreads();
    sp_stage(x + j0, r, nullptr, nj, nv, sx);
    __syncthreads();
    const int qb = (nj * wv) / 4, qe = (nj * (wv + 1)) / 4;
    if (i < r) {
      const double* mc = R.LU + int64_t(j0) * r + i;
      for (int j = qb; j < qe; j += kUc) {
        double m[kUc];
#pragma unroll
        for (int u = 0; u < kUc; ++u) {
          const int jr = j0 + j + u;
          m[u] = (j + u < qe && (TRI == 2 ? jr > i : jr <= i)) ? mc[int64_t(j + u) * r] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kUc; ++u)
          if (j + u < qe)
#pragma unroll
            for (int v = 0; v < kMaxV; ++v)
              if (v < nv) acc[v] += m[u] * sx[v][j + u];
      }
    }
  }
  if (RECT)
    for (int j0 = 0; j0 < R.k; j0 += kSpChunk) {
      const int nj = min(kSpChunk, R.k - j0);
      __syncthreads();
      sp_stage(A.u, A.N, R.sk + j0, nj, nv, sx);
      __syncthreads();
      const int qb = (nj * wv) / 4, qe = (nj * (wv + 1)) / 4;
      if (i < r) {
        const double* mc = R.Lsr + int64_t(j0) * r + i;
        for (int j = qb; j < qe; j += kUc) {
          double m[kUc];
#pragma unroll
          for (int u = 0; u < kUc; ++u) m[u] = j + u < qe ? mc[int64_t(j + u) * r] : 0.0;
#pragma unroll
          for (int u = 0; u < kUc; ++u)
            if (j + u < qe)
#pragma unroll
              for (int v = 0; v < kMaxV; ++v)
                if (v < nv) acc[v] += m[u] * sx[v][j + u];
        }
      }
    }
#pragma unroll
  for (int v = 0; v < kMaxV; ++v) sred[wv][v][lane] = acc[v];
  __syncthreads();
  if (wv == 0 && i < r)
#pragma unroll
    for (int v = 0; v < kMaxV; ++v)
      if (v < nv)
        out[v * r + i] = ((sred[0][v][lane] + sred[1][v][lane]) + (sred[2][v][lane] + sred[3][v][lane])) +
                         (TRI == 2 ? x[v * r + i] : 0.0);
}

// Inverses of the diagonal blocks of the records' L (unit lower) and U
// (upper) for the chained solves below: workgroup (b, i) inverts block b of
// record i; lane c builds column c of each inverse by substitution (L: down
// the rows, U: up the rows), so no lane reads another's column.  Rows and
// columns past a partial last block are the identity.
__global__ __launch_bounds__(64) void k_sp_dinv(SpArgs A, double* dinv) {
  const SpRec R = sp_rec(A, blockIdx.y);
  const int b = blockIdx.x, j0 = b * kNbT;
  if (j0 >= R.r) return;
  const int nb = min(kNbT, R.r - j0), r = R.r, c = threadIdx.x;
  __shared__ double sM[kNbT][kNbT + 1];
  __shared__ double sX[kNbT][kNbT + 1];
  for (int a = 0; a < kNbT; ++a)
    sM[a][c] = (a < nb && c < nb) ? R.LU[int64_t(j0 + a) * r + j0 + c] : (a == c ? 1.0 : 0.0);
  __syncthreads();
  double* out = dinv + (int64_t(blockIdx.y) * A.dnb + b) * 2 * kNbT * kNbT;
  for (int a = 0; a < kNbT; ++a) {  // L X = I, unit diagonal
    double acc = 0.0;
    for (int j = c; j < a; ++j) acc += sM[a][j] * sX[j][c];
    sX[a][c] = a == c ? 1.0 : (a > c ? -acc : 0.0);
  }
  for (int a = 0; a < kNbT; ++a) out[a * kNbT + c] = sX[a][c];
  for (int a = kNbT - 1; a >= 0; --a) {  // U X = I
    double acc = 0.0;
    for (int j = a + 1; j <= c; ++j) acc += sM[a][j] * sX[j][c];
    const double d = sM[a][a];
    sX[a][c] = a > c ? 0.0 : (a == c ? 1.0 / d : -acc / d);
  }
  for (int a = 0; a < kNbT; ++a) out[kNbT * kNbT + a * kNbT + c] = sX[a][c];
}

// ---------------------------------------------------------------------------
// The blocked triangular solve X = M^{-1} B of every record of a pass in one
// launch.  Workgroup (record, block j) owns rows 64j .. 64j + 63 of X: it
// subtracts the products of its row of 64 x 64 blocks of M with the blocks
// of X it depends on, each as soon as that block is written, multiplies the
// result by the stored inverse of its diagonal block and writes its block of
// X.  The block's values are their own flag: the pass's first kernel marks
// every entry of X pending (a signaling NaN, which no arithmetic produces),
// the owner stores the entries with relaxed device-scope atomic stores, and
// a reader polls them with relaxed device-scope atomic loads, both coherent
// across the chip, until none is pending: one memory round trip per block,
// with no cache write-back or invalidation.  The workgroups draw (record,
// block) from a ticket counter in the order in which the blocks become
// ready, so a workgroup only ever waits on one that has already started, and
// every wait ends however many workgroups are resident at once.  Each wait
// is also bounded in time; past the bound (not expected) the workgroup
// writes NaN in its block, so that the failure shows in the result instead
// of stalling the device.  Each next block of M is loaded into registers
// before its wait.
//   MODE 0: L X = B    (unit lower L of the record's LU; blocks first to last)
//   MODE 1: U X = B    (upper U; last to first)
//   MODE 2: U^T X = B  (first to last; U read by columns)
//   MODE 3: L^T X = B  (last to first; L read by columns)
// Grid (A.nbm, records), 256 threads; the ticket is zero and X pending at
// launch.
// ---------------------------------------------------------------------------
constexpr long long kWaitTicks = 20000000;  // 0.2 s of the 100 MHz constant clock (default bound)

// Wave 0 of a reader: block b0 .. b0 + nbb - 1 of X, every right-hand side,
// into sx (lane = row of the block), polled until no entry is pending.
// Returns false past the time bound (wait ticks of the constant clock).
__device__ __forceinline__ bool sp_read_block(const double* X, int r, int b0, int nbb, int nv,
                                              double (*sx)[kNbT], long long wait) {
  const int lane = threadIdx.x & 63;
  const uint64_t* X64 = reinterpret_cast<const uint64_t*>(X);
  uint64_t got[kMaxV];
#pragma unroll
  for (int v = 0; v < kMaxV; ++v) got[v] = kXPending;
  const long long t0 = wall_clock64();
  bool ok = true;
  for (;;) {
    int ready = 1;
#pragma unroll
    for (int v = 0; v < kMaxV; ++v)
      if (v < nv && lane < nbb && got[v] == kXPending)
        got[v] = __hip_atomic_load(X64 + int64_t(v) * r + b0 + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int v = 0; v < kMaxV; ++v)
      if (v < nv && lane < nbb && got[v] == kXPending) ready = 0;
    if (__all(ready)) break;
    if (wall_clock64() - t0 > wait) {
      ok = false;
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
#pragma unroll
  for (int v = 0; v < kMaxV; ++v) sx[v][lane] = (v < nv && lane < nbb) ? __longlong_as_double((long long)got[v]) : 0.0;
  return ok;
}

template <int MODE>
__global__ __launch_bounds__(256) void k_sp_chain(SpArgs A) {
  constexpr bool kFwd = MODE == 0 || MODE == 2;
  constexpr bool kTrans = MODE >= 2;
  constexpr bool kUseU = MODE == 1 || MODE == 2;
  __shared__ unsigned s_ticket;
  __shared__ int s_ok;
  __shared__ double sM[kNbT][kNbT + 1];
  __shared__ double sD[kNbT][kNbT + 1];  // the diagonal block's inverse, staged before any wait
  __shared__ double sx[kMaxV][kNbT];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) {
    s_ticket = atomicAdd(A.sync, 1u);
    s_ok = 1;
  }
  __syncthreads();
  const unsigned t = s_ticket;
  const int rec = int(t / unsigned(A.nbm)), jj = int(t % unsigned(A.nbm));
  const SpRec R = sp_rec(A, rec);
  const int r = R.r, nbk = (r + kNbT - 1) / kNbT;
  if (jj >= nbk) return;
  const int j = kFwd ? jj : nbk - 1 - jj;
  const int j0 = j * kNbT, nb = min(kNbT, r - j0), nv = A.nv;
  const int ndep = kFwd ? j : nbk - 1 - j;
  // Element q of a thread is e = tid + 256 q of a 64 x 64 tile at (a, c):
  // (e / 64, e % 64) for a row-major read, (e % 64, e / 64) for a column
  // read, so consecutive threads read consecutive addresses either way.
  double pre[16], dpre[16];
  auto load_block = [&](int b) {
    const int b0 = b * kNbT, nbb = min(kNbT, r - b0);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + 256 * q, hi = e >> 6, lo = e & 63;
      const int a = kTrans ? lo : hi, c = kTrans ? hi : lo;
      pre[q] = (a < nb && c < nbb)
                   ? (kTrans ? R.LU[int64_t(b0 + c) * r + j0 + a] : R.LU[int64_t(j0 + a) * r + b0 + c])
                   : 0.0;
    }
  };
  auto store_tile = [&](double (*dst)[kNbT + 1], const double* v) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + 256 * q, hi = e >> 6, lo = e & 63;
      dst[kTrans ? lo : hi][kTrans ? hi : lo] = v[q];
    }
  };
  {
    // the stored inverse of the diagonal block, row-major; transposed for U^T, L^T
    const double* Dg = A.dinv + (int64_t(rec) * A.dnb + j) * 2 * kNbT * kNbT + (kUseU ? kNbT * kNbT : 0);
#pragma unroll
    for (int q = 0; q < 16; ++q) dpre[q] = Dg[tid + 256 * q];
  }
  // into LDS now: it depends on no other block, and the barriers below order
  // these stores before the product that reads them
  store_tile(sD, dpre);
  double acc[kMaxV / 4];
#pragma unroll
  for (int q = 0; q < kMaxV / 4; ++q) {
    const int v = wv + 4 * q;
    acc[q] = (v < nv && lane < nb) ? R.B[v * r + j0 + lane] : 0.0;
  }
  if (ndep > 0) load_block(kFwd ? 0 : nbk - 1);
  for (int d = 0; d < ndep; ++d) {
    const int b = kFwd ? d : nbk - 1 - d;
    // wave 0 waits for X_b and stages it in LDS; the other waves store the
    // prefetched tile meanwhile
    if (wv == 0) {
      const int b0 = b * kNbT;
      if (!sp_read_block(R.X, r, b0, min(kNbT, r - b0), nv, sx, A.wait_ticks) && lane == 0) s_ok = 0;
    }
    store_tile(sM, pre);
    __syncthreads();
    if (d + 1 < ndep) load_block(kFwd ? d + 1 : nbk - 2 - d);
#pragma unroll
    for (int q = 0; q < kMaxV / 4; ++q) {
      const int v = wv + 4 * q;
      if (v < nv) {
        double sum = 0.0;
#pragma unroll 16
        for (int c = 0; c < kNbT; ++c) sum += sM[lane][c] * sx[v][c];
        acc[q] -= sum;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kMaxV / 4; ++q) sx[wv + 4 * q][lane] = acc[q];
  __syncthreads();
  const bool ok = s_ok != 0;
  // X_j = D_j^{-1} B_j: each thread its row (lane) of its right-hand sides,
  // written straight from registers, entry by entry visible to the readers
  uint64_t* X64 = reinterpret_cast<uint64_t*>(R.X);
#pragma unroll
  for (int q = 0; q < kMaxV / 4; ++q) {
    const int v = wv + 4 * q;
    if (v < nv) {
      double y = 0.0;
#pragma unroll 16
      for (int c = 0; c < kNbT; ++c) y += sD[lane][c] * sx[v][c];
      if (lane < nb)
        __hip_atomic_store(X64 + int64_t(v) * r + j0 + lane, (uint64_t)__double_as_longlong(ok ? y : __builtin_nan("")),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

}  // namespace

void launch_make_perm(const GroupRec* recs, int nrec, int32_t* iarena, int max_r, hipStream_t s) {
  (void)max_r;
  hipLaunchKernelGGL(k_make_perm, dim3(nrec), dim3(64), 0, s, recs, iarena);
  HIF_HIP(hipGetLastError());
}

void launch_make_perm_top(const int32_t* piv, int32_t* perm, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_make_perm_top, dim3(1), dim3(64), 0, s, piv, perm, n);
  HIF_HIP(hipGetLastError());
}

// Dynamic LDS of the staged sweeps goes up to kCapL doubles (128 KiB).
static void allow_large_lds() {
  static std::once_flag once;
  std::call_once(once, [] {
    const int bytes = kCapL * int(sizeof(double));
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sweep_lds<64>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sweep_lds<128>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sweep_lds<256>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sweep_lds<1024>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipGetLastError();
  });
}

// Sub-levels whose sweeps run through the multi-workgroup path for nv
// right-hand sides per pass: records too large for LDS with all of them, or
// few records (at most kSplitMaxRecords) of at least kSplitMinR redundant
// unknowns, which one workgroup each would leave most of the chip idle.
#ifndef HIF_SPLIT_MAX_RECORDS
#define HIF_SPLIT_MAX_RECORDS 64
#endif
#ifndef HIF_SPLIT_MIN_R
#define HIF_SPLIT_MIN_R 128
#endif
constexpr int kSplitMaxRecords = HIF_SPLIT_MAX_RECORDS;
constexpr int kSplitMinR = HIF_SPLIT_MIN_R;
static bool split_solve(const SubLevel& sub, int64_t N, int nv) {
  return 2 * sub.sum_r <= N &&
         (int64_t(sub.max_2rk) * nv > kCapL || (sub.nrec <= kSplitMaxRecords && sub.max_r >= kSplitMinR));
}

// A top block too large for LDS is solved like a large record with no
// skeleton through the many-workgroup triangular solves.
static bool top_split_solve(const hif_factor_s* H) {
  return H->ntop >= kTopSplitMin && 2 * H->ntop <= H->n;
}

// The blocked triangular solve X = M^{-1} B of every record of a pass, one
// launch (k_sp_chain); mode as there.
static void chain(const SpArgs& P, int mode, unsigned nr, hipStream_t s) {
  const dim3 g(unsigned(P.nbm), nr);
  if (mode == 0)
    hipLaunchKernelGGL(k_sp_chain<0>, g, dim3(256), 0, s, P);
  else if (mode == 1)
    hipLaunchKernelGGL(k_sp_chain<1>, g, dim3(256), 0, s, P);
  else if (mode == 2)
    hipLaunchKernelGGL(k_sp_chain<2>, g, dim3(256), 0, s, P);
  else
    hipLaunchKernelGGL(k_sp_chain<3>, g, dim3(256), 0, s, P);
}

// The sweeps proper.  work: min(nrhs, 8) * N doubles of scratch, reused by
// every group of 8 right-hand sides (all launches are ordered on s).
static void sweep_run(hif_factor_s* H, int op, const double* x, double* y, int64_t nrhs, hipStream_t s,
                      double* work) {
  const int64_t N = H->n;
  const int64_t tot = N * nrhs;
  if (x != y) {
    int64_t blocks = (tot + 255) / 256;
    if (blocks > (1 << 20)) blocks = 1 << 20;
    hipLaunchKernelGGL(k_copy, dim3(unsigned(blocks)), dim3(256), 0, s, x, y, tot);
    HIF_HIP(hipGetLastError());
  }
  const long long wait_ticks = H->opts.sweep_wait_us > 0 ? 100ll * H->opts.sweep_wait_us : kWaitTicks;
  for (int64_t v0 = 0; v0 < nrhs; v0 += 8) {
    const int nv = int(std::min<int64_t>(8, nrhs - v0));
    double* u = y + v0 * N;
    double* wk = work;
    // solve / solve_T of a sub-level go through LDS when a group fits; the
    // four sweeps of few large records are spread over many workgroups per
    // record:
    //   solve   up:   B = P(u_r - T^T u_s); X = L^{-1} B;   u_s -= L_sr X; u_r = X
    //           down: B = u_r - U_rs u_s;   X = U^{-1} B;   u_s -= T X;    u_r = X
    //   solve_T up:   B = u_r - T^T u_s;    X = U^{-T} B;   u_s -= U_rs^T X; u_r = X
    //           down: B = u_r - L_sr^T u_s; X = L^{-T} B;   u_r = P^T X;   u_s -= T u_r
    //   apply   up:   B = u_r; u_s += T u_r;      X = U B + U_rs u_s;       u_r = X
    //           down: B = u_r; u_s += L_sr u_r;   X = L B; u_r = P^T X;     u_r += T^T u_s
    //   apply_T up:   B = P u_r; u_s += T u_r;    X = L^T B + L_sr^T u_s;   u_r = X
    //           down: B = u_r; u_s += U_rs^T u_r; X = U^T B; u_r = X;       u_r += T^T u_s
    auto sweep = [&](const SubLevel& sub, int down) {
      SwArgs A{sub.rec.p, sub.iarena.p, sub.darena.p, u, wk, N, nv, op};
      if (split_solve(sub, N, nv)) {
        HIF_REQUIRE(sub.dinv.p && H->sync.p, HIF_EDEVICE,
                    "the diagonal-block inverses of a sub-level were not built");
        SpArgs P{sub.rec.p,  sub.iarena.p, sub.darena.p, sub.woff.p, u, wk, wk + nv * sub.sum_r, N, nv,
                 sub.dinv.p, sub.dinv_nb};
        P.sync = H->sync.p;
        P.wait_ticks = wait_ticks;
        P.nbm = (sub.max_r + kNbT - 1) / kNbT;
        const unsigned nr = unsigned(sub.nrec);
        const dim3 gr(unsigned((sub.max_r + 255) / 256), nr), gu(unsigned((sub.max_r + 63) / 64), nr);
        const dim3 gw(unsigned((sub.max_r + 15) / 16), nr);
        const dim3 gs(unsigned((sub.max_k + 15) / 16), nr), gt(unsigned((sub.max_k + 63) / 64), nr);
        const bool sk = sub.max_k > 0;
        if (op == 0 && !down) {
          hipLaunchKernelGGL((k_sp_first_cols<false, true>), gu, dim3(256), 0, s, P);
          chain(P, 0, nr, s);
          if (sk) hipLaunchKernelGGL(k_sp_skel_update<false>, gs, dim3(256), 0, s, P, 0, -1.0);
          hipLaunchKernelGGL(k_sp_scatter<false>, gr, dim3(256), 0, s, P, 0);
        } else if (op == 0) {
          hipLaunchKernelGGL(k_sp_down_first, gw, dim3(256), 0, s, P);
          chain(P, 1, nr, s);
          if (sk) hipLaunchKernelGGL(k_sp_skel_update<false>, gs, dim3(256), 0, s, P, 1, -1.0);
          hipLaunchKernelGGL(k_sp_scatter<false>, gr, dim3(256), 0, s, P, 0);
        } else if (op == 1 && !down) {
          hipLaunchKernelGGL((k_sp_first_cols<false, false>), gu, dim3(256), 0, s, P);
          chain(P, 2, nr, s);
          if (sk) hipLaunchKernelGGL(k_sp_skel_update_T<false>, gt, dim3(256), 0, s, P, -1.0);
          hipLaunchKernelGGL(k_sp_scatter<false>, gr, dim3(256), 0, s, P, 0);
        } else if (op == 1) {
          hipLaunchKernelGGL((k_sp_first_cols<true, false>), gu, dim3(256), 0, s, P);
          chain(P, 3, nr, s);
          hipLaunchKernelGGL(k_sp_scatter<true>, gr, dim3(256), 0, s, P, 0);
          if (sk) hipLaunchKernelGGL(k_sp_skel_update<true>, gs, dim3(256), 0, s, P, 1, -1.0);
        } else if (op == 2 && !down) {
          hipLaunchKernelGGL(k_sp_gather<false>, gr, dim3(256), 0, s, P);
          if (sk) hipLaunchKernelGGL(k_sp_skel_update<true>, gs, dim3(256), 0, s, P, 1, 1.0);
          hipLaunchKernelGGL((k_sp_rowmv<0, true>), gw, dim3(256), 0, s, P, 0);
          hipLaunchKernelGGL(k_sp_scatter<false>, gr, dim3(256), 0, s, P, 0);
        } else if (op == 2) {
          hipLaunchKernelGGL(k_sp_gather<false>, gr, dim3(256), 0, s, P);
          if (sk) hipLaunchKernelGGL(k_sp_skel_update<true>, gs, dim3(256), 0, s, P, 0, 1.0);
          hipLaunchKernelGGL((k_sp_rowmv<1, false>), gw, dim3(256), 0, s, P, 0);
          hipLaunchKernelGGL(k_sp_scatter<true>, gr, dim3(256), 0, s, P, 0);
          if (sk) hipLaunchKernelGGL((k_sp_first_cols<false, false, true>), gu, dim3(256), 0, s, P);
        } else if (!down) {
          hipLaunchKernelGGL(k_sp_gather<true>, gr, dim3(256), 0, s, P);
          if (sk) hipLaunchKernelGGL(k_sp_skel_update<true>, gs, dim3(256), 0, s, P, 1, 1.0);
          hipLaunchKernelGGL((k_sp_colmv<2, true>), gu, dim3(256), 0, s, P, 0);
          hipLaunchKernelGGL(k_sp_scatter<false>, gr, dim3(256), 0, s, P, 0);
        } else {
          hipLaunchKernelGGL(k_sp_gather<false>, gr, dim3(256), 0, s, P);
          if (sk) hipLaunchKernelGGL(k_sp_skel_update_T<true>, gt, dim3(256), 0, s, P, 1.0);
          hipLaunchKernelGGL((k_sp_colmv<3, false>), gu, dim3(256), 0, s, P, 0);
          hipLaunchKernelGGL(k_sp_scatter<false>, gr, dim3(256), 0, s, P, 0);
          if (sk) hipLaunchKernelGGL((k_sp_first_cols<false, false, true>), gu, dim3(256), 0, s, P);
        }
        return;
      }
      if (sub.max_2rk <= kCapL) {
        allow_large_lds();
        // LDS for as many right-hand sides per pass as fit (all of them when
        // the records are small); 1024 threads per record when the records
        // are too few to give every CU several workgroups
        const int nvb = std::max(1, std::min(nv, kCapL / sub.max_2rk));
        const int cap = nvb * sub.max_2rk;
        const size_t lds = size_t(cap) * sizeof(double);
        const int many = tuning().sweep_many_threads;
        if (sub.nrec >= kManyRecords && many == 64)
          hipLaunchKernelGGL(k_sweep_lds<64>, dim3(sub.nrec), dim3(64), lds, s, A, down, cap);
        else if (sub.nrec >= kManyRecords && many == 128)
          hipLaunchKernelGGL(k_sweep_lds<128>, dim3(sub.nrec), dim3(128), lds, s, A, down, cap);
        else if (sub.nrec >= kManyRecords)
          hipLaunchKernelGGL(k_sweep_lds<256>, dim3(sub.nrec), dim3(256), lds, s, A, down, cap);
        else
          hipLaunchKernelGGL(k_sweep_lds<1024>, dim3(sub.nrec), dim3(1024), lds, s, A, down, cap);
      } else if (down)
        hipLaunchKernelGGL(k_down, dim3(sub.nrec), dim3(kBlock), 0, s, A);
      else
        hipLaunchKernelGGL(k_up, dim3(sub.nrec), dim3(kBlock), 0, s, A);
    };
    for (auto& sub : H->subs)
      if (sub.nrec > 0) sweep(sub, 0);
    // A top block too large for LDS is swept like a large record with no
    // skeleton (k = 0), through the same chained triangular solves and
    // products: solve X = U^{-1} L^{-1} P u, solve_T X = P^T L^{-T} U^{-T} u,
    // apply X = P^T L U u, apply_T X = U^T L^T P u.
    const bool top_split = top_split_solve(H);
    if (top_split) {
      const int r = int(H->ntop);
      HIF_REQUIRE(H->top_rec.p && H->top_dinv.p && H->sync.p, HIF_EDEVICE,
                  "the top block's solve record was not built with the factors");
      const int nbk = (r + kNbT - 1) / kNbT;
      SpArgs P{H->top_rec.p, H->top_iarena.p, H->top_lu.p,  H->top_woff.p, u, wk, wk + int64_t(nv) * r, N, nv,
               H->top_dinv.p, nbk};
      P.sync = H->sync.p;
      P.wait_ticks = wait_ticks;
      P.nbm = nbk;
      const dim3 gr(unsigned((r + 255) / 256), 1), gu(unsigned((r + 63) / 64), 1), gw(unsigned((r + 15) / 16), 1);
      if (op == 0) {
        hipLaunchKernelGGL((k_sp_first_cols<false, true>), gu, dim3(256), 0, s, P);
        chain(P, 0, 1, s);
        hipLaunchKernelGGL(k_sp_scatter<false>, gr, dim3(256), 0, s, P, 0);
        hipLaunchKernelGGL(k_sp_down_first, gw, dim3(256), 0, s, P);
        chain(P, 1, 1, s);
        hipLaunchKernelGGL(k_sp_scatter<false>, gr, dim3(256), 0, s, P, 0);
      } else if (op == 1) {
        hipLaunchKernelGGL((k_sp_first_cols<false, false>), gu, dim3(256), 0, s, P);
        chain(P, 2, 1, s);
        hipLaunchKernelGGL(k_sp_scatter<false>, gr, dim3(256), 0, s, P, 0);
        hipLaunchKernelGGL((k_sp_first_cols<true, false>), gu, dim3(256), 0, s, P);
        chain(P, 3, 1, s);
        hipLaunchKernelGGL(k_sp_scatter<true>, gr, dim3(256), 0, s, P, 0);
      } else if (op == 2) {
        hipLaunchKernelGGL(k_sp_gather<false>, gr, dim3(256), 0, s, P);
        hipLaunchKernelGGL((k_sp_rowmv<0, false>), gw, dim3(256), 0, s, P, 0);
        hipLaunchKernelGGL((k_sp_rowmv<1, false>), gw, dim3(256), 0, s, P, 1);
        hipLaunchKernelGGL(k_sp_scatter<true>, gr, dim3(256), 0, s, P, 1);
      } else {
        hipLaunchKernelGGL(k_sp_gather<true>, gr, dim3(256), 0, s, P);
        hipLaunchKernelGGL((k_sp_colmv<2, false>), gu, dim3(256), 0, s, P, 0);
        hipLaunchKernelGGL((k_sp_colmv<3, false>), gu, dim3(256), 0, s, P, 1);
        hipLaunchKernelGGL(k_sp_scatter<false>, gr, dim3(256), 0, s, P, 1);
      }
    } else if (H->ntop > 0) {
      if (2 * H->ntop <= kCapL)
        hipLaunchKernelGGL(k_top_lds, dim3(1), dim3(1024), 0, s, H->top_lu.p, H->top_perm.p, int(H->ntop),
                           H->top_idx.p, u, N, nv, op);
      else
        hipLaunchKernelGGL(k_top, dim3(1), dim3(1024), 0, s, H->top_lu.p, H->top_piv.p, int(H->ntop), H->top_idx.p,
                           u, wk, N, nv, op);
    }
    for (auto it = H->subs.rbegin(); it != H->subs.rend(); ++it)
      if (it->nrec > 0) sweep(*it, 1);
    HIF_HIP(hipGetLastError());
  }
}



// Diagonal-block inverses of the sub-levels (and the top block) whose solve
// can take the multi-workgroup path, for any number of right-hand sides per
// pass (at most kMaxV).
static void build_dinv(hif_factor_s* H, hipStream_t s) {
  for (SubLevel& sub : H->subs) {
    if (sub.nrec == 0 || sub.dinv.p || !split_solve(sub, H->n, kMaxV)) continue;
    sub.dinv_nb = (sub.max_r + kNbT - 1) / kNbT;
    sub.dinv.alloc(size_t(sub.nrec) * sub.dinv_nb * 2 * kNbT * kNbT, &H->mem);
    SpArgs P{sub.rec.p, sub.iarena.p, sub.darena.p, sub.woff.p, nullptr, nullptr, nullptr, H->n, 1,
             nullptr, sub.dinv_nb};
    hipLaunchKernelGGL(k_sp_dinv, dim3(unsigned(sub.dinv_nb), unsigned(sub.nrec)), dim3(64), 0, s, P, sub.dinv.p);
  }
  HIF_HIP(hipGetLastError());
}

void prepare_sweeps(hif_factor_s* H, hipStream_t s) {
  build_dinv(H, s);
  // the ticket counter of the chained triangular solves
  bool chained = top_split_solve(H);
  for (const SubLevel& sub : H->subs) chained = chained || sub.dinv.p != nullptr;
  if (chained && !H->sync.p) H->sync.alloc(1, &H->mem);
  if (!top_split_solve(H) || H->top_rec.p) return;
  const int r = int(H->ntop);
  H->top_iarena.alloc(size_t(3) * r, &H->mem);
  HIF_HIP(hipMemcpyAsync(H->top_iarena.p, H->top_idx.p, sizeof(int32_t) * r, hipMemcpyDeviceToDevice, s));
  HIF_HIP(hipMemcpyAsync(H->top_iarena.p + r, H->top_piv.p, sizeof(int32_t) * r, hipMemcpyDeviceToDevice, s));
  HIF_HIP(hipMemcpyAsync(H->top_iarena.p + 2 * r, H->top_perm.p, sizeof(int32_t) * r, hipMemcpyDeviceToDevice, s));
  const GroupRec rec{r, 0, 0, 0};
  const int64_t wo = 0;
  H->top_rec.alloc(1, &H->mem);
  H->top_woff.alloc(1, &H->mem);
  HIF_HIP(hipMemcpyAsync(H->top_rec.p, &rec, sizeof(GroupRec), hipMemcpyHostToDevice, s));
  HIF_HIP(hipMemcpyAsync(H->top_woff.p, &wo, sizeof(int64_t), hipMemcpyHostToDevice, s));
  const int nbk = (r + kNbT - 1) / kNbT;
  H->top_dinv.alloc(size_t(nbk) * 2 * kNbT * kNbT, &H->mem);
  SpArgs P{H->top_rec.p, H->top_iarena.p, H->top_lu.p, H->top_woff.p, nullptr, nullptr, nullptr, H->n, 1,
           nullptr, nbk};
  hipLaunchKernelGGL(k_sp_dinv, dim3(unsigned(nbk), 1), dim3(64), 0, s, P, H->top_dinv.p);
  HIF_HIP(hipGetLastError());
  HIF_HIP(hipStreamSynchronize(s));  // the host values above are copied before they go out of scope
}

void sweep_impl(hif_factor_s* H, int op, const double* x, double* y, int64_t nrhs, hipStream_t s) {
  H->work.ensure(std::min<int64_t>(nrhs, 8) * H->n, &H->mem);
  sweep_run(H, op, x, y, nrhs, s, H->work.p);
}

// The launches of one solve u = F^{-1} f recorded into a HIP graph by stream
// capture on a private stream (kernel nodes only), then instantiated.  The
// sweep scratch is allocated before the capture starts.
void graph_solve_impl(hif_factor_s* H, const double* f, double* u, int64_t nrhs, hipStream_t cs,
                      hipGraph_t* graph, hipGraphExec_t* exec) {
  H->work.ensure(std::min<int64_t>(nrhs, 8) * H->n, &H->mem);
  allow_large_lds();
  HIF_HIP(hipStreamSynchronize(cs));
  HIF_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  try {
    sweep_run(H, 0, f, u, nrhs, cs, H->work.p);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(cs, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  HIF_HIP(hipStreamEndCapture(cs, graph));
  const hipError_t e = hipGraphInstantiate(exec, *graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(*graph);
    *graph = nullptr;
    throw Error{HIF_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
  }
}

// ---------------------------------------------------------------------------
// Solve without allocation (hif_solve_noalloc): the sweep scratch is this
// file-scope device array instead of the handle's work buffer.  Each device
// holds its own copy; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in).  Calls that overlap on one device share it and race.
// ---------------------------------------------------------------------------
namespace {
__device__ __align__(256) double scratch[kSolveScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

double* scratch_ptr() {
  int dev = 0;
  HIF_HIP(hipGetDevice(&dev));
  HIF_REQUIRE(dev >= 0 && dev < kMaxDevices, HIF_EDEVICE, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error{HIF_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}
}  // namespace

void sweep_noalloc_impl(hif_factor_s* H, const double* f, double* u, int64_t nrhs, hipStream_t s) {
  const int64_t need = std::min<int64_t>(nrhs, 8) * H->n;
  HIF_REQUIRE(need <= int64_t(kSolveScratchDoubles), HIF_EINVAL,
              "min(nrhs, 8) * n = " + std::to_string(need) + " exceeds the " +
                  std::to_string(kSolveScratchDoubles) + " doubles of the solve scratch");
  double* work = scratch_ptr();
  sweep_run(H, 0, f, u, nrhs, s, work);
}

}  // namespace hif
