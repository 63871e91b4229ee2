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

#include "common.h"

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
#pragma unroll
    for (int v = 0; v < kMaxV; ++v)
      if (v < nv) {
        const double t = wave_sum(acc[v]);
        if (lane == 0) y[v * ys + i] += sgn * t;
      }
  }
}

// y[v*ys + j] += sgn * sum_i M[i*ld + j] x[v*xs + i]   (one thread per column)
__device__ __forceinline__ void l_gemv_t(const double* __restrict__ M, int nrow, int ncol, int ld, const double* x, int xs, double* y,
                         int ys, int nv, double sgn) {
  for (int j = threadIdx.x; j < ncol; j += blockDim.x) {
    double acc[kMaxV];
#pragma unroll
    for (int v = 0; v < kMaxV; ++v) acc[v] = 0.0;
    for (int i0 = 0; i0 < nrow; i0 += kU) {
      double mv[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) mv[u] = i0 + u < nrow ? M[int64_t(i0 + u) * ld + j] : 0.0;
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (i0 + u < nrow) {
#pragma unroll
          for (int v = 0; v < kMaxV; ++v)
            if (v < nv) acc[v] += mv[u] * x[v * xs + i0 + u];
        }
    }
#pragma unroll
    for (int v = 0; v < kMaxV; ++v)
      if (v < nv) y[v * ys + j] += sgn * acc[v];
  }
}

// acc[v] = sum_{c < nb} seg[c * cs] x[v*xs + x0 + c]  (a row or column segment of LU)
__device__ __forceinline__ void seg_dot(const double* seg, int64_t cs, int nb, const double* x, int xs, int x0, int nv,
                                        double (&acc)[kMaxV]) {
#pragma unroll
  for (int v = 0; v < kMaxV; ++v) acc[v] = 0.0;
  for (int c0 = 0; c0 < nb; c0 += kU) {
    double l[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) l[u] = c0 + u < nb ? seg[(c0 + u) * cs] : 0.0;
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (c0 + u < nb) {
#pragma unroll
        for (int v = 0; v < kMaxV; ++v)
          if (v < nv) acc[v] += l[u] * x[v * xs + x0 + c0 + u];
      }
  }
}

// x = L^{-1} x, L the unit lower triangle of the row-major n x n LU.
__device__ __forceinline__ void l_solve_L(const double* __restrict__ LU, int n, double* x, int xs, int nv) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
  for (int j0 = 0; j0 < n; j0 += kNbT) {
    const int nb = min(kNbT, n - j0);
    const double* Lr = LU + int64_t(j0 + min(lane, nb - 1)) * n + j0;
    for (int v = wv; v < nv; v += nw) {
      double xi = lane < nb ? x[v * xs + j0 + lane] : 0.0;
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
          }
        }
      }
      if (lane < nb) x[v * xs + j0 + lane] = xi;
    }
    __syncthreads();
    for (int i = j0 + nb + tid; i < n; i += blockDim.x) {
      double acc[kMaxV];
      seg_dot(LU + int64_t(i) * n + j0, 1, nb, x, xs, j0, nv, acc);
#pragma unroll
      for (int v = 0; v < kMaxV; ++v)
        if (v < nv) x[v * xs + i] -= acc[v];
    }
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
    for (int v = wv; v < nv; v += nw) {
      double xi = lane < nb ? x[v * xs + j0 + lane] : 0.0;
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
          }
        }
      }
      if (lane < nb) x[v * xs + j0 + lane] = xi;
    }
    __syncthreads();
    for (int i = tid; i < j0; i += blockDim.x) {
      double acc[kMaxV];
      seg_dot(LU + int64_t(i) * n + j0, 1, nb, x, xs, j0, nv, acc);
#pragma unroll
      for (int v = 0; v < kMaxV; ++v)
        if (v < nv) x[v * xs + i] -= acc[v];
    }
    __syncthreads();
  }
}

// x = U^{-T} x (U^T lower with diagonal U_jj), forward over column blocks.
__device__ __forceinline__ void l_solve_UT(const double* __restrict__ LU, int n, double* x, int xs, int nv) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
  for (int j0 = 0; j0 < n; j0 += kNbT) {
    const int nb = min(kNbT, n - j0);
    const int cl = j0 + min(lane, nb - 1);
    for (int v = wv; v < nv; v += nw) {
      double xi = lane < nb ? x[v * xs + j0 + lane] : 0.0;
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
          }
        }
      }
      if (lane < nb) x[v * xs + j0 + lane] = xi;
    }
    __syncthreads();
    for (int i = j0 + nb + tid; i < n; i += blockDim.x) {
      double acc[kMaxV];
      seg_dot(LU + int64_t(j0) * n + i, n, nb, x, xs, j0, nv, acc);
#pragma unroll
      for (int v = 0; v < kMaxV; ++v)
        if (v < nv) x[v * xs + i] -= acc[v];
    }
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
    for (int v = wv; v < nv; v += nw) {
      double xi = lane < nb ? x[v * xs + j0 + lane] : 0.0;
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
          }
        }
      }
      if (lane < nb) x[v * xs + j0 + lane] = xi;
    }
    __syncthreads();
    for (int i = tid; i < j0; i += blockDim.x) {
      double acc[kMaxV];
      seg_dot(LU + int64_t(j0) * n + i, n, nb, x, xs, j0, nv, acc);
#pragma unroll
      for (int v = 0; v < kMaxV; ++v)
        if (v < nv) x[v * xs + i] -= acc[v];
    }
    __syncthreads();
  }
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

// One group per workgroup of BS threads; op 0 solve, 1 solve_T; down = 0 for
// the upward sweep (finest sub-level first), 1 for the downward one.  The LDS
// holds cap doubles (sized by the launch to the sub-level's largest record);
// the caller guarantees 2r + k <= cap.
template <int BS>
__global__ __launch_bounds__(BS) void k_sweep_lds(SwArgs A, int down, int cap) {
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
    } else if (!down) {
      if (k > 0) l_gemv_t(T, k, r, r, xs, k, xr, r, nv, -1.0);    // u_r -= T^T u_s
      __syncthreads();
      l_solve_UT(LU, r, xr, r, nv);                                // u_r = U^{-T} u_r
      if (k > 0) l_gemv_t(Urs, r, k, k, xr, r, xs, k, nv, -1.0);  // u_s -= U_rs^T u_r
    } else {
      if (k > 0) l_gemv_t(Lsr, k, r, r, xs, k, xr, r, nv, -1.0);  // u_r -= L_sr^T u_s
      __syncthreads();
      l_solve_LT(LU, r, xr, r, nv);                                // u_r = L^{-T} u_r
      l_permute(perm, r, xr, tp, nv, false);                       // u_r = P^T u_r
      if (k > 0) l_gemv_n(T, k, r, r, xr, r, xs, k, nv, -1.0);    // u_s -= T u_r
    }
    __syncthreads();
    for (int e = tid; e < nv * r; e += BS) u[(e / r) * N + rd[e % r]] = xr[e];
    for (int e = tid; e < nv * k; e += BS) u[(e / k) * N + sk[e % k]] = xs[e];
    __syncthreads();
  }
}

// Top block: x = A_L^{-1} x (op 0) or A_L^{-T} x (op 1); requires 2n <= kCapL.
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
    } else {
      l_solve_UT(LU, n, x, n, nv);
      l_solve_LT(LU, n, x, n, nv);
      l_permute(perm, n, x, tp, nv, false);
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
// Solve (op 0) for sub-levels with few, large records: each record is spread
// over many workgroups and all right-hand sides go through its factors in one
// pass (the LDS kernel above holds 2r + k entries per right-hand side and so
// rereads large factors once per right-hand side).  Per record, B holds the
// right-hand sides of the triangular solve and X its solution, both [nv][r]
// at nv * woff in the work buffer.  The products with T, L_sr and U_rs are
// spread over many workgroups per record; each triangular solve takes one
// launch per 64-row block and multiplies the block by the stored inverse of
// its diagonal block.
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

constexpr int kSpChunk = 512;  // skeleton entries staged in LDS per pass

// Up, first step: B(v, i) = (P (u_r - T^T u_s))(v, i): 64 rows i per
// workgroup, lane per row, the sum over the skeleton split between the 4 waves
// and added through LDS.
__global__ __launch_bounds__(256) void k_sp_up_first(SpArgs A) {
  const SpRec R = sp_rec(A, blockIdx.y);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;  // 64 rows per workgroup
  if (blockIdx.x * 64 >= R.r) return;
  const int nv = A.nv;
  __shared__ double sus[kMaxV][kSpChunk];
  __shared__ double sred[4][kMaxV][64];
  const int c = i < R.r ? R.perm[i] : 0;
  double acc[kMaxV];
#pragma unroll
  for (int v = 0; v < kMaxV; ++v) acc[v] = 0.0;
  for (int j0 = 0; j0 < R.k; j0 += kSpChunk) {
    const int nj = min(kSpChunk, R.k - j0);
    __syncthreads();
    for (int e = threadIdx.x; e < nv * nj; e += 256) sus[e / nj][e % nj] = A.u[(e / nj) * A.N + R.sk[j0 + e % nj]];
    __syncthreads();
    // wave wv takes the quarter [jb, je) of the chunk
    const int jb = (nj * wv) / 4, je = (nj * (wv + 1)) / 4;
    if (i < R.r) {
      const double* tc = R.T + int64_t(j0) * R.r + c;
      for (int j = jb; j < je; j += kU) {
        double t[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) t[u] = j + u < je ? tc[int64_t(j + u) * R.r] : 0.0;
#pragma unroll
        for (int u = 0; u < kU; ++u)
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
      if (v < nv)
        R.B[v * R.r + i] =
            A.u[v * A.N + R.rd[c]] - ((sred[0][v][lane] + sred[1][v][lane]) + (sred[2][v][lane] + sred[3][v][lane]));
}

// Down, first step: B(v, i) = (u_r - U_rs u_s)(v, i), one wave per row i.
__global__ __launch_bounds__(256) void k_sp_down_first(SpArgs A) {
  const SpRec R = sp_rec(A, blockIdx.y);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i0 = blockIdx.x * 16;  // 16 rows per workgroup, 4 per wave
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
    for (int e = threadIdx.x; e < nv * nj; e += 256) sus[e / nj][e % nj] = A.u[(e / nj) * A.N + R.sk[j0 + e % nj]];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + wv * 4 + q;
      if (i >= R.r) break;
      const double* mr = R.Urs + int64_t(i) * R.k + j0;
      for (int j = lane; j < nj; j += 64) {
        const double m = mr[j];
#pragma unroll
        for (int v = 0; v < kMaxV; ++v)
          if (v < nv) acc[q][v] += m * sus[v][j];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = i0 + wv * 4 + q;
    if (i >= R.r) break;
#pragma unroll
    for (int v = 0; v < kMaxV; ++v)
      if (v < nv) {
        const double t = wave_sum(acc[q][v]);
        if (lane == 0) R.B[v * R.r + i] = A.u[v * A.N + R.rd[i]] - t;
      }
  }
}

// u_s -= M X (M = L_sr or T, k x r), one wave per skeleton row; X staged in
// LDS by chunks of columns.
__global__ __launch_bounds__(256) void k_sp_skel_update(SpArgs A, int which) {
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
    for (int e = threadIdx.x; e < nv * nc; e += 256) sx[e / nc][e % nc] = R.X[(e / nc) * R.r + c0 + e % nc];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + wv * 4 + q;
      if (j >= R.k) break;
      const double* mr = M + int64_t(j) * R.r + c0;
      for (int c = lane; c < nc; c += 64) {
        const double m = mr[c];
#pragma unroll
        for (int v = 0; v < kMaxV; ++v)
          if (v < nv) acc[q][v] += m * sx[v][c];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = j0 + wv * 4 + q;
    if (j >= R.k) break;
#pragma unroll
    for (int v = 0; v < kMaxV; ++v)
      if (v < nv) {
        const double t = wave_sum(acc[q][v]);
        if (lane == 0) A.u[v * A.N + R.sk[j]] -= t;
      }
  }
}

// u_r = X.
__global__ __launch_bounds__(256) void k_sp_scatter(SpArgs A) {
  const SpRec R = sp_rec(A, blockIdx.y);
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= R.r) return;
  for (int v = 0; v < A.nv; ++v) A.u[v * A.N + R.rd[i]] = R.X[v * R.r + i];
}

// x = D^{-1} x for the nv right-hand sides of one 64-row block, with D^{-1}
// (the inverse of the block's diagonal block of L or U) in sD: row a per
// lane, right-hand sides v = wave, wave + 4.  256 threads; ends synchronized.
__device__ __forceinline__ void diag_apply(const double (*sD)[kNbT + 1], double (*sx)[kNbT], int nv) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double y[kMaxV / 4];
#pragma unroll
  for (int q = 0; q < kMaxV / 4; ++q) {
    const int v = wv + 4 * q;
    double acc = 0.0;
    if (v < nv)
#pragma unroll 16
      for (int c = 0; c < kNbT; ++c) acc += sD[lane][c] * sx[v][c];
    y[q] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kMaxV / 4; ++q)
    if (wv + 4 * q < nv) sx[wv + 4 * q][lane] = y[q];
  __syncthreads();
}

// Inverses of the diagonal blocks of the records' L (unit lower) and U
// (upper) for the blocked solves below: workgroup (b, i) inverts block b of
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

// Block b of x = L^{-1} x (unit lower L of the LU): workgroup 0 writes X of
// the block, workgroup w >= 1 updates B rows 64(b + w) .. +63; every
// workgroup first multiplies the block by the stored inverse of its diagonal
// block (spread over many workgroups: one workgroup walking all blocks of a
// large record is bound by the latency of its row updates).
__global__ __launch_bounds__(256) void k_sp_lsolve(SpArgs A, int b) {
  const SpRec R = sp_rec(A, blockIdx.y);
  const int j0 = b * kNbT;
  if (j0 >= R.r) return;
  const int w = blockIdx.x;
  const int i0 = j0 + w * kNbT;
  if (i0 >= R.r) return;
  const int nb = min(kNbT, R.r - j0), nv = A.nv, r = R.r;
  const int tid = threadIdx.x;
  __shared__ double sL[kNbT][kNbT + 1];
  __shared__ double sx[kMaxV][kNbT];
  const double* Li = A.dinv + (int64_t(blockIdx.y) * A.dnb + b) * 2 * kNbT * kNbT;
  for (int e = tid; e < kNbT * kNbT; e += 256) sL[e >> 6][e & 63] = Li[e];
  for (int e = tid; e < nv * kNbT; e += 256) {
    const int v = e >> 6, a = e & 63;
    sx[v][a] = a < nb ? R.B[v * r + j0 + a] : 0.0;
  }
  __syncthreads();
  diag_apply(sL, sx, nv);
  if (w == 0) {
    for (int e = tid; e < nv * nb; e += 256) R.X[(e / nb) * r + j0 + e % nb] = sx[e / nb][e % nb];
    return;
  }
  // rows i0 + tid / 4, four threads per row over 16 columns each
  const int i = i0 + (tid >> 2), part = tid & 3;
  double acc[kMaxV];
#pragma unroll
  for (int v = 0; v < kMaxV; ++v) acc[v] = 0.0;
  if (i < r) {
    const double* lr = R.LU + int64_t(i) * r + j0 + part * 16;
    double l[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) l[c] = part * 16 + c < nb ? lr[c] : 0.0;
#pragma unroll
    for (int c = 0; c < 16; ++c)
#pragma unroll
      for (int v = 0; v < kMaxV; ++v)
        if (v < nv) acc[v] += l[c] * sx[v][part * 16 + c];
  }
#pragma unroll
  for (int v = 0; v < kMaxV; ++v) {
    acc[v] += __shfl_xor(acc[v], 1, 64);
    acc[v] += __shfl_xor(acc[v], 2, 64);
  }
  if (i < r && part == 0)
#pragma unroll
    for (int v = 0; v < kMaxV; ++v)
      if (v < nv) R.B[v * r + i] -= acc[v];
}

// Block b of x = U^{-1} x (upper U of the LU), blocks visited last to first.
// Workgroup 0 writes X of the block; workgroup w >= 1 updates B rows
// 64(w - 1) .. +63 above the block.
__global__ __launch_bounds__(256) void k_sp_usolve(SpArgs A, int b) {
  const SpRec R = sp_rec(A, blockIdx.y);
  const int j0 = b * kNbT;
  if (j0 >= R.r) return;
  const int w = blockIdx.x;
  const int i0 = (w - 1) * kNbT;
  if (w > 0 && i0 >= j0) return;
  const int nb = min(kNbT, R.r - j0), nv = A.nv, r = R.r;
  const int tid = threadIdx.x;
  __shared__ double sU[kNbT][kNbT + 1];
  __shared__ double sx[kMaxV][kNbT];
  const double* Ui = A.dinv + (int64_t(blockIdx.y) * A.dnb + b) * 2 * kNbT * kNbT + kNbT * kNbT;
  for (int e = tid; e < kNbT * kNbT; e += 256) sU[e >> 6][e & 63] = Ui[e];
  for (int e = tid; e < nv * kNbT; e += 256) {
    const int v = e >> 6, a = e & 63;
    sx[v][a] = a < nb ? R.B[v * r + j0 + a] : 0.0;
  }
  __syncthreads();
  diag_apply(sU, sx, nv);
  if (w == 0) {
    for (int e = tid; e < nv * nb; e += 256) R.X[(e / nb) * r + j0 + e % nb] = sx[e / nb][e % nb];
    return;
  }
  const int i = i0 + (tid >> 2), part = tid & 3;
  double acc[kMaxV];
#pragma unroll
  for (int v = 0; v < kMaxV; ++v) acc[v] = 0.0;
  {
    const double* ur = R.LU + int64_t(i) * r + j0 + part * 16;
    double l[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) l[c] = part * 16 + c < nb ? ur[c] : 0.0;
#pragma unroll
    for (int c = 0; c < 16; ++c)
#pragma unroll
      for (int v = 0; v < kMaxV; ++v)
        if (v < nv) acc[v] += l[c] * sx[v][part * 16 + c];
  }
#pragma unroll
  for (int v = 0; v < kMaxV; ++v) {
    acc[v] += __shfl_xor(acc[v], 1, 64);
    acc[v] += __shfl_xor(acc[v], 2, 64);
  }
  if (part == 0)
#pragma unroll
    for (int v = 0; v < kMaxV; ++v)
      if (v < nv) R.B[v * r + i] -= acc[v];
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

// Sub-levels whose solve runs through the multi-workgroup path for nv
// right-hand sides per pass: records too large for LDS with all of them, or
// few large records.
static bool split_solve(const SubLevel& sub, int64_t N, int nv) {
  return 2 * sub.sum_r <= N && (int64_t(sub.max_2rk) * nv > kCapL || (sub.nrec <= 64 && sub.max_r >= 256));
}

// A top block too large for LDS is solved like a large record with no
// skeleton through the many-workgroup triangular solves.
static bool top_split_solve(const hif_factor_s* H) {
  return H->ntop >= kTopSplitMin && 2 * H->ntop <= H->n;
}

// The triangular solves of the multi-workgroup path: one launch per 64-row
// block.
static void trsv(const SpArgs& P, unsigned nr, int nbk, bool lower, hipStream_t s) {
  if (lower)
    for (int b = 0; b < nbk; ++b) hipLaunchKernelGGL(k_sp_lsolve, dim3(unsigned(nbk - b), nr), dim3(256), 0, s, P, b);
  else
    for (int b = nbk - 1; b >= 0; --b) hipLaunchKernelGGL(k_sp_usolve, dim3(unsigned(b + 1), nr), dim3(256), 0, s, P, b);
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
  for (int64_t v0 = 0; v0 < nrhs; v0 += 8) {
    const int nv = int(std::min<int64_t>(8, nrhs - v0));
    double* u = y + v0 * N;
    double* wk = work;
    // solve / solve_T of a sub-level go through LDS when a group fits; solve
    // of few large records is spread over many workgroups per record
    auto sweep = [&](const SubLevel& sub, int down) {
      SwArgs A{sub.rec.p, sub.iarena.p, sub.darena.p, u, wk, N, nv, op};
      const bool split = op == 0 && split_solve(sub, N, nv);
      if (split) {
        HIF_REQUIRE(sub.dinv.p, HIF_EDEVICE, "the diagonal-block inverses of a sub-level were not built");
        SpArgs P{sub.rec.p,  sub.iarena.p, sub.darena.p, sub.woff.p, u, wk, wk + nv * sub.sum_r, N, nv,
                 sub.dinv.p, sub.dinv_nb};
        const unsigned nr = unsigned(sub.nrec);
        const int nbk = (sub.max_r + kNbT - 1) / kNbT;
        const dim3 gr(unsigned((sub.max_r + 255) / 256), nr), gu(unsigned((sub.max_r + 63) / 64), nr);
        const dim3 gs(unsigned((sub.max_k + 15) / 16), nr);
        if (!down) {
          hipLaunchKernelGGL(k_sp_up_first, gu, dim3(256), 0, s, P);
          trsv(P, nr, nbk, true, s);
          if (sub.max_k > 0) hipLaunchKernelGGL(k_sp_skel_update, gs, dim3(256), 0, s, P, 0);
        } else {
          hipLaunchKernelGGL(k_sp_down_first, dim3(unsigned((sub.max_r + 15) / 16), nr), dim3(256), 0, s, P);
          trsv(P, nr, nbk, false, s);
          if (sub.max_k > 0) hipLaunchKernelGGL(k_sp_skel_update, gs, dim3(256), 0, s, P, 1);
        }
        hipLaunchKernelGGL(k_sp_scatter, gr, dim3(256), 0, s, P);
        return;
      }
      if (op <= 1 && sub.max_2rk <= kCapL) {
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
    // A top block too large for LDS is solved like a large record with no
    // skeleton (k = 0): the same blocked triangular solves spread over many
    // workgroups, with the up pass (P, L^{-1}) and the down pass (U^{-1}).
    const bool top_split = op == 0 && top_split_solve(H);
    if (top_split) {
      const int r = int(H->ntop);
      HIF_REQUIRE(H->top_rec.p && H->top_dinv.p, HIF_EDEVICE,
                  "the top block's solve record was not built with the factors");
      const int nbk = (r + kNbT - 1) / kNbT;
      SpArgs P{H->top_rec.p, H->top_iarena.p, H->top_lu.p,  H->top_woff.p, u, wk, wk + int64_t(nv) * r, N, nv,
               H->top_dinv.p, nbk};
      const dim3 gr(unsigned((r + 255) / 256), 1);
      hipLaunchKernelGGL(k_sp_up_first, dim3(unsigned((r + 63) / 64), 1), dim3(256), 0, s, P);
      trsv(P, 1, nbk, true, s);
      hipLaunchKernelGGL(k_sp_scatter, gr, dim3(256), 0, s, P);
      hipLaunchKernelGGL(k_sp_down_first, dim3(unsigned((r + 15) / 16), 1), dim3(256), 0, s, P);
      trsv(P, 1, nbk, false, s);
      hipLaunchKernelGGL(k_sp_scatter, gr, dim3(256), 0, s, P);
    } else if (H->ntop > 0) {
      if (op <= 1 && 2 * H->ntop <= kCapL)
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
