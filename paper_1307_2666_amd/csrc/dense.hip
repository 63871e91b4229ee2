// Per-group dense kernels of the factorization: batched assembly of the
// compressed blocks, batched interpolative decomposition, batched
// skeletonization / elimination, and the top block LU.
//
// All kernels run one workgroup per independent problem (the groups of one
// sub-level commute, Section 2.3), on row-major blocks in device memory.
#include <algorithm>
#include <climits>
#include <vector>

#include "batched.h"
#include "gemm.h"
#include "kernels.h"
#include "wave.h"

namespace hif {

// ---------------------------------------------------------------------------
// Block-wide reductions (wave64, up to 1024 threads).
// ---------------------------------------------------------------------------
struct ArgMax {
  double v;
  int i;
};

__device__ __forceinline__ ArgMax better(ArgMax a, ArgMax b) {
  // larger value wins; equal values go to the lower index
  if (b.v > a.v || (b.v == a.v && b.i < a.i)) return b;
  return a;
}

__device__ ArgMax block_argmax(ArgMax x) {
  __shared__ double sv[16];
  __shared__ int si[16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    ArgMax y{__shfl_xor(x.v, o, 64), __shfl_xor(x.i, o, 64)};
    x = better(x, y);
  }
  if (lane == 0) { sv[wv] = x.v; si[wv] = x.i; }
  __syncthreads();
  ArgMax r{-1.0, INT_MAX};
  for (int k = 0; k < nw; ++k) r = better(r, ArgMax{sv[k], si[k]});
  __syncthreads();
  return r;
}

// Exclusive scan of a 0/1 flag over the block; returns the prefix and sets *total.
__device__ int block_excl_scan(int flag, int* total) {
  __shared__ int sw[16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  unsigned long long bal = __ballot(flag);
  int pre = __popcll(bal & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
  if (lane == 0) sw[wv] = __popcll(bal);
  __syncthreads();
  int off = 0, tot = 0;
  for (int k = 0; k < nw; ++k) {
    if (k < wv) off += sw[k];
    tot += sw[k];
  }
  __syncthreads();
  *total = tot;
  return off + pre;
}

// ---------------------------------------------------------------------------
// Assembly (eqn proxy-id, Section 3.3; SCI-expanded near field, Section 4.3).
// Pass 1 fills the kernel entries: workgroup (x, g) owns rows
// [64x, 64x + 64) of the stacked block [Y_c; A_cc] of group g (row
// descriptions staged in LDS), thread t columns t, t + 256, ..., so that
// consecutive threads write consecutive addresses of a row; it also writes
// the partial squared norm of every column over its rows of Y_c.  Pass 2
// (one wave per column) sums those partials in chunk order and adds the SCI
// entries of the column, lanes over the entries; the results do not depend
// on the launch shape.
// ---------------------------------------------------------------------------
constexpr int kAsmRows = 64;
constexpr int kAsmThreads = 256;

template <int D>
__global__ __launch_bounds__(kAsmThreads) void k_asm_fill(AsmArgs A) {
  const int g = blockIdx.y;
  const int64_t c0 = A.gstart[g];
  const int n = int(A.gstart[g + 1] - c0);
  const int64_t f0 = A.nf_start[g];
  const int nf = int(A.nf_start[g + 1] - f0);
  const int P = A.nproxy;
  const int m = A.sym ? nf + P : 2 * nf + 2 * P;
  const int r0 = blockIdx.x * kAsmRows;
  if (r0 >= m + n) return;
  const int r1 = min(r0 + kAsmRows, m + n), nr = r1 - r0;
  double* Y = A.Y + A.yoff[g];
  double* Acc = A.Acc + A.aoff[g];
  double* Scc = A.Scc + A.aoff[g];
  const int32_t* cols = A.cord + c0;
  const int32_t* nfi = A.nf_idx + f0;
  const int roff = A.sym ? nf : 2 * nf;  // first proxy row
  const bool f32 = A.fp32 != 0;
  // row descriptions: source point (or proxy point), kind, point index, factors
  __shared__ double sx[kAsmRows][D];
  __shared__ double sb[kAsmRows], swc[kAsmRows];
  __shared__ int skind[kAsmRows], sidx[kAsmRows];
  if (threadIdx.x < nr) {
    const int r = r0 + threadIdx.x;
    int kind, i = -1;
    double xi[D];
    if (r < nf) {
      kind = 0;
      i = nfi[r];
    } else if (!A.sym && r < 2 * nf) {
      kind = 1;
      i = nfi[r - nf];
    } else if (r < m) {
      const int p = A.sym ? r - roff : (r - roff) % P;
      kind = (A.sym || r - roff < P) ? 2 : 3;
      const double R = A.gpid ? A.pR[A.gpid[g]] : A.R;
#pragma unroll
      for (int k = 0; k < D; ++k) xi[k] = A.zc[int64_t(g) * D + k] + R * A.proxy_u[p * D + k];
    } else {
      kind = 4;
      i = cols[r - m];
    }
    if (i >= 0) {
#pragma unroll
      for (int k = 0; k < D; ++k) xi[k] = A.pts[int64_t(i) * D + k];
    }
#pragma unroll
    for (int k = 0; k < D; ++k) sx[threadIdx.x][k] = xi[k];
    sb[threadIdx.x] = i >= 0 ? A.b[i] : 0.0;
    swc[threadIdx.x] = i >= 0 ? A.w[i] * A.c[i] : 0.0;
    skind[threadIdx.x] = kind;
    sidx[threadIdx.x] = i;
  }
  __syncthreads();
  for (int col = threadIdx.x; col < n; col += kAsmThreads) {
    const int j = cols[col];
    double xj[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xj[k] = A.pts[int64_t(j) * D + k];
    const double aj = A.a[j], bj = A.b[j], cj = A.c[j], wj = A.w[j], sj = A.selfk[j];
    double k2 = 0.0;
    for (int rr = 0; rr < nr; ++rr) {
      const int r = r0 + rr;
      const int kind = skind[rr];
      double r2 = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const double t = sx[rr][k] - xj[k];
        r2 += t * t;
      }
      if (kind == 4) {
        const int i = sidx[rr];
        double v;
        if (i == j)
          v = aj + bj * sj * cj;
        else
          v = sb[rr] * green_mixed<D>(r2, f32) * wj * cj;
        const int rc = r - m;
        Acc[int64_t(rc) * n + col] = entry_prec(v, f32);
        Scc[int64_t(rc) * n + col] = 0.0;
      } else {
        const double gk = green_mixed<D>(r2, f32);
        double v;
        if (kind == 0)
          v = sb[rr] * gk * wj * cj;           // b_i G w_j c_j
        else if (kind == 1)
          v = bj * gk * swc[rr];               // b_j G w_i c_i
        else if (kind == 2)
          v = gk * wj * cj;                    // G(|x_p - x_j|) w_j c_j
        else
          v = bj * gk * wj;                    // b_j G(|x_p - x_j|) w_j
        v = entry_prec(v, f32);
        Y[int64_t(r) * n + col] = v;
        k2 += v * v;
      }
    }
    if (r0 < m) A.kpart[int64_t(blockIdx.x) * A.kstride + c0 + col] = k2;
  }
}

__global__ __launch_bounds__(256) void k_asm_finish(AsmArgs A) {
  const int g = blockIdx.y;
  const int64_t c0 = A.gstart[g];
  const int n = int(A.gstart[g + 1] - c0);
  const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (col >= n) return;  // uniform per wave
  const int64_t f0 = A.nf_start[g];
  const int nf = int(A.nf_start[g + 1] - f0);
  const int P = A.nproxy;
  const int m = A.sym ? nf + P : 2 * nf + 2 * P;
  double* Y = A.Y + A.yoff[g];
  double* Acc = A.Acc + A.aoff[g];
  double* Scc = A.Scc + A.aoff[g];
  const int32_t* nfi = A.nf_idx + f0;
  const int j = A.cord[c0 + col];
  // squared norm of the kernel part: chunk partials in chunk order
  const int nch = (m + kAsmRows - 1) / kAsmRows;
  double k2 = 0.0;
  for (int x = lane; x < nch; x += 64) k2 += A.kpart[int64_t(x) * A.kstride + c0 + col];
  k2 = wave_sum(k2);
  // SCI part: row j of the store holds (j, i) with values (S_ji, S_ij); the
  // entries of a row have distinct i, so the lanes write distinct rows.
  double s2 = 0.0;
  const int64_t e0 = A.srow[j], e1 = A.srow[j + 1];
  for (int64_t e = e0 + lane; e < e1; e += 64) {
    const int i = int(A.skey[e] & 0xffffffffu);
    const double2 sv = A.sval[e];
    if (A.grp_of[i] == g) {
      const int pr = A.pos_of[i];
      Acc[int64_t(pr) * n + col] += sv.y;
      Scc[int64_t(pr) * n + col] = sv.y;
    } else {
      // position of i in the (ascending) near-field list
      int lo = 0, hi = nf;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (nfi[mid] < i) lo = mid + 1; else hi = mid;
      }
      if (lo < nf && nfi[lo] == i) {
        Y[int64_t(lo) * n + col] += sv.y;
        s2 += sv.y * sv.y;
        if (!A.sym) {
          Y[int64_t(nf + lo) * n + col] += sv.x;
          s2 += sv.x * sv.x;
        }
      }
    }
  }
  s2 = wave_sum(s2);
  if (lane == 0) {
    A.colK2[c0 + col] = k2;
    A.colS2[c0 + col] = s2;
  }
}

void launch_assemble(const AsmArgs& A, hipStream_t s) {
  if (A.ngroups == 0) return;
  const dim3 g1(unsigned((A.max_rows + kAsmRows - 1) / kAsmRows), unsigned(A.ngroups));
  if (A.dim == 2)
    hipLaunchKernelGGL(k_asm_fill<2>, g1, dim3(kAsmThreads), 0, s, A);
  else
    hipLaunchKernelGGL(k_asm_fill<3>, g1, dim3(kAsmThreads), 0, s, A);
  const dim3 g2(unsigned((A.max_cols + 3) / 4), unsigned(A.ngroups));
  hipLaunchKernelGGL(k_asm_finish, g2, dim3(256), 0, s, A);
  HIF_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Interpolative decomposition (Lemma 2.2): column-pivoted Householder QR of
// the m x n block, stopped at the first pivot with |R_ii| <= tol |R_00|
// (Section 2.2), then T = R11^{-1} R12 by back substitution.  Thread t owns
// columns t + u B (u < U); pivoting only marks columns (no data movement).
// Trailing column norms are recomputed after every reflection.  On exit the
// block holds T in rows 0..k-1 of the redundant columns.
// ---------------------------------------------------------------------------
constexpr int kIdMaxRows = 4096;  // rows of the block the pivoted QR runs on (after row compression)
constexpr int kChunk = 8;

template <int U>
__global__ __launch_bounds__(1024) void k_id(IdArgs A) {
  const int q = blockIdx.x;
  double* M = A.base + A.moff[q];
  const int ld = A.ld[q], m = A.rows[q], n = A.cols[q];
  if (n <= A.skip_cols) return;
  const double tol = A.tol[q];
  int32_t* perm = A.perm + A.poff[q];
  const int tid = threadIdx.x, B = blockDim.x;
  __shared__ double s_alpha, s_v0, s_beta;
  __shared__ int s_p, s_k;
  __shared__ double sv[kIdMaxRows];  // Householder vector of the current step (rows i..m-1)

  double nrm[U];
  int state[U];  // -2 absent, -1 trailing, >= 0 pivot step
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int col = tid + u * B;
    state[u] = col < n ? -1 : -2;
    double s = 0.0;
    if (col < n) {
      int r = 0;
      for (; r + kChunk <= m; r += kChunk) {
        double y[kChunk];
#pragma unroll
        for (int c = 0; c < kChunk; ++c) y[c] = M[int64_t(r + c) * ld + col];
#pragma unroll
        for (int c = 0; c < kChunk; ++c) s += y[c] * y[c];
      }
      for (; r < m; ++r) {
        const double y = M[int64_t(r) * ld + col];
        s += y * y;
      }
    }
    nrm[u] = s;
  }
  const int kmax = m < n ? m : n;
  double r00 = 0.0;
  int k = kmax;
  for (int i = 0; i < kmax; ++i) {
    ArgMax loc{-1.0, INT_MAX};
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (state[u] == -1) loc = better(loc, ArgMax{nrm[u], tid + u * B});
    const ArgMax best = block_argmax(loc);
    const double nb = sqrt(best.v > 0.0 ? best.v : 0.0);
    if (i == 0) r00 = nb;
    if (!(best.v > 0.0) || !(nb > tol * r00)) {
      k = i;
      break;
    }
    const int p = best.i;
    // stage the pivot column below row i
    for (int r = i + 1 + tid; r < m; r += B) sv[r] = M[int64_t(r) * ld + p];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (tid + u * B == p) {
        state[u] = i;
        const double x0 = M[int64_t(i) * ld + p];
        const double alpha = -copysign(nb, x0);
        const double v0 = x0 - alpha;
        const double vtv = best.v - x0 * x0 + v0 * v0;
        s_alpha = alpha;
        s_v0 = v0;
        s_beta = vtv > 0.0 ? 2.0 / vtv : 0.0;
        s_p = p;
        perm[i] = p;
        if (A.alpha) A.alpha[q * A.astride + i] = alpha;
      }
    __syncthreads();
    const double v0 = s_v0, beta = s_beta;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (state[u] != -1) continue;
      const int col = tid + u * B;
      double* Mc = M + col;
      double w = v0 * Mc[int64_t(i) * ld];
      {
        int r = i + 1;
        for (; r + kChunk <= m; r += kChunk) {
          double y[kChunk];
#pragma unroll
          for (int c = 0; c < kChunk; ++c) y[c] = Mc[int64_t(r + c) * ld];
#pragma unroll
          for (int c = 0; c < kChunk; ++c) w += sv[r + c] * y[c];
        }
        for (; r < m; ++r) w += sv[r] * Mc[int64_t(r) * ld];
      }
      w *= beta;
      Mc[int64_t(i) * ld] -= w * v0;
      double s = 0.0;
      {
        int r = i + 1;
        for (; r + kChunk <= m; r += kChunk) {
          double y[kChunk];
#pragma unroll
          for (int c = 0; c < kChunk; ++c) y[c] = Mc[int64_t(r + c) * ld];
#pragma unroll
          for (int c = 0; c < kChunk; ++c) {
            y[c] -= w * sv[r + c];
            s += y[c] * y[c];
          }
#pragma unroll
          for (int c = 0; c < kChunk; ++c) Mc[int64_t(r + c) * ld] = y[c];
        }
        for (; r < m; ++r) {
          const double y = Mc[int64_t(r) * ld] - w * sv[r];
          Mc[int64_t(r) * ld] = y;
          s += y * y;
        }
      }
      nrm[u] = s;
    }
    __syncthreads();
    if (tid == (p % B)) M[int64_t(i) * ld + p] = s_alpha;
  }
  if (tid == 0) s_k = k;
  __syncthreads();
  k = s_k;
  // T = R11^{-1} R12, R11[a][b] = M[a][perm[b]]; written in place over R12
  // (or left to the blocked triangular solve).
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (state[u] != -1 || A.alpha) continue;
    const int col = tid + u * B;
    for (int a = k - 1; a >= 0; --a) {
      double t = M[int64_t(a) * ld + col];
      for (int b2 = a + 1; b2 < k; ++b2) t -= M[int64_t(a) * ld + perm[b2]] * M[int64_t(b2) * ld + col];
      M[int64_t(a) * ld + col] = t / M[int64_t(a) * ld + perm[a]];
    }
  }
  // Redundant columns in ascending order after the skeleton.
  int base = 0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int col = tid + u * B;
    const int flag = (state[u] == -1) ? 1 : 0;
    int tot = 0;
    const int pre = block_excl_scan(flag, &tot);
    if (flag) perm[k + base + pre] = col;
    base += tot;
    if (u * B + B >= n) break;
  }
  if (tid == 0) A.rank[q] = k;
  if (A.Tout && !A.alpha) {
    __syncthreads();
    const int r = n - k;
    double* T = A.Tout + A.toff[q];
    for (int e = tid; e < k * r; e += B) {
      const int a = e / r, b2 = e % r;
      T[e] = M[int64_t(a) * ld + perm[k + b2]];
    }
  }
}

// T = R11^{-1} R12 for the blocked pivoted QR below: R11[a][b] = M[a][perm[b]]
// above the diagonal, R11[a][a] = alpha[a], R12 in rows 0..k-1 of the
// redundant columns.  State of problem q lives at q * stride.
struct IdmState {
  double* alpha;  // [nprob * stride] R_ii
  int64_t stride;
};

// T = R11^{-1} R12 in place over R12, by blocks of 64 rows from the bottom
// (one launch per row block a0..a0+63): workgroup (tile, q) takes 64
// redundant columns, subtracts R11[a0:a1, a1:k] T[a1:k, :] on the matrix
// cores (pivot columns gathered through perm), then solves with the 64 x 64
// diagonal block in LDS.  R11[a][b] = M[a][perm[b]] above the diagonal,
// R11[a][a] = alpha[a].
constexpr int kTb64 = 64;
__global__ __launch_bounds__(256) void k_idm_T_block(IdArgs A, IdmState S, int a0) {
  const int q = blockIdx.y;
  const int n = A.cols[q], k = A.rank[q];
  if (a0 >= k) return;
  const int nr = n - k;
  const int c0 = blockIdx.x * kTb64;
  if (c0 >= nr) return;
  const int a1 = min(a0 + kTb64, k), nb = a1 - a0, nc = min(kTb64, nr - c0);
  double* M = A.base + A.moff[q];
  const int ld = A.ld[q];
  const int32_t* perm = A.perm + A.poff[q];
  const double* al = S.alpha + q * S.stride;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = wv >> 1, wc = wv & 1;
  __shared__ int scol[kTb64];
  __shared__ double sA[kTb64][17], sB[16][kTb64 + 1];
  __shared__ double sX[kTb64][kTb64 + 1];  // right-hand sides, then the solution
  __shared__ double sU[kTb64][kTb64 + 1];  // diagonal block
  if (tid < kTb64) scol[tid] = tid < nc ? perm[k + c0 + tid] : perm[k + c0];
  __syncthreads();
  // 1. acc = R11[a0:a1, a1:k] T[a1:k, cols]
  double4_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = double4_t{0.0, 0.0, 0.0, 0.0};
  for (int b0 = a1; b0 < k; b0 += 16) {
    for (int e = tid; e < kTb64 * 16; e += 256) {
      const int i = e >> 4, kk = e & 15;
      const int b = b0 + kk;
      sA[i][kk] = (i < nb && b < k) ? M[int64_t(a0 + i) * ld + perm[b]] : 0.0;
      const int kk2 = e >> 6, j = e & 63;
      const int b2 = b0 + kk2;
      sB[kk2][j] = (b2 < k && j < nc) ? M[int64_t(b2) * ld + scol[j]] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      double af[2], bf[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) af[x] = sA[wr * 32 + x * 16 + li][kk + lk];
#pragma unroll
      for (int y = 0; y < 2; ++y) bf[y] = sB[kk + lk][wc * 32 + y * 16 + li];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = mfma_f64(af[x], bf[y], acc[x][y]);
    }
    __syncthreads();
  }
  // 2. right-hand sides R12[a0:a1, cols] - acc and the diagonal block
  for (int e = tid; e < kTb64 * kTb64; e += 256) {
    const int i = e >> 6, j = e & 63;
    sX[i][j] = (i < nb && j < nc) ? M[int64_t(a0 + i) * ld + scol[j]] : 0.0;
    sU[i][j] = (i < nb && j < nb) ? (i == j ? al[a0 + i] : (j > i ? M[int64_t(a0 + i) * ld + perm[a0 + j]] : 0.0))
                                  : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) sX[wr * 32 + x * 16 + 4 * v + lk][wc * 32 + y * 16 + li] -= acc[x][y][v];
  __syncthreads();
  // 3. back substitution with the diagonal block, one thread per column
  if (tid < nc) {
    const int j = tid;
    for (int i = nb - 1; i >= 0; --i) {
      double t = sX[i][j];
      for (int b = i + 1; b < nb; ++b) t -= sU[i][b] * sX[b][j];
      sX[i][j] = t / sU[i][i];
    }
    for (int i = 0; i < nb; ++i) M[int64_t(a0 + i) * ld + scol[j]] = sX[i][j];
  }
}

// Compact copy of T (k x r row-major) for callers that ask for it.
__global__ __launch_bounds__(256) void k_idm_Tcopy(IdArgs A) {
  const int q = blockIdx.y;
  const int n = A.cols[q], k = A.rank[q];
  const int nr = n - k;
  const int b2 = blockIdx.x * 256 + threadIdx.x;
  if (b2 >= nr) return;
  const double* M = A.base + A.moff[q];
  const int ld = A.ld[q];
  const int col = A.perm[A.poff[q] + k + b2];
  double* T = A.Tout + A.toff[q];
  for (int a = 0; a < k; ++a) T[int64_t(a) * nr + b2] = M[int64_t(a) * ld + col];
}

// ---------------------------------------------------------------------------
// Blocked column-pivoted QR on the uncompressed block (no row compression
// first): the pivot sequence and rank rule of k_id, with the updates of up to
// kBq reflectors delayed as in LAPACK's xLAQPS (Quintana-Orti, Sun and
// Bischof's BLAS-3 QRP).  With Y0 the block at the start of a block of steps,
// after j reflectors Y = Y0 - V F^T, V = [v_0 .. v_{j-1}] (zero above each
// step row) and F(:, j) = beta_j (Y0^T v_j - F V^T v_j).  Per step:
//  - k_bq_piv (one workgroup per problem) picks the column of largest
//    downdated norm, brings it up to date from V and F, applies the rank rule
//    to its exact norm, forms the reflector and aux = -beta V^T v;
//  - k_bq_cols reads every trailing column once (rows at and below the step,
//    still at their block-start values), forms its entry of F, finalizes its
//    entry of R in the step row and downdates its norm.
// After the block, k_bq_update applies Y -= V F^T to the rows below the block
// on the matrix cores and recomputes the norms exactly.  A downdate that
// leaves a squared norm at or below sqrt(eps) times its last exact value
// ends the problem's block early (the xLAQPS safeguard): the problem idles
// until the update.  Rows above the step are final R rows; T = R11^{-1} R12
// comes from k_idm_T_block.
// ---------------------------------------------------------------------------
constexpr int kBq = 32;        // reflectors per block
static_assert(kBq == kRs, "the pivot kernel reduces its kBq products with wave_rs32");
constexpr int kBqT = 512;      // threads of the pivot kernel
constexpr int kBcGroups = 16;  // row groups of the column kernel (32 columns each)
constexpr int kBcV = 2048;     // rows of v staged in LDS by the column kernel
constexpr double kTol3z = 1.0536712127723509e-08;  // sqrt(2^-53)

struct BqCtl {  // written by k_bq_piv only, except stale (k_bq_cols sets, k_bq_update clears)
  int k;        // steps done
  int i0;       // first step of the open block
  int go;       // 1: k_bq_cols runs step cur
  int cur;
  int p;        // pivot column of step cur
  int done;
  int stale;
  int pad;
  double beta;
  double r00;
};

struct BqState {
  double* nrm;    // [nprob * stride] downdated squared norms (rows >= k)
  double* nrm0;   // [nprob * stride] squared norms at the last exact computation
  int32_t* st;    // [nprob * stride] -2 absent, -1 trailing, >= 0 pivot step
  double* F;      // [nprob * stride][kBq]
  double* V;      // [nprob][kBq][vld] reflectors of the open block, column-major
  double* aux;    // [nprob][kBq]
  double* alpha;  // [nprob * stride] R_ii
  BqCtl* ctl;     // [nprob]
  int64_t stride;
  int64_t vld;
};

__global__ __launch_bounds__(256) void k_bq_init(IdArgs A, BqState S) {
  const int q = blockIdx.y;
  const int m = A.rows[q], n = A.cols[q];
  const int c0 = blockIdx.x * 64;
  if (c0 >= n) return;
  const double* M = A.base + A.moff[q];
  const int ld = A.ld[q];
  const int lc = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int col = c0 + lc;
  __shared__ double sp[4][64];
  double s = 0.0;
  if (col < n)
    for (int r = rg; r < m; r += 4) {
      const double y = M[int64_t(r) * ld + col];
      s += y * y;
    }
  sp[rg][lc] = s;
  __syncthreads();
  if (rg == 0 && col < n) {
    const int64_t o = q * S.stride + col;
    const double t = sp[0][lc] + sp[1][lc] + sp[2][lc] + sp[3][lc];
    S.nrm[o] = t;
    S.nrm0[o] = t;
    S.st[o] = -1;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    BqCtl c{};
    S.ctl[q] = c;
    A.rank[q] = min(m, n);
  }
}

// Slot j of the block: step k of problem blockIdx.x.
__global__ __launch_bounds__(kBqT) void k_bq_piv(IdArgs A, BqState S, int j) {
  const int q = blockIdx.x;
  BqCtl* C = S.ctl + q;
  const int m = A.rows[q], n = A.cols[q];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int k = C->k;
  const int i0 = j == 0 ? k : C->i0;
  if (C->done || C->stale || k >= min(m, n)) {
    if (tid == 0) {
      C->go = 0;
      C->i0 = i0;
      if (!C->done && k >= min(m, n)) {
        C->done = 1;
        A.rank[q] = k;
      }
    }
    return;
  }
  const int i = k, jb = i - i0;  // reflectors already in the block
  const double* nrm = S.nrm + q * S.stride;
  int32_t* st = S.st + q * S.stride;
  ArgMax loc{-1.0, INT_MAX};
  for (int c = tid; c < n; c += kBqT)
    if (st[c] == -1) loc = better(loc, ArgMax{nrm[c], c});
  const ArgMax best = block_argmax(loc);
  __shared__ double sf[kBq], sred[16][kBq], sx0[1], sss[16];
  const int p = best.i;
  if (p != INT_MAX && tid < jb) sf[tid] = S.F[(q * S.stride + p) * kBq + tid];
  __syncthreads();
  double* M = A.base + A.moff[q];
  const int ld = A.ld[q];
  double* V = S.V + q * kBq * S.vld;
  const int64_t vld = S.vld;
  // One pass over the rows: the pivot column brought up to date (kept as
  // column jb of V), its squared norm and P = V(i:, 0:jb)^T col.  With
  // v = col - alpha e_i, aux = -beta V(i:, 0:jb)^T v = -beta (P - alpha V(i, 0:jb)).
  double ss = 0.0;
  double part[kBq];
#pragma unroll
  for (int jj = 0; jj < kBq; ++jj) part[jj] = 0.0;
  // The pivot column is a strided gather (one row per cache line): the
  // gathers of kPivU rows per thread are issued before any of them is used.
  constexpr int kPivU = 8;
  if (p != INT_MAX)
    for (int r0 = i + tid; r0 < m; r0 += kBqT * kPivU) {
      double xs[kPivU];
#pragma unroll
      for (int u = 0; u < kPivU; ++u) {
        const int r = r0 + u * kBqT;
        xs[u] = r < m ? M[int64_t(r) * ld + p] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kPivU; ++u) {
        const int r = r0 + u * kBqT;
        if (r >= m) break;
        double x = xs[u];
        double vv[kBq];  // all loads first
#pragma unroll
        for (int jj = 0; jj < kBq; ++jj) vv[jj] = jj < jb ? V[jj * vld + r] : 0.0;
#pragma unroll
        for (int jj = 0; jj < kBq; ++jj)
          if (jj < jb) x -= vv[jj] * sf[jj];
        V[jb * vld + r] = x;
        ss += x * x;
        if (r == i) sx0[0] = x;
#pragma unroll
        for (int jj = 0; jj < kBq; ++jj) part[jj] += vv[jj] * x;
      }
    }
  ss = wave_sum(ss);
  if (lane == 0) sss[wv] = ss;
  {
    // all jb products in one reduce-scatter (part[jj] is zero for jj >= jb):
    // lanes 2c and 2c + 1 end with the wave's sum for column c
    const double t = wave_rs32(part);
    if ((lane & 1) == 0 && (lane >> 1) < jb) sred[wv][lane >> 1] = t;
  }
  __syncthreads();
  ss = 0.0;
#pragma unroll
  for (int w = 0; w < kBqT / 64; ++w) ss += sss[w];
  const double nb = sqrt(ss);
  const double r00 = i == 0 ? nb : C->r00;
  if (p == INT_MAX || !(ss > 0.0) || !(nb > A.tol[q] * r00)) {
    if (tid == 0) {
      C->go = 0;
      C->i0 = i0;
      C->done = 1;
      A.rank[q] = i;
    }
    return;
  }
  const double x0 = sx0[0];
  const double alpha = -copysign(nb, x0);
  const double v0 = x0 - alpha;
  const double vtv = ss - x0 * x0 + v0 * v0;
  const double beta = vtv > 0.0 ? 2.0 / vtv : 0.0;
  if (tid == 0) V[jb * vld + i] = v0;
  if (tid < jb) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kBqT / 64; ++w) t += sred[w][tid];
    S.aux[q * kBq + tid] = -beta * (t - alpha * V[tid * vld + i]);
  }
  if (tid == 0) {
    st[p] = i;
    S.alpha[q * S.stride + i] = alpha;
    A.perm[A.poff[q] + i] = p;
    C->i0 = i0;
    C->k = i + 1;
    C->cur = i;
    C->p = p;
    C->go = 1;
    C->beta = beta;
    if (i == 0) C->r00 = nb;
  }
}

// Workgroup (b, q): columns 32b..32b+31 of problem q, thread (c, g) =
// (tid % 32, tid / 32) sums rows i + g + 16u of column c.
__global__ __launch_bounds__(32 * kBcGroups) void k_bq_cols(IdArgs A, BqState S) {
  const int q = blockIdx.y;
  const BqCtl ctl = S.ctl[q];  // one read of the whole control block
  if (!ctl.go) return;
  const int n = A.cols[q];
  const int c0 = blockIdx.x * 32;
  if (c0 >= n) return;
  const int m = A.rows[q];
  const int i = ctl.cur, jb = i - ctl.i0;
  const double beta = ctl.beta;
  const int tid = threadIdx.x, c = tid & 31, g = tid >> 5;
  const double* V = S.V + q * kBq * S.vld;
  const int64_t vld = S.vld;
  const int mr = m - i;
  const double* vcol = V + jb * vld + i;  // v(i + rr)
  __shared__ double sv[kBcV];
  __shared__ double sp[kBcGroups][32];
  __shared__ double saux[kBq], svi[kBq + 1];
  __shared__ double sF[32][kBq + 1];  // F rows of the 32 columns (contiguous in F)
  const bool lds = mr <= kBcV;
  if (lds)
    for (int rr = tid; rr < mr; rr += 32 * kBcGroups) sv[rr] = vcol[rr];
  if (tid < jb) saux[tid] = S.aux[q * kBq + tid];
  if (tid <= jb) svi[tid] = V[tid * vld + i];
  {
    const int n32 = min(32, n - c0);
    const double* F0 = S.F + (q * S.stride + c0) * kBq;
    for (int e = tid; e < 32 * kBq; e += 32 * kBcGroups) {
      const int cc = e / kBq, jj = e % kBq;
      sF[cc][jj] = (cc < n32 && jj < jb) ? F0[e] : 0.0;
    }
  }
  __syncthreads();
  const double* vs = lds ? sv : vcol;
  const int col = c0 + c;
  const int64_t o = q * S.stride + col;
  const bool upd = col < n && S.st[o] == -1;
  double* M = A.base + A.moff[q];
  const int ld = A.ld[q];
  double d = 0.0;
  // the finishing thread's own loads, issued before the pass and the stores
  double r0 = 0.0, old = 0.0, old0 = 0.0;
  if (g == 0 && upd) {
    r0 = M[int64_t(i) * ld + col];
    old = S.nrm[o];
    old0 = S.nrm0[o];
  }
  if (upd) {
    const double* y = M + int64_t(i) * ld + col;
    int rr = g;
    for (; rr + 7 * kBcGroups < mr; rr += 8 * kBcGroups) {
      double yy[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) yy[u] = y[int64_t(rr + u * kBcGroups) * ld];
#pragma unroll
      for (int u = 0; u < 8; ++u) d += yy[u] * vs[rr + u * kBcGroups];
    }
    for (; rr < mr; rr += kBcGroups) d += y[int64_t(rr) * ld] * vs[rr];
  }
  sp[g][c] = d;
  __syncthreads();
  if (g == 0 && upd) {
    double t = 0.0;
#pragma unroll
    for (int g2 = 0; g2 < kBcGroups; ++g2) t += sp[g2][c];
    double* yi = M + int64_t(i) * ld + col;
    double r = r0;
    double f = beta * t;
    for (int jj = 0; jj < jb; ++jj) {
      const double fj = sF[c][jj];
      f += fj * saux[jj];
      r -= svi[jj] * fj;
    }
    S.F[o * kBq + jb] = f;
    r -= svi[jb] * f;
    *yi = r;
    if (old > 0.0) {
      const double nw = old - r * r;
      if (nw <= kTol3z * old0) S.ctl[q].stale = 1;
      S.nrm[o] = nw > 0.0 ? nw : 0.0;
    }
  }
}

// Y(k:, c) -= V(k:, 0:ns) F(c, 0:ns)^T for the trailing columns, then exact
// norms.  Workgroup (b, q): columns 64b..64b+63, wave w 16 of them; rows in
// tiles of 16 on the matrix cores.
__global__ __launch_bounds__(256) void k_bq_update(IdArgs A, BqState S) {
  const int q = blockIdx.y;
  BqCtl* C = S.ctl + q;
  const int n = A.cols[q], m = A.rows[q];
  const int c0 = blockIdx.x * 64;
  if (c0 >= n) return;
  const int k = C->k, ns = k - C->i0;
  if (C->done || ns <= 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  __shared__ double sF[64][kBq + 1];
  __shared__ int sup[64];
  for (int e = tid; e < 64 * kBq; e += 256) {
    const int cc = e / kBq, jj = e % kBq;
    const int col = c0 + cc;
    const bool up = col < n && S.st[q * S.stride + col] == -1;
    sF[cc][jj] = (up && jj < ns) ? S.F[(q * S.stride + col) * kBq + jj] : 0.0;
    if (jj == 0) sup[cc] = up ? 1 : 0;
  }
  __syncthreads();
  if (blockIdx.x == 0 && tid == 0) C->stale = 0;
  const int cw = 16 * wv + li;  // this lane's column (as B operand / output column)
  const int col = c0 + cw;
  const bool up = sup[cw] != 0;
  double* M = A.base + A.moff[q];
  const int ld = A.ld[q];
  const double* V = S.V + q * kBq * S.vld;
  const int64_t vld = S.vld;
  double bf[kBq / 4];
#pragma unroll
  for (int s = 0; s < kBq / 4; ++s) bf[s] = sF[cw][4 * s + lk];
  double nsum = 0.0;
  for (int r0 = k; r0 < m; r0 += 16) {
    double a[kBq / 4], y[4];
#pragma unroll
    for (int s = 0; s < kBq / 4; ++s) {
      const int jj = 4 * s + lk, r = r0 + li;
      a[s] = (jj < ns && r < m) ? V[jj * vld + r] : 0.0;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = r0 + 4 * v + lk;
      y[v] = (up && r < m) ? M[int64_t(r) * ld + col] : 0.0;
    }
    double4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < kBq / 4; ++s) acc = mfma_f64(a[s], bf[s], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = r0 + 4 * v + lk;
      if (up && r < m) {
        const double t = y[v] - acc[v];
        M[int64_t(r) * ld + col] = t;
        nsum += t * t;
      }
    }
  }
  nsum += __shfl_xor(nsum, 16, 64);
  nsum += __shfl_xor(nsum, 32, 64);
  if (lk == 0 && up) {
    const int64_t o = q * S.stride + col;
    S.nrm[o] = nsum;
    S.nrm0[o] = nsum;
  }
}

// Redundant columns (state -1) in ascending order after the k pivots.
__global__ __launch_bounds__(1024) void k_bq_perm(IdArgs A, BqState S) {
  const int q = blockIdx.x;
  const int n = A.cols[q];
  const int k = A.rank[q];
  const int32_t* st = S.st + q * S.stride;
  int32_t* perm = A.perm + A.poff[q];
  int base = 0;
  for (int c0 = 0; c0 < n; c0 += blockDim.x) {
    const int c = c0 + threadIdx.x;
    const int flag = (c < n && st[c] == -1) ? 1 : 0;
    int tot = 0;
    const int pre = block_excl_scan(flag, &tot);
    if (flag) perm[k + base + pre] = c;
    base += tot;
  }
}

// Copy rows [0, rows) of every problem between two layouts (rows = the
// problem's row count, or its rank when `upto_rank`); workgroup (x, q) copies
// rows 8x..8x+7.
__global__ __launch_bounds__(256) void k_bq_copy(IdArgs src, IdArgs dst, int upto_rank) {
  const int q = blockIdx.y;
  const int n = src.cols[q];
  const int rows = upto_rank ? dst.rank[q] : src.rows[q];
  const double* S0 = src.base + src.moff[q];
  double* D0 = dst.base + dst.moff[q];
  const int lds = src.ld[q], ldd = dst.ld[q];
  for (int r = blockIdx.x * 8; r < min(rows, int(blockIdx.x) * 8 + 8); ++r)
    for (int c = threadIdx.x; c < n; c += 256) D0[int64_t(r) * ldd + c] = S0[int64_t(r) * lds + c];
}

void launch_id_blocked(const IdArgs& A0, int max_rows, int max_cols, hipStream_t s) {
  if (A0.nprob == 0) return;
  // The pivoted QR streams the trailing columns of every problem at every
  // step, 32 columns (256 bytes of a row) per workgroup: it runs on a copy
  // whose rows start on 128-byte lines (row stride padded to 16 doubles), so
  // that each row segment spans two lines instead of three.  Only rows
  // 0..k-1 (R11 and T) are copied back.
  std::vector<int32_t> hr(A0.nprob), hcl(A0.nprob);
  HIF_HIP(hipMemcpyAsync(hr.data(), A0.rows, sizeof(int32_t) * A0.nprob, hipMemcpyDeviceToHost, s));
  HIF_HIP(hipMemcpyAsync(hcl.data(), A0.cols, sizeof(int32_t) * A0.nprob, hipMemcpyDeviceToHost, s));
  HIF_HIP(hipStreamSynchronize(s));
  std::vector<int64_t> hzo(A0.nprob);
  std::vector<int32_t> hzl(A0.nprob);
  int64_t ztot = 0;
  for (int q = 0; q < A0.nprob; ++q) {
    hzl[q] = (hcl[q] + 15) & ~15;
    hzo[q] = ztot;
    ztot += int64_t(hr[q]) * hzl[q];
  }
  DBuf<double> Z;
  DBuf<int64_t> zoff;
  DBuf<int32_t> zld;
  Z.alloc(ztot + 16, nullptr);
  zoff.alloc(A0.nprob, nullptr);
  zld.alloc(A0.nprob, nullptr);
  HIF_HIP(hipMemcpyAsync(zoff.p, hzo.data(), sizeof(int64_t) * A0.nprob, hipMemcpyHostToDevice, s));
  HIF_HIP(hipMemcpyAsync(zld.p, hzl.data(), sizeof(int32_t) * A0.nprob, hipMemcpyHostToDevice, s));
  IdArgs A = A0;
  A.base = Z.p;
  A.moff = zoff.p;
  A.ld = zld.p;
  hipLaunchKernelGGL(k_bq_copy, dim3(unsigned((max_rows + 7) / 8), unsigned(A0.nprob)), dim3(256), 0, s, A0, A, 0);
  const int64_t stride = max_cols, vld = (max_rows + 15) & ~15;
  const int64_t total = stride * A.nprob;
  DBuf<double> nrm, nrm0, F, V, aux, alpha;
  DBuf<int32_t> st;
  DBuf<BqCtl> ctl;
  nrm.alloc(total, nullptr);
  nrm0.alloc(total, nullptr);
  st.alloc(total, nullptr);
  F.alloc(total * kBq, nullptr);
  V.alloc(int64_t(A.nprob) * kBq * vld, nullptr);
  aux.alloc(int64_t(A.nprob) * kBq, nullptr);
  alpha.alloc(total, nullptr);
  ctl.alloc(A.nprob, nullptr);
  BqState S{nrm.p, nrm0.p, st.p, F.p, V.p, aux.p, alpha.p, ctl.p, stride, vld};
  const unsigned np = unsigned(A.nprob);
  hipLaunchKernelGGL(k_bq_init, dim3(unsigned((max_cols + 63) / 64), np), dim3(256), 0, s, A, S);
  const dim3 gcols(unsigned((max_cols + 31) / 32), np), gupd(unsigned((max_cols + 63) / 64), np);
  std::vector<BqCtl> hc(A.nprob);
  // every block takes at least one step of each unfinished problem
  bool all = false;
  for (int blk = 0; blk <= max_cols && !all; ++blk) {
    for (int j = 0; j < kBq; ++j) {
      hipLaunchKernelGGL(k_bq_piv, dim3(np), dim3(kBqT), 0, s, A, S, j);
      hipLaunchKernelGGL(k_bq_cols, gcols, dim3(32 * kBcGroups), 0, s, A, S);
    }
    hipLaunchKernelGGL(k_bq_update, gupd, dim3(256), 0, s, A, S);
    HIF_HIP(hipMemcpyAsync(hc.data(), ctl.p, sizeof(BqCtl) * A.nprob, hipMemcpyDeviceToHost, s));
    HIF_HIP(hipStreamSynchronize(s));
    all = true;
    for (const BqCtl& c : hc) all = all && c.done;
  }
  if (!all) throw Error{HIF_EDEVICE, "blocked pivoted QR did not finish"};
  hipLaunchKernelGGL(k_bq_perm, dim3(np), dim3(1024), 0, s, A, S);
  std::vector<int32_t> hk(A.nprob);
  HIF_HIP(hipMemcpyAsync(hk.data(), A.rank, sizeof(int32_t) * A.nprob, hipMemcpyDeviceToHost, s));
  HIF_HIP(hipStreamSynchronize(s));
  int kmax = 0;
  for (int v : hk) kmax = std::max(kmax, v);
  IdmState T{alpha.p, stride};
  const dim3 tg(unsigned((max_cols + kTb64 - 1) / kTb64), np);
  for (int a0 = ((kmax - 1) / kTb64) * kTb64; kmax > 0 && a0 >= 0; a0 -= kTb64)
    hipLaunchKernelGGL(k_idm_T_block, tg, dim3(256), 0, s, A, T, a0);
  if (A.Tout)
    hipLaunchKernelGGL(k_idm_Tcopy, dim3(unsigned((max_cols + 255) / 256), np), dim3(256), 0, s, A);
  hipLaunchKernelGGL(k_bq_copy, dim3(unsigned((max_rows + 7) / 8), np), dim3(256), 0, s, A, A0, 1);
  HIF_HIP(hipGetLastError());
  HIF_HIP(hipStreamSynchronize(s));  // the state buffers are released on return
}

bool id_blocked_fits(int nprob, int max_rows, int max_cols) {
  // many small problems go to the one-workgroup ID after row compression
  (void)max_rows;
  return nprob <= 512 && max_cols >= 128;
}

// ---------------------------------------------------------------------------
// Register-resident pivoted QR for many problems of at most 64 CB columns and
// NW RB rows (after row compression): one workgroup of NW waves per problem,
// thread (c, g) = (tid % 64, tid / 64) holds rows g + NW u (u < RB) of columns
// c + 64j (j < CB) for the whole factorization; norms, the pivot column and
// the column sums go through LDS.  Same pivots, norms (recomputed every step)
// and rank rule as k_id; writes rows 0..k-1 (R) back, R_ii to alpha and the
// permutation, and leaves T to k_idm_T_block.
// ---------------------------------------------------------------------------
template <int CB, int RB, int NW>
__global__ __launch_bounds__(64 * NW) void k_id_reg(IdArgs A, IdmState S) {
  constexpr int NC = 64 * CB, NR = NW * RB, NT = 64 * NW;
  const int q = blockIdx.x;
  double* M = A.base + A.moff[q];
  const int ld = A.ld[q], m = A.rows[q], n = A.cols[q];
  if (n > NC || min(m, n) > NR) return;  // left to k_id (id_in_registers says the same)
  const double tol = A.tol[q];
  int32_t* perm = A.perm + A.poff[q];
  const int tid = threadIdx.x, c = tid & 63, g = tid >> 6;
  __shared__ double sred[NW][NC];
  __shared__ double snrm[NC], sw[NC], sv[NR];
  __shared__ int sst[NC];
  __shared__ int s_p;
  double y[CB][RB];
#pragma unroll
  for (int j = 0; j < CB; ++j)
#pragma unroll
    for (int u = 0; u < RB; ++u) {
      const int r = g + NW * u, col = c + 64 * j;
      y[j][u] = (r < m && col < n) ? M[int64_t(r) * ld + col] : 0.0;
    }
  // initial squared norms
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    double t = 0.0;
#pragma unroll
    for (int u = 0; u < RB; ++u) t += y[j][u] * y[j][u];
    sred[g][c + 64 * j] = t;
  }
  __syncthreads();
  for (int col = tid; col < NC; col += NT) {
    double t = 0.0;
#pragma unroll
    for (int g2 = 0; g2 < NW; ++g2) t += sred[g2][col];
    snrm[col] = t;
    sst[col] = col < n ? -1 : -2;
  }
  __syncthreads();
  const int kmax = m < n ? m : n;
  double r00 = 0.0;
  int k = kmax;
  for (int i = 0; i < kmax; ++i) {
    // pivot: largest trailing norm, ties to the lowest column (wave 0)
    if (g == 0) {
      ArgMax loc{-1.0, INT_MAX};
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        const int col = c + 64 * j;
        if (sst[col] == -1) loc = better(loc, ArgMax{snrm[col], col});
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        ArgMax y2{__shfl_xor(loc.v, o, 64), __shfl_xor(loc.i, o, 64)};
        loc = better(loc, y2);
      }
      if (c == 0) s_p = loc.i;
    }
    __syncthreads();
    const int p = s_p;
    const double nv2 = p == INT_MAX ? 0.0 : snrm[p];
    const double nb = sqrt(nv2 > 0.0 ? nv2 : 0.0);
    if (i == 0) r00 = nb;
    if (p == INT_MAX || !(nv2 > 0.0) || !(nb > tol * r00)) {
      k = i;
      break;
    }
    // the pivot column below the diagonal to LDS
    if (c == (p & 63)) {
#pragma unroll
      for (int j = 0; j < CB; ++j)
        if (j == (p >> 6))
#pragma unroll
          for (int u = 0; u < RB; ++u) sv[g + NW * u] = y[j][u];
    }
    __syncthreads();
    const double x0 = sv[i];
    const double alpha = -copysign(nb, x0);
    const double v0 = x0 - alpha;
    const double vtv = nv2 - x0 * x0 + v0 * v0;
    const double beta = vtv > 0.0 ? 2.0 / vtv : 0.0;
    // column sums v^T y over rows >= i
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      double d = 0.0;
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int r = g + NW * u;
        if (r >= i) d += (r == i ? v0 : sv[r]) * y[j][u];
      }
      sred[g][c + 64 * j] = d;
    }
    __syncthreads();
    for (int col = tid; col < NC; col += NT) {
      double t = 0.0;
#pragma unroll
      for (int g2 = 0; g2 < NW; ++g2) t += sred[g2][col];
      sw[col] = beta * t;
    }
    __syncthreads();
    // update of the trailing columns and their new norms (rows > i)
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int col = c + 64 * j;
      const bool upd = sst[col] == -1 && col != p;
      const double w = sw[col];
      double s2 = 0.0;
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int r = g + NW * u;
        if (upd && r >= i) {
          y[j][u] -= w * (r == i ? v0 : sv[r]);
          if (r > i) s2 += y[j][u] * y[j][u];
        }
      }
      sred[g][col] = s2;
    }
    __syncthreads();
    for (int col = tid; col < NC; col += NT) {
      if (sst[col] == -1 && col != p) {
        double t = 0.0;
#pragma unroll
        for (int g2 = 0; g2 < NW; ++g2) t += sred[g2][col];
        snrm[col] = t;
      }
    }
    if (tid == 0) {
      sst[p] = i;
      perm[i] = p;
      S.alpha[q * S.stride + i] = alpha;
    }
    __syncthreads();
  }
  // rows 0..k-1 back (R above the diagonal and R12), then the redundant
  // columns in ascending order after the pivots
#pragma unroll
  for (int j = 0; j < CB; ++j)
#pragma unroll
    for (int u = 0; u < RB; ++u) {
      const int r = g + NW * u, col = c + 64 * j;
      if (r < k && col < n) M[int64_t(r) * ld + col] = y[j][u];
    }
  if (tid == 0) A.rank[q] = k;
  int base = 0;
  for (int c0 = 0; c0 < NC; c0 += NT) {
    const int col = c0 + tid;
    const int flag = (col < NC && sst[col] == -1) ? 1 : 0;
    int tot = 0;
    const int pre = block_excl_scan(flag, &tot);
    if (flag) perm[k + base + pre] = col;
    base += tot;
  }
}

static void launch_id_small(const IdArgs& A, int max_cols, hipStream_t s);

// Problems in registers (all of them up to 128 columns; up to 192 columns in
// batches of up to 256), the others by k_id without its triangular solve; T
// for all by row blocks.
static void launch_id_reg(const IdArgs& A0, int max_cols, hipStream_t s) {
  const int64_t stride = max_cols;
  DBuf<double> alpha;
  alpha.alloc(stride * A0.nprob, nullptr);
  IdmState S{alpha.p, stride};
  const unsigned np = unsigned(A0.nprob);
  IdArgs A = A0;
  A.alpha = alpha.p;
  A.astride = stride;
  A.skip_cols = 192;
  // waves per problem from the launch-shape table; a wave holds 64 * CB / NW
  // rows of every column
  const hif_tuning tu = tuning();
  if (max_cols <= 64) {
    if (tu.id_reg_waves[0] == 16)
      hipLaunchKernelGGL((k_id_reg<1, 4, 16>), dim3(np), dim3(1024), 0, s, A, S);
    else if (tu.id_reg_waves[0] == 8)
      hipLaunchKernelGGL((k_id_reg<1, 8, 8>), dim3(np), dim3(512), 0, s, A, S);
    else
      hipLaunchKernelGGL((k_id_reg<1, 16, 4>), dim3(np), dim3(256), 0, s, A, S);
  } else if (max_cols <= 128) {
    if (tu.id_reg_waves[1] == 16)
      hipLaunchKernelGGL((k_id_reg<2, 8, 16>), dim3(np), dim3(1024), 0, s, A, S);
    else if (tu.id_reg_waves[1] == 4)
      hipLaunchKernelGGL((k_id_reg<2, 32, 4>), dim3(np), dim3(256), 0, s, A, S);
    else
      hipLaunchKernelGGL((k_id_reg<2, 16, 8>), dim3(np), dim3(512), 0, s, A, S);
  } else {
    if (tu.id_reg_waves[2] == 8)
      hipLaunchKernelGGL((k_id_reg<3, 24, 8>), dim3(np), dim3(512), 0, s, A, S);
    else
      hipLaunchKernelGGL((k_id_reg<3, 12, 16>), dim3(np), dim3(1024), 0, s, A, S);
    if (max_cols > 192) launch_id_small(A, max_cols, s);
  }
  std::vector<int32_t> hk(A.nprob);
  HIF_HIP(hipMemcpyAsync(hk.data(), A.rank, sizeof(int32_t) * A.nprob, hipMemcpyDeviceToHost, s));
  HIF_HIP(hipStreamSynchronize(s));
  int kmax = 0;
  for (int v : hk) kmax = std::max(kmax, v);
  const dim3 tg(unsigned((max_cols + kTb64 - 1) / kTb64), np);
  for (int a0 = ((kmax - 1) / kTb64) * kTb64; kmax > 0 && a0 >= 0; a0 -= kTb64)
    hipLaunchKernelGGL(k_idm_T_block, tg, dim3(256), 0, s, A, S, a0);
  if (A.Tout)
    hipLaunchKernelGGL(k_idm_Tcopy, dim3(unsigned((max_cols + 255) / 256), np), dim3(256), 0, s, A);
  HIF_HIP(hipGetLastError());
  HIF_HIP(hipStreamSynchronize(s));  // alpha is released on return
}

void launch_id(const IdArgs& A, int max_cols, hipStream_t s) {
  if (A.nprob == 0) return;
  // the pivoted QR runs on min(m, n) <= max_cols rows
  if (max_cols > 48 && max_cols <= 256) {  // tiny problems: one wave each in k_id
    launch_id_reg(A, max_cols, s);
    return;
  }
  launch_id_small(A, max_cols, s);
}

static void launch_id_small(const IdArgs& A, int max_cols, hipStream_t s) {
  // the pivoted QR runs on min(m, n) <= max_cols rows, staged in LDS
  if (max_cols > kIdMaxRows) throw Error{HIF_EUNSUPPORTED, "ID problem with more than 4096 columns"};
  int block = 64;
  while (block < max_cols && block < 1024) block *= 2;
  int U = (max_cols + block - 1) / block;
  if (U <= 1)
    hipLaunchKernelGGL(k_id<1>, dim3(A.nprob), dim3(block), 0, s, A);
  else if (U <= 2)
    hipLaunchKernelGGL(k_id<2>, dim3(A.nprob), dim3(block), 0, s, A);
  else if (U <= 4)
    hipLaunchKernelGGL(k_id<4>, dim3(A.nprob), dim3(block), 0, s, A);
  else if (U <= 8)
    hipLaunchKernelGGL(k_id<8>, dim3(A.nprob), dim3(block), 0, s, A);
  else if (U <= 16)
    hipLaunchKernelGGL(k_id<16>, dim3(A.nprob), dim3(block), 0, s, A);
  else
    throw Error{HIF_EUNSUPPORTED, "ID problem with more than 16384 columns"};
  HIF_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Row compression before the ID.  By Lemma 3.1 an ID of any matrix with the
// same row space is an ID of Y; with Y = Q R0 (Householder, no pivoting) the
// n x n upper-triangular R0 has exactly the column norms and pivot sequence of
// Y, so the pivoted QR then runs on R0 instead of the tall m x n block.
// Blocked right-looking Householder QR: panels of kRqNb columns factored in
// place, H = I - V T V^T (compact WY), trailing update W = T^T V^T Y_t,
// Y_t -= V W on the matrix cores.  Scratch per problem: V (m x kRqNb),
// W (kRqNb x n), G (kRqNb x kRqNb).
// ---------------------------------------------------------------------------
constexpr int kRqNb = 16;

// One step of a wave reduce-scatter of 16 values (see k_rowqr).
template <int H>
__device__ __forceinline__ void rs16_step(double (&p)[kRqNb], int lane) {
  const bool up = (lane & (4 * H)) != 0;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const double send = up ? p[i] : p[i + H];
    const double keep = up ? p[i + H] : p[i];
    p[i] = keep + __shfl_xor(send, 4 * H, 64);
  }
}

__global__ __launch_bounds__(256) void k_rowqr(RowQrArgs A) {
  const int q = blockIdx.x;
  const int m = A.rows[q], n = A.cols[q];
  if (m <= n) return;
  double* M = A.base + A.moff[q];
  const int ld = A.ld[q];
  double* V = A.scratch + A.soff[q];
  double* W = V + int64_t(m) * kRqNb;
  double* Gm = W + int64_t(kRqNb) * n;
  __shared__ double lds[kGemmLds];
  __shared__ double sT[kRqNb][kRqNb];
  __shared__ double sbeta[kRqNb];
  __shared__ double sred[4][kRqNb + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int j0 = 0; j0 < n; j0 += kRqNb) {
    const int jb = min(kRqNb, n - j0);
    // --- panel factorization (rows j0..m-1, columns j0..j0+jb-1) ---
    // Two passes over the rows per column: dot products (writing V), then the
    // update, which also accumulates the next column's norm.  Rows go in
    // chunks of 4 per thread so that many loads are in flight.
    double ss = 0.0;
    {
      double s0 = 0.0;
      for (int r = j0 + tid; r < m; r += 256) {
        const double y = M[int64_t(r) * ld + j0];
        s0 += y * y;
      }
      s0 = wave_sum(s0);
      if (lane == 0) sred[wv][0] = s0;
      __syncthreads();
      ss = sred[0][0] + sred[1][0] + sred[2][0] + sred[3][0];
      __syncthreads();
    }
    for (int r = j0 + tid; r < m; r += 256)
      for (int c = 0; c < kRqNb; ++c) V[int64_t(r - j0) * kRqNb + c] = 0.0;
    for (int jj = 0; jj < jb; ++jj) {
      const int j = j0 + jj;
      const int nc = jb - jj - 1;  // remaining panel columns
      const double x0 = M[int64_t(j) * ld + j];
      const double nrm = sqrt(ss);
      const double alpha = nrm > 0.0 ? -copysign(nrm, x0) : 0.0;
      const double v0 = x0 - alpha;
      const double vtv = ss - x0 * x0 + v0 * v0;
      const double beta = vtv > 0.0 ? 2.0 / vtv : 0.0;
      double part[kRqNb];
#pragma unroll
      for (int c = 0; c < kRqNb; ++c) part[c] = 0.0;
      for (int r0 = j + tid; r0 < m; r0 += 4 * 256) {
        double vr[4], y[4][kRqNb];
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const int r = r0 + qq * 256;
          vr[qq] = 0.0;
          if (r < m) vr[qq] = r == j ? v0 : M[int64_t(r) * ld + j];
#pragma unroll
          for (int c = 0; c < kRqNb; ++c) y[qq][c] = (r < m && c < nc) ? M[int64_t(r) * ld + j + 1 + c] : 0.0;
        }
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const int r = r0 + qq * 256;
          if (r < m) V[int64_t(r - j0) * kRqNb + jj] = vr[qq];
#pragma unroll
          for (int c = 0; c < kRqNb; ++c) part[c] += vr[qq] * y[qq][c];
        }
      }
      {
        // all 16 sums at once: lane pairs reduce-scatter, lane l ends with index l >> 2
        rs16_step<8>(part, lane);
        rs16_step<4>(part, lane);
        rs16_step<2>(part, lane);
        rs16_step<1>(part, lane);
        double t = part[0] + __shfl_xor(part[0], 1, 64);
        t += __shfl_xor(t, 2, 64);
        if ((lane & 3) == 0) sred[wv][lane >> 2] = t;
      }
      __syncthreads();
      double wc[kRqNb];
#pragma unroll
      for (int c = 0; c < kRqNb; ++c)
        wc[c] = c < nc ? beta * (sred[0][c] + sred[1][c] + sred[2][c] + sred[3][c]) : 0.0;
      __syncthreads();
      double snext = 0.0;
      for (int r0 = j + tid; r0 < m; r0 += 4 * 256) {
        double vr[4], y[4][kRqNb];
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const int r = r0 + qq * 256;
          vr[qq] = 0.0;
          if (r < m) vr[qq] = r == j ? v0 : M[int64_t(r) * ld + j];
#pragma unroll
          for (int c = 0; c < kRqNb; ++c) y[qq][c] = (r < m && c < nc) ? M[int64_t(r) * ld + j + 1 + c] : 0.0;
        }
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const int r = r0 + qq * 256;
#pragma unroll
          for (int c = 0; c < kRqNb; ++c) y[qq][c] -= wc[c] * vr[qq];
          if (r > j && r < m && nc > 0) snext += y[qq][0] * y[qq][0];
          if (r < m) {
#pragma unroll
            for (int c = 0; c < kRqNb; ++c)
              if (c < nc) M[int64_t(r) * ld + j + 1 + c] = y[qq][c];
          }
        }
      }
      if (tid == 0) sbeta[jj] = beta;
      snext = wave_sum(snext);
      if (lane == 0) sred[wv][0] = snext;
      __syncthreads();
      ss = sred[0][0] + sred[1][0] + sred[2][0] + sred[3][0];
      if (tid == 0) M[int64_t(j) * ld + j] = alpha;
      __syncthreads();
    }
    const int nt = n - j0 - jb;
    if (nt <= 0) break;
    const int mp = m - j0;
    // --- T of the compact WY form: T_ii = beta_i, T(0:i, i) = -beta_i T(0:i,0:i) V(:,0:i)^T v_i ---
    wg_gemm(jb, jb, mp, 1.0, V, kRqNb, true, V, kRqNb, false, 0.0, Gm, kRqNb, lds);
    if (tid == 0) {
      for (int i = 0; i < jb; ++i) {
        sT[i][i] = sbeta[i];
        for (int p = 0; p < i; ++p) {
          double t = 0.0;
          for (int l = p; l < i; ++l) t += sT[p][l] * Gm[l * kRqNb + i];
          sT[p][i] = -sbeta[i] * t;
        }
        for (int p = i + 1; p < jb; ++p) sT[p][i] = 0.0;
      }
    }
    __syncthreads();
    // --- trailing update of columns j0+jb..n-1 ---
    double* Yt = M + int64_t(j0) * ld + j0 + jb;
    wg_gemm(jb, nt, mp, 1.0, V, kRqNb, true, Yt, ld, false, 0.0, W, nt, lds);
    for (int c = tid; c < nt; c += 256) {  // W <- T^T W (lower triangular T^T), bottom row first
      for (int i = jb - 1; i >= 0; --i) {
        double t = 0.0;
        for (int p = 0; p <= i; ++p) t += sT[p][i] * W[int64_t(p) * nt + c];
        W[int64_t(i) * nt + c] = t;
      }
    }
    __syncthreads();
    wg_gemm(mp, nt, jb, -1.0, V, kRqNb, false, W, nt, false, 1.0, Yt, ld, lds);
  }
  // R0 = upper triangle of the leading n x n block; clear what lies below it.
  for (int64_t e = tid; e < int64_t(n) * n; e += 256) {
    const int r = int(e / n), c = int(e % n);
    if (c < r) M[int64_t(r) * ld + c] = 0.0;
  }
}

void launch_rowqr_auto(const RowQrArgs& A, int max_rows, int max_cols, hipStream_t s) {
  // Few large problems: per-panel launches spread each problem over many
  // workgroups; many small ones: one fused workgroup per problem.
  if (max_rows <= 32 * kTsqrStack || (A.nprob < 1024 && max_cols >= 96))
    launch_qr_batched(A, max_rows, max_cols, s);
  else
    launch_rowqr(A, s);
}

void launch_rowqr(const RowQrArgs& A, hipStream_t s) {
  if (A.nprob == 0) return;
  hipLaunchKernelGGL(k_rowqr, dim3(A.nprob), dim3(256), 0, s, A);
  HIF_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// LU with partial pivoting (row interchanges, LAPACK convention: rows j and
// piv[j] swapped at step j) of an n x n row-major block, by one workgroup.
// ---------------------------------------------------------------------------
__device__ void block_lu(double* A, int n, int ld, int32_t* piv, int32_t* status) {
  const int tid = threadIdx.x, B = blockDim.x;
  for (int j = 0; j < n; ++j) {
    ArgMax loc{-1.0, INT_MAX};
    for (int i = j + tid; i < n; i += B) loc = better(loc, ArgMax{fabs(A[int64_t(i) * ld + j]), i});
    const ArgMax best = block_argmax(loc);
    if (!(best.v > 0.0)) {
      if (tid == 0) { piv[j] = j; atomicOr(status, 1); }
      return;
    }
    const int p = best.i;
    if (tid == 0) piv[j] = p;
    if (p != j)
      for (int col = tid; col < n; col += B) {
        double t = A[int64_t(j) * ld + col];
        A[int64_t(j) * ld + col] = A[int64_t(p) * ld + col];
        A[int64_t(p) * ld + col] = t;
      }
    __syncthreads();
    const double inv = 1.0 / A[int64_t(j) * ld + j];
    for (int i = j + 1 + tid; i < n; i += B) A[int64_t(i) * ld + j] *= inv;
    __syncthreads();
    const int w = n - j - 1;
    const int64_t tot = int64_t(w) * w;
    for (int64_t e = tid; e < tot; e += B) {
      const int i = j + 1 + int(e / w), l = j + 1 + int(e % w);
      A[int64_t(i) * ld + l] -= A[int64_t(i) * ld + j] * A[int64_t(j) * ld + l];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Skeletonization of one group (Lemma 2.4) and elimination of its redundant
// DOFs (Lemma 2.1).  In (redundant, skeleton) order, Q^T A_cc Q has the blocks
//   B_sr = A_sr - A_ss T,  B_rs = A_rs - T^T A_ss,  B_rr = A_rr - A_rs T - T^T B_sr,
// and B_ss = A_ss.  A partial LU of M = [B_rr B_rs; B_sr S_ss] over its first
// r columns, pivoting among the redundant rows only, gives
//   P B_rr = L U,  U_rs = L^{-1} P B_rs,  L_sr = B_sr U^{-1},
// and leaves S_ss - L_sr U_rs = S_old(s,s) - B_sr B_rr^{-1} B_rs, the updated
// SCI block, in the trailing corner (M's skeleton block starts as the old
// SCI block S_old(s,s) instead of A_ss).  These are the factors R_p and S_p
// of Lemma 2.1 with the block LDU folded into (L, U).  The four products with
// T and the trailing updates of the blocked LU run on the matrix cores.
// ---------------------------------------------------------------------------
constexpr int kLuNb = 16;

struct ElimView {
  int r, k, n;
  int64_t c0;
  int32_t *rd, *sk, *piv;
  double *T, *Lsr, *Urs, *LU, *M;
  const double *Y, *Acc, *Scc;
  int32_t *rdl, *skl, *rlo, *rhi;
  const int32_t* cord;
};

__device__ ElimView elim_view(const ElimArgs& A, int g, const GroupRec& R) {
  ElimView v;
  v.r = R.r;
  v.k = R.k;
  v.c0 = A.gstart[g];
  v.n = int(A.gstart[g + 1] - v.c0);
  v.rd = A.iarena + R.idx;
  v.sk = v.rd + v.r;
  v.piv = v.sk + v.k;
  v.T = A.darena + R.off;
  v.Lsr = v.T + int64_t(v.k) * v.r;
  v.Urs = v.Lsr + int64_t(v.k) * v.r;
  v.LU = v.Urs + int64_t(v.r) * v.k;
  v.Y = A.Y + A.yoff[g];
  v.Acc = A.Acc + A.aoff[g];
  v.Scc = A.Scc + A.aoff[g];
  v.M = A.Mw + A.aoff[g];
  v.rdl = A.loc + v.c0;  // rd_loc (r) then sk_loc (k): the (redundant, skeleton) order
  v.skl = v.rdl + v.r;
  v.rlo = A.rlo + v.c0;
  v.rhi = A.rhi + v.c0;
  v.cord = A.cord + v.c0;
  return v;
}

// Skeleton / redundant lists in class order.
__device__ void elim_lists(const ElimArgs& A, int g, const ElimView& v) {
  const int tid = threadIdx.x, B = blockDim.x;
  for (int q = A.cls_first[g]; q < A.cls_first[g + 1]; ++q) {
    const int col0 = A.cls_col0[q], nq = A.cls_n[q], kq = A.cls_rank[q];
    const int so = A.cls_skoff[q], ro = A.cls_rdoff[q];
    const int32_t* pq = A.perm + v.c0 + col0;
    for (int j = tid; j < nq; j += B) {
      const int gl = col0 + pq[j];
      if (j < kq) {
        v.skl[so + j] = gl;
        v.sk[so + j] = v.cord[gl];
      } else {
        const int bb = ro + (j - kq);
        v.rdl[bb] = gl;
        v.rd[bb] = v.cord[gl];
        v.rlo[bb] = so;
        v.rhi[bb] = so + kq;
      }
    }
  }
}

// T (k x r, block diagonal over the classes) and M = A_cc in (redundant,
// skeleton) order; this workgroup does share `part` of `nparts`.
__device__ void elim_gather(const ElimView& v, int part, int nparts) {
  const int B = blockDim.x;
  const int64_t e0 = int64_t(part) * B + threadIdx.x, es = int64_t(nparts) * B;
  const int r = v.r, k = v.k, n = v.n;
  for (int64_t e = e0; e < int64_t(k) * r; e += es) {
    const int a = int(e / r), bb = int(e % r);
    const int lo = v.rlo[bb];
    v.T[e] = (a >= lo && a < v.rhi[bb]) ? v.Y[int64_t(a - lo) * n + v.rdl[bb]] : 0.0;
  }
  for (int64_t e = e0; e < int64_t(n) * n; e += es) {
    const int i = int(e / n), j = int(e % n);
    v.M[e] = v.Acc[int64_t(v.rdl[i]) * n + v.rdl[j]];
  }
}

__device__ void elim_setup(const ElimArgs& A, int g, const ElimView& v) {
  elim_lists(A, g, v);
  __syncthreads();
  elim_gather(v, 0, 1);
  __syncthreads();
}

// The skeleton block of M starts as the old SCI block S_old(s,s).
__device__ void elim_sss(const ElimView& v, int part, int nparts) {
  const int n = v.n, r = v.r, k = v.k;
  double* Mss = v.M + int64_t(r) * n + r;
  for (int64_t e = int64_t(part) * blockDim.x + threadIdx.x; e < int64_t(k) * k; e += int64_t(nparts) * blockDim.x) {
    const int a = int(e / k), a2 = int(e % k);
    Mss[int64_t(a) * n + a2] = v.Scc[int64_t(v.skl[a]) * n + v.skl[a2]];
  }
}

// Factors into the record, the updated SCI block into the new entries.
__device__ void elim_finish(const ElimArgs& A, int g, const ElimView& v, int part, int nparts) {
  const int64_t e0 = int64_t(part) * blockDim.x + threadIdx.x, es = int64_t(nparts) * blockDim.x;
  const int n = v.n, r = v.r, k = v.k;
  const double* Mss = v.M + int64_t(r) * n + r;
  for (int64_t e = e0; e < int64_t(r) * r; e += es) v.LU[e] = v.M[(e / r) * n + e % r];
  for (int64_t e = e0; e < int64_t(r) * k; e += es) v.Urs[e] = v.M[(e / k) * n + r + e % k];
  for (int64_t e = e0; e < int64_t(k) * r; e += es) v.Lsr[e] = v.M[(r + e / r) * n + e % r];
  uint64_t* nk = A.newkey + A.newoff[g];
  double2* nv = A.newval + A.newoff[g];
  for (int64_t e = e0; e < int64_t(k) * k; e += es) {
    const int a = int(e / k), a2 = int(e % k);
    nk[e] = (uint64_t(uint32_t(v.sk[a])) << 32) | uint32_t(v.sk[a2]);
    nv[e] = make_double2(Mss[int64_t(a) * n + a2], Mss[int64_t(a2) * n + a]);
  }
}

__global__ __launch_bounds__(256) void k_eliminate(ElimArgs A) {
  const int g = blockIdx.x;
  const int ri = A.grec[g];
  if (ri < 0) return;
  const GroupRec R = A.recs[ri];
  const ElimView v = elim_view(A, g, R);
  const int r = v.r, k = v.k, n = v.n;
  const int tid = threadIdx.x, B = blockDim.x;
  __shared__ double lds[kGemmLds];
  double* M = v.M;
  int32_t* piv = v.piv;
  elim_setup(A, g, v);
  // the skeletonization transform Q^T A_cc Q
  double* Mrr = M;
  double* Mrs = M + r;
  double* Msr = M + int64_t(r) * n;
  double* Mss = Msr + r;
  if (k > 0) {
    if (A.fp32) {
      wg_gemm_f32(r, r, k, -1.0, Mrs, n, false, v.T, r, false, 1.0, Mrr, n, lds);
      wg_gemm_f32(k, r, k, -1.0, Mss, n, false, v.T, r, false, 1.0, Msr, n, lds);
      wg_gemm_f32(r, r, k, -1.0, v.T, r, true, Msr, n, false, 1.0, Mrr, n, lds);
      wg_gemm_f32(r, k, k, -1.0, v.T, r, true, Mss, n, false, 1.0, Mrs, n, lds);
    } else {
      wg_gemm(r, r, k, -1.0, Mrs, n, false, v.T, r, false, 1.0, Mrr, n, lds);   // A_rr - A_rs T
      wg_gemm(k, r, k, -1.0, Mss, n, false, v.T, r, false, 1.0, Msr, n, lds);   // B_sr
      wg_gemm(r, r, k, -1.0, v.T, r, true, Msr, n, false, 1.0, Mrr, n, lds);    // B_rr
      wg_gemm(r, k, k, -1.0, v.T, r, true, Mss, n, false, 1.0, Mrs, n, lds);    // B_rs
    }
    elim_sss(v, 0, 1);
    __syncthreads();
  }
  // blocked partial LU over the first r columns
  for (int j0 = 0; j0 < r; j0 += kLuNb) {
    const int jb = min(kLuNb, r - j0);
    for (int j = j0; j < j0 + jb; ++j) {
      ArgMax loc2{-1.0, INT_MAX};
      for (int i = j + tid; i < r; i += B) loc2 = better(loc2, ArgMax{fabs(M[int64_t(i) * n + j]), i});
      const ArgMax best = block_argmax(loc2);
      if (!(best.v > 0.0)) {
        if (tid == 0) atomicOr(A.status, 1);
        return;
      }
      const int p = best.i;
      if (tid == 0) piv[j] = p;
      if (p != j)
        for (int col = tid; col < n; col += B) {
          const double t = M[int64_t(j) * n + col];
          M[int64_t(j) * n + col] = M[int64_t(p) * n + col];
          M[int64_t(p) * n + col] = t;
        }
      __syncthreads();
      const double inv = 1.0 / M[int64_t(j) * n + j];
      const int w = j0 + jb - j - 1;
      for (int i = j + 1 + tid; i < n; i += B) {
        double* row = M + int64_t(i) * n;
        const double l = row[j] * inv;
        row[j] = l;
        for (int c = 1; c <= w; ++c) row[j + c] -= l * M[int64_t(j) * n + j + c];
      }
      __syncthreads();
    }
    const int nt = n - j0 - jb;
    if (nt > 0) {
      for (int c = j0 + jb + tid; c < n; c += B)
        for (int i = j0 + 1; i < j0 + jb; ++i) {
          double val = M[int64_t(i) * n + c];
          for (int p = j0; p < i; ++p) val -= M[int64_t(i) * n + p] * M[int64_t(p) * n + c];
          M[int64_t(i) * n + c] = val;
        }
      __syncthreads();
      wg_gemm(n - j0 - jb, nt, jb, -1.0, M + int64_t(j0 + jb) * n + j0, n, false, M + int64_t(j0) * n + j0 + jb, n,
              false, 1.0, M + int64_t(j0 + jb) * n + j0 + jb, n, lds);
    }
  }
  elim_finish(A, g, v, 0, 1);
}

// Split path for sub-levels with few, large groups: setup, M_ss, finish as
// kernels of their own; the transform and the partial LU run as batched
// multi-workgroup launches in between.
__global__ __launch_bounds__(256) void k_elim_lists(ElimArgs A) {
  const int g = blockIdx.x;
  const int ri = A.grec[g];
  if (ri < 0) return;
  const GroupRec R = A.recs[ri];
  elim_lists(A, g, elim_view(A, g, R));
}

__global__ __launch_bounds__(256) void k_elim_gather(ElimArgs A) {
  const int g = blockIdx.y;
  const int ri = A.grec[g];
  if (ri < 0) return;
  const GroupRec R = A.recs[ri];
  elim_gather(elim_view(A, g, R), blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void k_elim_sss(ElimArgs A) {
  const int g = blockIdx.y;
  const int ri = A.grec[g];
  if (ri < 0) return;
  const GroupRec R = A.recs[ri];
  if (R.k > 0) elim_sss(elim_view(A, g, R), blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void k_elim_finish(ElimArgs A) {
  const int g = blockIdx.y;
  const int ri = A.grec[g];
  if (ri < 0) return;
  const GroupRec R = A.recs[ri];
  elim_finish(A, g, elim_view(A, g, R), blockIdx.x, gridDim.x);
}

// Workgroups per group for the copy kernels: about 16K entries each.
static unsigned elim_parts(const ElimArgs& A) {
  const int64_t n = A.max_n;
  return unsigned(std::min<int64_t>(256, std::max<int64_t>(1, n * n / 16384)));
}

void launch_elim_setup(const ElimArgs& A, hipStream_t s) {
  if (A.ngroups == 0) return;
  hipLaunchKernelGGL(k_elim_lists, dim3(A.ngroups), dim3(256), 0, s, A);
  hipLaunchKernelGGL(k_elim_gather, dim3(elim_parts(A), A.ngroups), dim3(256), 0, s, A);
  HIF_HIP(hipGetLastError());
}
void launch_elim_sss(const ElimArgs& A, hipStream_t s) {
  if (A.ngroups == 0) return;
  hipLaunchKernelGGL(k_elim_sss, dim3(elim_parts(A), A.ngroups), dim3(256), 0, s, A);
  HIF_HIP(hipGetLastError());
}
void launch_elim_finish(const ElimArgs& A, hipStream_t s) {
  if (A.ngroups == 0) return;
  hipLaunchKernelGGL(k_elim_finish, dim3(elim_parts(A), A.ngroups), dim3(256), 0, s, A);
  HIF_HIP(hipGetLastError());
}

void launch_eliminate(const ElimArgs& A, hipStream_t s) {
  if (A.ngroups == 0) return;
  hipLaunchKernelGGL(k_eliminate, dim3(A.ngroups), dim3(256), 0, s, A);
  HIF_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Top block (Section 3.1, level L): D's last block A_L(s_L, s_L).
// ---------------------------------------------------------------------------
template <int D>
__global__ void k_top_assemble(TopArgs A) {
  const int64_t n = A.n;
  const int64_t tot = n * n;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t ri = e / n, ci = e % n;
    const int i = A.idx[ri], j = A.idx[ci];
    double v;
    if (i == j) {
      v = A.a[i] + A.b[i] * A.selfk[i] * A.c[i];
    } else {
      double r2 = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        double t = A.pts[int64_t(i) * D + k] - A.pts[int64_t(j) * D + k];
        r2 += t * t;
      }
      v = A.b[i] * green_mixed<D>(r2, A.fp32 != 0) * A.w[j] * A.c[j];
    }
    A.A[e] = entry_prec(v, A.fp32 != 0);
  }
}

__global__ void k_top_sci(TopArgs A) {
  const int64_t ri = blockIdx.x;
  const int i = A.idx[ri];
  for (int64_t e = A.srow[i] + threadIdx.x; e < A.srow[i + 1]; e += blockDim.x) {
    const int j = int(A.skey[e] & 0xffffffffu);
    A.A[ri * A.n + A.pos_of[j]] += A.sval[e].x;
  }
}

__global__ void k_top_lu(TopArgs A) { block_lu(A.A, int(A.n), int(A.n), A.piv, A.status); }

void launch_top(const TopArgs& A, hipStream_t s) {
  if (A.n == 0) return;
  const int64_t tot = A.n * A.n;
  int blocks = int((tot + 255) / 256);
  if (blocks > 65536) blocks = 65536;
  if (A.dim == 2)
    hipLaunchKernelGGL(k_top_assemble<2>, dim3(blocks), dim3(256), 0, s, A);
  else
    hipLaunchKernelGGL(k_top_assemble<3>, dim3(blocks), dim3(256), 0, s, A);
  HIF_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_top_sci, dim3(unsigned(A.n)), dim3(64), 0, s, A);
  HIF_HIP(hipGetLastError());
  if (A.n <= 256) {
    hipLaunchKernelGGL(k_top_lu, dim3(1), dim3(1024), 0, s, A);
    HIF_HIP(hipGetLastError());
  }
}

// ---------------------------------------------------------------------------
// Stand-alone batched ID (hif_id_batched).
// ---------------------------------------------------------------------------
__global__ void k_copy_ld(const int32_t* cols, int32_t* ld, int nb) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb) ld[i] = cols[i];
}

void id_batched_impl(double* mats, const int64_t* off, const int32_t* rows, const int32_t* cols,
                     const double* tol, int32_t batch, int32_t max_cols, int32_t* rank,
                     int32_t* perm, const int64_t* off_perm, double* T, const int64_t* off_t,
                     hipStream_t s) {
  DBuf<int32_t> ld;
  ld.alloc(size_t(batch), nullptr);
  hipLaunchKernelGGL(k_copy_ld, dim3((batch + 255) / 256), dim3(256), 0, s, cols, ld.p, batch);
  HIF_HIP(hipGetLastError());
  // Row compression first, as in the factorization.
  std::vector<int32_t> hr(batch), hc(batch);
  HIF_HIP(hipMemcpyAsync(hr.data(), rows, sizeof(int32_t) * batch, hipMemcpyDeviceToHost, s));
  HIF_HIP(hipMemcpyAsync(hc.data(), cols, sizeof(int32_t) * batch, hipMemcpyDeviceToHost, s));
  HIF_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> hr2(batch);
  std::vector<int64_t> hso(batch);
  int64_t qt = 0;
  int max_rows = 1;
  for (int p = 0; p < batch; ++p) {
    HIF_REQUIRE(hc[p] >= 1 && hc[p] <= max_cols && hr[p] >= 1, HIF_EINVAL,
                "every matrix needs 1 <= cols <= max_cols and rows >= 1");
    hr2[p] = std::min(hr[p], hc[p]);
    hso[p] = qt;
    max_rows = std::max(max_rows, hr[p]);
    if (hr[p] > hc[p]) qt += rowqr_scratch(hr[p], hc[p]);
  }
  DBuf<int32_t> rows2;
  DBuf<int64_t> soff;
  DBuf<double> scratch;
  rows2.alloc(batch, nullptr);
  soff.alloc(batch, nullptr);
  scratch.alloc(qt + 1, nullptr);
  HIF_HIP(hipMemcpyAsync(rows2.p, hr2.data(), sizeof(int32_t) * batch, hipMemcpyHostToDevice, s));
  HIF_HIP(hipMemcpyAsync(soff.p, hso.data(), sizeof(int64_t) * batch, hipMemcpyHostToDevice, s));
  RowQrArgs Q;
  Q.base = mats;
  Q.moff = off;
  Q.ld = ld.p;
  Q.rows = rows;
  Q.cols = cols;
  Q.scratch = scratch.p;
  Q.soff = soff.p;
  Q.nprob = batch;
  double smn = 0.0, snn = 0.0;
  for (int p = 0; p < batch; ++p) {
    smn += double(hr[p]) * hc[p];
    snn += double(hc[p]) * hc[p];
  }
  const bool direct = id_blocked_fits(batch, max_rows, max_cols) && smn <= 1.25 * snn;
  if (!direct && rowqr_split_fits(max_rows, max_cols)) {
    std::vector<int64_t> ho(batch);
    HIF_HIP(hipMemcpyAsync(ho.data(), off, sizeof(int64_t) * batch, hipMemcpyDeviceToHost, s));
    HIF_HIP(hipStreamSynchronize(s));
    launch_rowqr_split(mats, ho, hc, hr, hc, nullptr, s);
  } else if (!direct) {
    launch_rowqr_auto(Q, max_rows, max_cols, s);
  }
  IdArgs A;
  A.base = mats;
  A.moff = off;
  A.ld = ld.p;
  A.rows = direct ? rows : rows2.p;
  A.cols = cols;
  A.tol = tol;
  A.rank = rank;
  A.perm = perm;
  A.poff = off_perm;
  A.Tout = T;
  A.toff = off_t;
  A.nprob = batch;
  if (direct)
    launch_id_blocked(A, max_rows, max_cols, s);
  else if (id_blocked_fits(batch, max_cols, max_cols))
    launch_id_blocked(A, max_cols, max_cols, s);  // on R0: rows <= columns
  else
    launch_id(A, max_cols, s);
  HIF_HIP(hipStreamSynchronize(s));
}

}  // namespace hif
