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
#pragma unroll
      for (int k = 0; k < D; ++k) xi[k] = A.zc[int64_t(g) * D + k] + A.R * A.proxy_u[p * D + k];
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
  // T = R11^{-1} R12, R11[a][b] = M[a][perm[b]]; written in place over R12.
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (state[u] != -1) continue;
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
  if (A.Tout) {
    __syncthreads();
    const int r = n - k;
    double* T = A.Tout + A.toff[q];
    for (int e = tid; e < k * r; e += B) {
      const int a = e / r, b2 = e % r;
      T[e] = M[int64_t(a) * ld + perm[k + b2]];
    }
  }
}

// ---------------------------------------------------------------------------
// Multi-workgroup ID for few large problems: the same column-pivoted
// Householder QR as k_id (recomputed norms, ties to the lowest column, rank
// rule of Section 2.2), one launch per pivot step.  Workgroup (b, q) owns
// columns 64b..64b+63 of problem q; every workgroup finds the pivot from the
// norms of the previous step (double-buffered, so no workgroup reads what
// another writes in the same launch), applies the reflector to its columns
// and recomputes their norms.  The pivot column keeps its Householder vector
// below the diagonal and R_ii goes to alpha.  State of problem q lives at
// q * stride.
// ---------------------------------------------------------------------------
struct IdmState {
  double* nrm;    // [2][nprob * stride] squared norms of the rows below the step
  int32_t* st;    // [2][nprob * stride] -2 absent, -1 trailing, >= 0 pivot step
  double* alpha;  // [nprob * stride] R_ii
  double* r00;    // [nprob]
  int32_t* done;  // [nprob]
  int64_t stride;
  int64_t total;  // nprob * stride
};
constexpr int kIdmCols = 64;
constexpr int kIdmThreads = 256;

__global__ __launch_bounds__(kIdmThreads) void k_idm_init(IdArgs A, IdmState S) {
  const int q = blockIdx.y;
  const int m = A.rows[q], n = A.cols[q];
  const int c0 = blockIdx.x * kIdmCols;
  if (c0 >= n) return;
  const double* M = A.base + A.moff[q];
  const int ld = A.ld[q];
  const int lc = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int col = c0 + lc;
  __shared__ double sp[4][kIdmCols];
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
    S.nrm[o] = sp[0][lc] + sp[1][lc] + sp[2][lc] + sp[3][lc];
    S.st[o] = -1;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S.done[q] = 0;
    A.rank[q] = min(m, n);
  }
}

__global__ __launch_bounds__(kIdmThreads) void k_idm_step(IdArgs A, IdmState S, int i) {
  const int q = blockIdx.y;
  const int m = A.rows[q], n = A.cols[q];
  const int c0 = blockIdx.x * kIdmCols;
  if (c0 >= n || i >= min(m, n) || S.done[q]) return;
  const int cur = i & 1, nxt = cur ^ 1;
  const double* nrm = S.nrm + cur * S.total + q * S.stride;
  const int32_t* st = S.st + cur * S.total + q * S.stride;
  ArgMax loc{-1.0, INT_MAX};
  for (int c = threadIdx.x; c < n; c += kIdmThreads)
    if (st[c] == -1) loc = better(loc, ArgMax{nrm[c], c});
  const ArgMax best = block_argmax(loc);
  const double nb = sqrt(best.v > 0.0 ? best.v : 0.0);
  const double r00 = i == 0 ? nb : S.r00[q];
  if (!(best.v > 0.0) || !(nb > A.tol[q] * r00)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      A.rank[q] = i;
      S.done[q] = 1;
    }
    return;
  }
  if (i == 0 && blockIdx.x == 0 && threadIdx.x == 0) S.r00[q] = nb;
  const int p = best.i;
  double* M = A.base + A.moff[q];
  const int ld = A.ld[q];
  const double x0 = M[int64_t(i) * ld + p];
  const double alpha = -copysign(nb, x0);
  const double v0 = x0 - alpha;
  const double vtv = best.v - x0 * x0 + v0 * v0;
  const double beta = vtv > 0.0 ? 2.0 / vtv : 0.0;
  const int lc = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int col = c0 + lc;
  const int state = col < n ? st[col] : -2;
  const bool upd = state == -1 && col != p;
  __shared__ double sp[4][kIdmCols];
  const double* vp = M + p;   // pivot column, rows > i hold the vector
  double* yc = M + col;
  double dot = 0.0;
  if (upd) {
    if (rg == 0) dot = v0 * yc[int64_t(i) * ld];
    int r = i + 1 + rg;
    for (; r + 28 < m; r += 32) {
      double vv[8], yy[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        vv[u] = vp[int64_t(r + 4 * u) * ld];
        yy[u] = yc[int64_t(r + 4 * u) * ld];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) dot += vv[u] * yy[u];
    }
    for (; r < m; r += 4) dot += vp[int64_t(r) * ld] * yc[int64_t(r) * ld];
  }
  sp[rg][lc] = dot;
  __syncthreads();
  const double w = beta * (sp[0][lc] + sp[1][lc] + sp[2][lc] + sp[3][lc]);
  __syncthreads();
  double s2 = 0.0;
  if (upd) {
    if (rg == 0) yc[int64_t(i) * ld] -= w * v0;
    int r = i + 1 + rg;
    for (; r + 28 < m; r += 32) {
      double vv[8], yy[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        vv[u] = vp[int64_t(r + 4 * u) * ld];
        yy[u] = yc[int64_t(r + 4 * u) * ld];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        yy[u] -= w * vv[u];
        s2 += yy[u] * yy[u];
        yc[int64_t(r + 4 * u) * ld] = yy[u];
      }
    }
    for (; r < m; r += 4) {
      const double y = yc[int64_t(r) * ld] - w * vp[int64_t(r) * ld];
      yc[int64_t(r) * ld] = y;
      s2 += y * y;
    }
  }
  sp[rg][lc] = s2;
  __syncthreads();
  if (rg == 0 && col < n) {
    const int64_t o = nxt * S.total + q * S.stride + col;
    if (upd) {
      S.nrm[o] = sp[0][lc] + sp[1][lc] + sp[2][lc] + sp[3][lc];
      S.st[o] = -1;
    } else if (col == p) {
      S.st[o] = i;
      S.alpha[q * S.stride + i] = alpha;
      A.perm[A.poff[q] + i] = p;
    } else {
      S.st[o] = state;
    }
  }
}

// Same step when at most kIrRows * kIrGroups rows are left below it:
// workgroup (b, q) owns 32 columns, thread (c, g) = (tid % 32, tid / 32)
// keeps rows i + g + 32u (u < kIrRows) of column c in registers between the
// dot product and the update, so every entry is read and written once per
// step; the Householder vector is staged in LDS.
constexpr int kIrCols = 32;
constexpr int kIrGroups = 32;
constexpr int kIrRows = 28;
constexpr int kIrMaxRows = kIrRows * kIrGroups;

__global__ __launch_bounds__(1024) void k_idm_step_reg(IdArgs A, IdmState S, int i) {
  const int q = blockIdx.y;
  const int m = A.rows[q], n = A.cols[q];
  const int c0 = blockIdx.x * kIrCols;
  if (c0 >= n || i >= min(m, n) || S.done[q]) return;
  const int cur = i & 1, nxt = cur ^ 1;
  const double* nrm = S.nrm + cur * S.total + q * S.stride;
  const int32_t* st = S.st + cur * S.total + q * S.stride;
  ArgMax loc{-1.0, INT_MAX};
  for (int c = threadIdx.x; c < n; c += 1024)
    if (st[c] == -1) loc = better(loc, ArgMax{nrm[c], c});
  const ArgMax best = block_argmax(loc);
  const double nb = sqrt(best.v > 0.0 ? best.v : 0.0);
  const double r00 = i == 0 ? nb : S.r00[q];
  if (!(best.v > 0.0) || !(nb > A.tol[q] * r00)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      A.rank[q] = i;
      S.done[q] = 1;
    }
    return;
  }
  if (i == 0 && blockIdx.x == 0 && threadIdx.x == 0) S.r00[q] = nb;
  const int p = best.i;
  double* M = A.base + A.moff[q];
  const int ld = A.ld[q];
  const double x0 = M[int64_t(i) * ld + p];
  const double alpha = -copysign(nb, x0);
  const double v0 = x0 - alpha;
  const double vtv = best.v - x0 * x0 + v0 * v0;
  const double beta = vtv > 0.0 ? 2.0 / vtv : 0.0;
  const int mr = m - i;  // <= kIrMaxRows (checked on the host)
  __shared__ double sv[kIrMaxRows];
  __shared__ double sp[16][kIrCols];
  const int tid = threadIdx.x, c = tid & 31, g = tid >> 5, wv = tid >> 6;
  for (int rr = tid; rr < mr; rr += 1024) sv[rr] = rr == 0 ? v0 : M[int64_t(i + rr) * ld + p];
  const int col = c0 + c;
  const int state = col < n ? st[col] : -2;
  const bool upd = state == -1 && col != p;
  double* yc = M + int64_t(i) * ld + col;  // row i of this column
  double y[kIrRows];
#pragma unroll
  for (int u = 0; u < kIrRows; ++u) {
    const int rr = g + kIrGroups * u;
    y[u] = (upd && rr < mr) ? yc[int64_t(rr) * ld] : 0.0;
  }
  __syncthreads();
  double dot = 0.0;
#pragma unroll
  for (int u = 0; u < kIrRows; ++u) {
    const int rr = g + kIrGroups * u;
    if (rr < mr) dot += sv[rr] * y[u];
  }
  dot += __shfl_xor(dot, 32, 64);
  if ((tid & 63) < 32) sp[wv][c] = dot;
  __syncthreads();
  double tdot = 0.0;
#pragma unroll
  for (int w2 = 0; w2 < 16; ++w2) tdot += sp[w2][c];
  const double w = beta * tdot;
  __syncthreads();
  double s2 = 0.0;
#pragma unroll
  for (int u = 0; u < kIrRows; ++u) {
    const int rr = g + kIrGroups * u;
    if (rr < mr) {
      y[u] -= w * sv[rr];
      if (rr > 0) s2 += y[u] * y[u];
    }
  }
  if (upd) {
#pragma unroll
    for (int u = 0; u < kIrRows; ++u) {
      const int rr = g + kIrGroups * u;
      if (rr < mr) yc[int64_t(rr) * ld] = y[u];
    }
  }
  s2 += __shfl_xor(s2, 32, 64);
  if ((tid & 63) < 32) sp[wv][c] = s2;
  __syncthreads();
  if (g == 0 && col < n) {
    const int64_t o = nxt * S.total + q * S.stride + col;
    if (upd) {
      double t = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < 16; ++w2) t += sp[w2][c];
      S.nrm[o] = t;
      S.st[o] = -1;
    } else if (col == p) {
      S.st[o] = i;
      S.alpha[q * S.stride + i] = alpha;
      A.perm[A.poff[q] + i] = p;
    } else {
      S.st[o] = state;
    }
  }
}

// Redundant columns in ascending order after the skeleton (one workgroup per problem).
__global__ __launch_bounds__(1024) void k_idm_perm(IdArgs A, IdmState S) {
  const int q = blockIdx.x;
  const int n = A.cols[q];
  const int k = A.rank[q];
  const int32_t* st = S.st + (k & 1) * S.total + q * S.stride;
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

static void launch_id_multi(const IdArgs& A, int max_cols, hipStream_t s) {
  const int64_t stride = max_cols;
  const int64_t total = stride * A.nprob;
  DBuf<double> nrm, alpha, r00;
  DBuf<int32_t> st, done;
  nrm.alloc(2 * total, nullptr);
  st.alloc(2 * total, nullptr);
  alpha.alloc(total, nullptr);
  r00.alloc(A.nprob, nullptr);
  done.alloc(A.nprob, nullptr);
  IdmState S{nrm.p, st.p, alpha.p, r00.p, done.p, stride, total};
  const dim3 grid(unsigned((max_cols + kIdmCols - 1) / kIdmCols), unsigned(A.nprob));
  const dim3 grid_reg(unsigned((max_cols + kIrCols - 1) / kIrCols), unsigned(A.nprob));
  hipLaunchKernelGGL(k_idm_init, grid, dim3(kIdmThreads), 0, s, A, S);
  std::vector<int32_t> hd(A.nprob);
  // the ID runs on the compressed block (rows <= cols <= max_cols): steps
  // with at most kIrMaxRows rows left keep the columns in registers
  for (int i = 0; i < max_cols; ++i) {
    if (max_cols - i <= kIrMaxRows)
      hipLaunchKernelGGL(k_idm_step_reg, grid_reg, dim3(1024), 0, s, A, S, i);
    else
      hipLaunchKernelGGL(k_idm_step, grid, dim3(kIdmThreads), 0, s, A, S, i);
    if ((i & 15) == 15) {  // stop launching once every problem has met the rank rule
      HIF_HIP(hipMemcpyAsync(hd.data(), done.p, sizeof(int32_t) * A.nprob, hipMemcpyDeviceToHost, s));
      HIF_HIP(hipStreamSynchronize(s));
      bool all = true;
      for (int v : hd) all = all && v;
      if (all) break;
    }
  }
  hipLaunchKernelGGL(k_idm_perm, dim3(A.nprob), dim3(1024), 0, s, A, S);
  // ranks bound the row blocks of the triangular solve
  std::vector<int32_t> hk(A.nprob);
  HIF_HIP(hipMemcpyAsync(hk.data(), A.rank, sizeof(int32_t) * A.nprob, hipMemcpyDeviceToHost, s));
  HIF_HIP(hipStreamSynchronize(s));
  int kmax = 0;
  for (int v : hk) kmax = std::max(kmax, v);
  const dim3 tg(unsigned((max_cols + kTb64 - 1) / kTb64), unsigned(A.nprob));
  for (int a0 = ((kmax - 1) / kTb64) * kTb64; kmax > 0 && a0 >= 0; a0 -= kTb64)
    hipLaunchKernelGGL(k_idm_T_block, tg, dim3(256), 0, s, A, S, a0);
  if (A.Tout)
    hipLaunchKernelGGL(k_idm_Tcopy, dim3(unsigned((max_cols + 255) / 256), unsigned(A.nprob)), dim3(256), 0, s, A);
  HIF_HIP(hipGetLastError());
  HIF_HIP(hipStreamSynchronize(s));  // the state buffers are released on return
}

void launch_id(const IdArgs& A, int max_cols, hipStream_t s) {
  if (A.nprob == 0) return;
  if (A.nprob <= 2048 && max_cols >= 128) {
    launch_id_multi(A, max_cols, s);
    return;
  }
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
  launch_rowqr_auto(Q, max_rows, max_cols, s);
  IdArgs A;
  A.base = mats;
  A.moff = off;
  A.ld = ld.p;
  A.rows = rows2.p;
  A.cols = cols;
  A.tol = tol;
  A.rank = rank;
  A.perm = perm;
  A.poff = off_perm;
  A.Tout = T;
  A.toff = off_t;
  A.nprob = batch;
  launch_id(A, max_cols, s);
  HIF_HIP(hipStreamSynchronize(s));
}

}  // namespace hif
