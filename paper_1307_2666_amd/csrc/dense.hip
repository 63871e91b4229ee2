// Per-group dense kernels of the factorization: batched assembly of the
// compressed blocks, batched interpolative decomposition, batched
// skeletonization / elimination, and the top block LU.
//
// All kernels run one workgroup per independent problem (the groups of one
// sub-level commute, Section 2.3), on row-major blocks in device memory.
#include <climits>

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
// Thread t owns columns t, t+B, ...; each column is filled top to bottom so
// consecutive threads write consecutive addresses of a row.
// ---------------------------------------------------------------------------
template <int D>
__global__ void k_assemble(AsmArgs A) {
  const int g = blockIdx.x;
  const int64_t c0 = A.gstart[g];
  const int n = int(A.gstart[g + 1] - c0);
  const int64_t f0 = A.nf_start[g];
  const int nf = int(A.nf_start[g + 1] - f0);
  const int P = A.nproxy;
  const int m = A.sym ? nf + P : 2 * nf + 2 * P;
  double* Y = A.Y + A.yoff[g];
  double* Acc = A.Acc + A.aoff[g];
  double* Scc = A.Scc + A.aoff[g];
  const int32_t* cols = A.cord + c0;
  const int32_t* nfi = A.nf_idx + f0;
  double z[D];
#pragma unroll
  for (int k = 0; k < D; ++k) z[k] = A.zc[int64_t(g) * D + k];

  for (int col = threadIdx.x; col < n; col += blockDim.x) {
    const int j = cols[col];
    double xj[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xj[k] = A.pts[int64_t(j) * D + k];
    const double wcj = A.w[j] * A.c[j];
    const double bj = A.b[j];
    double k2 = 0.0;
    // near-field kernel rows: b_i G(|x_i - x_j|) w_j c_j
    for (int r = 0; r < nf; ++r) {
      const int i = nfi[r];
      double r2 = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        double t = A.pts[int64_t(i) * D + k] - xj[k];
        r2 += t * t;
      }
      double v = A.b[i] * green_r2<D>(r2) * wcj;
      Y[int64_t(r) * n + col] = v;
      k2 += v * v;
    }
    int roff = nf;
    if (!A.sym) {
      // transposed row block A(c, c^N)^T: b_j G w_i c_i
      for (int r = 0; r < nf; ++r) {
        const int i = nfi[r];
        double r2 = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          double t = A.pts[int64_t(i) * D + k] - xj[k];
          r2 += t * t;
        }
        double v = bj * green_r2<D>(r2) * A.w[i] * A.c[i];
        Y[int64_t(nf + r) * n + col] = v;
        k2 += v * v;
      }
      roff = 2 * nf;
    }
    // proxy rows: G(|x_p - x_j|) w_j c_j  (and b_j G w_j for the row side)
    for (int p = 0; p < P; ++p) {
      double r2 = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        double xp = z[k] + A.R * A.proxy_u[p * D + k];
        double t = xp - xj[k];
        r2 += t * t;
      }
      const double gk = green_r2<D>(r2);
      double v = gk * wcj;
      Y[int64_t(roff + p) * n + col] = v;
      k2 += v * v;
      if (!A.sym) {
        double v2 = bj * gk * A.w[j];
        Y[int64_t(roff + P + p) * n + col] = v2;
        k2 += v2 * v2;
      }
    }
    // A_cc column: a_j delta + b_i K_ij c_j
    for (int r = 0; r < n; ++r) {
      const int i = cols[r];
      double v;
      if (i == j) {
        v = A.a[j] + A.b[j] * A.selfk[j] * A.c[j];
      } else {
        double r2 = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          double t = A.pts[int64_t(i) * D + k] - xj[k];
          r2 += t * t;
        }
        v = A.b[i] * green_r2<D>(r2) * wcj;
      }
      Acc[int64_t(r) * n + col] = v;
      Scc[int64_t(r) * n + col] = 0.0;
    }
    // SCI part: row j of the store holds (j, i) with values (S_ji, S_ij).
    double s2 = 0.0;
    const int64_t e0 = A.srow[j], e1 = A.srow[j + 1];
    for (int64_t e = e0; e < e1; ++e) {
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
          int mid = (lo + hi) >> 1;
          if (nfi[mid] < i) lo = mid + 1; else hi = mid;
        }
        if (lo < nf && nfi[lo] == i) {
          double yk = Y[int64_t(lo) * n + col];
          double yt = yk + sv.y;
          Y[int64_t(lo) * n + col] = yt;
          s2 += sv.y * sv.y;
          if (!A.sym) {
            double yk2 = Y[int64_t(nf + lo) * n + col];
            Y[int64_t(nf + lo) * n + col] = yk2 + sv.x;
            s2 += sv.x * sv.x;
          }
        }
      }
    }
    A.colK2[c0 + col] = k2;
    A.colS2[c0 + col] = s2;
  }
}

void launch_assemble(const AsmArgs& A, int block, hipStream_t s) {
  if (A.ngroups == 0) return;
  if (A.dim == 2)
    hipLaunchKernelGGL(k_assemble<2>, dim3(A.ngroups), dim3(block), 0, s, A);
  else
    hipLaunchKernelGGL(k_assemble<3>, dim3(A.ngroups), dim3(block), 0, s, A);
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
template <int U>
__global__ void k_id(IdArgs A) {
  const int q = blockIdx.x;
  double* M = A.base + A.moff[q];
  const int ld = A.ld[q], m = A.rows[q], n = A.cols[q];
  const double tol = A.tol[q];
  int32_t* perm = A.perm + A.poff[q];
  const int tid = threadIdx.x, B = blockDim.x;
  __shared__ double s_alpha, s_v0, s_beta;
  __shared__ int s_p, s_k;

  double nrm[U];
  int state[U];  // -2 absent, -1 trailing, >= 0 pivot step
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int col = tid + u * B;
    state[u] = col < n ? -1 : -2;
    double s = 0.0;
    if (col < n)
      for (int r = 0; r < m; ++r) {
        double y = M[int64_t(r) * ld + col];
        s += y * y;
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
      double w = v0 * M[int64_t(i) * ld + col];
      for (int r = i + 1; r < m; ++r) w += M[int64_t(r) * ld + p] * M[int64_t(r) * ld + col];
      w *= beta;
      M[int64_t(i) * ld + col] -= w * v0;
      double s = 0.0;
      for (int r = i + 1; r < m; ++r) {
        double y = M[int64_t(r) * ld + col] - w * M[int64_t(r) * ld + p];
        M[int64_t(r) * ld + col] = y;
        s += y * y;
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

void launch_id(const IdArgs& A, int max_cols, hipStream_t s) {
  if (A.nprob == 0) return;
  int block = 64;
  while (block < max_cols && block < 256) block *= 2;
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
    throw Error{HIF_EUNSUPPORTED, "ID problem with more than 4096 columns"};
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
// DOFs (Lemma 2.1):
//   B_sr = A_sr - A_ss T,  B_rs = A_rs - T^T A_ss,
//   B_rr = A_rr - A_rs T - T^T B_sr,
//   LU(B_rr), G = B_rr^{-1} B_rs, E = B_sr B_rr^{-1},
//   new S(s,s) = S_old(s,s) - B_sr G.
// T = diag(T_q) over the split classes, so every product over the skeleton
// index runs only over the class of the redundant column.
// ---------------------------------------------------------------------------
__global__ void k_eliminate(ElimArgs A) {
  const int g = blockIdx.x;
  const int ri = A.grec[g];
  if (ri < 0) return;
  const GroupRec R = A.recs[ri];
  const int r = R.r, k = R.k;
  const int64_t c0 = A.gstart[g];
  const int n = int(A.gstart[g + 1] - c0);
  const int tid = threadIdx.x, B = blockDim.x;
  int32_t* rd = A.iarena + R.idx;
  int32_t* sk = rd + r;
  int32_t* piv = sk + k;
  double* T = A.darena + R.off;
  double* E = T + int64_t(k) * r;
  double* Gm = E + int64_t(k) * r;
  double* LU = Gm + int64_t(r) * k;
  const double* Y = A.Y + A.yoff[g];
  double* Acc = A.Acc + A.aoff[g];
  const double* Scc = A.Scc + A.aoff[g];
  int32_t* rdl = A.loc + c0;
  int32_t* skl = rdl + r;
  int32_t* rlo = A.rlo + c0;
  int32_t* rhi = A.rhi + c0;
  const int32_t* cord = A.cord + c0;

  // 1. skeleton / redundant lists in class order.
  for (int q = A.cls_first[g]; q < A.cls_first[g + 1]; ++q) {
    const int col0 = A.cls_col0[q], nq = A.cls_n[q], kq = A.cls_rank[q];
    const int so = A.cls_skoff[q], ro = A.cls_rdoff[q];
    const int32_t* pq = A.perm + c0 + col0;
    for (int j = tid; j < nq; j += B) {
      const int gl = col0 + pq[j];
      if (j < kq) {
        skl[so + j] = gl;
        sk[so + j] = cord[gl];
      } else {
        const int bb = ro + (j - kq);
        rdl[bb] = gl;
        rd[bb] = cord[gl];
        rlo[bb] = so;
        rhi[bb] = so + kq;
      }
    }
  }
  __syncthreads();
  // 2. dense block-diagonal T (k x r).
  for (int64_t e = tid; e < int64_t(k) * r; e += B) {
    const int a = int(e / r), bb = int(e % r);
    const int lo = rlo[bb];
    T[e] = (a >= lo && a < rhi[bb]) ? Y[int64_t(a - lo) * n + rdl[bb]] : 0.0;
  }
  __syncthreads();
  // 3. B_sr (into E) and B_rs (into G).
  for (int64_t e = tid; e < int64_t(k) * r; e += B) {
    const int a = int(e / r), bb = int(e % r);
    const double* arow = Acc + int64_t(skl[a]) * n;
    double v = arow[rdl[bb]];
    for (int l = rlo[bb]; l < rhi[bb]; ++l) v -= arow[skl[l]] * T[int64_t(l) * r + bb];
    E[e] = v;
  }
  for (int64_t e = tid; e < int64_t(r) * k; e += B) {
    const int bb = int(e / k), a = int(e % k);
    double v = Acc[int64_t(rdl[bb]) * n + skl[a]];
    for (int l = rlo[bb]; l < rhi[bb]; ++l) v -= T[int64_t(l) * r + bb] * Acc[int64_t(skl[l]) * n + skl[a]];
    Gm[e] = v;
  }
  __syncthreads();
  // 4. B_rr (into LU).
  for (int64_t e = tid; e < int64_t(r) * r; e += B) {
    const int bb = int(e / r), ee = int(e % r);
    const double* arow = Acc + int64_t(rdl[bb]) * n;
    double v = arow[rdl[ee]];
    for (int l = rlo[ee]; l < rhi[ee]; ++l) v -= arow[skl[l]] * T[int64_t(l) * r + ee];
    for (int l = rlo[bb]; l < rhi[bb]; ++l) v -= T[int64_t(l) * r + bb] * E[int64_t(l) * r + ee];
    LU[e] = v;
  }
  __syncthreads();
  // 5. LU(B_rr).
  block_lu(LU, r, r, piv, A.status);
  __syncthreads();
  // 6. G = B_rr^{-1} B_rs, one column of G per thread.
  for (int a = tid; a < k; a += B) {
    for (int j = 0; j < r; ++j) {
      const int p = piv[j];
      if (p != j) {
        double t = Gm[int64_t(j) * k + a];
        Gm[int64_t(j) * k + a] = Gm[int64_t(p) * k + a];
        Gm[int64_t(p) * k + a] = t;
      }
    }
    for (int i = 1; i < r; ++i) {
      double v = Gm[int64_t(i) * k + a];
      for (int j = 0; j < i; ++j) v -= LU[int64_t(i) * r + j] * Gm[int64_t(j) * k + a];
      Gm[int64_t(i) * k + a] = v;
    }
    for (int i = r - 1; i >= 0; --i) {
      double v = Gm[int64_t(i) * k + a];
      for (int j = i + 1; j < r; ++j) v -= LU[int64_t(i) * r + j] * Gm[int64_t(j) * k + a];
      Gm[int64_t(i) * k + a] = v / LU[int64_t(i) * r + i];
    }
  }
  __syncthreads();
  // 7. new S block (k x k) = S_old(s,s) - B_sr G, staged in the A_cc scratch.
  double* NS = Acc;
  for (int64_t e = tid; e < int64_t(k) * k; e += B) {
    const int a = int(e / k), a2 = int(e % k);
    double v = Scc[int64_t(skl[a]) * n + skl[a2]];
    const double* er = E + int64_t(a) * r;
    for (int bb = 0; bb < r; ++bb) v -= er[bb] * Gm[int64_t(bb) * k + a2];
    NS[e] = v;
  }
  __syncthreads();
  {
    uint64_t* nk = A.newkey + A.newoff[g];
    double2* nv = A.newval + A.newoff[g];
    for (int64_t e = tid; e < int64_t(k) * k; e += B) {
      const int a = int(e / k), a2 = int(e % k);
      nk[e] = (uint64_t(uint32_t(sk[a])) << 32) | uint32_t(sk[a2]);
      nv[e] = make_double2(NS[e], NS[int64_t(a2) * k + a]);
    }
  }
  // 8. E = B_sr B_rr^{-1}, one row per thread: x P^T L U = b.
  for (int a = tid; a < k; a += B) {
    double* x = E + int64_t(a) * r;
    for (int j = 0; j < r; ++j) {  // y U = b
      double v = x[j];
      for (int i = 0; i < j; ++i) v -= x[i] * LU[int64_t(i) * r + j];
      x[j] = v / LU[int64_t(j) * r + j];
    }
    for (int j = r - 2; j >= 0; --j) {  // z L = y (unit lower)
      double v = x[j];
      for (int i = j + 1; i < r; ++i) v -= x[i] * LU[int64_t(i) * r + j];
      x[j] = v;
    }
    for (int j = r - 1; j >= 0; --j) {  // x = z P
      const int p = piv[j];
      if (p != j) {
        double t = x[j];
        x[j] = x[p];
        x[p] = t;
      }
    }
  }
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
      v = A.b[i] * green_r2<D>(r2) * A.w[j] * A.c[j];
    }
    A.A[e] = v;
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
  hipLaunchKernelGGL(k_top_lu, dim3(1), dim3(1024), 0, s, A);
  HIF_HIP(hipGetLastError());
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
  IdArgs A;
  A.base = mats;
  A.moff = off;
  A.ld = ld.p;
  A.rows = rows;
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
