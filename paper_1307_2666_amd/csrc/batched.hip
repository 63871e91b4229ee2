// Per-panel batched kernels for the coarse sub-levels, where a few large
// problems would leave most compute units idle if each ran in one workgroup:
// the row compression before the ID (blocked Householder QR) and the partial
// LU of the elimination (and of the top block) are split into a panel kernel
// (one workgroup per problem) and a trailing-update kernel (one workgroup per
// 64-column tile per problem) launched once per panel of 16 columns.  The
// updates run on the matrix cores (v_mfma_f64_16x16x4f64) with operands read
// straight from device memory in the instruction's lane layout.
#include <algorithm>
#include <map>
#include <climits>
#include <vector>

#include "batched.h"
#include "gemm.h"
#include "wave.h"

namespace hif {

namespace {

constexpr int kNb = 16;     // panel width
constexpr int kTileN = 64;  // columns per update workgroup

struct AM {
  double v;
  int i;
};
__device__ __forceinline__ AM am_better(AM a, AM b) {
  if (b.v > a.v || (b.v == a.v && b.i < a.i)) return b;
  return a;
}
__device__ __forceinline__ double pick16(const double (&y)[kNb], int j) {
  double r = 0.0;
#pragma unroll
  for (int c = 0; c < kNb; ++c)
    if (c == j) r = y[c];
  return r;
}

// Block-wide argmax (larger value, ties to the lower index) for up to 1024 threads.
// The caller must pass a barrier between two calls (the slots are
// rewritten by the next call).
__device__ AM block_argmax_n(AM x) {
  __shared__ double sv[16];
  __shared__ int si[16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    AM y{__shfl_xor(x.v, o, 64), __shfl_xor(x.i, o, 64)};
    x = am_better(x, y);
  }
  if (lane == 0) { sv[wv] = x.v; si[wv] = x.i; }
  __syncthreads();
  AM r{-1.0, INT_MAX};
  for (int k = 0; k < nw; ++k) r = am_better(r, AM{sv[k], si[k]});
  return r;
}

__device__ AM block_argmax256(AM x) {
  __shared__ double sv[4];
  __shared__ int si[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    AM y{__shfl_xor(x.v, o, 64), __shfl_xor(x.i, o, 64)};
    x = am_better(x, y);
  }
  if (lane == 0) { sv[wv] = x.v; si[wv] = x.i; }
  __syncthreads();
  AM r{-1.0, INT_MAX};
  for (int k = 0; k < 4; ++k) r = am_better(r, AM{sv[k], si[k]});
  __syncthreads();
  return r;
}

constexpr int kQrThreads = 1024;            // trailing-update workgroup
constexpr int kQrWaves = kQrThreads / 64;
constexpr int kQpThreads = 512;             // panel workgroup (register budget of 256 VGPRs)
constexpr int kQpWaves = kQpThreads / 64;

__device__ __forceinline__ double bsumQ(double v, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < kQpWaves; ++w) t += red[w];
  __syncthreads();
  return t;
}

// ---------------------------------------------------------------------------
// Row compression, panel j0 of every problem: Householder vectors of columns
// j0..j0+jb-1 (rows j0..m-1) into V (m x 16, zero above the diagonal), R's
// diagonal into the block, and T of the compact WY form I - V T V^T into Tq.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kQpThreads) void k_qr_panel(QrBatch A, int j0) {
  const int q = blockIdx.x;
  const int m = A.rows[q], n = A.cols[q];
  if (m <= n || j0 >= n) return;
  double* M = A.base + A.moff[q];
  const int ld = A.ld[q];
  double* V = A.scratch + A.soff[q];
  double* Tq = V + int64_t(m) * kNb;
  const int jb = min(kNb, n - j0);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  __shared__ double red[kQpWaves];
  __shared__ double sred[kQpWaves][kNb + 1];
  __shared__ double sbeta[kNb];
  __shared__ double sG[kQpWaves][kNb * kNb];
  for (int r = j0 + tid; r < m; r += kQpThreads)
#pragma unroll
    for (int c = 0; c < kNb; ++c) V[int64_t(r - j0) * kNb + c] = 0.0;
  double s0 = 0.0;
  for (int r = j0 + tid; r < m; r += kQpThreads) {
    const double y = M[int64_t(r) * ld + j0];
    s0 += y * y;
  }
  double ss = bsumQ(s0, red);
  for (int jj = 0; jj < jb; ++jj) {
    const int j = j0 + jj;
    const int nc = jb - jj - 1;
    const double x0 = M[int64_t(j) * ld + j];
    const double nrm = sqrt(ss);
    const double alpha = nrm > 0.0 ? -copysign(nrm, x0) : 0.0;
    const double v0 = x0 - alpha;
    const double vtv = ss - x0 * x0 + v0 * v0;
    const double beta = vtv > 0.0 ? 2.0 / vtv : 0.0;
    double part[kNb];
#pragma unroll
    for (int c = 0; c < kNb; ++c) part[c] = 0.0;
    for (int r0 = j + tid; r0 < m; r0 += 4 * kQpThreads) {
      double vr[4], y[4][kNb];
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const int r = r0 + qq * kQpThreads;
        vr[qq] = 0.0;
        if (r < m) vr[qq] = r == j ? v0 : M[int64_t(r) * ld + j];
#pragma unroll
        for (int c = 0; c < kNb; ++c) y[qq][c] = (r < m && c < nc) ? M[int64_t(r) * ld + j + 1 + c] : 0.0;
      }
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const int r = r0 + qq * kQpThreads;
        if (r < m) V[int64_t(r - j0) * kNb + jj] = vr[qq];
#pragma unroll
        for (int c = 0; c < kNb; ++c) part[c] += vr[qq] * y[qq][c];
      }
    }
#pragma unroll
    for (int c = 0; c < kNb; ++c) {
      if (c >= nc) break;
      const double t = wave_sum(part[c]);
      if (lane == 0) sred[wv][c] = t;
    }
    __syncthreads();
    double wc[kNb];
#pragma unroll
    for (int c = 0; c < kNb; ++c) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kQpWaves; ++w) t += sred[w][c];
      wc[c] = c < nc ? beta * t : 0.0;
    }
    __syncthreads();
    double snext = 0.0;
    for (int r0 = j + tid; r0 < m; r0 += 4 * kQpThreads) {
      double vr[4], y[4][kNb];
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const int r = r0 + qq * kQpThreads;
        vr[qq] = 0.0;
        if (r < m) vr[qq] = r == j ? v0 : M[int64_t(r) * ld + j];
#pragma unroll
        for (int c = 0; c < kNb; ++c) y[qq][c] = (r < m && c < nc) ? M[int64_t(r) * ld + j + 1 + c] : 0.0;
      }
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const int r = r0 + qq * kQpThreads;
#pragma unroll
        for (int c = 0; c < kNb; ++c) y[qq][c] -= wc[c] * vr[qq];
        if (r > j && r < m && nc > 0) snext += y[qq][0] * y[qq][0];
        if (r < m) {
#pragma unroll
          for (int c = 0; c < kNb; ++c)
            if (c < nc) M[int64_t(r) * ld + j + 1 + c] = y[qq][c];
        }
      }
    }
    if (tid == 0) sbeta[jj] = beta;
    ss = bsumQ(snext, red);
    if (tid == 0) M[int64_t(j) * ld + j] = alpha;
  }
  // G = V^T V on the matrix cores: every wave sums its own 4-row slices.
  {
    double4_t acc = {0.0, 0.0, 0.0, 0.0};
    const int mp = m - j0;
    const int li = lane & 15, lk = lane >> 4;
    for (int kb = wv * 4; kb < mp; kb += 4 * kQpWaves) {
      const int r = kb + lk;
      const double a = r < mp ? V[int64_t(r) * kNb + li] : 0.0;
      acc = mfma_f64(a, a, acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) sG[wv][(4 * v + lk) * kNb + li] = acc[v];
  }
  __syncthreads();
  __shared__ double T[kNb][kNb];
  for (int e = tid; e < kNb * kNb; e += kQpThreads) T[e / kNb][e % kNb] = 0.0;
  __syncthreads();
  if (tid == 0) {
    for (int i = 0; i < jb; ++i) {
      T[i][i] = sbeta[i];
      for (int p = 0; p < i; ++p) {
        double t = 0.0;
        for (int l = p; l < i; ++l) {
          const int e = l * kNb + i;
          double gsum = 0.0;
          for (int w = 0; w < kQpWaves; ++w) gsum += sG[w][e];
          t += T[p][l] * gsum;
        }
        T[p][i] = -sbeta[i] * t;
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < kNb * kNb; e += kQpThreads) Tq[e] = T[e / kNb][e % kNb];
}

// Trailing update of one 64-column tile: W = T^T V^T Y_t (split over the
// waves along the rows), then Y_t -= V W.
__global__ __launch_bounds__(kQrThreads) void k_qr_update(QrBatch A, int j0) {
  const int q = blockIdx.y;
  const int m = A.rows[q], n = A.cols[q];
  if (m <= n || j0 >= n) return;
  const int jb = min(kNb, n - j0);
  const int c0 = j0 + jb + blockIdx.x * kTileN;
  if (c0 >= n) return;
  const int nt = min(kTileN, n - c0);
  double* M = A.base + A.moff[q];
  const int ld = A.ld[q];
  const double* V = A.scratch + A.soff[q];
  const double* Tq = V + int64_t(m) * kNb;
  const int mp = m - j0;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  __shared__ double sW[kQrWaves][kNb][kTileN + 1];
  __shared__ double sW2[kNb][kTileN + 1];
  // 1. partial W per wave over rows kb = 4*wv, 4*wv + 16, ...
  double4_t acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = double4_t{0.0, 0.0, 0.0, 0.0};
  for (int kb = wv * 4; kb < mp; kb += 4 * kQrWaves) {
    const int r = kb + lk;
    const bool ok = r < mp;
    const double a = ok ? V[int64_t(r) * kNb + li] : 0.0;
    const double* yr = M + int64_t(j0 + (ok ? r : 0)) * ld + c0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int col = t * 16 + li;
      const double b = (ok && col < nt) ? yr[col] : 0.0;
      acc[t] = mfma_f64(a, b, acc[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) sW[wv][4 * v + lk][t * 16 + li] = acc[t][v];
  __syncthreads();
  // 2. W = T^T (sum of the partials), T upper triangular.
  for (int e = tid; e < kNb * kTileN; e += kQrThreads) {
    const int i = e / kTileN, c = e % kTileN;
    double s = 0.0;
    for (int p = 0; p <= i; ++p) {
      double w = 0.0;
#pragma unroll
      for (int q2 = 0; q2 < kQrWaves; ++q2) w += sW[q2][p][c];
      s += Tq[p * kNb + i] * w;
    }
    sW2[i][c] = s;
  }
  __syncthreads();
  // 3. Y_t -= V W, 16-row tiles spread over the waves.
  for (int rt = wv * 16; rt < mp; rt += 16 * kQrWaves) {
    double4_t d[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) d[t] = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < kNb; ks += 4) {
      const int r = rt + li;
      const double a = r < mp ? V[int64_t(r) * kNb + ks + lk] : 0.0;
#pragma unroll
      for (int t = 0; t < 4; ++t) d[t] = mfma_f64(a, sW2[ks + lk][t * 16 + li], d[t]);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = rt + 4 * v + lk, col = t * 16 + li;
        if (r < mp && col < nt) M[int64_t(j0 + r) * ld + c0 + col] -= d[t][v];
      }
  }
}

__global__ void k_qr_clear_lower(QrBatch A) {
  const int q = blockIdx.y;
  const int m = A.rows[q], n = A.cols[q];
  if (m <= n) return;
  double* M = A.base + A.moff[q];
  const int ld = A.ld[q];
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < int64_t(n) * n;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int r = int(e / n), c = int(e % n);
    if (c < r) M[int64_t(r) * ld + c] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Communication-avoiding row compression (TSQR panels).  Panel j0 (columns
// j0..j0+jb-1, rows j0..m-1) is split into nck balanced chunks of at most
// kTsqrRows rows.  Each chunk is factored by its own workgroup (one row per
// thread, in registers); with nck > 1 the chunk R factors are stacked and the
// stack is factored again.  The trailing columns are then updated chunk by
// chunk with the chunk's compact WY form, and the chunk top rows with the
// stack's.  The final R rows of the panel land in rows j0..j0+jb-1; all that
// later steps read is R (the orthogonal factor is never formed).
// ---------------------------------------------------------------------------
constexpr int kTb = kTsqrNb;
static_assert(kTb == kRs, "the panel width is the reduce-scatter width");

struct PanelGeom {
  int mp, jb, nck;
};
__device__ __forceinline__ PanelGeom panel_geom(int m, int n, int j0, int cr) {
  PanelGeom g;
  g.mp = m - j0;
  g.jb = min(kTb, n - j0);
  g.nck = (g.mp + cr - 1) / cr;
  return g;
}
__device__ __forceinline__ int chunk_lo(int c, int mp, int nck) { return (c * mp) / nck; }

__device__ __forceinline__ double pick(const double (&y)[kTb], int j) {
  double r = 0.0;
#pragma unroll
  for (int c = 0; c < kTb; ++c)
    if (c == j) r = y[c];
  return r;
}


// Householder QR of a block of at most RPT * blockDim.x rows and jb <= kTb
// columns held RPT rows per thread (thread t: rows t + u * blockDim.x; rows
// past the block are zero).  Per column one reduction round gives, over the
// rows below the diagonal, the squared norm and the products with the later
// columns; the first kTb threads then turn them into the reflector (alpha,
// v0, beta) and the update coefficient of every column, which all threads
// read back from LDS.  On return rows < jb hold R (upper part) and rows > jj
// hold the Householder vector of column jj below the diagonal; v0 (its
// diagonal entry) and beta = 2 / v^T v are in sv0 / sbeta.
// LDS: sred [2][NW][kTb], srow [2][kTb], scf [2][kTb + 2].
template <int NW, int RPT>
__device__ void rowblock_qr(double (&y)[RPT][kTb], int jb, double* sred, double* srow, double* scf, double* sv0,
                            double* sbeta, double* sG) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int t0 = threadIdx.x, B = blockDim.x;
  if (t0 >= jb && t0 < kTb) {  // columns past a partial panel: no reflector
    sv0[t0] = 0.0;
    sbeta[t0] = 0.0;
  }
  for (int jj = 0; jj < jb; ++jj) {
    const int b = jj & 1;  // double-buffered: one barrier pair per column
    double* red = sred + b * NW * kTb;
    double* row = srow + b * kTb;
    double* cf = scf + b * (kTb + 2);
    double yj[RPT];
#pragma unroll
    for (int u = 0; u < RPT; ++u) yj[u] = pick(y[u], jj);
    if (t0 == jj) {  // jj < kTb <= B: row jj is slot 0 of thread jj
#pragma unroll
      for (int c = 0; c < kTb; ++c) row[c] = y[0][c];
    }
    double p[kTb];
    {
      double e[RPT];
#pragma unroll
      for (int u = 0; u < RPT; ++u) e[u] = t0 + u * B > jj ? yj[u] : 0.0;
#pragma unroll
      for (int c = 0; c < kTb; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < RPT; ++u) acc += e[u] * y[u][c];
        p[c] = acc;
      }
    }
    const double w = wave_rs32(p);
    if ((lane & 1) == 0) red[wv * kTb + (lane >> 1)] = w;
    __syncthreads();
    if (t0 < kTb) {
      const int c = t0;
      double sc = 0.0, sj = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < NW; ++w2) {
        sc += red[w2 * kTb + c];
        sj += red[w2 * kTb + jj];
      }
      const double x0 = row[jj];
      const double ss = sj + x0 * x0;
      const double nrm = sqrt(ss);
      const double alpha = nrm > 0.0 ? -copysign(nrm, x0) : 0.0;
      const double v0 = x0 - alpha;
      const double vtv = sj + v0 * v0;
      const double beta = vtv > 0.0 ? 2.0 / vtv : 0.0;
      cf[c] = (c > jj && c < jb) ? beta * (v0 * row[c] + sc) : 0.0;
      // column jj of G = V^T V above the diagonal: rows > jj of column c < jj
      // hold its reflector, row jj its entry V(jj, c)
      if (c < jj) sG[c * (kTb + 1) + jj] = sc + row[c] * v0;
      if (c == 0) {
        cf[kTb] = alpha;
        cf[kTb + 1] = v0;
        sv0[jj] = v0;
        sbeta[jj] = beta;
      }
    }
    __syncthreads();
    const double alpha = cf[kTb], v0 = cf[kTb + 1];
    double coef[kTb];
#pragma unroll
    for (int c = 0; c < kTb; ++c) coef[c] = cf[c];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int t = t0 + u * B;
      if (t >= jj) {
        const double vt = t == jj ? v0 : yj[u];
#pragma unroll
        for (int c = 0; c < kTb; ++c) y[u][c] -= coef[c] * vt;
        if (u == 0 && t == jj) {  // row jj < kTb lives in slot 0
#pragma unroll
          for (int c = 0; c < kTb; ++c)
            if (c == jj) y[u][c] = alpha;
        }
      }
    }
  }
  __syncthreads();
}

// Row t of V (rows x kTb, zero above the diagonal and past column jb).
__device__ __forceinline__ void store_vrow(const double (&y)[kTb], int t, int jb, const double* sv0, double* Vrow) {
#pragma unroll
  for (int c = 0; c < kTb; ++c) Vrow[c] = (c < jb && t > c) ? y[c] : ((c < jb && t == c) ? sv0[c] : 0.0);
}

// T of the compact WY form I - V T V^T (T upper triangular) from beta and the
// upper part of G = V^T V that rowblock_qr left in sG.
__device__ void build_T(const double* sbeta, const double* sG, double* Tout) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // T(p, i) = -beta_i sum_{l < i} T(p, l) G(l, i) for p < i, T(i, i) = beta_i:
  // one wave, lane p keeps row p of T in registers (no barriers)
  if (wv == 0) {
    const int p = lane & (kTb - 1);
    double trow[kTb];
#pragma unroll
    for (int l = 0; l < kTb; ++l) trow[l] = 0.0;
#pragma unroll
    for (int i = 0; i < kTb; ++i) {
      const double b = sbeta[i];
      // no branch on b, so that the G reads can be issued ahead of the
      // chain; for b == 0 (no reflector, G unset) acc is discarded below
      double acc = 0.0;
#pragma unroll
      for (int l = 0; l < i; ++l) acc += trow[l] * sG[l * (kTb + 1) + i];
      trow[i] = p == i ? b : ((p < i && b != 0.0) ? -b * acc : 0.0);
    }
    if (lane < kTb)
#pragma unroll
      for (int l = 0; l < kTb; ++l) Tout[p * kTb + l] = trow[l];
  }
}

// K1: QR of one chunk of the panel (chunks of at most cr = BS * RPT rows).
template <int BS, int RPT>
__global__ __launch_bounds__(BS) void k_tsqr_chunk(QrBatch A, int j0, int cr, int half) {
  const int q = blockIdx.y, c = blockIdx.x;
  const int m = A.rows[q], n = A.cols[q];
  if (m <= n || j0 >= n) return;
  const PanelGeom g = panel_geom(m, n, j0, cr);
  if (c >= g.nck) return;
  const int lo = chunk_lo(c, g.mp, g.nck), rows = chunk_lo(c + 1, g.mp, g.nck) - lo;
  double* M = A.base + A.moff[q];
  const int ld = A.ld[q];
  const TsqrLayout L = tsqr_layout(m);
  double* S0 = A.scratch + A.soff[q] + half * L.total;
  const int t0 = threadIdx.x;
  __shared__ double sred[2 * (BS / 64) * kTb], srow[2 * kTb], scf[2 * (kTb + 2)], sv0[kTb], sbeta[kTb];
  __shared__ double sG[kTb * (kTb + 1)];
  double y[RPT][kTb];
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int t = t0 + u * BS;
    const double* src = M + int64_t(j0 + lo + (t < rows ? t : 0)) * ld + j0;
#pragma unroll
    for (int cc = 0; cc < kTb; ++cc) y[u][cc] = (t < rows && cc < g.jb) ? src[cc] : 0.0;
  }
  rowblock_qr<BS / 64, RPT>(y, g.jb, sred, srow, scf, sv0, sbeta, sG);
  double* V = S0 + L.V + int64_t(lo) * kTb;
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int t = t0 + u * BS;
    if (t < rows) store_vrow(y[u], t, g.jb, sv0, V + int64_t(t) * kTb);
  }
  if (g.nck == 1) {
    if (t0 < g.jb) {
      double* dst = M + int64_t(j0 + t0) * ld + j0;
#pragma unroll
      for (int cc = 0; cc < kTb; ++cc)
        if (cc < g.jb) dst[cc] = cc >= t0 ? y[0][cc] : 0.0;
    }
  } else if (t0 < kTb) {
    double* dst = S0 + L.S + int64_t(c * kTb + t0) * kTb;
#pragma unroll
    for (int cc = 0; cc < kTb; ++cc) dst[cc] = (t0 < g.jb && cc >= t0 && cc < g.jb) ? y[0][cc] : 0.0;
  }
  __syncthreads();
  build_T(sbeta, sG, S0 + L.Tc + int64_t(c) * kTb * kTb);
}

// K2: QR of the stacked chunk R factors (nck > 1); writes the panel's R.
template <int BS, int RPT>
__global__ __launch_bounds__(BS) void k_tsqr_stack(QrBatch A, int j0, int cr, int half) {
  const int q = blockIdx.x;
  const int m = A.rows[q], n = A.cols[q];
  if (m <= n || j0 >= n) return;
  const PanelGeom g = panel_geom(m, n, j0, cr);
  if (g.nck < 2) return;
  const int srows = g.nck * kTb;
  double* M = A.base + A.moff[q];
  const int ld = A.ld[q];
  const TsqrLayout L = tsqr_layout(m);
  double* S0 = A.scratch + A.soff[q] + half * L.total;
  const int t = threadIdx.x;
  __shared__ double sred[2 * (BS / 64) * kTb], srow[2 * kTb], scf[2 * (kTb + 2)], sv0[kTb], sbeta[kTb];
  __shared__ double sG[kTb * (kTb + 1)];
  double y[RPT][kTb];
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int tu = t + u * BS;
    const double* src = S0 + L.S + int64_t(tu < srows ? tu : 0) * kTb;
#pragma unroll
    for (int cc = 0; cc < kTb; ++cc) y[u][cc] = tu < srows ? src[cc] : 0.0;
  }
  rowblock_qr<BS / 64, RPT>(y, g.jb, sred, srow, scf, sv0, sbeta, sG);
  double* V = S0 + L.Vs;
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int tu = t + u * BS;
    if (tu < srows) store_vrow(y[u], tu, g.jb, sv0, V + int64_t(tu) * kTb);
  }
  if (t < g.jb) {
    double* dst = M + int64_t(j0 + t) * ld + j0;
#pragma unroll
    for (int cc = 0; cc < kTb; ++cc)
      if (cc < g.jb) dst[cc] = cc >= t ? y[0][cc] : 0.0;
  }
  __syncthreads();
  build_T(sbeta, sG, S0 + L.Ts);
}

// Y <- (I - V T V^T)^T Y for one 64-column tile: P = V^T Y, W = T^T P,
// Y -= V W.  rowp(r) gives the address of row r of the tile.  256 threads;
// wave w owns columns 16w..16w+15 and needs nothing from the other waves:
// in the 16x16x4 FP64 MFMA layout, element v of an accumulator tile holds
// rows 4v + (lane / 16) of column lane % 16, which is exactly the B operand
// of K-step v, so P feeds W = T^T P and W feeds Y -= V W from registers.
template <class RowP>
__device__ void apply_wy_tile(const double* V, int rows, const double* Tm, RowP rowp, int nt) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ct = wv * 16;
  const bool colok = ct + li < nt;
  // 1. P (kTb x 16): rows 0-15 in p0, 16-31 in p1, from one read of Y
  double4_t p0 = {0.0, 0.0, 0.0, 0.0}, p1 = {0.0, 0.0, 0.0, 0.0};
  for (int kb = 0; kb < rows; kb += 32) {  // 8 steps of 4 rows, loads issued first
    double a0[8], a1[8], b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int r = kb + 4 * u + lk;
      const bool ok = r < rows;
      a0[u] = ok ? V[int64_t(r) * kTb + li] : 0.0;
      a1[u] = ok ? V[int64_t(r) * kTb + 16 + li] : 0.0;
      b[u] = (ok && colok) ? rowp(r)[ct + li] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      p0 = mfma_f64(a0[u], b[u], p0);
      p1 = mfma_f64(a1[u], b[u], p1);
    }
  }
  // 2. W = T^T P (T upper triangular, zero below the diagonal): A(i, k) = T(k, i)
  double4_t w0 = {0.0, 0.0, 0.0, 0.0}, w1 = {0.0, 0.0, 0.0, 0.0};
  {
    double t0[8], t1[8];
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) {
      t0[s2] = Tm[(4 * s2 + lk) * kTb + li];
      t1[s2] = Tm[(4 * s2 + lk) * kTb + 16 + li];
    }
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) {
      const double bp = s2 < 4 ? p0[s2 & 3] : p1[s2 & 3];
      w0 = mfma_f64(t0[s2], bp, w0);
      w1 = mfma_f64(t1[s2], bp, w1);
    }
  }
  // 3. Y -= V W over 16-row tiles
  for (int rt = 0; rt < rows; rt += 16) {
    double a[8], y[4];
    const int ra = rt + li;
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) a[s2] = ra < rows ? V[int64_t(ra) * kTb + 4 * s2 + lk] : 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = rt + 4 * v + lk;
      y[v] = (r < rows && colok) ? rowp(r)[ct + li] : 0.0;
    }
    double4_t d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) d = mfma_f64(a[s2], s2 < 4 ? w0[s2 & 3] : w1[s2 & 3], d);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = rt + 4 * v + lk;
      if (r < rows && colok) rowp(r)[ct + li] = y[v] - d[v];
    }
  }
}

// The same update for chunks of at most 256 rows with the wave's 256 x 16
// slice of Y held in registers from the first product to the write-back, so
// that Y is read once and written once (element v of row tile t is row
// 16t + 4v + lane / 16, column lane % 16: the B operand of K-step 4t + v).
__device__ __forceinline__ void apply_wy_tile_reg(const double* V, int rows, const double* Tm, double* Y0, int64_t ld, int nt) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ct = wv * 16;
  const bool colok = ct + li < nt;
  double yv[16][4];
#pragma unroll
  for (int t = 0; t < 16; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * t + 4 * v + lk;
      yv[t][v] = (r < rows && colok) ? Y0[int64_t(r) * ld + ct + li] : 0.0;
    }
  // 1. P = V^T Y (rows past the chunk are zero in yv; V rows there are not read)
  double4_t p0 = {0.0, 0.0, 0.0, 0.0}, p1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    if (16 * t >= rows) break;
    double a0[4], a1[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * t + 4 * v + lk;
      a0[v] = r < rows ? V[int64_t(r) * kTb + li] : 0.0;
      a1[v] = r < rows ? V[int64_t(r) * kTb + 16 + li] : 0.0;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      p0 = mfma_f64(a0[v], yv[t][v], p0);
      p1 = mfma_f64(a1[v], yv[t][v], p1);
    }
  }
  // 2. W = T^T P
  double4_t w0 = {0.0, 0.0, 0.0, 0.0}, w1 = {0.0, 0.0, 0.0, 0.0};
  {
    double t0[8], t1[8];
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) {
      t0[s2] = Tm[(4 * s2 + lk) * kTb + li];
      t1[s2] = Tm[(4 * s2 + lk) * kTb + 16 + li];
    }
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) {
      const double bp = s2 < 4 ? p0[s2 & 3] : p1[s2 & 3];
      w0 = mfma_f64(t0[s2], bp, w0);
      w1 = mfma_f64(t1[s2], bp, w1);
    }
  }
  // 3. Y -= V W, written back
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    if (16 * t >= rows) break;
    double a[8];
    const int ra = 16 * t + li;
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) a[s2] = ra < rows ? V[int64_t(ra) * kTb + 4 * s2 + lk] : 0.0;
    double4_t d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) d = mfma_f64(a[s2], s2 < 4 ? w0[s2 & 3] : w1[s2 & 3], d);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * t + 4 * v + lk;
      if (r < rows && colok) Y0[int64_t(r) * ld + ct + li] = yv[t][v] - d[v];
    }
  }
}

// The same update with the chunk's V and T staged in LDS first (one coalesced
// pass per workgroup), so that the fragments the matrix cores consume come
// from LDS rather than from scattered global loads inside the product loops.
// sV holds V with row stride kVs = kTb + 1 doubles: a Y-phase fragment reads
// 16 rows at one column offset, which then fall on different banks.
constexpr int kVs = kTb + 1;
constexpr size_t kApplyLds = (size_t(kTsqrRows) * kVs + kTb * kTb) * sizeof(double);
__device__ __forceinline__ void apply_wy_tile_lds(const double* sV, int rows, const double* sT, double* Y0, int64_t ld, int nt) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ct = wv * 16;
  const bool colok = ct + li < nt;
  double yv[16][4];
#pragma unroll
  for (int t = 0; t < 16; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * t + 4 * v + lk;
      yv[t][v] = (r < rows && colok) ? Y0[int64_t(r) * ld + ct + li] : 0.0;
    }
  // 1. P = V^T Y.  The fragments of row tile t + 1 are read while tile t is
  // multiplied (one tile ahead, no further: the scheduling barrier keeps the
  // compiler from hoisting every tile's reads and spilling).
  double4_t p0 = {0.0, 0.0, 0.0, 0.0}, p1 = {0.0, 0.0, 0.0, 0.0};
  double a0[4], a1[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = 4 * v + lk;
    a0[v] = r < rows ? sV[r * kVs + li] : 0.0;
    a1[v] = r < rows ? sV[r * kVs + 16 + li] : 0.0;
  }
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    if (16 * t < rows) {  // guarded, not broken out of: the loop must unroll fully
    double b0[4], b1[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * (t + 1) + 4 * v + lk;
      b0[v] = (t < 15 && r < rows) ? sV[r * kVs + li] : 0.0;
      b1[v] = (t < 15 && r < rows) ? sV[r * kVs + 16 + li] : 0.0;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      p0 = mfma_f64(a0[v], yv[t][v], p0);
      p1 = mfma_f64(a1[v], yv[t][v], p1);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      a0[v] = b0[v];
      a1[v] = b1[v];
    }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  // 2. W = T^T P
  double4_t w0 = {0.0, 0.0, 0.0, 0.0}, w1 = {0.0, 0.0, 0.0, 0.0};
  {
    double t0[8], t1[8];
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) {
      t0[s2] = sT[(4 * s2 + lk) * kTb + li];
      t1[s2] = sT[(4 * s2 + lk) * kTb + 16 + li];
    }
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) {
      const double bp = s2 < 4 ? p0[s2 & 3] : p1[s2 & 3];
      w0 = mfma_f64(t0[s2], bp, w0);
      w1 = mfma_f64(t1[s2], bp, w1);
    }
  }
  // 3. Y -= V W, written back; fragments one row tile ahead as in 1.
  double a[8];
#pragma unroll
  for (int s2 = 0; s2 < 8; ++s2) a[s2] = li < rows ? sV[li * kVs + 4 * s2 + lk] : 0.0;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    if (16 * t < rows) {
    double b[8];
    const int rb = 16 * (t + 1) + li;
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) b[s2] = (t < 15 && rb < rows) ? sV[rb * kVs + 4 * s2 + lk] : 0.0;
    double4_t d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) d = mfma_f64(a[s2], s2 < 4 ? w0[s2 & 3] : w1[s2 & 3], d);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * t + 4 * v + lk;
      if (r < rows && colok) Y0[int64_t(r) * ld + ct + li] = yv[t][v] - d[v];
    }
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) a[s2] = b[s2];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// The same update with the chunk's rows split between two waves per 16
// columns (wave w: columns 16 (w % CG), rows 128 (w / CG) .. + 127), so that
// each wave holds half the slice of Y and more waves fit per SIMD; the two
// halves add their partial products V^T Y through LDS before both form W.
template <int CG>
__device__ __forceinline__ void apply_wy_tile_split(const double* V, int rows, const double* Tm, double* Y0,
                                                    int64_t ld, int nt, double* sP) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int cg = wv % CG, hf = wv / CG;
  const int li = lane & 15, lk = lane >> 4;
  const int ct = cg * 16, r0 = hf * 128;
  const bool colok = ct + li < nt;
  double yv[8][4];
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = r0 + 16 * t + 4 * v + lk;
      yv[t][v] = (r < rows && colok) ? Y0[int64_t(r) * ld + ct + li] : 0.0;
    }
  double4_t p0 = {0.0, 0.0, 0.0, 0.0}, p1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    if (r0 + 16 * t < rows) {
      double a0[4], a1[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + 16 * t + 4 * v + lk;
        a0[v] = r < rows ? V[int64_t(r) * kTb + li] : 0.0;
        a1[v] = r < rows ? V[int64_t(r) * kTb + 16 + li] : 0.0;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        p0 = mfma_f64(a0[v], yv[t][v], p0);
        p1 = mfma_f64(a1[v], yv[t][v], p1);
      }
    }
  }
  // sP[cg][hf][8][64]: each lane's 8 accumulator entries, by lane
  double* mine = sP + (cg * 2 + hf) * 8 * 64;
  const double* other = sP + (cg * 2 + (1 - hf)) * 8 * 64;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    mine[e * 64 + lane] = p0[e];
    mine[(4 + e) * 64 + lane] = p1[e];
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    p0[e] += other[e * 64 + lane];
    p1[e] += other[(4 + e) * 64 + lane];
  }
  double4_t w0 = {0.0, 0.0, 0.0, 0.0}, w1 = {0.0, 0.0, 0.0, 0.0};
  {
    double t0[8], t1[8];
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) {
      t0[s2] = Tm[(4 * s2 + lk) * kTb + li];
      t1[s2] = Tm[(4 * s2 + lk) * kTb + 16 + li];
    }
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) {
      const double bp = s2 < 4 ? p0[s2 & 3] : p1[s2 & 3];
      w0 = mfma_f64(t0[s2], bp, w0);
      w1 = mfma_f64(t1[s2], bp, w1);
    }
  }
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    if (r0 + 16 * t < rows) {
      double a[8];
      const int ra = r0 + 16 * t + li;
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2) a[s2] = ra < rows ? V[int64_t(ra) * kTb + 4 * s2 + lk] : 0.0;
      double4_t d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2) d = mfma_f64(a[s2], s2 < 4 ? w0[s2 & 3] : w1[s2 & 3], d);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + 16 * t + 4 * v + lk;
        if (r < rows && colok) Y0[int64_t(r) * ld + ct + li] = yv[t][v] - d[v];
      }
    }
  }
}

// K3 for chunks of at most 256 rows, rows split over two waves per 16 columns
// (CG groups of 16 columns per workgroup, 2 CG waves).
template <int CG>
__global__ __launch_bounds__(128 * CG) void k_tsqr_apply_chunk_split(QrBatch A, int j0, int cr, int half, int cbeg,
                                                                    int cend) {
  const int q = blockIdx.z, c = blockIdx.y;
  const int m = A.rows[q], n = A.cols[q];
  if (m <= n || j0 >= n) return;
  const PanelGeom g = panel_geom(m, n, j0, cr);
  if (c >= g.nck) return;
  const int c0 = cbeg + blockIdx.x * 16 * CG, ce = min(n, cend);
  if (c0 >= ce) return;
  const int nt = min(16 * CG, ce - c0);
  const int lo = chunk_lo(c, g.mp, g.nck), rows = chunk_lo(c + 1, g.mp, g.nck) - lo;
  double* M = A.base + A.moff[q];
  const int ld = A.ld[q];
  const TsqrLayout L = tsqr_layout(m);
  const double* S0 = A.scratch + A.soff[q] + half * L.total;
  __shared__ double sP[CG * 2 * 8 * 64];
  apply_wy_tile_split<CG>(S0 + L.V + int64_t(lo) * kTb, rows, S0 + L.Tc + int64_t(c) * kTb * kTb,
                          M + int64_t(j0 + lo) * ld + c0, ld, nt, sP);
}

// K3 for chunks of at most 256 rows, V and T in LDS (kApplyLds bytes of
// dynamic LDS), NW waves of 16 columns each: workgroup (x, chunk, problem)
// updates columns cbeg + 16 NW x .. + 16 NW - 1.
template <int NW>
__global__ __launch_bounds__(64 * NW) void k_tsqr_apply_chunk_lds(QrBatch A, int j0, int cr, int half, int cbeg,
                                                                  int cend) {
  const int q = blockIdx.z, c = blockIdx.y;
  const int m = A.rows[q], n = A.cols[q];
  if (m <= n || j0 >= n) return;
  const PanelGeom g = panel_geom(m, n, j0, cr);
  if (c >= g.nck) return;
  const int c0 = cbeg + blockIdx.x * 16 * NW, ce = min(n, cend);
  if (c0 >= ce) return;
  const int nt = min(16 * NW, ce - c0);
  const int lo = chunk_lo(c, g.mp, g.nck), rows = chunk_lo(c + 1, g.mp, g.nck) - lo;
  double* M = A.base + A.moff[q];
  const int ld = A.ld[q];
  const TsqrLayout L = tsqr_layout(m);
  const double* S0 = A.scratch + A.soff[q] + half * L.total;
  extern __shared__ double smem[];
  double* sV = smem;
  double* sT = smem + kTsqrRows * kVs;
  const double* V = S0 + L.V + int64_t(lo) * kTb;
  const double* Tm = S0 + L.Tc + int64_t(c) * kTb * kTb;
  for (int e = threadIdx.x; e < rows * kTb; e += 64 * NW) sV[(e / kTb) * kVs + e % kTb] = V[e];
  for (int e = threadIdx.x; e < kTb * kTb; e += 64 * NW) sT[e] = Tm[e];
  __syncthreads();
  apply_wy_tile_lds(sV, rows, sT, M + int64_t(j0 + lo) * ld + c0, ld, nt);
}

// K3: trailing update of chunk blockIdx.y, column tile blockIdx.x.
__global__ __launch_bounds__(256) void k_tsqr_apply_chunk(QrBatch A, int j0, int cr, int half, int cbeg, int cend) {
  const int q = blockIdx.z, c = blockIdx.y;
  const int m = A.rows[q], n = A.cols[q];
  if (m <= n || j0 >= n) return;
  const PanelGeom g = panel_geom(m, n, j0, cr);
  if (c >= g.nck) return;
  const int c0 = cbeg + blockIdx.x * 64, ce = min(n, cend);
  if (c0 >= ce) return;
  const int nt = min(64, ce - c0);
  const int lo = chunk_lo(c, g.mp, g.nck), rows = chunk_lo(c + 1, g.mp, g.nck) - lo;
  double* M = A.base + A.moff[q];
  const int ld = A.ld[q];
  const TsqrLayout L = tsqr_layout(m);
  const double* S0 = A.scratch + A.soff[q] + half * L.total;
  double* Y0 = M + int64_t(j0 + lo) * ld + c0;
  apply_wy_tile(S0 + L.V + int64_t(lo) * kTb, rows, S0 + L.Tc + int64_t(c) * kTb * kTb,
                [=](int r) { return Y0 + int64_t(r) * ld; }, nt);
}

// K3 for chunks of at most 256 rows, Y held in registers; NW waves of 16
// columns each.
template <int NW>
__global__ __launch_bounds__(64 * NW, 8 / NW) void k_tsqr_apply_chunk_reg(QrBatch A, int j0, int cr, int half, int cbeg,
                                                                          int cend) {
  const int q = blockIdx.z, c = blockIdx.y;
  const int m = A.rows[q], n = A.cols[q];
  if (m <= n || j0 >= n) return;
  const PanelGeom g = panel_geom(m, n, j0, cr);
  if (c >= g.nck) return;
  const int c0 = cbeg + blockIdx.x * 16 * NW, ce = min(n, cend);
  if (c0 >= ce) return;
  const int nt = min(16 * NW, ce - c0);
  const int lo = chunk_lo(c, g.mp, g.nck), rows = chunk_lo(c + 1, g.mp, g.nck) - lo;
  double* M = A.base + A.moff[q];
  const int ld = A.ld[q];
  const TsqrLayout L = tsqr_layout(m);
  const double* S0 = A.scratch + A.soff[q] + half * L.total;
  apply_wy_tile_reg(S0 + L.V + int64_t(lo) * kTb, rows, S0 + L.Tc + int64_t(c) * kTb * kTb,
                    M + int64_t(j0 + lo) * ld + c0, ld, nt);
}


// The stack update with the rows split between RG waves per 16 columns
// (wave w: columns 16 (w % CG), row blocks of 32 taken round-robin by the RG
// waves w / CG): each wave forms a partial V^T Y over its rows, the RG
// partials are added through LDS, and every wave then forms W and updates its
// own rows.  rowp(r) gives the address of row r of the tile.
template <int CG, int RG, class RowP>
__device__ __forceinline__ void apply_wy_tile_rg(const double* V, int rows, const double* Tm, RowP rowp, int nt,
                                                 double* sP) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int cg = wv % CG, rg = wv / CG;
  const int li = lane & 15, lk = lane >> 4;
  const int ct = cg * 16;
  const bool colok = ct + li < nt;
  double4_t p0 = {0.0, 0.0, 0.0, 0.0}, p1 = {0.0, 0.0, 0.0, 0.0};
  for (int kb = 32 * rg; kb < rows; kb += 32 * RG) {
    double a0[8], a1[8], b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int r = kb + 4 * u + lk;
      const bool ok = r < rows;
      a0[u] = ok ? V[int64_t(r) * kTb + li] : 0.0;
      a1[u] = ok ? V[int64_t(r) * kTb + 16 + li] : 0.0;
      b[u] = (ok && colok) ? rowp(r)[ct + li] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      p0 = mfma_f64(a0[u], b[u], p0);
      p1 = mfma_f64(a1[u], b[u], p1);
    }
  }
  double* mine = sP + (cg * RG + rg) * 8 * 64;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    mine[e * 64 + lane] = p0[e];
    mine[(4 + e) * 64 + lane] = p1[e];
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      s0 += sP[(cg * RG + g) * 8 * 64 + e * 64 + lane];
      s1 += sP[(cg * RG + g) * 8 * 64 + (4 + e) * 64 + lane];
    }
    p0[e] = s0;
    p1[e] = s1;
  }
  double4_t w0 = {0.0, 0.0, 0.0, 0.0}, w1 = {0.0, 0.0, 0.0, 0.0};
  {
    double t0[8], t1[8];
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) {
      t0[s2] = Tm[(4 * s2 + lk) * kTb + li];
      t1[s2] = Tm[(4 * s2 + lk) * kTb + 16 + li];
    }
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) {
      const double bp = s2 < 4 ? p0[s2 & 3] : p1[s2 & 3];
      w0 = mfma_f64(t0[s2], bp, w0);
      w1 = mfma_f64(t1[s2], bp, w1);
    }
  }
  for (int rt = 16 * rg; rt < rows; rt += 16 * RG) {
    double a[8], y[4];
    const int ra = rt + li;
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) a[s2] = ra < rows ? V[int64_t(ra) * kTb + 4 * s2 + lk] : 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = rt + 4 * v + lk;
      y[v] = (r < rows && colok) ? rowp(r)[ct + li] : 0.0;
    }
    double4_t d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) d = mfma_f64(a[s2], s2 < 4 ? w0[s2 & 3] : w1[s2 & 3], d);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = rt + 4 * v + lk;
      if (r < rows && colok) rowp(r)[ct + li] = y[v] - d[v];
    }
  }
}

// K4 with the rows split between RG waves: the stack's WY form applied to the
// chunk top rows of 16 CG columns per workgroup (CG RG waves).
template <int CG, int RG>
__global__ __launch_bounds__(64 * CG * RG) void k_tsqr_apply_stack_rg(QrBatch A, int j0, int cr, int half, int cbeg,
                                                                     int cend) {
  const int q = blockIdx.y;
  const int m = A.rows[q], n = A.cols[q];
  if (m <= n || j0 >= n) return;
  const PanelGeom g = panel_geom(m, n, j0, cr);
  if (g.nck < 2) return;
  const int c0 = cbeg + blockIdx.x * 16 * CG, ce = min(n, cend);
  if (c0 >= ce) return;
  const int nt = min(16 * CG, ce - c0);
  double* M = A.base + A.moff[q];
  const int ld = A.ld[q];
  const TsqrLayout L = tsqr_layout(m);
  const double* S0 = A.scratch + A.soff[q] + half * L.total;
  const int mp = g.mp, nck = g.nck;
  double* Mc = M + int64_t(j0) * ld + c0;
  __shared__ double sP[CG * RG * 8 * 64];
  apply_wy_tile_rg<CG, RG>(S0 + L.Vs, nck * kTb, S0 + L.Ts,
                           [=](int r) { return Mc + int64_t(chunk_lo(r / kTb, mp, nck) + r % kTb) * ld; }, nt, sP);
}

// ---------------------------------------------------------------------------
// Partial LU (Lemma 2.1) of the n x n problems over their first r columns,
// pivoting among rows < r: panel j0 = columns j0..j0+jb-1 with row swaps over
// whole rows, then U12 = L11^{-1} A12 for the panel rows.
// ---------------------------------------------------------------------------
// Register-resident panel for panels of at most kLpRows rows (rows j0..n-1):
// thread t holds rows j0 + t and j0 + t + kLpThreads of the kNb panel
// columns for all kNb elimination steps; the pivot row is exchanged and
// broadcast through LDS.  The row interchanges are then applied in order to
// the columns outside the panel (one thread per column) and U12 is formed.
constexpr int kLpRows = 2048;  // rows of the largest register panel (1024 threads)

template <int kLpThreads>
__global__ __launch_bounds__(kLpThreads) void k_lu_panel_reg(LuBatch A, int j0) {
  const int q = blockIdx.x;
  const int n = A.n[q], r = A.r[q];
  if (j0 >= r) return;
  double* M = A.base + A.moff[q];
  int32_t* piv = A.piv + A.poff[q];
  const int jb = min(kNb, r - j0);
  const int tid = threadIdx.x;
  __shared__ double sA[kNb], sB[kNb];
  __shared__ int spiv[kNb];
  double y[2][kNb];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int R = j0 + tid + u * kLpThreads;
    const double* src = M + int64_t(R < n ? R : j0) * n + j0;
#pragma unroll
    for (int c = 0; c < kNb; ++c) y[u][c] = (R < n && c < jb) ? src[c] : 0.0;
  }
  for (int jj = 0; jj < jb; ++jj) {
    const int j = j0 + jj;
    AM loc{-1.0, INT_MAX};
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int R = j0 + tid + u * kLpThreads;
      if (R >= j && R < r) loc = am_better(loc, AM{fabs(pick16(y[u], jj)), R});
    }
    const AM best = block_argmax_n(loc);
    if (!(best.v > 0.0)) {
      if (tid == 0) atomicOr(A.status, 1);
      return;
    }
    const int p = best.i;
    // rows j (slot 0 of thread jj) and p trade places; everyone reads the new row j
    const int tp = (p - j0) % kLpThreads, up = (p - j0) / kLpThreads;
    if (tid == jj) {
#pragma unroll
      for (int c = 0; c < kNb; ++c) sA[c] = y[0][c];
    }
    if (tid == tp) {
#pragma unroll
      for (int c = 0; c < kNb; ++c) sB[c] = up == 0 ? y[0][c] : y[1][c];
    }
    if (tid == 0) spiv[jj] = p;
    __syncthreads();
    const double* prow = sB;  // the new row j, read from LDS
    if (p != j) {
      if (tid == jj) {
#pragma unroll
        for (int c = 0; c < kNb; ++c) y[0][c] = prow[c];
      }
      if (tid == tp) {
#pragma unroll
        for (int c = 0; c < kNb; ++c) {
          if (up == 0) y[0][c] = sA[c]; else y[1][c] = sA[c];
        }
      }
    }
    const double inv = 1.0 / prow[jj];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int R = j0 + tid + u * kLpThreads;
      if (R > j && R < n) {
        const double l = pick16(y[u], jj) * inv;
#pragma unroll
        for (int c = 0; c < kNb; ++c) {
          if (c == jj) y[u][c] = l;
          else if (c > jj) y[u][c] -= l * prow[c];
        }
      }
    }
    // Two barriers per step: the argmax slots are read before this step's
    // exchange barrier, which every thread passes before the next step
    // writes them; sA / sB are read after that barrier and before the next
    // step's argmax barrier, which precedes their next writes.
  }
  __syncthreads();  // sA / sB of the last step, before the code below
  // panel back to memory
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int R = j0 + tid + u * kLpThreads;
    if (R < n) {
      double* dst = M + int64_t(R) * n + j0;
#pragma unroll
      for (int c = 0; c < kNb; ++c)
        if (c < jb) dst[c] = y[u][c];
    }
  }
  if (tid < jb) piv[j0 + tid] = spiv[tid];
  // interchanges on the columns outside the panel, in order
  for (int col = tid; col < n; col += kLpThreads) {
    if (col >= j0 && col < j0 + jb) continue;
    for (int jj = 0; jj < jb; ++jj) {
      const int pj = spiv[jj];
      if (pj != j0 + jj) {
        const double t = M[int64_t(j0 + jj) * n + col];
        M[int64_t(j0 + jj) * n + col] = M[int64_t(pj) * n + col];
        M[int64_t(pj) * n + col] = t;
      }
    }
  }
  __syncthreads();  // the panel rows and the interchanges are in memory
  // the unit lower L11 of the panel, read once into LDS for every column
  __shared__ double sL11[kNb][kNb];
  for (int e = tid; e < kNb * kNb; e += kLpThreads) {
    const int a = e / kNb, b = e % kNb;
    sL11[a][b] = (a < jb && b < a) ? M[int64_t(j0 + a) * n + j0 + b] : 0.0;
  }
  __syncthreads();
  // U12 = L11^{-1} A12 (rows j0..j0+jb-1, columns j0+jb..n-1)
  for (int c = j0 + jb + tid; c < n; c += kLpThreads) {
    double x[kNb];
#pragma unroll
    for (int i = 0; i < kNb; ++i) x[i] = i < jb ? M[int64_t(j0 + i) * n + c] : 0.0;
#pragma unroll
    for (int i = 1; i < kNb; ++i) {
      if (i >= jb) break;
      double v = x[i];
#pragma unroll
      for (int p2 = 0; p2 < kNb; ++p2)
        if (p2 < i) v -= sL11[i][p2] * x[p2];
      x[i] = v;
    }
#pragma unroll
    for (int i = 1; i < kNb; ++i)
      if (i < jb) M[int64_t(j0 + i) * n + c] = x[i];
  }
}

// ---------------------------------------------------------------------------
// Multi-workgroup panel for panels taller than the register panels (the top
// block and the largest redundant blocks in 3D): rows in blocks of kLmRows
// per workgroup, one launch per column step.  Every workgroup reduces the
// block maxima left by the previous launch to the pivot (largest |a(i, j)|
// over unpivoted candidate rows i < r, ties to the lowest row), eliminates
// column j from its own unpivoted rows and leaves its block maximum of
// column j + 1 (double-buffered by step parity).  The pivot row is flagged,
// not moved, so no workgroup reads a row that another writes in the same
// launch; after the panel the interchanges go to piv in LAPACK order and are
// applied as one permutation, with U12 = L11^{-1} A12.
// ---------------------------------------------------------------------------
constexpr int kLmRows = 256;

struct LuPanelState {
  double* pv;      // [2][nprob][nblk] block maxima
  int32_t* pi;     // [2][nprob][nblk] their rows
  int32_t* flag;   // [nprob][fstride] -1 unpivoted, else the step (rows j0..)
  int32_t* prow;   // [nprob][kNb] pivot row of each step
  int nblk;
  int64_t fstride;
};

__global__ __launch_bounds__(256) void k_lum_init(LuBatch A, LuPanelState P, int j0) {
  const int q = blockIdx.y, blk = blockIdx.x;
  const int n = A.n[q], r = A.r[q];
  if (j0 >= r || j0 + blk * kLmRows >= n) return;
  const double* M = A.base + A.moff[q];
  const int i = j0 + blk * kLmRows + threadIdx.x;
  if (i < n) P.flag[q * P.fstride + (i - j0)] = -1;
  AM loc{-1.0, INT_MAX};
  if (i < r) loc = AM{fabs(M[int64_t(i) * n + j0]), i};
  const AM b = block_argmax256(loc);
  if (threadIdx.x == 0) {
    P.pv[q * P.nblk + blk] = b.v;
    P.pi[q * P.nblk + blk] = b.i;
  }
}

__global__ __launch_bounds__(256) void k_lum_step(LuBatch A, LuPanelState P, int j0, int jj) {
  const int q = blockIdx.y, blk = blockIdx.x;
  const int n = A.n[q], r = A.r[q];
  if (j0 >= r) return;
  const int jb = min(kNb, r - j0);
  const int rb0 = j0 + blk * kLmRows;
  if (jj >= jb || rb0 >= n) return;
  double* M = A.base + A.moff[q];
  const int tid = threadIdx.x;
  const int64_t cur = int64_t(jj & 1) * A.nprob * P.nblk, nxt = int64_t((jj + 1) & 1) * A.nprob * P.nblk;
  const int nbr = (r - j0 + kLmRows - 1) / kLmRows;  // blocks holding candidate rows
  AM loc{-1.0, INT_MAX};
  for (int b = tid; b < nbr; b += 256) loc = am_better(loc, AM{P.pv[cur + q * P.nblk + b], P.pi[cur + q * P.nblk + b]});
  const AM best = block_argmax256(loc);
  if (!(best.v > 0.0)) {
    if (blk == 0 && tid == 0) atomicOr(A.status, 1);
    return;
  }
  const int rp = best.i;
  __shared__ double sp[kNb];
  if (tid < kNb) sp[tid] = tid < jb ? M[int64_t(rp) * n + j0 + tid] : 0.0;
  __syncthreads();
  if (blk == 0 && tid == 0) P.prow[q * kNb + jj] = rp;
  const int i = rb0 + tid;
  AM nx{-1.0, INT_MAX};
  if (i < n && i != rp && P.flag[q * P.fstride + (i - j0)] < 0) {
    double* row = M + int64_t(i) * n + j0;
    double y[kNb];
#pragma unroll
    for (int c = 0; c < kNb; ++c) y[c] = (c >= jj && c < jb) ? row[c] : 0.0;
    const double l = pick16(y, jj) / sp[jj];
#pragma unroll
    for (int c = 0; c < kNb; ++c) {
      if (c == jj) row[c] = l;
      else if (c > jj && c < jb) {
        y[c] -= l * sp[c];
        row[c] = y[c];
      }
    }
    if (jj + 1 < jb && i < r) nx = AM{fabs(pick16(y, jj + 1)), i};
  }
  if (i == rp) P.flag[q * P.fstride + (i - j0)] = jj;
  const AM b2 = block_argmax256(nx);
  if (tid == 0) {
    P.pv[nxt + q * P.nblk + blk] = b2.v;
    P.pi[nxt + q * P.nblk + blk] = b2.i;
  }
}

// The panel's interchanges as a permutation of at most 2 kNb rows (one wave,
// lane a holds entry a: position dst receives physical row src), and piv.
__device__ void lum_perm(const LuPanelState& P, int q, int j0, int jb, int* s_dst, int* s_src, int* s_na,
                         int32_t* piv) {
  const int lane = threadIdx.x & 63;
  if (threadIdx.x >= 64) return;
  int dst = lane < jb ? j0 + lane : -1, src = dst, na = jb;
  for (int jj = 0; jj < jb; ++jj) {
    const int rp = P.prow[q * kNb + jj];
    const unsigned long long hit = __ballot(src == rp);
    int ap;
    if (hit) {
      ap = __ffsll(hit) - 1;
    } else {
      ap = na++;
      if (lane == ap) dst = src = rp;
    }
    const int pos = __shfl(dst, ap, 64);
    if (piv && lane == 0) piv[j0 + jj] = pos;
    const int s_jj = __shfl(src, jj, 64), s_ap = __shfl(src, ap, 64);
    if (lane == jj) src = s_ap;
    if (lane == ap) src = s_jj;
  }
  if (lane < na) {
    s_dst[lane] = dst;
    s_src[lane] = src;
  }
  if (lane == 0) *s_na = na;
}

// Columns outside the panel (mode 0): the interchanges, and right of the
// panel U12 = L11^{-1} A12 with L11 from the pivot rows' panel columns (not
// written here).  Mode 1: the interchanges of the panel columns.
__global__ __launch_bounds__(256) void k_lum_finish(LuBatch A, LuPanelState P, int j0, int mode) {
  const int q = blockIdx.y;
  const int n = A.n[q], r = A.r[q];
  if (j0 >= r) return;
  const int jb = min(kNb, r - j0);
  double* M = A.base + A.moff[q];
  __shared__ int s_dst[2 * kNb], s_src[2 * kNb], s_na;
  __shared__ double sL[kNb][kNb + 1];
  lum_perm(P, q, j0, jb, s_dst, s_src, &s_na, (mode == 0 && blockIdx.x == 0) ? A.piv + A.poff[q] : nullptr);
  __syncthreads();
  const int na = s_na;
  if (mode == 1) {
    const int e = threadIdx.x;  // one thread per panel column
    if (blockIdx.x != 0 || e >= jb) return;
    const int col = j0 + e;
    double v[2 * kNb];
#pragma unroll
    for (int a2 = 0; a2 < 2 * kNb; ++a2) v[a2] = a2 < na ? M[int64_t(s_src[a2]) * n + col] : 0.0;
#pragma unroll
    for (int a2 = 0; a2 < 2 * kNb; ++a2)
      if (a2 < na && s_src[a2] != s_dst[a2]) M[int64_t(s_dst[a2]) * n + col] = v[a2];
    return;
  }
  for (int e = threadIdx.x; e < kNb * kNb; e += 256) {
    const int i = e / kNb, c = e % kNb;
    sL[i][c] = (i < jb && c < jb) ? M[int64_t(s_src[i]) * n + j0 + c] : 0.0;
  }
  bool moved = false;
  for (int a2 = 0; a2 < na; ++a2) moved = moved || s_src[a2] != s_dst[a2];
  __syncthreads();
  const int col = blockIdx.x * 256 + threadIdx.x;
  if (col >= n || (col >= j0 && col < j0 + jb)) return;
  const bool right = col >= j0 + jb;
  if (!right && !moved) return;
  double v[2 * kNb];
#pragma unroll
  for (int a2 = 0; a2 < 2 * kNb; ++a2)
    v[a2] = (a2 < na && ((right && a2 < jb) || s_src[a2] != s_dst[a2])) ? M[int64_t(s_src[a2]) * n + col] : 0.0;
  if (right) {
#pragma unroll
    for (int i = 1; i < kNb; ++i) {
      if (i >= jb) break;
      double t = v[i];
#pragma unroll
      for (int p2 = 0; p2 < kNb; ++p2)
        if (p2 < i) t -= sL[i][p2] * v[p2];
      v[i] = t;
    }
  }
#pragma unroll
  for (int a2 = 0; a2 < 2 * kNb; ++a2)
    if (a2 < na && ((right && a2 < jb) || s_src[a2] != s_dst[a2])) M[int64_t(s_dst[a2]) * n + col] = v[a2];
}

// Trailing update A22 -= L21 U12 of one 64 x 64 tile (K = panel width).
__global__ __launch_bounds__(256) void k_lu_update(LuBatch A, int j0) {
  const int q = blockIdx.z;
  const int n = A.n[q], r = A.r[q];
  if (j0 >= r) return;
  const int jb = min(kNb, r - j0);
  const int s0 = j0 + jb;
  const int rt0 = s0 + blockIdx.y * 64, ct0 = s0 + blockIdx.x * 64;
  if (rt0 >= n || ct0 >= n) return;
  double* M = A.base + A.moff[q];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = wv >> 1, wc = wv & 1;
  if (A.fp32 && rt0 >= r && ct0 >= r) {
    // Schur update of the skeleton block (rows and columns >= r) in FP32
    float4_t d[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) d[a][b] = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kNb; ks += 4) {
      const int k = ks + lk;
      float af[2], bf[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int i = rt0 + wr * 32 + a * 16 + li;
        af[a] = (i < n && k < jb) ? float(M[int64_t(i) * n + j0 + k]) : 0.f;
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int c = ct0 + wc * 32 + b * 16 + li;
        bf[b] = (c < n && k < jb) ? float(M[int64_t(j0 + k) * n + c]) : 0.f;
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) d[a][b] = mfma_f32(af[a], bf[b], d[a][b]);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = rt0 + wr * 32 + a * 16 + 4 * lk + v;
          const int c = ct0 + wc * 32 + b * 16 + li;
          if (i < n && c < n) M[int64_t(i) * n + c] -= double(d[a][b][v]);
        }
    return;
  }
  double4_t d[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) d[a][b] = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < kNb; ks += 4) {
    const int k = ks + lk;
    double af[2], bf[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int i = rt0 + wr * 32 + a * 16 + li;
      af[a] = (i < n && k < jb) ? M[int64_t(i) * n + j0 + k] : 0.0;
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int c = ct0 + wc * 32 + b * 16 + li;
      bf[b] = (c < n && k < jb) ? M[int64_t(j0 + k) * n + c] : 0.0;
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) d[a][b] = mfma_f64(af[a], bf[b], d[a][b]);
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = rt0 + wr * 32 + a * 16 + 4 * v + lk;
        const int c = ct0 + wc * 32 + b * 16 + li;
        if (i < n && c < n) M[int64_t(i) * n + c] -= d[a][b][v];
      }
}

// Batched general GEMM, one 64 x 64 tile of C per workgroup:
// C = beta C + alpha op(A) op(B) for every entry of a problem table.
__global__ __launch_bounds__(256) void k_gemm_tiles(const GemmDesc* D, int nd) {
  const int q = blockIdx.z;
  if (q >= nd) return;
  const GemmDesc g = D[q];
  const int tm = blockIdx.y * kGemmTile, tn = blockIdx.x * kGemmTile;
  if (tm >= g.M || tn >= g.N) return;
  __shared__ double lds[kGemmLds];
  const int Mt = min(kGemmTile, g.M - tm), Nt = min(kGemmTile, g.N - tn);
  const double* Ap = g.ta ? g.A + tm : g.A + int64_t(tm) * g.lda;
  const double* Bp = g.tb ? g.B + int64_t(tn) * g.ldb : g.B + tn;
  if (g.fp32)
    wg_gemm_f32(Mt, Nt, g.K, g.alpha, Ap, g.lda, g.ta, Bp, g.ldb, g.tb, g.beta, g.C + int64_t(tm) * g.ldc + tn, g.ldc,
                lds);
  else
    wg_gemm(Mt, Nt, g.K, g.alpha, Ap, g.lda, g.ta, Bp, g.ldb, g.tb, g.beta, g.C + int64_t(tm) * g.ldc + tn, g.ldc,
            lds);
}

}  // namespace

// Second stream of the row compression's look-ahead, one per host thread and
// device, with the two events that order it against the caller's stream;
// created on first use and kept for the life of the thread (creating and
// destroying them per call costs a host wait on their work each time, and
// an event must not be destroyed while a stream still waits on it), or
// until release_thread_streams.
struct AuxStream {
  hipStream_t s2 = nullptr;
  hipEvent_t ev_fact = nullptr, ev_rest = nullptr;
};

static std::map<int, AuxStream>& aux_streams() {
  thread_local std::map<int, AuxStream> streams;
  return streams;
}

static const AuxStream& aux_stream() {
  std::map<int, AuxStream>& streams = aux_streams();
  int dev = 0;
  HIF_HIP(hipGetDevice(&dev));
  auto it = streams.find(dev);
  if (it != streams.end()) return it->second;
  AuxStream a;
  HIF_HIP(hipStreamCreateWithFlags(&a.s2, hipStreamNonBlocking));
  if (hipEventCreateWithFlags(&a.ev_fact, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&a.ev_rest, hipEventDisableTiming) != hipSuccess) {
    if (a.ev_fact) (void)hipEventDestroy(a.ev_fact);
    (void)hipStreamDestroy(a.s2);
    throw Error{HIF_EDEVICE, "creating the look-ahead events failed"};
  }
  return streams[dev] = a;
}

void release_thread_streams() {
  std::map<int, AuxStream>& streams = aux_streams();
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto& kv : streams) {
    (void)hipSetDevice(kv.first);
    (void)hipStreamSynchronize(kv.second.s2);
    dbuf_retire_stream(kv.second.s2);
    (void)hipEventDestroy(kv.second.ev_fact);
    (void)hipEventDestroy(kv.second.ev_rest);
    (void)hipStreamDestroy(kv.second.s2);
  }
  streams.clear();
  (void)hipSetDevice(cur);
}

// The LDS-staged chunk update asks for more than the default 64 KiB of
// dynamic LDS.
static void allow_apply_lds() {
  static std::once_flag once;
  std::call_once(once, [] {
    const int bytes = int(kApplyLds);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tsqr_apply_chunk_lds<2>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tsqr_apply_chunk_lds<4>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tsqr_apply_chunk_lds<8>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipGetLastError();
  });
}

void launch_qr_batched(const QrBatch& A, int max_rows, int max_cols, hipStream_t s) {
  if (A.nprob == 0) return;
  // chunks of 256 rows (one per thread), or of 1024 rows (two per thread)
  // when the stack of 256-row chunk factors would exceed kTsqrStack rows
  int rpt = 0;
  if (tsqr_chunks(max_rows) * kTsqrNb <= kTsqrStack)
    rpt = 1;
  else if (((max_rows + 4 * kTsqrRows - 1) / (4 * kTsqrRows)) * kTsqrNb <= kTsqrStack)
    rpt = 2;
  if (rpt > 0) {
    const int cr = rpt == 1 ? kTsqrRows : 4 * kTsqrRows;
    const unsigned nckmax = unsigned((max_rows + cr - 1) / cr);
    // Look-ahead: panel p is factored on s; its update of the next panel's
    // 32 columns also runs on s, and that of the remaining columns on a
    // second stream, overlapping the factorization of panel p + 1.  Panels
    // alternate between two scratch halves (p & 1), so that panel p + 1
    // never overwrites the V and T that the update of panel p still reads.
    // Orders: the update of panel p on any column follows that of panel
    // p - 1 (s waits for the remaining-columns update of p - 1 before its
    // own updates of panel p), and the remaining-columns update of p
    // follows the factorization of p (it waits for an event recorded after
    // the stack kernel).
    allow_apply_lds();
    const int uw = tuning().rowqr_update_waves, ukind = tuning().rowqr_update_kind, ulds = ukind == 1;
    const AuxStream& aux = aux_stream();
    hipStream_t s2 = aux.s2;
    hipEvent_t ev_fact = aux.ev_fact, ev_rest = aux.ev_rest;
    bool rest_pending = false;
    for (int j0 = 0, p = 0; j0 < max_cols; j0 += kTsqrNb, ++p) {
      const int half = p & 1;
      // two rows per thread: 128 threads per 256-row chunk, 512 per 1024-row chunk
      if (rpt == 1)
        hipLaunchKernelGGL((k_tsqr_chunk<128, 2>), dim3(nckmax, A.nprob), dim3(128), 0, s, A, j0, cr, half);
      else
        hipLaunchKernelGGL((k_tsqr_chunk<512, 2>), dim3(nckmax, A.nprob), dim3(512), 0, s, A, j0, cr, half);
      if (nckmax * kTsqrNb <= 256)  // block sized to the tallest stack (two rows per thread)
        hipLaunchKernelGGL((k_tsqr_stack<128, 2>), dim3(A.nprob), dim3(128), 0, s, A, j0, cr, half);
      else if (nckmax * kTsqrNb <= 512)
        hipLaunchKernelGGL((k_tsqr_stack<256, 2>), dim3(A.nprob), dim3(256), 0, s, A, j0, cr, half);
      else
        hipLaunchKernelGGL((k_tsqr_stack<512, 2>), dim3(A.nprob), dim3(512), 0, s, A, j0, cr, half);
      const int nb0 = j0 + kTsqrNb, nb1 = j0 + 2 * kTsqrNb;  // next panel: columns [nb0, nb1)
      if (nb0 >= max_cols) break;
      HIF_HIP(hipEventRecord(ev_fact, s));
      if (rest_pending) HIF_HIP(hipStreamWaitEvent(s, ev_rest, 0));  // remaining-columns update of p - 1
      rest_pending = false;
      if (nb1 < max_cols) {
        const unsigned tiles = unsigned((max_cols - nb1 + 63) / 64);
        HIF_HIP(hipStreamWaitEvent(s2, ev_fact, 0));
        const dim3 g8(unsigned((max_cols - nb1 + 127) / 128), nckmax, A.nprob), g4(tiles, nckmax, A.nprob);
        const dim3 gs2(unsigned((max_cols - nb1 + 31) / 32), nckmax, A.nprob);
        if (cr <= 256 && ukind == 2 && uw == 8)
          hipLaunchKernelGGL(k_tsqr_apply_chunk_split<4>, g4, dim3(512), 0, s2, A, j0, cr, half, nb1, max_cols);
        else if (cr <= 256 && ukind == 2)
          hipLaunchKernelGGL(k_tsqr_apply_chunk_split<2>, gs2, dim3(256), 0, s2, A, j0, cr, half, nb1, max_cols);
        else if (cr <= 256 && ulds && uw == 8)
          hipLaunchKernelGGL(k_tsqr_apply_chunk_lds<8>, g8, dim3(512), kApplyLds, s2, A, j0, cr, half, nb1, max_cols);
        else if (cr <= 256 && ulds)
          hipLaunchKernelGGL(k_tsqr_apply_chunk_lds<4>, g4, dim3(256), kApplyLds, s2, A, j0, cr, half, nb1, max_cols);
        else if (cr <= 256 && uw == 8)
          hipLaunchKernelGGL(k_tsqr_apply_chunk_reg<8>, g8, dim3(512), 0, s2, A, j0, cr, half, nb1, max_cols);
        else if (cr <= 256)
          hipLaunchKernelGGL(k_tsqr_apply_chunk_reg<4>, g4, dim3(256), 0, s2, A, j0, cr, half, nb1, max_cols);
        else
          hipLaunchKernelGGL(k_tsqr_apply_chunk, dim3(tiles, nckmax, A.nprob), dim3(256), 0, s2, A, j0, cr, half,
                             nb1, max_cols);
        hipLaunchKernelGGL((k_tsqr_apply_stack_rg<4, 2>), dim3(tiles, A.nprob), dim3(512), 0, s2, A, j0, cr, half, nb1,
                           max_cols);
        HIF_HIP(hipEventRecord(ev_rest, s2));
        rest_pending = true;
      }
      if (cr <= 256 && ulds)  // the next panel's 32 columns: two waves
        hipLaunchKernelGGL(k_tsqr_apply_chunk_lds<2>, dim3(1, nckmax, A.nprob), dim3(128), kApplyLds, s, A, j0, cr,
                           half, nb0, nb1);
      else if (cr <= 256)
        hipLaunchKernelGGL(k_tsqr_apply_chunk_reg<4>, dim3(1, nckmax, A.nprob), dim3(256), 0, s, A, j0, cr, half, nb0,
                           nb1);
      else
        hipLaunchKernelGGL(k_tsqr_apply_chunk, dim3(1, nckmax, A.nprob), dim3(256), 0, s, A, j0, cr, half, nb0, nb1);
      hipLaunchKernelGGL((k_tsqr_apply_stack_rg<2, 4>), dim3(1, A.nprob), dim3(512), 0, s, A, j0, cr, half, nb0, nb1);
    }
    if (rest_pending) HIF_HIP(hipStreamWaitEvent(s, ev_rest, 0));
    hipLaunchKernelGGL(k_qr_clear_lower, dim3(64, A.nprob), dim3(256), 0, s, A);
    HIF_HIP(hipGetLastError());
    return;
  }
  // taller problems: one workgroup per problem for the panel
  for (int j0 = 0; j0 < max_cols; j0 += kNb) {
    hipLaunchKernelGGL(k_qr_panel, dim3(A.nprob), dim3(kQpThreads), 0, s, A, j0);
    const int rem = max_cols - j0 - kNb;
    if (rem > 0) {
      const unsigned tiles = unsigned((rem + kTileN - 1) / kTileN);
      hipLaunchKernelGGL(k_qr_update, dim3(tiles, A.nprob), dim3(kQrThreads), 0, s, A, j0);
    }
  }
  hipLaunchKernelGGL(k_qr_clear_lower, dim3(64, A.nprob), dim3(256), 0, s, A);
  HIF_HIP(hipGetLastError());
}

// One rectangle copy per blockIdx.y: dst[r * dld + c] = src[r * sld + c].
struct BlockCopy {
  const double* src;
  double* dst;
  int32_t sld, dld, rows, cols;
};
__global__ void k_copy_blocks(const BlockCopy* d) {
  const BlockCopy c = d[blockIdx.y];
  const int64_t ne = int64_t(c.rows) * c.cols;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < ne; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t r = e / c.cols, k = e % c.cols;
    c.dst[r * c.dld + k] = c.src[r * c.sld + k];
  }
}

static void copy_blocks(const std::vector<BlockCopy>& h, MemTracker* mt, hipStream_t s) {
  if (h.empty()) return;
  DBuf<BlockCopy> d;
  d.alloc(h.size(), mt);
  HIF_HIP(hipMemcpyAsync(d.p, h.data(), sizeof(BlockCopy) * h.size(), hipMemcpyHostToDevice, s));
  for (size_t i = 0; i < h.size(); i += 65535) {
    const unsigned cnt = unsigned(std::min<size_t>(65535, h.size() - i));
    hipLaunchKernelGGL(k_copy_blocks, dim3(256, cnt), dim3(256), 0, s, d.p + i);
  }
  HIF_HIP(hipGetLastError());
}

void launch_rowqr_split(double* base, const std::vector<int64_t>& moff, const std::vector<int32_t>& ld,
                        const std::vector<int32_t>& rows, const std::vector<int32_t>& cols, MemTracker* mt,
                        hipStream_t s) {
  // The R factor of [Y_1; ...; Y_b] is that of [R_1; ...; R_b] with
  // Y_i = Q_i R_i (up to row signs, which the ID does not see), and only R
  // is needed.  Blocks of 4096..8192 rows (n <= 2048) shrink the stack at
  // least 2-fold a round; blocks of 16384..32768 rows (n <= 16384) leave a
  // stack of nb n rows, which a round of 2 blocks brings to one block.
  struct Prob {
    int64_t off;
    int32_t ld, rows, cols, orig;
  };
  int maxn = 1;
  std::vector<Prob> cur;
  for (size_t q = 0; q < rows.size(); ++q)
    if (rows[q] > cols[q]) {
      cur.push_back({moff[q], ld[q], rows[q], cols[q], int32_t(q)});
      maxn = std::max(maxn, cols[q]);
    }
  HIF_REQUIRE(maxn <= kTsqrSplitRows / 2, HIF_EUNSUPPORTED, "row compression of more than 16384 columns");
  const int B = maxn <= 2048 ? 8192 : kTsqrSplitRows;
  double* rbase = base;     // buffer of this round's problems
  DBuf<double> stack[2];    // stacks of R factors, alternating by round
  for (int round = 0; !cur.empty(); ++round) {
    std::vector<int64_t> h_off, h_soff;
    std::vector<int32_t> h_ld, h_rows, h_cols;
    std::vector<int32_t> nblk(cur.size());
    int64_t stot = 0, next_tot = 0;
    int maxr = 1, maxc = 1;
    for (size_t i = 0; i < cur.size(); ++i) {
      const Prob& p = cur[i];
      const int nb = p.rows > B ? (p.rows + B - 1) / B : 1;
      nblk[i] = nb;
      for (int b = 0; b < nb; ++b) {
        const int r0 = int(int64_t(p.rows) * b / nb), r1 = int(int64_t(p.rows) * (b + 1) / nb);
        h_off.push_back(p.off + int64_t(r0) * p.ld);
        h_ld.push_back(p.ld);
        h_rows.push_back(r1 - r0);
        h_cols.push_back(p.cols);
        h_soff.push_back(stot);
        stot += rowqr_scratch(r1 - r0, p.cols);
        maxr = std::max(maxr, r1 - r0);
        maxc = std::max(maxc, p.cols);
      }
      if (nb > 1) next_tot += int64_t(nb) * p.cols * p.cols;
    }
    const int np = int(h_off.size());
    DBuf<int64_t> d_off, d_soff;
    DBuf<int32_t> d_ld, d_rows, d_cols;
    DBuf<double> scratch;
    d_off.alloc(np, mt);
    d_soff.alloc(np, mt);
    d_ld.alloc(np, mt);
    d_rows.alloc(np, mt);
    d_cols.alloc(np, mt);
    scratch.alloc(stot + 1, mt);
    HIF_HIP(hipMemcpyAsync(d_off.p, h_off.data(), sizeof(int64_t) * np, hipMemcpyHostToDevice, s));
    HIF_HIP(hipMemcpyAsync(d_soff.p, h_soff.data(), sizeof(int64_t) * np, hipMemcpyHostToDevice, s));
    HIF_HIP(hipMemcpyAsync(d_ld.p, h_ld.data(), sizeof(int32_t) * np, hipMemcpyHostToDevice, s));
    HIF_HIP(hipMemcpyAsync(d_rows.p, h_rows.data(), sizeof(int32_t) * np, hipMemcpyHostToDevice, s));
    HIF_HIP(hipMemcpyAsync(d_cols.p, h_cols.data(), sizeof(int32_t) * np, hipMemcpyHostToDevice, s));
    QrBatch A{};
    A.base = rbase;
    A.moff = d_off.p;
    A.ld = d_ld.p;
    A.rows = d_rows.p;
    A.cols = d_cols.p;
    A.scratch = scratch.p;
    A.soff = d_soff.p;
    A.nprob = np;
    // every block has at most B <= kTsqrSplitRows rows: one TSQR stack
    launch_qr_batched(A, maxr, maxc, s);
    // Unsplit problems are done (copied home if they are stacks); split ones
    // become stacks of their blocks' n x n R factors (lower parts cleared).
    DBuf<double>& nxt = stack[round & 1];
    if (next_tot > 0) nxt.alloc(next_tot, mt);
    std::vector<Prob> next;
    std::vector<BlockCopy> gather, back;
    int64_t noff = 0;
    size_t k = 0;
    for (size_t i = 0; i < cur.size(); ++i) {
      const Prob& p = cur[i];
      const int nb = nblk[i];
      if (nb == 1) {
        if (round > 0)
          back.push_back({rbase + p.off, base + moff[p.orig], p.ld, ld[p.orig], p.cols, p.cols});
        ++k;
        continue;
      }
      for (int b = 0; b < nb; ++b, ++k)
        gather.push_back({rbase + h_off[k], nxt.p + noff + int64_t(b) * p.cols * p.cols, p.ld, p.cols, p.cols,
                          p.cols});
      next.push_back({noff, p.cols, nb * p.cols, p.cols, p.orig});
      noff += int64_t(nb) * p.cols * p.cols;
    }
    // both copies read this round's buffer, which the round after next
    // allocates over (stream-ordered)
    copy_blocks(back, mt, s);
    copy_blocks(gather, mt, s);
    cur.swap(next);
    rbase = nxt.p;
  }
}

void launch_lu_batched(const LuBatch& A, int max_r, int max_n, hipStream_t s) {
  if (A.nprob == 0) return;
  // state of the multi-workgroup panel (panels taller than kLpRows)
  DBuf<double> pv;
  DBuf<int32_t> pi, flag, prow;
  LuPanelState P{};
  if (max_n > kLpRows) {
    P.nblk = (max_n + kLmRows - 1) / kLmRows;
    P.fstride = max_n;
    pv.alloc(size_t(2) * A.nprob * P.nblk, nullptr);
    pi.alloc(size_t(2) * A.nprob * P.nblk, nullptr);
    flag.alloc(size_t(A.nprob) * max_n, nullptr);
    prow.alloc(size_t(A.nprob) * kNb, nullptr);
    P.pv = pv.p;
    P.pi = pi.p;
    P.flag = flag.p;
    P.prow = prow.p;
  }
  const hif_tuning tu = tuning();
  for (int j0 = 0; j0 < max_r; j0 += kNb) {
    if (max_n - j0 > kLpRows) {
      const dim3 g(unsigned((max_n - j0 + kLmRows - 1) / kLmRows), unsigned(A.nprob));
      hipLaunchKernelGGL(k_lum_init, g, dim3(256), 0, s, A, P, j0);
      for (int jj = 0; jj < kNb; ++jj) hipLaunchKernelGGL(k_lum_step, g, dim3(256), 0, s, A, P, j0, jj);
      hipLaunchKernelGGL(k_lum_finish, dim3(unsigned((max_n + 255) / 256), unsigned(A.nprob)), dim3(256), 0, s, A,
                         P, j0, 0);
      hipLaunchKernelGGL(k_lum_finish, dim3(1, unsigned(A.nprob)), dim3(256), 0, s, A, P, j0, 1);
    } else {
      // two rows per thread: at least (panel rows) / 2 threads; within that,
      // the thread count of the launch-shape table for the panel's size
      const int rows = max_n - j0;
      int threads = rows <= kLpRows / 4 ? tu.lu_panel_threads[0] : (rows <= kLpRows / 2 ? tu.lu_panel_threads[1] : 1024);
      if (2 * threads < rows) threads = rows <= kLpRows / 2 ? 512 : 1024;
      if (threads == 256)
        hipLaunchKernelGGL(k_lu_panel_reg<256>, dim3(A.nprob), dim3(256), 0, s, A, j0);
      else if (threads == 512)
        hipLaunchKernelGGL(k_lu_panel_reg<512>, dim3(A.nprob), dim3(512), 0, s, A, j0);
      else
        hipLaunchKernelGGL(k_lu_panel_reg<1024>, dim3(A.nprob), dim3(1024), 0, s, A, j0);
    }
    const int rem = max_n - j0 - 1;
    if (rem > 0) {
      const unsigned tiles = unsigned((rem + 63) / 64);
      hipLaunchKernelGGL(k_lu_update, dim3(tiles, tiles, A.nprob), dim3(256), 0, s, A, j0);
    }
  }
  HIF_HIP(hipGetLastError());
}

void launch_gemm_tiles(const GemmDesc* D, int nd, int max_m, int max_n, hipStream_t s) {
  if (nd == 0 || max_m <= 0 || max_n <= 0) return;
  const unsigned tx = unsigned((max_n + kGemmTile - 1) / kGemmTile), ty = unsigned((max_m + kGemmTile - 1) / kGemmTile);
  hipLaunchKernelGGL(k_gemm_tiles, dim3(tx, ty, nd), dim3(256), 0, s, D, nd);
  HIF_HIP(hipGetLastError());
}

}  // namespace hif
