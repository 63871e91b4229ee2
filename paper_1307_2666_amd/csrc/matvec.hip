// Exact on-the-fly y = A x for A = diag(a) + diag(b) K diag(c) (eqn 1.1 under
// the collocation of Section 3.1): K_ij = G(|x_i - x_j|) w_j off the
// diagonal, K_ii the cell integral.  O(N^2) pair evaluations; each workgroup
// owns 256 targets and streams the sources through LDS in tiles, all
// right-hand sides (up to 8 per pass) sharing one kernel evaluation per pair.
#include "common.h"

namespace hif {

namespace {

constexpr int kTile = 256;

// Natural logarithm of a positive normal x, within about 2 ulp, in some 30
// instructions (the library's double-precision log carries extra-precise
// steps that cost several times that, and the pair loop below is bound by
// it).  x = 2^e m with m in [sqrt(1/2), sqrt(2)); with s = (m - 1) / (m + 1),
// |s| <= 3 - 2 sqrt(2) < 0.1716, log m = 2 atanh(s) = 2 s sum_k s^(2k) /
// (2k + 1), whose terms past s^18 sum to below 2^-55 relative (s^2 < 0.0295);
// log x = e ln2_hi + (e ln2_lo + log m), ln2_hi holding 29 significant bits so
// that e ln2_hi is exact.
__device__ __forceinline__ double log_pos(double x) {
  double m = __builtin_amdgcn_frexp_mant(x);  // [0.5, 1)
  int e = __builtin_amdgcn_frexp_exp(x);
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    e -= 1;
  }
  const double f = m - 1.0;  // exact
  const double d = m + 1.0;
  double t = __builtin_amdgcn_rcp(d);
  t = fma(fma(-d, t, 1.0), t, t);  // one Newton step on 1 / d
  double q = f * t;
  q = fma(fma(-q, d, f), t, q);  // s = f / d, corrected once
  const double z = q * q;
  double p = 1.0 / 19.0;
  p = fma(p, z, 1.0 / 17.0);
  p = fma(p, z, 1.0 / 15.0);
  p = fma(p, z, 1.0 / 13.0);
  p = fma(p, z, 1.0 / 11.0);
  p = fma(p, z, 1.0 / 9.0);
  p = fma(p, z, 1.0 / 7.0);
  p = fma(p, z, 1.0 / 5.0);
  p = fma(p, z, 1.0 / 3.0);
  const double s2 = 2.0 * q;
  const double ed = double(e);
  const double lo = fma(s2 * z, p, ed * -4.2009150726810846e-11);  // + e ln2_lo
  return fma(ed, 0.6931471806019545, s2 + lo);
}

// G(r) from the squared distance for the pair loop (2D through log_pos).
template <int D>
__device__ __forceinline__ double green_pair(double r2) {
  if constexpr (D == 2) {
    return -0.5 * kInv2Pi * log_pos(r2);
  } else {
    return kInv4Pi * rsqrt(r2);
  }
}

// Each workgroup owns TPT * 256 targets (thread t: targets t + 256 u) and
// streams the sources through LDS in tiles of 256: the point and the
// weighted right-hand-side values of a source are read once per tile and
// serve TPT targets; all right-hand sides (up to 8 per pass) share one kernel
// evaluation per pair.  The self pair is dropped by a select, not a branch.
template <int D, int NR, int TPT>
__global__ __launch_bounds__(kTile) void k_matvec(const double* __restrict__ pts, int64_t n,
                                                  const double* __restrict__ a, const double* __restrict__ b,
                                                  const double* __restrict__ c, const double* __restrict__ w,
                                                  double w_const, const double* __restrict__ selfk,
                                                  double self_const, const double* __restrict__ x,
                                                  double* __restrict__ y, int64_t ldx, int nr) {
  __shared__ double sp[kTile][D];
  __shared__ double sq[kTile][NR];
  int64_t i[TPT];
  double xi[TPT][D];
  double acc[TPT][NR];
#pragma unroll
  for (int u = 0; u < TPT; ++u) {
    i[u] = (blockIdx.x * int64_t(TPT) + u) * kTile + threadIdx.x;
#pragma unroll
    for (int k = 0; k < D; ++k) xi[u][k] = i[u] < n ? pts[i[u] * D + k] : 4.0 + k;
#pragma unroll
    for (int v = 0; v < NR; ++v) acc[u][v] = 0.0;
  }
  for (int64_t j0 = 0; j0 < n; j0 += kTile) {
    const int64_t j = j0 + threadIdx.x;
    __syncthreads();
    if (j < n) {
#pragma unroll
      for (int k = 0; k < D; ++k) sp[threadIdx.x][k] = pts[j * D + k];
      const double wc = (w ? w[j] : w_const) * (c ? c[j] : 1.0);
#pragma unroll
      for (int v = 0; v < NR; ++v) sq[threadIdx.x][v] = v < nr ? wc * x[v * ldx + j] : 0.0;
    } else {
#pragma unroll
      for (int k = 0; k < D; ++k) sp[threadIdx.x][k] = 2.0 + k;  // far away, weight 0
#pragma unroll
      for (int v = 0; v < NR; ++v) sq[threadIdx.x][v] = 0.0;
    }
    __syncthreads();
    const int cnt = int(n - j0 < kTile ? n - j0 : kTile);
    int self_t[TPT];
#pragma unroll
    for (int u = 0; u < TPT; ++u) self_t[u] = (i[u] >= j0 && i[u] < j0 + kTile) ? int(i[u] - j0) : -1;
    for (int t = 0; t < cnt; ++t) {
      double q[NR];
#pragma unroll
      for (int v = 0; v < NR; ++v) q[v] = sq[t][v];
#pragma unroll
      for (int u = 0; u < TPT; ++u) {
        double r2 = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          const double dd = xi[u][k] - sp[t][k];
          r2 += dd * dd;
        }
        const bool self = t == self_t[u];
        const double g = self ? 0.0 : green_pair<D>(self ? 1.0 : r2);
#pragma unroll
        for (int v = 0; v < NR; ++v) acc[u][v] += g * q[v];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < TPT; ++u) {
    if (i[u] >= n) continue;
    const int64_t ii = i[u];
    const double ai = a ? a[ii] : 0.0, bi = b ? b[ii] : 1.0, ci = c ? c[ii] : 1.0;
    const double si = selfk ? selfk[ii] : self_const;
#pragma unroll
    for (int v = 0; v < NR; ++v)
      if (v < nr) {
        const double xv = x[v * ldx + ii];
        y[v * ldx + ii] = ai * xv + bi * (acc[u][v] + si * ci * xv);
      }
  }
}

template <int D, int TPT>
void launch_t(const double* pts, int64_t n, const double* a, const double* b, const double* c, const double* w,
              double w_const, const double* selfk, double self_const, const double* x, double* y, int64_t nrhs,
              hipStream_t s) {
  const unsigned blocks = unsigned((n + TPT * kTile - 1) / (TPT * kTile));
  for (int64_t v0 = 0; v0 < nrhs; v0 += 8) {
    const int nr = int(std::min<int64_t>(8, nrhs - v0));
    const double* xv = x + v0 * n;
    double* yv = y + v0 * n;
    if (nr == 1)
      hipLaunchKernelGGL((k_matvec<D, 1, TPT>), dim3(blocks), dim3(kTile), 0, s, pts, n, a, b, c, w, w_const, selfk,
                         self_const, xv, yv, n, nr);
    else if (nr <= 2)
      hipLaunchKernelGGL((k_matvec<D, 2, TPT>), dim3(blocks), dim3(kTile), 0, s, pts, n, a, b, c, w, w_const, selfk,
                         self_const, xv, yv, n, nr);
    else if (nr <= 4)
      hipLaunchKernelGGL((k_matvec<D, 4, TPT>), dim3(blocks), dim3(kTile), 0, s, pts, n, a, b, c, w, w_const, selfk,
                         self_const, xv, yv, n, nr);
    else
      hipLaunchKernelGGL((k_matvec<D, 8, TPT>), dim3(blocks), dim3(kTile), 0, s, pts, n, a, b, c, w, w_const, selfk,
                         self_const, xv, yv, n, nr);
    HIF_HIP(hipGetLastError());
  }
}

// Two targets per thread once there are enough targets to give every CU
// several workgroups of them.
template <int D>
void launch(const double* pts, int64_t n, const double* a, const double* b, const double* c, const double* w,
            double w_const, const double* selfk, double self_const, const double* x, double* y, int64_t nrhs,
            hipStream_t s) {
  if (n >= (int64_t(1) << 18))
    launch_t<D, 2>(pts, n, a, b, c, w, w_const, selfk, self_const, x, y, nrhs, s);
  else
    launch_t<D, 1>(pts, n, a, b, c, w, w_const, selfk, self_const, x, y, nrhs, s);
}

}  // namespace

void matvec_impl(const double* pts, int64_t n, int dim, const double* a, const double* b, const double* c,
                 const double* w, double w_const, const double* selfk, double self_const, const double* x,
                 double* y, int64_t nrhs, hipStream_t s) {
  if (dim == 2)
    launch<2>(pts, n, a, b, c, w, w_const, selfk, self_const, x, y, nrhs, s);
  else
    launch<3>(pts, n, a, b, c, w, w_const, selfk, self_const, x, y, nrhs, s);
}

}  // namespace hif
