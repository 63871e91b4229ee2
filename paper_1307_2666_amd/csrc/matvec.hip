// Exact on-the-fly y = A x for A = diag(a) + diag(b) K diag(c) (eqn 1.1 under
// the collocation of Section 3.1): K_ij = G(|x_i - x_j|) w_j off the
// diagonal, K_ii the cell integral.  O(N^2) pair evaluations; each workgroup
// owns 256 targets and streams the sources through LDS in tiles, all
// right-hand sides (up to 8 per pass) sharing one kernel evaluation per pair.
#include "common.h"

namespace hif {

namespace {

constexpr int kTile = 256;

template <int D, int NR>
__global__ __launch_bounds__(kTile) void k_matvec(const double* __restrict__ pts, int64_t n,
                                                  const double* __restrict__ a, const double* __restrict__ b,
                                                  const double* __restrict__ c, const double* __restrict__ w,
                                                  double w_const, const double* __restrict__ selfk,
                                                  double self_const, const double* __restrict__ x,
                                                  double* __restrict__ y, int64_t ldx, int nr) {
  __shared__ double sp[D][kTile];
  __shared__ double sq[NR][kTile];
  const int64_t i = blockIdx.x * int64_t(kTile) + threadIdx.x;
  const bool valid = i < n;
  double xi[D];
#pragma unroll
  for (int k = 0; k < D; ++k) xi[k] = valid ? pts[i * D + k] : 0.0;
  double acc[NR];
#pragma unroll
  for (int v = 0; v < NR; ++v) acc[v] = 0.0;
  for (int64_t j0 = 0; j0 < n; j0 += kTile) {
    const int64_t j = j0 + threadIdx.x;
    __syncthreads();
    if (j < n) {
#pragma unroll
      for (int k = 0; k < D; ++k) sp[k][threadIdx.x] = pts[j * D + k];
      const double wc = (w ? w[j] : w_const) * (c ? c[j] : 1.0);
#pragma unroll
      for (int v = 0; v < NR; ++v) sq[v][threadIdx.x] = v < nr ? wc * x[v * ldx + j] : 0.0;
    } else {
#pragma unroll
      for (int k = 0; k < D; ++k) sp[k][threadIdx.x] = 2.0 + k;  // far away, weight 0
#pragma unroll
      for (int v = 0; v < NR; ++v) sq[v][threadIdx.x] = 0.0;
    }
    __syncthreads();
    const int cnt = int(n - j0 < kTile ? n - j0 : kTile);
    const int self_t = (i >= j0 && i < j0 + kTile) ? int(i - j0) : -1;
    for (int t = 0; t < cnt; ++t) {
      if (t == self_t) continue;
      double r2 = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const double d = xi[k] - sp[k][t];
        r2 += d * d;
      }
      const double g = green_r2<D>(r2);
#pragma unroll
      for (int v = 0; v < NR; ++v) acc[v] += g * sq[v][t];
    }
  }
  if (!valid) return;
  const double ai = a ? a[i] : 0.0, bi = b ? b[i] : 1.0, ci = c ? c[i] : 1.0;
  const double si = selfk ? selfk[i] : self_const;
#pragma unroll
  for (int v = 0; v < NR; ++v)
    if (v < nr) {
      const double xv = x[v * ldx + i];
      y[v * ldx + i] = ai * xv + bi * (acc[v] + si * ci * xv);
    }
}

template <int D>
void launch(const double* pts, int64_t n, const double* a, const double* b, const double* c, const double* w,
            double w_const, const double* selfk, double self_const, const double* x, double* y, int64_t nrhs,
            hipStream_t s) {
  const unsigned blocks = unsigned((n + kTile - 1) / kTile);
  for (int64_t v0 = 0; v0 < nrhs; v0 += 8) {
    const int nr = int(std::min<int64_t>(8, nrhs - v0));
    const double* xv = x + v0 * n;
    double* yv = y + v0 * n;
    if (nr == 1)
      hipLaunchKernelGGL((k_matvec<D, 1>), dim3(blocks), dim3(kTile), 0, s, pts, n, a, b, c, w, w_const, selfk,
                         self_const, xv, yv, n, nr);
    else if (nr <= 2)
      hipLaunchKernelGGL((k_matvec<D, 2>), dim3(blocks), dim3(kTile), 0, s, pts, n, a, b, c, w, w_const, selfk,
                         self_const, xv, yv, n, nr);
    else if (nr <= 4)
      hipLaunchKernelGGL((k_matvec<D, 4>), dim3(blocks), dim3(kTile), 0, s, pts, n, a, b, c, w, w_const, selfk,
                         self_const, xv, yv, n, nr);
    else
      hipLaunchKernelGGL((k_matvec<D, 8>), dim3(blocks), dim3(kTile), 0, s, pts, n, a, b, c, w, w_const, selfk,
                         self_const, xv, yv, n, nr);
    HIF_HIP(hipGetLastError());
  }
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
