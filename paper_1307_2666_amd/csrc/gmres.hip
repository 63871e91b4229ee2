// Right-preconditioned GMRES (Section 5, Example 3: Lemma 5.1 and its
// corollary, with the factorization F ~ A of this handle as preconditioner):
// solve A u = f by GMRES on A F^{-1} y = f, u = F^{-1} y, x_0 = 0, no
// restart.  The transposed variant solves A^T u = f on A^T F^{-T} y = f with
// the same machinery.  A is the exact operator of eqn 1.1, applied pair by
// pair on the fly (the hif_matvec kernel) unless the handle was built with
// the FFT product enabled; F^{-1} is the solve sweep.  All right-hand
// sides iterate in lockstep; the Arnoldi basis, the products, the
// orthogonalization (classical Gram-Schmidt applied twice) and the norms run
// on the device with fixed-order two-stage reductions; only the small
// Hessenberg least-squares problems (Givens rotations) live on the host.
#include <cmath>
#include <vector>

#include "common.h"

namespace hif {

namespace {

constexpr int kSlices = 256;  // partial sums per dot product
constexpr int kThr = 256;

// part[(v*nvec + j)*kSlices + b] = sum over slice b of X[v][j][i] * Y[v][i]
__global__ __launch_bounds__(kThr) void k_mdot(const double* X, int64_t xs_rhs, const double* Y, int64_t ys_rhs,
                                               int64_t N, int nvec, double* part) {
  const int b = blockIdx.x, j = blockIdx.y, v = blockIdx.z;
  const int64_t lo = N * b / kSlices, hi = N * (b + 1) / kSlices;
  const double* x = X + v * xs_rhs + j * N;
  const double* y = Y + v * ys_rhs;
  double acc = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kThr) acc += x[i] * y[i];
  __shared__ double red[kThr / 64];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kThr / 64; ++w) t += red[w];
    part[(int64_t(v) * nvec + j) * kSlices + b] = t;
  }
}

// out[e] = sum_b part[e*kSlices + b] in slice order
__global__ void k_sum_parts(const double* part, int ne, double* out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  double t = 0.0;
  for (int b = 0; b < kSlices; ++b) t += part[int64_t(e) * kSlices + b];
  out[e] = t;
}

// Y[v][i] += sgn * sum_{j < nvec} X[v][j][i] * coef[v*cs + j]
__global__ __launch_bounds__(kThr) void k_vcomb(const double* X, int64_t xs_rhs, const double* coef, int cs,
                                                int nvec, double sgn, double* Y, int64_t ys_rhs, int64_t N) {
  const int v = blockIdx.y;
  const double* x = X + v * xs_rhs;
  double* y = Y + v * ys_rhs;
  const double* cv = coef + int64_t(v) * cs;
  for (int64_t i = blockIdx.x * int64_t(kThr) + threadIdx.x; i < N; i += int64_t(gridDim.x) * kThr) {
    double t = 0.0;
    for (int j = 0; j < nvec; ++j) t += x[int64_t(j) * N + i] * cv[j];
    y[i] += sgn * t;
  }
}

// Y[v][i] = X[v][i] * scale[v]
__global__ __launch_bounds__(kThr) void k_vscale(const double* X, int64_t xs_rhs, const double* scale, double* Y,
                                                 int64_t ys_rhs, int64_t N) {
  const int v = blockIdx.y;
  const double sc = scale[v];
  for (int64_t i = blockIdx.x * int64_t(kThr) + threadIdx.x; i < N; i += int64_t(gridDim.x) * kThr)
    Y[v * ys_rhs + i] = X[v * xs_rhs + i] * sc;
}

__global__ void k_zero(double* x, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    x[i] = 0.0;
}

unsigned grid_for(int64_t N) { return unsigned(std::min<int64_t>(1024, (N + kThr - 1) / kThr)); }

// Coefficients of A^T in the form the matvec evaluates.  With
// A_ij = b_i G_ij w_j c_j (i != j) and A_ii = a_i + b_i s_i c_i, the transpose
// is A^T_ij = (c_i w_i) G_ij b_j: row factor c w, column factor b, unit
// weights, and the whole diagonal carried by the a term (self term zero).
__global__ void k_transpose_coef(const double* a, const double* b, const double* c, const double* w,
                                 const double* sf, double* aT, double* bT, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    aT[i] = a[i] + b[i] * sf[i] * c[i];
    bT[i] = c[i] * w[i];
  }
}

// grad[i] = -sum_v lam[v][i] * u[v][i]
__global__ __launch_bounds__(kThr) void k_diag_grad(const double* lam, const double* u, double* grad, int64_t n,
                                                    int nr) {
  for (int64_t i = blockIdx.x * int64_t(kThr) + threadIdx.x; i < n; i += int64_t(gridDim.x) * kThr) {
    double t = 0.0;
    for (int v = 0; v < nr; ++v) t += lam[int64_t(v) * n + i] * u[int64_t(v) * n + i];
    grad[i] = -t;
  }
}

}  // namespace

void gmres_impl(hif_factor_s* H, const double* f, double* u, int64_t nrhs, double tol, int maxit, int32_t* iters,
                double* relres, bool trans, hipStream_t s) {
  const int64_t N = H->n;
  const int R = int(nrhs);
  const int K = maxit;
  // Basis V [R][K+1][N], work W [R][N], Z [R][N]; coefficient and partial buffers.
  DBuf<double> V, W, Z, part, hbuf, sbuf;
  V.alloc(size_t(R) * (K + 1) * N, nullptr);
  W.alloc(size_t(R) * N, nullptr);
  Z.alloc(size_t(R) * N, nullptr);
  part.alloc(size_t(R) * (K + 1) * kSlices, nullptr);
  hbuf.alloc(size_t(R) * (K + 1), nullptr);
  sbuf.alloc(size_t(R), nullptr);
  const int64_t vs = int64_t(K + 1) * N;  // RHS stride of V
  const unsigned gN = grid_for(N);

  auto dots = [&](const double* X, int64_t xs, const double* Y, int64_t ys, int nvec, std::vector<double>& out) {
    hipLaunchKernelGGL(k_mdot, dim3(kSlices, nvec, R), dim3(kThr), 0, s, X, xs, Y, ys, N, nvec, part.p);
    const int ne = R * nvec;
    hipLaunchKernelGGL(k_sum_parts, dim3((ne + 255) / 256), dim3(256), 0, s, part.p, ne, hbuf.p);
    HIF_HIP(hipGetLastError());
    out.resize(ne);
    HIF_HIP(hipMemcpyAsync(out.data(), hbuf.p, sizeof(double) * ne, hipMemcpyDeviceToHost, s));
    HIF_HIP(hipStreamSynchronize(s));
  };
  const int pre = trans ? 1 : 0;  // sweep: F^{-1} or F^{-T}
  auto matvec = [&](const double* x, double* y) { apply_A_impl(H, x, y, nrhs, trans, s); };

  // r_0 = f, beta = |f|, v_0 = f / beta
  std::vector<double> nrm;
  dots(f, N, f, N, 1, nrm);
  std::vector<double> beta(R), scale(R);
  for (int v = 0; v < R; ++v) {
    beta[v] = std::sqrt(nrm[v]);
    scale[v] = beta[v] > 0.0 ? 1.0 / beta[v] : 0.0;
  }
  HIF_HIP(hipMemcpyAsync(sbuf.p, scale.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_vscale, dim3(gN, R), dim3(kThr), 0, s, f, N, sbuf.p, V.p, vs, N);

  // Hessenberg (column-major per RHS), Givens rotations, rhs g of the LS problem
  std::vector<std::vector<double>> Hh(R, std::vector<double>(size_t(K + 1) * K, 0.0));
  std::vector<std::vector<double>> cs(R, std::vector<double>(K)), sn(R, std::vector<double>(K));
  std::vector<std::vector<double>> g(R, std::vector<double>(K + 1, 0.0));
  std::vector<int> done(R, 0), kused(R, 0);
  for (int v = 0; v < R; ++v) {
    g[v][0] = beta[v];
    if (!(beta[v] > 0.0)) done[v] = 1;
  }
  std::vector<double> h1, h2, coef(size_t(R) * (K + 1));
  int it = 0;
  for (; it < K; ++it) {
    bool all = true;
    for (int v = 0; v < R; ++v) all = all && done[v];
    if (all) break;
    // w = A F^{-1} v_it
    for (int v = 0; v < R; ++v)
      HIF_HIP(hipMemcpyAsync(W.p + v * N, V.p + v * vs + int64_t(it) * N, sizeof(double) * N,
                             hipMemcpyDeviceToDevice, s));
    sweep_impl(H, pre, W.p, Z.p, nrhs, s);
    matvec(Z.p, W.p);
    // classical Gram-Schmidt, twice
    const int nv = it + 1;
    dots(V.p, vs, W.p, N, nv, h1);
    HIF_HIP(hipMemcpyAsync(hbuf.p, h1.data(), sizeof(double) * R * nv, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_vcomb, dim3(gN, R), dim3(kThr), 0, s, V.p, vs, hbuf.p, nv, nv, -1.0, W.p, N, N);
    dots(V.p, vs, W.p, N, nv, h2);
    HIF_HIP(hipMemcpyAsync(hbuf.p, h2.data(), sizeof(double) * R * nv, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_vcomb, dim3(gN, R), dim3(kThr), 0, s, V.p, vs, hbuf.p, nv, nv, -1.0, W.p, N, N);
    dots(W.p, N, W.p, N, 1, nrm);
    for (int v = 0; v < R; ++v) {
      double* col = Hh[v].data() + size_t(it) * (K + 1);
      for (int j = 0; j < nv; ++j) col[j] = h1[size_t(v) * nv + j] + h2[size_t(v) * nv + j];
      const double hn = std::sqrt(nrm[v]);
      col[nv] = hn;
      scale[v] = (!done[v] && hn > 0.0) ? 1.0 / hn : 0.0;
      if (done[v]) continue;
      // apply previous rotations, then a new one that zeroes col[nv]
      for (int j = 0; j < it; ++j) {
        const double t = cs[v][j] * col[j] + sn[v][j] * col[j + 1];
        col[j + 1] = -sn[v][j] * col[j] + cs[v][j] * col[j + 1];
        col[j] = t;
      }
      const double a0 = col[it], b0 = col[nv];
      const double rr = std::hypot(a0, b0);
      cs[v][it] = rr > 0.0 ? a0 / rr : 1.0;
      sn[v][it] = rr > 0.0 ? b0 / rr : 0.0;
      col[it] = rr;
      col[nv] = 0.0;
      g[v][nv] = -sn[v][it] * g[v][it];
      g[v][it] = cs[v][it] * g[v][it];
      kused[v] = it + 1;
      // |g_{it+1}| is the residual norm of the LS solution; hn = 0 means the
      // Krylov space is invariant (exact solution reached)
      if (std::fabs(g[v][nv]) <= tol * beta[v] || !(hn > 0.0)) done[v] = 1;
    }
    HIF_HIP(hipMemcpyAsync(sbuf.p, scale.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_vscale, dim3(gN, R), dim3(kThr), 0, s, W.p, N, sbuf.p, V.p + int64_t(it + 1) * N, vs, N);
    HIF_HIP(hipGetLastError());
  }
  // y = R^{-1} g per RHS, then u = F^{-1} (V y)
  std::fill(coef.begin(), coef.end(), 0.0);
  for (int v = 0; v < R; ++v) {
    const int k = kused[v];
    for (int a = k - 1; a >= 0; --a) {
      double t = g[v][a];
      for (int b = a + 1; b < k; ++b) t -= Hh[v][size_t(b) * (K + 1) + a] * coef[size_t(v) * (K + 1) + b];
      const double d = Hh[v][size_t(a) * (K + 1) + a];
      coef[size_t(v) * (K + 1) + a] = d != 0.0 ? t / d : 0.0;
    }
    if (iters) iters[v] = k;
  }
  HIF_HIP(hipMemcpyAsync(hbuf.p, coef.data(), sizeof(double) * R * (K + 1), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_zero, dim3(gN), dim3(kThr), 0, s, W.p, int64_t(R) * N);
  // only the basis vectors built so far (0..it-1 carry coefficients)
  hipLaunchKernelGGL(k_vcomb, dim3(gN, R), dim3(kThr), 0, s, V.p, vs, hbuf.p, K + 1, it, 1.0, W.p, N, N);
  sweep_impl(H, pre, W.p, u, nrhs, s);
  // true residual |f - A u| / |f|
  matvec(u, W.p);
  std::vector<double> ones(R, -1.0);
  HIF_HIP(hipMemcpyAsync(sbuf.p, ones.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_vscale, dim3(gN, R), dim3(kThr), 0, s, W.p, N, sbuf.p, W.p, N, N);
  std::vector<double> fcoef(R, 1.0);
  HIF_HIP(hipMemcpyAsync(hbuf.p, fcoef.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_vcomb, dim3(gN, R), dim3(kThr), 0, s, f, N, hbuf.p, 1, 1, 1.0, W.p, N, N);
  dots(W.p, N, W.p, N, 1, nrm);
  if (relres)
    for (int v = 0; v < R; ++v) relres[v] = beta[v] > 0.0 ? std::sqrt(nrm[v]) / beta[v] : 0.0;
  HIF_HIP(hipStreamSynchronize(s));
}

void matvec_T_impl(hif_factor_s* H, const double* x, double* y, int64_t nrhs, hipStream_t s) {
  const int64_t N = H->n;
  DBuf<double> coefT;
  coefT.alloc(size_t(2) * N, nullptr);
  hipLaunchKernelGGL(k_transpose_coef, dim3(grid_for(N)), dim3(kThr), 0, s, H->a, H->b, H->c, H->w, H->selfk,
                     coefT.p, coefT.p + N, N);
  HIF_HIP(hipGetLastError());
  matvec_impl(H->pts, N, H->dim, coefT.p, coefT.p + N, H->b, nullptr, 1.0, nullptr, 0.0, x, y, nrhs, s);
}

void diag_grad_impl(const double* lam, const double* u, double* grad, int64_t n, int64_t nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_grad, dim3(grid_for(n)), dim3(kThr), 0, s, lam, u, grad, n, int(nrhs));
  HIF_HIP(hipGetLastError());
}

}  // namespace hif
