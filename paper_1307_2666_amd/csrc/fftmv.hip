// Exact products with A on a uniform grid by FFT convolution.
//
// The operator of eqn 1.1 under the discretization of Section 3.1 is
// A = diag(a) + diag(b) K diag(c) with K_ij = G(|x_i - x_j|) w_j (i != j) and
// K_ii = s_i.  When the points are the cell centres of the full n^d grid of
// step h = 1/n and w, s are constant, K_ij depends only on the grid offset
// g_i - g_j, so K is a symmetric d-level Toeplitz matrix: K z is the linear
// convolution of the grid array of z with the kernel array
// k(delta) = G(h |delta|) w (k(0) = s), computed exactly (up to rounding) by a
// zero-padded cyclic convolution of size (2n)^d.  This is the same product
// hif_matvec forms pair by pair, in O(N log N) instead of O(N^2); the paper
// accelerates its products with A by FFT in the same way for its refinement.
#include <hipfft/hipfft.h>

#include <cmath>
#include <map>
#include <memory>
#include <tuple>
#include <vector>

#include "common.h"

namespace hif {

struct FftOp {
  int n = 0, d = 2;
  int64_t M = 0;   // (2n)^d real points of the padded grid
  int64_t Mh = 0;  // (2n)^(d-1) (n + 1) complex points of its half spectrum
  DBuf<int64_t> gidx;           // padded-grid position of every point
  DBuf<hipfftDoubleComplex> kh; // spectrum of the kernel array
};

namespace {

constexpr int kThr = 256;

unsigned grid1(int64_t n) { return unsigned(std::min<int64_t>(4096, (n + kThr - 1) / kThr)); }

void fft_check(hipfftResult r, const char* what) {
  if (r != HIPFFT_SUCCESS)
    throw Error{HIF_EDEVICE, std::string("hipFFT ") + what + " failed (" + std::to_string(int(r)) + ")"};
}

// Plans by (device, stream, dimension, size, batch, direction), per host
// thread: creating a plan costs milliseconds, and a plan's work area must not
// be shared by transforms that may run concurrently (other threads or
// streams).  Kept for the life of the process.
hipfftHandle cached_plan(int d, int n2, int batch, hipfftType type, hipStream_t s) {
  using Key = std::tuple<int, hipStream_t, int, int, int, int>;
  thread_local std::map<Key, hipfftHandle>* cache = new std::map<Key, hipfftHandle>();
  int dev = 0;
  HIF_HIP(hipGetDevice(&dev));
  const Key key{dev, s, d, n2, batch, int(type)};
  auto it = cache->find(key);
  if (it != cache->end()) return it->second;
  int dims[3] = {n2, n2, n2};
  hipfftHandle p;
  fft_check(hipfftPlanMany(&p, d, dims, nullptr, 1, 0, nullptr, 1, 0, type, batch), "plan");
  const hipfftResult r = hipfftSetStream(p, s);
  if (r != HIPFFT_SUCCESS) hipfftDestroy(p);
  fft_check(r, "set stream");
  cache->emplace(key, p);
  return p;
}

// Kernel array over the padded grid: index o per dimension, offset o or
// o - 2n; offsets of magnitude n never pair two points and are left zero.
template <int D>
__global__ void k_fft_kernel_array(double* kr, int n, double h, double w, double self) {
  const int64_t n2 = 2 * int64_t(n);
  int64_t tot = n2 * n2;
  if (D == 3) tot *= n2;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x) {
    int64_t rem = e;
    double r2 = 0.0;
    bool edge = false;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const int o = int(rem % n2);
      rem /= n2;
      const int dlt = o < n ? o : o - int(n2);
      edge = edge || o == n;
      r2 += double(dlt) * double(dlt);
    }
    double v;
    if (edge)
      v = 0.0;
    else if (r2 == 0.0)
      v = self;
    else
      v = green_r2<D>(r2 * h * h) * w;
    kr[e] = v;
  }
}

__global__ void k_fft_zero(double* p, int64_t n) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
    p[e] = 0.0;
}

// P[v][gidx[i]] = s[i] x[v][i]
__global__ void k_fft_scatter(const double* x, const double* s, const int64_t* gidx, double* P, int64_t N,
                              int64_t M) {
  const int v = blockIdx.y;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < N; i += int64_t(gridDim.x) * blockDim.x)
    P[v * M + gidx[i]] = s[i] * x[v * N + i];
}

// S[v][k] *= kh[k]
__global__ void k_fft_mul(hipfftDoubleComplex* S, const hipfftDoubleComplex* kh, int64_t Mh) {
  const int v = blockIdx.y;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < Mh; e += int64_t(gridDim.x) * blockDim.x) {
    const hipfftDoubleComplex a = S[v * Mh + e], b = kh[e];
    S[v * Mh + e] = make_hipDoubleComplex(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
  }
}

// y[v][i] = a[i] x[v][i] + r[i] P[v][gidx[i]] / M
__global__ void k_fft_gather(const double* x, const double* a, const double* r, const int64_t* gidx,
                             const double* P, double* y, int64_t N, int64_t M, double inv) {
  const int v = blockIdx.y;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < N; i += int64_t(gridDim.x) * blockDim.x)
    y[v * N + i] = a[i] * x[v * N + i] + r[i] * (P[v * M + gidx[i]] * inv);
}

// Grid cell of every point if it is a cell centre of the n^d grid with the
// weight and self term of point 0 (else *bad = 1): owner[cell] = i, and the
// padded-grid position in gidx.
template <int D>
__global__ void k_fft_locate(const double* pts, const double* w, const double* sf, int64_t N, int n,
                             int32_t* owner, int64_t* cell_of, int64_t* gidx, int* bad) {
  const double h = 1.0 / n, w0 = w[0], s0 = sf[0];
  const int64_t n2 = 2 * int64_t(n);
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < N; i += int64_t(gridDim.x) * blockDim.x) {
    bool ok = w[i] == w0 && sf[i] == s0;
    int64_t cell = 0, padded = 0, mul = 1, pmul = 1;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double t = pts[i * D + k] / h - 0.5;
      const double g = rint(t);
      ok = ok && g >= 0.0 && g < double(n) && fabs(t - g) <= 1e-9;
      const int64_t gi = ok ? int64_t(g) : 0;
      cell += gi * mul;
      padded += gi * pmul;
      mul *= n;
      pmul *= n2;
    }
    if (!ok) *bad = 1;
    cell_of[i] = cell;
    gidx[i] = padded;
    if (ok) owner[cell] = int32_t(i);
  }
}

// Two points in one cell: one of them does not own it.
__global__ void k_fft_unique(const int32_t* owner, const int64_t* cell_of, int64_t N, int* bad) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < N; i += int64_t(gridDim.x) * blockDim.x)
    if (owner[cell_of[i]] != int32_t(i)) *bad = 1;
}

__global__ void k_fft_flag_init(int* bad) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *bad = 0;
}

}  // namespace

bool fft_ready(hif_factor_s* H, hipStream_t s) {
  if (H->fft_state != 0) return H->fft_state > 0;
  H->fft_state = -1;
  if (H->opts.fft_matvec != 1) return false;
  const int64_t N = H->n;
  const int n = int(std::llround(std::pow(double(N), 1.0 / H->dim)));
  int64_t nd = 1;
  for (int k = 0; k < H->dim; ++k) nd *= n;
  if (n < 1 || nd != N) return false;
  auto F = std::make_unique<FftOp>();
  F->n = n;
  F->d = H->dim;
  const int64_t n2 = 2 * int64_t(n);
  F->M = H->dim == 2 ? n2 * n2 : n2 * n2 * n2;
  F->Mh = (H->dim == 2 ? n2 : n2 * n2) * (int64_t(n) + 1);
  F->gidx.alloc(N, &H->mem);
  {
    DBuf<int32_t> owner;
    DBuf<int64_t> cell_of;
    DBuf<int> bad;
    owner.alloc(N, nullptr);
    cell_of.alloc(N, nullptr);
    bad.alloc(1, nullptr);
    hipLaunchKernelGGL(k_fft_flag_init, dim3(1), dim3(64), 0, s, bad.p);
    if (H->dim == 2)
      hipLaunchKernelGGL(k_fft_locate<2>, dim3(grid1(N)), dim3(kThr), 0, s, H->pts, H->w, H->selfk, N, n, owner.p,
                         cell_of.p, F->gidx.p, bad.p);
    else
      hipLaunchKernelGGL(k_fft_locate<3>, dim3(grid1(N)), dim3(kThr), 0, s, H->pts, H->w, H->selfk, N, n, owner.p,
                         cell_of.p, F->gidx.p, bad.p);
    hipLaunchKernelGGL(k_fft_unique, dim3(grid1(N)), dim3(kThr), 0, s, owner.p, cell_of.p, N, bad.p);
    HIF_HIP(hipGetLastError());
    int hb = 1;
    HIF_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIF_HIP(hipStreamSynchronize(s));
    if (hb) return false;
  }
  double w0 = 0.0, s0 = 0.0;
  HIF_HIP(hipMemcpyAsync(&w0, H->w, sizeof(double), hipMemcpyDeviceToHost, s));
  HIF_HIP(hipMemcpyAsync(&s0, H->selfk, sizeof(double), hipMemcpyDeviceToHost, s));
  HIF_HIP(hipStreamSynchronize(s));
  DBuf<double> kr;
  kr.alloc(F->M, nullptr);
  const double h = 1.0 / n;
  if (H->dim == 2)
    hipLaunchKernelGGL(k_fft_kernel_array<2>, dim3(grid1(F->M)), dim3(kThr), 0, s, kr.p, n, h, w0, s0);
  else
    hipLaunchKernelGGL(k_fft_kernel_array<3>, dim3(grid1(F->M)), dim3(kThr), 0, s, kr.p, n, h, w0, s0);
  HIF_HIP(hipGetLastError());
  F->kh.alloc(F->Mh, &H->mem);
  fft_check(hipfftExecD2Z(cached_plan(H->dim, int(n2), 1, HIPFFT_D2Z, s), kr.p, F->kh.p), "kernel transform");
  H->fft = F.release();
  H->fft_state = 1;
  return true;
}

void fft_release(hif_factor_s* H) {
  delete H->fft;
  H->fft = nullptr;
}

void fft_apply(hif_factor_s* H, const double* x, double* y, int64_t nrhs, bool trans, hipStream_t s) {
  FftOp& F = *H->fft;
  const int nb = int(nrhs);
  const hipfftHandle pf = cached_plan(F.d, 2 * F.n, nb, HIPFFT_D2Z, s);
  const hipfftHandle pi = cached_plan(F.d, 2 * F.n, nb, HIPFFT_Z2D, s);
  const int64_t N = H->n;
  DBuf<double> P;
  DBuf<hipfftDoubleComplex> S;
  P.alloc(size_t(nb) * F.M, nullptr);
  S.alloc(size_t(nb) * F.Mh, nullptr);
  // A^T = diag(a) + diag(c) K diag(b): K is symmetric here
  const double* pre = trans ? H->b : H->c;
  const double* post = trans ? H->c : H->b;
  hipLaunchKernelGGL(k_fft_zero, dim3(grid1(int64_t(nb) * F.M)), dim3(kThr), 0, s, P.p, int64_t(nb) * F.M);
  hipLaunchKernelGGL(k_fft_scatter, dim3(grid1(N), nb), dim3(kThr), 0, s, x, pre, F.gidx.p, P.p, N, F.M);
  HIF_HIP(hipGetLastError());
  fft_check(hipfftExecD2Z(pf, P.p, S.p), "forward transform");
  hipLaunchKernelGGL(k_fft_mul, dim3(grid1(F.Mh), nb), dim3(kThr), 0, s, S.p, F.kh.p, F.Mh);
  HIF_HIP(hipGetLastError());
  fft_check(hipfftExecZ2D(pi, S.p, P.p), "inverse transform");
  hipLaunchKernelGGL(k_fft_gather, dim3(grid1(N), nb), dim3(kThr), 0, s, x, H->a, post, F.gidx.p, P.p, y, N, F.M,
                     1.0 / double(F.M));
  HIF_HIP(hipGetLastError());
}

void apply_A_impl(hif_factor_s* H, const double* x, double* y, int64_t nrhs, bool trans, hipStream_t s) {
  if (fft_ready(H, s)) {
    fft_apply(H, x, y, nrhs, trans, s);
    return;
  }
  if (!trans) {
    matvec_impl(H->pts, H->n, H->dim, H->a, H->b, H->c, H->w, 0.0, H->selfk, 0.0, x, y, nrhs, s);
    return;
  }
  matvec_T_impl(H, x, y, nrhs, s);
}

}  // namespace hif
