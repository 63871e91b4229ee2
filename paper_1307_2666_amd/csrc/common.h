// Internal declarations shared by the HIF-IE library sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "hif.h"

namespace hif {

// ---------------------------------------------------------------------------
// Errors: a status plus a thread-local message; no exceptions cross the ABI.
// ---------------------------------------------------------------------------
struct Error {
  hif_status status;
  std::string msg;
};

void set_error(hif_status s, const std::string& msg);
hif_status fail(hif_status s, const std::string& msg);

#define HIF_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      throw ::hif::Error{HIF_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    }                                                                              \
  } while (0)

#define HIF_REQUIRE(cond, status, msg)                   \
  do {                                                   \
    if (!(cond)) throw ::hif::Error{(status), (msg)};    \
  } while (0)

// ---------------------------------------------------------------------------
// Device memory owned by the library, with an optional cap on the total.
// ---------------------------------------------------------------------------
struct MemTracker {
  size_t held = 0;
  size_t peak = 0;
  size_t cap = 0;  // 0 = no cap
};

// DBuf memory comes from the device's stream-ordered pool: allocations and
// frees are ordered on the stream of the ABI call that makes them (set per
// thread by StreamScope), so a block freed on a stream is reused only after
// the work queued before the free, and freeing does not synchronize the
// device.  The pool keeps freed memory for later calls.
inline hipStream_t& dbuf_stream() {
  static thread_local hipStream_t s = nullptr;
  return s;
}
// While set (ReleaseIdle), blocks released on this thread are known to be
// idle: no queued work on any stream uses them (a handle's teardown after
// waiting on every stream it was used on).  They go to a section of the
// cache that the next allocation of their size class on any stream may take,
// not to the section of the releasing stream.
inline bool& dbuf_idle() {
  static thread_local bool v = false;
  return v;
}
struct ReleaseIdle {
  bool prev;
  ReleaseIdle() : prev(dbuf_idle()) { dbuf_idle() = true; }
  ~ReleaseIdle() { dbuf_idle() = prev; }
  ReleaseIdle(const ReleaseIdle&) = delete;
  ReleaseIdle& operator=(const ReleaseIdle&) = delete;
};
// Cache key of the idle section (no stream has this value).
inline hipStream_t dbuf_idle_key() { return reinterpret_cast<hipStream_t>(~uintptr_t(0)); }
void dbuf_pool_setup();  // once per device: keep freed memory in the pool
// Host-side cache in front of the pool: a block freed on a stream is kept
// (per device and stream, by size class) and handed to the next
// allocation of that class on the same stream, which the stream orders after
// the block's last use; it saves the allocator's per-call host cost between
// the host's waits on the device.  Blocks released as idle (ReleaseIdle) are
// kept in a section any stream may take from.  At most kDbufCacheBytes stay
// cached (per process): a release that would pass the cap first returns the
// oldest idle blocks to the device, and goes back to the pool itself only
// when no idle block is left.  The pool's host cost per call grows with the
// blocks it has seen, so the cap is sized to hold a whole batch
// factorization's working set (its largest blocks alone take about 16 GiB
// for 48 problems of up to 256 x 256): 64 GiB, under a quarter of the 288 GB
// of an MI355X.  An allocation the device cannot serve returns every cached
// block first (dbuf_trim) and tries again.
// Blocks of kDbufDirectBytes or more bypass the pool (plain hipMalloc /
// hipFree: few and large, they would otherwise stay reserved in it) but not
// the cache: mapping and unmapping them takes the host up to hundreds of
// milliseconds once device memory is fragmented, so they are kept for reuse
// like the others and freed only when the cache is full or trimmed.
constexpr size_t kDbufCacheBytes = size_t(64) << 30;
constexpr size_t kDbufDirectBytes = size_t(1) << 30;
size_t dbuf_class(size_t bytes);                  // allocation size for a request
// cached block of at least cls bytes (cls becomes its size) or nullptr
void* dbuf_take(size_t& cls, hipStream_t s);
bool dbuf_give(void* p, size_t cls, hipStream_t s);  // true if cached
void dbuf_trim();  // return every cached and pooled free block to the device
struct StreamScope {
  hipStream_t prev;
  explicit StreamScope(hipStream_t s) : prev(dbuf_stream()) {
    dbuf_pool_setup();
    dbuf_stream() = s;
  }
  ~StreamScope() { dbuf_stream() = prev; }
  StreamScope(const StreamScope&) = delete;
  StreamScope& operator=(const StreamScope&) = delete;
};

template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;        // elements allocated
  size_t cls = 0;      // bytes of the underlying block
  MemTracker* mt = nullptr;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n), cls(o.cls), mt(o.mt) { o.p = nullptr; o.n = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; cls = o.cls; mt = o.mt; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DBuf() { release(); }
  void release() {
    if (p) {
      if (!dbuf_give(p, cls, dbuf_idle() ? dbuf_idle_key() : dbuf_stream())) {
        if (cls >= kDbufDirectBytes)
          (void)hipFree(p);
        else
          (void)hipFreeAsync(p, dbuf_stream());
      }
      if (mt) mt->held -= n * sizeof(T);
    }
    p = nullptr;
    n = 0;
  }
  // Allocate exactly n elements (contents undefined); frees what was held.
  void alloc(size_t cnt, MemTracker* tracker) {
    release();
    mt = tracker;
    if (cnt == 0) return;
    size_t bytes = cnt * sizeof(T);
    if (mt && mt->cap && mt->held + bytes > mt->cap)
      throw Error{HIF_ENOMEM, "device memory cap (opts.max_bytes) exceeded"};
    size_t c = dbuf_class(bytes);
    p = static_cast<T*>(dbuf_take(c, dbuf_stream()));
    if (!p) {
      auto get = [&]() {
        return c >= kDbufDirectBytes ? hipMalloc((void**)&p, c) : hipMallocAsync((void**)&p, c, dbuf_stream());
      };
      hipError_t e = get();
      if (e != hipSuccess) {  // once more after returning free blocks to the device
        (void)hipGetLastError();
        dbuf_trim();
        e = get();
      }
      if (e != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        throw Error{HIF_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
      }
    }
    cls = c;
    n = cnt;
    if (mt) { mt->held += bytes; if (mt->held > mt->peak) mt->peak = mt->held; }
  }
  // Grow-only: keep the allocation if it already holds cnt elements.
  void ensure(size_t cnt, MemTracker* tracker) {
    if (cnt <= n && p) return;
    alloc(cnt < 16 ? 16 : cnt + cnt / 8, tracker);
  }
};

// ---------------------------------------------------------------------------
// Factor records (Lemma 2.4): one per skeletonized index set with r > 0.
//  iarena + idx : rd[r], sk[k], piv[r]           (int32, global DOF ids / pivots)
//  darena + off : T (k x r), E (k x r), G (r x k), LU(B_rr) (r x r), all row-major.
// ---------------------------------------------------------------------------
struct GroupRec {
  int32_t r, k;
  int64_t idx;
  int64_t off;
};

struct SubLevel {
  int level = 0;
  int kind = 0;  // 0 cell, 1 face, 2 edge
  int nrec = 0;
  int max_r = 0, max_k = 0;
  int max_2rk = 0;  // max over records of 2r + k (LDS need of the staged sweeps, per RHS)
  // Record layout: iarena + idx = [rd (r) | sk (k) | piv (r) | perm (r)], where
  // piv are the LU row interchanges and perm the same permutation as a gather
  // index, (P x)[i] = x[perm[i]]; darena + off = [T (k x r) | L_sr (k x r) |
  // U_rs (r x k) | LU (r x r)], row-major.
  std::vector<GroupRec> hrec;
  DBuf<GroupRec> rec;
  // Work offsets of the multi-workgroup solve: record i uses [nv][r] at
  // nv * woff[i] in each of two work regions; sum_r = sum of r.
  DBuf<int64_t> woff;
  int64_t sum_r = 0;
  DBuf<int32_t> iarena;
  DBuf<double> darena;
  // Inverses of the 64 x 64 diagonal blocks of every record's L and U, for
  // the multi-workgroup solve: record i, block b at (i * dinv_nb + b) * 2 *
  // 4096, [L^{-1} | U^{-1}] row-major (built by prepare_sweeps where that
  // solve can run).
  DBuf<double> dinv;
  int dinv_nb = 0;
};

struct FftOp;  // FFT form of the exact operator on a uniform grid (fftmv.hip)

}  // namespace hif

struct hif_factor_s {
  int64_t n = 0;
  int dim = 2;
  int L = 0;
  double eps = 0;
  int leaf = 64;
  hif_opts opts{};
  int symmetric = 1;
  int nproxy = 64;
  double proxy_r = 1.5;
  hif::MemTracker mem;
  // Operator data, caller order: points [n][dim], then a, b, c, w, self [n] each.
  hif::DBuf<double> op;
  const double *pts = nullptr, *a = nullptr, *b = nullptr, *c = nullptr, *w = nullptr, *selfk = nullptr;
  // Factors.
  std::vector<hif::SubLevel> subs;
  int64_t ntop = 0;
  hif::DBuf<int32_t> top_idx, top_piv, top_perm;
  hif::DBuf<double> top_lu;
  // The top block as one record of the many-workgroup solve (k = 0),
  // built on the first solve that needs it: table, [idx | piv | perm], offsets.
  hif::DBuf<hif::GroupRec> top_rec;
  hif::DBuf<int32_t> top_iarena;
  hif::DBuf<int64_t> top_woff;
  hif::DBuf<double> top_dinv;  // its diagonal-block inverses, as SubLevel::dinv
  // Sweep scratch.
  hif::DBuf<double> work;
  // Ticket counter of the chained triangular solves (sweep.hip), cleared by
  // each pass before use.
  hif::DBuf<uint32_t> sync;
  hif_stats_t stats{};
  // Exact operator by FFT: 0 not set up yet, 1 ready (fft), -1 not applicable.
  int fft_state = 0;
  hif::FftOp* fft = nullptr;
  // Copies of one sub-level kept for hif_trace_get (opts.trace_sublevel).
  bool traced = false;
  hif::DBuf<int64_t> tr_gstart, tr_nfstart, tr_yoff, tr_aoff;
  hif::DBuf<int32_t> tr_dofs, tr_nf;
  hif::DBuf<double> tr_Y, tr_Acc;
  // The streams the handle's work was queued on, each with an event recorded
  // after the last such call there: hif_free waits on these events, not on
  // the whole device.
  std::mutex use_mu;
  std::vector<std::pair<hipStream_t, hipEvent_t>> uses;
  hif_factor_s() = default;
  hif_factor_s(const hif_factor_s&) = delete;
  hif_factor_s& operator=(const hif_factor_s&) = delete;
  ~hif_factor_s() {
    for (auto& u : uses) (void)hipEventDestroy(u.second);
  }
};

namespace hif {
// Records that h's work was queued on s up to this point (see uses).
void mark_use(hif_factor_s* h, hipStream_t s);
// Blocks until every call recorded by mark_use has finished on the device.
void wait_uses(hif_factor_s* h);
}  // namespace hif

namespace hif {

// ---------------------------------------------------------------------------
// Kernel functions (eqn laplace-kernel).
// ---------------------------------------------------------------------------
constexpr double kInv2Pi = 0.15915494309189533577;  // 1 / (2 pi)
constexpr double kInv4Pi = 0.07957747154594766788;  // 1 / (4 pi)

// G as a function of the squared distance r2 > 0.
template <int D>
__device__ __forceinline__ double green_r2(double r2) {
  if constexpr (D == 2) {
    return -0.5 * kInv2Pi * log(r2);
  } else {
    return kInv4Pi * rsqrt(r2);
  }
}

// Single-precision G for the mixed-precision assembly.
template <int D>
__device__ __forceinline__ float green_r2f(float r2) {
  if constexpr (D == 2) {
    return -0.5f * float(kInv2Pi) * logf(r2);
  } else {
    return float(kInv4Pi) * rsqrtf(r2);
  }
}

// Kernel value G(r) (r2 = r^2) in the precision of the factorization: FP64,
// or FP32 evaluation in the mixed-precision mode.
template <int D>
__device__ __forceinline__ double green_mixed(double r2, bool f32) {
  return f32 ? double(green_r2f<D>(float(r2))) : green_r2<D>(r2);
}
// An assembled entry, rounded to FP32 in the mixed-precision mode.
__device__ __forceinline__ double entry_prec(double v, bool f32) { return f32 ? double(float(v)) : v; }

// Closed-form integral of G over the element [-h/2, h/2]^d.
inline double self_integral(double h, int d) {
  if (d == 2) return -(h * h / (2.0 * M_PI)) * (std::log(h / std::sqrt(2.0)) - 1.5 + M_PI / 4.0);
  return h * h * (3.0 * std::log(2.0 + std::sqrt(3.0)) - M_PI / 2.0) / (4.0 * M_PI);
}

// Squared distance summed in coordinate order with every product and sum
// rounded separately (no FMA contraction), so equal inputs give the same
// value on any IEEE implementation; on dyadic grids it is exact, so Voronoi
// ties and the strict near-field test are decided exactly.
template <int D>
__device__ __forceinline__ double dist2_exact(const double* x, const double* z) {
#pragma clang fp contract(off)
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double t = x[k] - z[k];
    const double p = t * t;
    s = s + p;
  }
  return s;
}

// Wave / block reductions (wave64).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// Launch helpers implemented in the .hip sources.
// ---------------------------------------------------------------------------
struct Prim;  // rocPRIM wrappers (prim.hip)

// Sort (u64 key) ascending, in place via a double buffer; returns nothing.
void sort_u64(uint64_t* keys, uint64_t* tmp, size_t n, int end_bit, hipStream_t s,
              DBuf<unsigned char>& scratch, MemTracker* mt);
// Sort pairs (u64 key, int32 value) ascending by key (stable).
void sort_u64_i32(uint64_t* keys, uint64_t* ktmp, int32_t* vals, int32_t* vtmp, size_t n,
                  int end_bit, hipStream_t s, DBuf<unsigned char>& scratch, MemTracker* mt);
// Sort pairs (int32 key, int32 value) ascending by key (stable).
void sort_i32_i32(int32_t* keys, int32_t* ktmp, int32_t* vals, int32_t* vtmp, size_t n,
                  int end_bit, hipStream_t s, DBuf<unsigned char>& scratch, MemTracker* mt);
// Exclusive prefix sum of int64 counts; out has n+1 entries (out[n] = total).
void exclusive_scan_i64(const int64_t* in, int64_t* out, size_t n, hipStream_t s,
                        DBuf<unsigned char>& scratch, MemTracker* mt);
void exclusive_scan_i32(const int32_t* in, int32_t* out, size_t n, hipStream_t s,
                        DBuf<unsigned char>& scratch, MemTracker* mt);

// Factorization driver (factor.hip).
void factor_impl(hif_factor_s* H, const double* points, const hif_kernel* k, const double* a,
                 const double* b, const double* c, hipStream_t s);
// Level-synchronous factorization of independent problems together: every
// sub-level runs one launch sequence over the groups of all problems.  The
// handles hold their operators (prepare_problem) and share dim, symmetric
// compression and options; on return each holds its own factors.
void prepare_problem(hif_factor_s* H, const double* points, const hif_kernel* k, const double* a,
                     const double* b, const double* c, hipStream_t s);
void factor_fused_impl(const std::vector<hif_factor_s*>& hs, hipStream_t s);

// Gather form of the LU row interchanges of every record (sweep.hip).
void launch_make_perm(const GroupRec* recs, int nrec, int32_t* iarena, int max_r, hipStream_t s);
void launch_make_perm_top(const int32_t* piv, int32_t* perm, int n, hipStream_t s);

// Sweeps (sweep.hip): op 0 solve, 1 solve_T, 2 apply, 3 apply_T; scratch in
// the handle.  prepare_sweeps builds what the sweeps read besides the factor
// records (called once by the factorization).  sweep_noalloc_impl solves with
// the library's static device scratch of kSolveScratchDoubles doubles.
void sweep_impl(hif_factor_s* H, int op, const double* x, double* y, int64_t nrhs, hipStream_t s);
void prepare_sweeps(hif_factor_s* H, hipStream_t s);
void graph_solve_impl(hif_factor_s* H, const double* f, double* u, int64_t nrhs, hipStream_t cs,
                      hipGraph_t* graph, hipGraphExec_t* exec);
constexpr size_t kSolveScratchDoubles = HIF_SOLVE_NOALLOC_MAX;  // 32 MiB
void sweep_noalloc_impl(hif_factor_s* H, const double* f, double* u, int64_t nrhs, hipStream_t s);

// Right-preconditioned GMRES with the factorization and the exact matvec (gmres.hip).
// With trans, A^T u = f preconditioned by F^{-T}.
void gmres_impl(hif_factor_s* H, const double* f, double* u, int64_t nrhs, double tol, int maxit,
                int32_t* iters, double* relres, bool trans, hipStream_t s);

// Batch workers: destroy the calling thread's look-ahead streams
// (batched.hip), and move the blocks cached for a stream that has been
// synchronized and is about to be destroyed to the idle section, where any
// stream may take them (api.hip); a destroyed stream's own section would
// never be asked for again.
void release_thread_streams();
void dbuf_retire_stream(hipStream_t s);

// y = A^T x pair by pair (gmres.hip).
void matvec_T_impl(hif_factor_s* H, const double* x, double* y, int64_t nrhs, hipStream_t s);

// y = A x or A^T x with the handle's exact operator, by FFT convolution when
// the points form the full uniform grid (fftmv.hip); fft_release frees it.
void apply_A_impl(hif_factor_s* H, const double* x, double* y, int64_t nrhs, bool trans, hipStream_t s);
bool fft_ready(hif_factor_s* H, hipStream_t s);
void fft_release(hif_factor_s* H);

// grad = -sum over right-hand sides of lam (.) u (gmres.hip).
void diag_grad_impl(const double* lam, const double* u, double* grad, int64_t n, int64_t nrhs, hipStream_t s);

// Exact O(n^2) matvec (matvec.hip).
void matvec_impl(const double* pts, int64_t n, int dim, const double* a, const double* b,
                 const double* c, const double* w, double w_const, const double* selfk,
                 double self_const, const double* x, double* y, int64_t nrhs, hipStream_t s);

// Batched ID (dense.hip), the same kernel hif_factor uses.
void id_batched_impl(double* mats, const int64_t* off, const int32_t* rows, const int32_t* cols,
                     const double* tol, int32_t batch, int32_t max_cols, int32_t* rank,
                     int32_t* perm, const int64_t* off_perm, double* T, const int64_t* off_t,
                     hipStream_t s);

// Group assignment (factor.hip).
void partition_impl(const double* pts, int64_t n, int dim, const uint8_t* active, int kind,
                    int32_t S, int32_t* group, hipStream_t s);

// Launch-shape table (hif_tuning_set / hif_tuning_get): a snapshot for the
// dispatching code, and the checked replacement.
hif_tuning tuning();
bool set_tuning(const hif_tuning* t);  // nullptr: the built-in table; false if invalid

inline int ceil_log2(uint64_t v) {
  int b = 0;
  while ((uint64_t(1) << b) < v) ++b;
  return b;
}

}  // namespace hif
