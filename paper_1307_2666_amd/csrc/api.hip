// C ABI entry points (include/hif.h): argument checks on the host, handle
// lifecycle, error mapping.  No exception crosses the ABI.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <iterator>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "batched.h"
#include "common.h"
#include "tuning_gfx950.h"

// A captured solve: the graph and its executable instance.
struct hif_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hif_factor_s* h = nullptr;  // the handle whose factors the graph reads
};

namespace hif {

namespace {
thread_local std::string g_last_error;
}

void set_error(hif_status s, const std::string& msg) {
  (void)s;
  g_last_error = msg;
}

hif_status fail(hif_status s, const std::string& msg) {
  set_error(s, msg);
  return s;
}

void dbuf_pool_setup() {
  static std::mutex mu;
  static std::set<int> done;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  std::lock_guard<std::mutex> lk(mu);
  if (done.count(dev)) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t keep = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  }
  (void)hipGetLastError();
  done.insert(dev);
}

size_t dbuf_class(size_t bytes) {
  if (bytes <= 256) return 256;
  size_t p2 = 256;
  while (p2 < bytes) p2 <<= 1;
  if (p2 <= (size_t(1) << 20)) return p2;
  const size_t step = p2 / 16;  // eighths between the powers of two p2 / 2 and p2
  return (bytes + step - 1) / step * step;
}

namespace {
struct CacheKey {
  int dev;
  hipStream_t s;
  size_t cls;
  bool operator<(const CacheKey& o) const {
    if (dev != o.dev) return dev < o.dev;
    if (s != o.s) return s < o.s;
    return cls < o.cls;
  }
};
// Process-wide and never destroyed (freeing at exit could run after the HIP
// runtime is gone); the memory returns to the system with the process.
struct CacheEntry {
  void* p;
  uint64_t tick;  // when it was cached
};
using CacheMap = std::multimap<CacheKey, CacheEntry>;
struct DbufCache {
  std::mutex mu;
  CacheMap blocks;
  // the idle blocks, oldest first: a release that would pass the cap frees
  // these first (idle blocks have no pending work)
  std::map<uint64_t, CacheMap::iterator> idle_age;
  uint64_t tick = 0;
  size_t bytes = 0;
};
DbufCache& dbuf_cache() {
  static DbufCache* c = new DbufCache;
  return *c;
}
void cache_insert(DbufCache& c, const CacheKey& k, void* p, uint64_t tick) {
  const CacheMap::iterator it = c.blocks.emplace(k, CacheEntry{p, tick});
  if (k.s == dbuf_idle_key()) c.idle_age.emplace(tick, it);
  c.bytes += k.cls;
}
void cache_erase(DbufCache& c, CacheMap::iterator it) {
  if (it->first.s == dbuf_idle_key()) c.idle_age.erase(it->second.tick);
  c.bytes -= it->first.cls;
  c.blocks.erase(it);
}
// Returns a block to the device: blocks of a stream's section after the
// stream's queued work, idle ones at once.
void block_free(void* p, const CacheKey& k) {
  if (k.cls >= kDbufDirectBytes)
    (void)hipFree(p);
  else
    (void)hipFreeAsync(p, k.s == dbuf_idle_key() ? nullptr : k.s);
}
}  // namespace

void* dbuf_take(size_t& cls, hipStream_t s) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  DbufCache& c = dbuf_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  // the smallest cached block of at least cls bytes, up to a quarter more
  // (classes above 1 MiB are sixteenths of a power of two apart; smaller
  // ones are powers of two, so for them this is the exact class)
  auto fit = [&](hipStream_t key) {
    auto it = c.blocks.lower_bound(CacheKey{dev, key, cls});
    const bool ok = it != c.blocks.end() && it->first.dev == dev && it->first.s == key && it->first.cls <= cls + cls / 4;
    return ok ? it : c.blocks.end();
  };
  auto it = fit(s);
  if (it == c.blocks.end()) it = fit(dbuf_idle_key());  // idle blocks serve any stream
  if (it == c.blocks.end()) return nullptr;
  void* p = it->second.p;
  cls = it->first.cls;
  cache_erase(c, it);
  return p;
}

void dbuf_trim() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  {
    DbufCache& c = dbuf_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    for (auto it = c.blocks.begin(); it != c.blocks.end();) {
      const auto nx = std::next(it);
      if (it->first.dev == dev) {
        block_free(it->second.p, it->first);
        cache_erase(c, it);
      }
      it = nx;
    }
  }
  (void)hipDeviceSynchronize();
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
  (void)hipGetLastError();
}

void dbuf_retire_stream(hipStream_t s) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  DbufCache& c = dbuf_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  std::vector<std::pair<CacheKey, CacheEntry>> moved;
  for (auto it = c.blocks.lower_bound(CacheKey{dev, s, 0});
       it != c.blocks.end() && it->first.dev == dev && it->first.s == s;) {
    const auto nx = std::next(it);
    moved.push_back({CacheKey{dev, dbuf_idle_key(), it->first.cls}, it->second});
    cache_erase(c, it);
    it = nx;
  }
  for (const auto& m : moved) cache_insert(c, m.first, m.second.p, m.second.tick);
}

bool dbuf_give(void* p, size_t cls, hipStream_t s) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  DbufCache& c = dbuf_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  // past the cap, the oldest idle blocks of this device go back first: a
  // block just released is the likelier to be asked for again
  for (auto a = c.idle_age.begin(); c.bytes + cls > kDbufCacheBytes && a != c.idle_age.end();) {
    const auto nx = std::next(a);
    const CacheMap::iterator it = a->second;
    if (it->first.dev == dev) {
      block_free(it->second.p, it->first);
      cache_erase(c, it);  // erases a
    }
    a = nx;
  }
  if (c.bytes + cls > kDbufCacheBytes) return false;
  cache_insert(c, CacheKey{dev, s, cls}, p, ++c.tick);
  return true;
}

namespace {
std::mutex g_tune_mu;
hif_tuning builtin_tuning() {
  hif_tuning t{HIF_TUNED_ID_REG_WAVES, HIF_TUNED_LU_PANEL_THREADS, HIF_TUNED_ROWQR_UPDATE_WAVES,
               HIF_TUNED_ROWQR_UPDATE_KIND, HIF_TUNED_SWEEP_MANY_THREADS};
  return t;
}
hif_tuning g_tune = builtin_tuning();
}  // namespace

hif_tuning tuning() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_tune;
}

bool set_tuning(const hif_tuning* t) {
  const hif_tuning v = t ? *t : builtin_tuning();
  auto in = [](int x, std::initializer_list<int> ok) {
    for (int o : ok)
      if (x == o) return true;
    return false;
  };
  if (!in(v.id_reg_waves[0], {4, 8, 16}) || !in(v.id_reg_waves[1], {4, 8, 16}) || !in(v.id_reg_waves[2], {8, 16}) ||
      !in(v.lu_panel_threads[0], {256, 512, 1024}) || !in(v.lu_panel_threads[1], {512, 1024}) ||
      !in(v.rowqr_update_waves, {4, 8}) || !in(v.rowqr_update_kind, {0, 1, 2}) ||
      !in(v.sweep_many_threads, {64, 128, 256}))
    return false;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune = v;
  return true;
}

void mark_use(hif_factor_s* h, hipStream_t s) {
  std::lock_guard<std::mutex> lk(h->use_mu);
  for (auto& u : h->uses)
    if (u.first == s) {
      HIF_HIP(hipEventRecord(u.second, s));
      return;
    }
  hipEvent_t e = nullptr;
  HIF_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  h->uses.emplace_back(s, e);
  HIF_HIP(hipEventRecord(e, s));
}

void wait_uses(hif_factor_s* h) {
  std::lock_guard<std::mutex> lk(h->use_mu);
  for (auto& u : h->uses) (void)hipEventSynchronize(u.second);
}

// Runs f with DBuf memory ordered on stream s; errors become a status.
template <class F>
hif_status guarded(hipStream_t s, F&& f) {
  try {
    g_last_error.clear();
    StreamScope scope(s);
    f();
    return HIF_OK;
  } catch (const Error& e) {
    return fail(e.status, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(HIF_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(HIF_EDEVICE, e.what());
  } catch (...) {
    return fail(HIF_EDEVICE, "unknown error");
  }
}

static hif_status check_kernel(const hif_kernel* k) {
  if (!k) return fail(HIF_EINVAL, "kernel description is NULL");
  if (!(k->weights && k->self) && !(std::isfinite(k->h) && k->h > 0.0))
    return fail(HIF_EINVAL, "kernel.h must be finite and > 0 unless weights and self are both given");
  return HIF_OK;
}

}  // namespace hif

using namespace hif;

extern "C" {

hif_status hif_opts_default(hif_opts* o) {
  if (!o) return fail(HIF_EINVAL, "opts is NULL");
  o->precision = HIF_FP64;
  o->second_kind = -1;
  o->symmetric = -1;
  o->variant = HIF_VARIANT_HIFIE;
  o->n_proxy = 0;
  o->proxy_radius = 0.0;
  o->max_bytes = 0;
  o->row_compression = -1;
  o->fft_matvec = 0;
  o->trace_sublevel = -1;
  o->sweep_wait_us = 0;
  return HIF_OK;
}

const char* hif_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// Checks of hif_factor's problem arguments (everything but the handle).
static hif_status check_problem(const double* points, int64_t n, int dim, const hif_kernel* k, double eps,
                                int32_t leaf) {
  if (!points) return fail(HIF_EINVAL, "points is NULL");
  if (n < 1) return fail(HIF_EINVAL, "n must be >= 1");
  if (n > int64_t(INT32_MAX) - 1) return fail(HIF_EINVAL, "n must fit in int32");
  if (dim != 2 && dim != 3) return fail(HIF_EINVAL, "dim must be 2 or 3");
  if (hif_status s = check_kernel(k); s != HIF_OK) return s;
  if (!(eps > 0.0 && eps < 1.0)) return fail(HIF_EINVAL, "eps must satisfy 0 < eps < 1");
  if (leaf < 1) return fail(HIF_EINVAL, "leaf must be >= 1");
  return HIF_OK;
}

// Options with the defaults filled in and checked.
static hif_status resolve_opts(const hif_opts* opts, hif_opts* out) {
  hif_opts o;
  hif_opts_default(&o);
  if (opts) o = *opts;
  if (o.precision != HIF_FP64 && o.precision != HIF_FP32_MIXED)
    return fail(HIF_EINVAL, "opts.precision must be HIF_FP64 or HIF_FP32_MIXED");
  if (o.second_kind < -1 || o.second_kind > 1) return fail(HIF_EINVAL, "opts.second_kind must be -1, 0 or 1");
  if (o.symmetric < -1 || o.symmetric > 1) return fail(HIF_EINVAL, "opts.symmetric must be -1, 0 or 1");
  if (o.variant != HIF_VARIANT_HIFIE && o.variant != HIF_VARIANT_RSF)
    return fail(HIF_EINVAL, "opts.variant must be HIF_VARIANT_HIFIE or HIF_VARIANT_RSF");
  if (o.n_proxy < 0 || o.n_proxy > 8192) return fail(HIF_EINVAL, "opts.n_proxy must be in [0, 8192]");
  if (o.row_compression < -1 || o.row_compression > 1)
    return fail(HIF_EINVAL, "opts.row_compression must be -1, 0 or 1");
  if (o.fft_matvec != 0 && o.fft_matvec != 1) return fail(HIF_EINVAL, "opts.fft_matvec must be 0 or 1");
  if (o.sweep_wait_us < 0) return fail(HIF_EINVAL, "opts.sweep_wait_us must be >= 0");
  if (o.trace_sublevel < -1 || o.trace_sublevel >= HIF_MAX_SUBLEVELS)
    return fail(HIF_EINVAL, "opts.trace_sublevel must be -1 or a sub-level index");
  if (!(o.proxy_radius == 0.0 || (std::isfinite(o.proxy_radius) && o.proxy_radius > 0.5)))
    return fail(HIF_EINVAL, "opts.proxy_radius must be 0 (default) or > 0.5 cell widths");
  // second-kind modification by default in FP64 only: in FP32 the SCI-scaled
  // tolerance rho * eps falls below single-precision resolution
  if (o.second_kind < 0) o.second_kind = o.precision == HIF_FP64 ? 1 : 0;
  *out = o;
  return HIF_OK;
}

static std::unique_ptr<hif_factor_s> new_handle(int64_t n, int dim, double eps, int32_t leaf, const hif_opts& o) {
  std::unique_ptr<hif_factor_s> h(new hif_factor_s());
  h->n = n;
  h->dim = dim;
  h->eps = eps;
  h->leaf = leaf;
  h->opts = o;
  h->nproxy = o.n_proxy ? o.n_proxy : (dim == 2 ? 64 : 512);
  h->proxy_r = o.proxy_radius > 0.0 ? o.proxy_radius : 1.5;
  h->mem.cap = o.max_bytes;
  return h;
}

extern "C" {

hif_status hif_factor(const double* points, int64_t n, int dim, const hif_kernel* k, const double* a,
                      const double* b, const double* c, double eps, int32_t leaf, const hif_opts* opts,
                      hif_stream stream, hif_handle* out) {
  if (!out) return fail(HIF_EINVAL, "out is NULL");
  *out = nullptr;
  if (hif_status st = check_problem(points, n, dim, k, eps, leaf); st != HIF_OK) return st;
  hif_opts o;
  if (hif_status st = resolve_opts(opts, &o); st != HIF_OK) return st;
  hif_handle H = nullptr;
  hif_status st = guarded(hipStream_t(stream), [&] {
    std::unique_ptr<hif_factor_s> h = new_handle(n, dim, eps, leaf, o);
    factor_impl(h.get(), points, k, a, b, c, hipStream_t(stream));
    mark_use(h.get(), hipStream_t(stream));
    H = h.release();
  });
  if (st == HIF_OK) *out = H;
  return st;
}

// Level-synchronous factorization of the whole batch (nworkers == 0): every
// problem is checked and set up on its own (a failure stays with its
// problem), then the problems that share dim and the symmetric compression
// are factored together, each sub-level one launch sequence over all of
// them; a failure there is reported for every problem of that set.
static hif_status factor_batch_fused(const hif_problem* problems, int32_t count, const hif_opts* opts,
                                     hif_handle* out, std::vector<hif_status>& st, std::vector<std::string>& msg) {
  hif_opts o;
  if (hif_status e = resolve_opts(opts, &o); e != HIF_OK) return e;
  bool any = false;
  for (int32_t p = 0; p < count; ++p) {
    const hif_problem& q = problems[p];
    st[p] = check_problem(q.points, q.n, q.dim, &q.kernel, q.eps, q.leaf);
    if (st[p] != HIF_OK) msg[p] = g_last_error;
    any = any || st[p] == HIF_OK;
  }
  if (!any) return HIF_OK;
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
    return fail(HIF_EDEVICE, "creating the batch stream failed");
  std::vector<std::unique_ptr<hif_factor_s>> hs(count);
  for (int32_t p = 0; p < count; ++p) {
    const hif_problem& q = problems[p];
    if (st[p] == HIF_OK)
      st[p] = guarded(s, [&] {
        std::unique_ptr<hif_factor_s> h = new_handle(q.n, q.dim, q.eps, q.leaf, o);
        prepare_problem(h.get(), q.points, &q.kernel, q.a, q.b, q.c, s);
        hs[p] = std::move(h);
      });
    if (st[p] != HIF_OK) msg[p] = g_last_error;
  }
  // sets of problems that can share launches: same dim and symmetric compression
  std::vector<char> done(count, 0);
  for (int32_t p = 0; p < count; ++p) {
    if (!hs[p] || done[p]) continue;
    std::vector<int32_t> set;
    for (int32_t q = p; q < count; ++q)
      if (hs[q] && !done[q] && hs[q]->dim == hs[p]->dim && hs[q]->symmetric == hs[p]->symmetric) {
        set.push_back(q);
        done[q] = 1;
      }
    std::vector<hif_factor_s*> ptrs;
    for (int32_t q : set) ptrs.push_back(hs[q].get());
    const hif_status e = guarded(s, [&] { factor_fused_impl(ptrs, s); });
    for (int32_t q : set) {
      if (e == HIF_OK) {
        out[q] = hs[q].release();
      } else {
        st[q] = e;
        msg[q] = g_last_error;
        guarded(s, [&] { hs[q].reset(); });
      }
    }
  }
  (void)hipStreamSynchronize(s);
  release_thread_streams();
  dbuf_retire_stream(s);
  (void)hipStreamDestroy(s);
  return HIF_OK;
}

static hif_status factor_batch(const hif_problem* problems, int32_t count, const hif_opts* opts, int32_t nworkers,
                               hif_handle* out, hif_status* status) {
  if (count < 0) return fail(HIF_EINVAL, "count must be >= 0");
  if (count > 0 && (!problems || !out)) return fail(HIF_EINVAL, "problems and out must not be NULL");
  if (nworkers < 0 || nworkers > 16) return fail(HIF_EINVAL, "nworkers must be in [0, 16]");
  for (int32_t p = 0; p < count; ++p) {
    out[p] = nullptr;
    if (status) status[p] = HIF_OK;
  }
  if (count == 0) return HIF_OK;
  if (nworkers == 0) {
    std::vector<hif_status> st(count, HIF_OK);
    std::vector<std::string> msg(count);
    if (hif_status e = factor_batch_fused(problems, count, opts, out, st, msg); e != HIF_OK) return e;
    hif_status first = HIF_OK;
    std::string first_msg;
    for (int32_t p = 0; p < count; ++p) {
      if (status) status[p] = st[p];
      if (st[p] != HIF_OK && first == HIF_OK) {
        first = st[p];
        first_msg = "problem " + std::to_string(p) + ": " + msg[p];
      }
    }
    if (first != HIF_OK) return fail(first, first_msg);
    g_last_error.clear();
    return HIF_OK;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(HIF_EDEVICE, "no current HIP device");
  // largest problems first, so that the last ones to start are short
  std::vector<int32_t> order(count);
  for (int32_t p = 0; p < count; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t x, int32_t y) { return problems[x].n > problems[y].n; });
  std::vector<hif_status> st(count, HIF_OK);
  std::vector<std::string> msg(count);
  std::atomic<int32_t> next{0};
  std::atomic<int> setup_failed{0};
  auto work = [&]() {
    if (hipSetDevice(dev) != hipSuccess) {
      setup_failed = 1;
      return;
    }
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      setup_failed = 1;
      return;
    }
    for (;;) {
      const int32_t i = next++;
      if (i >= count) break;
      const int32_t p = order[i];
      const hif_problem& q = problems[p];
      hif_handle h = nullptr;
      st[p] = hif_factor(q.points, q.n, q.dim, &q.kernel, q.a, q.b, q.c, q.eps, q.leaf, opts, s, &h);
      if (st[p] != HIF_OK) msg[p] = g_last_error;
      out[p] = h;
    }
    // every handle's device work is complete when the batch returns; the
    // thread's streams are destroyed and the blocks cached for them become
    // idle blocks that any stream may take
    (void)hipStreamSynchronize(s);
    release_thread_streams();
    dbuf_retire_stream(s);
    (void)hipStreamDestroy(s);
  };
  {
    // workers that could not be started leave their share to the others
    // (or to this thread), which drain the same queue
    std::vector<std::thread> pool;
    const int nw = std::min<int>(nworkers, count);
    pool.reserve(nw);
    for (int w = 0; w < nw; ++w) {
      try {
        pool.emplace_back(work);
      } catch (const std::system_error&) {
        break;
      }
    }
    if (pool.empty()) work();
    for (auto& t : pool) t.join();
  }
  if (setup_failed) {
    for (int32_t p = 0; p < count; ++p)
      if (out[p] == nullptr && st[p] == HIF_OK) st[p] = HIF_EDEVICE;
  }
  hif_status first = HIF_OK;
  std::string first_msg;
  for (int32_t p = 0; p < count; ++p) {
    if (status) status[p] = st[p];
    if (st[p] != HIF_OK && first == HIF_OK) {
      first = st[p];
      first_msg = "problem " + std::to_string(p) + ": " + (msg[p].empty() ? "worker setup failed" : msg[p]);
    }
  }
  if (first != HIF_OK) return fail(first, first_msg);
  g_last_error.clear();
  return HIF_OK;
}

hif_status hif_factor_batch(const hif_problem* problems, int32_t count, const hif_opts* opts, int32_t nworkers,
                            hif_handle* out, hif_status* status) {
  try {
    return factor_batch(problems, count, opts, nworkers, out, status);
  } catch (const std::exception& e) {  // thread creation or host allocation
    return fail(HIF_EDEVICE, std::string("batch scheduling failed: ") + e.what());
  }
}

static hif_status sweep(hif_handle h, int op, const double* x, double* y, int64_t nrhs, hif_stream s) {
  if (!h) return fail(HIF_EINVAL, "handle is NULL");
  if (!x || !y) return fail(HIF_EINVAL, "vector pointer is NULL");
  if (nrhs < 1) return fail(HIF_EINVAL, "nrhs must be >= 1");
  return guarded(hipStream_t(s), [&] {
    sweep_impl(h, op, x, y, nrhs, hipStream_t(s));
    mark_use(h, hipStream_t(s));
  });
}

hif_status hif_solve(hif_handle h, const double* f, double* u, int64_t nrhs, hif_stream s) {
  return sweep(h, 0, f, u, nrhs, s);
}
hif_status hif_solve_T(hif_handle h, const double* f, double* u, int64_t nrhs, hif_stream s) {
  return sweep(h, 1, f, u, nrhs, s);
}
hif_status hif_apply(hif_handle h, const double* x, double* y, int64_t nrhs, hif_stream s) {
  return sweep(h, 2, x, y, nrhs, s);
}
hif_status hif_apply_T(hif_handle h, const double* x, double* y, int64_t nrhs, hif_stream s) {
  return sweep(h, 3, x, y, nrhs, s);
}

hif_status hif_solve_graph(hif_handle h, const double* f, double* u, int64_t nrhs, hif_graph* out) {
  if (!out) return fail(HIF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!h) return fail(HIF_EINVAL, "handle is NULL");
  if (!f || !u) return fail(HIF_EINVAL, "vector pointer is NULL");
  if (nrhs < 1) return fail(HIF_EINVAL, "nrhs must be >= 1");
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
    return fail(HIF_EDEVICE, "creating the capture stream failed");
  std::unique_ptr<hif_graph_s> g(new (std::nothrow) hif_graph_s());
  if (g) g->h = h;
  hif_status st = g ? guarded(cs, [&] { graph_solve_impl(h, f, u, nrhs, cs, &g->graph, &g->exec); })
                    : fail(HIF_ENOMEM, "host allocation failed");
  (void)hipStreamSynchronize(cs);
  dbuf_retire_stream(cs);
  (void)hipStreamDestroy(cs);
  if (st == HIF_OK) *out = g.release();
  return st;
}

hif_status hif_graph_launch(hif_graph g, hif_stream s) {
  if (!g) return fail(HIF_EINVAL, "graph is NULL");
  const hipError_t e = hipGraphLaunch(g->exec, hipStream_t(s));
  if (e != hipSuccess) return fail(HIF_EDEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
  return guarded(hipStream_t(s), [&] { mark_use(g->h, hipStream_t(s)); });
}

void hif_graph_free(hif_graph g) {
  if (!g) return;
  wait_uses(g->h);  // its replays are recorded on the handle, which outlives the graph
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

hif_status hif_solve_noalloc(hif_handle h, const double* f, double* u, int64_t nrhs, hif_stream s) {
  if (!h) return fail(HIF_EINVAL, "handle is NULL");
  if (!f || !u) return fail(HIF_EINVAL, "vector pointer is NULL");
  if (nrhs < 1) return fail(HIF_EINVAL, "nrhs must be >= 1");
  // no StreamScope: this call never touches the handle's pooled buffers
  try {
    g_last_error.clear();
    sweep_noalloc_impl(h, f, u, nrhs, hipStream_t(s));
    mark_use(h, hipStream_t(s));
    return HIF_OK;
  } catch (const Error& e) {
    return fail(e.status, e.msg);
  } catch (const std::exception& e) {
    return fail(HIF_EDEVICE, e.what());
  } catch (...) {
    return fail(HIF_EDEVICE, "unknown error");
  }
}

hif_status hif_matvec(const double* points, int64_t n, int dim, const hif_kernel* k, const double* a,
                      const double* b, const double* c, const double* x, double* y, int64_t nrhs, hif_stream s) {
  if (!points || !x || !y) return fail(HIF_EINVAL, "NULL pointer argument");
  if (x == y) return fail(HIF_EINVAL, "y must not alias x");
  if (n < 1) return fail(HIF_EINVAL, "n must be >= 1");
  if (dim != 2 && dim != 3) return fail(HIF_EINVAL, "dim must be 2 or 3");
  if (nrhs < 1) return fail(HIF_EINVAL, "nrhs must be >= 1");
  if (hif_status st = check_kernel(k); st != HIF_OK) return st;
  return guarded(hipStream_t(s), [&] {
    const double wc = k->weights ? 0.0 : std::pow(k->h, dim);
    const double sc = k->self ? 0.0 : self_integral(k->h, dim);
    matvec_impl(points, n, dim, a, b, c, k->weights, wc, k->self, sc, x, y, nrhs, hipStream_t(s));
  });
}

static hif_status gmres_any(hif_handle h, const double* f, double* u, int64_t nrhs, double tol, int32_t maxit,
                            int32_t* iters, double* relres, bool trans, hif_stream s) {
  if (!h) return fail(HIF_EINVAL, "handle is NULL");
  if (!f || !u) return fail(HIF_EINVAL, "vector pointer is NULL");
  if (f == u) return fail(HIF_EINVAL, "u must not alias f");
  if (nrhs < 1 || nrhs > 64) return fail(HIF_EINVAL, "nrhs must be in [1, 64]");
  if (!(tol > 0.0 && tol < 1.0)) return fail(HIF_EINVAL, "tol must satisfy 0 < tol < 1");
  if (maxit < 1 || maxit > 200) return fail(HIF_EINVAL, "maxit must be in [1, 200]");
  return guarded(hipStream_t(s),
                 [&] {
                   gmres_impl(h, f, u, nrhs, tol, maxit, iters, relres, trans, hipStream_t(s));
                   mark_use(h, hipStream_t(s));
                 });
}

hif_status hif_gmres(hif_handle h, const double* f, double* u, int64_t nrhs, double tol, int32_t maxit,
                     int32_t* iters, double* relres, hif_stream s) {
  return gmres_any(h, f, u, nrhs, tol, maxit, iters, relres, false, s);
}

hif_status hif_gmres_T(hif_handle h, const double* f, double* u, int64_t nrhs, double tol, int32_t maxit,
                       int32_t* iters, double* relres, hif_stream s) {
  return gmres_any(h, f, u, nrhs, tol, maxit, iters, relres, true, s);
}

hif_status hif_diag_grad(const double* lambda, const double* u, double* grad, int64_t n, int64_t nrhs,
                         hif_stream s) {
  if (!lambda || !u || !grad) return fail(HIF_EINVAL, "NULL pointer argument");
  if (n < 1) return fail(HIF_EINVAL, "n must be >= 1");
  if (nrhs < 1) return fail(HIF_EINVAL, "nrhs must be >= 1");
  if (grad == lambda || grad == u) return fail(HIF_EINVAL, "grad must not alias lambda or u");
  return guarded(hipStream_t(s), [&] { diag_grad_impl(lambda, u, grad, n, nrhs, hipStream_t(s)); });
}

hif_status hif_stats(hif_handle h, hif_stats_t* out) {
  if (!h || !out) return fail(HIF_EINVAL, "NULL argument");
  *out = h->stats;
  return HIF_OK;
}

void hif_free(hif_handle h) {
  if (!h) return;
  wait_uses(h);  // the handle's own work on every stream it was used on
  StreamScope scope(nullptr);
  ReleaseIdle idle;  // waited on above: the handle's blocks are idle
  fft_release(h);
  delete h;
}

hif_status hif_apply_A(hif_handle h, const double* x, double* y, int64_t nrhs, int transpose, int32_t* used_fft,
                       hif_stream s) {
  if (!h) return fail(HIF_EINVAL, "handle is NULL");
  if (!x || !y) return fail(HIF_EINVAL, "vector pointer is NULL");
  if (x == y) return fail(HIF_EINVAL, "y must not alias x");
  if (nrhs < 1 || nrhs > 64) return fail(HIF_EINVAL, "nrhs must be in [1, 64]");
  if (transpose != 0 && transpose != 1) return fail(HIF_EINVAL, "transpose must be 0 or 1");
  return guarded(hipStream_t(s), [&] {
    apply_A_impl(h, x, y, nrhs, transpose == 1, hipStream_t(s));
    mark_use(h, hipStream_t(s));
    if (used_fft) *used_fft = h->fft_state > 0 ? 1 : 0;
  });
}

hif_status hif_id_batched(double* mats, const int64_t* off, const int32_t* rows, const int32_t* cols,
                          const double* tol, int32_t batch, int32_t max_cols, int32_t* rank, int32_t* perm,
                          const int64_t* off_perm, double* T, const int64_t* off_t, hif_stream s) {
  if (batch < 0) return fail(HIF_EINVAL, "batch must be >= 0");
  if (batch == 0) return HIF_OK;
  if (!mats || !off || !rows || !cols || !tol || !rank || !perm || !off_perm)
    return fail(HIF_EINVAL, "NULL pointer argument");
  if ((T == nullptr) != (off_t == nullptr)) return fail(HIF_EINVAL, "T and off_t must both be given or both NULL");
  if (max_cols < 1 || max_cols > 4096) return fail(HIF_EINVAL, "max_cols must be in [1, 4096]");
  return guarded(hipStream_t(s), [&] {
    id_batched_impl(mats, off, rows, cols, tol, batch, max_cols, rank, perm, off_perm, T, off_t, hipStream_t(s));
  });
}

hif_status hif_trace_get(hif_handle h, int item, void* dst, int64_t cap, int64_t* count) {
  if (!h) return fail(HIF_EINVAL, "handle is NULL");
  if (!count) return fail(HIF_EINVAL, "count is NULL");
  if (!h->traced) return fail(HIF_EINVAL, "the factorization kept no trace (opts.trace_sublevel)");
  const void* src = nullptr;
  size_t esz = 0;
  int64_t n = 0;
  switch (item) {
    case HIF_TRACE_GROUP_START: src = h->tr_gstart.p; esz = 8; n = int64_t(h->tr_gstart.n); break;
    case HIF_TRACE_GROUP_DOFS: src = h->tr_dofs.p; esz = 4; n = int64_t(h->tr_dofs.n); break;
    case HIF_TRACE_NEAR_START: src = h->tr_nfstart.p; esz = 8; n = int64_t(h->tr_nfstart.n); break;
    case HIF_TRACE_NEAR_DOFS: src = h->tr_nf.p; esz = 4; n = int64_t(h->tr_nf.n); break;
    case HIF_TRACE_Y_OFF: src = h->tr_yoff.p; esz = 8; n = int64_t(h->tr_yoff.n); break;
    case HIF_TRACE_Y: src = h->tr_Y.p; esz = 8; n = int64_t(h->tr_Y.n); break;
    case HIF_TRACE_ACC_OFF: src = h->tr_aoff.p; esz = 8; n = int64_t(h->tr_aoff.n); break;
    case HIF_TRACE_ACC: src = h->tr_Acc.p; esz = 8; n = int64_t(h->tr_Acc.n); break;
    default: return fail(HIF_EINVAL, "unknown trace item");
  }
  *count = n;
  if (cap == 0 || n == 0) return HIF_OK;
  if (!dst) return fail(HIF_EINVAL, "dst is NULL");
  if (cap < n) return fail(HIF_ENOMEM, "dst holds fewer elements than the item");
  if (hipMemcpy(dst, src, esz * size_t(n), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(HIF_EDEVICE, "copying the trace to the host failed");
  return HIF_OK;
}

hif_status hif_tuning_get(hif_tuning* out) {
  if (!out) return fail(HIF_EINVAL, "out is NULL");
  *out = tuning();
  return HIF_OK;
}

hif_status hif_tuning_set(const hif_tuning* t) {
  if (!set_tuning(t)) return fail(HIF_EINVAL, "launch-shape table entry outside the allowed values");
  return HIF_OK;
}

hif_status hif_lu_batched(double* mats, const int64_t* off, const int32_t* n, const int32_t* r, int32_t* piv,
                          const int64_t* poff, int32_t batch, int32_t max_n, int32_t max_r, int32_t* status,
                          hif_stream s) {
  if (batch < 0) return fail(HIF_EINVAL, "batch must be >= 0");
  if (batch == 0) return HIF_OK;
  if (!mats || !off || !n || !r || !piv || !poff || !status) return fail(HIF_EINVAL, "NULL pointer argument");
  if (max_n < 1 || max_r < 0 || max_r > max_n) return fail(HIF_EINVAL, "need 0 <= max_r <= max_n and max_n >= 1");
  return guarded(hipStream_t(s), [&] {
    int32_t* st = status;
    LuBatch lb{};
    lb.base = mats;
    lb.moff = off;
    lb.n = n;
    lb.r = r;
    lb.piv = piv;
    lb.poff = poff;
    lb.status = st;
    lb.nprob = batch;
    launch_lu_batched(lb, max_r, max_n, hipStream_t(s));
  });
}

hif_status hif_partition(const double* points, int64_t n, int dim, const uint8_t* active, int kind, int32_t S,
                         int32_t* group, hif_stream s) {
  if (!points || !active || !group) return fail(HIF_EINVAL, "NULL pointer argument");
  if (n < 1) return fail(HIF_EINVAL, "n must be >= 1");
  if (dim != 2 && dim != 3) return fail(HIF_EINVAL, "dim must be 2 or 3");
  if (kind < 0 || kind > 2 || (kind == 1 && dim != 3)) return fail(HIF_EINVAL, "kind must be 0 (cell), 1 (face, 3D) or 2 (edge)");
  if (S < 1 || S > (1 << 20)) return fail(HIF_EINVAL, "S must be in [1, 2^20]");
  return guarded(hipStream_t(s), [&] { partition_impl(points, n, dim, active, kind, S, group, hipStream_t(s)); });
}

}  // extern "C"
