// HIF-IE / RSF factorization driver (Algorithms 3.1, 4.1, 4.2) and the index
// bookkeeping kernels it needs: tree depth, cell / face / edge partitions,
// near fields, split classes, and the store of Schur-complement interactions
// (SCIs).  The host only sequences launches and turns per-group sizes that
// depend on the ranks into offsets (one read-back per stage of a sub-level).
#include <algorithm>
#include <chrono>
#include <climits>
#include <numeric>

#include "batched.h"
#include "kernels.h"

namespace hif {

namespace {

constexpr int kThreads = 256;

inline unsigned nblocks(int64_t n, int t = kThreads) {
  int64_t b = (n + t - 1) / t;
  if (b < 1) b = 1;
  if (b > (1 << 20)) b = 1 << 20;
  return unsigned(b);
}

#define GRID_STRIDE(i, n) \
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < (n); i += int64_t(gridDim.x) * blockDim.x)

// ---------------------------------------------------------------------------
// Small utility kernels.
// ---------------------------------------------------------------------------
__global__ void k_iota(int32_t* a, int64_t n) { GRID_STRIDE(i, n) a[i] = int32_t(i); }
__global__ void k_fill_u8(uint8_t* a, int64_t n, uint8_t v) { GRID_STRIDE(i, n) a[i] = v; }
__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v) { GRID_STRIDE(i, n) a[i] = v; }
__global__ void k_fill_i64(int64_t* a, int64_t n, int64_t v) { GRID_STRIDE(i, n) a[i] = v; }
__global__ void k_fill_f64(double* a, int64_t n, double v) { GRID_STRIDE(i, n) a[i] = v; }
__global__ void k_copy_f64(const double* x, double* y, int64_t n) { GRID_STRIDE(i, n) y[i] = x[i]; }

// Input checks: bit 1 non-finite point, bit 2 point outside [0,1]^d,
// bit 4 non-finite coefficient / weight / self term.
__global__ void k_validate(const double* pts, int64_t n, int dim, const double* a, const double* b,
                           const double* c, const double* w, const double* sf, int32_t* flags) {
  GRID_STRIDE(i, n) {
    int f = 0;
    for (int k = 0; k < dim; ++k) {
      double x = pts[i * dim + k];
      if (!isfinite(x)) f |= 1;
      else if (x < 0.0 || x > 1.0) f |= 2;
    }
    if (!isfinite(a[i]) || !isfinite(b[i]) || !isfinite(c[i]) || !isfinite(w[i]) || !isfinite(sf[i])) f |= 4;
    if (f) atomicOr(flags, f);
  }
}

template <int D>
__device__ __forceinline__ void box_of(const double* x, int S, int* j) {
#pragma unroll
  for (int k = 0; k < D; ++k) {
    int v = int(floor(x[k] * double(S)));
    j[k] = v < 0 ? 0 : (v > S - 1 ? S - 1 : v);
  }
}

template <int D>
__device__ __forceinline__ int flat_box(const int* j, int S) {
  int f = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) f = f * S + j[k];
  return f;
}

template <int D>
__global__ void k_box_count(const double* pts, int64_t n, int S, int32_t* counts) {
  GRID_STRIDE(i, n) {
    int j[D];
    box_of<D>(pts + i * D, S, j);
    atomicAdd(&counts[flat_box<D>(j, S)], 1);
  }
}

__global__ void k_minmax(const int32_t* counts, int64_t m, int32_t* mm) {
  GRID_STRIDE(i, m) {
    atomicMin(&mm[0], counts[i]);
    atomicMax(&mm[1], counts[i]);
  }
}

// ---------------------------------------------------------------------------
// Partitions (Sections 3.1, 4.1, 4.2).  Centre families in the paper's order:
// 2D edges: x-integer, y-integer; 3D faces: x-, y-, z-integer; 3D edges:
// (x,y)-, (x,z)-, (y,z)-integer.  An integer coordinate takes m w for
// m = 1..S-1, a half coordinate (m + 1/2) w for m = 0..S-1; within a family
// the index is lexicographic with the first coordinate slowest.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ int family_mask(int kind, int fam) {
  if (kind == 1) return 1 << fam;  // faces
  if (D == 2) return 1 << fam;     // 2D edges
  return fam == 0 ? 3 : (fam == 1 ? 5 : 6);
}

template <int D>
__device__ __forceinline__ int family_count(int kind) {
  return kind == 0 ? 1 : (D == 2 ? 2 : 3);
}

template <int D>
__device__ int group_key(const double* x, int kind, int S) {
#pragma clang fp contract(off)
  int j[D];
  box_of<D>(x, S, j);
  if (kind == 0) return flat_box<D>(j, S);
  const double w = 1.0 / double(S);
  double best = INFINITY;
  int bidx = -1, off = 0;
  const int nf = family_count<D>(kind);
  for (int fam = 0; fam < nf; ++fam) {
    const int mask = family_mask<D>(kind, fam);
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0}, base[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
    int fsize = 1;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const bool integ = (mask >> k) & 1;
      base[k] = integ ? 1 : 0;
      cnt[k] = integ ? S - 1 : S;
      lo[k] = integ ? max(1, j[k] - 2) : max(0, j[k] - 2);
      hi[k] = integ ? min(S - 1, j[k] + 3) : min(S - 1, j[k] + 2);
      fsize *= cnt[k];
    }
    if (fsize > 0) {
      for (int m0 = lo[0]; m0 <= hi[0]; ++m0)
        for (int m1 = lo[1]; m1 <= hi[1]; ++m1)
          for (int m2 = (D == 3 ? lo[2] : 0); m2 <= (D == 3 ? hi[2] : 0); ++m2) {
            const int mm[3] = {m0, m1, m2};
            double z[D];
#pragma unroll
            for (int k = 0; k < D; ++k)
              z[k] = ((mask >> k) & 1) ? double(mm[k]) * w : (double(mm[k]) + 0.5) * w;
            const double d2 = dist2_exact<D>(x, z);
            if (d2 < best) {
              best = d2;
              int idx = 0;
#pragma unroll
              for (int k = 0; k < D; ++k) idx = idx * cnt[k] + (mm[k] - base[k]);
              bidx = off + idx;
            }
          }
    }
    off += fsize;
  }
  return bidx;
}

template <int D>
__device__ void centre_of(int key, int kind, int S, double* z) {
#pragma clang fp contract(off)
  const double w = 1.0 / double(S);
  if (kind == 0) {
    int r = key;
    for (int k = D - 1; k >= 0; --k) {
      z[k] = (double(r % S) + 0.5) * w;
      r /= S;
    }
    return;
  }
  const int nf = family_count<D>(kind);
  int off = 0;
  for (int fam = 0; fam < nf; ++fam) {
    const int mask = family_mask<D>(kind, fam);
    int cnt[D], fsize = 1;
    for (int k = 0; k < D; ++k) {
      cnt[k] = ((mask >> k) & 1) ? S - 1 : S;
      fsize *= cnt[k];
    }
    if (key < off + fsize) {
      int r = key - off;
      for (int k = D - 1; k >= 0; --k) {
        const int m = r % cnt[k];
        r /= cnt[k];
        z[k] = ((mask >> k) & 1) ? double(m + 1) * w : (double(m) + 0.5) * w;
      }
      return;
    }
    off += fsize;
  }
}

// Per-problem geometry of a sub-level when several independent problems are
// factored together (their DOFs concatenated): pid[j] is the problem of DOF
// j, and problem p has S[p] boxes per side, its group keys start at koff[p],
// its cells at coff[p] in the cell table, its proxy radius is R[p] and its ID
// precision eps[p].  With pid == nullptr there is one problem and the
// sub-level's scalars apply.
struct ProbGeo {
  const int32_t* pid = nullptr;
  const int32_t* S = nullptr;
  const int32_t* koff = nullptr;
  const int32_t* coff = nullptr;
  const double* R = nullptr;
  const double* eps = nullptr;
  const int32_t* gpid = nullptr;  // [G] problem of each group
};

// key = the problem's key offset (coff for cells with cell_keys, koff
// otherwise) + the point's group within its problem.
template <int D>
__global__ void k_group_key(const double* pts, const int32_t* act, int64_t nact, int kind, int S,
                            int32_t* key, int32_t* dof, ProbGeo pg, int cell_keys) {
  GRID_STRIDE(i, nact) {
    const int j = act[i];
    int s = S, off = 0;
    if (pg.pid) {
      const int p = pg.pid[j];
      s = pg.S[p];
      off = cell_keys ? pg.coff[p] : pg.koff[p];
    }
    key[i] = off + group_key<D>(pts + int64_t(j) * D, kind, s);
    dof[i] = j;
  }
}

template <int D>
__global__ void k_partition(const double* pts, int64_t n, const uint8_t* active, int kind, int S,
                            int32_t* group) {
  GRID_STRIDE(i, n) group[i] = active[i] ? group_key<D>(pts + i * D, kind, S) : -1;
}

__global__ void k_heads(const int32_t* skey, int64_t n, int32_t* head) {
  GRID_STRIDE(i, n) head[i] = (i == 0 || skey[i] != skey[i - 1]) ? 1 : 0;
}

// After an exclusive scan of the heads: group index of every position.
__global__ void k_group_setup(const int32_t* skey, const int32_t* sdof, int64_t n, const int32_t* head,
                              const int32_t* hscan, int64_t* gstart, int32_t* gkey, int32_t* grp_of,
                              const int32_t* pid, int32_t* gpid) {
  GRID_STRIDE(i, n) {
    const int g = hscan[i] + head[i] - 1;
    if (head[i]) {
      gstart[g] = i;
      gkey[g] = skey[i];
      if (pid) gpid[g] = pid[sdof[i]];
    }
    if (i == n - 1) gstart[g + 1] = n;
    grp_of[sdof[i]] = g;
  }
}

template <int D>
__global__ void k_centres(const int32_t* gkey, int G, int kind, int S, double* zc, ProbGeo pg) {
  GRID_STRIDE(g, G) {
    if (pg.pid) {
      const int p = pg.gpid[g];
      centre_of<D>(gkey[g] - pg.koff[p], kind, pg.S[p], zc + g * D);
    } else {
      centre_of<D>(gkey[g], kind, S, zc + g * D);
    }
  }
}

__global__ void k_cell_table(const int32_t* ckey, int64_t n, int32_t* lo, int32_t* hi) {
  GRID_STRIDE(i, n) {
    const int c = ckey[i];
    if (i == 0 || ckey[i - 1] != c) lo[c] = int32_t(i);
    if (i == n - 1 || ckey[i + 1] != c) hi[c] = int32_t(i + 1);
  }
}

// ---------------------------------------------------------------------------
// Near field c^N (Section 3.3, expanded by SCI partners per Section 4.3):
// DOFs of other groups strictly inside the proxy sphere about the group
// centre, plus every DOF sharing a stored SCI with the group.  Candidates are
// counted, emitted as (group, DOF) keys, sorted and deduplicated.
// ---------------------------------------------------------------------------
struct NfArgs {
  const double* pts;
  const int32_t* sdof;
  const int64_t* gstart;
  const double* zc;
  int G, S;
  double R, R2;
  const int32_t* cdof;
  const int32_t* cell_lo;
  const int32_t* cell_hi;
  const int32_t* grp_of;
  const int64_t* srow;
  const uint64_t* skey;
  int64_t* cnt;
  uint64_t* cand;
  const int64_t* cand_off;
  int shift;
  ProbGeo pg;
};

template <int D, bool FILL>
__global__ void k_nearfield(NfArgs A) {
  // group g is split over gridDim.x workgroups (slot g * gridDim.x + part):
  // the cells of its bounding box go round-robin to the parts, and each wave
  // takes one DOF of the group with its lanes over that DOF's SCI entries.
  // Candidates are sorted and de-duplicated afterwards, so the split and the
  // order of emission do not show in the result.
  const int g = blockIdx.y, part = blockIdx.x, NP = gridDim.x;
  const int64_t slot = int64_t(g) * NP + part;
  // the group's problem: its boxes per side, proxy radius and cells
  int S = A.S, coff = 0;
  double R = A.R, R2 = A.R2;
  if (A.pg.pid) {
    const int p = A.pg.gpid[g];
    S = A.pg.S[p];
    R = A.pg.R[p];
    R2 = R * R;
    coff = A.pg.coff[p];
  }
  double z[D];
#pragma unroll
  for (int k = 0; k < D; ++k) z[k] = A.zc[int64_t(g) * D + k];
  int lo[3] = {0, 0, 0}, ext[3] = {1, 1, 1};
#pragma unroll
  for (int k = 0; k < D; ++k) {
    lo[k] = max(0, int(floor((z[k] - R) * double(S))) - 1);
    const int hi = min(S - 1, int(floor((z[k] + R) * double(S))) + 1);
    ext[k] = hi - lo[k] + 1;
  }
  __shared__ unsigned long long s_cnt;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  int64_t local = 0;
  uint64_t* out = FILL ? A.cand + A.cand_off[slot] : nullptr;
  const unsigned long long cap = FILL ? (unsigned long long)(A.cand_off[slot + 1] - A.cand_off[slot]) : 0ull;
  auto emit = [&](int j) {
    if (FILL) {
      unsigned long long pos = atomicAdd(&s_cnt, 1ull);
      if (pos < cap) out[pos] = (uint64_t(g) << A.shift) | uint64_t(uint32_t(j));
    } else {
      ++local;
    }
  };
  const int ncell = ext[0] * ext[1] * ext[2];
  for (int cl = part; cl < ncell; cl += NP) {
    const int cc[3] = {lo[0] + cl / (ext[1] * ext[2]), lo[1] + (cl / ext[2]) % ext[1], lo[2] + cl % ext[2]};
    int cid = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) cid = cid * S + cc[k];
    cid += coff;
    const int b = A.cell_lo[cid], e = A.cell_hi[cid];
    for (int i = b + threadIdx.x; i < e; i += blockDim.x) {
      const int j = A.cdof[i];
      if (A.grp_of[j] == g) continue;
      if (dist2_exact<D>(A.pts + int64_t(j) * D, z) < R2) emit(j);
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int64_t p = A.gstart[g] + int64_t(part) * nw + wv; p < A.gstart[g + 1]; p += int64_t(NP) * nw) {
    const int i = A.sdof[p];
    for (int64_t e = A.srow[i] + lane; e < A.srow[i + 1]; e += 64) {
      const int j = int(A.skey[e] & 0xffffffffu);
      if (A.grp_of[j] != g) emit(j);
    }
  }
  if (!FILL) {
    __shared__ long long sp[16];
    long long v = local;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sp[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      long long t = 0;
      for (int k = 0; k < int(blockDim.x + 63) / 64; ++k) t += sp[k];
      A.cnt[slot] = t;
    }
  }
}

__global__ void k_unique_flags(const uint64_t* keys, int64_t n, int64_t* flag) {
  GRID_STRIDE(i, n) flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

__global__ void k_unique_compact(const uint64_t* keys, int64_t n, const int64_t* flag, const int64_t* pos,
                                 int shift, int32_t* nf_idx) {
  GRID_STRIDE(i, n) {
    if (flag[i]) nf_idx[pos[i]] = int32_t(keys[i] & ((uint64_t(1) << shift) - 1));
  }
}

// Offsets out[0..nseg] of the segments (key >> shift) of n > 0 sorted keys:
// out[s] = index (pos[e] if pos is given) of the first key of segment >= s,
// out[nseg] = total.  Every entry is written exactly once: each boundary
// fills the offsets of the segments it passes, so no atomics are needed.
__global__ void k_csr_from_sorted(const uint64_t* keys, int64_t n, int shift, int64_t nseg, const int64_t* pos,
                                  int64_t total, int64_t* out) {
  GRID_STRIDE(e, n) {
    const int64_t sg = int64_t(keys[e] >> shift);
    const int64_t val = pos ? pos[e] : e;
    const int64_t prev = e == 0 ? -1 : int64_t(keys[e - 1] >> shift);
    if (prev != sg)
      for (int64_t t = prev + 1; t <= sg; ++t) out[t] = val;
    if (e == n - 1)
      for (int64_t t = sg + 1; t <= nseg; ++t) out[t] = total;
  }
}

__global__ void k_i32_to_i64(const int32_t* a, int64_t* b, int64_t n) { GRID_STRIDE(i, n) b[i] = a[i]; }

// ---------------------------------------------------------------------------
// Split classes (Section 4.4, Lemma 4.2): columns with the same structural
// SCI pattern over the near field.  Pattern sets are compared through two
// order-independent 64-bit hashes plus their size; classes are ordered by
// their first column and keep ascending column order inside.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

struct ClsArgs {
  const int32_t* sdof;
  const int64_t* gstart;
  const int32_t* grp_of;
  const int64_t* srow;
  const uint64_t* skey;
  uint64_t* h1;
  uint64_t* h2;
  int32_t* hc;
  int32_t* rep;
  int32_t* newpos;
  int32_t* cord;
  int32_t* pos_of;
  int32_t* ncls;
  int split;
  // fill pass
  const int32_t* cls_first;
  int32_t* cls_col0;
  int32_t* cls_n;
  int32_t* cls_group;
};

// Exclusive scan of a 0/1 flag over the workgroup (wave64); sets *total.
__device__ int cls_excl_scan(int flag, int* total) {
  __shared__ int sw[16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  const unsigned long long bal = __ballot(flag);
  const int pre = __popcll(bal & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
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

// Key of every column (thread per column of all groups): a hash of the set of
// its SCI rows outside its own group (Section 4.4 splits a group's columns by
// that sparsity pattern).
__global__ void k_class_hash(ClsArgs A, int64_t ncol) {
  GRID_STRIDE(e, ncol) {
    uint64_t a = 0, b = 0;
    int c = 0;
    if (A.split) {
      const int j = A.sdof[e];
      const int g = A.grp_of[j];
      for (int64_t t = A.srow[j]; t < A.srow[j + 1]; ++t) {
        const int i = int(A.skey[t] & 0xffffffffu);
        if (A.grp_of[i] != g) {
          a += mix64(uint64_t(i));
          b ^= mix64(uint64_t(i) * 0x2545f4914f6cdd1dull + 17);
          ++c;
        }
      }
    }
    A.h1[e] = a;
    A.h2[e] = b;
    A.hc[e] = c;
    A.rep[e] = -1;
  }
}

// Second-kind classes of group g (Section 4.4): columns with the same key
// form one class.  Classes are numbered by their first column, columns keep
// their order within a class; one round per class finds the first unassigned
// column, assigns every column with its key and places them (work
// O(classes x n) per group).
__global__ void k_class_prep(ClsArgs A) {
  const int g = blockIdx.x;
  const int64_t c0 = A.gstart[g];
  const int n = int(A.gstart[g + 1] - c0);
  __shared__ int s_first;
  int ncls = 0, placed = 0, from = 0;
  for (;;) {
    if (threadIdx.x == 0) s_first = INT_MAX;
    __syncthreads();
    for (int p = from + int(threadIdx.x); p < n; p += blockDim.x)
      if (A.rep[c0 + p] < 0) atomicMin(&s_first, p);
    __syncthreads();
    const int p0 = s_first;
    if (p0 == INT_MAX) break;
    const uint64_t a = A.h1[c0 + p0], b = A.h2[c0 + p0];
    const int cc = A.hc[c0 + p0];
    // members in column order, placed after the classes found so far
    for (int base = p0; base < n; base += blockDim.x) {
      const int p = base + int(threadIdx.x);
      const int flag = (p < n && A.rep[c0 + p] < 0 && A.h1[c0 + p] == a && A.h2[c0 + p] == b && A.hc[c0 + p] == cc)
                           ? 1 : 0;
      int tot = 0;
      const int pre = cls_excl_scan(flag, &tot);
      if (flag) {
        const int np = placed + pre;
        A.rep[c0 + p] = p0;
        A.newpos[c0 + p] = np;
        const int j = A.sdof[c0 + p];
        A.cord[c0 + np] = j;
        A.pos_of[j] = np;
      }
      placed += tot;
    }
    ++ncls;
    from = p0 + 1;
  }
  if (threadIdx.x == 0) A.ncls[g] = ncls;
}

__global__ void k_class_fill(ClsArgs A) {
  const int g = blockIdx.x;
  const int64_t c0 = A.gstart[g];
  const int n = int(A.gstart[g + 1] - c0);
  for (int p = threadIdx.x; p < n; p += blockDim.x) {
    if (A.rep[c0 + p] != p) continue;
    int ci = 0, cnt = 0;
    for (int q = 0; q < n; ++q) {
      const int rq = A.rep[c0 + q];
      ci += (rq == q && q < p);
      cnt += (rq == p);
    }
    const int slot = A.cls_first[g] + ci;
    A.cls_col0[slot] = A.newpos[c0 + p];
    A.cls_n[slot] = cnt;
    A.cls_group[slot] = g;
  }
}

// Per class: local tolerance rho eps with rho = min(1, |Y^K| / |Y^S|) (Section 4.4).
__global__ void k_class_tol(int nc, const int32_t* cls_group, const int32_t* cls_col0, const int32_t* cls_n,
                            const int64_t* gstart, const double* colK2, const double* colS2, double eps,
                            int second_kind, const int64_t* yoff, const int64_t* nf_start, int sym,
                            int nproxy, int64_t* moff, int32_t* ld, int32_t* rows, double* tol,
                            int64_t* poff, ProbGeo pg) {
  GRID_STRIDE(q, nc) {
    const int g = cls_group[q];
    if (pg.pid) eps = pg.eps[pg.gpid[g]];
    const int64_t c0 = gstart[g];
    const int n = int(gstart[g + 1] - c0);
    const int col0 = cls_col0[q], nq = cls_n[q];
    double k2 = 0.0, s2 = 0.0;
    for (int j = 0; j < nq; ++j) {
      k2 += colK2[c0 + col0 + j];
      s2 += colS2[c0 + col0 + j];
    }
    double rho = 1.0;
    if (second_kind && s2 > 0.0) rho = fmin(1.0, sqrt(k2) / sqrt(s2));
    tol[q] = rho * eps;
    const int nf = int(nf_start[g + 1] - nf_start[g]);
    moff[q] = yoff[g] + col0;
    ld[q] = n;
    rows[q] = sym ? nf + nproxy : 2 * nf + 2 * nproxy;
    poff[q] = c0 + col0;
  }
}

// ---------------------------------------------------------------------------
// SCI store maintenance.
// ---------------------------------------------------------------------------
__global__ void k_mark_inactive(const GroupRec* recs, int nrec, const int32_t* iarena, uint8_t* active) {
  const int ri = blockIdx.x;
  if (ri >= nrec) return;
  const GroupRec R = recs[ri];
  for (int b = threadIdx.x; b < R.r; b += blockDim.x) active[iarena[R.idx + b]] = 0;
}

__global__ void k_sci_keep(const uint64_t* key, int64_t nnz, const uint8_t* active, const int32_t* grp_of,
                           const int32_t* grec, int64_t* keep) {
  GRID_STRIDE(e, nnz) {
    const int i = int(key[e] >> 32), j = int(key[e] & 0xffffffffu);
    int kp = 0;
    if (active[i] && active[j]) {
      // DOFs of a problem that sits this sub-level out have no group (-1)
      const int gi = grp_of[i], gj = grp_of[j];
      kp = (gi != gj) || gi < 0 || (grec[gi] < 0);
    }
    keep[e] = kp;
  }
}

__global__ void k_sci_compact(const uint64_t* key, const double2* val, int64_t nnz, const int64_t* keep,
                              const int64_t* pos, uint64_t* okey, double2* oval, int32_t* oidx) {
  GRID_STRIDE(e, nnz) {
    if (keep[e]) {
      const int64_t p = pos[e];
      okey[p] = key[e];
      oval[p] = val[e];
      oidx[p] = int32_t(p);
    }
  }
}

__global__ void k_append(const uint64_t* nkey, const double2* nval, int64_t nn, int64_t base, uint64_t* okey,
                         double2* oval, int32_t* oidx) {
  GRID_STRIDE(e, nn) {
    okey[base + e] = nkey[e];
    oval[base + e] = nval[e];
    oidx[base + e] = int32_t(base + e);
  }
}

__global__ void k_gather_val(const double2* in, const int32_t* idx, int64_t n, double2* out) {
  GRID_STRIDE(e, n) out[e] = in[idx[e]];
}


__global__ void k_active_keep(const int32_t* act, int64_t nact, const uint8_t* active, int32_t* keep) {
  GRID_STRIDE(i, nact) keep[i] = active[act[i]] ? 1 : 0;
}

__global__ void k_active_compact(const int32_t* act, int64_t nact, const int32_t* keep, const int32_t* pos,
                                 int32_t* out) {
  GRID_STRIDE(i, nact) if (keep[i]) out[pos[i]] = act[i];
}

// Descriptors of a sub-batch of IDs (classes idx[0..n)), and its ranks back.
__global__ void k_id_gather(int n, const int32_t* idx, const int64_t* moff, const int32_t* ld, const int32_t* rows,
                            const int32_t* cols, const double* tol, const int64_t* poff, int64_t* omoff, int32_t* old,
                            int32_t* orows, int32_t* ocols, double* otol, int64_t* opoff) {
  GRID_STRIDE(i, n) {
    const int q = idx[i];
    omoff[i] = moff[q];
    old[i] = ld[q];
    orows[i] = rows[q];
    ocols[i] = cols[q];
    otol[i] = tol[q];
    opoff[i] = poff[q];
  }
}

__global__ void k_id_scatter_rank(int n, const int32_t* idx, const int32_t* rank_s, int32_t* rank) {
  GRID_STRIDE(i, n) rank[idx[i]] = rank_s[i];
}

// Number of entries of the ascending list a[0..n) below v (one thread,
// binary search).
__global__ void k_count_below(const int32_t* a, int64_t n, int32_t v, int64_t* out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (a[mid] < v) lo = mid + 1; else hi = mid;
  }
  *out = lo;
}

// Subtract off from the DOF indices (redundant, then skeleton) of every record.
__global__ void k_rebase_records(const GroupRec* recs, int nrec, int32_t* iarena, int32_t off) {
  const int ri = blockIdx.x;
  if (ri >= nrec) return;
  const GroupRec R = recs[ri];
  for (int e = threadIdx.x; e < R.r + R.k; e += blockDim.x) iarena[R.idx + e] -= off;
}

__global__ void k_sub_i32(const int32_t* a, int64_t n, int32_t off, int32_t* out) {
  GRID_STRIDE(i, n) out[i] = a[i] - off;
}

__global__ void k_pos_scatter(const int32_t* idx, int64_t n, int32_t* pos_of) {
  GRID_STRIDE(i, n) pos_of[idx[i]] = int32_t(i);
}

// Coincident points: pairwise comparison inside each leaf box (boxes with
// more than 4096 points are skipped).
__global__ void k_coincident(const double* pts, int D, const int32_t* cdof, const int32_t* lo, const int32_t* hi,
                             int32_t* flag) {
  const int b = lo[blockIdx.x], e = hi[blockIdx.x];
  const int n = e - b;
  if (n < 2 || n > 4096) return;
  const int64_t pairs = int64_t(n) * (n - 1) / 2;
  for (int64_t t = threadIdx.x; t < pairs; t += blockDim.x) {
    // t -> (i, j), i < j
    int i = int((sqrt(8.0 * double(t) + 1.0) - 1.0) / 2.0);
    while (int64_t(i + 1) * (i + 2) / 2 <= t) ++i;
    while (int64_t(i) * (i + 1) / 2 > t) --i;
    const int j = int(t - int64_t(i) * (i + 1) / 2);
    const int pi = cdof[b + i + 1], pj = cdof[b + j];
    bool same = true;
    for (int k = 0; k < D; ++k) same = same && (pts[int64_t(pi) * D + k] == pts[int64_t(pj) * D + k]);
    if (same) atomicOr(flag, 1);
  }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
template <class T>
void to_host(std::vector<T>& h, const T* d, size_t n, hipStream_t s) {
  h.resize(n);
  if (n) HIF_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s));
  HIF_HIP(hipStreamSynchronize(s));
}

template <class T>
void to_dev(T* d, const std::vector<T>& h, hipStream_t s) {
  if (!h.empty()) HIF_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

template <class T>
T scalar_at(const T* d, hipStream_t s) {
  T v{};
  HIF_HIP(hipMemcpyAsync(&v, d, sizeof(T), hipMemcpyDeviceToHost, s));
  HIF_HIP(hipStreamSynchronize(s));
  return v;
}

// Phase timing with HIP events recorded on the factorization's stream.  The
// events come from a pool owned by the timer: created on first use, recorded
// again after every flush and destroyed with the timer, so a factorization
// creates a few dozen events instead of one per mark (thousands per
// factorization, from every worker thread of a batch).
struct Timer {
  hipStream_t s;
  std::vector<hipEvent_t> pool;  // every event created so far
  size_t used = 0;               // events recorded since the last flush
  std::vector<int> phase;
  void mark(int ph) {
    if (used == pool.size()) {
      hipEvent_t e;
      HIF_HIP(hipEventCreate(&e));
      pool.push_back(e);
    }
    HIF_HIP(hipEventRecord(pool[used], s));
    ++used;
    phase.push_back(ph);
  }
  void flush(double* acc, double* acc2 = nullptr) {
    if (used >= 2) {
      HIF_HIP(hipEventSynchronize(pool[used - 1]));
      for (size_t i = 1; i < used; ++i) {
        float ms = 0.f;
        HIF_HIP(hipEventElapsedTime(&ms, pool[i - 1], pool[i]));
        acc[phase[i]] += ms;
        if (acc2) acc2[phase[i]] += ms;
      }
    } else if (used == 1) {
      HIF_HIP(hipEventSynchronize(pool[0]));
    }
    used = 0;
    phase.clear();
  }
  ~Timer() {
    // a pending record must complete before its event is destroyed
    if (used > 0) (void)hipEventSynchronize(pool[used - 1]);
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

enum { PH_PART = 0, PH_ASM = 1, PH_ID = 2, PH_ELIM = 3, PH_SCI = 4, PH_TOP = 5, PH_HOST = 6, PH_QR = 7 };

struct Factorizer {
  hif_factor_s* H;
  hipStream_t s;
  int D;
  int64_t N;
  MemTracker* mt;
  Timer tm;
  // operator (owned for the duration of the factorization)
  const double *pts, *a, *b, *c, *w, *sf;
  // state
  DBuf<uint8_t> active;
  DBuf<int32_t> act, act2;
  int64_t nact = 0;
  DBuf<int32_t> grp_of, pos_of;
  DBuf<uint64_t> skey, skey2;
  DBuf<double2> sval, sval2;
  DBuf<int64_t> srow;
  int64_t snnz = 0;
  DBuf<double> proxy_u;
  // scratch
  DBuf<unsigned char> prim;
  DBuf<int32_t> key, dof, ktmp, vtmp, head, hscan, gkey, cell_lo, cell_hi, ckey, cdof;
  DBuf<int64_t> gstart, cnt, cand_off, flag64, pos64, nf_start;
  DBuf<double> zc;
  DBuf<uint64_t> cand, cand2;
  DBuf<int32_t> nf_idx;
  DBuf<uint64_t> h1, h2;
  DBuf<int32_t> hc, rep, newpos, cord, ncls;
  DBuf<int32_t> cls_first, cls_col0, cls_n, cls_group, cls_rank, cls_skoff, cls_rdoff, cls_ld, cls_rows, perm;
  DBuf<int64_t> cls_moff, cls_poff, yoff, aoff, newoff;
  DBuf<double> cls_tol, Y, Acc, Scc, Mw, colK2, colS2, kpart, qr_scratch;
  DBuf<int32_t> cls_rows2;
  DBuf<int64_t> cls_soff;
  DBuf<GemmDesc> gdesc;
  DBuf<int64_t> lu_moff, lu_poff;
  DBuf<int32_t> lu_n, lu_r;
  DBuf<int32_t> grec, loc, rlo, rhi, status, sidx, sidx2;
  DBuf<uint64_t> newkey;
  DBuf<double2> newval;
  DBuf<int32_t> akeep, apos;
  DBuf<int32_t> sub_idx, sub_ld, sub_rows, sub_cols, sub_rank;
  DBuf<int64_t> sub_moff, sub_poff;
  DBuf<double> sub_tol;
  // Several independent problems factored together (level-synchronous
  // batch): their DOFs are concatenated, deepest tree first, so that the
  // problems still taking part in a level hold a prefix of the ascending
  // active list.  Problem p has tree depth pL[p], DOFs [poff[p], poff[p+1]),
  // ID precision peps[p].  One problem: multi == false and none of this is used.
  bool multi = false;
  int nprob = 1;
  std::vector<int> pL;
  std::vector<int64_t> poff;
  std::vector<double> peps;
  DBuf<int32_t> pid, dS, dkoff, dcoff, gpid;
  DBuf<int64_t> cut;
  DBuf<double> dR, deps;
  // per sub-level: problem of each record (host), for the split into handles
  std::vector<std::vector<int32_t>> rec_prob;

  void sublevel(int lvl, int kind);
  void top();
  void top_multi(const std::vector<hif_factor_s*>& hs);
};

void Factorizer::sublevel(int lvl, int kind) {
  const int L = H->L;
  const int S = 1 << (L - lvl);
  const double w_l = 1.0 / double(S);
  const double R = H->proxy_r * w_l;
  const double R2 = R * R;
  const int P = H->nproxy;
  const int sym = H->symmetric;
  const int split = H->opts.second_kind ? 1 : 0;
  const int si = int(H->subs.size());
  SubLevel sub;
  sub.level = lvl;
  sub.kind = kind;
  hif_stats_t& st = H->stats;
  st.sub_kind[si] = kind;
  // Several problems: the ones whose tree is deep enough take part; their
  // active DOFs are the first nact of the list, and every DOF starts the
  // sub-level without a group.
  const int64_t nact_all = nact;
  ProbGeo pg{};
  int ncent = 1, ncell = 1;
  for (int k = 0; k < D; ++k) {
    ncent *= S;
    ncell *= S;
  }
  ncent *= (kind == 0 ? 1 : 3);
  if (multi) {
    int np = 0;
    while (np < nprob && pL[np] > lvl) ++np;
    std::vector<int32_t> hS(np), hk(np + 1), hc(np + 1);
    std::vector<double> hR(np), he(np);
    hk[0] = hc[0] = 0;
    for (int q = 0; q < np; ++q) {
      const int Sq = 1 << (pL[q] - lvl);
      int nc = 1;
      for (int k = 0; k < D; ++k) nc *= Sq;
      hS[q] = Sq;
      hc[q + 1] = hc[q] + nc;
      hk[q + 1] = hk[q] + nc * (kind == 0 ? 1 : 3);
      hR[q] = H->proxy_r / double(Sq);
      he[q] = peps[q];
    }
    ncent = hk[np];
    ncell = hc[np];
    dS.ensure(nprob, mt);
    dkoff.ensure(nprob + 1, mt);
    dcoff.ensure(nprob + 1, mt);
    dR.ensure(nprob, mt);
    deps.ensure(nprob, mt);
    to_dev(dS.p, hS, s);
    to_dev(dkoff.p, hk, s);
    to_dev(dcoff.p, hc, s);
    to_dev(dR.p, hR, s);
    to_dev(deps.p, he, s);
    hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(N)), dim3(kThreads), 0, s, grp_of.p, N, -1);
    if (np < nprob) {
      cut.ensure(1, mt);
      hipLaunchKernelGGL(k_count_below, dim3(1), dim3(64), 0, s, act.p, nact, int32_t(poff[np]), cut.p);
      HIF_HIP(hipGetLastError());
      nact = scalar_at(cut.p, s);
    }
    pg.pid = pid.p;
    pg.S = dS.p;
    pg.koff = dkoff.p;
    pg.coff = dcoff.p;
    pg.R = dR.p;
    pg.eps = deps.p;
  }
  st.sub_active[si] = nact;
  if (nact == 0) {
    nact = nact_all;
    H->subs.push_back(std::move(sub));
    if (multi) rec_prob.emplace_back();
    return;
  }
  tm.mark(PH_HOST);

  // ---- partition of the active DOFs into groups -------------------------
  key.ensure(nact, mt);
  dof.ensure(nact, mt);
  ktmp.ensure(nact, mt);
  vtmp.ensure(nact, mt);
  head.ensure(nact, mt);
  hscan.ensure(nact + 1, mt);
  if (D == 2)
    hipLaunchKernelGGL(k_group_key<2>, dim3(nblocks(nact)), dim3(kThreads), 0, s, pts, act.p, nact, kind, S, key.p,
                       dof.p, pg, 0);
  else
    hipLaunchKernelGGL(k_group_key<3>, dim3(nblocks(nact)), dim3(kThreads), 0, s, pts, act.p, nact, kind, S, key.p,
                       dof.p, pg, 0);
  HIF_HIP(hipGetLastError());
  sort_i32_i32(key.p, ktmp.p, dof.p, vtmp.p, nact, ceil_log2(uint64_t(ncent) + 1), s, prim, mt);
  hipLaunchKernelGGL(k_heads, dim3(nblocks(nact)), dim3(kThreads), 0, s, key.p, nact, head.p);
  exclusive_scan_i32(head.p, hscan.p, nact, s, prim, mt);
  const int G = scalar_at(hscan.p + nact, s);
  gstart.ensure(G + 1, mt);
  gkey.ensure(G, mt);
  if (multi) {
    gpid.ensure(G, mt);
    pg.gpid = gpid.p;
  }
  hipLaunchKernelGGL(k_group_setup, dim3(nblocks(nact)), dim3(kThreads), 0, s, key.p, dof.p, nact, head.p, hscan.p,
                     gstart.p, gkey.p, grp_of.p, pg.pid, multi ? gpid.p : nullptr);
  zc.ensure(int64_t(G) * D, mt);
  if (D == 2)
    hipLaunchKernelGGL(k_centres<2>, dim3(nblocks(G)), dim3(kThreads), 0, s, gkey.p, G, kind, S, zc.p, pg);
  else
    hipLaunchKernelGGL(k_centres<3>, dim3(nblocks(G)), dim3(kThreads), 0, s, gkey.p, G, kind, S, zc.p, pg);
  HIF_HIP(hipGetLastError());
  st.sub_groups[si] = G;

  // ---- level-l cell binning of the active DOFs (geometric candidates) ----
  ckey.ensure(nact, mt);
  cdof.ensure(nact, mt);
  cell_lo.ensure(ncell, mt);
  cell_hi.ensure(ncell, mt);
  if (D == 2)
    hipLaunchKernelGGL(k_group_key<2>, dim3(nblocks(nact)), dim3(kThreads), 0, s, pts, act.p, nact, 0, S, ckey.p,
                       cdof.p, pg, 1);
  else
    hipLaunchKernelGGL(k_group_key<3>, dim3(nblocks(nact)), dim3(kThreads), 0, s, pts, act.p, nact, 0, S, ckey.p,
                       cdof.p, pg, 1);
  sort_i32_i32(ckey.p, ktmp.p, cdof.p, vtmp.p, nact, ceil_log2(uint64_t(ncell) + 1), s, prim, mt);
  hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(ncell)), dim3(kThreads), 0, s, cell_lo.p, int64_t(ncell), 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(ncell)), dim3(kThreads), 0, s, cell_hi.p, int64_t(ncell), 0);
  hipLaunchKernelGGL(k_cell_table, dim3(nblocks(nact)), dim3(kThreads), 0, s, ckey.p, nact, cell_lo.p, cell_hi.p);
  HIF_HIP(hipGetLastError());

  // ---- near fields --------------------------------------------------------
  const int shift = ceil_log2(uint64_t(N) + 1);
  const int gbits = ceil_log2(uint64_t(G) + 1);
  NfArgs nfa{};
  nfa.pts = pts;
  nfa.sdof = dof.p;
  nfa.gstart = gstart.p;
  nfa.zc = zc.p;
  nfa.G = G;
  nfa.S = S;
  nfa.R = R;
  nfa.R2 = R2;
  nfa.cdof = cdof.p;
  nfa.cell_lo = cell_lo.p;
  nfa.cell_hi = cell_hi.p;
  nfa.grp_of = grp_of.p;
  nfa.srow = srow.p;
  nfa.skey = skey.p;
  // workgroups per group: enough to fill the GPU when groups are few
  const int NP = int(std::min<int64_t>(64, std::max<int64_t>(1, 2048 / G)));
  const int64_t nslot = int64_t(G) * NP;
  cnt.ensure(nslot, mt);
  cand_off.ensure(nslot + 1, mt);
  nfa.cnt = cnt.p;
  nfa.shift = shift;
  nfa.pg = pg;
  if (D == 2)
    hipLaunchKernelGGL((k_nearfield<2, false>), dim3(NP, G), dim3(kThreads), 0, s, nfa);
  else
    hipLaunchKernelGGL((k_nearfield<3, false>), dim3(NP, G), dim3(kThreads), 0, s, nfa);
  HIF_HIP(hipGetLastError());
  exclusive_scan_i64(cnt.p, cand_off.p, nslot, s, prim, mt);
  const int64_t ncand = scalar_at(cand_off.p + nslot, s);
  cand.ensure(ncand, mt);
  cand2.ensure(ncand, mt);
  nfa.cand = cand.p;
  nfa.cand_off = cand_off.p;
  if (D == 2)
    hipLaunchKernelGGL((k_nearfield<2, true>), dim3(NP, G), dim3(kThreads), 0, s, nfa);
  else
    hipLaunchKernelGGL((k_nearfield<3, true>), dim3(NP, G), dim3(kThreads), 0, s, nfa);
  HIF_HIP(hipGetLastError());
  sort_u64(cand.p, cand2.p, ncand, shift + gbits, s, prim, mt);
  flag64.ensure(ncand, mt);
  pos64.ensure(ncand + 1, mt);
  nf_start.ensure(G + 1, mt);
  hipLaunchKernelGGL(k_unique_flags, dim3(nblocks(ncand)), dim3(kThreads), 0, s, cand.p, ncand, flag64.p);
  exclusive_scan_i64(flag64.p, pos64.p, ncand, s, prim, mt);
  const int64_t nnf = scalar_at(pos64.p + ncand, s);
  nf_idx.ensure(nnf, mt);
  hipLaunchKernelGGL(k_unique_compact, dim3(nblocks(ncand)), dim3(kThreads), 0, s, cand.p, ncand, flag64.p, pos64.p,
                     shift, nf_idx.p);
  if (ncand > 0)
    hipLaunchKernelGGL(k_csr_from_sorted, dim3(nblocks(ncand)), dim3(kThreads), 0, s, cand.p, ncand, shift,
                       int64_t(G), pos64.p, nnf, nf_start.p);
  else
    hipLaunchKernelGGL(k_fill_i64, dim3(nblocks(G + 1)), dim3(kThreads), 0, s, nf_start.p, int64_t(G + 1),
                       int64_t(0));
  HIF_HIP(hipGetLastError());
  st.sub_near[si] = nnf;

  // ---- split classes and class-ordered group DOFs -------------------------
  h1.ensure(nact, mt);
  h2.ensure(nact, mt);
  hc.ensure(nact, mt);
  rep.ensure(nact, mt);
  newpos.ensure(nact, mt);
  cord.ensure(nact, mt);
  ncls.ensure(G, mt);
  ClsArgs ca{};
  ca.sdof = dof.p;
  ca.gstart = gstart.p;
  ca.grp_of = grp_of.p;
  ca.srow = srow.p;
  ca.skey = skey.p;
  ca.h1 = h1.p;
  ca.h2 = h2.p;
  ca.hc = hc.p;
  ca.rep = rep.p;
  ca.newpos = newpos.p;
  ca.cord = cord.p;
  ca.pos_of = pos_of.p;
  ca.ncls = ncls.p;
  ca.split = split;
  hipLaunchKernelGGL(k_class_hash, dim3(nblocks(nact)), dim3(kThreads), 0, s, ca, int64_t(nact));
  hipLaunchKernelGGL(k_class_prep, dim3(G), dim3(kThreads), 0, s, ca);
  HIF_HIP(hipGetLastError());
  tm.mark(PH_PART);
  std::vector<int32_t> h_ncls;
  std::vector<int64_t> h_gstart, h_nf;
  to_host(h_ncls, ncls.p, G, s);
  to_host(h_gstart, gstart.p, G + 1, s);
  to_host(h_nf, nf_start.p, G + 1, s);
  std::vector<int32_t> h_cls_first(G + 1, 0);
  std::vector<int64_t> h_yoff(G), h_aoff(G);
  int64_t ytot = 0, atot = 0;
  int maxn = 1, maxmn = 1;
  for (int g = 0; g < G; ++g) {
    h_cls_first[g + 1] = h_cls_first[g] + h_ncls[g];
    const int64_t n = h_gstart[g + 1] - h_gstart[g];
    const int64_t nf = h_nf[g + 1] - h_nf[g];
    const int64_t m = sym ? nf + P : 2 * nf + 2 * P;
    h_yoff[g] = ytot;
    h_aoff[g] = atot;
    ytot += m * n;
    atot += n * n;
    maxn = std::max<int>(maxn, int(n));
    maxmn = std::max<int>(maxmn, int(m + n));
  }
  const int NC = h_cls_first[G];
  st.sub_classes[si] = NC;
  cls_first.ensure(G + 1, mt);
  to_dev(cls_first.p, h_cls_first, s);
  yoff.ensure(G, mt);
  aoff.ensure(G, mt);
  to_dev(yoff.p, h_yoff, s);
  to_dev(aoff.p, h_aoff, s);
  cls_col0.ensure(NC, mt);
  cls_n.ensure(NC, mt);
  cls_group.ensure(NC, mt);
  ca.cls_first = cls_first.p;
  ca.cls_col0 = cls_col0.p;
  ca.cls_n = cls_n.p;
  ca.cls_group = cls_group.p;
  hipLaunchKernelGGL(k_class_fill, dim3(G), dim3(kThreads), 0, s, ca);
  HIF_HIP(hipGetLastError());
  tm.mark(PH_HOST);

  // ---- assembly of Y_c and A_cc -------------------------------------------
  Y.ensure(ytot, mt);
  Acc.ensure(atot, mt);
  Scc.ensure(atot, mt);
  Mw.ensure(atot, mt);
  colK2.ensure(nact, mt);
  colS2.ensure(nact, mt);
  AsmArgs aa{};
  aa.dim = D;
  aa.sym = sym;
  aa.nproxy = P;
  aa.ngroups = G;
  aa.R = R;
  aa.pts = pts;
  aa.a = a;
  aa.b = b;
  aa.c = c;
  aa.w = w;
  aa.selfk = sf;
  aa.proxy_u = proxy_u.p;
  aa.cord = cord.p;
  aa.gstart = gstart.p;
  aa.nf_idx = nf_idx.p;
  aa.nf_start = nf_start.p;
  aa.zc = zc.p;
  aa.yoff = yoff.p;
  aa.aoff = aoff.p;
  aa.Y = Y.p;
  aa.Acc = Acc.p;
  aa.Scc = Scc.p;
  aa.colK2 = colK2.p;
  aa.colS2 = colS2.p;
  aa.grp_of = grp_of.p;
  aa.pos_of = pos_of.p;
  aa.srow = srow.p;
  aa.skey = skey.p;
  aa.sval = sval.p;
  aa.fp32 = H->opts.precision == HIF_FP32_MIXED;
  aa.gpid = pg.gpid;
  aa.pR = pg.R;
  aa.max_rows = maxmn;
  aa.kstride = nact;
  kpart.ensure(size_t((maxmn + 63) / 64) * size_t(nact), mt);
  aa.kpart = kpart.p;
  aa.max_cols = maxn;
  launch_assemble(aa, s);
  cls_tol.ensure(NC, mt);
  cls_moff.ensure(NC, mt);
  cls_ld.ensure(NC, mt);
  cls_rows.ensure(NC, mt);
  cls_poff.ensure(NC, mt);
  cls_rank.ensure(NC, mt);
  perm.ensure(nact, mt);
  hipLaunchKernelGGL(k_class_tol, dim3(nblocks(NC)), dim3(kThreads), 0, s, NC, cls_group.p, cls_col0.p, cls_n.p,
                     gstart.p, colK2.p, colS2.p, H->eps, split, yoff.p, nf_start.p, sym, P, cls_moff.p, cls_ld.p,
                     cls_rows.p, cls_tol.p, cls_poff.p, pg);
  HIF_HIP(hipGetLastError());
  if (H->opts.trace_sublevel == si && !multi) {
    // a copy of this sub-level as assembled, for step-by-step checks
    auto keep = [&](auto& dst, const auto* src, int64_t count) {
      dst.alloc(count, mt);
      if (count > 0) HIF_HIP(hipMemcpyAsync(dst.p, src, sizeof(*src) * count, hipMemcpyDeviceToDevice, s));
    };
    keep(H->tr_gstart, gstart.p, G + 1);
    keep(H->tr_dofs, cord.p, nact);
    keep(H->tr_nfstart, nf_start.p, G + 1);
    keep(H->tr_nf, nf_idx.p, nnf);
    keep(H->tr_yoff, yoff.p, G);
    keep(H->tr_Y, Y.p, ytot);
    keep(H->tr_aoff, aoff.p, G);
    keep(H->tr_Acc, Acc.p, atot);
    H->traced = true;
  }
  tm.mark(PH_ASM);

  // ---- interpolative decompositions (one per class) -----------------------
  std::vector<int32_t> h_cls_n, h_cls_col0;
  to_host(h_cls_n, cls_n.p, NC, s);
  to_host(h_cls_col0, cls_col0.p, NC, s);
  int maxq = 1;
  for (int q = 0; q < NC; ++q) maxq = std::max(maxq, h_cls_n[q]);
  std::vector<int32_t> h_rows2(NC), h_rowsm(NC);
  std::vector<int64_t> h_soff(NC);
  int64_t qtot = 0;
  int maxm = 1;
  for (int g = 0; g < G; ++g) {
    const int64_t nf = h_nf[g + 1] - h_nf[g];
    const int64_t m = sym ? nf + P : 2 * nf + 2 * P;
    maxm = std::max<int>(maxm, int(m));
    for (int q = h_cls_first[g]; q < h_cls_first[g + 1]; ++q) {
      const int64_t nq = h_cls_n[q];
      h_rowsm[q] = int32_t(m);
      h_rows2[q] = int32_t(std::min<int64_t>(m, nq));
      h_soff[q] = qtot;
      if (m > nq) qtot += rowqr_scratch(m, nq);
    }
  }
  cls_rows2.ensure(NC, mt);
  cls_soff.ensure(NC, mt);
  to_dev(cls_rows2.p, h_rows2, s);
  to_dev(cls_soff.p, h_soff, s);
  // blocked pivoted QR straight on Y, or row compression then the pivoted QR of R0
  const int rc = H->opts.row_compression;
  // auto: on Y directly only when Y is nearly square (every step then streams
  // about as many rows as it would after compression, and the QR of Y is saved)
  double smn = 0.0, snn = 0.0;
  for (int g = 0; g < G; ++g) {
    const int64_t nf = h_nf[g + 1] - h_nf[g];
    const double m = double(sym ? nf + P : 2 * nf + 2 * P);
    for (int q = h_cls_first[g]; q < h_cls_first[g + 1]; ++q) {
      smn += m * h_cls_n[q];
      snn += double(h_cls_n[q]) * h_cls_n[q];
    }
  }
  const bool direct = id_blocked_fits(NC, maxm, maxq) && (rc == 0 || (rc < 0 && smn <= 1.25 * snn));
  // After row compression the classes of a sub-level can take two paths at
  // once: those of at most kIdRegCols columns the register-resident kernel,
  // the larger ones the blocked pivoted QR (whose steps then stream only the
  // large classes).  Used when a sub-level mixes both sizes, or holds more
  // large classes than the blocked path takes in one batch.
  constexpr int kIdRegCols = 192;
  std::vector<int32_t> sel_small, sel_large;
  int max_small = 1, max_large = 1;
  for (int q = 0; q < NC; ++q) {
    if (h_cls_n[q] <= kIdRegCols) {
      sel_small.push_back(q);
      max_small = std::max(max_small, h_cls_n[q]);
    } else {
      sel_large.push_back(q);
      max_large = std::max(max_large, h_cls_n[q]);
    }
  }
  const bool split_id = !direct && !sel_large.empty() && (!sel_small.empty() || NC > 512);
  const bool blocked_r0 = !direct && !split_id && id_blocked_fits(NC, maxq, maxq);
  // problems taller than one TSQR stack: row blocks, then their stacked R factors
  const bool tall_split = !direct && rowqr_split_fits(maxm, maxq);
  if (!direct && !tall_split) qr_scratch.ensure(qtot + 1, mt);
  tm.mark(PH_HOST);
  RowQrArgs qa{};
  qa.base = Y.p;
  qa.moff = cls_moff.p;
  qa.ld = cls_ld.p;
  qa.rows = cls_rows.p;
  qa.cols = cls_n.p;
  qa.scratch = qr_scratch.p;
  qa.soff = cls_soff.p;
  qa.nprob = NC;
  if (tall_split) {
    std::vector<int64_t> h_moff;
    std::vector<int32_t> h_ld;
    to_host(h_moff, cls_moff.p, NC, s);
    to_host(h_ld, cls_ld.p, NC, s);
    launch_rowqr_split(Y.p, h_moff, h_ld, h_rowsm, h_cls_n, mt, s);
  } else if (!direct) {
    launch_rowqr_auto(qa, maxm, maxq, s);
  }
  tm.mark(PH_QR);
  IdArgs ia{};
  ia.base = Y.p;
  ia.moff = cls_moff.p;
  ia.ld = cls_ld.p;
  ia.rows = direct ? cls_rows.p : cls_rows2.p;
  ia.cols = cls_n.p;
  ia.tol = cls_tol.p;
  ia.rank = cls_rank.p;
  ia.perm = perm.p;
  ia.poff = cls_poff.p;
  ia.Tout = nullptr;
  ia.toff = nullptr;
  ia.nprob = NC;
  if (direct) {
    launch_id_blocked(ia, maxm, maxq, s);
  } else if (blocked_r0) {
    launch_id_blocked(ia, maxq, maxq, s);  // on R0: rows <= columns
  } else if (split_id) {
    // two sub-batches with gathered descriptors; their ranks go back to the
    // class order (the permutations land in place through their offsets)
    auto run = [&](const std::vector<int32_t>& sel, bool blocked, int maxc) {
      if (sel.empty()) return;
      const int ns = int(sel.size());
      sub_idx.ensure(ns, mt);
      sub_moff.ensure(ns, mt);
      sub_poff.ensure(ns, mt);
      sub_ld.ensure(ns, mt);
      sub_rows.ensure(ns, mt);
      sub_cols.ensure(ns, mt);
      sub_rank.ensure(ns, mt);
      sub_tol.ensure(ns, mt);
      to_dev(sub_idx.p, sel, s);
      hipLaunchKernelGGL(k_id_gather, dim3(nblocks(ns)), dim3(kThreads), 0, s, ns, sub_idx.p, cls_moff.p, cls_ld.p,
                         cls_rows2.p, cls_n.p, cls_tol.p, cls_poff.p, sub_moff.p, sub_ld.p, sub_rows.p, sub_cols.p,
                         sub_tol.p, sub_poff.p);
      IdArgs sa = ia;
      sa.moff = sub_moff.p;
      sa.ld = sub_ld.p;
      sa.rows = sub_rows.p;
      sa.cols = sub_cols.p;
      sa.tol = sub_tol.p;
      sa.rank = sub_rank.p;
      sa.poff = sub_poff.p;
      sa.nprob = ns;
      if (blocked)
        launch_id_blocked(sa, maxc, maxc, s);
      else
        launch_id(sa, maxc, s);
      hipLaunchKernelGGL(k_id_scatter_rank, dim3(nblocks(ns)), dim3(kThreads), 0, s, ns, sub_idx.p, sub_rank.p,
                         cls_rank.p);
      HIF_HIP(hipGetLastError());
      HIF_HIP(hipStreamSynchronize(s));  // the host index list is released on return
    };
    run(sel_large, true, max_large);
    run(sel_small, false, max_small);
  } else {
    launch_id(ia, maxq, s);
  }
  tm.mark(PH_ID);

  // ---- records: sizes from the ranks ---------------------------------------
  std::vector<int32_t> h_rank, h_gpid;
  to_host(h_rank, cls_rank.p, NC, s);
  if (multi) to_host(h_gpid, gpid.p, G, s);
  std::vector<int32_t> h_grec(G, -1), h_skoff(NC), h_rdoff(NC);
  std::vector<int> rec_g;
  std::vector<int64_t> h_newoff(G, 0);
  int64_t itot = 0, dtot = 0, ntot_new = 0, skel = 0;
  double idfl = 0.0, elfl = 0.0, idby = 0.0, rqfl = 0.0;
  for (int g = 0; g < G; ++g) {
    int kk = 0, rr = 0;
    const int64_t nf = h_nf[g + 1] - h_nf[g];
    const int64_t m = sym ? nf + P : 2 * nf + 2 * P;
    for (int q = h_cls_first[g]; q < h_cls_first[g + 1]; ++q) {
      h_skoff[q] = kk;
      h_rdoff[q] = rr;
      kk += h_rank[q];
      rr += h_cls_n[q] - h_rank[q];
      const double nq = h_cls_n[q], kq = h_rank[q];
      idfl += 4.0 * m * nq * kq - 2.0 * kq * kq * (m + nq) + 4.0 * kq * kq * kq / 3.0 + kq * kq * (nq - kq);
      // sum_{i<k} (a - i)(b - i), b = columns and a = rows the pivoted QR runs on
      const double a2 = direct ? double(m) : double(std::min<int64_t>(m, h_cls_n[q]));
      const double sab = kq * a2 * nq - (a2 + nq) * kq * (kq - 1.0) / 2.0 + (kq - 1.0) * kq * (2.0 * kq - 1.0) / 6.0;
      if (direct) {
        // each step reads the trailing block once; each finished block of
        // reflectors reads and writes the rows below it once
        idby += 8.0 * sab;
        for (int e = 32; e <= h_rank[q] && e < std::min<int64_t>(m, h_cls_n[q]); e += 32)
          idby += 16.0 * (double(m) - e) * (nq - e);
      } else {
        // blocked on R0 (rows m' = min(m, n)) as on Y; in registers (k_id_reg):
        // R0 read once and rows 0..k-1 written once; otherwise every step reads
        // and writes the trailing block of R0
        if (blocked_r0 || (split_id && h_cls_n[q] > kIdRegCols)) {
          idby += 8.0 * sab;
          for (int e = 32; e <= h_rank[q] && e < a2; e += 32) idby += 16.0 * (a2 - e) * (nq - e);
        } else if (id_in_registers(split_id ? max_small : maxq, int(a2), h_cls_n[q])) {
          idby += 8.0 * (a2 + kq) * nq;
        } else {
          idby += 16.0 * sab;
        }
        if (m > h_cls_n[q]) rqfl += 2.0 * m * nq * nq - 2.0 * nq * nq * nq / 3.0;
      }
    }
    skel += kk;
    h_newoff[g] = ntot_new;
    if (rr > 0) {
      GroupRec R;
      R.r = rr;
      R.k = kk;
      R.idx = itot;
      R.off = dtot;
      h_grec[g] = int32_t(sub.hrec.size());
      sub.hrec.push_back(R);
      rec_g.push_back(g);
      itot += 3 * int64_t(rr) + kk;
      dtot += 3 * int64_t(kk) * rr + int64_t(rr) * rr;
      ntot_new += int64_t(kk) * kk;
      sub.max_r = std::max(sub.max_r, rr);
      sub.max_k = std::max(sub.max_k, kk);
      sub.max_2rk = std::max(sub.max_2rk, 2 * rr + kk);
      const double r3 = rr, k3 = kk;
      elfl += 6.0 * r3 * r3 * k3 + 4.0 * k3 * k3 * r3 + 2.0 / 3.0 * r3 * r3 * r3 + 4.0 * r3 * r3 * k3 + 2.0 * k3 * k3 * r3;
    }
  }
  if (multi) {
    rec_prob.emplace_back();
    for (int g : rec_g) rec_prob.back().push_back(h_gpid[g]);
  }
  st.sub_skel[si] = skel;
  st.sub_id_flops[si] = idfl;
  st.sub_id_bytes[si] = idby;
  st.sub_rowqr_flops[si] = rqfl;
  st.sub_elim_flops[si] = elfl;
  sub.nrec = int(sub.hrec.size());
  sub.rec.alloc(sub.nrec, mt);
  to_dev(sub.rec.p, sub.hrec, s);
  {
    std::vector<int64_t> hw(sub.nrec);
    sub.sum_r = 0;
    for (int i = 0; i < sub.nrec; ++i) {
      hw[i] = sub.sum_r;
      sub.sum_r += sub.hrec[i].r;
    }
    sub.woff.alloc(sub.nrec, mt);
    to_dev(sub.woff.p, hw, s);
  }
  sub.iarena.alloc(itot, mt);
  sub.darena.alloc(dtot, mt);
  grec.ensure(G, mt);
  to_dev(grec.p, h_grec, s);
  cls_skoff.ensure(NC, mt);
  cls_rdoff.ensure(NC, mt);
  to_dev(cls_skoff.p, h_skoff, s);
  to_dev(cls_rdoff.p, h_rdoff, s);
  newoff.ensure(G, mt);
  to_dev(newoff.p, h_newoff, s);
  newkey.ensure(ntot_new, mt);
  newval.ensure(ntot_new, mt);
  loc.ensure(nact, mt);
  rlo.ensure(nact, mt);
  rhi.ensure(nact, mt);
  tm.mark(PH_HOST);

  // ---- skeletonization and elimination -------------------------------------
  ElimArgs ea{};
  ea.ngroups = G;
  ea.cord = cord.p;
  ea.gstart = gstart.p;
  ea.grec = grec.p;
  ea.recs = sub.rec.p;
  ea.iarena = sub.iarena.p;
  ea.darena = sub.darena.p;
  ea.Y = Y.p;
  ea.yoff = yoff.p;
  ea.Acc = Acc.p;
  ea.Scc = Scc.p;
  ea.Mw = Mw.p;
  ea.aoff = aoff.p;
  ea.cls_first = cls_first.p;
  ea.cls_col0 = cls_col0.p;
  ea.cls_n = cls_n.p;
  ea.cls_rank = cls_rank.p;
  ea.cls_skoff = cls_skoff.p;
  ea.cls_rdoff = cls_rdoff.p;
  ea.perm = perm.p;
  ea.loc = loc.p;
  ea.rlo = rlo.p;
  ea.rhi = rhi.p;
  ea.newkey = newkey.p;
  ea.newval = newval.p;
  ea.newoff = newoff.p;
  ea.status = status.p;
  int max_nrec = 0;
  for (int g : rec_g) max_nrec = std::max<int>(max_nrec, int(h_gstart[g + 1] - h_gstart[g]));
  ea.max_n = max_nrec;
  ea.fp32 = H->opts.precision == HIF_FP32_MIXED;
  if (sub.nrec > 0 && (max_nrec > 256 || (sub.nrec < 256 && max_nrec > 96))) {
    // split path: setup, transform GEMMs, M_ss, batched partial LU, finish
    launch_elim_setup(ea, s);
    std::vector<GemmDesc> d1, d2;
    int mm = 1, mn = 1;
    std::vector<int64_t> hm, hp;
    std::vector<int32_t> hn, hr;
    for (int i = 0; i < sub.nrec; ++i) {
      const GroupRec& R = sub.hrec[i];
      const int g = rec_g[i];
      const int n = int(h_gstart[g + 1] - h_gstart[g]);
      double* M = Mw.p + h_aoff[g];
      double* T = sub.darena.p + R.off;
      const int r = R.r, k = R.k;
      if (k > 0) {
        d1.push_back(GemmDesc{r, r, k, 0, 0, n, r, n, -1.0, 1.0, M + r, T, M});                      // A_rr - A_rs T
        d1.push_back(GemmDesc{k, r, k, 0, 0, n, r, n, -1.0, 1.0, M + int64_t(r) * n + r, T,
                              M + int64_t(r) * n});                                                  // B_sr
        d2.push_back(GemmDesc{r, r, k, 1, 0, r, n, n, -1.0, 1.0, T, M + int64_t(r) * n, M});        // B_rr
        d2.push_back(GemmDesc{r, k, k, 1, 0, r, n, n, -1.0, 1.0, T, M + int64_t(r) * n + r, M + r}); // B_rs
        mm = std::max(mm, std::max(r, k));
        mn = std::max(mn, std::max(r, k));
      }
      hm.push_back(h_aoff[g]);
      hp.push_back(R.idx + r + k);
      hn.push_back(n);
      hr.push_back(r);
    }
    if (!d1.empty()) {
      gdesc.ensure(d1.size() + d2.size(), mt);
      std::vector<GemmDesc> all(d1);
      all.insert(all.end(), d2.begin(), d2.end());
      for (auto& d : all) d.fp32 = ea.fp32;
      to_dev(gdesc.p, all, s);
      launch_gemm_tiles(gdesc.p, int(d1.size()), mm, mn, s);
      launch_gemm_tiles(gdesc.p + d1.size(), int(d2.size()), mm, mn, s);
      launch_elim_sss(ea, s);
    }
    lu_moff.ensure(sub.nrec, mt);
    lu_poff.ensure(sub.nrec, mt);
    lu_n.ensure(sub.nrec, mt);
    lu_r.ensure(sub.nrec, mt);
    to_dev(lu_moff.p, hm, s);
    to_dev(lu_poff.p, hp, s);
    to_dev(lu_n.p, hn, s);
    to_dev(lu_r.p, hr, s);
    LuBatch lb{};
    lb.base = Mw.p;
    lb.moff = lu_moff.p;
    lb.n = lu_n.p;
    lb.r = lu_r.p;
    lb.piv = sub.iarena.p;
    lb.poff = lu_poff.p;
    lb.status = status.p;
    lb.nprob = sub.nrec;
    lb.fp32 = ea.fp32;
    launch_lu_batched(lb, sub.max_r, max_nrec, s);
    launch_elim_finish(ea, s);
    HIF_HIP(hipStreamSynchronize(s));  // descriptor tables are host vectors
  } else {
    launch_eliminate(ea, s);
  }
  if (sub.nrec > 0) launch_make_perm(sub.rec.p, sub.nrec, sub.iarena.p, sub.max_r, s);
  tm.mark(PH_ELIM);

  // ---- SCI store update, active set ----------------------------------------
  if (sub.nrec > 0) {
    hipLaunchKernelGGL(k_mark_inactive, dim3(sub.nrec), dim3(64), 0, s, sub.rec.p, sub.nrec, sub.iarena.p, active.p);
    HIF_HIP(hipGetLastError());
  }
  int64_t kept = 0;
  if (snnz > 0) {
    flag64.ensure(snnz, mt);
    pos64.ensure(snnz + 1, mt);
    hipLaunchKernelGGL(k_sci_keep, dim3(nblocks(snnz)), dim3(kThreads), 0, s, skey.p, snnz, active.p, grp_of.p, grec.p,
                       flag64.p);
    exclusive_scan_i64(flag64.p, pos64.p, snnz, s, prim, mt);
    kept = scalar_at(pos64.p + snnz, s);
  }
  const int64_t nnz2 = kept + ntot_new;
  skey2.ensure(nnz2, mt);
  sval2.ensure(nnz2, mt);
  sidx.ensure(nnz2, mt);
  sidx2.ensure(nnz2, mt);
  if (snnz > 0 && kept > 0)
    hipLaunchKernelGGL(k_sci_compact, dim3(nblocks(snnz)), dim3(kThreads), 0, s, skey.p, sval.p, snnz, flag64.p,
                       pos64.p, skey2.p, sval2.p, sidx.p);
  if (ntot_new > 0)
    hipLaunchKernelGGL(k_append, dim3(nblocks(ntot_new)), dim3(kThreads), 0, s, newkey.p, newval.p, ntot_new, kept,
                       skey2.p, sval2.p, sidx.p);
  HIF_HIP(hipGetLastError());
  skey.ensure(nnz2, mt);
  sval.ensure(nnz2, mt);
  // sort (key, idx) then gather values; keys land back in skey2 / skey
  if (nnz2 > 0) {
    sort_u64_i32(skey2.p, skey.p, sidx.p, sidx2.p, nnz2, 32 + shift, s, prim, mt);
    HIF_HIP(hipMemcpyAsync(skey.p, skey2.p, nnz2 * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_gather_val, dim3(nblocks(nnz2)), dim3(kThreads), 0, s, sval2.p, sidx.p, nnz2, sval.p);
  }
  snnz = nnz2;
  if (snnz > 0)
    hipLaunchKernelGGL(k_csr_from_sorted, dim3(nblocks(snnz)), dim3(kThreads), 0, s, skey.p, snnz, 32, N,
                       static_cast<const int64_t*>(nullptr), snnz, srow.p);
  else
    hipLaunchKernelGGL(k_fill_i64, dim3(nblocks(N + 1)), dim3(kThreads), 0, s, srow.p, N + 1, int64_t(0));
  HIF_HIP(hipGetLastError());
  // active list (every problem's DOFs, also those of problems that sat out)
  nact = nact_all;
  akeep.ensure(nact, mt);
  apos.ensure(nact + 1, mt);
  hipLaunchKernelGGL(k_active_keep, dim3(nblocks(nact)), dim3(kThreads), 0, s, act.p, nact, active.p, akeep.p);
  exclusive_scan_i32(akeep.p, apos.p, nact, s, prim, mt);
  const int64_t nact2 = scalar_at(apos.p + nact, s);
  act2.ensure(nact2, mt);
  hipLaunchKernelGGL(k_active_compact, dim3(nblocks(nact)), dim3(kThreads), 0, s, act.p, nact, akeep.p, apos.p, act2.p);
  HIF_HIP(hipGetLastError());
  std::swap(act, act2);
  nact = nact2;
  tm.mark(PH_SCI);
  tm.flush(st.t_phase_ms, st.sub_t_ms[si]);
  const int32_t bad = scalar_at(status.p, s);
  HIF_REQUIRE(bad == 0, HIF_ESINGULAR, "zero pivot in a redundant block B_rr (Lemma 2.1 needs it nonsingular)");
  H->subs.push_back(std::move(sub));
}

void Factorizer::top() {
  tm.mark(PH_HOST);
  H->ntop = nact;
  const int64_t n = nact;
  H->top_idx.alloc(n, mt);
  H->top_piv.alloc(n, mt);
  H->top_perm.alloc(n, mt);
  H->top_lu.alloc(n * n, mt);
  if (n > 0) {
    HIF_HIP(hipMemcpyAsync(H->top_idx.p, act.p, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_pos_scatter, dim3(nblocks(n)), dim3(kThreads), 0, s, act.p, n, pos_of.p);
    TopArgs ta{};
    ta.dim = D;
    ta.fp32 = H->opts.precision == HIF_FP32_MIXED;
    ta.n = n;
    ta.pts = pts;
    ta.a = a;
    ta.b = b;
    ta.c = c;
    ta.w = w;
    ta.selfk = sf;
    ta.idx = H->top_idx.p;
    ta.pos_of = pos_of.p;
    ta.srow = srow.p;
    ta.skey = skey.p;
    ta.sval = sval.p;
    ta.A = H->top_lu.p;
    ta.piv = H->top_piv.p;
    ta.status = status.p;
    launch_top(ta, s);
    if (n > 256) {  // blocked LU spread over the whole GPU
      lu_moff.ensure(1, mt);
      lu_poff.ensure(1, mt);
      lu_n.ensure(1, mt);
      lu_r.ensure(1, mt);
      std::vector<int64_t> z = {0};
      std::vector<int32_t> nn = {int32_t(n)};
      to_dev(lu_moff.p, z, s);
      to_dev(lu_poff.p, z, s);
      to_dev(lu_n.p, nn, s);
      to_dev(lu_r.p, nn, s);
      LuBatch lb{};
      lb.base = H->top_lu.p;
      lb.moff = lu_moff.p;
      lb.n = lu_n.p;
      lb.r = lu_r.p;
      lb.piv = H->top_piv.p;
      lb.poff = lu_poff.p;
      lb.status = status.p;
      lb.nprob = 1;
      launch_lu_batched(lb, int(n), int(n), s);
      HIF_HIP(hipStreamSynchronize(s));
    }
    launch_make_perm_top(H->top_piv.p, H->top_perm.p, int(n), s);
  }
  tm.mark(PH_TOP);
  tm.flush(H->stats.t_phase_ms);
  const int32_t bad = scalar_at(status.p, s);
  HIF_REQUIRE(bad == 0, HIF_ESINGULAR, "zero pivot in the top block A_L (Lemma 2.1 needs it nonsingular)");
}

// Top blocks of several problems factored together: each problem's active
// DOFs (a contiguous range of the ascending active list) form its A_L; the
// blocks are assembled one by one, LU-factored together (one batched launch
// sequence for all blocks above 256 unknowns) and handed to the problems'
// handles with indices local to each problem.
void Factorizer::top_multi(const std::vector<hif_factor_s*>& hs) {
  tm.mark(PH_HOST);
  std::vector<int64_t> bounds(nprob + 1, 0);
  bounds[nprob] = nact;
  cut.ensure(1, mt);
  for (int q = 1; q < nprob; ++q) {
    hipLaunchKernelGGL(k_count_below, dim3(1), dim3(64), 0, s, act.p, nact, int32_t(poff[q]), cut.p);
    HIF_HIP(hipGetLastError());
    bounds[q] = scalar_at(cut.p, s);
  }
  std::vector<int64_t> aoffs(nprob + 1, 0), ioffs(nprob + 1, 0);
  for (int q = 0; q < nprob; ++q) {
    const int64_t n = bounds[q + 1] - bounds[q];
    aoffs[q + 1] = aoffs[q] + n * n;
    ioffs[q + 1] = ioffs[q] + n;
  }
  DBuf<double> lu;
  DBuf<int32_t> piv;
  lu.alloc(aoffs[nprob], mt);
  piv.alloc(ioffs[nprob], mt);
  std::vector<int64_t> hm, hp;
  std::vector<int32_t> hn;
  int maxn = 0;
  for (int q = 0; q < nprob; ++q) {
    const int64_t n = bounds[q + 1] - bounds[q];
    if (n == 0) continue;
    const int32_t* gidx = act.p + bounds[q];
    hipLaunchKernelGGL(k_pos_scatter, dim3(nblocks(n)), dim3(kThreads), 0, s, gidx, n, pos_of.p);
    TopArgs ta{};
    ta.dim = D;
    ta.fp32 = H->opts.precision == HIF_FP32_MIXED;
    ta.n = n;
    ta.pts = pts;
    ta.a = a;
    ta.b = b;
    ta.c = c;
    ta.w = w;
    ta.selfk = sf;
    ta.idx = gidx;
    ta.pos_of = pos_of.p;
    ta.srow = srow.p;
    ta.skey = skey.p;
    ta.sval = sval.p;
    ta.A = lu.p + aoffs[q];
    ta.piv = piv.p + ioffs[q];
    ta.status = status.p;
    launch_top(ta, s);
    if (n > 256) {
      hm.push_back(aoffs[q]);
      hp.push_back(ioffs[q]);
      hn.push_back(int32_t(n));
      maxn = std::max<int>(maxn, int(n));
    }
  }
  if (!hn.empty()) {  // blocked LU of every block above 256 unknowns in one launch sequence
    const int nb = int(hn.size());
    lu_moff.ensure(nb, mt);
    lu_poff.ensure(nb, mt);
    lu_n.ensure(nb, mt);
    lu_r.ensure(nb, mt);
    to_dev(lu_moff.p, hm, s);
    to_dev(lu_poff.p, hp, s);
    to_dev(lu_n.p, hn, s);
    to_dev(lu_r.p, hn, s);
    LuBatch lb{};
    lb.base = lu.p;
    lb.moff = lu_moff.p;
    lb.n = lu_n.p;
    lb.r = lu_r.p;
    lb.piv = piv.p;
    lb.poff = lu_poff.p;
    lb.status = status.p;
    lb.nprob = nb;
    launch_lu_batched(lb, maxn, maxn, s);
    HIF_HIP(hipStreamSynchronize(s));
  }
  for (int q = 0; q < nprob; ++q) {
    hif_factor_s* Hq = hs[q];
    const int64_t n = bounds[q + 1] - bounds[q];
    Hq->ntop = n;
    Hq->top_idx.alloc(n, &Hq->mem);
    Hq->top_piv.alloc(n, &Hq->mem);
    Hq->top_perm.alloc(n, &Hq->mem);
    Hq->top_lu.alloc(n * n, &Hq->mem);
    if (n == 0) continue;
    hipLaunchKernelGGL(k_sub_i32, dim3(nblocks(n)), dim3(kThreads), 0, s, act.p + bounds[q], n, int32_t(poff[q]),
                       Hq->top_idx.p);
    HIF_HIP(hipMemcpyAsync(Hq->top_lu.p, lu.p + aoffs[q], sizeof(double) * n * n, hipMemcpyDeviceToDevice, s));
    HIF_HIP(hipMemcpyAsync(Hq->top_piv.p, piv.p + ioffs[q], sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    launch_make_perm_top(Hq->top_piv.p, Hq->top_perm.p, int(n), s);
  }
  HIF_HIP(hipGetLastError());
  tm.mark(PH_TOP);
  tm.flush(H->stats.t_phase_ms);
  const int32_t bad = scalar_at(status.p, s);
  HIF_REQUIRE(bad == 0, HIF_ESINGULAR, "zero pivot in a top block A_L (Lemma 2.1 needs it nonsingular)");
}

}  // namespace

// ---------------------------------------------------------------------------
// Copies the operator into the handle (points, then a (0 if absent), b, c
// (1 if absent), weight (h^d) and self term), checks the inputs, decides the
// symmetric compression (Section 5: b_i = s c_i w_i for one scalar s) and the
// tree depth (boxes split while they hold more than leaf points; only trees
// whose leaves all sit at one depth are handled, Section 3.1), and rejects
// coincident points.
void prepare_problem(hif_factor_s* H, const double* points, const hif_kernel* kr, const double* a_in,
                     const double* b_in, const double* c_in, hipStream_t s) {
  const int D = H->dim;
  const int64_t N = H->n;
  MemTracker* mt = &H->mem;
  DBuf<double>& op = H->op;
  op.alloc(int64_t(N) * (D + 5), mt);
  double* pts = op.p;
  double* a = pts + N * D;
  double* b = a + N;
  double* c = b + N;
  double* w = c + N;
  double* sf = w + N;
  HIF_HIP(hipMemcpyAsync(pts, points, sizeof(double) * N * D, hipMemcpyDeviceToDevice, s));
  auto fill_or_copy = [&](double* dst, const double* src, double v) {
    if (src)
      HIF_HIP(hipMemcpyAsync(dst, src, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    else
      hipLaunchKernelGGL(k_fill_f64, dim3(nblocks(N)), dim3(kThreads), 0, s, dst, N, v);
  };
  fill_or_copy(a, a_in, 0.0);
  fill_or_copy(b, b_in, 1.0);
  fill_or_copy(c, c_in, 1.0);
  fill_or_copy(w, kr->weights, std::pow(kr->h, D));
  fill_or_copy(sf, kr->self, kr->self ? 0.0 : self_integral(kr->h, D));
  HIF_HIP(hipGetLastError());
  H->pts = pts;
  H->a = a;
  H->b = b;
  H->c = c;
  H->w = w;
  H->selfk = sf;

  DBuf<int32_t> status;
  status.alloc(2, mt);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, status.p, int64_t(2), 0);
  hipLaunchKernelGGL(k_validate, dim3(nblocks(N)), dim3(kThreads), 0, s, pts, N, D, a, b, c, w, sf, status.p);
  HIF_HIP(hipGetLastError());
  const int32_t vflags = scalar_at(status.p, s);
  HIF_REQUIRE(!(vflags & 1), HIF_EINVAL, "non-finite point coordinate");
  HIF_REQUIRE(!(vflags & 2), HIF_EINVAL, "point outside the unit box [0,1]^d");
  HIF_REQUIRE(!(vflags & 4), HIF_EINVAL, "non-finite a, b, c, weight or self term");

  if (H->opts.symmetric < 0) {
    std::vector<double> hb, hc, hw;
    to_host(hb, b, N, s);
    to_host(hc, c, N, s);
    to_host(hw, w, N, s);
    bool sym = true;
    const double cw0 = hc[0] * hw[0], b0 = hb[0];
    for (int64_t i = 0; i < N && sym; ++i) sym = (hb[i] * cw0 == hc[i] * hw[i] * b0);
    H->symmetric = sym ? 1 : 0;
  } else {
    H->symmetric = H->opts.symmetric;
  }

  {
    DBuf<int32_t> counts, mm;
    mm.alloc(2, mt);
    // Depths with fewer than N / leaf boxes always hold a box with more than
    // leaf points; start one depth before the first that could satisfy the
    // rule (its minimum count decides uniformity when the rule holds at once).
    int L0 = 0;
    while (L0 < 24 && (int64_t(1) << (D * L0)) * int64_t(H->leaf) < N) ++L0;
    int L = L0 > 0 ? L0 - 1 : 0;
    int32_t prev_min = INT_MAX;
    for (;;) {
      const int64_t S = int64_t(1) << L;
      int64_t nb = 1;
      for (int k = 0; k < D; ++k) nb *= S;
      HIF_REQUIRE(nb <= 64 * N + 4096 && L <= 24, HIF_EUNSUPPORTED,
                  "adaptive tree too deep for a uniform-depth factorization (clustered or coincident points)");
      counts.ensure(nb, mt);
      hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(nb)), dim3(kThreads), 0, s, counts.p, nb, 0);
      if (D == 2)
        hipLaunchKernelGGL(k_box_count<2>, dim3(nblocks(N)), dim3(kThreads), 0, s, pts, N, int(S), counts.p);
      else
        hipLaunchKernelGGL(k_box_count<3>, dim3(nblocks(N)), dim3(kThreads), 0, s, pts, N, int(S), counts.p);
      std::vector<int32_t> init = {INT_MAX, 0};
      to_dev(mm.p, init, s);
      hipLaunchKernelGGL(k_minmax, dim3(nblocks(nb)), dim3(kThreads), 0, s, counts.p, nb, mm.p);
      HIF_HIP(hipGetLastError());
      std::vector<int32_t> h;
      to_host(h, mm.p, 2, s);
      if (h[1] <= H->leaf) break;
      prev_min = h[0];
      ++L;
    }
    HIF_REQUIRE(L == 0 || prev_min > H->leaf, HIF_EUNSUPPORTED,
                "adaptive tree leaves are not all at one depth (non-uniform point distribution)");
    H->L = L;
  }
  HIF_REQUIRE(H->L <= HIF_MAX_SUBLEVELS / 3, HIF_EUNSUPPORTED, "tree deeper than the statistics arrays allow");

  // coincident points: compare pairs inside every leaf box
  {
    const int S = 1 << H->L;
    int ncell = 1;
    for (int k = 0; k < D; ++k) ncell *= S;
    DBuf<int32_t> iota, ckey, cdof, ktmp, vtmp, lo, hi;
    DBuf<unsigned char> prim;
    iota.alloc(N, mt);
    ckey.alloc(N, mt);
    cdof.alloc(N, mt);
    ktmp.alloc(N, mt);
    vtmp.alloc(N, mt);
    lo.alloc(ncell, mt);
    hi.alloc(ncell, mt);
    hipLaunchKernelGGL(k_iota, dim3(nblocks(N)), dim3(kThreads), 0, s, iota.p, N);
    if (D == 2)
      hipLaunchKernelGGL(k_group_key<2>, dim3(nblocks(N)), dim3(kThreads), 0, s, pts, iota.p, N, 0, S, ckey.p,
                         cdof.p, ProbGeo{}, 0);
    else
      hipLaunchKernelGGL(k_group_key<3>, dim3(nblocks(N)), dim3(kThreads), 0, s, pts, iota.p, N, 0, S, ckey.p,
                         cdof.p, ProbGeo{}, 0);
    sort_i32_i32(ckey.p, ktmp.p, cdof.p, vtmp.p, N, ceil_log2(uint64_t(ncell) + 1), s, prim, mt);
    hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(ncell)), dim3(kThreads), 0, s, lo.p, int64_t(ncell), 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(ncell)), dim3(kThreads), 0, s, hi.p, int64_t(ncell), 0);
    hipLaunchKernelGGL(k_cell_table, dim3(nblocks(N)), dim3(kThreads), 0, s, ckey.p, N, lo.p, hi.p);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, status.p, int64_t(2), 0);
    hipLaunchKernelGGL(k_coincident, dim3(ncell), dim3(kThreads), 0, s, pts, D, cdof.p, lo.p, hi.p, status.p);
    HIF_HIP(hipGetLastError());
    const int32_t dup = scalar_at(status.p, s);
    HIF_REQUIRE(dup == 0, HIF_EINVAL, "coincident points (the kernel is singular at r = 0)");
  }
}

namespace {

// Proxy directions (Section 3.3): circle p -> (cos 2 pi p / P, sin 2 pi p / P);
// sphere: spherical Fibonacci points z = 1 - (2p+1)/P, phi = p pi (3 - sqrt 5).
std::vector<double> proxy_directions(int D, int P) {
  std::vector<double> u(size_t(P) * D);
  for (int p = 0; p < P; ++p) {
    if (D == 2) {
      const double t = 2.0 * M_PI * double(p) / double(P);
      u[2 * p] = std::cos(t);
      u[2 * p + 1] = std::sin(t);
    } else {
      const double z = 1.0 - (2.0 * p + 1.0) / double(P);
      const double rho = std::sqrt(1.0 - z * z);
      const double phi = double(p) * M_PI * (3.0 - std::sqrt(5.0));
      u[3 * p] = rho * std::cos(phi);
      u[3 * p + 1] = rho * std::sin(phi);
      u[3 * p + 2] = z;
    }
  }
  return u;
}

// Sub-level kinds of one level: cells, then (faces and) edges; RSF: cells only.
std::vector<int> level_kinds(const hif_factor_s* H) {
  if (H->opts.variant == HIF_VARIANT_RSF) return {0};
  if (H->dim == 2) return {0, 2};
  return {0, 1, 2};
}

// Factorizer state for the DOFs of a handle whose operator is in place:
// everything active, no SCIs, no groups.
void init_state(Factorizer& F) {
  const int64_t N = F.N;
  MemTracker* mt = F.mt;
  hipStream_t s = F.s;
  F.status.alloc(2, mt);
  F.active.alloc(N, mt);
  F.act.alloc(N, mt);
  F.grp_of.alloc(N, mt);
  F.pos_of.alloc(N, mt);
  F.srow.alloc(N + 1, mt);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, F.status.p, int64_t(2), 0);
  hipLaunchKernelGGL(k_fill_u8, dim3(nblocks(N)), dim3(kThreads), 0, s, F.active.p, N, uint8_t(1));
  hipLaunchKernelGGL(k_iota, dim3(nblocks(N)), dim3(kThreads), 0, s, F.act.p, N);
  hipLaunchKernelGGL(k_fill_i64, dim3(nblocks(N + 1)), dim3(kThreads), 0, s, F.srow.p, N + 1, int64_t(0));
  hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(N)), dim3(kThreads), 0, s, F.grp_of.p, N, -1);
  HIF_HIP(hipGetLastError());
  F.nact = N;
  const std::vector<double> u = proxy_directions(F.D, F.H->nproxy);
  F.proxy_u.alloc(u.size(), mt);
  to_dev(F.proxy_u.p, u, s);
}

// m_f and the per-handle statistics that follow from the records.
void record_stats(hif_factor_s* H) {
  hif_stats_t& st = H->stats;
  st.n = H->n;
  st.dim = H->dim;
  st.levels = H->L;
  st.n_sublevels = int32_t(H->subs.size());
  st.top_size = H->ntop;
  int64_t fb = 0;
  for (auto& sub : H->subs)
    for (auto& R : sub.hrec) fb += 8 * (3 * int64_t(R.k) * R.r + int64_t(R.r) * R.r) + 4 * (2 * int64_t(R.r) + R.k);
  fb += 8 * H->ntop * H->ntop + 8 * H->ntop;
  st.factor_bytes = fb;
}

}  // namespace

void factor_impl(hif_factor_s* H, const double* points, const hif_kernel* kr, const double* a_in,
                 const double* b_in, const double* c_in, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  prepare_problem(H, points, kr, a_in, b_in, c_in, s);
  Factorizer F{};
  F.H = H;
  F.s = s;
  F.D = H->dim;
  F.N = H->n;
  F.mt = &H->mem;
  F.tm.s = s;
  F.pts = H->pts;
  F.a = H->a;
  F.b = H->b;
  F.c = H->c;
  F.w = H->w;
  F.sf = H->selfk;
  init_state(F);
  const std::vector<int> kinds = level_kinds(H);
  for (int lvl = 0; lvl < H->L; ++lvl)
    for (int kind : kinds) F.sublevel(lvl, kind);
  F.top();
  record_stats(H);
  prepare_sweeps(H, s);
  HIF_HIP(hipStreamSynchronize(s));
  H->stats.t_factor_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  // the blocks this factorization released on the caller's stream are idle
  // now: any stream may take them (and the oldest may be evicted), rather
  // than only later work on this stream
  dbuf_retire_stream(s);
}

void factor_fused_impl(const std::vector<hif_factor_s*>& hs_in, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  const int P = int(hs_in.size());
  if (P == 0) return;
  // deepest tree first: the problems that take part in a level then hold a
  // prefix of the active list
  std::vector<hif_factor_s*> hs(hs_in);
  std::stable_sort(hs.begin(), hs.end(), [](const hif_factor_s* x, const hif_factor_s* y) { return x->L > y->L; });
  const int D = hs[0]->dim;
  std::vector<int64_t> poff(P + 1, 0);
  for (int q = 0; q < P; ++q) poff[q + 1] = poff[q] + hs[q]->n;
  const int64_t N = poff[P];
  HIF_REQUIRE(N <= int64_t(INT32_MAX) - 1, HIF_EINVAL, "the problems of a fused batch must have fewer than 2^31 points in all");
  // the batch as one operator: points and coefficients concatenated
  hif_factor_s B;
  B.n = N;
  B.dim = D;
  B.L = hs[0]->L;
  B.eps = hs[0]->eps;
  B.leaf = hs[0]->leaf;
  B.opts = hs[0]->opts;
  B.symmetric = hs[0]->symmetric;
  B.nproxy = hs[0]->nproxy;
  B.proxy_r = hs[0]->proxy_r;
  B.mem.cap = hs[0]->opts.max_bytes;
  MemTracker* mt = &B.mem;
  B.op.alloc(N * (D + 5), mt);
  double* pts = B.op.p;
  double* co[5];
  for (int t = 0; t < 5; ++t) co[t] = pts + N * D + int64_t(t) * N;
  for (int q = 0; q < P; ++q) {
    const hif_factor_s* Hq = hs[q];
    const int64_t n = Hq->n;
    HIF_HIP(hipMemcpyAsync(pts + poff[q] * D, Hq->pts, sizeof(double) * n * D, hipMemcpyDeviceToDevice, s));
    const double* src[5] = {Hq->a, Hq->b, Hq->c, Hq->w, Hq->selfk};
    for (int t = 0; t < 5; ++t)
      HIF_HIP(hipMemcpyAsync(co[t] + poff[q], src[t], sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  }
  B.pts = pts;
  B.a = co[0];
  B.b = co[1];
  B.c = co[2];
  B.w = co[3];
  B.selfk = co[4];
  Factorizer F{};
  F.H = &B;
  F.s = s;
  F.D = D;
  F.N = N;
  F.mt = mt;
  F.tm.s = s;
  F.pts = B.pts;
  F.a = B.a;
  F.b = B.b;
  F.c = B.c;
  F.w = B.w;
  F.sf = B.selfk;
  F.multi = true;
  F.nprob = P;
  F.poff = poff;
  for (int q = 0; q < P; ++q) {
    F.pL.push_back(hs[q]->L);
    F.peps.push_back(hs[q]->eps);
  }
  F.pid.alloc(N, mt);
  for (int q = 0; q < P; ++q)
    hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(hs[q]->n)), dim3(kThreads), 0, s, F.pid.p + poff[q], hs[q]->n,
                       int32_t(q));
  init_state(F);
  const std::vector<int> kinds = level_kinds(&B);
  for (int lvl = 0; lvl < B.L; ++lvl)
    for (int kind : kinds) F.sublevel(lvl, kind);
  F.top_multi(hs);

  // Each problem's records, copied out of the batch's sub-levels into its
  // own handle with DOF indices local to the problem.
  for (size_t si = 0; si < B.subs.size(); ++si) {
    SubLevel& bs = B.subs[si];
    const std::vector<int32_t>& rp = F.rec_prob[si];
    int rb = 0;
    for (int q = 0; q < P; ++q) {
      if (hs[q]->L <= bs.level) continue;
      int re = rb;
      while (re < bs.nrec && rp[re] == q) ++re;
      hif_factor_s* Hq = hs[q];
      SubLevel out;
      out.level = bs.level;
      out.kind = bs.kind;
      out.nrec = re - rb;
      const int sq = int(Hq->subs.size());
      Hq->stats.sub_kind[sq] = bs.kind;
      if (out.nrec > 0) {
        const GroupRec& R0 = bs.hrec[rb];
        const GroupRec& R1 = bs.hrec[re - 1];
        const int64_t i0 = R0.idx, i1 = R1.idx + 3 * int64_t(R1.r) + R1.k;
        const int64_t d0 = R0.off, d1 = R1.off + 3 * int64_t(R1.k) * R1.r + int64_t(R1.r) * R1.r;
        out.iarena.alloc(i1 - i0, &Hq->mem);
        out.darena.alloc(d1 - d0, &Hq->mem);
        HIF_HIP(hipMemcpyAsync(out.iarena.p, bs.iarena.p + i0, sizeof(int32_t) * (i1 - i0),
                               hipMemcpyDeviceToDevice, s));
        HIF_HIP(hipMemcpyAsync(out.darena.p, bs.darena.p + d0, sizeof(double) * (d1 - d0),
                               hipMemcpyDeviceToDevice, s));
        std::vector<int64_t> hw(out.nrec);
        for (int i = rb; i < re; ++i) {
          GroupRec R = bs.hrec[i];
          R.idx -= i0;
          R.off -= d0;
          hw[i - rb] = out.sum_r;
          out.sum_r += R.r;
          out.max_r = std::max(out.max_r, R.r);
          out.max_k = std::max(out.max_k, R.k);
          out.max_2rk = std::max(out.max_2rk, 2 * R.r + R.k);
          Hq->stats.sub_skel[sq] += R.k;
          out.hrec.push_back(R);
        }
        out.rec.alloc(out.nrec, &Hq->mem);
        to_dev(out.rec.p, out.hrec, s);
        out.woff.alloc(out.nrec, &Hq->mem);
        to_dev(out.woff.p, hw, s);
        hipLaunchKernelGGL(k_rebase_records, dim3(out.nrec), dim3(64), 0, s, out.rec.p, out.nrec, out.iarena.p,
                           int32_t(poff[q]));
        HIF_HIP(hipGetLastError());
        HIF_HIP(hipStreamSynchronize(s));  // the host tables above are copied before they go out of scope
      }
      Hq->stats.sub_groups[sq] = out.nrec;
      Hq->subs.push_back(std::move(out));
      rb = re;
    }
    // the batch's copy is no longer needed
    bs.iarena.release();
    bs.darena.release();
  }
  HIF_HIP(hipStreamSynchronize(s));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (int q = 0; q < P; ++q) {
    hif_factor_s* Hq = hs[q];
    record_stats(Hq);
    // phase times and the wall time are those of the whole batch
    for (int k = 0; k < 8; ++k) Hq->stats.t_phase_ms[k] = B.stats.t_phase_ms[k];
    Hq->stats.t_factor_ms = ms;
    prepare_sweeps(Hq, s);
  }
  HIF_HIP(hipStreamSynchronize(s));
}

void partition_impl(const double* pts, int64_t n, int dim, const uint8_t* active, int kind, int32_t S,
                    int32_t* group, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(k_partition<2>, dim3(nblocks(n)), dim3(kThreads), 0, s, pts, n, active, kind, S, group);
  else
    hipLaunchKernelGGL(k_partition<3>, dim3(nblocks(n)), dim3(kThreads), 0, s, pts, n, active, kind, S, group);
  HIF_HIP(hipGetLastError());
  HIF_HIP(hipStreamSynchronize(s));
}

}  // namespace hif
