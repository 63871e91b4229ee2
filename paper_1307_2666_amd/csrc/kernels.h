// Launch interfaces of the per-group dense kernels (dense.hip) used by the
// factorization driver (factor.hip).  Internal, not part of the ABI.
#pragma once

#include "common.h"

namespace hif {

// Batched assembly of the compressed blocks Y_c (eqn proxy-id; the column
// block Y'_c of Section 5 when symmetric) and of A_cc, one workgroup per group.
struct AsmArgs {
  int dim = 2, sym = 1, nproxy = 64, ngroups = 0;
  int max_rows = 0, max_cols = 0;  // max over groups of rows(Y_c) + n_c, and of n_c
  int fp32 = 0;                 // mixed precision: kernel entries evaluated and rounded in FP32
  double R = 0;                 // absolute proxy radius of this sub-level
  const double *pts, *a, *b, *c, *w, *selfk;
  const double* proxy_u;        // [nproxy][dim] unit directions
  const int32_t* cord;          // group DOFs, class order, groups concatenated
  const int64_t* gstart;        // [G+1]
  const int32_t* nf_idx;        // near-field DOFs (ascending per group)
  const int64_t* nf_start;      // [G+1]
  const double* zc;             // [G][dim] group centres
  const int64_t* yoff;          // [G] offset of Y_c (row-major m x n)
  const int64_t* aoff;          // [G] offset of A_cc / S_cc (row-major n x n)
  double *Y, *Acc, *Scc;
  double *colK2, *colS2;        // per cord position: squared norms of kernel / SCI part of Y
  double* kpart;                // [row chunk][kstride]: partial squared norms of the kernel part
  int64_t kstride = 0;          // = number of cord positions of the sub-level
  const int32_t* grp_of;        // per DOF: group of this sub-level (-1 inactive)
  const int32_t* pos_of;        // per DOF: position within its group (class order)
  const int64_t* srow;          // SCI store CSR row pointer [N+1]
  const uint64_t* skey;         // (i << 32 | j)
  const double2* sval;          // (S_ij, S_ji)
  // several problems factored together: problem of each group and proxy
  // radius of each problem (nullptr: one problem, radius R)
  const int32_t* gpid = nullptr;
  const double* pR = nullptr;
};
void launch_assemble(const AsmArgs& A, hipStream_t s);

// Batched interpolative decomposition by column-pivoted Householder QR
// (Lemma 2.2, Section 2.2), one workgroup per problem, in place.
struct IdArgs {
  double* base;
  const int64_t* moff;   // offset of element (0,0) of problem q
  const int32_t* ld;     // row stride (row-major)
  const int32_t* rows;
  const int32_t* cols;
  const double* tol;
  int32_t* rank;
  int32_t* perm;         // per problem: cols entries (skeleton pivots, then redundant ascending)
  const int64_t* poff;
  double* Tout;          // optional compact copy of T (k x r row-major)
  const int64_t* toff;
  int nprob = 0;
  // one-workgroup ID only: when alpha is set, R_ii goes to alpha[q * astride + i]
  // and T is left to the blocked triangular solve; problems with at most
  // skip_cols columns are left to another kernel
  double* alpha = nullptr;
  int64_t astride = 0;
  int skip_cols = 0;
};
void launch_id(const IdArgs& A, int max_cols, hipStream_t s);
// Blocked pivoted QR on the uncompressed problems (rows up to max_rows), same
// outputs as launch_id; id_blocked_fits says whether a batch suits it.
void launch_id_blocked(const IdArgs& A, int max_rows, int max_cols, hipStream_t s);
bool id_blocked_fits(int nprob, int max_rows, int max_cols);
// Whether launch_id runs a problem of rows x cols (after row compression) in
// registers, in a batch whose widest problem has max_cols columns.
inline bool id_in_registers(int max_cols, int rows, int cols) {
  if (max_cols <= 48) return false;
  if (max_cols <= 128) return true;
  return max_cols <= 256 && cols <= 192 && rows <= 192;
}

// Row compression Y = Q R0 (blocked Householder, no pivoting) before the ID;
// R0 overwrites the leading n x n block of each problem with m > n.
struct RowQrArgs {
  double* base;
  const int64_t* moff;
  const int32_t* ld;
  const int32_t* rows;
  const int32_t* cols;
  double* scratch;       // per problem: rowqr_scratch(m, n) doubles
  const int64_t* soff;
  int nprob = 0;
};
void launch_rowqr(const RowQrArgs& A, hipStream_t s);
void launch_rowqr_auto(const RowQrArgs& A, int max_rows, int max_cols, hipStream_t s);

// Batched skeletonization + elimination (Lemma 2.4 with Lemma 2.1), one
// workgroup per group with a record.
struct ElimArgs {
  int ngroups = 0;
  int max_n = 0;               // largest group of the sub-level (sizes the copy grids)
  int fp32 = 0;                // mixed precision: transform GEMMs on FP32 matrix cores
  const int32_t* cord;
  const int64_t* gstart;
  const int32_t* grec;          // [G] record index or -1
  const GroupRec* recs;
  int32_t* iarena;
  double* darena;
  const double* Y;              // IDs in place (T_q in rows 0..k_q-1)
  const int64_t* yoff;
  const double* Acc;
  const double* Scc;
  double* Mw;                   // workspace, same layout as Acc
  const int64_t* aoff;
  const int32_t* cls_first;     // [G+1] classes of group g
  const int32_t* cls_col0;      // group-local first column of class q
  const int32_t* cls_n;         // columns of class q
  const int32_t* cls_rank;      // skeleton size of class q
  const int32_t* cls_skoff;     // offset of class q within the group's skeleton list
  const int32_t* cls_rdoff;     // offset of class q within the group's redundant list
  const int32_t* perm;          // class perms, slot at gstart[g] + col0
  int32_t* loc;                 // scratch [total group size]: rd_loc then sk_loc
  int32_t* rlo;                 // scratch [total group size]
  int32_t* rhi;
  uint64_t* newkey;             // new SCI entries (k x k per group)
  double2* newval;
  const int64_t* newoff;        // [G]
  int32_t* status;              // set to 1 on a zero pivot
};
void launch_eliminate(const ElimArgs& A, hipStream_t s);
void launch_elim_setup(const ElimArgs& A, hipStream_t s);
void launch_elim_sss(const ElimArgs& A, hipStream_t s);
void launch_elim_finish(const ElimArgs& A, hipStream_t s);

// Top block A_L(s_L, s_L) = diag(a) + bKc + S, then LU with partial pivoting.
struct TopArgs {
  int dim = 2;
  int fp32 = 0;                 // mixed precision: kernel entries in FP32
  int64_t n = 0;
  const double *pts, *a, *b, *c, *w, *selfk;
  const int32_t* idx;           // top DOFs ascending
  const int32_t* pos_of;        // per DOF: position in idx
  const int64_t* srow;
  const uint64_t* skey;
  const double2* sval;
  double* A;                    // n x n row-major
  int32_t* piv;
  int32_t* status;
};
void launch_top(const TopArgs& A, hipStream_t s);

}  // namespace hif
