/*
 * hif.h -- C ABI of the MI355X (gfx950) HIF-IE library.
 *
 * Hierarchical interpolative factorization for integral equations
 * (K. L. Ho and L. Ying, arXiv 1307.2666).  The library factors the dense
 * matrix of the discretized integral equation
 *
 *     a(x) u(x) + b(x) int K(|x - y|) c(y) u(y) dy = f(x)          (eqn 1.1)
 *
 * on collocation points x_i:  A = diag(a) + diag(b) K diag(c), with
 * K_ij = G(|x_i - x_j|) w_j for i != j (one-point rule, Section 5) and K_ii the
 * integral of G over the element of x_i (eqn kernel-integral, Section 3.1).
 * G is the Laplace fundamental solution (eqn laplace-kernel): -log(r)/(2 pi)
 * in 2D, 1/(4 pi r) in 3D.  The factorization F ~ A is the generalized LU
 * decomposition of eqns (hifie2) / (hifie3) built by Algorithms 4.1 / 4.2
 * (or the RSF of Algorithm 3.1, eqn rskelf); F and F^{-1} are applied in
 * factored form.
 *
 * Conventions for every call:
 *  - Pointers to arrays are DEVICE pointers on the current HIP device unless
 *    stated otherwise.  All floating point arrays are IEEE double.
 *  - points: [n][dim] row-major (point i at points[i*dim .. i*dim+dim-1]),
 *    inside the closed unit box [0,1]^dim.
 *  - a, b, c, weights, self: [n], in the caller's point order.
 *  - Right-hand sides and solutions: [nrhs][n], each vector contiguous,
 *    caller's point order.  In-place calls (x == y, f == u) are allowed.
 *  - stream: a hipStream_t passed as void* (NULL = the null stream).
 *  - Inputs are borrowed for the duration of the call only; hif_factor copies
 *    what later calls need into the handle.  The handle owns all device
 *    memory it allocates until hif_free.  A handle serves one stream at a
 *    time.
 *  - Errors: every call returns a hif_status; negative values are errors and
 *    hif_last_error() gives a message (thread-local).  Nothing is thrown
 *    across the ABI.  Argument checks that need no device data (NULL
 *    pointers, sizes, dim, eps, leaf, option ranges) run on the host before
 *    any device work.
 */
#ifndef HIF_H
#define HIF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hif_factor_s* hif_handle;  /* opaque, library-owned */
typedef void* hif_stream;                 /* hipStream_t */

typedef enum {
  HIF_OK = 0,
  HIF_EINVAL = -1,        /* bad argument, non-finite input, point outside [0,1]^d, coincident points */
  HIF_ENOMEM = -2,        /* device allocation failed or opts.max_bytes exceeded */
  HIF_ESINGULAR = -3,     /* zero pivot in a redundant block B_rr or the top block (Lemma 2.1) */
  HIF_EDEVICE = -4,       /* HIP runtime error */
  HIF_EUNSUPPORTED = -5   /* valid request the library does not handle (e.g. non-uniform tree depth) */
} hif_status;

enum { HIF_FP64 = 0, HIF_FP32_MIXED = 1 };
enum { HIF_VARIANT_HIFIE = 0, HIF_VARIANT_RSF = 1 };

/*
 * Kernel description (Laplace only).  Off-diagonal weight w_j = weights[j]
 * if given, else h^dim.  Diagonal K_ii = self[i] if given, else the closed
 * form of the integral of G over the cube of side h centred at x_i:
 *   2D: -(h^2/(2 pi)) (log(h/sqrt 2) - 3/2 + pi/4),
 *   3D: h^2 (3 log(2 + sqrt 3) - pi/2) / (4 pi).
 */
typedef struct {
  double h;                 /* grid step (> 0 unless both arrays are given) */
  const double* weights;    /* optional [n] device */
  const double* self;       /* optional [n] device */
} hif_kernel;

/*
 * Factorization options.  hif_opts_default fills the defaults.
 *  precision:    HIF_FP64, or HIF_FP32_MIXED: kernel entries evaluated and
 *                rounded in FP32, the skeletonization GEMMs and the Schur
 *                update of the skeleton block on FP32 matrix cores with FP32
 *                accumulation; the row compression, pivoted QR (rank
 *                decisions), the LU of the redundant blocks and of the top
 *                block, the SCI store and the sweeps stay FP64.  Meant as a
 *                preconditioner for hif_gmres.
 *  second_kind:  1 = Section 4.4 modification (rho-scaled local tolerance and
 *                split compression by SCI sparsity pattern; "hifie2x/3x"),
 *                0 = plain compression, -1 = auto (1 in FP64, 0 in FP32_MIXED).
 *  symmetric:    1 = compress only the column block Y'_c (Section 5; valid
 *                when A is symmetric), 0 = full Y_c of eqn proxy-id,
 *                -1 = auto (symmetric iff b_i == s c_i w_i for one scalar s).
 *  variant:      HIF_VARIANT_HIFIE (Algorithms 4.1/4.2) or HIF_VARIANT_RSF
 *                (Algorithm 3.1, cells only).
 *  n_proxy:      proxy points, 0 = 64 (2D circle) / 512 (3D sphere) (Section 3.3).
 *  proxy_radius: proxy radius in units of the cell width, 0 = 1.5 (Section 3.3).
 *  max_bytes:    cap on device memory the factorization may hold, 0 = none.
 *  row_compression: how the IDs of a sub-level with few large problems run
 *                (Section 2.2 leaves the QR organization open):
 *                1 = Householder QR of Y first, then the pivoted QR of its
 *                n x n R factor; 0 = pivoted QR directly on Y; -1 = auto
 *                (0 only when Y is nearly square: sum of m n over the
 *                sub-level's problems at most 1.25 times the sum of n^2).
 *                Either way the pivoted QR delays the updates of 32
 *                reflectors; both give the same ID up to rounding.
 *  trace_sublevel: -1 (default) = nothing; s >= 0 = keep copies of
 *                sub-level s's groups, near fields and assembled blocks for
 *                hif_trace_get (step-by-step checks; costs memory and time).
 *  fft_matvec:   products with the exact operator inside hif_gmres,
 *                hif_gmres_T and hif_apply_A: 0 (default) = pair by pair,
 *                evaluated on the fly as hif_matvec; 1 = by FFT convolution
 *                when the points form the full uniform grid with constant
 *                weights and self terms (see hif_apply_A), else pair by pair.
 *  sweep_wait_us: bound, in microseconds, on each wait of the sweeps'
 *                chained triangular solves (a workgroup waiting for a block
 *                of the solution another one computes); 0 (default) =
 *                200000.  A workgroup whose wait passes the bound writes NaN
 *                into its block and finishes, so that the failure shows in
 *                the result instead of stalling the device.  Waits are never
 *                expected to come near the default; a tiny bound is for
 *                testing that path.
 */
typedef struct {
  int precision;
  int second_kind;
  int symmetric;
  int variant;
  int n_proxy;
  double proxy_radius;
  size_t max_bytes;
  int row_compression;
  int fft_matvec;
  int trace_sublevel;
  int sweep_wait_us;
} hif_opts;

#define HIF_MAX_SUBLEVELS 64

/* Statistics of a factorization (the quantities of Section 5 plus timings). */
typedef struct {
  int64_t n;
  int32_t dim;
  int32_t levels;                 /* tree depth L */
  int32_t n_sublevels;            /* 2L (2D) or 3L (3D); L for RSF */
  int64_t top_size;               /* |s_L| */
  int64_t factor_bytes;           /* m_f: bytes of stored factors */
  double t_factor_ms;             /* wall time of hif_factor */
  double t_phase_ms[8];           /* partition+near field, assembly, ID (pivoted QR),
                                     elimination, SCI update, top LU, host sync/alloc,
                                     row compression before the ID */
  int32_t sub_kind[HIF_MAX_SUBLEVELS];     /* 0 cell, 1 face, 2 edge */
  int32_t sub_groups[HIF_MAX_SUBLEVELS];   /* nonempty groups */
  int64_t sub_active[HIF_MAX_SUBLEVELS];   /* active DOFs entering the sub-level */
  int64_t sub_skel[HIF_MAX_SUBLEVELS];     /* sum of skeleton sizes */
  int64_t sub_near[HIF_MAX_SUBLEVELS];     /* sum of near-field sizes */
  int64_t sub_classes[HIF_MAX_SUBLEVELS];  /* ID problems solved (split classes) */
  double sub_id_flops[HIF_MAX_SUBLEVELS];  /* algorithmic flops of the IDs */
  double sub_elim_flops[HIF_MAX_SUBLEVELS];/* algorithmic flops of the eliminations */
  double sub_t_ms[HIF_MAX_SUBLEVELS][8];   /* per sub-level split of t_phase_ms */
  double sub_id_bytes[HIF_MAX_SUBLEVELS];  /* pivoted-QR traffic, summed over classes, m' rows
                                              (m' = min(m, n) after row compression, m on Y):
                                              blocked kernel: every step i < k reads the trailing
                                              block, 8 (m' - i)(n - i), and every full block of 32
                                              reflectors ending at step e < k reads and writes the
                                              rows below it, 16 (m' - e)(n - e); block held in
                                              registers: 8 (m' + k) n; one-workgroup streaming
                                              kernel: every step reads and writes the trailing
                                              block, 16 (m' - i)(n - i) */
  double sub_rowqr_flops[HIF_MAX_SUBLEVELS]; /* row compression: 2 m n^2 - 2 n^3 / 3 per class with m > n */
} hif_stats_t;

/* Fill *opts with the defaults listed above.  Returns HIF_EINVAL if opts is NULL. */
hif_status hif_opts_default(hif_opts* opts);

/*
 * Build F ~ A by HIF-IE (Algorithms 4.1/4.2) or RSF (Algorithm 3.1).
 *   points, n, dim: collocation points (see conventions), dim in {2, 3}.
 *   k:    kernel weights / self terms (must not be NULL).
 *   a:    [n] or NULL (a = 0, first kind);  b, c: [n] or NULL (= 1).
 *   eps:  relative ID precision, 0 < eps < 1 (Section 2.2).
 *   leaf: maximum points per leaf box (>= 1); the adaptive tree must have
 *         all its leaves at one depth, else HIF_EUNSUPPORTED.
 *   opts: NULL for defaults.
 *   out:  receives the handle (set to NULL on error).
 * Host-blocking: sizes that depend on the ranks are read back once per
 * sub-level.  Coincident points, non-finite values or points outside the
 * unit box give HIF_EINVAL; a singular B_rr or top block HIF_ESINGULAR.
 */
hif_status hif_factor(const double* points, int64_t n, int dim, const hif_kernel* k,
                      const double* a, const double* b, const double* c,
                      double eps, int32_t leaf, const hif_opts* opts,
                      hif_stream stream, hif_handle* out);

/*
 * The four factored sweeps.  x, y (f, u): [nrhs][n] device, caller's point
 * order, nrhs >= 1; in place (x == y) allowed.  Stream-ordered and
 * asynchronous; the first call of a handle may allocate sweep scratch
 * (nrhs * n doubles, kept until hif_free).  HIF_EINVAL on a NULL handle or
 * vector or nrhs < 1.
 */
/* y = F x (generalized FMM; eqn hifie2/hifie3 first line: the product of the
 * factors U_l^{-*}, D, V_l^{-1} of Lemma 2.4 / eqn rskelf). */
hif_status hif_apply(hif_handle h, const double* x, double* y, int64_t nrhs, hif_stream stream);
/* y = F^T x: the transpose of the same factored product, as the power
 * iteration of Section 5 needs A^* and F^* to estimate e_a = |A - F| / |A|. */
hif_status hif_apply_T(hif_handle h, const double* x, double* y, int64_t nrhs, hif_stream stream);
/* u = F^{-1} f (direct solver / preconditioner; eqn hifie2/hifie3 second line). */
hif_status hif_solve(hif_handle h, const double* f, double* u, int64_t nrhs, hif_stream stream);
/* u = F^{-T} f: the transposed inverse (eqn hifie2/hifie3 second line,
 * transposed), used with A^* for e_s = |I - A F^{-1}| in Section 5 and for
 * adjoint solves. */
hif_status hif_solve_T(hif_handle h, const double* f, double* u, int64_t nrhs, hif_stream stream);

/*
 * Solve sweeps recorded once as a HIP graph and replayed (for repeated
 * solves with the same factors, vectors and right-hand-side count, e.g. the
 * solves of a batch of factorizations, where the launch overhead of the
 * sweeps matters).  hif_solve_graph captures the launches hif_solve would
 * make for u = F^{-1} f (eqn hifie2/hifie3 second line) on a private stream
 * (kernel nodes only) and instantiates the graph; hif_graph_launch replays it
 * on a stream, reading f and writing u at the addresses given at capture.
 * f, u: [nrhs][n] device arrays that must stay valid while the graph is used;
 * f == u allowed.  The graph uses the handle's factors and sweep scratch:
 * free the graph before the handle, and do not overlap replays (or other
 * sweeps) of one handle on different streams.  hif_solve_graph is
 * host-blocking and allocates the sweep scratch before capturing;
 * hif_graph_launch is stream-ordered.  HIF_EINVAL on NULL arguments or
 * nrhs < 1, HIF_EDEVICE if capture or instantiation fails.
 */
typedef struct hif_graph_s* hif_graph;
hif_status hif_solve_graph(hif_handle h, const double* f, double* u, int64_t nrhs, hif_graph* out);
hif_status hif_graph_launch(hif_graph g, hif_stream stream);
/* Blocks until the replays of the graph (and the handle's other work) have
 * finished, then destroys the graph.  NULL is a no-op. */
void hif_graph_free(hif_graph g);

/*
 * u = F^{-1} f exactly as hif_solve, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the sweep scratch is a static device array of the
 * library, HIF_SOLVE_NOALLOC_MAX doubles per GPU (32 MiB, held by every GPU
 * the library runs on until the process ends), instead of the handle's
 * buffer.  The call allocates nothing and calls no allocating routine; the
 * handle must come from hif_factor (the factors hold everything else the
 * sweeps read).  Requires min(nrhs, 8) * n <= HIF_SOLVE_NOALLOC_MAX, else
 * HIF_EINVAL before any device work.  Arguments, layouts and results as
 * hif_solve.  Every call on one GPU shares that GPU's scratch: calls that
 * overlap on one GPU (different streams or host threads without ordering)
 * race and give wrong results.  The scratch needs no clearing (it is written
 * before it is read).  Stream-ordered.
 */
#define HIF_SOLVE_NOALLOC_MAX (4u << 20)
hif_status hif_solve_noalloc(hif_handle h, const double* f, double* u, int64_t nrhs, hif_stream stream);

/*
 * y = A x evaluated exactly on the fly in O(n^2) (the operator of eqn 1.1
 * under the discretization of Section 3.1; no factorization involved).
 * Arguments as in hif_factor; x, y: [nrhs][n], y must not alias x.
 * Stream-ordered.
 */
hif_status hif_matvec(const double* points, int64_t n, int dim, const hif_kernel* k,
                      const double* a, const double* b, const double* c,
                      const double* x, double* y, int64_t nrhs, hif_stream stream);

/*
 * Iterative refinement by GMRES with F^{-1} as preconditioner (Section 5,
 * Example 3: Lemma 5.1 and its corollary bound the iteration count by the
 * accuracy of F): solve A u = f with A the exact operator of this handle
 * (pair by pair as hif_matvec, from the points and coefficients given to
 * hif_factor; by FFT only with opts.fft_matvec = 1) and F^{-1} (hif_solve)
 * as right preconditioner:
 * GMRES on A F^{-1} y = f, u = F^{-1} y, starting from zero, no restart.
 *   f, u:   [nrhs][n] device, must not alias; u receives the solution.
 *   nrhs:   1..64; all right-hand sides iterate together.
 *   tol:    stop a right-hand side once its Arnoldi residual estimate is
 *           <= tol |f| (0 < tol < 1).
 *   maxit:  iteration cap, 1..200; the Krylov basis takes
 *           nrhs * (maxit + 1) * n doubles of device memory during the call.
 *   iters:  optional host [nrhs]: iterations used.
 *   relres: optional host [nrhs]: true relative residual |f - A u| / |f|
 *           recomputed with the exact operator at the end.
 * Host-blocking.  Non-convergence within maxit is not an error (check relres).
 */
hif_status hif_gmres(hif_handle h, const double* f, double* u, int64_t nrhs, double tol, int32_t maxit,
                     int32_t* iters, double* relres, hif_stream stream);

/*
 * The same refinement for the transposed system A^T u = f (the paper needs
 * A^T and F^{-T} for its error estimates, Section 5; here they solve the
 * adjoint equation of a differentiated solve): GMRES on A^T F^{-T} y = f,
 * u = F^{-T} y, with A^T applied exactly (the matvec of hif_matvec with the
 * row and column factors exchanged) and F^{-T} = hif_solve_T.
 * Arguments, limits, memory and errors as hif_gmres; relres is
 * |f - A^T u| / |f|.
 */
hif_status hif_gmres_T(hif_handle h, const double* f, double* u, int64_t nrhs, double tol, int32_t maxit,
                       int32_t* iters, double* relres, hif_stream stream);

/*
 * y = A x (transpose = 0) or y = A^T x (transpose = 1) with the exact
 * operator of this handle (eqn 1.1 under the discretization of Section 3.1,
 * from the points and coefficients given to hif_factor; the operator the
 * hif_gmres refinements use).  When the points are the cell centres of the
 * full n^d grid on the unit square/cube (any order) with constant weights and
 * self terms, and opts.fft_matvec = 1 asked for it, K is a d-level Toeplitz matrix
 * and the product runs as a zero-padded FFT convolution of size (2n)^d in
 * O(n^d log n) (the acceleration the paper uses for its products with A);
 * otherwise pair by pair as hif_matvec.  Both give the same product up to
 * rounding.
 *   x, y:     [nrhs][n] device, must not alias.  nrhs: 1..64.
 *   used_fft: optional host int, set to 1 if the FFT path ran, else 0.
 * Stream-ordered (the first call may block while it sets up the FFT).
 */
hif_status hif_apply_A(hif_handle h, const double* x, double* y, int64_t nrhs, int transpose, int32_t* used_fft,
                       hif_stream stream);

/*
 * Gradient with respect to the diagonal coefficient a of eqn 1.1 of a scalar
 * loss L(u) of the solution of the linear system of Section 3.1,
 * A u = f with A = diag(a) + diag(b) K diag(c).  (The paper does not
 * differentiate its solver; this is the adjoint of that system.)  With
 * lambda = A^{-T} dL/du (hif_solve_T, or hif_gmres_T for the refined
 * system), dL/df = lambda and
 *   grad[i] = dL/da_i = -sum_r lambda[r][i] u[r][i],
 * summed over the nrhs right-hand sides that share the operator.
 *   lambda, u: [nrhs][n] device; grad: [n] device, overwritten, must not
 *   alias lambda or u.  Stream-ordered; HIF_EINVAL on NULL or sizes < 1.
 */
hif_status hif_diag_grad(const double* lambda, const double* u, double* grad, int64_t n, int64_t nrhs,
                         hif_stream stream);

/* Copy the statistics of a factorization into *out (host memory). */
hif_status hif_stats(hif_handle h, hif_stats_t* out);

/*
 * One problem of hif_factor_batch: the arguments of hif_factor for it.
 */
typedef struct {
  const double* points;
  int64_t n;
  int dim;
  hif_kernel kernel;
  const double *a, *b, *c;
  double eps;
  int32_t leaf;
} hif_problem;

/*
 * Factor independent problems together, with the same opts.  The paper
 * factors one operator at a time; the groups of a sub-level are independent
 * (Section 2.3: the products over a level can be taken in any order), across
 * problems as within one.
 *   nworkers = 0: level-synchronous: sub-level l of every problem (level
 *             l counted from the leaves; problems with shallower trees drop
 *             out first) runs as one launch sequence over the concatenated
 *             groups of all problems, with one host read-back of the ranks
 *             per stage for the whole batch; the top blocks are LU-factored
 *             in one batched launch sequence.  Problems that share dim and
 *             the symmetric compression are factored together.  Each handle
 *             then owns its factors, as from hif_factor; its phase times
 *             (hif_stats) are those of the whole batch.
 *   nworkers = 1..16: that many host threads, each with a HIP stream of its
 *             own, run hif_factor on the problems largest first.
 *   problems: [count] host array; the arrays it points to are device arrays
 *             as for hif_factor and must stay valid until the call returns.
 *   out:      [count] host array of handles (NULL where a problem failed).
 *   status:   optional [count] host array of per-problem statuses.
 * Blocks until every factorization's device work is done; the handles then
 * serve any stream.  Returns HIF_OK, or the first failing problem's status
 * (hif_last_error names the problem); the other handles are still valid.
 * Invalid arguments of one problem fail that problem alone; in the
 * level-synchronous mode a failure of the joint factorization (a singular
 * block, the memory cap, which then applies to the whole set) is reported
 * for every problem factored with it.
 */
hif_status hif_factor_batch(const hif_problem* problems, int32_t count, const hif_opts* opts, int32_t nworkers,
                            hif_handle* out, hif_status* status);

/*
 * Launch shapes the factorization picks by problem size, per size bucket:
 *   id_reg_waves[b]: waves (of 64 lanes) per problem of the register-resident
 *     pivoted QR of the IDs, for problems of at most 64 (b = 0), 128 (b = 1)
 *     and 192 (b = 2) columns after row compression; each wave holds
 *     64 * (b + 1) / waves rows of every column.  Allowed: 4, 8 or 16 for
 *     b = 0 and 1, 8 or 16 for b = 2.
 *   lu_panel_threads[b]: threads of the register-resident LU panel (partial
 *     pivoting, Lemma 2.1) for panels of at most 512 (b = 0) and 1024 (b = 1)
 *     rows; allowed 256, 512 or 1024 for b = 0, 512 or 1024 for b = 1.
 *   rowqr_update_waves: waves (16 columns each) per workgroup of the
 *     trailing update that the row compression (Householder QR of Y before
 *     each ID) runs beside the factorization of the next panel; 4 or 8.
 *   rowqr_update_kind: 0 holds each wave's 256 rows x 16 columns of Y in
 *     registers and reads the chunk's reflectors from memory inside the
 *     products, 1 stages the reflectors in LDS first, 2 splits the rows
 *     between two waves per 16 columns (half the registers per wave, the
 *     partial products added through LDS).
 *   sweep_many_threads: threads per record of the solve's sweeps on
 *     sub-levels of at least 1024 records (the many small records of the
 *     lower levels); 64, 128 or 256.
 * The built-in table comes from paper_1307_2666_amd/tune.py, which times the
 * candidates with hif_id_batched and hif_lu_batched, the row-compression
 * shapes on whole factorizations and the sweep shapes on solves.  hif_tuning_set(NULL)
 * restores it; any other call replaces the table for the whole process (calls
 * already queued keep the shapes they were launched with).  HIF_EINVAL for an
 * entry outside the allowed values (the table is then unchanged).
 */
typedef struct {
  int32_t id_reg_waves[3];
  int32_t lu_panel_threads[2];
  int32_t rowqr_update_waves;
  int32_t rowqr_update_kind;
  int32_t sweep_many_threads;
} hif_tuning;
hif_status hif_tuning_get(hif_tuning* out);
hif_status hif_tuning_set(const hif_tuning* t);

/*
 * Batched partial LU with partial pivoting (Lemma 2.1): the kernel the
 * factorization uses on the transformed blocks [B_rr B_rs; B_sr B_ss] of
 * the skeletonized groups and on the top block, exposed on its own.  Matrix
 * p is mats + off[p], n[p] x n[p] row-major; its first r[p] columns are
 * eliminated with pivot rows chosen among rows < r[p] (the redundant block):
 * on return rows/columns < r[p] hold the unit-lower L11 and upper U11 of
 * P B_rr = L11 U11, the rows < r[p] of columns >= r[p] hold
 * U12 = L11^{-1} P B_rs, the columns < r[p] of rows >= r[p] hold
 * L21 = B_sr U11^{-1}, and the trailing block holds the Schur complement
 * B_ss - L21 U12.  piv + poff[p] receives the r[p] row interchanges
 * (row j swapped with row piv[j], in order j = 0..r-1).  off, poff (int64),
 * n, r (int32): device arrays of length batch; max_n, max_r: the largest n
 * and r.  status: device int32 that the caller clears; set to nonzero on a
 * zero pivot (HIF_ESINGULAR is not returned: the call is asynchronous).
 * Stream-ordered; allocates nothing.  HIF_EINVAL on NULL arrays, batch < 0,
 * or max_r > max_n.
 */
hif_status hif_lu_batched(double* mats, const int64_t* off, const int32_t* n, const int32_t* r, int32_t* piv,
                          const int64_t* poff, int32_t batch, int32_t max_n, int32_t max_r, int32_t* status,
                          hif_stream stream);

/*
 * What hif_factor kept of sub-level opts.trace_sublevel (sub-levels counted
 * from 0 in factor order: level 0 cells, then its faces / edges, level 1
 * cells, ...), as it stood after assembly and before the IDs:
 *   HIF_TRACE_GROUP_START  int64 [G+1]: group g's DOFs are GROUP_DOFS[start[g]..start[g+1])
 *   HIF_TRACE_GROUP_DOFS   int32: the groups' DOFs (caller's indices), each group's
 *                          columns in the order of its second-kind classes
 *   HIF_TRACE_NEAR_START   int64 [G+1], HIF_TRACE_NEAR_DOFS int32: the near field
 *                          c^N of every group (Section 4.3), ascending
 *   HIF_TRACE_Y_OFF        int64 [G], HIF_TRACE_Y double: group g's compressed block
 *                          (eqn proxy-id; Y'_c when symmetric) at Y + off[g],
 *                          row-major, rows = near field then proxy points
 *                          (non-symmetric: near-field rows, near-field
 *                          columns transposed, then the two proxy blocks),
 *                          columns = the group's DOFs in GROUP_DOFS order
 *   HIF_TRACE_ACC_OFF      int64 [G], HIF_TRACE_ACC double: A_cc (kernel and SCI
 *                          entries), row-major n_c x n_c, same order
 * dst: host buffer of cap elements of the item's type; *count (host) receives
 * the number of elements (call with cap = 0 to size the buffer).
 * HIF_EINVAL for an unknown item, a NULL count, or a handle factored without
 * a trace of an existing sub-level; HIF_ENOMEM (nothing copied) if cap is
 * too small and not 0.
 */
enum { HIF_TRACE_GROUP_START = 0, HIF_TRACE_GROUP_DOFS = 1, HIF_TRACE_NEAR_START = 2, HIF_TRACE_NEAR_DOFS = 3,
       HIF_TRACE_Y_OFF = 4, HIF_TRACE_Y = 5, HIF_TRACE_ACC_OFF = 6, HIF_TRACE_ACC = 7 };
hif_status hif_trace_get(hif_handle h, int item, void* dst, int64_t cap, int64_t* count);

/* Release a handle and all its device memory (NULL is a no-op).  Blocks the
 * host until the handle's own work has finished on every stream it was used
 * on (each call records an event on its stream), without waiting for other
 * work on the device; graphs made from the handle must be freed first. */
void hif_free(hif_handle h);

/* Message of the last error on this thread ("" if none). */
const char* hif_last_error(void);

/*
 * Batched interpolative decomposition (Lemma 2.2 with the adaptive rank rule
 * of Section 2.2): the kernel hif_factor uses for every compression, exposed
 * on its own.  For p = 0..batch-1, matrix p is Y_p = mats + off[p], row-major
 * with rows[p] rows, cols[p] columns and leading dimension cols[p].
 * Pivot i is kept iff |R_ii| > tol[p] |R_00| (column-pivoted Householder QR,
 * norms recomputed each step, ties to the lowest column index).
 * Outputs (device): rank[p]; perm + off_perm[p]: cols[p] entries, the skeleton
 * columns in pivot order followed by the redundant columns in ascending order;
 * T + off_t[p]: rank x (cols - rank) row-major interpolation matrix with
 * Y[:, redundant] ~= Y[:, skeleton] T.  mats is overwritten.  All offset and
 * size arrays are device arrays of length batch (int64 offsets, int32 sizes).
 */
hif_status hif_id_batched(double* mats, const int64_t* off, const int32_t* rows,
                          const int32_t* cols, const double* tol, int32_t batch,
                          int32_t max_cols, int32_t* rank, int32_t* perm,
                          const int64_t* off_perm, double* T, const int64_t* off_t,
                          hif_stream stream);

/*
 * Group assignment of one sub-level (Sections 3.1, 4.1, 4.2): for every
 * active point (active[i] != 0), group[i] = index of its cell (kind 0,
 * containing box, first coordinate slowest), face (kind 1, 3D) or edge
 * (kind 2) centre among the interior centres of a grid of S boxes per side,
 * enumerated family by family in the paper's order with the first index
 * slowest; nearest centre by squared distance, ties to the lowest index.
 * Inactive points get -1.  group: [n] int32 device.
 */
hif_status hif_partition(const double* points, int64_t n, int dim, const uint8_t* active,
                         int kind, int32_t S, int32_t* group, hif_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* HIF_H */
