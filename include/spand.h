/* spand.h -- C ABI of the MI355X sparsified nested dissection library (libspand.so).
 *
 * Solves A x = b for a sparse symmetric positive-definite A (Cambier et al.,
 * "An algebraic sparsified nested dissection algorithm using low-rank
 * approximations", Sec. 1, eq. (1)) with CG preconditioned by the approximate
 * factorization M of Algorithm 3 (OrthS: block Cholesky elimination, block
 * diagonal scaling, orthogonal sparsification, merge), M^T A M ~ I (Sec. 2.8).
 *
 * Conventions
 *  - Every call returns spand_status; SPAND_OK == 0.  No call aborts or prints.
 *    The text of the last error of a handle is available from spand_error_string.
 *  - The caller owns every array it passes; the library keeps no caller pointer
 *    after a call returns.  The handle owns copies of what it needs and all
 *    device memory it allocates; spand_destroy releases them.
 *  - "host" arrays are ordinary CPU memory.  "device" arrays are HIP device
 *    memory on the current device (e.g. a torch tensor's data_ptr()).
 *  - Matrices are given as the FULL symmetric CSR pattern (both triangles and
 *    the diagonal), rows 0..n-1, column indices sorted within a row.
 *  - A handle is not thread-safe; distinct handles are independent.
 *  - State machine: analyze -> factor* -> solve*.  factor may be repeated with
 *    new values (same pattern) or new tol/skip/prec; solve before any
 *    successful factor returns SPAND_E_STATE.
 */
#ifndef SPAND_H
#define SPAND_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spand_ctx* spand_t;

typedef enum {
  SPAND_OK = 0,
  SPAND_E_INVALID = 1, /* bad argument, non-symmetric pattern, non-finite value */
  SPAND_E_NOT_SPD = 2, /* a Cholesky pivot failed; site in spand_stats.fail_* */
  SPAND_E_NOCONV = 3,  /* PCG hit maxit; x, iters, relres are still written */
  SPAND_E_NOMEM = 4,   /* device or host allocation failed */
  SPAND_E_HIP = 5,     /* a HIP runtime call failed (text in spand_error_string) */
  SPAND_E_STATE = 6,   /* call out of order (e.g. solve before factor) */
  SPAND_E_BREAKDOWN = 7 /* PCG produced a non-finite residual; x, iters, relres are still written */
} spand_status;

/* Arithmetic of the dense Schur-complement products (TRSM-by-inverse and SYRK of
 * the elimination, Sec. 2.4).  Trailing storage, Cholesky pivots, CPQR, the apply
 * and PCG are FP64 in every mode. */
typedef enum { SPAND_FP64 = 0, SPAND_FP32 = 1, SPAND_BF16X3 = 2 } spand_prec;

/* Sparsification variant (Sec. 2.6, compared in Sec. 3.1 and Sec. 4.1):
 *   SPAND_ORTHS  block scaling (Sec. 2.5), then orthogonal sparsification (Sec. 2.6.1): the method
 *   SPAND_IN     interpolative sparsification (Sec. 2.6.2) without block scaling
 *   SPAND_INS    block scaling, then interpolative sparsification */
typedef enum { SPAND_ORTHS = 0, SPAND_IN = 1, SPAND_INS = 2 } spand_variant;

/* Per-run statistics (the paper's metrics of Sec. 4: t_P, t_F, t_S, n_CG,
 * size_Top, mem_F). Times in seconds measured with host clocks around the calls,
 * after device synchronisation. */
typedef struct {
  double t_analyze;      /* t_P: ordering, clustering and symbolic pattern */
  double t_factor;       /* t_F: numerical factorization (excludes analyze) */
  double t_solve;        /* t_S: total PCG time of the last solve */
  int64_t n;             /* matrix dimension */
  int32_t levels;        /* ND tree depth (root = level 1, leaves = level L) */
  int32_t n_steps;       /* = levels */
  int32_t last_iters;    /* max PCG iteration count over the RHS of the last solve */
  int32_t s_top;         /* size of the top separator right before its elimination */
  int64_t m_F;           /* stored factor entries (L_s, G_ns, L_p, Householder) */
  double schur_flops;    /* algorithmic flops of the elimination's Schur products (Sec. 2.4):
                            sum over eliminated s of |N_s||s|^2 (TRSM) + |N_s|(|N_s|+1)|s| (SYRK) */
  double schur_seconds;  /* device time of the whole elimination phase (HIP events); it also
                            holds the pivot-block Cholesky and the ordered Schur reduction */
  int32_t fail_step;     /* on SPAND_E_NOT_SPD: elimination step (1-based) */
  int32_t fail_cluster;  /* ... cluster id within that step */
  int32_t fail_phase;    /* ... 0 = elimination, 1 = scaling, 2 = interpolative sparsification
                            (the Cholesky of C_ff, Sec. 2.6.2) */
  int32_t cpqr_one_launch_steps; /* steps of the last factor whose CPQRs (Sec. 2.6.1) ran in
                                    one launch, each interface waiting for its neighbours of
                                    earlier colour classes only */
  /* Per-step profile of the last factor (the paper's time/memory per level,
   * Sec. 4.4): device seconds (HIP events) of each phase of step t (t = 1..32):
   * [t-1][0] assembly/merge, [1] elimination, [2] scaling, [3] sparsification;
   * and the cumulative stored factor entries after step t. */
  double step_phase_seconds[32][4];
  int64_t step_m_F[32];
  /* The truncated CPQRs of the last factor (Sec. 2.6.1).  For an interface with an
   * m x n block A_pn and k Householder steps the algorithmic work is
   *   sum_{j<k} [2(m-j)(n-j) + 4(m-j)(n-j-1) + 3(m-j)]  (column norms, reflector, update)
   *   + 2(m-k)(n-k) when it stops before min(m, n)      (the norms that end it). */
  double cpqr_flops;
  double cpqr_seconds;    /* summed device time of the CPQR launches (HIP events) */
  int64_t cpqr_launches;
  /* The preconditioner applies of the last solve (Sec. 2.8).  Algorithmic HBM bytes
   * of one apply on nrhs columns: every stored factor entry read twice (forward and
   * backward sweep, 8 B each) plus the n x nrhs vector read and written per sweep. */
  double apply_bytes;
  double apply_seconds;   /* summed device time of the applies (HIP events) */
  int64_t apply_calls;
  int32_t apply_graph;    /* 1 if the last solve replayed its apply from a captured graph */
  int32_t cpqr_lds_slot_interfaces; /* interfaces of the last factor whose CPQR teams kept a
                                       column in LDS beside their register columns */
  /* Interfaces of the last factor by the register layout of their CPQR: one workgroup
   * (32 rows x 2 columns per lane), one workgroup of the wide layout (teams of 2
   * lanes, 28 rows x 3 columns), several workgroups with 32 x 2, several with 20 x 3. */
  int64_t cpqr_interfaces[4];
  /* Interfaces of the last factor by the kernels of their apply (Sec. 2.8 scaling and
   * Householder products): the fused one-wave kernel for at most 64 dofs, the fused
   * kernel for 65..fuse_max dofs (see spand_tuning), the tiled kernels otherwise. */
  int64_t apply_interfaces[3];
  /* Residual replacements in the last solve: columns whose recursive residual met
   * rtol while the true residual did not, and which went on from the true one. */
  int64_t pcg_replacements;
  /* Interfaces of the last factor whose CPQR ran in the global-memory kernel for
   * interfaces beyond the register layouts (more than 2048 rows, more columns than
   * the co-resident slabs hold, or at least tuning.cpqr_big_min rows). */
  int64_t cpqr_big_interfaces;
  /* Doubles of apply scratch per right-hand side that the last factorization needs
   * (spand_apply_noalloc holds 8 Mi doubles in all). */
  int64_t apply_scratch_per_rhs;
} spand_stats;

/* Kernel-shape and path parameters of a handle.  None of them changes what is
 * computed; they change how the work is cut into launches (and, for chol_group,
 * the order of the roundings inside the blocked Cholesky updates).
 *   chol_group    64-wide block columns per trailing-update group of the blocked
 *                 Cholesky and of the left scaling (1..4; default 3)
 *   fuse128_min   the apply's fused one-wave kernel also takes interfaces of 65..128
 *                 dofs when a step has at least this many of them (default 256;
 *                 0 = always, -1 = never)
 *   gemm_syrk     output tile of the batched matrix-core GEMM of the Schur SYRK
 *   gemm_chol     ... of the trailing updates of the blocked Cholesky (pivot blocks and
 *                 the rows below them)
 *   gemm_scale    ... of the left scaling and the compact-WY T factors
 *                 (0: 64 x 64, 1: 128 x 128, 2: 32 x 32 output tiles; every tile adds the
 *                 products of an entry in one order, so results agree bit for bit; the
 *                 BF16x3 products always use 64 x 64)
 *   cpqr_big_min  interfaces of at least this many dofs take the global-memory CPQR
 *                 kernel, which is otherwise kept for interfaces beyond the register
 *                 layouts (0 = only those; default 0)
 */
typedef struct {
  int32_t chol_group;
  int32_t fuse128_min;
  int32_t gemm_syrk;
  int32_t cpqr_big_min;
  int32_t gemm_chol;
  int32_t gemm_scale;
  int32_t reserved[2];
} spand_tuning;

/* Ordering, clustering and symbolic factorization (Algorithm 2, Sec. 2.3, with a
 * geometric vertex separator, or a graph one when no coordinates are given;
 * cluster hierarchy, Sec. 2.7; fill pattern, Sec. 2.4).
 *   n        matrix dimension (>= 1)
 *   rowptr   host, n+1 entries, rowptr[0] = 0
 *   colind   host, rowptr[n] entries, sorted per row, pattern symmetric, diagonal present
 *   dim      2 or 3: coords host, n*dim doubles, row-major (x, y[, z]) per vertex, and
 *            the separator cuts the widest coordinate axis at its lower median;
 *            0: coords must be NULL, and the separator is a breadth-first level
 *            structure of the graph from a pseudo-peripheral root (George-Liu), cut at
 *            the lower median level
 *   levels   ND tree depth L >= 1 (2^(L-1) leaves)
 *   out      receives the new handle (NULL on failure)
 * Host-only: touches no GPU.  Errors: SPAND_E_INVALID, SPAND_E_NOMEM. */
spand_status spand_analyze(int64_t n, const int64_t* rowptr, const int32_t* colind,
                           int32_t dim, const double* coords, int32_t levels, spand_t* out);

/* Numerical factorization, Algorithm 3 (OrthS), on the GPU.
 *   values   device, rowptr[n] doubles in the CSR order given to analyze
 *   tol      sparsification tolerance eps >= 0: keep the leading CPQR steps with
 *            |R_jj| >= eps |R_00| (Sec. 4 intro); eps = 0 keeps full rank
 *   skip     number of initial elimination steps without scaling/sparsification
 *            (skip >= levels gives the exact ND Cholesky, "Direct" in Sec. 4)
 *   prec     arithmetic of the Schur products (spand_prec)
 * Synchronises the handle's stream.  Errors: SPAND_E_INVALID (negative tol,
 * non-finite values), SPAND_E_NOT_SPD (site in stats), SPAND_E_NOMEM, SPAND_E_HIP. */
spand_status spand_factor(spand_t h, const double* values, double tol, int32_t skip, spand_prec prec);

/* PCG with the preconditioner M M^T, x0 = 0, FP64 (Sec. 4: stop at ||Ax-b||/||b|| <= rtol).
 * A column stops when its true residual meets rtol; the recursive residual is the
 * cheap test that triggers forming the true one (residual replacement otherwise).
 *   nrhs     number of right-hand sides (>= 1)
 *   b        device, n x nrhs column-major
 *   x        device, n x nrhs column-major, output
 *   rtol     relative residual target on the recursive residual (e.g. 1e-12)
 *   maxit    iteration cap (>= 1)
 *   iters    host, nrhs ints: iterations taken per RHS (0 for b = 0)
 *   relres   host, nrhs doubles: true relative residual ||b - A x|| / ||b|| at exit
 * Errors: SPAND_E_STATE (no factor), SPAND_E_INVALID (non-finite b),
 * SPAND_E_BREAKDOWN (a residual norm became NaN or Inf, e.g. from a corrupted factor;
 * that column stops, outputs still written), SPAND_E_NOCONV (some RHS hit maxit;
 * outputs still written), SPAND_E_HIP. */
spand_status spand_solve(spand_t h, int32_t nrhs, const double* b, double* x, double rtol,
                         int32_t maxit, int32_t* iters, double* relres);

/* Preconditioner apply z = M M^T r (Sec. 2.8) for nrhs columns; r, z device n x nrhs
 * column-major (may not alias).  Errors: SPAND_E_STATE, SPAND_E_HIP. */
spand_status spand_apply(spand_t h, int32_t nrhs, const double* r, double* z);

/* spand_apply for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same apply
 * z = M M^T r, with the apply's scratch in a fixed 64 MiB array of the library (8 Mi
 * doubles per GPU, held until the process ends) instead of the handle's workspace.
 * It calls no allocator and does not synchronize: the kernels are enqueued on the
 * handle's stream and z is ready when that stream reaches them.  All calls on one
 * GPU share the array, so calls that overlap on one GPU (other streams, other
 * handles, other threads) race; the array is fully written before it is read, so
 * nothing carries over from one call to the next.  It needs
 * spand_stats.apply_scratch_per_rhs * nrhs doubles of scratch (a property of the
 * factorization); a call needing more than the array holds returns
 * SPAND_E_INVALID, with the size needed in spand_error_string, and runs nothing.  Other errors:
 * SPAND_E_STATE, SPAND_E_HIP. */
spand_status spand_apply_noalloc(spand_t h, int32_t nrhs, const double* r, double* z);

/* Use this HIP stream (hipStream_t passed as void*) for all later device work of
 * the handle; NULL selects the default stream. */
spand_status spand_set_stream(spand_t h, void* hip_stream);

/* Inside spand_solve the preconditioner apply of every PCG iteration works on the
 * same vectors, so by default it is captured once per solve into a HIP graph (on a
 * private stream) and replayed on the handle's stream.  enable = 0 launches it
 * kernel by kernel instead; results are identical.  If the runtime refuses the
 * capture, spand_solve falls back to kernel-by-kernel launches. */
spand_status spand_set_apply_graph(spand_t h, int32_t enable);

/* Set or read the tuning parameters of h (spand_tuning).  The set applies from the
 * next factor on.  Errors: SPAND_E_INVALID for a value out of range. */
spand_status spand_set_tuning(spand_t h, const spand_tuning* t);
spand_status spand_get_tuning(spand_t h, spand_tuning* t);

/* Select the sparsification variant (spand_variant) of the later factors of h; the
 * default is SPAND_ORTHS.  For SPAND_IN and SPAND_INS each interface p is split by the
 * truncated CPQR of A_np (pivoting over the dofs of p, the rule of spand_factor's tol)
 * into coarse dofs c (the pivots) and fine dofs f; T_cf = R_11^{-1} R_12 interpolates
 * A_nf ~ A_nc T_cf; the congruence with T_p = [I 0; -T_cf I] forms C_ff and C_cf, the
 * f-n coupling is dropped and f is eliminated against c (Sec. 2.6.2).  The
 * factorization may then lose positive definiteness: SPAND_E_NOT_SPD, with fail_phase
 * 2 when the Cholesky of C_ff fails.  Limits of these variants: interfaces of at most
 * 4096 dofs and A_np of at most 7680 rows (SPAND_E_INVALID beyond); the batched
 * calls accept SPAND_ORTHS handles only.  Errors: SPAND_E_INVALID for an unknown
 * variant. */
spand_status spand_set_variant(spand_t h, spand_variant v);
spand_status spand_get_variant(spand_t h, spand_variant* v);

/* Autotuner of the kernel shapes (spand_tuning) for this matrix and these settings.
 * Coordinate descent over the parameters in turn (the GEMM tile of the Cholesky
 * updates, the Cholesky grouping, the SYRK tile, the scaling tile, the apply's fusion
 * threshold), each candidate timed on this handle's own factorization (the device
 * time of the factor phases the parameter acts on, best of reps runs) or, for the
 * fusion threshold, on its apply with nrhs columns; a candidate replaces the current
 * choice only if it is at least 2% faster.  The handle ends factored (values, tol,
 * skip, prec as in spand_factor) with the chosen tuning, which *out receives (may be
 * NULL).  When the environment variable SPAND_TUNE_CACHE names a file, a choice
 * stored there for the same matrix size, pattern size, levels, tol, skip, prec, nrhs
 * and GPU architecture is taken without measuring, and a new choice is appended.
 * The search factors the matrix about 16 x reps times.  Errors as spand_factor and
 * spand_apply; SPAND_E_NOMEM if the timing vectors (2 n nrhs doubles) cannot be
 * allocated. */
spand_status spand_autotune(spand_t h, const double* values, double tol, int32_t skip, spand_prec prec, int32_t nrhs,
                            int32_t reps, spand_tuning* out);

/* Copy the statistics of the last analyze/factor/solve into *s. */
spand_status spand_get_stats(spand_t h, spand_stats* s);

/* Per-vertex separator ids of Algorithm 2: S, L, R as level * 2^32 + index
 * ("none" = 0); host arrays of n entries each. */
spand_status spand_get_ordering(spand_t h, int64_t* S, int64_t* L, int64_t* R);

/* The nested-dissection elimination order of the vertices (Algorithm 2's output
 * order): perm[k] = the k-th vertex eliminated, sorted by the step of its separator
 * (leaves first), then by the cluster of that step it belongs to (canonical cluster
 * order), then by vertex id.  host array of n entries. */
spand_status spand_get_permutation(spand_t h, int64_t* perm);

/* Symbolic structure of elimination step `step` (1-based; level = levels - step + 1).
 * counts (host, 6 entries) receives: number of clusters nc, number eliminated ne,
 * number of blocks before elimination nb, number of blocks among remaining clusters
 * after fill na, ND level, total neighbour entries of the eliminated clusters. */
spand_status spand_step_counts(spand_t h, int32_t step, int64_t* counts);

/* Arrays of step `step`, sized by spand_step_counts (any pointer may be NULL):
 *   keys    nc*3 int64: S, L, R of each cluster in cluster order (pointers truncated)
 *   parent  nc int32: cluster id at the next step (-1 if eliminated or last step)
 *   colour  nc int32: sparsification colour (-1 for eliminated clusters)
 *   before  nb*2 int32: block pairs (i, j), i >= j, sorted, before elimination
 *   after   na*2 int32: block pairs among remaining clusters after fill */
spand_status spand_step_structure(spand_t h, int32_t step, int64_t* keys, int32_t* parent,
                                  int32_t* colour, int32_t* before, int32_t* after);

/* After a factor: sizes (nc int32) of every cluster of step `step` before its
 * elimination and ranks (nc int32) kept after sparsification (= size when not
 * sparsified, -1 for eliminated clusters). */
spand_status spand_step_ranks(spand_t h, int32_t step, int32_t* sizes, int32_t* ranks);

/* Batched factorization of P independent problems (the 256-problem workload: many
 * small grids factored together).  hs: P distinct handles from spand_analyze (host
 * array); values: host array of P device pointers, values[q] as in spand_factor for
 * hs[q]; tol, skip, prec as in spand_factor, shared by all problems.
 * The problems are factored in lockstep: step t of every problem runs in the same
 * launches (one set of elimination, scaling, sparsification and merge kernels per
 * step for the whole batch, with the descriptors of all problems concatenated), on
 * one stream: that of hs[0], or a stream created for the call when hs[0] has none.
 * The tuning of hs[0] applies to all.  Each problem's result is the one spand_factor
 * gives it alone (no problem's arithmetic depends on another's).  Every handle ends
 * in the state spand_factor would leave it in: a problem that fails (not SPD,
 * non-finite values) is dropped from the run and the others go on.  The device
 * times in each handle's stats are those of the shared launches.
 * Returns SPAND_OK, or the status of the first failing problem in handle order, with
 * spand_error_string(NULL) naming it and spand_error_string(hs[q]) holding its error.
 * SPAND_E_INVALID if P < 1, a handle is NULL or repeated. */
spand_status spand_factor_batch(int32_t P, spand_t* hs, const double* const* values, double tol, int32_t skip,
                                spand_prec prec);

/* Batched PCG: problem q solves nrhs right-hand sides b[q] -> x[q] (device, n_q x nrhs
 * column-major) with hs[q] as in spand_solve.  iters and relres are host arrays of
 * P * nrhs entries, problem q at offset q * nrhs.  The problems iterate in lockstep on
 * the stream of hs[0] (or one created for the call): each half of an iteration of
 * every problem (SpMV, dot products and updates; the preconditioner applies) is one
 * captured HIP graph, replayed every iteration, and one copy per iteration brings
 * every residual norm to the host.  Each problem's iterates are those spand_solve
 * gives it alone.  Errors as spand_factor_batch; a problem that hits maxit returns
 * SPAND_E_NOCONV with its outputs written, one that breaks down SPAND_E_BREAKDOWN. */
spand_status spand_solve_batch(int32_t P, spand_t* hs, int32_t nrhs, const double* const* b, double* const* x,
                               double rtol, int32_t maxit, int32_t* iters, double* relres);

/* Text of the last error on h (or, when h is NULL, of the last failed analyze or
 * batched call on this thread).
 * Valid until the next call on h. */
const char* spand_error_string(spand_t h);

/* Release the handle and all its memory.  NULL-safe. */
void spand_destroy(spand_t h);

#ifdef __cplusplus
}
#endif

#endif /* SPAND_H */
