/*
 * hodlr.h - C ABI of the MI355X (gfx950) HODLR QR library.
 *
 * The library computes the QR decomposition A ~= Q R of a square HODLR matrix
 * A with Q = I - Y T Y^T (compact WY representation, Schreiber & Van Loan),
 * following Algorithm hQR of Kressner & Susnjara, "Fast QR decomposition of
 * HODLR matrices" (Sec. 4).  Y (unit lower triangular), T and R (upper
 * triangular) are HODLR matrices of the same level and partition as A.
 *
 * Conventions shared by every entry point
 *  - All arithmetic is IEEE binary64.
 *  - Matrices are column-major.  A HODLR matrix of level l on the partition
 *    n = n_1 + ... + n_{2^l} (Sec. 2.1, eq. integerpart) has 2^l dense leaves
 *    and, for every internal node v of its binary tree (heap numbering: root 1,
 *    children 2v and 2v+1), an upper block A(I_left, I_right) = U V^T and a
 *    lower block A(I_right, I_left) = U V^T (eq. factoroffdiagonal with
 *    V = A_R^T).  Blocks are listed in level order (depth 0 .. l-1, nodes left
 *    to right), the upper block of a node before its lower block.
 *  - "device" pointers are HIP device memory on the current device, "host"
 *    pointers are ordinary host memory.  The caller owns every array it passes;
 *    the library owns the handles and all device memory behind them.  Device
 *    memory comes from the allocator installed with hodlr_set_allocator, else
 *    from hipMalloc (memory held by a handle) and hipMallocAsync (temporaries
 *    of one call).
 *  - Every call returns a hodlr_status.  Argument errors are detected on the
 *    host before any work is queued; hodlr_last_error() then describes the
 *    failure (thread-local string).  No call aborts or throws.
 *  - Work is queued on the given stream (0 = the null stream).  hodlr_build
 *    and hodlr_qr synchronise that stream before returning (they read back a
 *    few scalars).  hodlr_apply_q, hodlr_solve, hodlr_matmul and
 *    hodlr_qr_matmul are stream-ordered and asynchronous: they replay launch
 *    sequences the handle cached when it was made (a product's on its first
 *    call), take their temporaries from the allocator on the call's stream,
 *    and return without waiting for the device.
 *  - Threads: a finished hodlr_t or hodlr_qr_t is not modified by the calls
 *    that read it, so apply_q, solve and the products may run on one handle
 *    from several threads and streams at once (each call has its own
 *    temporaries).  A handle must outlive the work queued with it: release it
 *    only after that work is done.  hodlr_qr_time / hodlr_qr_profile and the
 *    batched calls create private handles.  hodlr_qr_refactor rewrites the
 *    factorisations it is given: no other call may use them meanwhile.
 */
#ifndef HODLR_H
#define HODLR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hodlr_s hodlr_t;       /* device-resident HODLR matrix            */
typedef struct hodlr_qr_s hodlr_qr_t; /* device-resident factors {Y, T, R}       */
typedef void *hodlr_stream_t;         /* a hipStream_t                           */

typedef enum {
  HODLR_OK = 0,
  HODLR_EINVAL = -1,     /* invalid argument (sizes, partition, ranks, NULL)      */
  HODLR_ENOMEM = -2,     /* device allocation failed                              */
  HODLR_ENONFINITE = -3, /* NaN or Inf in the input                               */
  HODLR_ECAPACITY = -4,  /* an off-diagonal rank outgrew the capacity; retry with
                            a larger rank_cap or a looser eps                      */
  HODLR_EDEVICE = -5,    /* a HIP call failed; hodlr_last_error() has its text     */
  HODLR_ENOTBUILT = -6   /* the library was loaded without device code            */
} hodlr_status;

/*
 * hodlr_set_allocator - route the library's device memory through the caller's
 * allocator (for example a framework's caching allocator).  alloc(bytes,
 * stream, ctx) returns device memory usable in stream order on `stream` (NULL
 * on failure, reported as HODLR_ENOMEM); release(ptr, stream, ctx) gives it
 * back, called once the work using it has been queued on `stream`.  Both NULL:
 * back to hipMalloc / hipMallocAsync.  Handles keep the allocator they were
 * made with; calls made later use the one installed at the time of the call.
 * Returns HODLR_EINVAL if exactly one of alloc, release is NULL.
 */
hodlr_status hodlr_set_allocator(void *(*alloc)(size_t bytes, void *stream, void *ctx),
                                 void (*release)(void *ptr, void *stream, void *ctx), void *ctx);

/* hodlr_qr / hodlr_qr_time flags.  By default the launches are issued directly,
 * with the T-factor steps of every node (T~12 and T12, Alg. hQR) on a second
 * stream beside the main chain, joined back into the caller's stream. */
#define HODLR_QR_GRAPH 1u       /* capture the launch sequence once per call (per
                                   handle for hodlr_qr_time) in its serial order
                                   on one stream and replay it as a HIP graph     */
#define HODLR_QR_ONE_STREAM 2u  /* direct launches, all on the caller's stream in
                                   the serial order                                */
#define HODLR_QR_BY_SHAPE 4u    /* hodlr_qr_batched: run the groups of equal shape one
                                   after another instead of one merged sequence    */
#define HODLR_QR_KEEP 8u        /* keep the schedule (launch lists, workspace and, with
                                   HODLR_QR_GRAPH, the graph) for hodlr_qr_refactor */

/*
 * hodlr_build - copy a HODLR matrix to the device.
 *
 *  n, levels      order and level l >= 0 of the matrix.
 *  leaf_off       host, 2^l + 1 prefix offsets of the partition (leaf_off[0] = 0,
 *                 leaf_off[2^l] = n, strictly increasing).
 *  leaves         host, the dense leaves one after another, leaf j column-major
 *                 n_j x n_j starting at leaves + leaf_data_off[j].
 *  leaf_data_off  host, 2^l offsets (in doubles) into `leaves`.
 *  U, u_off       host, block b's left factor (rows_b x rank_b, column-major) at
 *                 U + u_off[b]; blocks in the order stated above (2^(l+1) - 2 of
 *                 them).
 *  V, v_off       host, block b's right factor (cols_b x rank_b) at V + v_off[b].
 *  ranks          host, rank_b of every block, 0 <= rank_b <= min(rows_b, cols_b,
 *                 rank_cap).
 *  rank_cap       capacity (columns) reserved for every off-diagonal factor of A
 *                 and of the factors Y, T, R computed from it; 1..64.
 *  out            receives the new handle (release with hodlr_free).
 * Returns HODLR_EINVAL for an inconsistent partition or rank, HODLR_ENONFINITE
 * if any input entry is NaN/Inf, HODLR_ENOMEM if the device is full.
 */
hodlr_status hodlr_build(int64_t n, int32_t levels, const int64_t *leaf_off,
                         const double *leaves, const int64_t *leaf_data_off,
                         const double *U, const int64_t *u_off,
                         const double *V, const int64_t *v_off,
                         const int32_t *ranks, int32_t rank_cap,
                         hodlr_stream_t stream, hodlr_t **out);

/*
 * hodlr_build_rect - copy an m x n rectangular HODLR matrix (Sec. 6) to the
 * device: leaf j is m_j x n_j with m_j >= n_j, on the row partition row_off
 * (host, 2^l + 1 offsets from 0 to m) and the column partition col_off (from 0
 * to n); leaf j column-major with leading dimension m_j; block b's left factor
 * has rows_b rows of the row partition, its right factor cols_b rows of the
 * column partition; otherwise as hodlr_build.  Products (hodlr_matmul: X has
 * n rows and Z m rows, or m and n with trans) and the norm estimate accept it.
 */
hodlr_status hodlr_build_rect(int64_t m, int64_t n, int32_t levels, const int64_t *row_off,
                              const int64_t *col_off, const double *leaves, const int64_t *leaf_data_off,
                              const double *U, const int64_t *u_off, const double *V, const int64_t *v_off,
                              const int32_t *ranks, int32_t rank_cap, hodlr_stream_t stream, hodlr_t **out);

/*
 * hodlr_qr - hQR factorisation A ~= (I - Y T Y^T) R  (Algorithm hQR, Sec. 4).
 *
 *  eps    truncation tolerance >= 0.  Recompressions of A-valued blocks (the
 *         sum S~, the new upper block of R, the low-rank update of the trailing
 *         HODLR part) keep singular values > eps*anorm; the off-diagonal blocks
 *         of T keep singular values > eps (as written in the algorithm).
 *  anorm  |A|_2 used for the threshold; if anorm <= 0 it is estimated on the
 *         device, as the first step of the factorisation's launch sequence, by
 *         50 steps of power iteration on A^T A (see hodlr_norm2_est).
 *  flags  0, HODLR_QR_GRAPH or HODLR_QR_ONE_STREAM; every choice gives
 *         bitwise identical factors.
 *  out    receives the factors (release with hodlr_qr_free).  A is not modified.
 * Returns HODLR_ECAPACITY if a rank outgrew rank_cap (or a recompression width
 * exceeded 128); the partial factors are then released.
 *
 * A rectangular A (hodlr_build_rect, Sec. 6) gets the permuted QR of that
 * section: block column j is reduced onto the first n_j rows of leaf j (its
 * pivot rows) and every other row of it becomes zero.  Y (m x n) then has
 * upper blocks as well, over the rows of a node's first child left unreduced
 * by it ("free rows", compressed at eps*anorm); T is n x n on the column
 * partition; R is zero outside the pivot rows, and hodlr_qr_factor(F, 'R') /
 * hodlr_qr_matmul(F, 'R', ...) act with R on its pivot rows in column order (an
 * n x n upper triangular HODLR matrix).  Q is m x m: hodlr_apply_q takes m-row
 * operands.
 */
hodlr_status hodlr_qr(const hodlr_t *A, double eps, double anorm, uint32_t flags,
                      hodlr_stream_t stream, hodlr_qr_t **out);

/*
 * hodlr_qr_batched - hodlr_qr of `count` independent matrices A[0..count-1] at
 * once (Algorithm hQR for each).  Matrices with the same partition and
 * rank_cap share one schedule: every launch of it carries the jobs of all of
 * them, so they advance through the recursion in lockstep.  When the matrices
 * have several shapes (and one rank_cap) the schedules of the shapes are merged
 * into one launch sequence: at each step the schedule with the most launches
 * left picks the kernel, and every schedule whose next launch runs the same
 * kernel variant joins that launch (flag HODLR_QR_BY_SHAPE: the shapes one after
 * another instead).  Each factorisation computes exactly what hodlr_qr
 * computes for that matrix alone (bitwise: no kernel mixes jobs).
 *  anorm  host array of count values (<= 0: estimate) or NULL (estimate all).
 *  out    host array of count handles, released with hodlr_qr_free one by one.
 * On error no handle is returned; the message names the first failing matrix.
 */
hodlr_status hodlr_qr_batched(const hodlr_t *const *A, int32_t count, double eps,
                              const double *anorm, uint32_t flags, hodlr_stream_t stream,
                              hodlr_qr_t **out);

/*
 * hodlr_qr_batched_time - as hodlr_qr_time for hodlr_qr_batched: per-run
 * durations (ms, host array of reps) of factorising the whole batch.
 */
hodlr_status hodlr_qr_batched_time(const hodlr_t *const *A, int32_t count, double eps,
                                   const double *anorm, uint32_t flags, int32_t warmup,
                                   int32_t reps, hodlr_stream_t stream, double *ms);

/*
 * hodlr_qr_refactor - factorise new matrices into factorisations made with
 * HODLR_QR_KEEP, replaying their kept schedules (no planning, no allocation of
 * schedule memory; with HODLR_QR_GRAPH the captured graph is launched again).
 * A[i] must have F[i]'s partition and rank_cap; the thresholds are those of the
 * first factorisation (its given |A|_2, or a new estimate of |A[i]|_2 when it
 * estimated).  The factorisations of one hodlr_qr_batched call share one
 * schedule and must all be passed together.  F[i]'s apply-Q / solve / product
 * calls see the new factors.  Blocks the host until the device has finished
 * (it reads the error flags); HODLR_ECAPACITY as hodlr_qr.
 */
hodlr_status hodlr_qr_refactor(hodlr_qr_t *const *F, const hodlr_t *const *A, int32_t count, uint32_t flags,
                               hodlr_stream_t stream);

/*
 * hodlr_apply_q - X <- Q X (trans = 0) or X <- Q^T X (trans = 1), with
 * Q = I - Y T Y^T (eq. compactwy): W = Y^T X, W <- op(T) W, X <- X - Y W, in
 * blocks of at most 64 columns.  X: device, n x nrhs, leading dimension
 * ldx >= n (< 2^31).  Stream-ordered and asynchronous; temporaries 2 n
 * min(nrhs, 64) doubles plus the products' projections, from the allocator.
 */
hodlr_status hodlr_apply_q(const hodlr_qr_t *F, int32_t trans, int64_t nrhs, double *X,
                           int64_t ldx, hodlr_stream_t stream);

/*
 * hodlr_apply_q_noalloc - hodlr_apply_q for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same launch sequence and kernels, with its temporaries in a
 * static device array of 32 MiB that the library holds on every device it runs
 * on until the process ends.  It calls no hipMalloc, hipFree or allocating
 * routine.  The array holds the product projections of the factor (2 x the
 * tree's nodes x rank_cap x 64 doubles) plus two n x s blocks; s, the columns
 * processed per pass, is chosen as large as fits (at most 64).  A factor whose
 * projections and two n-row columns do not fit is refused with HODLR_EINVAL
 * (n = 65536 with rank_cap 16 fits with s = 16).  All calls on one device share
 * the array: calls that overlap on one device (other streams, other threads)
 * race and must be serialised by the caller; a call leaves the array's
 * contents behind and the next call overwrites them.
 */
hodlr_status hodlr_apply_q_noalloc(const hodlr_qr_t *F, int32_t trans, int64_t nrhs, double *X,
                                   int64_t ldx, hodlr_stream_t stream);

/*
 * hodlr_solve - B <- R^{-1} Q^T B, i.e. the solution of A x = b for every
 * column of B (device, n x nrhs, ldb >= n).  Back substitution with the upper
 * triangular HODLR R runs leaf by leaf from the last one
 * (x2 = R22^{-1} c2, c1 <- c1 - R12 x2, x1 = R11^{-1} c1).  Stream-ordered and
 * asynchronous.  A rectangular factorisation is refused (HODLR_EINVAL): use
 * hodlr_lstsq.
 */
hodlr_status hodlr_solve(const hodlr_qr_t *F, int64_t nrhs, double *B, int64_t ldb,
                         hodlr_stream_t stream);

/*
 * hodlr_lstsq - least-squares solutions x = argmin |A x - b|_2 of every column
 * of B from the (permuted) QR: B <- Q^T B (device, m x nrhs, ldb >= m), then X
 * (device, n x nrhs, ldx >= n) <- R_p^{-1} (the pivot rows of Q^T B in column
 * order), with R_p the n x n triangular factor on the pivot rows.  For a square
 * factorisation it is hodlr_solve with the result in X.  Stream-ordered and
 * asynchronous.
 */
hodlr_status hodlr_lstsq(const hodlr_qr_t *F, int64_t nrhs, double *B, int64_t ldb, double *X, int64_t ldx,
                         hodlr_stream_t stream);

/*
 * hodlr_matmul - Z <- op(A) X for the HODLR matrix A (HODLR matrix times a
 * dense block, Table 1's matrix-vector product applied to nrhs columns).
 * trans = 0: op(A) = A, 1: A^T.  X, Z: device, n x nrhs, distinct.  A may be
 * a factor view from hodlr_qr_factor.  Stream-ordered and asynchronous (the
 * first call per (A, trans) builds and uploads its launch sequence).
 */
hodlr_status hodlr_matmul(const hodlr_t *A, int32_t trans, int64_t nrhs, const double *X,
                          int64_t ldx, double *Z, int64_t ldz, hodlr_stream_t stream);

/*
 * hodlr_qr_matmul - Z <- op(M) X for one factor M of F: which = 'Y' (unit lower),
 * 'T' (upper) or 'R' (upper).  Same operand rules as hodlr_matmul.
 */
hodlr_status hodlr_qr_matmul(const hodlr_qr_t *F, char which, int32_t trans, int64_t nrhs,
                             const double *X, int64_t ldx, double *Z, int64_t ldz,
                             hodlr_stream_t stream);

/*
 * hodlr_norm2_est - |A|_2 estimate: x0 = (1,...,1)/sqrt(n), 'iters' steps of
 * x <- A^T A x / |A^T A x|, result |A x|.  Synchronises the stream; *out host.
 */
hodlr_status hodlr_norm2_est(const hodlr_t *A, int32_t iters, hodlr_stream_t stream,
                             double *out);

/* Factor summary (host struct filled by hodlr_qr_info). */
typedef struct {
  int64_t n;
  int32_t levels;
  int32_t rank_cap;
  int32_t max_rank_y, max_rank_t, max_rank_r; /* largest off-diagonal ranks          */
  double anorm, tau_a, tau_t;                 /* thresholds actually used             */
  double flops;        /* algorithmic FP64 flops of the factorisation (counted on the
                          device from the realised sizes and ranks, Table 1 and the
                          cost terms of Sec. 4.1), the |A|_2 estimate excluded       */
  int64_t n_truncations; /* recompressions performed                                 */
  int64_t n_launches;    /* kernel launches in one factorisation                     */
  int64_t device_bytes;  /* device memory held by the factors                        */
  double norm_flops;     /* flops of the |A|_2 estimate (0 when anorm was given); not
                            part of `flops`                                           */
} hodlr_qr_info_t;

hodlr_status hodlr_qr_info(const hodlr_qr_t *F, hodlr_qr_info_t *info);

/*
 * hodlr_export / hodlr_qr_export - copy a matrix (or one factor of F:
 * which = 'Y', 'T', 'R') back to host memory in the hodlr_build layout.
 * leaves: sum n_j^2 doubles.  U, V: room for (2^(l+1) - 2) blocks of
 * rank_cap columns each, packed as rows_b*rank_b (U) and cols_b*rank_b (V)
 * at the offsets written to u_off / v_off; ranks: 2^(l+1) - 2 ints.
 * For Y the stored leaf is the unit lower triangle (ones on the diagonal), for
 * T and R the upper triangle; blocks that are zero by structure get rank 0.
 * Synchronous.
 */
hodlr_status hodlr_export(const hodlr_t *A, double *leaves, double *U, int64_t *u_off,
                          double *V, int64_t *v_off, int32_t *ranks);
hodlr_status hodlr_qr_export(const hodlr_qr_t *F, char which, double *leaves, double *U,
                             int64_t *u_off, double *V, int64_t *v_off, int32_t *ranks);

/*
 * hodlr_qr_time - run the factorisation of A `reps` times on `stream` after
 * `warmup` untimed runs, bracketing each run with HIP events on that stream,
 * and return the per-run durations in ms (host array of reps doubles).  The
 * factors of the last run are discarded.
 */
hodlr_status hodlr_qr_time(const hodlr_t *A, double eps, double anorm, uint32_t flags,
                           int32_t warmup, int32_t reps, hodlr_stream_t stream, double *ms);

/*
 * hodlr_qr_profile - diagnostic: run one factorisation launch by launch on
 * `stream`, each launch issued through hipExtLaunchKernel with a pair of HIP
 * events that the dispatch itself stamps at its start and end (so a duration
 * excludes launch gaps and matches a kernel trace), and accumulate per
 * kernel type (index = type, names from hodlr_op_name, hodlr_op_count types):
 * ms[type] total duration, counts[type] launches, flops[type] algorithmic FP64
 * flops credited to that kernel type (same counting rules as hodlr_qr_info).
 * Host arrays of ntypes entries.  Synchronous and much slower than hodlr_qr.
 */
hodlr_status hodlr_qr_profile(const hodlr_t *A, double eps, double anorm, int32_t ntypes,
                              double *ms, int64_t *counts, double *flops,
                              hodlr_stream_t stream);
const char *hodlr_op_name(int32_t type);
int32_t hodlr_op_count(void);

/*
 * hodlr_qr_factor - borrowed view of one factor of F as a HODLR matrix:
 * which = 'Y' (unit lower triangular leaves, lower blocks), 'T' or 'R' (upper
 * triangular leaves, upper blocks).  The view stays valid while F lives; it
 * can be passed to hodlr_matmul and hodlr_export; hodlr_free ignores it, and
 * hodlr_qr / hodlr_qr_batched reject it (HODLR_EINVAL).
 */
hodlr_status hodlr_qr_factor(const hodlr_qr_t *F, char which, const hodlr_t **view);

/*
 * hodlr_check - wait for the work queued on `stream` and report the conditions
 * the device flagged for F: HODLR_ECAPACITY if a rank outgrew rank_cap, a
 * recompression outgrew 128 columns or a stacked leaf column outgrew 1024 rows;
 * HODLR_OK otherwise.
 */
hodlr_status hodlr_check(const hodlr_qr_t *F, hodlr_stream_t stream);

/*
 * hodlr_qr_ranklog - the decision of every recompression T_tau (Sec. 2.1.1) of
 * the factorisation, one record of 7 int32 each: (site, a, b, c, d, w, k) with
 * w the input width and k the kept rank (#{sigma_i > tau}).  Sites and keys:
 *   0 left-orthogonalisation of a lower block (a, b = its first row, column);
 *   1 i-th recompression of the sum S~ at the node covering [a, b) (c = i);
 *   2 the node's new upper block of R;
 *   3 the -_H update at node [a, b) of the block whose first row, column are c, d;
 *   4 i-th recompression of the sum T~12 at node [a, b) (c = i).
 * recs: host, room for `cap` records, or NULL to query *count only.  Synchronous.
 */
hodlr_status hodlr_qr_ranklog(const hodlr_qr_t *F, int32_t *recs, int64_t cap, int64_t *count);

/*
 * hodlr_plan_check - build the factorisation schedule of `count` matrices on
 * the partition (n, levels, leaf_off) with rank capacity rank_cap without a
 * device (every address virtual), and test it for hazards: every pair of
 * launches the two streams may run at the same time (lane order plus the
 * schedule's events) and every pair of jobs inside one launch is checked for a
 * write that overlaps the other's reads or writes (byte ranges from the jobs'
 * descriptors, ranks at capacity).  flags: HODLR_QR_ONE_STREAM checks the serial
 * order, HODLR_CHECK_ESTIMATE includes the |A|_2 estimate, HODLR_CHECK_PLANT
 * plants a known hazard (self test).  stats (host, 5): launches, launches of the
 * second stream, launch pairs checked, conflicting pairs, conflicting job pairs
 * within launches.  msg (host, msglen bytes, may be NULL): the first conflict.
 */
#define HODLR_CHECK_ESTIMATE 0x100u
#define HODLR_CHECK_PLANT 0x200u
hodlr_status hodlr_plan_check(int64_t n, int32_t levels, const int64_t *leaf_off, int32_t rank_cap,
                              int32_t count, uint32_t flags, int64_t *stats, char *msg, int64_t msglen);

/*
 * hodlr_plan_check_set - hodlr_plan_check of the merged launch sequence that
 * hodlr_qr_batched runs for `count` matrices of each of `nshapes` partitions
 * (n[i], levels[i]); leaf_off holds the partitions' leaf offsets one after
 * another (2^levels[i] + 1 entries each).  With nshapes == 1 it is
 * hodlr_plan_check; with more, HODLR_CHECK_PLANT gives every shape's schedule
 * the same workspace (a planted hazard between the jobs of merged launches).
 */
hodlr_status hodlr_plan_check_set(int32_t nshapes, const int64_t *n, const int32_t *levels,
                                  const int64_t *leaf_off, int32_t rank_cap, int32_t count, uint32_t flags,
                                  int64_t *stats, char *msg, int64_t msglen);

/*
 * Launch shapes of the schedules (an autotuned table, measured on MI355X).
 * mm_rt64_rows: product launches over at least this many output rows take 64
 * rows per block of threads, smaller ones 16; tr_small_chunks (1..4):
 * recompressions whose factors span at most this many 256-row chunks (rank
 * capacity <= 32) run in one launch, larger ones in two.  Only the launch shape
 * changes, not what is computed (results agree to rounding).
 * hodlr_tuning: the values schedules for order n and rank_cap get now.
 * hodlr_set_tuning: use `t` for every schedule built afterwards (NULL: the
 * table again); process-wide, takes effect at the next planning (a factor's
 * cached apply / solve / product sequences keep theirs).
 */
typedef struct {
  int32_t mm_rt64_rows;
  int32_t tr_small_chunks;
} hodlr_tuning_t;
hodlr_status hodlr_tuning(int64_t n, int32_t rank_cap, hodlr_tuning_t *out);
hodlr_status hodlr_set_tuning(const hodlr_tuning_t *t);

void hodlr_free(hodlr_t *A);        /* NULL-safe; ignores factor views */
void hodlr_qr_free(hodlr_qr_t *F);  /* NULL-safe */
const char *hodlr_last_error(void); /* thread-local; empty string if none */
const char *hodlr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HODLR_H */
