/*
 * rg.h -- C ABI of librg.so: rank-Greville recursive least squares on
 * MI355X (gfx950).
 *
 * The operation (Staub & Steinmann, "Efficient Recursive Least Squares Solver
 * for Rank-Deficient Matrices"): a stream receives observation rows
 * Gamma_i in R^m with targets y_i and keeps the minimum-norm least-squares
 * solution x_n = A_n^+ Y_n of the rows seen so far (introduction, definition
 * of the least-squares solution and its pseudoinverse form).  Each pushed row
 * is one call of Algorithm 1 (UpdateLeastSquares): projection gamma = Ct Gamma,
 * rejection Gamma_r = Gamma - C^T gamma, the rank test of Section 3, then the
 * independent update (Theorems 4 and 6) or the dependent update (Theorems 5
 * and 6).  The state is a full-rank factorisation: C (r x m, the accepted
 * rows), its dual basis Ct = (C C^T)^-1 C and P^-1 = (B^T B)^-1 (Section 2.1),
 * plus the solution in coordinates w = C x, so that x = Ct^T w.
 *
 * Conventions for every call:
 *  - Pointers marked (device) are HIP device pointers; (host) are host
 *    pointers.  The caller owns every buffer it passes and keeps it valid
 *    until the handle's HIP stream has passed the call.
 *  - Calls are ordered on the handle's HIP stream (rg_options.stream).  Only
 *    rg_rank / rg_batch_rank / rg_status_flags / rg_batch_flags synchronise
 *    that stream.
 *  - All state lives in one device workspace allocated by rg_init /
 *    rg_batch_init and freed by rg_destroy; pushes never allocate.
 *  - Errors: invalid arguments return RG_E_INVALID and leave the state
 *    untouched.  Conditions found on the device while rows are applied set a
 *    sticky per-stream flag (RG_FLAG_*): that row and every later row of that
 *    stream are ignored until rg_reset.  Pushes are asynchronous and return
 *    RG_OK once the work is enqueued, except that rg_push_rows returns
 *    RG_E_STATE (enqueueing nothing) once a synchronising call on the handle
 *    (rg_rank, rg_status_flags, rg_check, rg_batch_*) has seen the stream
 *    flagged.  rg_check / rg_batch_status map the flags to status codes.  No
 *    C++ exception crosses this boundary.
 *  - Element types: RG_F32 streams take float rows/targets and keep C and Ct
 *    in FP32, P^-1 in FP64 (FP32 Sherman-Morrison downdates lose positive
 *    definiteness on ill-conditioned bases), and the rejection, its norm, the
 *    rank decision, the Greville denominators, their reciprocals and w are
 *    FP64.  RG_F64 streams take double inputs and keep everything in FP64.
 *  - Factored form: the streams of the blocked on-chip classes, and the
 *    stream of a one-stream handle that no on-chip class holds (it runs in
 *    blocks of 16 rows over the whole GPU), keep the dual basis Ct = H^-1 C
 *    of Section 2.1 as C (the accepted input rows, exact in either element
 *    type) and H^-1 = (C C^T)^-1 in FP64; rg_batch_get_state forms Ct on
 *    request.  The rounding of x then grows like kappa(C)^2 2^-52 rather
 *    than kappa(C) times the state's unit roundoff.  FP64 streams project
 *    each block's rejections a second time, so that their rank decisions
 *    hold at FP64 tolerances.
 *  - Placement: FP32 streams take one of rg_class_count() on-chip classes
 *    (0 .. rg_class_count()-1).  The FP64 stream of a one-stream handle with
 *    m <= 128 and r_max <= 64 takes the on-chip class rg_class_count()
 *    (blocked, FP64 state, factored form); FP64 streams of batches run in the
 *    global-memory kernel, whose explicit Ct keeps the rank decision at FP64
 *    tolerances for larger kappa(C).  A stream alone in a handle that no
 *    class holds runs over the whole GPU; other streams run in the
 *    global-memory kernel.  RG_OPT_GENERIC_KERNEL and the variants of
 *    Section 2.2 select the global-memory kernel.
 */
#ifndef RG_H
#define RG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RG_OK = 0,
    RG_E_INVALID = 1,        /* bad argument; nothing was done */
    RG_E_NOMEM = 2,          /* device or host allocation failed (init only) */
    RG_E_DEVICE = 3,         /* a HIP runtime call failed */
    RG_E_RANK_CAPACITY = 4,  /* the stream holds RG_FLAG_RANK_CAPACITY */
    RG_E_NONFINITE = 5,      /* the stream holds RG_FLAG_NONFINITE */
    RG_E_STATE = 6,          /* the stream is flagged (for a push: flagged streams
                                take no rows until rg_reset; from rg_check: it
                                holds RG_FLAG_DENOMINATOR) */
    RG_E_UNSUPPORTED = 7     /* valid request outside the library's limits */
} rg_status;

typedef enum { RG_F32 = 0, RG_F64 = 1 } rg_dtype;

/* Sticky per-stream flags, set on the device. */
#define RG_FLAG_NONFINITE     0x1u  /* a row or target was NaN/Inf */
#define RG_FLAG_RANK_CAPACITY 0x2u  /* an independent row arrived at r == r_max */
#define RG_FLAG_DENOMINATOR   0x4u  /* 1 + gamma^T zeta not finite or <= 0 */

/* Option bits. */
#define RG_OPT_NO_REPROJECT   0x1u  /* skip the second projection pass of independent rows */
#define RG_OPT_GENERIC_KERNEL 0x2u  /* force the global-memory kernel (testing) */
#define RG_OPT_SERIAL_CLASSES 0x4u  /* launch the size classes one after another on the
                                       handle's stream instead of on forked streams */
#define RG_OPT_ROW_BY_ROW     0x8u  /* never apply rows in blocks: every row is one call of
                                       Algorithm 1 (reference path for the blocked variant) */
#define RG_OPT_DEPENDENT_BLOCKS_ONLY 0x10u  /* blocks take dependent rows only; independent
                                              rows are taken one at a time */
#define RG_OPT_ORTHOGONAL     0x20u  /* orthogonal rank factorization (Section 2.2, alpha = 1):
                                       C stores the rejections Gamma_r, whose rows are
                                       mutually orthogonal; same x and rank as Algorithm 1 */
#define RG_OPT_ORTHONORMAL    0x40u  /* orthonormal variant (alpha = 1 / ||Gamma_r||): C has
                                       orthonormal rows and C-tilde = C.  Streams with either
                                       variant bit run in the global-memory kernel; setting
                                       both bits is RG_E_INVALID */
#define RG_OPT_ONE_WG_PER_STREAM 0x80u  /* blocked on-chip classes: one workgroup per stream
                                          instead of the persistent grid (as many workgroups
                                          as fit on the chip, each taking streams from a
                                          queue, longest expected cost first) */
#define RG_OPT_EXPLICIT_REJECTIONS 0x100u  /* blocked on-chip classes: always form the
                                    rejections of a block, also when every row of it is
                                    dependent beyond doubt from ||Gamma||^2 - gamma^T v and
                                    its rounding bound (testing; results agree to rounding) */

typedef struct {
    int32_t dtype;   /* rg_dtype */
    int32_t r_max;   /* rank capacity per stream (<= m); <= 0 means m.  Used
                        only by rg_init; rg_batch_init takes per-stream values */
    double eps;      /* rank-test threshold of Section 3: a row is dependent
                        iff ||Gamma_r|| < eps or ||Gamma_r|| < eps ||Gamma||.
                        eps < 0 selects the default: for RG_F64 the paper's
                        (m^2 r + m r + m) 2^-52 at the current rank r, for
                        RG_F32 1e-3.  eps = 0 is the exact test Gamma_r == 0. */
    void *stream;    /* hipStream_t for every call on the handle; NULL = null stream */
    uint32_t flags;  /* RG_OPT_* */
} rg_options;

typedef struct rg_ctx *rg_handle;

/* Fill *opt with the defaults (RG_F32, r_max = m, eps = -1, null stream). */
void rg_default_options(rg_options *opt);

/* ---- one stream -------------------------------------------------------- */

/* Create a stream with m regressors (m >= 1) in the empty state (rank 0,
 * x = 0, i.e. A_0^+ = 0).  opt may be NULL.  An RG_F32 stream that an
 * on-chip size class holds runs in one workgroup; any other stream runs in
 * blocks of 16 rows over the whole GPU (unless RG_OPT_GENERIC_KERNEL or an
 * orthogonal variant selects the one-workgroup generic kernel). */
rg_status rg_init(rg_handle *out, int32_t m, const rg_options *opt);

/* Push k >= 0 rows: gamma (device, k x m row-major, dtype of the handle),
 * y (device, k).  Rows are applied in order, each as one call of
 * Algorithm 1.  k = 0 is a no-op. */
rg_status rg_push_rows(rg_handle h, const void *gamma, const void *y, int64_t k);

/* Write x_n = Ct^T w (device, m elements of the handle's dtype). */
rg_status rg_solution(rg_handle h, void *x);

/* Current rank r (host).  Synchronises the handle's stream. */
rg_status rg_rank(rg_handle h, int32_t *r);

/* Sticky RG_FLAG_* bits (host).  Synchronises the handle's stream. */
rg_status rg_status_flags(rg_handle h, uint32_t *flags);

/* Synchronise the handle's stream and return the stream's condition as a
 * status: RG_OK (no flag), RG_E_NONFINITE, RG_E_RANK_CAPACITY or RG_E_STATE
 * (RG_FLAG_DENOMINATOR), in that order of precedence when several flags are
 * set.  Single-stream handles only (RG_E_INVALID otherwise). */
rg_status rg_check(rg_handle h);

/* Back to the empty state (rank 0, x = 0, flags cleared); stream-ordered. */
rg_status rg_reset(rg_handle h);

/* Release the workspace.  Synchronises the handle's stream first. */
rg_status rg_destroy(rg_handle h);

/* ---- B independent streams --------------------------------------------- */

/* Create B >= 1 streams; m (host, B) gives each stream's regressor count and
 * r_max (host, B, nullable = m) its rank capacity.  opt->r_max is ignored.
 * Streams are numbered 0..B-1 everywhere below. */
rg_status rg_batch_init(rg_handle *out, int32_t B, const int32_t *m, const int32_t *r_max,
                        const rg_options *opt);

/* rg_batch_init on a workspace the caller provides: ws (device, at least
 * rg_workspace_bytes(B, m, r_max, opt->dtype) bytes, 256-byte aligned) holds
 * all device state of the handle, and the library allocates no device memory
 * for it; the caller keeps ws valid until rg_destroy, which does not free it.
 * ws_bytes smaller than needed or a misaligned ws is RG_E_INVALID.  The
 * handle itself (host) and, for batches whose streams fall into two or more
 * kernel classes, its auxiliary HIP streams and events are still created. */
rg_status rg_batch_init_ws(rg_handle *out, int32_t B, const int32_t *m, const int32_t *r_max,
                           const rg_options *opt, void *ws, size_t ws_bytes);

/* Check a packed row layout on the host before it is pushed: copies row_ptr
 * (device, B+1) and gamma_off (device, B) to the host (synchronising the
 * handle's stream) and returns RG_E_INVALID unless row_ptr starts at 0, never
 * decreases and ends at n_rows (the length of y), and every stream's rows
 * [gamma_off[b], gamma_off[b] + n_b m_b) lie inside [0, n_elems) (the length
 * of gamma) without overlapping another stream's.  rg_batch_push itself does
 * not read these arrays on the host. */
rg_status rg_batch_check_layout(rg_handle h, const int64_t *row_ptr, const int64_t *gamma_off, int64_t n_rows,
                                int64_t n_elems);

/* Per-stream condition (host, B rg_status values, as rg_check gives for one
 * stream).  Synchronises. */
rg_status rg_batch_status(rg_handle h, int32_t *status);

/* Push rows to every stream at once.  Stream b receives the rows
 * row_ptr[b] .. row_ptr[b+1]-1 of the packed target vector y (device), and
 * its rows start at element gamma_off[b] of gamma (device, each stream's
 * rows row-major n_b x m_b).  row_ptr (device, B+1 int64, non-decreasing) and
 * gamma_off (device, B int64) must describe in-bounds, non-overlapping rows:
 * the library does not read them on the host, except on a handle of one
 * stream that runs over the whole GPU (no on-chip size class holds it, and
 * neither RG_OPT_GENERIC_KERNEL nor an orthogonal variant is set): there it
 * copies row_ptr[0..1] and gamma_off[0] to the host,
 * waiting for the handle's stream, since that path enqueues one pass of
 * kernels per block of rows.  Streams are processed
 * concurrently in one persistent launch, largest expected cost first (see
 * rg_batch_plan). */
rg_status rg_batch_push(rg_handle h, const void *gamma, const void *y, const int64_t *row_ptr,
                        const int64_t *gamma_off);

/* Optional scheduling hint: rows_hint (host, B) = rows each stream will get
 * per push.  Streams are then taken longest first by rows * m * r_max
 * (default: m * m * r_max). */
rg_status rg_batch_plan(rg_handle h, const int64_t *rows_hint);

/* Write every x_b (device) packed back to back: x_b starts at element
 * sum_{c<b} m_c. */
rg_status rg_batch_solution(rg_handle h, void *x);

/* Ranks (host, B int32).  Synchronises. */
rg_status rg_batch_rank(rg_handle h, int32_t *r);

/* Flags (host, B uint32).  Synchronises. */
rg_status rg_batch_flags(rg_handle h, uint32_t *flags);

/* Kernel class of every stream (host, B int32): 0 .. rg_class_count()-1 for
 * FP32 streams, rg_class_count() for the FP64 stream of a one-stream handle
 * in the FP64 on-chip class,
 * or -1 for the global-memory kernel.  Fixed at init; does not synchronise. */
rg_status rg_batch_classes(rg_handle h, int32_t *cls);

/* Copy stream b's state to caller buffers (device; any may be NULL): C and
 * Ct as r x m row-major in the handle dtype, Pinv as r x r row-major doubles,
 * w as r doubles,
 * where r is the current rank (read it first with rg_batch_rank).
 * Synchronises the handle's stream; meant for tests and checkpoints. */
rg_status rg_batch_get_state(rg_handle h, int32_t b, void *C, void *Ct, void *Pinv, double *w);

/* Adjoint of the solve at constant rank (derivative of the rank-r truncated
 * pseudoinverse, Golub-Pereyra) for a loss L(x): given g = dL/dx (device,
 * packed like rg_batch_solution) and the rows A and targets Y that were
 * pushed since the last reset (device, laid out as in rg_batch_push), write
 * dL/dA (device, laid out like A) and dL/dY (device, laid out like Y):
 *   dL/dY = A s,  dL/dA = -(A s) x^T + (Y - A x) s^T + (A t) p^T,
 * with s = Ct^T P^-1 Ct g, t = Ct^T P^-1 Ct x, p = g - C^T Ct g, built from
 * the maintained factorisation (A^+ A^+T = Ct^T P^-1 Ct, A^+ A = C^T Ct). */
rg_status rg_batch_adjoint(rg_handle h, const void *A, const void *Y, const int64_t *row_ptr,
                           const int64_t *a_off, const void *g, void *dA, void *dY);

/* Pseudoinverse of every stream from its maintained factorisation (Theorem 1:
 * A^+ = Ct^T P^-1 B^T with B = A Ct^T): given the rows A that were pushed since
 * the last reset (device, laid out as in rg_batch_push), write A^+ of stream b
 * (device, m_b x n_b row-major, at element offset a_off[b], i.e. the same
 * number of elements and offset as the stream's rows; n_b = row_ptr[b+1] -
 * row_ptr[b]).  FP64 sums, stored in the handle dtype.  O(n m r) per stream;
 * stream-ordered. */
rg_status rg_batch_pinv(rg_handle h, const void *A, const int64_t *row_ptr, const int64_t *a_off, void *Ap);

/* ---- pseudoinverse maintained row by row (Theorems 2 and 3) ----------- */

/* Device bytes of the workspace rg_pinv_track needs (0 for invalid sizes):
 * per problem C and Ct (r_max x m), P^-1 (r_max x r_max), the coordinate
 * factor B (n x r_max) of A = B C, and beta (n), all FP64. */
size_t rg_pinv_track_workspace_bytes(int32_t B, int32_t n, int32_t m, int32_t r_max);

/* Push the n rows of each of B problems (all with n rows of m regressors)
 * through Algorithm 1 and maintain the pseudoinverse recursively
 * (Theorem 2, independent row: A^+ <- [A^+ - K beta^T, K] with
 * K = Gamma_r / ||Gamma_r||^2; Theorem 3, dependent row: the same with
 * K = Ct^T zeta / (1 + gamma^T zeta); beta = B zeta, zeta = P^-1 gamma).
 * O(m n) per row, FP64, base rank factorization, one workgroup per problem.
 *   A     device, B x n x m row-major (row i of problem b at (b n + i) m)
 *   Y     device, B x n targets
 *   eps   rank threshold of Section 3; < 0 takes the default
 *         (m^2 r + m r + m) eps_M at the rank before each row; NaN is invalid
 *   Ap    device output, B x m x n: A_n^+ of each problem, row-major
 *   X     device output, B x m: the minimum-norm least-squares solution
 *   rank  device output, B int32; flags device output, B uint32 (RG_FLAG_*)
 *   work  device workspace of at least rg_pinv_track_workspace_bytes bytes,
 *         owned by the caller; its contents on entry do not matter
 *   stream  hipStream_t to enqueue on (NULL = default stream)
 * A row that is not finite, an independent row at r == r_max or a
 * non-positive 1 + gamma^T zeta sets the flag and ends that problem: its later
 * columns of Ap and its X are then undefined.  r_max <= m; r_max >= min(n, m)
 * never runs out of capacity in exact arithmetic.  A, Y and Ap may be NULL
 * when n == 0.  Invalid arguments return RG_E_INVALID before any device work;
 * LDS needs over 160 KiB (3 m + 2 r_max doubles) return RG_E_UNSUPPORTED.
 * Stream-ordered; the caller synchronises before reading the outputs. */
rg_status rg_pinv_track(const double *A, const double *Y, int32_t B, int32_t n, int32_t m, int32_t r_max,
                        double eps, double *Ap, double *X, int32_t *rank, uint32_t *flags, void *work,
                        size_t work_bytes, void *stream);

/* rg_pinv_track with q >= 1 right-hand sides: Y (device, B x n x q; row i of
 * problem b has the q targets Y[(b n + i) q + c]) and X (device output,
 * B x m x q, the minimum-norm least-squares solutions X = A^+ Y, row-major).
 * Every right-hand side takes the same gain K per row, X <- X + K (y_i^T -
 * Gamma^T X); with Y = I_n, X equals A^+.  A non-finite target in any column
 * sets RG_FLAG_NONFINITE.  The LDS need grows by q doubles (RG_E_UNSUPPORTED
 * past 160 KiB); otherwise as rg_pinv_track, which is this call with q = 1. */
rg_status rg_pinv_track_rhs(const double *A, const double *Y, int32_t B, int32_t n, int32_t m, int32_t q,
                            int32_t r_max, double eps, double *Ap, double *X, int32_t *rank, uint32_t *flags,
                            void *work, size_t work_bytes, void *stream);

/* rg_pinv_track for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation and outputs, with the workspace taken from a fixed
 * device array inside the library instead of a caller buffer.  That array
 * holds rg_pinv_track_noalloc_max_bytes() bytes (32 MiB) on every GPU the
 * library runs on, for the life of the process; problems whose
 * rg_pinv_track_workspace_bytes exceeds it return RG_E_UNSUPPORTED before
 * any device work.  The call allocates nothing: no hipMalloc, no hipFree.
 * The caller still passes A, Y and the outputs (device, as for
 * rg_pinv_track).  Every call on one GPU shares that GPU's array, so calls
 * that overlap on one GPU (other streams, other threads) race and must be
 * ordered by the caller; the array's contents on entry do not matter.  The
 * first call on a device looks up the array's device address (once per
 * device, with that device current). */
rg_status rg_pinv_track_noalloc(const double *A, const double *Y, int32_t B, int32_t n, int32_t m, int32_t r_max,
                                double eps, double *Ap, double *X, int32_t *rank, uint32_t *flags, void *stream);

/* Size in bytes of the fixed device array rg_pinv_track_noalloc works in. */
size_t rg_pinv_track_noalloc_max_bytes(void);

/* ---- kernel size classes (tuning) -------------------------------------- */

/* FP32 streams run in one of rg_class_count() on-chip kernel classes, or in
 * the global-memory kernel.  By default a stream takes the smallest class that
 * holds it; a tuning tool can measure the classes and install rules instead.
 * Class rg_class_count() holds FP64 streams only and takes no rules. */
int32_t rg_class_count(void);

/* Shape of class cls (0 .. rg_class_count(), the last the FP64 class):
 * largest rank capacity, largest m, threads per stream (host outputs, each
 * nullable).  RG_E_INVALID for cls out of range. */
rg_status rg_class_info(int32_t cls, int32_t *r_max_cap, int32_t *m_cap, int32_t *threads);

/* *fits (host) = 1 if class cls can hold a stream with m regressors and rank
 * capacity r_max (including its on-chip memory at that capacity), else 0. */
rg_status rg_class_fits(int32_t cls, int32_t m, int32_t r_max, int32_t *fits);

/* Install process-wide placement rules, used by every later rg_init /
 * rg_batch_init (handles already created keep their classes).  A stream with
 * m regressors and capacity r_max takes the class of the first rule k with
 * m <= m_hi[k] and r_max <= r_max_hi[k] whose class can hold it; cls[k] = -1
 * selects the global-memory kernel.  Streams no rule places get the default.
 * The arrays (host, n entries) are copied; n = 0 restores the default.  Not
 * safe to call while another thread creates a handle. */
rg_status rg_set_class_rules(const int32_t *m_hi, const int32_t *r_max_hi, const int32_t *cls, int32_t n);

/* ---- measurement ------------------------------------------------------- */

/* LDS read-bandwidth probe, the reference for the on-chip kernels' state
 * traffic: launches blocks workgroups of 256 threads on stream (hipStream_t,
 * NULL = default); each thread reads 128 bytes of LDS per iteration for iters
 * iterations, so one launch reads blocks * 256 * 128 * iters bytes.  out
 * (device, blocks * 256 floats) receives a value that depends on the reads.
 * Stream-ordered; time it with events around the call. */
rg_status rg_probe_lds_read(void *out, int32_t blocks, int32_t iters, void *stream);

/* Device bytes the workspace of such a batch takes. */
size_t rg_workspace_bytes(int32_t B, const int32_t *m, const int32_t *r_max, int32_t dtype);

/* Static description of a status code. */
const char *rg_status_string(rg_status s);

#ifdef __cplusplus
}
#endif
#endif /* RG_H */
