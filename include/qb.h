/*
 * qb.h -- C ABI of the MI355X (gfx950) blocked randomized QB library.
 *
 * Method: Martinsson & Voronin, "A randomized blocked algorithm for
 * efficiently computing rank-revealing factorizations of matrices",
 * randQB_b (Figure 4, Sections 4.1-4.4) and its power-iteration form
 * randQB_pb (Figure 6, Section 5.2).  Given an m x n matrix A and a
 * tolerance eps, it returns Q (m x k, orthonormal columns), B (k x n) and
 * the rank k, built b columns at a time, such that ||A - Q B||_F <= eps
 * (Section 1.1, problem statement; Section 4.2, adaptive rank).
 *
 * Conventions for every entry point
 *   - matrices are column-major (LAPACK order); an m x n matrix X with
 *     leading dimension ldx >= m holds entry (i, j) at X[i + j * ldx];
 *   - matrix pointers are DEVICE pointers on the current HIP device; the
 *     caller owns every buffer, the library allocates no device memory;
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream);
 *     all device work is ordered on it.  Entry points that return host
 *     values synchronise that stream before returning;
 *   - return value: 0 on success, > 0 a warning (outputs valid), < 0 an
 *     error (outputs undefined, *k set to 0 where present).  The library
 *     never prints and never aborts.
 *
 * Not thread-safe for concurrent calls that share a workspace.
 */
#ifndef QB_H
#define QB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define QB_OK               0   /* stopped with ||A - QB||_F <= eps        */
#define QB_KMAX             1   /* k reached kmax < min(m, n) before eps   */
#define QB_RANK_EXHAUSTED   2   /* the residual is at the rounding level of
                                   the downdate, or k = min(m, n), or a
                                   block kept no column, before eps        */
#define QB_NOT_CONVERGED    3   /* qb_svd: the Jacobi sweeps reached their
                                   cap (60) before every column pair was
                                   orthogonal to 1e-15; outputs valid      */
#define QB_EINVAL          -1   /* invalid argument                        */
#define QB_ENONFINITE      -2   /* A holds a NaN or an infinity            */
#define QB_EWORKSPACE      -3   /* workspace NULL or smaller than required */
#define QB_EHIP            -4   /* a HIP runtime call failed               */
#define QB_ENODEVICE       -5   /* no usable gfx950 device                 */
#define QB_ETOOBIG         -6   /* qb_factor_noalloc: the problem needs more
                                   workspace than its fixed scratch        */

/* ---- stop reasons (qb_info.stop_reason) -------------------------------- */
#define QB_STOP_TOL_TRACKED 0   /* ||A||^2 - sum ||B_i||^2 <= eps^2 - delta */
#define QB_STOP_TOL_DIRECT  1   /* inside the band: ||A^(i)||_F^2 <= eps^2  */
#define QB_STOP_RANK_CAP    2   /* k = min(m, n)                           */
#define QB_STOP_EXHAUSTED   3   /* block kept no column / rounding floor   */
#define QB_STOP_KMAX        4   /* k = kmax < min(m, n)                    */
#define QB_STOP_ZERO        5   /* ||A||_F <= eps: k = 0                   */

/* ---- flags ------------------------------------------------------------- */
#define QB_OVERWRITE_A    (1u << 0)  /* A becomes the residual (Figure 4
                                        overwrites A); no copy is made     */
/* precision of the sampling products A*Omega, A^T*Q, A*Z (Fig. 6 (3),(5),(6)).
 * With P >= 1 the last A*Z of each block, whose columns span Q_i, runs in
 * float64 in every mode: a rounded product would leave in Q_i a component
 * outside range(A) that no later block removes once k = min(m, n) < m. */
#define QB_SAMPLE_F64     (0u << 4)
#define QB_SAMPLE_F32     (1u << 4)
#define QB_SAMPLE_BF16X3  (2u << 4)
/* Exact-range sample: A Omega_i is formed as the exact product, on the int8
 * MFMA with int32 sums, of A on a fixed-point grid (2^(E-55), E fixed by
 * ||A||_F so every entry lies below 2^(E-1); eight base-128 int8 digits per
 * entry) and the sketch rounded to a grid of 1/16 (int8, clipped at
 * +-127/16), then rounded once to float64.  The sample thus lies in range(A)
 * to float64 accuracy, so the factorisation reaches the tolerances of the
 * float64 form even at k = min(m, n) < m, where a rounded low-precision
 * sample floors at its own accuracy.  The sketch is the quantised Gaussian,
 * a different (equally valid) sketch from the float64 form's.  Power
 * iterations, if any, run in float64 in this mode.  Depth (n) per call is
 * unlimited (split in chunks of at most 2^17). */
#define QB_SAMPLE_INT8X8  (3u << 4)
#define QB_SAMPLE_MASK    (3u << 4)
/* precision of the projection B_i = Q_i^T A^(i-1) (Fig. 4 (4), Fig. 6 (9)).
 * The downdate, the residual norm and the stopping rule stay float64, so
 * ||A - QB||_F <= eps still holds when the call returns QB_OK; but a B below
 * float64 leaves its own rounding error in the residual, so the attainable
 * error floors near 1e-7 (f32) and 1e-5 (bf16x3) of ||A||_F.  Sweep
 * variants: they report that floor; they do not reach tight tolerances. */
#define QB_BGEMM_F64      (0u << 6)
#define QB_BGEMM_F32      (1u << 6)
#define QB_BGEMM_BF16X3   (2u << 6)
#define QB_BGEMM_MASK     (3u << 6)
/* Section 5.4 / Figure 8 comparison: skip the orthonormalisation between
 * applications of A and A^T, i.e. Y = (A A^T)^P A Omega_i, then Q_i = orth(Y).
 * Without it a pass resolves nothing below sigma_1 tau^(1/(2P+1)), tau = 2^-20
 * the relative column size orth can separate; the blocked scheme recovers
 * the rest in later blocks. */
#define QB_POWER_NO_ORTH  (1u << 8)
/* Stop after the first block whatever its kept width: the unblocked randQB
 * (Figure 3) and randQB_p (Figure 5) with l = b.  Returns QB_KMAX (stop
 * reason QB_STOP_KMAX) unless the tolerance was met. */
#define QB_SINGLE_BLOCK   (1u << 9)
/* Queue no work past the stop decision.  By default qb_factor, while the
 * host reads block i's stop quantities, already queues the sketch and the
 * sampling product of block i + 1 on `stream` (assuming no column was
 * dropped); when the run stops there, that work is left queued and writes
 * the workspace (sketch, sample and split-K partial areas; never A, Q or B)
 * after qb_factor has returned.  Work ordered after `stream` is unaffected;
 * a caller that hands the workspace to another stream without ordering it
 * after `stream` must pass this flag. */
#define QB_NO_SPECULATE   (1u << 10)

/* Per-call report.  The trace arrays are optional HOST arrays owned by the
 * caller (set the pointers to NULL or trace_cap to 0 to skip).  Entry i
 * describes block i: kept columns, tracked indicator E_i = ||A||_F^2 -
 * sum_{j<=i} ||B_j||_F^2, and direct D_i = ||A^(i)||_F^2. */
typedef struct qb_info {
  int64_t k;              /* rank of the factorisation (columns of Q)      */
  int32_t blocks;         /* number of blocks added                        */
  int32_t stop_reason;    /* QB_STOP_*                                     */
  double  normA2;         /* ||A||_F^2                                     */
  double  indicator;      /* last E_i                                      */
  double  resid2;         /* last D_i                                      */
  int32_t trace_cap;      /* capacity of the trace arrays                  */
  int32_t trace_len;      /* entries written (<= trace_cap)                */
  int32_t* trace_w;       /* kept columns per block                        */
  double* trace_E;        /* E_i per block                                 */
  double* trace_D;        /* D_i per block                                 */
} qb_info;

/* Bytes of device workspace qb_factor needs for these sizes.  kmax < 0
 * means min(m, n); kmax = 0 is a capacity of zero columns.  Returns 0 for
 * sizes qb_factor rejects (see qb_factor: m, n, b, kmax). */
size_t qb_workspace_bytes(int64_t m, int64_t n, int32_t b, int64_t kmax, uint32_t flags);

/*
 * qb_factor -- blocked adaptive randomized QB (randQB_pb; randQB_b when
 * power_iters = 0).
 *
 *  A            m x n input, lda >= m.  Read-only unless QB_OVERWRITE_A, in
 *               which case it holds the final residual A - Q B on return.
 *               1 <= m < 2^24 - 1, 1 <= n <= 65535 * 64 (the limits of the
 *               kernels' 32-bit tile offsets and of the downdate grid).
 *  eps          Frobenius tolerance, finite and >= 0.
 *  b            block size >= 1.  Each block adds at most b columns.
 *  power_iters  P >= 0 power iterations per block (Figure 6 steps (4)-(7)).
 *  seed         64-bit seed of the Gaussian sketch: entry (i, j) of the
 *               n x infinity sketch depends only on (seed, i, j) (Philox4x32-10
 *               with counter (i/2, j, 0, 0), Box-Muller), so block i uses
 *               sketch columns [k, k + w) whatever b is.
 *  Q, ldq       output, m x kmax, ldq >= m.  Columns [0, k) are written.
 *  B, ldb       output, kmax x n, ldb >= kmax.  Rows [0, k) are written.
 *               lda, ldq and ldb are below 2^24; 1 <= b <= 256.
 *  kmax         capacity (max rank), 0 <= kmax <= min(m, n); kmax < 0 means
 *               min(m, n) (then Q and B must hold min(m, n) columns/rows).
 *  k            HOST out: the rank.
 *  info         HOST in/out, may be NULL.
 *  workspace    device buffer of at least qb_workspace_bytes(...) bytes,
 *               256-byte aligned.
 *  flags        QB_OVERWRITE_A, one QB_SAMPLE_* and one QB_BGEMM_* value,
 *               QB_POWER_NO_ORTH, QB_SINGLE_BLOCK, QB_NO_SPECULATE.
 *
 * Synchronises `stream` once per block (to read the stop quantities).  On
 * return the stream may still hold the speculative sketch and sample of
 * one further block, which write only the workspace (QB_NO_SPECULATE).
 * Errors: QB_EINVAL (arguments, sizes), QB_EWORKSPACE (NULL or too small),
 * QB_ENODEVICE (no current device, or not a gfx950), QB_ENONFINITE,
 * QB_EHIP.
 */
int qb_factor(const double* A, int64_t m, int64_t n, int64_t lda,
              double eps, int32_t b, int32_t power_iters, uint64_t seed,
              double* Q, int64_t ldq, double* B, int64_t ldb, int64_t kmax,
              int64_t* k, qb_info* info, void* workspace, size_t ws_bytes,
              void* stream, uint32_t flags);

/*
 * qb_factor_noalloc -- qb_factor for callers that cannot allocate: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and errors as qb_factor, with no
 * workspace argument: the workspace is a fixed device array of
 * QB_NOALLOC_SCRATCH_BYTES inside the library, one per device, held from
 * the library's load until the process ends.  The call allocates nothing
 * (no hipMalloc, hipFree, pinned host memory or events): the per-block
 * stop quantities are copied to a host stack buffer and the stream is
 * synchronised instead, and the stream is idle when the call returns.
 * Keep qb_profile_enable off, as its events are created on demand.
 *
 * Limit: problems for which qb_workspace_bytes(m, n, b, kmax, flags)
 * exceeds QB_NOALLOC_SCRATCH_BYTES are rejected with QB_ETOOBIG before any
 * device work (QB_OVERWRITE_A saves the m x n residual copy).  Every call
 * on a device shares that device's scratch, which keeps the last call's
 * contents (no result depends on them): calls that overlap on one device,
 * from different streams or threads, race and must be serialised by the
 * caller.
 */
#define QB_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int qb_factor_noalloc(const double* A, int64_t m, int64_t n, int64_t lda,
                      double eps, int32_t b, int32_t power_iters, uint64_t seed,
                      double* Q, int64_t ldq, double* B, int64_t ldb, int64_t kmax,
                      int64_t* k, qb_info* info, void* stream, uint32_t flags);

/* Human-readable name of a status code (static string). */
const char* qb_status_string(int status);

/* ---- component entry points (same kernels the factorisation uses) ------
 * Leading dimensions are below 2^24.  Like qb_factor they return
 * QB_ENODEVICE when the current device is not a gfx950. */

/* Columns [col0, col0 + w) of the Gaussian sketch (Figure 4 step (2);
 * Section 4.1 eq. (OmegaBlock)): out is n x w, ld >= n, device. */
int qb_sketch(uint64_t seed, int64_t n, int64_t col0, int32_t w,
              double* out, int64_t ld, void* stream);

/* orth(X) (Section 2.4) by Cholesky QR applied twice with column dropping:
 * Q (m x w, ldq >= m, may alias X only if ldq == ldx) receives the kept
 * columns first, then zero columns; *kept (HOST out) is their number.
 * X is m x w, ldx >= m, 1 <= w <= 256.  Workspace: qb_orth_workspace_bytes. */
size_t qb_orth_workspace_bytes(int64_t m, int32_t w);
int qb_orth(const double* X, int64_t m, int32_t w, int64_t ldx,
            double* Q, int64_t ldq, int32_t* kept,
            void* workspace, size_t ws_bytes, void* stream);

/* Y = X * W (m x w) in the requested sampling precision (QB_SAMPLE_*):
 * X m x K (ldx), W K x w (ldw), Y m x w (ldy); w <= 256.  This is the
 * product of Figure 4 step (3) and Figure 6 step (6).  QB_SAMPLE_INT8X8
 * computes the exact product of W rounded to the 1/16 grid (clipped at
 * +-127/16) with X on the fixed-point grid that ||X||_F fixes (see the
 * flag), rounded once to float64.
 * Workspace: qb_gemm_workspace_bytes(m, K, w), 256-byte aligned. */
size_t qb_gemm_workspace_bytes(int64_t m, int64_t K, int32_t w);
int qb_sample(const double* X, int64_t m, int64_t K, int64_t ldx,
              const double* W, int32_t w, int64_t ldw,
              double* Y, int64_t ldy, uint32_t precision,
              void* workspace, size_t ws_bytes, void* stream);

/* C = Q^T X (w x N) in the requested precision: Q is K x w (ldq), X is
 * K x N (ldx), C is w x N (ldc); w <= 256.  Figure 4 step (4), Figure 6
 * steps (5) and (9).  precision: QB_SAMPLE_F64, _F32 or _BF16X3.
 * Workspace: qb_gemm_workspace_bytes(N, K, w), 256-byte aligned. */
int qb_project(const double* Qm, int64_t K, int32_t w, int64_t ldq,
               const double* X, int64_t N, int64_t ldx,
               double* C, int64_t ldc, uint32_t precision,
               void* workspace, size_t ws_bytes, void* stream);

/* R <- R - Q B (Figure 4 step (5)) with the fused residual norm:
 * R m x n (ldr), Q m x w (ldq), B w x n (ldb); *resid2 (HOST out, may be
 * NULL) receives ||R||_F^2 after the update.
 * Workspace: qb_downdate_workspace_bytes(m, n). */
size_t qb_downdate_workspace_bytes(int64_t m, int64_t n);
int qb_downdate(double* R, int64_t m, int64_t n, int64_t ldr,
                const double* Qm, int32_t w, int64_t ldq,
                const double* B, int64_t ldb, double* resid2,
                void* workspace, size_t ws_bytes, void* stream);

/* ||X||_F^2 (notation of Section 2.1) with a compensated final sum;
 * *out (HOST) receives it, *nonfinite (HOST, may be NULL) is set to 1 if X
 * holds a NaN or infinity.  Workspace: qb_downdate_workspace_bytes(m, n). */
int qb_frob2(const double* X, int64_t m, int64_t n, int64_t ldx,
             double* out, int32_t* nonfinite,
             void* workspace, size_t ws_bytes, void* stream);

/* ---- standard factorisations from Q B (Section 3.3) ------------------------
 * Inputs: Q (m x k, orthonormal columns, ldq >= m) and B (k x n, ldb >= k)
 * as produced by qb_factor, device, column-major; 1 <= k <= min(m, 4096).
 * Outputs are caller-owned device arrays; workspaces come from the
 * *_workspace_bytes calls (0 = invalid sizes), 256-byte aligned.  Errors:
 * QB_EINVAL (sizes, leading dimensions, NULL), QB_EWORKSPACE, QB_EHIP. */

/* Low-rank SVD (Section 3.3.1): Q B = U diag(S) V^T with U (m x k, ldu >= m)
 * and V (n x k, ldv >= n) orthonormal and S (k) non-increasing.  The SVD of
 * B is computed by one-sided Jacobi on B^T (high relative accuracy); a
 * zero singular value gets a zero column in V.  *sweeps (HOST, may be NULL)
 * receives the number of Jacobi sweeps.  Truncation to a rank is left to
 * the caller (S is sorted).  Returns QB_OK or QB_NOT_CONVERGED. */
size_t qb_svd_workspace_bytes(int64_t m, int64_t n, int64_t k);
int qb_svd(const double* Q, int64_t m, int64_t k, int64_t ldq,
           const double* B, int64_t n, int64_t ldb,
           double* U, int64_t ldu, double* S, double* V, int64_t ldv,
           int32_t* sweeps, void* workspace, size_t ws_bytes, void* stream);

/* Partial column-pivoted QR (Section 3.3.2): A P ~ Q B P = Qhat R with
 * Qhat = Q Q_tilde (m x k, ldqh >= m), R (k x n upper trapezoidal,
 * ldr >= k) and perm (n, device int64): column j of Qhat R is column
 * perm[j] of Q B.  Householder QR of B with column pivoting: column norms
 * recomputed every step, ties to the smallest index, R_jj = -sign(pivot
 * entry) * norm. */
size_t qb_pivoted_qr_workspace_bytes(int64_t m, int64_t n, int64_t k);
int qb_pivoted_qr(const double* Q, int64_t m, int64_t k, int64_t ldq,
                  const double* B, int64_t n, int64_t ldb,
                  double* Qhat, int64_t ldqh, double* R, int64_t ldr, int64_t* perm,
                  void* workspace, size_t ws_bytes, void* stream);

/* ---- batched QB ------------------------------------------------------------
 * Many independent factorisations (Figure 4, P = 0) advanced together: each
 * step of the block loop is one launch over every problem still active, and
 * each problem stops by the rule of qb_factor on its own.  Inputs are float
 * (the storage of the batched workload); every stored value and product is
 * float64, so each problem follows the float64 qb_factor.  Callers that
 * cannot afford one float64 copy of every input in the workspace should
 * split the batch. */
typedef struct qb_problem {
  /* inputs */
  const float* A;         /* device, column-major, m x n, lda >= m          */
  int64_t m, n, lda;
  double eps;             /* absolute Frobenius tolerance                    */
  uint64_t seed;          /* sketch seed (the Philox key of qb_sketch)       */
  int64_t kmax;           /* cap on k, < 0 for min(m, n)                     */
  double* Q;              /* device, m x kmax, ldq >= m (float64)            */
  int64_t ldq;
  double* B;              /* device, kmax x n, ldb >= kmax (float64)         */
  int64_t ldb;
  int32_t b;              /* block size, 1 <= b <= 64                        */
  /* outputs */
  int32_t status;         /* as qb_factor; QB_ENONFINITE for a NaN or Inf    */
  int32_t stop_reason;    /* QB_STOP_*                                       */
  int32_t blocks;
  int64_t k;
  double normA2, resid2;  /* ||A||_F^2 and the final ||A - QB||_F^2         */
} qb_problem;

/* Workspace for a batch (0 when any problem is invalid): one float64 copy
 * of each A plus O((m + n) b) and 8 MiB of split-K partials per problem. */
size_t qb_factor_batched_workspace_bytes(const qb_problem* probs, int32_t count);
/* probs: HOST array; every problem's outputs are written there.  Returns
 * QB_OK when the batch ran (see each problem's status), QB_EINVAL when any
 * problem is invalid (nothing runs), QB_EWORKSPACE or QB_EHIP.  Each
 * problem's stop decision is taken on the device; eight block iterations
 * at a time run as one HIP graph launch on `stream`, after which the call
 * reads the problems' state (which are still active) and, once they need
 * much smaller launches, captures the graph again for them.  It thus
 * synchronises the stream once per eight iterations and returns with the
 * stream idle.  It keeps a pinned host staging buffer per calling thread,
 * grown to the largest batch seen, for the problem records. */
int qb_factor_batched(qb_problem* probs, int32_t count, void* workspace, size_t ws_bytes,
                      void* stream);

/* Tile classes of the batched products (process-wide).  Each product role
 * of a block iteration takes, per panel width class (0: w <= 16, 1: w <= 32,
 * 2: w <= 64), one output tile class.  Every allowed class computes the
 * same products (results may differ in the last bits, as the depth split
 * follows the tile count); B_i and the downdate allow every class but
 * 16 x 16, the others any class.  For the tuner
 * (paper_1503_07157_amd/autotune.py) and for callers with their own
 * measurements; batched calls that start after a change use it.
 * qb_batched_set_tile returns QB_OK or QB_EINVAL (unknown role, class or
 * width class, or a class not allowed for the role); qb_batched_get_tile
 * returns the class or QB_EINVAL. */
#define QB_TILE_64X64 0
#define QB_TILE_16X16 1
#define QB_TILE_32X32 2
#define QB_TILE_64X32 3  /* 64 rows x 32 columns: panels as the N side */
#define QB_TILE_32X64 4  /* 32 rows x 64 columns: panels as the M side */
#define QB_ROLE_SAMPLE 0     /* R Omega_i                */
#define QB_ROLE_GRAM 1       /* X^T X of each CholQR pass */
#define QB_ROLE_APPLY 2      /* X T^{-1}                  */
#define QB_ROLE_REPROJ_C 3   /* Qbar^T Q_i                */
#define QB_ROLE_REPROJ_Q 4   /* Q_i - Qbar C              */
#define QB_ROLE_B 5          /* B_i = Q_i^T R             */
#define QB_ROLE_DOWNDATE 6   /* R - Q_i B_i               */
#define QB_ROLES 7
int qb_batched_set_tile(int32_t role, int32_t width_class, int32_t tile_class);
int qb_batched_get_tile(int32_t role, int32_t width_class);

/* ---- adjoint of the fixed-sketch map A -> (Q, B) ----------------------------
 * With the sketch (seed), the block width b, the number of blocks s and the
 * number of power iterations P fixed, the blocked scheme (Figure 4, with the
 * power iterations of Figure 6 and the re-projection of Section 4.3) maps A
 * to Q = [Q_1 .. Q_s] (m x s b) and B = [B_1; ..; B_s] (s b x n) smoothly
 * wherever every orthonormalisation sees a full-column-rank matrix; that
 * map is qb_factor(A, eps = 0, b, P, seed) with kmax = s b when no column
 * is dropped.
 *
 * qb_adjoint writes dA = J^T (dQ, dB), the gradient of <dQ, Q> + <dB, B>
 * with respect to A (m x n, lda), given A and the forward's Q (m x s b, ldq)
 * and B (s b x n, ldb).  dQ (m x s b, lddq) or dB (s b x n, lddb) may be
 * NULL for a zero upstream gradient.  Only Q and B of the forward are used:
 * the samples and power-iteration intermediates are recomputed.  All
 * matrices are float64, column-major, device memory; dA (ldda >= m) is
 * overwritten and must not alias the inputs.
 *
 * Requirements: 1 <= b <= 256, s >= 1, s b <= min(m, n), 0 <= P <= 8,
 * leading dimensions below 2^24.  Returns QB_OK; QB_RANK_EXHAUSTED when a
 * recomputed orthonormalisation dropped a column (the map is not
 * differentiable there; dA is then unspecified); QB_EINVAL, QB_EWORKSPACE
 * or QB_EHIP.  Synchronises the stream before returning. */
size_t qb_adjoint_workspace_bytes(int64_t m, int64_t n, int32_t b, int32_t blocks,
                                  int32_t power_iters);
int qb_adjoint(const double* A, int64_t m, int64_t n, int64_t lda, int32_t b, int32_t blocks,
               int32_t power_iters, uint64_t seed, const double* Q, int64_t ldq, const double* B,
               int64_t ldb, const double* dQ, int64_t lddq, const double* dB, int64_t lddb,
               double* dA, int64_t ldda, void* workspace, size_t ws_bytes, void* stream);

/* ---- measurement ---------------------------------------------------------
 * Optional per-kernel timing: when enabled, every kernel launch of the
 * library is bracketed by two HIP events on the stream it runs on and
 * tagged with the algorithmic flops and bytes of the operation (for a
 * product of an M x K by a K x N matrix: 2 M N K flops and one read of each
 * operand plus one write of the result).  qb_profile_enable clears the
 * counters; qb_profile_read waits for the pending events and returns the
 * totals for kernel class `kernel` (0 <= kernel < qb_profile_count()). */
int qb_profile_enable(int on);
int32_t qb_profile_count(void);
const char* qb_profile_name(int32_t kernel);
int qb_profile_read(int32_t kernel, double* ms, int64_t* launches, double* flops, double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* QB_H */
