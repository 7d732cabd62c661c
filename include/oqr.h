/*
 * oqr.h -- oblique QR factorisation on one MI355X (gfx950), plain C ABI.
 *
 * Given a symmetric positive definite m x m operator A and a full-rank m x n
 * matrix Z (m >= n), compute Z = Q R with R (n x n) upper triangular with a
 * positive diagonal and Q^T A Q = I (Lowery & Langou, "Stability Analysis of
 * QR factorization in an Oblique Inner Product", Section 1).  The pair is
 * unique: R is the Cholesky factor of the normal-equation matrix Z^T A Z.
 *
 * Conventions shared by every entry point
 *   - Matrices are column-major with a leading dimension: element (i, j) of
 *     X is X[i + j * ldx].  A torch caller passes an (n, m) row-major tensor,
 *     which is the same memory.
 *   - Pointers named *_dev, and the matrix pointers A->a, Z, Q, R, are device
 *     pointers owned by the caller.  Descriptor structs (oqr_op, oqr_opts) are
 *     host memory read during the call only.
 *   - The library allocates nothing inside a call.  Scratch memory is the
 *     caller's workspace `ws` of at least oqr_workspace_bytes(...) bytes
 *     (256-byte aligned); its contents on entry are irrelevant.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream)
 *     and the call returns without synchronising.
 *   - The return value reports host-detectable errors only (oqr_status).
 *     Numerical failure is reported on the device in *info_dev, following
 *     LAPACK potrf: 0 = success; k > 0 = the k-th pivot of the n x n
 *     Cholesky factorisation was not positive (or NaN) after all shifted
 *     retries.  On info_dev != 0 the contents of Q are unspecified.
 *   - Q may alias Z (same pointer and ld): the triangular solve is done in
 *     place.  No other aliasing is allowed (A, R, ws, info distinct).
 *   - R is written in full: strictly lower triangle set to 0.
 *   - Dense A must be stored in full and symmetric (A = A^T).  The FP64
 *     CholQR passes read only its upper block triangle (the blocks of 64 rows
 *     on and above the diagonal) and form Z^T A Z = Z^T (U + D) Z + (U Z)^T Z
 *     with U the strictly upper blocks and D the diagonal ones; the other
 *     entry points read the whole of A.
 */
#ifndef OQR_H
#define OQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes (host-detectable errors). */
typedef enum {
  OQR_OK = 0,
  OQR_E_ARG = 1,          /* bad size, leading dimension, null pointer or option */
  OQR_E_NOT_SPD = 2,      /* reserved: numerical failure is reported in info_dev */
  OQR_E_HIP = 3,          /* a HIP launch or runtime call failed */
  OQR_E_WORKSPACE = 4,    /* workspace too small or misaligned */
  OQR_E_UNSUPPORTED = 5,  /* valid request the library does not implement (n or a leading
                             dimension beyond the limits below OQR_MAX_N) */
  OQR_E_SCRATCH = 6       /* oqr_cholqr2_noalloc: the request needs more than its fixed scratch */
} oqr_status;

/* Storage type of A, Z, Q and R. */
typedef enum { OQR_F64 = 0, OQR_F32 = 1 } oqr_dtype;

/* Kind of operator A. */
typedef enum {
  OQR_OP_DENSE = 0,       /* explicit m x m symmetric matrix */
  OQR_OP_STENCIL7 = 1,    /* matrix-free 7-point operator on an nx x ny x nz grid */
  OQR_OP_TRIDIAG = 2      /* symmetric tridiagonal matrix (the sparse workload of Section 8) */
} oqr_op_kind;

/* The operator A.
 *   dense:   a = device pointer to A (column-major, full symmetric storage),
 *            lda >= m.  Single-instance entry points take dtype = OQR_F64.
 *   stencil: m = nx*ny*nz, grid index p = x + nx*(y + ny*z);
 *            (A z)_p = center*z_p + off*(sum of z_q over the face neighbours
 *            q of p inside the grid) -- homogeneous Dirichlet boundary.  The
 *            Dirichlet 3D Laplacian (h = 1) plus s*I is center = 6 + s,
 *            off = -1.  a and lda are ignored.
 *   tridiag: a = device pointer to 2m-1 doubles, the diagonal d (m values)
 *            followed by the off-diagonal e (m-1 values): A(i,i) = d_i,
 *            A(i,i+1) = A(i+1,i) = e_i; lda must equal m (the offset of e). */
typedef struct oqr_op {
  int32_t kind;
  int32_t dtype;
  const void* a;
  int64_t lda;
  int32_t nx, ny, nz;
  int32_t reserved;
  double center;
  double off;
} oqr_op;

/* Arithmetic of the operator product A*Z (dense A) or of the Gram product
 * Z^T W (stencil A) within one CholQR pass.  Gram accumulation across tiles,
 * the Cholesky factorisation and the triangular solve are FP64 always.
 *   FP64    : FP64 throughout.
 *   BF16X2  : operands split into two bfloat16 slices (hi = bf16(x),
 *             lo = bf16(x - hi)), products hi*hi + hi*lo + lo*hi on MFMA,
 *             FP32 accumulation inside a tile of K, FP64 across tiles.
 *   BF16X3  : three slices, the six products with slice indices i + j < 3.
 *   FP32    : operands rounded to FP32 (nearest), products on FP32 MFMA,
 *             FP32 accumulation inside a tile of K (at most 960 rows for
 *             the dense product, 256 for the Gram), FP64 across tiles.
 *             For the 7-point operator A Z is formed in FP64 first (the
 *             unfused path) and the Gram runs in FP32.
 * Every reduced-precision pass (BF16X2, BF16X3, FP32) starts with the shift
 * of oqr_opts (unit roundoff u_p = 2^-24). */
typedef enum { OQR_P_FP64 = 0, OQR_P_FP32 = 1, OQR_P_BF16X2 = 2, OQR_P_BF16X3 = 3 } oqr_prec;

/* Gram-Schmidt variants for oqr_gs (Section 6 and the comments of Section 8). */
typedef enum {
  OQR_GS_CGS = 0,         /* classical Gram-Schmidt */
  OQR_GS_MGS_ROW = 1,     /* modified, R computed a row at a time (A applied once per column) */
  OQR_GS_MGS_COL = 2,     /* modified, R computed a column at a time (A inside the inner loop) */
  OQR_GS_CGS2 = 3         /* classical with one reorthogonalisation */
} oqr_gs_variant;

/* Options.  NULL means the defaults of oqr_default_opts().
 *   pass1, pass2  oqr_prec of the first and second CholQR pass (CholQR uses pass1 only).
 *   shift_c       first-attempt shift s = shift_c * u_p * max_i G_ii added to the
 *                 diagonal of G before the Cholesky factorisation, with u_p = 2^-24
 *                 for reduced-precision passes; FP64 passes start unshifted.  On a
 *                 failed pivot the factorisation is redone from the kept G with the
 *                 constant multiplied by 10 (an unshifted FP64 pass retries with
 *                 shift_c * 2^-53), at most max_retries times.
 *   max_retries   number of shifted retries (0..16).
 *   gs_variant    oqr_gs_variant, used by oqr_gs only. */
typedef struct oqr_opts {
  int32_t pass1;
  int32_t pass2;
  double shift_c;
  int32_t max_retries;
  int32_t gs_variant;
} oqr_opts;

/* Algorithms, for the workspace query. */
typedef enum {
  OQR_ALG_CHOLQR = 0, OQR_ALG_CHOLQR2 = 1, OQR_ALG_CHOL_A = 2, OQR_ALG_EIG_A = 3, OQR_ALG_GS = 4,
  OQR_ALG_PRE_CHOLQR = 5
} oqr_alg;

/* Largest n the single-instance kernels support. */
#define OQR_MAX_N 256

/* Size limits of the single-instance entry points, oqr_check and oqr_gls: the
 * kernels address operands with 32-bit byte offsets from a base that moves
 * with the tile, a tile spanning up to c = min(columns, 256) columns of an
 * operand (dense operator) or c = min(columns, 64) (stencil, tridiagonal).
 * Each leading dimension (of Z and Q with n columns, of B with k columns),
 * and m + 32, must not exceed (2^31 - 1) / (8 c) rows: at n >= 64 that is
 * 1048575 rows for a dense operator with n >= 256 and 4194303 otherwise; and
 * n * ldr must not exceed (2^31 - 1) / 8.
 * Beyond that the call returns OQR_E_UNSUPPORTED before touching the device. */

/* Fills *opts with the defaults: pass1 = pass2 = FP64, shift_c = 1, max_retries = 3, CGS. */
void oqr_default_opts(oqr_opts* opts);

/* Workspace bytes needed by algorithm `alg` for this operator and size
 * (0 on invalid arguments). */
size_t oqr_workspace_bytes(int32_t alg, const oqr_op* A, int64_t m, int64_t n, const oqr_opts* opts);

/* CHOLQR-A (Algorithm 1, Section 2): W = A Z, G = Z^T W, R = chol(G [+ shift]),
 * Q = Z R^{-1} by row-wise substitution (FP64).  Precision of A Z / Z^T W is
 * opts->pass1.  Arguments as described at the top of this file. */
int oqr_cholqr(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n,
               double* Q, int64_t ldq, double* R, int64_t ldr, const oqr_opts* opts,
               void* ws, size_t ws_bytes, int32_t* info_dev, void* stream);

/* CholQR2-A: CHOLQR-A twice, (Q1, R1) = CHOLQR(A, Z) in precision pass1,
 * (Q, R2) = CHOLQR(A, Q1) in precision pass2, R = R2 R1.  Like the
 * preconditioning step of PRE-CHOLQR (Algorithm 2, Section 3), the first
 * pass removes the kappa(Z) dependence of the loss of orthogonality; the
 * analysis of Theorem 2.1 with Z = Q1 gives loss c m n u ||A|| ||Q||^2.
 * info_dev reports the first pass that failed (its pivot index). */
int oqr_cholqr2(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n,
                double* Q, int64_t ldq, double* R, int64_t ldr, const oqr_opts* opts,
                void* ws, size_t ws_bytes, int32_t* info_dev, void* stream);

/* Allocation-free CholQR2-A, for callers that cannot allocate device memory
 * or pass a workspace (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels, results (bit
 * for bit) and info_dev convention as oqr_cholqr2, without ws / ws_bytes:
 * the scratch is a device array of OQR_NOALLOC_SCRATCH_BYTES owned by the
 * library, one per device, held from the first use on that device until the
 * process ends.  The first call on a device looks up the array's device
 * address (hipGetSymbolAddress, with that device current) and keeps it; make
 * that first call outside any graph capture.  No call allocates (no hipMalloc,
 * no hipFree, no allocating library routine); the caller still passes Z, Q,
 * R and info_dev.
 * Limits: a request whose oqr_cholqr2 workspace (oqr_workspace_bytes with
 * OQR_ALG_CHOLQR2) exceeds OQR_NOALLOC_SCRATCH_BYTES returns OQR_E_SCRATCH
 * before anything is enqueued.  Every call on one device shares that device's
 * scratch, which keeps the last call's contents (nothing in it needs to start
 * at zero): calls that overlap on one device (two streams, two host threads)
 * race and give undefined results; calls on one stream are ordered and safe. */
#define OQR_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
size_t oqr_noalloc_scratch_bytes(void);
int oqr_cholqr2_noalloc(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n,
                        double* Q, int64_t ldq, double* R, int64_t ldr, const oqr_opts* opts,
                        int32_t* info_dev, void* stream);

/* PRE-CHOLQR-A (Algorithm 2, Section 3): Householder QR of Z in the Euclidean
 * product, Z = Y U (Y orthonormal, diag(U) > 0), then CHOLQR-A on Y in FP64,
 * Y = Q S, and R = S U.  Dense or stencil A.  info_dev as oqr_cholqr.  Q may
 * alias Z. */
int oqr_pre_cholqr(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n,
                   double* Q, int64_t ldq, double* R, int64_t ldr, const oqr_opts* opts,
                   void* ws, size_t ws_bytes, int32_t* info_dev, void* stream);

/* CHOL-EQR (Algorithm 3, Section 4), dense or tridiagonal A: C = chol(A)
 * upper (A = C^T C; upper bidiagonal for a tridiagonal A), W = C Z,
 * Householder [Y, R] = qr(W) with positive diag(R), Q = C^{-1} Y.
 * info_dev = k if the k-th pivot of chol(A) failed (no shift is applied to
 * A).  FP64 throughout.  Stencil operators: OQR_E_UNSUPPORTED. */
int oqr_chol_a(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n,
               double* Q, int64_t ldq, double* R, int64_t ldr, const oqr_opts* opts,
               void* ws, size_t ws_bytes, int32_t* info_dev, void* stream);

/* EQR-SYEV (Algorithm 4, Section 5), dense A only: A = V D V^T (cyclic
 * Jacobi), X = V^T Z, W = D^{1/2} X, [Y, R] = qr(W), U = D^{-1/2} Y, Q = V U.
 * info_dev = 1 if an eigenvalue is not positive, 2 if Jacobi did not
 * converge.  FP64 throughout. */
int oqr_eig_a(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n,
              double* Q, int64_t ldq, double* R, int64_t ldr, const oqr_opts* opts,
              void* ws, size_t ws_bytes, int32_t* info_dev, void* stream);

/* Gram-Schmidt in the A inner product (Section 6), variant opts->gs_variant.
 * info_dev = j if ||v_j||_A^2 was not positive at column j (1-based).  FP64. */
int oqr_gs(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n,
           double* Q, int64_t ldq, double* R, int64_t ldr, const oqr_opts* opts,
           void* ws, size_t ws_bytes, int32_t* info_dev, void* stream);

/* Generalised least squares (Section 1): X = R^{-1} Q^T A B, the minimiser of
 * ||Z x - b||_A for each column b of B, from an oblique QR (Q, R) of Z
 * computed by any of the entry points above.  B: m x k (ldb >= m), X: n x k
 * (ldx >= n), Q m x n, R n x n upper; all device memory, X must not overlap
 * B, Q or R.  FP64.  Returns OQR_E_ARG for bad sizes or pointers. */
size_t oqr_gls_workspace_bytes(const oqr_op* A, int64_t m, int64_t n, int64_t k);
int oqr_gls(const oqr_op* A, const double* Q, int64_t ldq, const double* R, int64_t ldr, int64_t m, int64_t n,
            const double* B, int64_t ldb, int64_t k, double* X, int64_t ldx, void* ws, size_t ws_bytes,
            void* stream);

/* Error measures of Section 7, computed on the device in FP64 (a report, not
 * a reference): out_dev[0] = ||I - Q^T A Q||_F (upper bound of the 2-norm
 * and within sqrt(n) of it), out_dev[1] = ||Z - Q R||_F / ||Z||_F. */
int oqr_check(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n,
              const double* Q, int64_t ldq, const double* R, int64_t ldr,
              void* ws, size_t ws_bytes, double* out_dev, void* stream);

/* One item of a batch (device memory).  a: dense A_i (column-major, lda);
 * z, q, r: Z_i, Q_i, R_i with their leading dimensions.  Storage type is the
 * batch's dtype.  q may alias z. */
typedef struct oqr_batch_item {
  const void* a;
  const void* z;
  void* q;
  void* r;
  int64_t lda, ldz, ldq, ldr;
  int32_t m, n;
} oqr_batch_item;

/* info_dev values of oqr_cholqr2_batched, one per instance: 0 success; k > 0 the
 * Cholesky of the Gram broke down at pivot k in spite of the allowed shifted
 * retries; OQR_BATCH_BAD_ITEM the item breaks the limits stated below, checked
 * on the device before anything of the instance is read or written. */
enum { OQR_BATCH_BAD_ITEM = -1 };

/* Workspace bytes for oqr_cholqr2_batched: a few int32 per instance plus the
 * partial Grams of up to min(batch, 512) cooperative instances (8 parts of
 * 32 KiB each), about 256 KiB per instance up to 128 MiB in all. */
size_t oqr_batched_workspace_bytes(int64_t batch, int32_t max_m, int32_t max_n, int32_t dtype);

/* Tuning of the batched launch.  Instances are classed by m (buckets
 * m < 512, < 1024, < 2048, < 4096, < 8192, >= 8192) and by n (n <= 8, <= 16,
 * <= 32, <= 64); each class runs the Gram phase with one tile shape:
 *   shape 0: row blocks of 128 rows, K steps of 32   shape 1: 64 x 32
 *   shape 2: 128 x 16                                shape 3: 64 x 16
 * Shapes change the grouping of the FP64 sums (not the arithmetic), so
 * results differ between shapes by rounding only.  wg_per_cu: 1..3
 * persistent workgroups per compute unit; sort: 1 = take instances largest
 * (m^2 n) first, 0 = in index order.  A table tuned on the caller's batch
 * comes from the binding's autotuner (it times the shapes class by class). */
#define OQR_BATCH_MBUCKETS 6
#define OQR_BATCH_NCLASSES 4
#define OQR_BATCH_SHAPES 4
typedef struct oqr_batch_tuning {
  int32_t wg_per_cu;
  int32_t sort;
  uint8_t shape[OQR_BATCH_MBUCKETS][OQR_BATCH_NCLASSES];
  /* Cooperative instances: with split_m > 0 (and sort = 1, batch <= 8192), up
   * to 512 of the largest instances with m >= split_m run each pass as `parts`
   * workgroups (1..8) over interleaved row blocks, their partial Grams summed
   * in part order by one workgroup that then factors and solves; the other
   * instances run in the persistent launch.  0 = no split. */
  int32_t split_m;
  int32_t parts;
} oqr_batch_tuning;

/* Fills *tuning with the built-in configuration (2 workgroups per compute
 * unit, sorted, shape 0 for every class, no split), used when NULL is passed. */
void oqr_batched_default_tuning(oqr_batch_tuning* tuning);

/* Batched CholQR2-A over `batch` independent dense instances in one
 * persistent launch: workgroups take instances from a device work queue
 * (largest first), each instance runs both passes inside one workgroup with
 * FP64 Gram accumulation, Cholesky (shift/retry as in opts) and substitution.
 * Cooperative instances (tuning split_m > 0) run before it in four staged
 * launches (Gram parts, then sum + Cholesky + substitution, for each pass).
 * items_dev: device array of `batch` items with 1 <= n_i <= max_n <= 64,
 * n_i <= m_i <= max_m, non-null pointers, lda >= m_i, ldz >= m_i, ldq >= m_i,
 * ldr >= n_i, and A_i, Z_i and Q_i each spanning at most 2^31 - 1 bytes
 * ((m_i - 1) lda + m_i elements, (n_i - 1) ldz + m_i, (n_i - 1) ldq + m_i);
 * an item outside these limits gets OQR_BATCH_BAD_ITEM.  dtype: OQR_F64 or
 * OQR_F32 (FP32 storage, widened to FP64 on load: every product, the Gram, the
 * Cholesky and the substitution are FP64; Q and R are rounded to FP32 on
 * store).  info_dev: `batch` int32, one per instance (values above).  Host
 * errors: OQR_E_ARG for batch, max_m, max_n, dtype, tuning or options out of
 * range; OQR_E_UNSUPPORTED for a precision other than FP64.  The call
 * allocates nothing and may be captured in a hipGraph.
 * tuning: host struct read during the call (NULL = oqr_batched_default_tuning). */
int oqr_cholqr2_batched(int64_t batch, const oqr_batch_item* items_dev, int32_t dtype,
                        int32_t max_m, int32_t max_n, const oqr_opts* opts,
                        const oqr_batch_tuning* tuning, void* ws, size_t ws_bytes,
                        int32_t* info_dev, void* stream);

/* Timing aid: from oqr_trace_start(name) until oqr_trace_stop, every launch
 * of the named kernel ("gemm_f64", "gemm_split", "gram", "chol", "trsm",
 * "stencil", "split_z", "batch", "symm_diag") made by this process is
 * bracketed by a pair of HIP
 * events recorded on its stream (events are created on first use and reused).
 * oqr_trace_stop waits for the recorded events and returns the summed kernel
 * time in milliseconds and the number of launches.  Not thread-safe; do not
 * trace while capturing a graph. */
int oqr_trace_start(const char* kernel);
int oqr_trace_stop(double* total_ms, int32_t* count);

/* Human-readable text for a status code. */
const char* oqr_status_string(int status);

/* ABI version (major*10000 + minor*100 + patch). */
int oqr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* OQR_H */
