// Baseline algorithms of the paper behind the same ABI, FP64, correctness first:
//   oqr_gs      Gram-Schmidt in the A inner product (Section 6): CGS, MGS row/column oriented
//               (the two implementations of Section 8's comments), CGS2;
//   oqr_chol_a  CHOL-EQR (Algorithm 3, Section 4): blocked Cholesky of A, W = C Z, Householder QR
//               of W, Q = C^{-1} Y;
//   oqr_eig_a   EQR-SYEV (Algorithm 4, Section 5): cyclic two-sided Jacobi A = V D V^T (parallel
//               round-robin ordering), X = V^T Z, W = D^{1/2} X, Householder QR, Q = V D^{-1/2} Y.
// The level-2 and level-1 pieces are small generic kernels launched per column; the O(m^2 n) and
// O(m^3) products run on the FP64 MFMA kernels of the hot path where they fit.
#include "common.hpp"

#include <climits>
#include <math.h>

namespace oqr {
namespace {

constexpr int NT = 256;
constexpr int CH = 2048;          // rows per chunk of a column reduction

#define OQR_TRY(expr)                       \
  do {                                      \
    hipError_t e_ = (expr);                 \
    if (e_ != hipSuccess) return OQR_E_HIP; \
  } while (0)

__device__ double block_sum256(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  return s;
}

// ---- generic column kernels ------------------------------------------------------------------

// partial[ch * nc + c] = sum over rows of chunk ch of X(i, c) * Y(i, c or 0)
__global__ __launch_bounds__(NT) void colsdot_kernel(const double* __restrict__ X, int64_t ldx,
                                                      const double* __restrict__ Y, int64_t ldy, int ycols,
                                                      int m, int nc, double* __restrict__ partial,
                                                      const int32_t* __restrict__ info) {
  __shared__ double red[NT / 64];
  if (info && info[0]) return;
  const int c = blockIdx.y, ch = blockIdx.x;
  const int r0 = ch * CH, r1 = min(m, r0 + CH);
  const double* x = X + (int64_t)c * ldx;
  const double* y = Y + (int64_t)(ycols ? c : 0) * ldy;
  double s = 0.0;
  for (int i = r0 + threadIdx.x; i < r1; i += NT) s += x[i] * y[i];
  s = block_sum256(s, red);
  if (threadIdx.x == 0) partial[(int64_t)ch * nc + c] = s;
}

// out[c * ostride] = alpha * sum_ch partial[ch * nc + c] (chunk order)
__global__ void chunks_sum_kernel(const double* __restrict__ partial, int nch, int nc, double alpha,
                                  double* __restrict__ out, int64_t ostride, const int32_t* __restrict__ info) {
  if (info && info[0]) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  double s = 0.0;
  for (int ch = 0; ch < nch; ++ch) s += partial[(int64_t)ch * nc + c];
  out[(int64_t)c * ostride] = alpha * s;
}

hipError_t cols_dot(const double* X, int64_t ldx, const double* Y, int64_t ldy, int ycols, int m, int nc,
                    double* partial, double* out, int64_t ostride, double alpha, const int32_t* info,
                    hipStream_t s) {
  if (nc <= 0) return hipSuccess;
  const int nch = ceil_div(m, CH);
  colsdot_kernel<<<dim3(nch, nc), NT, 0, s>>>(X, ldx, Y, ldy, ycols, m, nc, partial, info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  chunks_sum_kernel<<<ceil_div(nc, 256), 256, 0, s>>>(partial, nch, nc, alpha, out, ostride, info);
  return hipGetLastError();
}

// y = A x for dense A: partial over column chunks, then summed in chunk order.
constexpr int GKC = 1024;
__global__ __launch_bounds__(NT) void gemv_partial_kernel(const double* __restrict__ A, int64_t lda,
                                                           const double* __restrict__ x, int m,
                                                           double* __restrict__ partial,
                                                           const int32_t* __restrict__ info) {
  if (info && info[0]) return;
  const int i = blockIdx.x * NT + threadIdx.x;
  const int k0 = blockIdx.y * GKC, k1 = min(m, k0 + GKC);
  if (i >= m) return;
  double s = 0.0;
  for (int k = k0; k < k1; ++k) s += A[(int64_t)k * lda + i] * x[k];
  partial[(int64_t)blockIdx.y * m + i] = s;
}
__global__ void vec_chunks_sum_kernel(const double* __restrict__ partial, int nch, int m, double* __restrict__ y,
                                      const int32_t* __restrict__ info) {
  if (info && info[0]) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += partial[(int64_t)c * m + i];
  y[i] = s;
}

// v = z - X r  (X: m x j, r on the device, contiguous)
__global__ void sub_matvec_kernel(const double* __restrict__ z, const double* __restrict__ X, int64_t ldx,
                                  const double* __restrict__ r, int j, int m, double* __restrict__ v,
                                  const int32_t* __restrict__ info) {
  if (info && info[0]) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double s = z[i];
  for (int k = 0; k < j; ++k) s -= X[(int64_t)k * ldx + i] * r[k];
  v[i] = s;
}

// rjj = sqrt(vAv[0]); q = v / rjj; info = col + 1 when vAv is not positive
__global__ void normalize_kernel(const double* __restrict__ v, const double* __restrict__ vav, int m,
                                 double* __restrict__ q, double* __restrict__ rjj, int col,
                                 int32_t* __restrict__ info) {
  if (info[0]) return;
  const double d = vav[0];
  if (!(d > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) info[0] = col + 1;
    return;
  }
  const double r = sqrt(d);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) q[i] = v[i] / r;
  if (blockIdx.x == 0 && threadIdx.x == 0) rjj[0] = r;
}

// V(:, c) -= q * r[c * rstride] for c in [0, nc)
__global__ void rank1_sub_kernel(double* __restrict__ V, int64_t ldv, const double* __restrict__ q,
                                 const double* __restrict__ r, int64_t rstride, int m, int nc,
                                 const int32_t* __restrict__ info) {
  if (info && info[0]) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * nc) return;
  const int c = (int)(idx / m), i = (int)(idx % m);
  V[(int64_t)c * ldv + i] -= q[i] * r[(int64_t)c * rstride];
}

// v -= r0 * q  (r0 on the device)
__global__ void axpy_dev_kernel(double* __restrict__ v, const double* __restrict__ q, const double* __restrict__ r0,
                                int m, const int32_t* __restrict__ info) {
  if (info && info[0]) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) v[i] -= r0[0] * q[i];
}

__global__ void add_vec_kernel(double* __restrict__ a, const double* __restrict__ b, int n,
                               const int32_t* __restrict__ info) {
  if (info && info[0]) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] += b[i];
}

__global__ void zero_matrix_kernel(double* __restrict__ X, int64_t ldx, int m, int n) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * n) return;
  X[(idx / m) * ldx + idx % m] = 0.0;
}

hipError_t zero_matrix(double* X, int64_t ldx, int m, int n, hipStream_t s) {
  const int64_t total = (int64_t)m * n;
  if (!total) return hipSuccess;
  zero_matrix_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(X, ldx, m, n);
  return hipGetLastError();
}

// ---- the operator on one vector ----------------------------------------------------------------

struct OpCtx {
  const oqr_op* A;
  int m;
  double* gemv_partial;    // ceil(m / GKC) * m doubles (dense)
};

hipError_t apply_vec(const OpCtx& op, const double* x, double* y, const int32_t* info, hipStream_t s) {
  if (op.A->kind != OQR_OP_DENSE) return launch_sparse_apply(op.A, x, op.m, y, op.m, 1, s);
  const int nch = ceil_div(op.m, GKC);
  gemv_partial_kernel<<<dim3(ceil_div(op.m, NT), nch), NT, 0, s>>>((const double*)op.A->a, op.A->lda, x, op.m,
                                                                  op.gemv_partial, info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  vec_chunks_sum_kernel<<<ceil_div(op.m, 256), 256, 0, s>>>(op.gemv_partial, nch, op.m, y, info);
  return hipGetLastError();
}

// ---- Householder QR of a tall-skinny W (m x n, in place) --------------------------------------
// LAPACK convention: H_j = I - tau_j v_j v_j^T, v_j(j) = 1, v_j stored below the diagonal of W.

__global__ __launch_bounds__(1024) void hh_gen_kernel(double* __restrict__ W, int64_t ldw, int m, int j,
                                                       double* __restrict__ tau) {
  __shared__ double red[16];
  double* x = W + (int64_t)j * ldw;
  double s = 0.0;
  for (int i = j + 1 + threadIdx.x; i < m; i += 1024) s += x[i] * x[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  double sig = 0.0;
  for (int w = 0; w < 16; ++w) sig += red[w];
  const double x0 = x[j];
  __syncthreads();
  if (sig == 0.0) {                 // already upper triangular in this column: H = I
    if (threadIdx.x == 0) tau[j] = 0.0;
    return;
  }
  const double nrm = sqrt(x0 * x0 + sig);
  const double beta = (x0 >= 0.0) ? -nrm : nrm;
  const double scale = 1.0 / (x0 - beta);
  for (int i = j + 1 + threadIdx.x; i < m; i += 1024) x[i] *= scale;
  if (threadIdx.x == 0) {
    tau[j] = (beta - x0) / beta;
    x[j] = beta;
  }
}

// Apply H_j to columns [c0, c0 + gridDim.x) of C (rows j..m-1): c := c - tau (v^T c) v.
__global__ __launch_bounds__(NT) void hh_apply_kernel(const double* __restrict__ Wv, int64_t ldw, int m, int j,
                                                       const double* __restrict__ tau, double* __restrict__ C,
                                                       int64_t ldc, int c0) {
  __shared__ double red[NT / 64];
  const int c = c0 + blockIdx.x;
  const double t = tau[j];
  if (t == 0.0) return;
  const double* v = Wv + (int64_t)j * ldw;
  double* col = C + (int64_t)c * ldc;
  double s = (threadIdx.x == 0) ? col[j] : 0.0;
  for (int i = j + 1 + threadIdx.x; i < m; i += NT) s += v[i] * col[i];
  s = block_sum256(s, red);
  const double ts = t * s;
  if (threadIdx.x == 0) col[j] -= ts;
  for (int i = j + 1 + threadIdx.x; i < m; i += NT) col[i] -= ts * v[i];
}

// Y = [I_n; 0] (m x n)
__global__ void eye_kernel(double* __restrict__ Y, int64_t ldy, int m, int n) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * n) return;
  const int c = (int)(idx / m), i = (int)(idx % m);
  Y[(int64_t)c * ldy + i] = (i == c) ? 1.0 : 0.0;
}

// R = sign-fixed upper triangle of W; Y(:, c) *= sign(R_cc)
__global__ void hh_finish_kernel(const double* __restrict__ W, int64_t ldw, int m, int n, double* __restrict__ R,
                                 int64_t ldr, double* __restrict__ Y, int64_t ldy) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (int64_t)n * n) {
    const int c = (int)(idx / n), i = (int)(idx % n);
    const double sg = (W[(int64_t)i * ldw + i] < 0.0) ? -1.0 : 1.0;
    R[(int64_t)c * ldr + i] = (i <= c) ? sg * W[(int64_t)c * ldw + i] : 0.0;
  }
  if (idx < (int64_t)m * n) {
    const int c = (int)(idx / m), i = (int)(idx % m);
    const double sg = (W[(int64_t)c * ldw + c] < 0.0) ? -1.0 : 1.0;
    Y[(int64_t)c * ldy + i] *= sg;
  }
}

// Householder QR: W (m x n) is overwritten by the reflectors; R (n x n) and Y (m x n) with
// positive diag(R) are returned.  tau: n doubles.
hipError_t householder_qr(double* W, int64_t ldw, int m, int n, double* tau, double* R, int64_t ldr, double* Y,
                          int64_t ldy, hipStream_t s) {
  for (int j = 0; j < n; ++j) {
    hh_gen_kernel<<<1, 1024, 0, s>>>(W, ldw, m, j, tau);
    if (j + 1 < n) hh_apply_kernel<<<n - j - 1, NT, 0, s>>>(W, ldw, m, j, tau, W, ldw, j + 1);
  }
  const int64_t total = (int64_t)m * n;
  eye_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(Y, ldy, m, n);
  for (int j = n - 1; j >= 0; --j) hh_apply_kernel<<<n - j, NT, 0, s>>>(W, ldw, m, j, tau, Y, ldy, j);
  hh_finish_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(W, ldw, m, n, R, ldr, Y, ldy);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_householder_qr(double* W, int64_t ldw, int64_t m, int64_t n, double* tau, double* R, int64_t ldr,
                                 double* Y, int64_t ldy, hipStream_t s) {
  return householder_qr(W, ldw, (int)m, (int)n, tau, R, ldr, Y, ldy, s);
}

// =================================================================================================
// Gram-Schmidt in the A inner product
// =================================================================================================

size_t gs_workspace_bytes(const oqr_op* A, int64_t m, int64_t n) {
  size_t b = 0;
  b += align256((size_t)ceil_div(m, GKC) * m * sizeof(double));     // gemv partials
  b += align256((size_t)ceil_div(m, CH) * (n > 0 ? n : 1) * sizeof(double));   // column-dot partials
  b += align256((size_t)m * n * sizeof(double));                    // V (MGS working copy)
  b += align256((size_t)m * sizeof(double)) * 3;                    // p, w, v
  b += align256((size_t)(n + 8) * sizeof(double)) * 2;              // r scratch, scalars
  (void)A;
  return b;
}

int gs_run(const oqr_op* A, const double* Z, int64_t ldz, int64_t m64, int64_t n64, double* Q, int64_t ldq,
           double* R, int64_t ldr, int variant, void* ws, int32_t* info, hipStream_t s) {
  const int m = (int)m64, n = (int)n64;
  char* p = (char*)ws;
  auto take = [&](size_t bytes) {
    char* r = p;
    p += align256(bytes);
    return (double*)r;
  };
  OpCtx op{A, m, take((size_t)ceil_div(m, GKC) * m * sizeof(double))};
  double* part = take((size_t)ceil_div(m, CH) * n * sizeof(double));
  double* V = take((size_t)m * n * sizeof(double));
  double* pv = take((size_t)m * sizeof(double));
  double* wv = take((size_t)m * sizeof(double));
  double* vv = take((size_t)m * sizeof(double));
  double* rs = take((size_t)(n + 8) * sizeof(double));
  double* sc = take((size_t)(n + 8) * sizeof(double));
  const int gb = ceil_div(m, 256);
  OQR_TRY(zero_matrix(R, ldr, n, n, s));

  // ||v||_A^2 -> sc[0]; then q_j = v / sqrt(sc[0]), R_jj
  auto finish_column = [&](const double* v, int j) -> int {
    OQR_TRY(apply_vec(op, v, wv, info, s));
    OQR_TRY(cols_dot(v, m, wv, m, 0, m, 1, part, sc, 1, 1.0, info, s));
    normalize_kernel<<<gb, 256, 0, s>>>(v, sc, m, Q + (int64_t)j * ldq, R + (int64_t)j * ldr + j, j, info);
    OQR_TRY(hipGetLastError());
    return OQR_OK;
  };

  if (variant == OQR_GS_CGS || variant == OQR_GS_CGS2) {
    const int rounds = (variant == OQR_GS_CGS2) ? 2 : 1;
    for (int j = 0; j < n; ++j) {
      const double* zj = Z + (int64_t)j * ldz;
      if (j == 0) {
        OQR_TRY(hipMemcpyAsync(vv, zj, (size_t)m * sizeof(double), hipMemcpyDeviceToDevice, s));
      } else if (variant == OQR_GS_CGS) {
        // r_{1:j-1,j} = Q^T (A z_j); v = z_j - Q r
        OQR_TRY(apply_vec(op, zj, pv, info, s));
        OQR_TRY(cols_dot(Q, ldq, pv, m, 0, m, j, part, R + (int64_t)j * ldr, 1, 1.0, info, s));
        sub_matvec_kernel<<<gb, 256, 0, s>>>(zj, Q, ldq, R + (int64_t)j * ldr, j, m, vv, info);
        OQR_TRY(hipGetLastError());
      } else {
        OQR_TRY(hipMemcpyAsync(vv, zj, (size_t)m * sizeof(double), hipMemcpyDeviceToDevice, s));
        for (int rd = 0; rd < rounds; ++rd) {
          // h = Q^T (A v); v -= Q h; r += h
          OQR_TRY(apply_vec(op, vv, pv, info, s));
          OQR_TRY(cols_dot(Q, ldq, pv, m, 0, m, j, part, rs, 1, 1.0, info, s));
          sub_matvec_kernel<<<gb, 256, 0, s>>>(vv, Q, ldq, rs, j, m, wv, info);
          OQR_TRY(hipGetLastError());
          OQR_TRY(hipMemcpyAsync(vv, wv, (size_t)m * sizeof(double), hipMemcpyDeviceToDevice, s));
          add_vec_kernel<<<ceil_div(j, 256), 256, 0, s>>>(R + (int64_t)j * ldr, rs, j, info);
          OQR_TRY(hipGetLastError());
        }
      }
      if (int rc = finish_column(vv, j)) return rc;
    }
    return OQR_OK;
  }
  if (variant == OQR_GS_MGS_ROW) {
    // V = Z; for i: q_i = v_i / ||v_i||_A; p = A q_i; r_{i,i+1:} = p^T V(:, i+1:); V(:, i+1:) -= q_i r
    for (int c = 0; c < n; ++c)
      OQR_TRY(hipMemcpyAsync(V + (int64_t)c * m, Z + (int64_t)c * ldz, (size_t)m * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
    for (int i = 0; i < n; ++i) {
      if (int rc = finish_column(V + (int64_t)i * m, i)) return rc;
      const int rest = n - i - 1;
      if (!rest) break;
      OQR_TRY(apply_vec(op, Q + (int64_t)i * ldq, pv, info, s));
      OQR_TRY(cols_dot(V + (int64_t)(i + 1) * m, m, pv, m, 0, m, rest, part, R + (int64_t)(i + 1) * ldr + i, ldr, 1.0,
                       info, s));
      const int64_t tot = (int64_t)m * rest;
      rank1_sub_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(V + (int64_t)(i + 1) * m, m, Q + (int64_t)i * ldq,
                                                                     R + (int64_t)(i + 1) * ldr + i, ldr, m, rest, info);
      OQR_TRY(hipGetLastError());
    }
    return OQR_OK;
  }
  // MGS_COL: for j: v = z_j; for i < j: r_ij = q_i^T (A v); v -= r_ij q_i; then normalise
  for (int j = 0; j < n; ++j) {
    OQR_TRY(hipMemcpyAsync(vv, Z + (int64_t)j * ldz, (size_t)m * sizeof(double), hipMemcpyDeviceToDevice, s));
    for (int i = 0; i < j; ++i) {
      OQR_TRY(apply_vec(op, vv, pv, info, s));
      OQR_TRY(cols_dot(Q + (int64_t)i * ldq, ldq, pv, m, 0, m, 1, part, R + (int64_t)j * ldr + i, 1, 1.0, info, s));
      axpy_dev_kernel<<<gb, 256, 0, s>>>(vv, Q + (int64_t)i * ldq, R + (int64_t)j * ldr + i, m, info);
      OQR_TRY(hipGetLastError());
    }
    if (int rc = finish_column(vv, j)) return rc;
  }
  return OQR_OK;
}

// =================================================================================================
// Generalised least squares (Section 1): X = R^{-1} Q^T (A B)
// =================================================================================================
namespace {
// X(:, c) = R^{-1} Y(:, c) by back-substitution, one thread per right-hand side.
__global__ void back_subst_kernel(const double* __restrict__ R, int64_t ldr, int n, const double* __restrict__ Y,
                                  int k, double* __restrict__ X, int64_t ldx) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  const double* y = Y + (int64_t)c * n;
  double* x = X + (int64_t)c * ldx;
  for (int i = n - 1; i >= 0; --i) {
    double s = y[i];
    for (int j = i + 1; j < n; ++j) s -= R[(int64_t)j * ldr + i] * x[j];
    x[i] = s / R[(int64_t)i * ldr + i];
  }
}
}  // namespace

size_t gls_workspace_bytes(const oqr_op* A, int64_t m, int64_t n, int64_t k) {
  (void)A;
  return align256((size_t)m * k * sizeof(double)) + align256((size_t)n * k * sizeof(double)) +
         align256((size_t)ceil_div(m, CH) * n * sizeof(double));
}

int gls_run(const oqr_op* A, const double* Q, int64_t ldq, const double* R, int64_t ldr, int64_t m64, int64_t n64,
            const double* B, int64_t ldb, int64_t k64, double* X, int64_t ldx, void* ws, hipStream_t s) {
  const int m = (int)m64, n = (int)n64, k = (int)k64;
  char* p = (char*)ws;
  double* Wb = (double*)p;
  p += align256((size_t)m * k * sizeof(double));
  double* Y = (double*)p;
  p += align256((size_t)n * k * sizeof(double));
  double* part = (double*)p;
  // W = A B
  if (A->kind != OQR_OP_DENSE) {
    OQR_TRY(launch_sparse_apply(A, B, ldb, Wb, m, k, s));
  } else {
    OQR_TRY(launch_gemm_f64((const double*)A->a, A->lda, B, ldb, Wb, m, m, k, nullptr, s));
  }
  // Y = Q^T W, column by column (chunked dot products summed in chunk order)
  for (int c = 0; c < k; ++c)
    OQR_TRY(cols_dot(Q, ldq, Wb + (int64_t)c * m, m, 0, m, n, part, Y + (int64_t)c * n, 1, 1.0, nullptr, s));
  back_subst_kernel<<<ceil_div(k, 64), 64, 0, s>>>(R, ldr, n, Y, k, X, ldx);
  OQR_TRY(hipGetLastError());
  return OQR_OK;
}

// =================================================================================================
// CHOL-EQR: C = chol(A) (blocked, upper), W = C Z, [Y, R] = qr(W), Q = C^{-1} Y
// =================================================================================================
namespace {

constexpr int PB = 64;    // panel width of the blocked Cholesky of A and of the block back-substitution

// Panel solve: rows k0..k0+kb-1 of C, columns [k0+kb, m): X = R_kk^{-T} X (forward substitution),
// one thread per column; R_kk (upper) staged in LDS.
__global__ __launch_bounds__(NT) void panel_solve_kernel(double* __restrict__ C, int64_t ldc, int m, int k0, int kb,
                                                          const int32_t* __restrict__ info) {
  __shared__ double Rk[PB][PB + 1];
  if (info[0]) return;
  for (int e = threadIdx.x; e < PB * PB; e += NT) {
    const int i = e % PB, j = e / PB;
    Rk[i][j] = (i < kb && j < kb) ? C[(int64_t)(k0 + j) * ldc + k0 + i] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  const int col = k0 + kb + blockIdx.x * NT + threadIdx.x;
  if (col >= m) return;
  double* x = C + (int64_t)col * ldc + k0;
  for (int p = 0; p < kb; ++p) {
    double a = x[p];
    for (int q = 0; q < p; ++q) a -= Rk[q][p] * x[q];
    x[p] = a / Rk[p][p];
  }
}

// Trailing update of the upper 64x64 tiles (I <= J) of C[k1:m, k1:m] -= P^T P, P = C[k0:k1, k1:m].
__global__ __launch_bounds__(NT) void syrk_update_kernel(double* __restrict__ C, int64_t ldc, int m, int k0, int kb,
                                                          const int32_t* __restrict__ info) {
  if (info[0]) return;
  const int k1 = k0 + kb;
  const int nbt = (m - k1 + 63) / 64;
  int t = blockIdx.x, I = 0;
  while (t >= nbt - I) { t -= nbt - I; ++I; }
  const int J = I + t;
  const int I0 = k1 + 64 * I, J0 = k1 + 64 * J;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane >> 4, lj = lane & 15;
  f64x4 acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = I0 + wave * 16 + 4 * r + li, j = J0 + b * 16 + lj;
      acc[b][r] = (i < m && j < m) ? C[(int64_t)j * ldc + i] : 0.0;
    }
  for (int kk = 0; kk < kb; kk += 4) {
    const int row = k0 + kk + li;
    const int ca = I0 + wave * 16 + lj;
    const double a = (row < k1 && ca < m) ? -C[(int64_t)ca * ldc + row] : 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int cb = J0 + b * 16 + lj;
      const double bv = (row < k1 && cb < m) ? C[(int64_t)cb * ldc + row] : 0.0;
      acc[b] = mfma_f64(a, bv, acc[b]);
    }
  }
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = I0 + wave * 16 + 4 * r + li, j = J0 + b * 16 + lj;
      if (i < m && j < m && i <= j) C[(int64_t)j * ldc + i] = acc[b][r];
    }
}

// Unblocked Cholesky of the diagonal block C[k0:k0+kb, k0:k0+kb] (upper, in place) in LDS;
// info = k0 + k + 1 on the first non-positive (or NaN) pivot k.
__global__ __launch_bounds__(NT) void chol_diag_kernel(double* __restrict__ C, int64_t ldc, int k0, int kb,
                                                        int32_t* __restrict__ info) {
  __shared__ double L[PB][PB + 1];
  if (info[0]) return;
  for (int e = threadIdx.x; e < PB * PB; e += NT) {
    const int i = e % PB, j = e / PB;
    L[i][j] = (i <= j && j < kb) ? C[(int64_t)(k0 + j) * ldc + k0 + i] : 0.0;
  }
  for (int k = 0; k < kb; ++k) {
    __syncthreads();
    const double d = L[k][k];
    if (!(d > 0.0)) {                  // uniform: every thread read the same pivot
      if (threadIdx.x == 0) info[0] = k0 + k + 1;
      return;
    }
    const double r = sqrt(d);
    __syncthreads();
    for (int j = k + 1 + threadIdx.x; j < kb; j += NT) L[k][j] /= r;
    if (threadIdx.x == 0) L[k][k] = r;
    __syncthreads();
    const int w = kb - k - 1;
    for (int e = threadIdx.x; e < w * w; e += NT) {
      const int i = k + 1 + e % w, j = k + 1 + e / w;
      if (i <= j) L[i][j] -= L[k][i] * L[k][j];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < PB * PB; e += NT) {
    const int i = e % PB, j = e / PB;
    if (i <= j && j < kb) C[(int64_t)(k0 + j) * ldc + k0 + i] = L[i][j];
  }
}

__global__ void copy_upper_kernel(const double* __restrict__ A, int64_t lda, double* __restrict__ C, int64_t ldc,
                                  int m) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * m) return;
  const int j = (int)(idx / m), i = (int)(idx % m);
  C[(int64_t)j * ldc + i] = (i <= j) ? A[(int64_t)j * lda + i] : 0.0;
}

// Back-substitution C X = Y for upper C (m x m), n right-hand sides, block row [b0, b0 + bb):
// X_b = C_bb^{-1} (Y_b - C_{b, b0+bb:} X_{b0+bb:}); one workgroup per 64-column block of X.
__global__ __launch_bounds__(NT) void back_block_kernel(const double* __restrict__ C, int64_t ldc, int m, int b0,
                                                         int bb, double* __restrict__ X, int64_t ldx, int n,
                                                         const int32_t* __restrict__ info) {
  __shared__ double Acc[PB][PB + 1];    // [row of block][column of X block]
  __shared__ double Cb[PB][PB + 1];
  if (info[0]) return;
  const int c0 = blockIdx.x * 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane >> 4, lj = lane & 15;
  f64x4 acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = b0 + wave * 16 + 4 * r + li, c = c0 + b * 16 + lj;
      acc[b][r] = (i < b0 + bb && c < n) ? X[(int64_t)c * ldx + i] : 0.0;
    }
  const int e0 = b0 + bb;
  for (int k = e0; k < m; k += 4) {
    const int kr = k + li;
    const int ra = b0 + wave * 16 + lj;
    const double a = (kr < m && ra < b0 + bb) ? -C[(int64_t)kr * ldc + ra] : 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int c = c0 + b * 16 + lj;
      const double bv = (kr < m && c < n) ? X[(int64_t)c * ldx + kr] : 0.0;
      acc[b] = mfma_f64(a, bv, acc[b]);
    }
  }
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) Acc[wave * 16 + 4 * r + li][b * 16 + lj] = acc[b][r];
  for (int e = threadIdx.x; e < PB * PB; e += NT) {
    const int i = e % PB, j = e / PB;
    Cb[i][j] = (i < bb && j < bb) ? C[(int64_t)(b0 + j) * ldc + b0 + i] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  const int c = threadIdx.x;             // one thread per column of the block
  if (c < 64 && c0 + c < n) {
    for (int p = bb - 1; p >= 0; --p) {
      double a = Acc[p][c];
      for (int q = p + 1; q < bb; ++q) a -= Cb[p][q] * Acc[q][c];
      Acc[p][c] = a / Cb[p][p];
    }
    for (int p = 0; p < bb; ++p) X[(int64_t)(c0 + c) * ldx + b0 + p] = Acc[p][c];
  }
}

}  // namespace


size_t chol_a_workspace_bytes(int64_t m, int64_t n) {
  size_t b = 0;
  b += align256((size_t)m * m * sizeof(double));   // C
  b += align256((size_t)m * n * sizeof(double));   // W
  b += align256(euclid_qr_ws_bytes(m, n));         // the Euclidean QR
  return b;
}

int chol_a_run(const oqr_op* A, const double* Z, int64_t ldz, int64_t m64, int64_t n64, double* Q, int64_t ldq,
               double* R, int64_t ldr, void* ws, int32_t* info, hipStream_t s) {
  const int m = (int)m64, n = (int)n64;
  char* p = (char*)ws;
  double* C = (double*)p;
  p += align256((size_t)m * m * sizeof(double));
  double* W = (double*)p;
  p += align256((size_t)m * n * sizeof(double));
  void* qr_ws = p;
  const int64_t mm = (int64_t)m * m;
  copy_upper_kernel<<<(unsigned)((mm + 255) / 256), 256, 0, s>>>((const double*)A->a, A->lda, C, m, m);
  OQR_TRY(hipGetLastError());
  // blocked right-looking Cholesky, upper: C = chol(A)
  for (int k0 = 0; k0 < m; k0 += PB) {
    const int kb = min(PB, m - k0);
    chol_diag_kernel<<<1, NT, 0, s>>>(C, m, k0, kb, info);
    OQR_TRY(hipGetLastError());
    const int rest = m - k0 - kb;
    if (rest <= 0) break;
    panel_solve_kernel<<<ceil_div(rest, NT), NT, 0, s>>>(C, m, m, k0, kb, info);
    OQR_TRY(hipGetLastError());
    const int nbt = ceil_div(rest, 64);
    syrk_update_kernel<<<nbt * (nbt + 1) / 2, NT, 0, s>>>(C, m, m, k0, kb, info);
    OQR_TRY(hipGetLastError());
  }
  // W = C Z  (C upper, zero below the diagonal)
  OQR_TRY(launch_gemm_f64(C, m, Z, ldz, W, m, m, n, nullptr, s));
  // [Y, R] = qr(W): Y goes to Q
  OQR_TRY(launch_euclid_qr(W, m, m, n, qr_ws, R, ldr, Q, ldq, s));
  // Q = C^{-1} Y (block back-substitution from the bottom)
  const int nb = ceil_div(m, PB);
  for (int b = nb - 1; b >= 0; --b) {
    const int b0 = b * PB, bb = min(PB, m - b0);
    back_block_kernel<<<ceil_div(n, 64), NT, 0, s>>>(C, m, m, b0, bb, Q, ldq, n, info);
    OQR_TRY(hipGetLastError());
  }
  return OQR_OK;
}

// =================================================================================================
// CHOL-EQR for a tridiagonal A: C upper bidiagonal (c_i on the diagonal, f_i above), A = C^T C
// =================================================================================================
namespace {

// Pivots of the tridiagonal Cholesky (LDL^T form): p_0 = d_0, p_i = d_i - e_{i-1}^2 / p_{i-1}.  The
// recurrence is evaluated in chunks of TK pivots: each map p -> d - e^2 / p is the 2 x 2 matrix
// [d, -e^2; 1, 0] acting on homogeneous (x, y) with p = x / y, so (1) every chunk forms the product of
// its maps (one wave per chunk, a product tree over the lanes), (2) one workgroup scans these products
// to the homogeneous start value of every chunk, (3) every chunk runs the recurrence itself from its
// start.  Products are rescaled by powers of two (exact).  info = first pivot (1-based) that is not
// positive.
constexpr int TK = 256;
constexpr int SCAN_NT = 1024;

struct M2 {
  double a, b, c, d;   // [a b; c d]
};

__device__ __forceinline__ M2 m2_mul(const M2& x, const M2& y) {   // x * y
  return {fma(x.a, y.a, x.b * y.c), fma(x.a, y.b, x.b * y.d), fma(x.c, y.a, x.d * y.c), fma(x.c, y.b, x.d * y.d)};
}

__device__ __forceinline__ M2 m2_norm(M2 x) {
  const double mx = fmax(fmax(fabs(x.a), fabs(x.b)), fmax(fabs(x.c), fabs(x.d)));
  if (mx == 0.0 || !isfinite(mx)) return x;
  const int ex = ilogb(mx);
  return {ldexp(x.a, -ex), ldexp(x.b, -ex), ldexp(x.c, -ex), ldexp(x.d, -ex)};
}

__device__ __forceinline__ M2 m2_shfl_down(const M2& x, int o) {
  return {__shfl_down(x.a, o), __shfl_down(x.b, o), __shfl_down(x.c, o), __shfl_down(x.d, o)};
}

// F[k] = M_{s+TK} ... M_{s+1} for chunk k (s = k TK), k < nch - 1.  One wave per chunk; lane l owns
// maps s + 1 + 4l .. s + 4 + 4l.
__global__ __launch_bounds__(64) void tridiag_chunk_maps_kernel(const double* __restrict__ t, int m, int nch,
                                                                double* __restrict__ F,
                                                                const int32_t* __restrict__ info) {
  const int k = blockIdx.x, l = threadIdx.x;
  if (info[0] || k >= nch - 1) return;
  const int i0 = k * TK + 1 + 4 * l;   // <= m - 1: chunk k + 1 exists
  M2 P = {1.0, 0.0, 0.0, 1.0};
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const double di = t[i0 + u], e = t[m + i0 + u - 1];
    P = m2_norm(m2_mul({di, -e * e, 1.0, 0.0}, P));
  }
  // ordered product over the lanes: later lanes on the left
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const M2 Q = m2_shfl_down(P, o);
    if ((l & (2 * o - 1)) == 0) P = m2_norm(m2_mul(Q, P));
  }
  if (l == 0) {
    F[4 * k] = P.a;
    F[4 * k + 1] = P.b;
    F[4 * k + 2] = P.c;
    F[4 * k + 3] = P.d;
  }
}

// xy[k] = homogeneous start of chunk k: (F_{k-1} ... F_0)(d_0, 1).  One workgroup: each thread composes
// a run of chunk maps, a scan over the threads in LDS gives every run its prefix, the runs are then
// walked again.
__global__ __launch_bounds__(SCAN_NT) void tridiag_chunk_starts_kernel(const double* __restrict__ t, int nch,
                                                                      const double* __restrict__ F,
                                                                      double* __restrict__ xy,
                                                                      const int32_t* __restrict__ info) {
  __shared__ M2 S[SCAN_NT];
  if (info[0]) return;
  const int tid = threadIdx.x;
  const int per = (nch + SCAN_NT - 1) / SCAN_NT;
  const int k0 = min(nch, tid * per), k1 = min(nch, k0 + per);
  auto fmap = [&](int k) -> M2 {   // the map from chunk k's start to chunk k + 1's start
    if (k >= nch - 1) return {1.0, 0.0, 0.0, 1.0};
    return {F[4 * k], F[4 * k + 1], F[4 * k + 2], F[4 * k + 3]};
  };
  M2 G = {1.0, 0.0, 0.0, 1.0};
  for (int k = k0; k < k1; ++k) G = m2_norm(m2_mul(fmap(k), G));
  S[tid] = G;
  __syncthreads();
  for (int o = 1; o < SCAN_NT; o <<= 1) {
    M2 v = S[tid];
    if (tid >= o) v = m2_norm(m2_mul(v, S[tid - o]));
    __syncthreads();
    S[tid] = v;
    __syncthreads();
  }
  double x = t[0], y = 1.0;
  if (tid > 0) {
    const M2 E = S[tid - 1];
    const double nx = fma(E.a, x, E.b * y), ny = fma(E.c, x, E.d * y);
    x = nx;
    y = ny;
  }
  for (int k = k0; k < k1; ++k) {
    xy[2 * k] = x;
    xy[2 * k + 1] = y;
    const M2 Fk = fmap(k);
    double nx = fma(Fk.a, x, Fk.b * y), ny = fma(Fk.c, x, Fk.d * y);
    const double mx = fmax(fabs(nx), fabs(ny));
    if (mx != 0.0 && isfinite(mx)) {
      const int ex = ilogb(mx);
      nx = ldexp(nx, -ex);
      ny = ldexp(ny, -ex);
    }
    x = nx;
    y = ny;
  }
}

__global__ void tridiag_chunk_pivots_kernel(const double* __restrict__ t, int m, int nch,
                                            const double* __restrict__ xy, double* __restrict__ p,
                                            int32_t* __restrict__ fail, const int32_t* __restrict__ info) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (info[0] || k >= nch) return;
  const int s0 = k * TK, s1 = min(m, s0 + TK);
  double pi = xy[2 * k] / xy[2 * k + 1];
  int32_t f = 0;
  for (int i0 = s0; i0 < s1 && !f; i0 += 16) {
    double dn[16], en[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {   // d_{i+1}, e_i (clamped into the array; used only when i + 1 < m)
      const int i = (m >= 2) ? min(i0 + u, m - 2) : -1;
      dn[u] = t[i + 1];
      en[u] = t[(m >= 2) ? m + i : 0];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int i = i0 + u;
      if (i >= s1 || f) break;
      if (!(pi > 0.0)) {
        f = i + 1;
        break;
      }
      p[i] = pi;
      if (i + 1 < m) pi = dn[u] - en[u] * en[u] / pi;
    }
  }
  fail[k] = f;
}

// info = the failed pivot of the first chunk that has one (chunks after a failure carry meaningless
// starts, so only the first one counts).  One wave.
__global__ __launch_bounds__(64) void tridiag_first_fail_kernel(const int32_t* __restrict__ fail, int nch,
                                                                int32_t* __restrict__ info) {
  if (info[0]) return;
  int kmin = INT_MAX;
  for (int k = threadIdx.x; k < nch; k += 64)
    if (fail[k] && k < kmin) kmin = k;
  for (int o = 32; o > 0; o >>= 1) kmin = min(kmin, __shfl_xor(kmin, o));
  if (threadIdx.x == 0 && kmin != INT_MAX) info[0] = fail[kmin];
}

// c_i = sqrt(p_i), rc_i = 1 / c_i, f_i = e_i / c_i
__global__ void tridiag_factor_kernel(const double* __restrict__ t, const double* __restrict__ p, int m,
                                      double* __restrict__ c, double* __restrict__ rc, double* __restrict__ f,
                                      const int32_t* __restrict__ info) {
  if (info[0]) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double ci = sqrt(p[i]), ri = 1.0 / ci;
  c[i] = ci;
  rc[i] = ri;
  if (i + 1 < m) f[i] = t[m + i] * ri;
}

// W = C Z: w_i = c_i z_i + f_i z_{i+1}
__global__ void bidiag_apply_kernel(const double* __restrict__ c, const double* __restrict__ f, int m,
                                    const double* __restrict__ Z, int64_t ldz, double* __restrict__ W, int64_t ldw,
                                    int n, const int32_t* __restrict__ info) {
  if (info[0]) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * n) return;
  const int64_t j = idx / m;
  const int i = (int)(idx % m);
  const double* z = Z + j * ldz;
  double w = c[i] * z[i];
  if (i + 1 < m) w += f[i] * z[i + 1];
  W[j * ldw + i] = w;
}

// Q = C^{-1} Y in place (Q holds Y): q_i = a_i + b_i q_{i+1} with a_i = y_i / c_i, b_i = -f_i / c_i
// (q_m = 0), in chunks of TK rows: (1) per chunk and column the chunk's own solution with q = 0 past
// its end, and the coefficient B_i = b_i ... b_end of the value past the end (the same for every
// column); (2) per column, the values at the chunk starts, last chunk first; (3) q_i += B_i q_next.
__global__ void bidiag_back_local_kernel(const double* __restrict__ rc, const double* __restrict__ f, int m, int nch,
                                         double* __restrict__ Q, int64_t ldq, int n, double* __restrict__ Bc,
                                         const int32_t* __restrict__ info) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (info[0] || idx >= (int64_t)nch * n) return;
  const int k = (int)(idx % nch), j = (int)(idx / nch);
  const int s0 = k * TK, s1 = min(m, s0 + TK);
  double* q = Q + (int64_t)j * ldq;
  double a = 0.0, B = 1.0;
  for (int i1 = s1; i1 > s0; i1 -= 16) {   // rows i1 - 1 down to max(s0, i1 - 16)
    double rv[16], fv[16], qv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int i = max(i1 - 1 - u, s0);
      rv[u] = rc[i];
      fv[u] = f[min(i, m - 2 >= 0 ? m - 2 : 0)];
      qv[u] = q[i];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int i = i1 - 1 - u;
      if (i < s0) break;
      const double bi = (i + 1 < m) ? -fv[u] * rv[u] : 0.0;
      a = fma(bi, a, qv[u] * rv[u]);
      B *= bi;
      q[i] = a;
      if (j == 0) Bc[i] = B;
    }
  }
}

// qn[j][k] = q_j at the start of chunk k + 1 (0 past the end): V_k = a_k + B_k V_{k+1} over the chunk
// starts, as a scan of affine maps over one workgroup per column.
__global__ __launch_bounds__(SCAN_NT) void bidiag_back_starts_kernel(const double* __restrict__ Bc, int m, int nch,
                                                                    const double* __restrict__ Q, int64_t ldq, int n,
                                                                    double* __restrict__ qn,
                                                                    const int32_t* __restrict__ info) {
  __shared__ double Sa[SCAN_NT], Sb[SCAN_NT];
  const int j = blockIdx.x;
  if (info[0] || j >= n) return;
  const double* q = Q + (int64_t)j * ldq;
  const int tid = threadIdx.x;
  const int per = (nch + SCAN_NT - 1) / SCAN_NT;
  // position kk walks the chunks from the last (kk = 0) to the first; g_kk(x) = a + b x
  const int kk0 = min(nch, tid * per), kk1 = min(nch, kk0 + per);
  double ga = 0.0, gb = 1.0;   // composite of this thread's maps, later ones outside
  for (int kk = kk0; kk < kk1; ++kk) {
    const int s0 = (nch - 1 - kk) * TK;
    const double a = q[s0], b = Bc[s0];
    ga = fma(b, ga, a);
    gb = b * gb;
  }
  Sa[tid] = ga;
  Sb[tid] = gb;
  __syncthreads();
  for (int o = 1; o < SCAN_NT; o <<= 1) {
    double va = Sa[tid], vb = Sb[tid];
    if (tid >= o) {
      va = fma(vb, Sa[tid - o], va);
      vb = vb * Sb[tid - o];
    }
    __syncthreads();
    Sa[tid] = va;
    Sb[tid] = vb;
    __syncthreads();
  }
  double x = (tid > 0) ? Sa[tid - 1] : 0.0;   // V past this run (applied to V = 0 past the end)
  for (int kk = kk0; kk < kk1; ++kk) {
    const int k = nch - 1 - kk, s0 = k * TK;
    qn[(int64_t)j * nch + k] = x;
    x = fma(Bc[s0], x, q[s0]);
  }
}

__global__ void bidiag_back_fix_kernel(const double* __restrict__ Bc, int m, int nch, double* __restrict__ Q,
                                       int64_t ldq, int n, const double* __restrict__ qn,
                                       const int32_t* __restrict__ info) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (info[0] || idx >= (int64_t)m * n) return;
  const int64_t j = idx / m;
  const int i = (int)(idx % m);
  const double nx = qn[j * nch + i / TK];
  if (nx != 0.0) Q[j * ldq + i] = fma(Bc[i], nx, Q[j * ldq + i]);
}

}  // namespace

size_t chol_a_tridiag_workspace_bytes(int64_t m, int64_t n) {
  const int64_t nch = (m + TK - 1) / TK;
  return align256((size_t)m * sizeof(double)) * 4 + align256((size_t)m * n * sizeof(double)) +
         align256(euclid_qr_ws_bytes(m, n)) + align256((size_t)nch * 4 * sizeof(double)) +
         align256((size_t)nch * 2 * sizeof(double)) + align256((size_t)nch * sizeof(int32_t)) +
         align256((size_t)nch * n * sizeof(double));
}

int chol_a_tridiag_run(const oqr_op* A, const double* Z, int64_t ldz, int64_t m64, int64_t n64, double* Q,
                       int64_t ldq, double* R, int64_t ldr, void* ws, int32_t* info, hipStream_t s) {
  const int m = (int)m64, n = (int)n64;
  const double* t = (const double*)A->a;
  char* p = (char*)ws;
  auto take = [&](size_t bytes) {
    char* r = p;
    p += align256(bytes);
    return (double*)r;
  };
  double* piv = take((size_t)m * sizeof(double));
  double* c = take((size_t)m * sizeof(double));
  double* rc = take((size_t)m * sizeof(double));
  double* f = take((size_t)m * sizeof(double));
  double* Wt = take((size_t)m * n * sizeof(double));
  double* qr_ws = take(euclid_qr_ws_bytes(m, n));
  const int nch = ceil_div(m, TK);
  double* F = take((size_t)nch * 4 * sizeof(double));
  double* p0 = take((size_t)nch * 2 * sizeof(double));   // homogeneous chunk starts
  int32_t* fail = (int32_t*)take((size_t)nch * sizeof(int32_t));
  double* qn = take((size_t)nch * n * sizeof(double));
  if (nch > 1) {
    tridiag_chunk_maps_kernel<<<nch - 1, 64, 0, s>>>(t, m, nch, F, info);
    OQR_TRY(hipGetLastError());
  }
  tridiag_chunk_starts_kernel<<<1, SCAN_NT, 0, s>>>(t, nch, F, p0, info);
  OQR_TRY(hipGetLastError());
  tridiag_chunk_pivots_kernel<<<ceil_div(nch, 64), 64, 0, s>>>(t, m, nch, p0, piv, fail, info);
  OQR_TRY(hipGetLastError());
  tridiag_first_fail_kernel<<<1, 64, 0, s>>>(fail, nch, info);
  OQR_TRY(hipGetLastError());
  tridiag_factor_kernel<<<ceil_div(m, 256), 256, 0, s>>>(t, piv, m, c, rc, f, info);
  OQR_TRY(hipGetLastError());
  const int64_t mn = (int64_t)m * n;
  bidiag_apply_kernel<<<(unsigned)((mn + 255) / 256), 256, 0, s>>>(c, f, m, Z, ldz, Wt, m, n, info);
  OQR_TRY(hipGetLastError());
  OQR_TRY(launch_euclid_qr(Wt, m, m, n, qr_ws, R, ldr, Q, ldq, s));
  double* Bc = piv;   // the pivots are no longer needed
  bidiag_back_local_kernel<<<ceil_div((int64_t)nch * n, 64), 64, 0, s>>>(rc, f, m, nch, Q, ldq, n, Bc, info);
  OQR_TRY(hipGetLastError());
  bidiag_back_starts_kernel<<<n, SCAN_NT, 0, s>>>(Bc, m, nch, Q, ldq, n, qn, info);
  OQR_TRY(hipGetLastError());
  bidiag_back_fix_kernel<<<(unsigned)((mn + 255) / 256), 256, 0, s>>>(Bc, m, nch, Q, ldq, n, qn, info);
  OQR_TRY(hipGetLastError());
  return OQR_OK;
}

// =================================================================================================
// EQR-SYEV: cyclic two-sided Jacobi, A = V D V^T
// =================================================================================================
namespace {

// Round-robin pairing on M (even) indices: index M-1 is fixed; round r pairs (r, M-1) and
// ((r + k) mod (M-1), (r - k) mod (M-1)) for k = 1 .. M/2 - 1.
__device__ __forceinline__ void rr_pair(int r, int k, int M, int& p, int& q) {
  if (k == 0) {
    p = r;
    q = M - 1;
  } else {
    p = (r + k) % (M - 1);
    q = (r - k + (M - 1)) % (M - 1);
  }
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
}

// Columns p, q of A and V for every pair of round r; the rotation (c, s) zeroing A_pq is computed
// from the values before the round and stored for the row pass.  One workgroup per pair.
__global__ __launch_bounds__(NT) void jacobi_cols_kernel(double* __restrict__ A, int64_t lda, double* __restrict__ V,
                                                          int64_t ldv, int m, int M, int r, double* __restrict__ cs,
                                                          int32_t* __restrict__ rotated,
                                                          const int32_t* __restrict__ done) {
  if (done[0]) return;
  int p, q;
  rr_pair(r, blockIdx.x, M, p, q);
  __shared__ double s_c, s_s;
  if (q >= m) {                        // the padding index: no rotation
    if (threadIdx.x == 0) {
      cs[2 * blockIdx.x] = 1.0;
      cs[2 * blockIdx.x + 1] = 0.0;
    }
    return;
  }
  if (threadIdx.x == 0) {
    const double app = A[(int64_t)p * lda + p], aqq = A[(int64_t)q * lda + q], apq = A[(int64_t)q * lda + p];
    double c = 1.0, s = 0.0;
    // rotate unless a_pq is negligible relative to sqrt(a_pp a_qq) (relative accuracy of Jacobi)
    if (fabs(apq) > 1.1102230246251565e-16 * sqrt(fabs(app * aqq)) && apq != 0.0) {
      const double zeta = (aqq - app) / (2.0 * apq);
      const double t = fabs(zeta) > 1e100 ? 0.5 / zeta
                                          : (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
      c = 1.0 / sqrt(1.0 + t * t);
      s = t * c;
      atomicAdd(rotated, 1);
    }
    s_c = c;
    s_s = s;
    cs[2 * blockIdx.x] = c;
    cs[2 * blockIdx.x + 1] = s;
  }
  __syncthreads();
  const double c = s_c, s = s_s;
  if (s == 0.0) return;
  double* ap = A + (int64_t)p * lda;
  double* aq = A + (int64_t)q * lda;
  double* vp = V + (int64_t)p * ldv;
  double* vq = V + (int64_t)q * ldv;
  for (int i = threadIdx.x; i < m; i += NT) {
    const double x = ap[i], y = aq[i];
    ap[i] = c * x - s * y;
    aq[i] = s * x + c * y;
    const double u = vp[i], w = vq[i];
    vp[i] = c * u - s * w;
    vq[i] = s * u + c * w;
  }
}

// Rows p, q of A for every pair of round r (after the column pass).
__global__ __launch_bounds__(NT) void jacobi_rows_kernel(double* __restrict__ A, int64_t lda, int m, int M, int r,
                                                          const double* __restrict__ cs,
                                                          const int32_t* __restrict__ done) {
  if (done[0]) return;
  int p, q;
  rr_pair(r, blockIdx.x, M, p, q);
  if (q >= m) return;
  const double c = cs[2 * blockIdx.x], s = cs[2 * blockIdx.x + 1];
  if (s == 0.0) return;
  for (int j = threadIdx.x; j < m; j += NT) {
    const double x = A[(int64_t)j * lda + p], y = A[(int64_t)j * lda + q];
    A[(int64_t)j * lda + p] = c * x - s * y;
    A[(int64_t)j * lda + q] = s * x + c * y;
  }
  __syncthreads();
  // the rotation annihilates a_pq; store the exact zero instead of its rounding residue
  if (threadIdx.x == 0) {
    A[(int64_t)q * lda + p] = 0.0;
    A[(int64_t)p * lda + q] = 0.0;
  }
}

// After a sweep: done = (no rotation happened); reset the counter.
__global__ void jacobi_sweep_end_kernel(int32_t* __restrict__ rotated, int32_t* __restrict__ done,
                                        int32_t* __restrict__ sweeps) {
  if (done[0]) return;
  sweeps[0] += 1;
  if (rotated[0] == 0) done[0] = 1;
  rotated[0] = 0;
}

// d = diag(A); info = 1 if some d_i <= 0, 2 if Jacobi did not converge
__global__ void jacobi_finish_kernel(const double* __restrict__ A, int64_t lda, int m, double* __restrict__ d,
                                     const int32_t* __restrict__ done, int32_t* __restrict__ info) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && !done[0] && info[0] == 0) info[0] = 2;
  if (i >= m) return;
  const double v = A[(int64_t)i * lda + i];
  d[i] = v;
  if (!(v > 0.0)) atomicCAS(info, 0, 1);
}

// B = V^T (m x m transpose)
__global__ void transpose_kernel(const double* __restrict__ V, int64_t ldv, double* __restrict__ B, int64_t ldb,
                                 int m) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int y = threadIdx.y; y < 32; y += 8) {
    const int i = bx + threadIdx.x, j = by + y;
    tile[y][threadIdx.x] = (i < m && j < m) ? V[(int64_t)j * ldv + i] : 0.0;
  }
  __syncthreads();
  for (int y = threadIdx.y; y < 32; y += 8) {
    const int i = by + threadIdx.x, j = bx + y;
    if (i < m && j < m) B[(int64_t)j * ldb + i] = tile[threadIdx.x][y];
  }
}

// X(i, c) *= d_i^{power} (power = +1/2 or -1/2)
__global__ void diag_scale_kernel(double* __restrict__ X, int64_t ldx, int m, int n, const double* __restrict__ d,
                                  int inverse, const int32_t* __restrict__ info) {
  if (info[0]) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * n) return;
  const int c = (int)(idx / m), i = (int)(idx % m);
  const double s = sqrt(d[i]);
  X[(int64_t)c * ldx + i] = inverse ? X[(int64_t)c * ldx + i] / s : X[(int64_t)c * ldx + i] * s;
}

constexpr int MAX_SWEEPS = 30;

}  // namespace

size_t eig_a_workspace_bytes(int64_t m, int64_t n) {
  size_t b = 0;
  b += align256((size_t)m * m * sizeof(double)) * 3;    // A copy, V, V^T
  b += align256((size_t)m * n * sizeof(double)) * 2;    // X/W, U
  b += align256((size_t)(m + 8) * sizeof(double));      // d
  b += align256((size_t)(m + 2) * sizeof(double));      // rotations (c, s) per pair
  b += align256(euclid_qr_ws_bytes(m, n));              // the Euclidean QR
  b += align256(64);                                    // counters
  return b;
}

int eig_a_run(const oqr_op* A, const double* Z, int64_t ldz, int64_t m64, int64_t n64, double* Q, int64_t ldq,
              double* R, int64_t ldr, void* ws, int32_t* info, hipStream_t s) {
  const int m = (int)m64, n = (int)n64;
  char* p = (char*)ws;
  auto take = [&](size_t bytes) {
    char* r = p;
    p += align256(bytes);
    return r;
  };
  double* Ac = (double*)take((size_t)m * m * sizeof(double));
  double* V = (double*)take((size_t)m * m * sizeof(double));
  double* Vt = (double*)take((size_t)m * m * sizeof(double));
  double* X = (double*)take((size_t)m * n * sizeof(double));
  double* U = (double*)take((size_t)m * n * sizeof(double));
  double* d = (double*)take((size_t)(m + 8) * sizeof(double));
  double* cs = (double*)take((size_t)(m + 2) * sizeof(double));
  void* qr_ws = take(euclid_qr_ws_bytes(m, n));
  int32_t* cnt = (int32_t*)take(64);          // [0] rotated, [1] done, [2] sweeps
  OQR_TRY(launch_copy_matrix((const double*)A->a, A->lda, Ac, m, m, m, s));
  eye_kernel<<<(unsigned)(((int64_t)m * m + 255) / 256), 256, 0, s>>>(V, m, m, m);
  OQR_TRY(hipGetLastError());
  OQR_TRY(launch_fill_i32(cnt, 0, 16, s));
  const int M = (m % 2) ? m + 1 : m;
  if (m > 1) {
    for (int sw = 0; sw < MAX_SWEEPS; ++sw) {
      for (int r = 0; r < M - 1; ++r) {
        jacobi_cols_kernel<<<M / 2, NT, 0, s>>>(Ac, m, V, m, m, M, r, cs, cnt, cnt + 1);
        jacobi_rows_kernel<<<M / 2, NT, 0, s>>>(Ac, m, m, M, r, cs, cnt + 1);
      }
      jacobi_sweep_end_kernel<<<1, 1, 0, s>>>(cnt, cnt + 1, cnt + 2);
      OQR_TRY(hipGetLastError());
    }
  } else {
    OQR_TRY(launch_fill_i32(cnt + 1, 1, 1, s));
  }
  jacobi_finish_kernel<<<ceil_div(m, 256), 256, 0, s>>>(Ac, m, m, d, cnt + 1, info);
  OQR_TRY(hipGetLastError());
  // X = V^T Z; W = D^{1/2} X; [Y, R] = qr(W); U = D^{-1/2} Y; Q = V U
  transpose_kernel<<<dim3(ceil_div(m, 32), ceil_div(m, 32)), dim3(32, 8), 0, s>>>(V, m, Vt, m, m);
  OQR_TRY(hipGetLastError());
  OQR_TRY(launch_gemm_f64(Vt, m, Z, ldz, X, m, m, n, nullptr, s));
  const int64_t mn = (int64_t)m * n;
  diag_scale_kernel<<<(unsigned)((mn + 255) / 256), 256, 0, s>>>(X, m, m, n, d, 0, info);
  OQR_TRY(hipGetLastError());
  OQR_TRY(launch_euclid_qr(X, m, m, n, qr_ws, R, ldr, U, m, s));
  diag_scale_kernel<<<(unsigned)((mn + 255) / 256), 256, 0, s>>>(U, m, m, n, d, 1, info);
  OQR_TRY(hipGetLastError());
  OQR_TRY(launch_gemm_f64(V, m, U, m, Q, ldq, m, n, nullptr, s));
  return OQR_OK;
}

}  // namespace oqr
