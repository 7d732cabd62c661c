// Small dense kernels of the CholQR pass: the n x n Cholesky factorisation of
// the Gram matrix (step 3 of Algorithm 1, R = chol(C)) with the shift-and-retry
// rule, the triangular product R = R2 R1 that combines two passes, and fills.
//
// Cholesky: one workgroup of 1024 threads, blocked right-looking with 32x32
// blocks, working in place in R (global memory, L2-resident):
//   (a) the diagonal block is factored in LDS (one entry per thread),
//   (b) the block row to its right is solved column by column,
//       R_KJ = R_KK^{-T} G_KJ (substitution, one thread per column),
//   (c) the trailing upper blocks get G_IJ -= R_KI^T R_KJ on FP64 MFMA.
// A pivot that is not positive (or NaN) restarts the factorisation from the
// kept G with a larger diagonal shift; after the last retry the 1-based pivot
// index goes to info (LAPACK potrf convention).
#include "common.hpp"

#include <math.h>

namespace oqr {
namespace {

constexpr int CB = 32;
constexpr int NTC = 1024;

__global__ __launch_bounds__(NTC) void chol_kernel(const double* __restrict__ G, int n, double* __restrict__ R,
                                                    int64_t ldr, double unit, double c_first, double c_retry,
                                                    int max_retries, int32_t* __restrict__ info,
                                                    double* __restrict__ shift_used) {
  __shared__ double Dk[CB][CB + 1];
  __shared__ double P[CB][OQR_MAX_N + 2];     // P[p][j] = R(k0 + p, j), j absolute column
  __shared__ double red[NTC / 64];
  __shared__ double s_dmax;
  __shared__ int s_fail;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  if (info[0] != 0) return;                   // an earlier pass failed

  // max_i G_ii (estimator of ||G||_2 for the shift)
  double v = (t < n) ? G[(int64_t)t * n + t] : 0.0;
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  if (lane == 0) red[wave] = v;
  __syncthreads();
  if (t == 0) {
    double mx = 0.0;
    for (int w = 0; w < NTC / 64; ++w) mx = fmax(mx, red[w]);
    s_dmax = mx;
  }
  __syncthreads();
  const double dmax = s_dmax;
  const int npad = (n + CB - 1) / CB * CB;

  double c = c_first;
  for (int attempt = 0;; ++attempt) {
    const double s = c * unit * dmax;
    for (int idx = t; idx < n * n; idx += NTC) {
      const int j = idx / n, i = idx % n;
      R[(int64_t)j * ldr + i] = (i <= j) ? G[(int64_t)j * n + i] + (i == j ? s : 0.0) : 0.0;
    }
    if (t == 0) s_fail = 0;
    __syncthreads();

    for (int k0 = 0; k0 < n; k0 += CB) {
      const int kb = min(CB, n - k0);
      // (a) factor the diagonal block in LDS
      const int di = t >> 5, dj = t & 31;
      Dk[di][dj] = (di < kb && dj < kb) ? R[(int64_t)(k0 + dj) * ldr + k0 + di] : (di == dj ? 1.0 : 0.0);
      __syncthreads();
      for (int k = 0; k < kb; ++k) {
        const double piv = Dk[k][k];
        if (!(piv > 0.0)) {                    // every thread reads the same value: uniform exit
          if (t == 0) s_fail = k0 + k + 1;
          break;
        }
        const double rkk = sqrt(piv);
        double nv = 0.0;
        bool wr = false;
        if (di == k && dj >= k) {
          nv = (dj == k) ? rkk : Dk[k][dj] / rkk;
          wr = true;
        } else if (di > k && dj >= di) {
          nv = Dk[di][dj] - (Dk[k][di] / rkk) * (Dk[k][dj] / rkk);
          wr = true;
        }
        __syncthreads();
        if (wr) Dk[di][dj] = nv;
        __syncthreads();
      }
      __syncthreads();
      if (s_fail) break;
      // (b) write the factored block, solve the block row R_KJ = R_KK^{-T} G_KJ
      if (di < kb && dj < kb && di <= dj) R[(int64_t)(k0 + dj) * ldr + k0 + di] = Dk[di][dj];
      const int k1 = k0 + kb;
      const int jcol = k1 + t;
      if (jcol < npad) {
        double x[CB];
#pragma unroll
        for (int p = 0; p < CB; ++p) {
          double acc = (p < kb && jcol < n) ? R[(int64_t)jcol * ldr + k0 + p] : 0.0;
#pragma unroll
          for (int q = 0; q < p; ++q) acc -= Dk[q][p] * x[q];
          x[p] = (p < kb && jcol < n) ? acc / Dk[p][p] : 0.0;
        }
#pragma unroll
        for (int p = 0; p < CB; ++p) {
          P[p][jcol] = x[p];
          if (p < kb && jcol < n) R[(int64_t)jcol * ldr + k0 + p] = x[p];
        }
      }
      __syncthreads();
      // (c) trailing update of the upper 32x32 blocks (I, J), k1 <= I <= J
      const int nbt = (n - k1 + CB - 1) / CB;
      const int pairs = nbt * (nbt + 1) / 2;
      for (int pr = wave; pr < pairs; pr += NTC / 64) {
        int a = 0, rem = pr;
        while (rem >= nbt - a) { rem -= nbt - a; ++a; }
        const int b = a + rem;
        const int I0 = k1 + a * CB, J0 = k1 + b * CB;
        f64x4 acc[2][2];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = I0 + 16 * x + 4 * r + (lane >> 4), j = J0 + 16 * y + (lane & 15);
              acc[x][y][r] = (i < n && j < n) ? R[(int64_t)j * ldr + i] : 0.0;
            }
#pragma unroll
        for (int kk = 0; kk < CB; kk += 4) {
          const int kr = kk + (lane >> 4);
          double av[2], bv[2];
#pragma unroll
          for (int x = 0; x < 2; ++x) av[x] = -P[kr][I0 + 16 * x + (lane & 15)];
#pragma unroll
          for (int y = 0; y < 2; ++y) bv[y] = P[kr][J0 + 16 * y + (lane & 15)];
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) acc[x][y] = mfma_f64(av[x], bv[y], acc[x][y]);
        }
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = I0 + 16 * x + 4 * r + (lane >> 4), j = J0 + 16 * y + (lane & 15);
              if (i < n && j < n && i <= j) R[(int64_t)j * ldr + i] = acc[x][y][r];
            }
      }
      __syncthreads();
    }
    __syncthreads();
    const int fail = s_fail;
    if (!fail) {
      if (t == 0 && shift_used) *shift_used = s;
      break;
    }
    if (attempt >= max_retries) {
      if (t == 0) {
        info[0] = fail;
        if (shift_used) *shift_used = s;
      }
      break;
    }
    c = (c == 0.0) ? c_retry : c * 10.0;
    __syncthreads();
  }
}

// R = R2 * R1 for upper triangular n x n factors.
__global__ void trmm_upper_kernel(const double* __restrict__ R2, int64_t ld2, const double* __restrict__ R1,
                                  int64_t ld1, double* __restrict__ R, int64_t ldr, int n,
                                  const int32_t* __restrict__ info) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int j = (int)(idx / n), i = (int)(idx % n);
  if (info && info[0] != 0) return;
  double s = 0.0;
  if (i <= j)
    for (int k = i; k <= j; ++k) s += R2[(int64_t)k * ld2 + i] * R1[(int64_t)j * ld1 + k];
  R[(int64_t)j * ldr + i] = s;
}

__global__ void copy_matrix_kernel(const double* __restrict__ X, int64_t ldx, double* __restrict__ Y, int64_t ldy,
                                   int64_t m, int64_t n) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * n) return;
  const int64_t j = idx / m, i = idx % m;
  Y[j * ldy + i] = X[j * ldx + i];
}

__global__ void fill_i32_kernel(int32_t* p, int32_t v, int64_t count) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) p[idx] = v;
}

}  // namespace

hipError_t launch_chol_small(const double* G, int64_t n, double* R, int64_t ldr, double unit, double c_first,
                             double c_retry, int max_retries, int32_t* info, double* shift_used, hipStream_t s) {
  chol_kernel<<<1, NTC, 0, s>>>(G, (int)n, R, ldr, unit, c_first, c_retry, max_retries, info, shift_used);
  return hipGetLastError();
}

hipError_t launch_trmm_upper(const double* R2, int64_t ld2, const double* R1, int64_t ld1, double* R, int64_t ldr,
                             int64_t n, const int32_t* info, hipStream_t s) {
  const int64_t total = n * n;
  trmm_upper_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(R2, ld2, R1, ld1, R, ldr, (int)n, info);
  return hipGetLastError();
}

hipError_t launch_copy_matrix(const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t m, int64_t n,
                              hipStream_t s) {
  const int64_t total = m * n;
  if (total == 0) return hipSuccess;
  copy_matrix_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(X, ldx, Y, ldy, m, n);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  fill_i32_kernel<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(p, v, count);
  return hipGetLastError();
}

}  // namespace oqr
