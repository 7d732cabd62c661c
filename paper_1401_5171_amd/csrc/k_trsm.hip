// Triangular solve Q = Z R^{-1} (step 4 of CHOLQR, Algorithm 1), FP64.
//
// Each row of Q solves q_i R = z_i by substitution, which is the row-wise
// backward-stable solve the residual bound of Theorem 2.1 rests on:
// q_ij = (z_ij - sum_{k<j} q_ik r_kj) / r_jj, with k ascending.  One thread per
// row (coalesced across the rows of a column-major Z); columns are processed
// in blocks of 32 held in registers; R is read with uniform addresses.
// Q may alias Z: a block of Z is read before the same columns of Q are written.
#include "common.hpp"

namespace oqr {
namespace {

constexpr int JB = 32;
constexpr int NT = 64;

__global__ __launch_bounds__(NT) void trsm_kernel(const double* Z, int64_t ldz, const double* __restrict__ R,
                                                  int64_t ldr, double* Q, int64_t ldq, int m, int n,
                                                  const int32_t* __restrict__ info) {
  if (info[0] != 0) return;
  const int i = blockIdx.x * NT + threadIdx.x;
  const bool ok = i < m;
  for (int j0 = 0; j0 < n; j0 += JB) {
    const int jb = min(JB, n - j0);
    double x[JB];
#pragma unroll
    for (int c = 0; c < JB; ++c) x[c] = (ok && c < jb) ? Z[(int64_t)(j0 + c) * ldz + i] : 0.0;
    for (int k = 0; k < j0; ++k) {
      const double qk = ok ? Q[(int64_t)k * ldq + i] : 0.0;
      const double* rk = R + (int64_t)j0 * ldr + k;
#pragma unroll
      for (int c = 0; c < JB; ++c)
        if (c < jb) x[c] -= qk * rk[(int64_t)c * ldr];
    }
#pragma unroll
    for (int c = 0; c < JB; ++c) {
      if (c < jb) {
        const double* rc = R + (int64_t)(j0 + c) * ldr + j0;
#pragma unroll
        for (int p = 0; p < c; ++p) x[c] -= x[p] * rc[p];
        x[c] = x[c] / rc[c];
      }
    }
    if (ok) {
#pragma unroll
      for (int c = 0; c < JB; ++c)
        if (c < jb) Q[(int64_t)(j0 + c) * ldq + i] = x[c];
    }
  }
}

// W = A Z for the 7-point operator: one thread per (grid point, column).
__global__ void stencil_apply_kernel(const double* __restrict__ Z, int64_t ldz, double* __restrict__ W, int64_t ldw,
                                     int nx, int ny, int nz, double center, double off, int64_t n) {
  const int64_t m = (int64_t)nx * ny * nz;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * n) return;
  const int64_t j = idx / m, p = idx % m;
  const int x = (int)(p % nx);
  const int y = (int)((p / nx) % ny);
  const int zc = (int)(p / ((int64_t)nx * ny));
  const double* z = Z + j * ldz;
  const int64_t sy = nx, sz = (int64_t)nx * ny;
  double nb = 0.0;
  if (x > 0) nb += z[p - 1];
  if (x < nx - 1) nb += z[p + 1];
  if (y > 0) nb += z[p - sy];
  if (y < ny - 1) nb += z[p + sy];
  if (zc > 0) nb += z[p - sz];
  if (zc < nz - 1) nb += z[p + sz];
  W[j * ldw + p] = center * z[p] + off * nb;
}

}  // namespace

hipError_t launch_trsm(const double* Z, int64_t ldz, const double* R, int64_t ldr, double* Q, int64_t ldq,
                       int64_t m, int64_t n, const int32_t* info, hipStream_t s) {
  trsm_kernel<<<ceil_div(m, NT), NT, 0, s>>>(Z, ldz, R, ldr, Q, ldq, (int)m, (int)n, info);
  return hipGetLastError();
}

hipError_t launch_stencil_apply(const oqr_op* op, const double* Z, int64_t ldz, double* W, int64_t ldw, int64_t n,
                                hipStream_t s) {
  const int64_t m = (int64_t)op->nx * op->ny * op->nz;
  const int64_t total = m * n;
  stencil_apply_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(Z, ldz, W, ldw, op->nx, op->ny, op->nz,
                                                                        op->center, op->off, n);
  return hipGetLastError();
}

}  // namespace oqr
