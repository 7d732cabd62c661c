// Device-side error report (Section 7 measures): ||I - Q^T A Q||_F and
// ||Z - Q R||_F / ||Z||_F, in FP64 with fixed-order reductions.
#include "common.hpp"

namespace oqr {
namespace {

constexpr int NT = 256;

__device__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x / 64); ++w) s += red[w];
  return s;
}

// part[2*b] = sum over rows of block b of |Z - QR|^2, part[2*b+1] = sum |Z|^2.
__global__ __launch_bounds__(NT) void residual_kernel(const double* __restrict__ Z, int64_t ldz,
                                                      const double* __restrict__ Q, int64_t ldq,
                                                      const double* __restrict__ R, int64_t ldr, int m, int n,
                                                      double* __restrict__ part) {
  __shared__ double red[NT / 64];
  const int i = blockIdx.x * NT + threadIdx.x;
  double e2 = 0.0, z2 = 0.0;
  if (i < m) {
    for (int j = 0; j < n; ++j) {
      double qr = 0.0;
      for (int k = 0; k <= j; ++k) qr += Q[(int64_t)k * ldq + i] * R[(int64_t)j * ldr + k];
      const double z = Z[(int64_t)j * ldz + i];
      const double d = z - qr;
      e2 += d * d;
      z2 += z * z;
    }
  }
  const double se = block_sum(e2, red);
  const double sz = block_sum(z2, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = se;
    part[2 * blockIdx.x + 1] = sz;
  }
}

__global__ __launch_bounds__(NT) void finish_kernel(const double* __restrict__ G, int n,
                                                    const double* __restrict__ part, int nparts,
                                                    double* __restrict__ out) {
  __shared__ double red[NT / 64];
  double o = 0.0;
  for (int idx = threadIdx.x; idx < n * n; idx += NT) {
    const int j = idx / n, i = idx % n;
    const double d = G[idx] - (i == j ? 1.0 : 0.0);
    o += d * d;
  }
  const double so = block_sum(o, red);
  double e = 0.0, z = 0.0;
  if (threadIdx.x == 0) {
    for (int b = 0; b < nparts; ++b) {
      e += part[2 * b];
      z += part[2 * b + 1];
    }
    out[0] = sqrt(so);
    out[1] = sqrt(e) / sqrt(z);
  }
}

}  // namespace

size_t check_workspace_bytes(const oqr_op* A, int64_t m, int64_t n) {
  (void)A;
  size_t b = align256((size_t)m * n * sizeof(double));
  b += align256(gram_partial_bytes(m, n));
  b += align256((size_t)n * n * sizeof(double));
  b += align256((size_t)2 * ceil_div(m, NT) * sizeof(double));
  return b;
}

int check_run(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n, const double* Q, int64_t ldq,
              const double* R, int64_t ldr, void* ws, size_t ws_bytes, double* out, hipStream_t s) {
  (void)ws_bytes;
  char* p = (char*)ws;
  double* W = (double*)p;
  p += align256((size_t)m * n * sizeof(double));
  double* partial = (double*)p;
  p += align256(gram_partial_bytes(m, n));
  double* G = (double*)p;
  p += align256((size_t)n * n * sizeof(double));
  double* part = (double*)p;
  hipError_t e;
  if (A->kind == OQR_OP_DENSE)
    e = launch_gemm_f64((const double*)A->a, A->lda, Q, ldq, W, m, m, n, nullptr, s);
  else
    e = launch_sparse_apply(A, Q, ldq, W, m, n, s);
  if (e != hipSuccess) return OQR_E_HIP;
  if (launch_gram_f64(Q, ldq, W, m, m, n, partial, G, s) != hipSuccess) return OQR_E_HIP;
  const int nb = ceil_div(m, NT);
  residual_kernel<<<nb, NT, 0, s>>>(Z, ldz, Q, ldq, R, ldr, (int)m, (int)n, part);
  if (hipGetLastError() != hipSuccess) return OQR_E_HIP;
  finish_kernel<<<1, NT, 0, s>>>(G, (int)n, part, nb, out);
  if (hipGetLastError() != hipSuccess) return OQR_E_HIP;
  return OQR_OK;
}

}  // namespace oqr
