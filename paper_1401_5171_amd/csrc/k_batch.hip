// Batched CholQR2-A over many independent dense instances in one persistent launch.
//
// Workgroups (256 threads) take instances from a device work queue (atomic counter over an order
// array sorted by decreasing cost) until the queue is empty, and run both CHOLQR passes of an
// instance on their own (Algorithm 1 twice, R = R2 R1):
//   G = X^T A X  row block by row block: W_b = A_b X on FP64 MFMA, then G += X_b^T W_b, so W is
//                never stored; G stays in the MFMA accumulators,
//   R = chol(G + s I) in LDS with the shift-and-retry rule of the single-instance path,
//   X <- X R^{-1}  row-wise substitution, four lanes per row,
// and finally R = R2 R1.  Storage is FP64 or FP32 (FP32 values are widened to FP64 on load, so all
// arithmetic is FP64 and the shift rule is the FP64 one).  n_i <= 64; m_i >= n_i.  One failing instance sets its own info and never
// stops the batch.  The launch allocates nothing and issues no memset (the queue counter is cleared
// by a kernel), so a caller may capture it in a graph.
#include "common.hpp"

#include <math.h>

namespace oqr {
namespace {

constexpr int NT = 256;
constexpr int NB = 64;        // max n
constexpr int BR = 64;        // rows of A per block
constexpr int BK = 16;        // K step of the A X product
constexpr int LD = NB + 1;

constexpr double U64 = 1.1102230246251565e-16;

template <class T>
__device__ __forceinline__ double ldv(const T* p, int64_t i, bool ok) {
  const T v = p[ok ? i : 0];
  return ok ? (double)v : 0.0;
}

struct Tiles {
  double As[BK][BR + 1];      // A tile: As[k][i]
  double Xs[BK][LD];          // X tile: Xs[k][j]
};
struct Smem {
  union {
    Tiles tl;                 // during the K loop of W_b = A_b X
    double Ws[BR][LD];        // W_b (rows of the block x columns); R1 at the end
  };
  double Gs[NB][LD];          // Gram, then the factor R (upper)
  double diag[NB];
  int idx;
  int fail;
  double dmax;
};

// One CHOLQR pass on instance (A, X) in place: X <- X R^{-1}, R into smem Gs (upper, zero lower).
// Returns 0 or the failing pivot (1-based).
template <class T>
__device__ int cholqr_pass_wg(const T* A, int64_t lda, const T* Xin, int64_t ldxin, T* X, int64_t ldx, int m,
                              int n, double unit, double c_first, double c_retry, int max_retries, Smem& S) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int li = lane >> 4, lj = lane & 15;
  const int nbk = (n + 15) / 16;              // 16-column blocks of n
  // ---- G = X^T A X ----------------------------------------------------------------------------
  f64x4 g[4];                                 // wave owns G rows 16 wave .. + 15, column blocks 0..3
#pragma unroll
  for (int b = 0; b < 4; ++b) g[b] = f64x4{0, 0, 0, 0};
  for (int r0 = 0; r0 < m; r0 += BR) {
    f64x4 w[4];                               // wave owns W_b rows 16 wave .. + 15
#pragma unroll
    for (int b = 0; b < 4; ++b) w[b] = f64x4{0, 0, 0, 0};
    for (int k0 = 0; k0 < m; k0 += BK) {
      // A tile: rows r0..r0+63, columns k0..k0+15 (column-major: contiguous rows)
#pragma unroll
      for (int q = 0; q < BR * BK / NT; ++q) {
        const int e = t + NT * q, i = e % BR, k = e / BR;
        S.tl.As[k][i] = ldv(A, (int64_t)(k0 + k) * lda + r0 + i, r0 + i < m && k0 + k < m);
      }
      // X tile: rows k0..k0+15, columns 0..63
#pragma unroll
      for (int q = 0; q < BK * NB / NT; ++q) {
        const int e = t + NT * q, k = e % BK, j = e / BK;
        S.tl.Xs[k][j] = ldv(Xin, (int64_t)j * ldxin + k0 + k, j < n && k0 + k < m);
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        const double a = S.tl.As[kk + li][wave * 16 + lj];
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if (b < nbk) w[b] = mfma_f64(a, S.tl.Xs[kk + li][b * 16 + lj], w[b]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) S.Ws[wave * 16 + 4 * r + li][b * 16 + lj] = w[b][r];
    __syncthreads();
    // G += X_b^T W_b: A operand X_b^T (rows of G = columns of X), B operand W_b
#pragma unroll 4
    for (int kk = 0; kk < BR; kk += 4) {
      const int row = r0 + kk + li;
      const int col = wave * 16 + lj;
      const double a = ldv(Xin, (int64_t)col * ldxin + row, row < m && col < n);
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (b < nbk) g[b] = mfma_f64(a, S.Ws[kk + li][b * 16 + lj], g[b]);
    }
    __syncthreads();
  }
  // ---- R = chol(G + s I), retries from the accumulators ------------------------------------------
  // max diag(G): diagonal entries sit in block b == wave, element r with 4r + li == lj
  if (t < NB) S.diag[t] = 0.0;
  __syncthreads();
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (b == wave && 4 * r + li == lj) S.diag[wave * 16 + lj] = g[b][r];
  __syncthreads();
  if (t == 0) {
    double mx = 0.0;
    for (int i = 0; i < n; ++i) mx = fmax(mx, S.diag[i]);
    S.dmax = mx;
  }
  __syncthreads();
  double c = c_first;
  int fail = 0;
  for (int attempt = 0;; ++attempt) {
    const double s = c * unit * S.dmax;
    // G (upper triangle, symmetric use) into Gs; identity beyond n
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = wave * 16 + 4 * r + li, j = b * 16 + lj;
        double v = g[b][r] + (i == j ? s : 0.0);
        if (i >= n || j >= n) v = (i == j) ? 1.0 : 0.0;
        S.Gs[i][j] = v;
      }
    if (t == 0) S.fail = 0;
    __syncthreads();
    // right-looking, upper: one entry per thread-slot, two barriers per pivot
    for (int k = 0; k < n; ++k) {
      const double piv = S.Gs[k][k];
      if (!(piv > 0.0)) {
        if (t == 0) S.fail = k + 1;
        break;
      }
      const double rkk = sqrt(piv);
      double nv[NB * NB / NT];
#pragma unroll
      for (int q = 0; q < NB * NB / NT; ++q) {
        const int e = t + NT * q, i = e / NB, j = e % NB;
        double v = S.Gs[i][j];
        if (i == k && j >= k) v = (j == k) ? rkk : v / rkk;
        else if (i > k && j >= i) v = v - (S.Gs[k][i] / rkk) * (S.Gs[k][j] / rkk);
        nv[q] = v;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < NB * NB / NT; ++q) {
        const int e = t + NT * q, i = e / NB, j = e % NB;
        S.Gs[i][j] = nv[q];
      }
      __syncthreads();
    }
    __syncthreads();
    fail = S.fail;
    if (!fail || attempt >= max_retries) break;
    c = (c == 0.0) ? c_retry : c * 10.0;
    __syncthreads();
  }
  if (fail) return fail;
  // zero the strictly lower triangle
  for (int e = t; e < NB * NB; e += NT) {
    const int i = e / NB, j = e % NB;
    if (i > j) S.Gs[i][j] = 0.0;
  }
  __syncthreads();
  // ---- X <- X R^{-1}: four lanes per row (lane `sub` owns columns sub + 4e), the pivot column's
  // value broadcast within the quad; q_ij = (x_ij - sum_{k<j} q_ik r_kj) / r_jj, k ascending ---------
  {
    const int sub = t & 3;
    for (int r0 = 0; r0 < m; r0 += NT / 4) {
      const int row = r0 + (t >> 2);
      const bool ok = row < m;
      double x[NB / 4];
#pragma unroll
      for (int e = 0; e < NB / 4; ++e) x[e] = ldv(Xin, (int64_t)(sub + 4 * e) * ldxin + row, ok && sub + 4 * e < n);
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c < n) {
          const int owner = c & 3, ec = c >> 2;
          const double qo = x[ec] / S.Gs[c][c];
          const double qv = __shfl(qo, (lane & ~3) | owner);
          if (sub == owner) x[ec] = qv;
#pragma unroll
          for (int e = 0; e < NB / 4; ++e) {
            const double upd = x[e] - qv * S.Gs[c][sub + 4 * e];
            x[e] = (sub + 4 * e > c) ? upd : x[e];
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
#pragma unroll
      for (int e = 0; e < NB / 4; ++e)
        if (ok && sub + 4 * e < n) X[(int64_t)(sub + 4 * e) * ldx + row] = (T)x[e];
    }
  }
  __syncthreads();
  return 0;
}

template <class T>
__global__ __launch_bounds__(NT) void batch_kernel(const oqr_batch_item* __restrict__ items,
                                                    const int32_t* __restrict__ order, int batch,
                                                    int32_t* __restrict__ counter, int32_t* __restrict__ info,
                                                    double c_retry, int max_retries) {
  __shared__ Smem S;
  const int t = threadIdx.x;
  for (;;) {
    if (t == 0) S.idx = atomicAdd(counter, 1);
    __syncthreads();
    const int slot = S.idx;
    __syncthreads();
    if (slot >= batch) break;
    const int id = order[slot];
    const oqr_batch_item it = items[id];
    const T* A = (const T*)it.a;
    const T* Z = (const T*)it.z;
    T* Q = (T*)it.q;
    T* R = (T*)it.r;
    const int m = it.m, n = it.n;
    // pass 1 (Z -> Q), pass 2 (Q in place); both FP64 arithmetic
    int f = cholqr_pass_wg<T>(A, it.lda, Z, it.ldz, Q, it.ldq, m, n, U64, 0.0, c_retry, max_retries, S);
    if (f) {
      if (t == 0) info[id] = f;
      __syncthreads();
      continue;
    }
    double r1[NB * NB / NT];                    // R1, kept in registers across pass 2
#pragma unroll
    for (int q = 0; q < NB * NB / NT; ++q) {
      const int e = t + NT * q, i = e / NB, j = e % NB;
      r1[q] = S.Gs[i][j];
    }
    __syncthreads();
    f = cholqr_pass_wg<T>(A, it.lda, Q, it.ldq, Q, it.ldq, m, n, U64, 0.0, c_retry, max_retries, S);
    if (f) {
      if (t == 0) info[id] = f;
      __syncthreads();
      continue;
    }
    // R = R2 R1: R2 in Gs, R1 into Ws
#pragma unroll
    for (int q = 0; q < NB * NB / NT; ++q) {
      const int e = t + NT * q, i = e / NB, j = e % NB;
      S.Ws[i][j] = r1[q];
    }
    __syncthreads();
    for (int e = t; e < n * n; e += NT) {
      const int i = e % n, j = e / n;
      double s = 0.0;
      if (i <= j)
        for (int k = i; k <= j; ++k) s += S.Gs[i][k] * S.Ws[k][j];
      R[(int64_t)j * it.ldr + i] = (T)s;
    }
    if (t == 0) info[id] = 0;
    __syncthreads();
  }
}

// order[] = instance indices sorted by decreasing cost m^2 n (one workgroup, bitonic sort in LDS).
constexpr int SORT_MAX = 8192;
__global__ __launch_bounds__(1024) void order_kernel(const oqr_batch_item* __restrict__ items, int batch,
                                                     int32_t* __restrict__ order, int32_t* __restrict__ counter,
                                                     int32_t* __restrict__ info) {
  __shared__ unsigned long long key[SORT_MAX];
  const int t = threadIdx.x;
  int p2 = 1;
  while (p2 < batch) p2 <<= 1;
  // key = (2^50 - cost) << 13 | index: ascending keys = descending cost, ties by index
  for (int i = t; i < p2; i += 1024) {
    unsigned long long k = ~0ull;                      // padding sorts last
    if (i < batch) {
      const double cost = fmin((double)items[i].m * items[i].m * items[i].n, 1125899906842624.0);
      k = ((unsigned long long)(1125899906842624.0 - cost) << 13) | (unsigned long long)i;
    }
    key[i] = k;
  }
  __syncthreads();
  for (int size = 2; size <= p2; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = t; i < p2; i += 1024) {
        const int j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const unsigned long long a = key[i], b = key[j];
          if ((a > b) == up) {
            key[i] = b;
            key[j] = a;
          }
        }
      }
      __syncthreads();
    }
  for (int i = t; i < batch; i += 1024) {
    order[i] = (int32_t)(key[i] & (SORT_MAX - 1));
    info[i] = 0;
  }
  if (t == 0) counter[0] = 0;
}

__global__ void identity_order_kernel(int batch, int32_t* order, int32_t* counter, int32_t* info) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < batch) {
    order[i] = i;
    info[i] = 0;
  }
  if (i == 0) counter[0] = 0;
}

struct TileCfg {
  int wg_per_cu;
  int sort;
};
const TileCfg kTiles[] = {{2, 1}, {1, 1}, {2, 1}, {3, 1}, {2, 0}};   // id 0 = default
constexpr int kNumTiles = 4;                                          // ids 1..4

}  // namespace
}  // namespace oqr

using namespace oqr;

extern "C" {

int oqr_batched_tile_count(void) { return kNumTiles; }

size_t oqr_batched_workspace_bytes(int64_t batch, int32_t max_m, int32_t max_n, int32_t dtype) {
  (void)max_m;
  (void)max_n;
  (void)dtype;
  if (batch < 0) return 0;
  return align256(sizeof(int32_t) * 64) + align256(sizeof(int32_t) * (size_t)(batch > 0 ? batch : 1));
}

int oqr_cholqr2_batched(int64_t batch, const oqr_batch_item* items_dev, int32_t dtype, int32_t max_m, int32_t max_n,
                        const oqr_opts* opts, int32_t tile, void* ws, size_t ws_bytes, int32_t* info_dev,
                        void* stream) {
  if (batch < 0 || batch > (1 << 30)) return OQR_E_ARG;
  if (batch == 0) return OQR_OK;
  if (!items_dev || !info_dev || max_m < 1 || max_n < 1 || max_n > NB || max_m < max_n) return OQR_E_ARG;
  if (dtype != OQR_F64 && dtype != OQR_F32) return OQR_E_ARG;
  if (tile < 0 || tile > kNumTiles) return OQR_E_ARG;
  oqr_opts o;
  if (opts) o = *opts;
  else oqr_default_opts(&o);
  if (!(o.shift_c >= 0.0) || o.max_retries < 0 || o.max_retries > 16) return OQR_E_ARG;
  if (o.pass1 != OQR_P_FP64 || o.pass2 != OQR_P_FP64) return OQR_E_UNSUPPORTED;
  const size_t need = oqr_batched_workspace_bytes(batch, max_m, max_n, dtype);
  if (!ws || ws_bytes < need || ((uintptr_t)ws & 255u)) return OQR_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  int32_t* counter = (int32_t*)ws;
  int32_t* order = (int32_t*)((char*)ws + align256(sizeof(int32_t) * 64));
  const TileCfg cfg = kTiles[tile];
  if (cfg.sort && batch <= SORT_MAX)
    order_kernel<<<1, 1024, 0, s>>>(items_dev, (int)batch, order, counter, info_dev);
  else
    identity_order_kernel<<<(unsigned)((batch + 255) / 256), 256, 0, s>>>((int)batch, order, counter, info_dev);
  if (hipGetLastError() != hipSuccess) return OQR_E_HIP;
  // compute-unit count, queried once per device (outside any graph capture: the first call)
  static int cu_count[64] = {0};
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64) {
    if (cu_count[dev] == 0) {
      int v = 0;
      if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
        cu_count[dev] = v;
    }
    if (cu_count[dev] > 0) cus = cu_count[dev];
  }
  int64_t grid = (int64_t)cus * cfg.wg_per_cu;
  if (grid > batch) grid = batch;
  trace_pre(K_BATCH, s);
  if (dtype == OQR_F64)
    batch_kernel<double><<<(unsigned)grid, NT, 0, s>>>(items_dev, order, (int)batch, counter, info_dev, o.shift_c,
                                                       o.max_retries);
  else
    batch_kernel<float><<<(unsigned)grid, NT, 0, s>>>(items_dev, order, (int)batch, counter, info_dev, o.shift_c,
                                                      o.max_retries);
  const hipError_t e = hipGetLastError();
  trace_post(K_BATCH, s);
  return e == hipSuccess ? OQR_OK : OQR_E_HIP;
}

}  // extern "C"
