// Gram matrix G = X^T Y (step 2 of CHOLQR, Algorithm 1: C = Z^T B), upper triangle.
//
// The reduction runs over the m rows.  The grid is (upper 64x64 tiles of G) x
// (row chunks); every workgroup writes its tile of a per-chunk partial in
// FP64, and a second kernel sums the partials in chunk order, so the result is
// deterministic (no atomics).  Only tiles with I <= J are computed; the
// reduction writes both triangles of G from the upper one.
#include "common.hpp"

namespace oqr {
namespace {

constexpr int TB = 64;      // tile edge
constexpr int NT = 256;

struct GramPlan {
  int nb, tiles, chunks, kc;
};

GramPlan plan(int64_t m, int64_t n) {
  GramPlan p;
  p.nb = ceil_div(n, TB);
  p.tiles = p.nb * (p.nb + 1) / 2;
  int want = ceil_div(1024, p.tiles);
  int maxc = ceil_div(m, 256);
  p.chunks = want < maxc ? want : maxc;
  if (p.chunks < 1) p.chunks = 1;
  int64_t kc = (m + p.chunks - 1) / p.chunks;
  kc = (kc + 31) / 32 * 32;
  p.kc = (int)kc;
  p.chunks = ceil_div(m, kc);
  return p;
}

__device__ __forceinline__ void tile_of(int t, int nb, int& I, int& J) {
  // t enumerates the upper tiles row by row: (0,0) (0,1) .. (0,nb-1) (1,1) ..
  int i = 0;
  while (t >= nb - i) { t -= nb - i; ++i; }
  I = i;
  J = i + t;
}

// ---- FP64 ------------------------------------------------------------------------------------
constexpr int BK = 16;
constexpr int PAD = 8;

__global__ __launch_bounds__(NT) void gram_f64_kernel(const double* __restrict__ X, int64_t ldx,
                                                       const double* __restrict__ Y, int64_t ldy, int m, int n,
                                                       int nb, int kc, double* __restrict__ partial) {
  __shared__ double Xs[BK][TB + PAD];
  __shared__ double Ys[BK][TB + PAD];
  int I, J;
  tile_of(blockIdx.x, nb, I, J);
  const int c = blockIdx.y;
  const int r0 = c * kc, r1 = min(m, r0 + kc);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int I0 = I * TB, J0 = J * TB;
  f64x4 acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = f64x4{0, 0, 0, 0};
  const int lk = t % BK, lc = t / BK;   // k = lk, column = lc + 16 r
  double rx[4], ry[4];
  auto load = [&](int k0) {
    const int k = k0 + lk;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int cx = I0 + lc + 16 * r, cy = J0 + lc + 16 * r;
      rx[r] = sel_load(X, (int64_t)cx * ldx + k, k < r1 && cx < n);
      ry[r] = sel_load(Y, (int64_t)cy * ldy + k, k < r1 && cy < n);
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      Xs[lk][lc + 16 * r] = rx[r];
      Ys[lk][lc + 16 * r] = ry[r];
    }
  };
  load(r0);
  store();
  __syncthreads();
  for (int k0 = r0; k0 < r1; k0 += BK) {
    const bool more = k0 + BK < r1;
    if (more) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      const double a = Xs[kr][wave * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[b] = mfma_f64(a, Ys[kr][b * 16 + (lane & 15)], acc[b]);
    }
    __syncthreads();
    if (more) {
      store();
      __syncthreads();
    }
  }
  double* P = partial + (int64_t)c * n * n;
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = I0 + wave * 16 + 4 * r + (lane >> 4);
      const int j = J0 + b * 16 + (lane & 15);
      if (i < n && j < n) P[(int64_t)j * n + i] = acc[b][r];
    }
}

// ---- split bfloat16 ---------------------------------------------------------------------------
constexpr int BKS = 32;
constexpr int KT = 256;
constexpr int SPAD = 8;

template <int S>
__global__ __launch_bounds__(NT) void gram_split_kernel(const double* __restrict__ X, int64_t ldx,
                                                         const double* __restrict__ Y, int64_t ldy, int m, int n,
                                                         int nb, int kc, double* __restrict__ partial) {
  __shared__ __attribute__((aligned(16))) unsigned short Xs[S][TB][BKS + SPAD];
  __shared__ __attribute__((aligned(16))) unsigned short Ys[S][TB][BKS + SPAD];
  int I, J;
  tile_of(blockIdx.x, nb, I, J);
  const int c = blockIdx.y;
  const int r0 = c * kc, r1 = min(m, r0 + kc);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int I0 = I * TB, J0 = J * TB;
  f32x4 acc[4];
  double dacc[4][4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    acc[b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int r = 0; r < 4; ++r) dacc[b][r] = 0.0;
  }
  // thread: column lc = t / 4 (0..63), k = (t % 4) * 8 .. +7
  const int lq = t % 4, lc = t / 4;
  double rx[8], ry[8];
  auto load = [&](int k0) {
    const int cx = I0 + lc, cy = J0 + lc;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + lq * 8 + e;
      rx[e] = sel_load(X, (int64_t)cx * ldx + k, k < r1 && cx < n);
      ry[e] = sel_load(Y, (int64_t)cy * ldy + k, k < r1 && cy < n);
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      unsigned short sx[S], sy[S];
      split_bf16<S>(rx[e], sx);
      split_bf16<S>(ry[e], sy);
#pragma unroll
      for (int s = 0; s < S; ++s) {
        Xs[s][lc][lq * 8 + e] = sx[s];
        Ys[s][lc][lq * 8 + e] = sy[s];
      }
    }
  };
  load(r0);
  store();
  __syncthreads();
  int since = 0;
  for (int k0 = r0; k0 < r1; k0 += BKS) {
    const bool more = k0 + BKS < r1;
    if (more) load(k0 + BKS);
    const int kb = 8 * (lane >> 4);
    bf16x8 a[S], b[S][4];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      a[s] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&Xs[s][wave * 16 + (lane & 15)][kb]));
#pragma unroll
      for (int q = 0; q < 4; ++q)
        b[s][q] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&Ys[s][q * 16 + (lane & 15)][kb]));
    }
#pragma unroll
    for (int p = S - 1; p >= 0; --p)
#pragma unroll
      for (int q = S - 1 - p; q >= 0; --q)
#pragma unroll
        for (int bb = 0; bb < 4; ++bb)
          acc[bb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[p], b[q][bb], acc[bb], 0, 0, 0);
    since += BKS;
    if (since == KT || !more) {
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) dacc[bb][r] += (double)acc[bb][r];
        acc[bb] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
      since = 0;
    }
    __syncthreads();
    if (more) {
      store();
      __syncthreads();
    }
  }
  double* P = partial + (int64_t)c * n * n;
#pragma unroll
  for (int bb = 0; bb < 4; ++bb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = I0 + wave * 16 + 4 * (lane >> 4) + r;
      const int j = J0 + bb * 16 + (lane & 15);
      if (i < n && j < n) P[(int64_t)j * n + i] = dacc[bb][r];
    }
}

// G(i, j) = G(j, i) = sum_c partial[c](i, j) for i <= j, summed in chunk order.
__global__ void gram_reduce_kernel(const double* __restrict__ partial, int n, int chunks, double* __restrict__ G) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int j = (int)(idx / n), i = (int)(idx % n);
  if (i > j) return;
  double s = 0.0;
  for (int c = 0; c < chunks; ++c) s += partial[(int64_t)c * n * n + idx];
  G[(int64_t)j * n + i] = s;
  G[(int64_t)i * n + j] = s;
}

}  // namespace

size_t gram_partial_bytes(int64_t m, int64_t n) {
  GramPlan p = plan(m, n);
  return (size_t)p.chunks * n * n * sizeof(double);
}

static hipError_t reduce(const double* partial, int64_t n, int chunks, double* G, hipStream_t s) {
  const int64_t total = n * n;
  gram_reduce_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(partial, (int)n, chunks, G);
  return hipGetLastError();
}

hipError_t launch_gram_f64(const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t m, int64_t n,
                           double* partial, double* G, hipStream_t s) {
  GramPlan p = plan(m, n);
  gram_f64_kernel<<<dim3(p.tiles, p.chunks), NT, 0, s>>>(X, ldx, Y, ldy, (int)m, (int)n, p.nb, p.kc, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return reduce(partial, n, p.chunks, G, s);
}

hipError_t launch_gram_split(const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t m, int64_t n,
                             int slices, double* partial, double* G, hipStream_t s) {
  GramPlan p = plan(m, n);
  if (slices == 2)
    gram_split_kernel<2><<<dim3(p.tiles, p.chunks), NT, 0, s>>>(X, ldx, Y, ldy, (int)m, (int)n, p.nb, p.kc, partial);
  else
    gram_split_kernel<3><<<dim3(p.tiles, p.chunks), NT, 0, s>>>(X, ldx, Y, ldy, (int)m, (int)n, p.nb, p.kc, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return reduce(partial, n, p.chunks, G, s);
}

}  // namespace oqr
