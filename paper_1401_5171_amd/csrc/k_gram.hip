// Gram matrix G = X^T Y (step 2 of CHOLQR, Algorithm 1: C = Z^T B), upper triangle.
//
// The reduction runs over the m rows.  The grid is (upper 64x64 tiles of G) x
// (row chunks); every workgroup writes its tile of a per-chunk partial in
// FP64, and a second kernel sums the partials in chunk order, so the result is
// deterministic (no atomics).  Only tiles with I <= J are computed; the
// reduction writes both triangles of G from the upper one.
#include <type_traits>

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

// SYM: G = X^T Y + X2^T X (the symmetric assembly Z^T Wsym + Woff^T Z with X = Z, Y = Wsym, X2 = Woff).
// F32 (not with SYM): the FP32 operand Gram, X and Y rounded to FP32 as they leave LDS, products on
// v_mfma_f32_16x16x4_f32, FP32 sums over KT32 rows folded into FP64 (the accumulators then follow the
// FP32 instruction's row layout).
constexpr int KT32 = 256;
template <bool SYM, bool F32 = false>
__global__ __launch_bounds__(NT) void gram_f64_kernel(const double* __restrict__ X, int64_t ldx,
                                                       const double* __restrict__ Y, int64_t ldy,
                                                       const double* __restrict__ X2, int64_t ldx2, int m, int n,
                                                       int nb, int kc, double* __restrict__ partial) {
  __shared__ double Xs[BK][TB + PAD];
  __shared__ double Ys[BK][TB + PAD];
  __shared__ double X2s[SYM ? BK : 1][TB + PAD];    // X2 columns of block I
  __shared__ double XJs[SYM ? BK : 1][TB + PAD];    // X columns of block J
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
  double rx[4], ry[4], rx2[SYM ? 4 : 1], rxj[SYM ? 4 : 1];
  // the 64 columns of blocks I and J through buffer resources based at the block (offsets stay below
  // 2^31 bytes); branch-free loads, lanes past r1 or n masked with kOOB (they read 0), so that the next
  // K step's loads stay in flight during this step's products
  const int wi = min(TB, n - I0), wj = min(TB, n - J0);
  const bufrsrc bx = make_buf(X + (int64_t)I0 * ldx, ((int64_t)(wi - 1) * ldx + m) * 8);
  const bufrsrc by = make_buf(Y + (int64_t)J0 * ldy, ((int64_t)(wj - 1) * ldy + m) * 8);
  const bufrsrc bx2 = make_buf(SYM ? X2 + (int64_t)I0 * ldx2 : X, SYM ? ((int64_t)(wi - 1) * ldx2 + m) * 8 : 0);
  const bufrsrc bxj = make_buf(X + (int64_t)J0 * ldx, ((int64_t)(wj - 1) * ldx + m) * 8);
  auto load = [&](int k0) {
    const int k = k0 + lk;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = lc + 16 * r;
      const uint32_t mx = (k < r1 && I0 + c < n) ? 0u : kOOB, my = (k < r1 && J0 + c < n) ? 0u : kOOB;
      rx[r] = buf_f64(bx, ((uint32_t)((int64_t)c * ldx + k) * 8u) | mx);
      ry[r] = buf_f64(by, ((uint32_t)((int64_t)c * ldy + k) * 8u) | my);
      if (SYM) {
        rx2[r] = buf_f64(bx2, ((uint32_t)((int64_t)c * ldx2 + k) * 8u) | mx);
        rxj[r] = buf_f64(bxj, ((uint32_t)((int64_t)c * ldx + k) * 8u) | my);
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      Xs[lk][lc + 16 * r] = rx[r];
      Ys[lk][lc + 16 * r] = ry[r];
      if (SYM) {
        X2s[lk][lc + 16 * r] = rx2[r];
        XJs[lk][lc + 16 * r] = rxj[r];
      }
    }
  };
  static_assert(!(SYM && F32), "the FP32 Gram has no symmetric assembly");
  f32x4 acc32[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc32[b] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto fold32 = [&]() {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[b][r] += (double)acc32[b][r];
      acc32[b] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  };
  load(r0);
  store();
  __syncthreads();
  int step = 0;
  for (int k0 = r0; k0 < r1; k0 += BK) {
    const bool more = k0 + BK < r1;
    load(k0 + BK);                        // past r1: zeros, never stored
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      const double a = Xs[kr][wave * 16 + (lane & 15)];
      if constexpr (F32) {
        const float a32 = (float)a;
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc32[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a32, (float)Ys[kr][b * 16 + (lane & 15)], acc32[b], 0, 0, 0);
      } else {
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[b] = mfma_f64(a, Ys[kr][b * 16 + (lane & 15)], acc[b]);
      }
      if (SYM) {
        const double a2 = X2s[kr][wave * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[b] = mfma_f64(a2, XJs[kr][b * 16 + (lane & 15)], acc[b]);
      }
    }
    if (F32 && ++step == KT32 / BK) {
      fold32();
      step = 0;
    }
    __syncthreads();
    if (more) {
      store();
      __syncthreads();
    }
  }
  if (F32) fold32();
  double* P = partial + (int64_t)c * n * n;
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = I0 + wave * 16 + (F32 ? 4 * (lane >> 4) + r : 4 * r + (lane >> 4));
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
  // blocks I and J through buffer resources based at the block; branch-free loads masked with kOOB
  // past r1 or n, so that the next K step's loads overlap this step's products
  const bufrsrc bx = make_buf(X + (int64_t)I0 * ldx, ((int64_t)(min(TB, n - I0) - 1) * ldx + m) * 8);
  const bufrsrc by = make_buf(Y + (int64_t)J0 * ldy, ((int64_t)(min(TB, n - J0) - 1) * ldy + m) * 8);
  auto load = [&](int k0) {
    const uint32_t cmx = I0 + lc < n ? 0u : kOOB, cmy = J0 + lc < n ? 0u : kOOB;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + lq * 8 + e;
      const uint32_t km = k < r1 ? 0u : kOOB;
      rx[e] = buf_f64(bx, ((uint32_t)((int64_t)lc * ldx + k) * 8u) | cmx | km);
      ry[e] = buf_f64(by, ((uint32_t)((int64_t)lc * ldy + k) * 8u) | cmy | km);
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
    load(k0 + BKS);                       // past r1: zeros, never stored
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

// ---- all upper tiles per workgroup (n <= 128) ---------------------------------------------------
// One workgroup owns a chunk of rows and every upper 64x64 tile of G, so X and Y are read once.  Tile
// loads are unconditional buffer loads (rows past m read as zero) issued one K step ahead and consumed
// only at the next LDS store.  One buffer resource per 64-column block keeps offsets below 2 GB.
constexpr int NCH_FULL = 512;    // target number of row chunks

struct FullPlan {
  int chunks, kc;
};
FullPlan full_plan(int64_t m, int kstep) {
  FullPlan p;
  int64_t kc = (m + NCH_FULL - 1) / NCH_FULL;
  if (kc < 64) kc = 64;
  kc = (kc + kstep - 1) / kstep * kstep;
  p.kc = (int)kc;
  p.chunks = ceil_div(m, kc);
  return p;
}

__device__ __forceinline__ bufrsrc block_buf(const double* base, int64_t ld, int m, int n, int r0, int c0) {
  const int cols = min(TB, n - c0);
  return make_buf(base + (int64_t)c0 * ld + r0, ((int64_t)(cols - 1) * ld + (m - r0)) * 8);
}

template <int NBT, bool SYM>
__global__ __launch_bounds__(NT, 2) void gram_full_f64_kernel(const double* __restrict__ X, int64_t ldx,
                                                             const double* __restrict__ Y, int64_t ldy,
                                                             const double* __restrict__ X2, int64_t ldx2, int m,
                                                             int n, int kc, double* __restrict__ partial) {
  __shared__ double Xs[NBT][BK][TB + 1];
  __shared__ double Ys[NBT][BK][TB + 1];
  __shared__ double X2s[SYM ? NBT : 1][BK][TB + 1];
  const int c = blockIdx.x;
  const int r0 = c * kc, r1 = min(m, r0 + kc);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int li = lane >> 4, lj = lane & 15;
  bufrsrc xb[NBT], yb[NBT], x2b[NBT];
#pragma unroll
  for (int b = 0; b < NBT; ++b) {
    xb[b] = block_buf(X, ldx, m, n, r0, b * TB);
    yb[b] = block_buf(Y, ldy, m, n, r0, b * TB);
    if (SYM) x2b[b] = block_buf(X2, ldx2, m, n, r0, b * TB);
  }
  // thread: k = t % BK, columns lc + 16 q (q = 0..3) of each block
  const int lk = t % BK, lc = t / BK;
  double rx[NBT][4], ry[NBT][4], rx2[SYM ? NBT : 1][4];
  auto load = [&](int k0) {
    const int k = k0 + lk;                    // absolute row
#pragma unroll
    for (int b = 0; b < NBT; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int col = lc + 16 * q;
        const uint32_t ox = (k < r1) ? (uint32_t)((int64_t)col * ldx + (k - r0)) * 8u : kOOB;
        const uint32_t oy = (k < r1) ? (uint32_t)((int64_t)col * ldy + (k - r0)) * 8u : kOOB;
        rx[b][q] = buf_f64(xb[b], ox);
        ry[b][q] = buf_f64(yb[b], oy);
        if (SYM) {
          const uint32_t o2 = (k < r1) ? (uint32_t)((int64_t)col * ldx2 + (k - r0)) * 8u : kOOB;
          rx2[b][q] = buf_f64(x2b[b], o2);
        }
      }
  };
  // Of the diagonal tiles only the 16 x 16 blocks on or above the diagonal are formed (the reduction
  // reads the upper triangle): with two column blocks, wave w takes row band w of tile (0,0) and band
  // 3 - w of tile (1,1), blocks q >= band (five per wave); with one, the ten blocks are dealt to the
  // waves in turn (block w + 4 v).  The off-diagonal tile (0,1): band w, all four column blocks.
  // Every entry sums the same products in the same order as when whole tiles were formed.
  const int wb = __builtin_amdgcn_readfirstlane(wave);
  f64x4 acc[NBT == 2 ? 1 : 1][4], accd[2][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[0][q] = accd[0][q] = accd[1][q] = f64x4{0, 0, 0, 0};
  auto d1 = [](int d, int& rb, int& qb) {       // block d of a lone diagonal tile, row order
    rb = d < 4 ? 0 : (d < 7 ? 1 : (d < 9 ? 2 : 3));
    qb = d < 4 ? d : (d < 7 ? d - 3 : (d < 9 ? d - 5 : 3));
  };
  load(r0);
  for (int k0 = r0; k0 < r1; k0 += BK) {
#pragma unroll
    for (int b = 0; b < NBT; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        Xs[b][lk][lc + 16 * q] = rx[b][q];
        Ys[b][lk][lc + 16 * q] = ry[b][q];
        if (SYM) X2s[b][lk][lc + 16 * q] = rx2[b][q];
      }
    __syncthreads();
    load(k0 + BK);                            // past r1: kOOB, zeros
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + li;
      if constexpr (NBT == 2) {
        {
          const double a = Xs[0][kr][wb * 16 + lj];
          const double a2 = SYM ? X2s[0][kr][wb * 16 + lj] : 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            acc[0][q] = mfma_f64(a, Ys[1][kr][q * 16 + lj], acc[0][q]);
            if (SYM) acc[0][q] = mfma_f64(a2, Xs[1][kr][q * 16 + lj], acc[0][q]);
          }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int b = h ? 3 - wb : wb;       // wave-uniform: the tests below branch
          const double a = Xs[h][kr][b * 16 + lj];
          const double a2 = SYM ? X2s[h][kr][b * 16 + lj] : 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (q >= b) {
              accd[h][q] = mfma_f64(a, Ys[h][kr][q * 16 + lj], accd[h][q]);
              if (SYM) accd[h][q] = mfma_f64(a2, Xs[h][kr][q * 16 + lj], accd[h][q]);
            }
        }
      } else {
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          const int d = wb + 4 * v;
          if (d < 10) {
            int rb, qb;
            d1(d, rb, qb);
            const double a = Xs[0][kr][rb * 16 + lj];
            const double a2 = SYM ? X2s[0][kr][rb * 16 + lj] : 0.0;
            accd[0][v] = mfma_f64(a, Ys[0][kr][qb * 16 + lj], accd[0][v]);
            if (SYM) accd[0][v] = mfma_f64(a2, Xs[0][kr][qb * 16 + lj], accd[0][v]);
          }
        }
      }
    }
    __syncthreads();
  }
  double* P = partial + (int64_t)c * n * n;
  auto put = [&](int i0, int j0, const f64x4& v) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + 4 * r + li, j = j0 + lj;
      if (i < n && j < n) P[(int64_t)j * n + i] = v[r];
    }
  };
  if constexpr (NBT == 2) {
#pragma unroll
    for (int q = 0; q < 4; ++q) put(wb * 16, TB + q * 16, acc[0][q]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int b = h ? 3 - wb : wb;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q >= b) put(h * TB + b * 16, h * TB + q * 16, accd[h][q]);
    }
  } else {
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      const int d = wb + 4 * v;
      if (d < 10) {
        int rb, qb;
        d1(d, rb, qb);
        put(rb * 16, qb * 16, accd[0][v]);
      }
    }
  }
}

// ---- all upper tiles per workgroup, 128 < n <= 256, symmetric assembly from layers --------------
// G = Z^T W + W^T Z (upper triangle) with W = sum_h Y_h, the H partial layers of the product summed as
// they are loaded (in layer order, as the layer sum would): the FP64 dense pass's W' = T Z needs no
// separate sum.  Eight waves, one workgroup per CU; a workgroup owns a chunk of rows and the ten upper
// 64 x 64 tiles, so Z and W are read once: waves 0-3 take tiles (0,1) (0,2) (0,3) and the diagonal
// tiles (0,0) (1,1), waves 4-7 tiles (1,2) (1,3) (2,3) and (2,2) (3,3).  Wave w (b = w & 3) owns rows
// 16 b .. 16 b + 15 of block I of its off-diagonal tiles and of its first diagonal tile, and rows
// 16 (3 - b) .. of its second; in a diagonal tile only the 16 x 16 blocks on or above the diagonal are
// formed, so every wave forms 4 - b + b + 1 = 5 of them.  Every entry sums the same products in the
// same order as when whole diagonal tiles were formed.
constexpr int NTW = 512, NBW = 4, WOFF = 3;
constexpr int WO_I[2][WOFF] = {{0, 0, 0}, {1, 1, 2}};
constexpr int WO_J[2][WOFF] = {{1, 2, 3}, {2, 3, 3}};
constexpr int WD_T[2][2] = {{0, 1}, {2, 3}};

FullPlan wide_plan(int64_t m) {
  FullPlan p;
  const int cus = device_cu_count();
  int64_t kc = (m + cus - 1) / cus;
  if (kc < BK) kc = BK;
  kc = (kc + BK - 1) / BK * BK;
  p.kc = (int)kc;
  p.chunks = ceil_div(m, kc);
  return p;
}

template <int G>
__device__ __forceinline__ void wide_tiles(const double (&Xs)[NBW][BK][TB + 1], const double (&Ys)[NBW][BK][TB + 1],
                                           int kr, int wb, int lj, f64x4 (&acc)[WOFF][4], f64x4 (&accd)[2][4]) {
#pragma unroll
  for (int u = 0; u < WOFF; ++u) {
    const int I = WO_I[G][u], J = WO_J[G][u];
    const double a = Xs[I][kr][16 * wb + lj], a2 = Ys[I][kr][16 * wb + lj];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc[u][q] = mfma_f64(a, Ys[J][kr][q * 16 + lj], acc[u][q]);
      acc[u][q] = mfma_f64(a2, Xs[J][kr][q * 16 + lj], acc[u][q]);
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int I = WD_T[G][h], b = h ? 3 - wb : wb;   // wb is wave-uniform (scalar): the tests branch
    const double a = Xs[I][kr][16 * b + lj], a2 = Ys[I][kr][16 * b + lj];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q >= b) {
        accd[h][q] = mfma_f64(a, Ys[I][kr][q * 16 + lj], accd[h][q]);
        accd[h][q] = mfma_f64(a2, Xs[I][kr][q * 16 + lj], accd[h][q]);
      }
  }
}

__global__ __launch_bounds__(NTW, 1) void gram_wide_symm_kernel(const double* __restrict__ X, int64_t ldx,
                                                                 const double* __restrict__ Y, int64_t ldy,
                                                                 int64_t ystride, int layers, int m, int n, int kc,
                                                                 double* __restrict__ partial) {
  __shared__ double Xs[NBW][BK][TB + 1];
  __shared__ double Ys[NBW][BK][TB + 1];
  const int c = blockIdx.x;
  const int r0 = c * kc, r1 = min(m, r0 + kc);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int li = lane >> 4, lj = lane & 15;
  const int grp = wave >> 2, wb = __builtin_amdgcn_readfirstlane(wave & 3);
  // thread: row k = t % BK of the step, columns lc + 32 q (q = 0..7); columns past n lie beyond the
  // size bound of the resource and read zero, rows past r1 are masked
  const int lk = t % BK, lc = t / BK;
  const bufrsrc xb = make_buf(X + r0, ((int64_t)(n - 1) * ldx + (m - r0)) * 8);
  double rx[8], ry[8];
  auto load = [&](int k0) {
    const int k = k0 + lk;
    const uint32_t mk = k < r1 ? 0u : kOOB;
#pragma unroll
    for (int q = 0; q < 8; ++q) rx[q] = buf_f64(xb, ((uint32_t)((int64_t)(lc + 32 * q) * ldx + (k - r0)) * 8u) | mk);
#pragma unroll
    for (int q = 0; q < 8; ++q) ry[q] = 0.0;
    for (int h = 0; h < layers; ++h) {
      const bufrsrc yb = make_buf(Y + h * ystride + r0, ((int64_t)(n - 1) * ldy + (m - r0)) * 8);
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = buf_f64(yb, ((uint32_t)((int64_t)(lc + 32 * q) * ldy + (k - r0)) * 8u) | mk);
#pragma unroll
      for (int q = 0; q < 8; ++q) ry[q] += v[q];
    }
  };
  f64x4 acc[WOFF][4], accd[2][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int u = 0; u < WOFF; ++u) acc[u][q] = f64x4{0, 0, 0, 0};
    accd[0][q] = accd[1][q] = f64x4{0, 0, 0, 0};
  }
  load(r0);
  for (int k0 = r0; k0 < r1; k0 += BK) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int col = lc + 32 * q;
      Xs[col >> 6][lk][col & 63] = rx[q];
      Ys[col >> 6][lk][col & 63] = ry[q];
    }
    __syncthreads();
    load(k0 + BK);                            // past r1: masked, zeros
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      if (grp == 0) wide_tiles<0>(Xs, Ys, kk + li, wb, lj, acc, accd);
      else wide_tiles<1>(Xs, Ys, kk + li, wb, lj, acc, accd);
    }
    __syncthreads();
  }
  double* P = partial + (int64_t)c * n * n;
#pragma unroll
  for (int u = 0; u < WOFF; ++u) {
    const int I = grp ? WO_I[1][u] : WO_I[0][u], J = grp ? WO_J[1][u] : WO_J[0][u];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = I * TB + 16 * wb + 4 * r + li;
        const int j = J * TB + q * 16 + lj;
        if (i < n && j < n) P[(int64_t)j * n + i] = acc[u][q][r];
      }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int I = grp ? WD_T[1][h] : WD_T[0][h], b = h ? 3 - wb : wb;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q >= b) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = I * TB + 16 * b + 4 * r + li;
          const int j = I * TB + q * 16 + lj;
          if (i < n && j < n) P[(int64_t)j * n + i] = accd[h][q][r];
        }
      }
  }
}

template <int S, int NBT>
__global__ __launch_bounds__(NT, 2) void gram_full_split_kernel(const double* __restrict__ X, int64_t ldx,
                                                               const double* __restrict__ Y, int64_t ldy, int m,
                                                               int n, int kc, double* __restrict__ partial) {
  __shared__ __attribute__((aligned(16))) unsigned short Xs[NBT][S][TB][BKS + SPAD];
  __shared__ __attribute__((aligned(16))) unsigned short Ys[NBT][S][TB][BKS + SPAD];
  const int c = blockIdx.x;
  const int r0 = c * kc, r1 = min(m, r0 + kc);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  bufrsrc xb[NBT], yb[NBT];
#pragma unroll
  for (int b = 0; b < NBT; ++b) {
    xb[b] = block_buf(X, ldx, m, n, r0, b * TB);
    yb[b] = block_buf(Y, ldy, m, n, r0, b * TB);
  }
  // thread: column lc = t / 4 (0..63) of each block, rows (t % 4) * 8 .. +7
  const int lq = t % 4, lc = t / 4;
  double rx[NBT][8], ry[NBT][8];
  auto load = [&](int k0) {
#pragma unroll
    for (int b = 0; b < NBT; ++b)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = k0 + lq * 8 + e;
        const uint32_t ox = (k < r1) ? (uint32_t)((int64_t)lc * ldx + (k - r0)) * 8u : kOOB;
        const uint32_t oy = (k < r1) ? (uint32_t)((int64_t)lc * ldy + (k - r0)) * 8u : kOOB;
        rx[b][e] = buf_f64(xb[b], ox);
        ry[b][e] = buf_f64(yb[b], oy);
      }
  };
  constexpr int NTILE = NBT * (NBT + 1) / 2;
  f32x4 acc[NTILE][4];
  double dacc[NTILE][4][4];
#pragma unroll
  for (int u = 0; u < NTILE; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc[u][q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) dacc[u][q][r] = 0.0;
    }
  load(r0);
  int since = 0;
  for (int k0 = r0; k0 < r1; k0 += BKS) {
#pragma unroll
    for (int b = 0; b < NBT; ++b)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        unsigned short sx[S], sy[S];
        split_bf16<S>(rx[b][e], sx);
        split_bf16<S>(ry[b][e], sy);
#pragma unroll
        for (int s2 = 0; s2 < S; ++s2) {
          Xs[b][s2][lc][lq * 8 + e] = sx[s2];
          Ys[b][s2][lc][lq * 8 + e] = sy[s2];
        }
      }
    __syncthreads();
    load(k0 + BKS);
    const int kb = 8 * (lane >> 4);
    int u = 0;
#pragma unroll
    for (int I = 0; I < NBT; ++I) {
      bf16x8 a[S];
#pragma unroll
      for (int s2 = 0; s2 < S; ++s2)
        a[s2] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&Xs[I][s2][wave * 16 + (lane & 15)][kb]));
#pragma unroll
      for (int J = I; J < NBT; ++J, ++u) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          bf16x8 b[S];
#pragma unroll
          for (int s2 = 0; s2 < S; ++s2)
            b[s2] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&Ys[J][s2][q * 16 + (lane & 15)][kb]));
#pragma unroll
          for (int p = S - 1; p >= 0; --p)
#pragma unroll
            for (int q2 = S - 1 - p; q2 >= 0; --q2)
              acc[u][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[p], b[q2], acc[u][q], 0, 0, 0);
        }
      }
    }
    since += BKS;
    if (since == KT || k0 + BKS >= r1) {
#pragma unroll
      for (int u2 = 0; u2 < NTILE; ++u2)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
          for (int r = 0; r < 4; ++r) dacc[u2][q][r] += (double)acc[u2][q][r];
          acc[u2][q] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
      since = 0;
    }
    __syncthreads();
  }
  double* P = partial + (int64_t)c * n * n;
  int u = 0;
#pragma unroll
  for (int I = 0; I < NBT; ++I)
#pragma unroll
    for (int J = I; J < NBT; ++J, ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = I * TB + wave * 16 + 4 * (lane >> 4) + r;
          const int j = J * TB + q * 16 + (lane & 15);
          if (i < n && j < n) P[(int64_t)j * n + i] = dacc[u][q][r];
        }
}

// G(i, j) = G(j, i) = sum_c partial[c](i, j) for i <= j.  Eight interleaved partial sums (chunk c goes
// to sum c mod 8) keep eight loads in flight; they are combined in a fixed order, so the result does
// not depend on timing.
// A workgroup reduces 64 consecutive entries with eight waves: wave u sums the partials of chunks u,
// u + 8, u + 16, ... in that order (64 consecutive entries per load: coalesced), and the eight sums of
// an entry (i <= j) are combined as ((s0 + s1) + (s2 + s3)) + ((s4 + s5) + (s6 + s7)) through LDS; both
// triangles of G are written.
__global__ __launch_bounds__(512) void gram_reduce_kernel(const double* __restrict__ partial, int n, int chunks,
                                                          double* __restrict__ G) {
  __shared__ double sh[8][64];
  const int u = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t idx = (int64_t)blockIdx.x * 64 + l, nn = (int64_t)n * n;
  const int j = (int)(idx / n), i = (int)(idx % n);
  const bool active = idx < nn && i <= j;
  double s = 0.0;
  if (active) {
    int c = u;
    for (; c + 56 < chunks; c += 64) {        // eight loads in flight, added in chunk order
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = partial[(int64_t)(c + 8 * q) * nn + idx];
#pragma unroll
      for (int q = 0; q < 8; ++q) s += v[q];
    }
    for (; c < chunks; c += 8) s += partial[(int64_t)c * nn + idx];
  }
  sh[u][l] = s;
  __syncthreads();
  if (u == 0 && active) {
    const double t = ((sh[0][l] + sh[1][l]) + (sh[2][l] + sh[3][l])) + ((sh[4][l] + sh[5][l]) + (sh[6][l] + sh[7][l]));
    G[(int64_t)j * n + i] = t;
    G[(int64_t)i * n + j] = t;
  }
}


// ---- G = Z^T (A Z) for the 7-point operator, A Z never stored -----------------------------------
// Steps 1 and 2 of CHOLQR (Algorithm 1) in one pass when A is the matrix-free stencil: the operand Y
// of the Gram product is A Z, formed in registers from Z, so A Z costs no HBM traffic.  A workgroup
// owns SP = 16 consecutive points p of the grid plane and a range of planes z, and marches through z:
// each K step is the 16 rows k = z nx ny + p of all n columns.  A 16-lane row of a wave holds the 16
// points of one column, so
//   x-neighbours: the lane to the left or right (DPP row shift); the two points beyond the region's
//                 ends are loaded by lanes 0 and 15 only;
//   z-neighbours: planes z - 1 and z + 1 of the same lane, kept in registers as the march goes on;
//   y-neighbours: two loads (rows +-nx, L2 hits: regions adjacent in y run on the same XCD).
// Out-of-grid neighbours read as zero (buffer loads past the resource, or masked).
constexpr int SP = 16;     // plane points per region = rows per K step

// v = old where the DPP source lane lies outside the 16-lane row
template <int CTRL>
__device__ __forceinline__ double row_shift(double old, double v) {
  const long long o = __double_as_longlong(old), x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)o, (int)x, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(x >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int DPP_ROW_SHL1 = 0x101;   // lane i reads lane i + 1
constexpr int DPP_ROW_SHR1 = 0x111;   // lane i reads lane i - 1

template <int NBT>
__global__ __launch_bounds__(NT, 2) void stencil_gram_kernel(const double* __restrict__ Z, int64_t ldz, int n,
                                                            int nx, int ny, int nz, double center, double off,
                                                            int nreg, int zparts, int zlen,
                                                            double* __restrict__ partial) {
  constexpr int NQ = 4 * NBT;                 // columns per thread: cg + 16 q
  __shared__ double Xs[NBT][SP][TB + 1];
  __shared__ double Ys[NBT][SP][TB + 1];
  const int G = gridDim.x;
  const int L = (G & 7) ? (int)blockIdx.x : (int)(blockIdx.x & 7) * (G >> 3) + (int)(blockIdx.x >> 3);
  const int reg0 = L / zparts, zpart = L % zparts, nrb = G / zparts;   // regions reg0, reg0 + nrb, ...
  const int z0 = zpart * zlen, z1 = min(nz, z0 + zlen);
  const int sxy = nx * ny;
  const int m = sxy * nz;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int li = lane >> 4, lj = lane & 15;
  const int lk = lane & 15, cg = t >> 4;      // point p0 + lk, columns cg + 16 q
  // one buffer resource per 16-column group (scalar registers): column cg of group g is column
  // 16 g + cg of Z, and a thread's offsets are the same in every group
  bufrsrc zb[NQ];
#pragma unroll
  for (int g = 0; g < NQ; ++g) {
    const int c0 = 16 * g, cols = min(16, n - c0);
    zb[g] = make_buf(Z + (int64_t)c0 * ldz, cols > 0 ? ((int64_t)(cols - 1) * ldz + m) * 8 : 0);
  }
  // per region: the thread's point, its neighbour masks and offsets.  Invalid loads get bit 31 of the
  // offset set (past every resource: zero); masks are ORed after the plane offset is added, rather
  // than selected, so that the compiler keeps one unconditional load.  Lane 0 loads the point before
  // the region, lane 15 the point after it (the x-neighbours beyond the DPP row).
  bool in = false, xl = false, xr = false;
  uint32_t o_c = 0, m_c = 0, m_e = 0, m_ym = 0, m_yp = 0, o_e = 0, o_ym = 0, o_yp = 0;
  auto set_region = [&](int reg) {
    const int p = reg * SP + lk;
    in = p < sxy;
    const int x = p % nx, y = p / nx;
    xl = in && x > 0;
    xr = in && x < nx - 1;
    const bool yl = in && y > 0, yr = in && y < ny - 1;
    const int de = (lk == 0 && xl) ? -1 : (lk == SP - 1 && xr) ? 1 : 0;
    o_c = (uint32_t)(((int64_t)cg * ldz + p) * 8);
    m_c = in ? 0u : kOOB;
    m_e = de ? 0u : kOOB;
    m_ym = yl ? 0u : kOOB;
    m_yp = yr ? 0u : kOOB;
    o_e = o_c + (uint32_t)(de * 8);
    o_ym = o_c - (uint32_t)nx * 8u;
    o_yp = o_c + (uint32_t)nx * 8u;
  };
  auto plane = [&](int zz) -> uint32_t { return (uint32_t)zz * (uint32_t)sxy * 8u; };
  // the centres of planes z - 1, z, z + 1 rotate through three arrays (static roles after unrolling)
  double ca[NQ], cbv[NQ], cc[NQ], e[NQ], ym[NQ], yp[NQ];
  // centre of plane zz (zero outside the grid)
  auto load_c = [&](double (&v)[NQ], int zz) {
    const uint32_t mz = (zz >= 0 && zz < nz) ? 0u : kOOB;
    const uint32_t oc = (o_c + plane(zz)) | (m_c | mz);
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = buf_f64(zb[q], oc);
  };
  // edge and y-neighbours of plane zz
  auto load_n = [&](int zz) {
    const uint32_t mz = zz < z1 ? 0u : kOOB, pz = plane(zz);
    const uint32_t oe = (o_e + pz) | (m_e | mz), om = (o_ym + pz) | (m_ym | mz), op = (o_yp + pz) | (m_yp | mz);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      e[q] = buf_f64(zb[q], oe);
      ym[q] = buf_f64(zb[q], om);
      yp[q] = buf_f64(zb[q], op);
    }
  };
  // Diagonal tiles (I, I): only their 16 x 16 blocks on or above the diagonal are needed (10 of 16);
  // those NBT x 10 blocks are dealt to the waves in turn (block wave + 4 v), so that no wave computes
  // a block the reduction never reads.  Off-diagonal tiles: wave w owns their rows 16 w .. 16 w + 15.
  // Every output element accumulates over the same K in the same order either way.
  constexpr int ND = 10 * NBT, DV = (ND + 3) / 4, NOFF = NBT * (NBT - 1) / 2;
  f64x4 accd[DV];
  f64x4 acco[NOFF > 0 ? NOFF : 1][4];
#pragma unroll
  for (int v = 0; v < DV; ++v) accd[v] = f64x4{0, 0, 0, 0};
#pragma unroll
  for (int u = 0; u < (NOFF > 0 ? NOFF : 1); ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) acco[u][q] = f64x4{0, 0, 0, 0};
  // block d of the diagonal tiles: tile d / 10, then (row block, column block) in row order
  auto dblock = [](int d, int& I, int& rb, int& qb) {
    I = d / 10;
    const int r = d % 10;
    rb = r < 4 ? 0 : (r < 7 ? 1 : (r < 9 ? 2 : 3));
    qb = r < 4 ? r : (r < 7 ? r - 3 : (r < 9 ? r - 5 : 3));
  };
  // plane z: cm, c0, cp hold the centres of z - 1, z, z + 1; cm is refilled with plane z + 2
  auto step = [&](int z, double (&cm)[NQ], double (&c0)[NQ], double (&cp)[NQ]) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double xm = row_shift<DPP_ROW_SHR1>(e[q], c0[q]);
      double xp = row_shift<DPP_ROW_SHL1>(e[q], c0[q]);
      xm = xl ? xm : 0.0;
      xp = xr ? xp : 0.0;
      const double w = center * c0[q] + off * (((xm + xp) + (ym[q] + yp[q])) + (cm[q] + cp[q]));
      Xs[q >> 2][lk][cg + 16 * (q & 3)] = c0[q];
      Ys[q >> 2][lk][cg + 16 * (q & 3)] = in ? w : 0.0;
    }
    __syncthreads();
    load_c(cm, z + 2);
    load_n(z + 1);
#pragma unroll
    for (int kk = 0; kk < SP; kk += 4) {
      const int kr = kk + li;
#pragma unroll
      for (int v = 0; v < DV; ++v) {
        const int d = wave + 4 * v;
        if (d < ND) {                          // wave-uniform
          int I, rb, qb;
          dblock(d, I, rb, qb);
          accd[v] = mfma_f64(Xs[I][kr][rb * 16 + lj], Ys[I][kr][qb * 16 + lj], accd[v]);
        }
      }
      int u = 0;
#pragma unroll
      for (int I = 0; I < NBT; ++I) {
        const double a = Xs[I][kr][wave * 16 + lj];
#pragma unroll
        for (int J = I + 1; J < NBT; ++J, ++u)
#pragma unroll
          for (int q = 0; q < 4; ++q) acco[u][q] = mfma_f64(a, Ys[J][kr][q * 16 + lj], acco[u][q]);
      }
    }
    __syncthreads();
  };
  for (int reg = reg0; reg < nreg; reg += nrb) {
    set_region(reg);
    load_c(ca, z0 - 1);
    load_c(cbv, z0);
    load_c(cc, z0 + 1);
    load_n(z0);
    for (int z = z0; z < z1; z += 3) {
      step(z, ca, cbv, cc);
      if (z + 1 < z1) step(z + 1, cbv, cc, ca);
      if (z + 2 < z1) step(z + 2, cc, ca, cbv);
    }
  }
  double* P = partial + (int64_t)blockIdx.x * n * n;
#pragma unroll
  for (int v = 0; v < DV; ++v) {
    const int d = wave + 4 * v;
    if (d < ND) {
      int I, rb, qb;
      dblock(d, I, rb, qb);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = I * TB + rb * 16 + 4 * r + li;
        const int j = I * TB + qb * 16 + lj;
        if (i < n && j < n) P[(int64_t)j * n + i] = accd[v][r];
      }
    }
  }
  int u = 0;
#pragma unroll
  for (int I = 0; I < NBT; ++I)
#pragma unroll
    for (int J = I + 1; J < NBT; ++J, ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = I * TB + wave * 16 + 4 * r + li;
          const int j = J * TB + q * 16 + lj;
          if (i < n && j < n) P[(int64_t)j * n + i] = acco[u][q][r];
        }
}

// ---- split-bfloat16 variant of the fused stencil Gram --------------------------------------------
// Same march, DPP neighbours and register rotation as stencil_gram_kernel.  The thread that forms an
// element of X = Z and Y = A Z (in FP64) rounds both to FP32 and splits them into S bfloat16 slices in
// LDS (as the split operator product does), so every element is split once; the products with slice indices p + q < S run on
// v_mfma_f32_16x16x16_bf16 (K = 16 = one plane), accumulated in FP32 over KT rows and then folded into
// FP64, as in the unfused split Gram.  512 threads (two waves per SIMD): a thread holds columns
// cg + 32 j of its point; wave w owns the 16-row block w & 3 of every output tile and half w >> 2 of
// the (tile, column block) pairs.
constexpr int NT2 = 512;
constexpr int SKP = 4;     // LDS padding (bf16 elements) after a column's 16 k values

typedef short s16x4 __attribute__((ext_vector_type(4)));

// upper 64 x 64 tiles in order (0,0) (0,1) (1,1) for two column blocks, (0,0) for one
__host__ __device__ constexpr int tile_row(int u, int nbt) { return nbt == 1 ? 0 : (u == 2 ? 1 : 0); }
__host__ __device__ constexpr int tile_col(int u, int nbt) { return nbt == 1 ? 0 : (u == 0 ? 0 : 1); }

template <int S, int NBT>
__global__ __launch_bounds__(NT2, 1) void stencil_gram_split_kernel(const double* __restrict__ Z, int64_t ldz, int n,
                                                                   int nx, int ny, int nz, double center,
                                                                   double off, int nreg, int zparts, int zlen,
                                                                   double* __restrict__ partial) {
  constexpr int NQ = 2 * NBT;                 // columns per thread: cg + 32 j
  constexpr int NTILE = NBT * (NBT + 1) / 2;
  constexpr int NP = 2 * NTILE;               // (tile, column block) pairs per wave
  __shared__ __attribute__((aligned(16))) unsigned short Xs[NBT][S][TB][SP + SKP];
  __shared__ __attribute__((aligned(16))) unsigned short Ys[NBT][S][TB][SP + SKP];
  const int G = gridDim.x;
  const int L = (G & 7) ? (int)blockIdx.x : (int)(blockIdx.x & 7) * (G >> 3) + (int)(blockIdx.x >> 3);
  const int reg0 = L / zparts, zpart = L % zparts, nrb = G / zparts;   // regions reg0, reg0 + nrb, ...
  const int z0 = zpart * zlen, z1 = min(nz, z0 + zlen);
  const int sxy = nx * ny;
  const int m = sxy * nz;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int lk = lane & 15, cg = t >> 4;      // point p0 + lk; columns cg + 32 j
  const int kq = lane >> 4, lj = lane & 15;   // MFMA fragment: k = 4 kq .. 4 kq + 3, row / column lj
  const int rb = wave & 3, hf = wave >> 2;
  // one buffer resource per 32-column group; column cg of group g is column 32 g + cg of Z
  bufrsrc zb[NQ];
#pragma unroll
  for (int g = 0; g < NQ; ++g) {
    const int c0 = 32 * g, cols = min(32, n - c0);
    zb[g] = make_buf(Z + (int64_t)c0 * ldz, cols > 0 ? ((int64_t)(cols - 1) * ldz + m) * 8 : 0);
  }
  bool in = false, xl = false, xr = false;
  uint32_t o_c = 0, m_c = 0, m_e = 0, m_ym = 0, m_yp = 0, o_e = 0, o_ym = 0, o_yp = 0;
  auto set_region = [&](int reg) {       // as in stencil_gram_kernel
    const int p = reg * SP + lk;
    in = p < sxy;
    const int x = p % nx, y = p / nx;
    xl = in && x > 0;
    xr = in && x < nx - 1;
    const bool yl = in && y > 0, yr = in && y < ny - 1;
    const int de = (lk == 0 && xl) ? -1 : (lk == SP - 1 && xr) ? 1 : 0;
    o_c = (uint32_t)(((int64_t)cg * ldz + p) * 8);
    m_c = in ? 0u : kOOB;
    m_e = de ? 0u : kOOB;
    m_ym = yl ? 0u : kOOB;
    m_yp = yr ? 0u : kOOB;
    o_e = o_c + (uint32_t)(de * 8);
    o_ym = o_c - (uint32_t)nx * 8u;
    o_yp = o_c + (uint32_t)nx * 8u;
  };
  auto plane = [&](int zz) -> uint32_t { return (uint32_t)zz * (uint32_t)sxy * 8u; };
  double ca[NQ], cbv[NQ], cc[NQ], e[NQ], ym[NQ], yp[NQ];
  auto load_c = [&](double (&v)[NQ], int zz) {
    const uint32_t mz = (zz >= 0 && zz < nz) ? 0u : kOOB;
    const uint32_t oc = (o_c + plane(zz)) | (m_c | mz);
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = buf_f64(zb[q], oc);
  };
  auto load_n = [&](int zz) {
    const uint32_t mz = zz < z1 ? 0u : kOOB, pz = plane(zz);
    const uint32_t oe = (o_e + pz) | (m_e | mz), om = (o_ym + pz) | (m_ym | mz), op = (o_yp + pz) | (m_yp | mz);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      e[q] = buf_f64(zb[q], oe);
      ym[q] = buf_f64(zb[q], om);
      yp[q] = buf_f64(zb[q], op);
    }
  };
  f32x4 acc[NP];
  double dacc[NP][4];
#pragma unroll
  for (int v = 0; v < NP; ++v) {
    acc[v] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int r = 0; r < 4; ++r) dacc[v][r] = 0.0;
  }
  // the MFMAs of half H of the pairs: pair g = H NP + v is tile g / 4, column block g % 4
  auto mfma_half = [&](auto hc) {
    constexpr int H = decltype(hc)::value;
    s16x4 a[NBT][S];
#pragma unroll
    for (int I = 0; I < NBT; ++I)
#pragma unroll
      for (int s2 = 0; s2 < S; ++s2) a[I][s2] = *reinterpret_cast<const s16x4*>(&Xs[I][s2][rb * 16 + lj][4 * kq]);
#pragma unroll
    for (int v = 0; v < NP; ++v) {
      const int g = H * NP + v, u = g >> 2, qb = g & 3;
      const int I = tile_row(u, NBT), J = tile_col(u, NBT);
      s16x4 b[S];
#pragma unroll
      for (int s2 = 0; s2 < S; ++s2) b[s2] = *reinterpret_cast<const s16x4*>(&Ys[J][s2][qb * 16 + lj][4 * kq]);
#pragma unroll
      for (int p1 = S - 1; p1 >= 0; --p1)
#pragma unroll
        for (int q2 = S - 1 - p1; q2 >= 0; --q2)
          acc[v] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[I][p1], b[q2], acc[v], 0, 0, 0);
    }
  };
  int since = 0;
  // FP64 -> FP32 -> S bfloat16 slices, two elements (columns cg and cg + 32 of block b) per
  // v_cvt_pk_bf16_f32 (nearest even); the FP32 remainders are exact
  auto store_split = [&](unsigned short (&T)[NBT][S][TB][SP + SKP], int b, double v0, double v1) {
    f32x2 r = f32x2{(float)v0, (float)v1};
#pragma unroll
    for (int s2 = 0; s2 < S; ++s2) {
      const unsigned w = __builtin_bit_cast(unsigned, __builtin_convertvector(r, bf16x2));
      T[b][s2][cg][lk] = (unsigned short)(w & 0xffffu);
      T[b][s2][cg + 32][lk] = (unsigned short)(w >> 16);
      if (s2 + 1 < S) {
        r.x -= __uint_as_float(w << 16);
        r.y -= __uint_as_float(w & 0xffff0000u);
      }
    }
  };
  auto step = [&](int z, double (&cm)[NQ], double (&c0)[NQ], double (&cp)[NQ]) {
    double w[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double xm = row_shift<DPP_ROW_SHR1>(e[q], c0[q]);
      double xp = row_shift<DPP_ROW_SHL1>(e[q], c0[q]);
      xm = xl ? xm : 0.0;
      xp = xr ? xp : 0.0;
      w[q] = in ? center * c0[q] + off * (((xm + xp) + (ym[q] + yp[q])) + (cm[q] + cp[q])) : 0.0;
    }
#pragma unroll
    for (int b = 0; b < NBT; ++b) {
      store_split(Xs, b, c0[2 * b], c0[2 * b + 1]);
      store_split(Ys, b, w[2 * b], w[2 * b + 1]);
    }
    __syncthreads();
    load_c(cm, z + 2);
    load_n(z + 1);
    if (hf == 0)
      mfma_half(std::integral_constant<int, 0>{});
    else
      mfma_half(std::integral_constant<int, 1>{});
    since += SP;
    if (since == KT || z == z1 - 1) {
#pragma unroll
      for (int v = 0; v < NP; ++v) {
#pragma unroll
        for (int r = 0; r < 4; ++r) dacc[v][r] += (double)acc[v][r];
        acc[v] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
      since = 0;
    }
    __syncthreads();
  };
  for (int reg = reg0; reg < nreg; reg += nrb) {
    set_region(reg);
    load_c(ca, z0 - 1);
    load_c(cbv, z0);
    load_c(cc, z0 + 1);
    load_n(z0);
    for (int z = z0; z < z1; z += 3) {
      step(z, ca, cbv, cc);
      if (z + 1 < z1) step(z + 1, cbv, cc, ca);
      if (z + 2 < z1) step(z + 2, cc, ca, cbv);
    }
  }
  double* P = partial + (int64_t)blockIdx.x * n * n;
  auto write_half = [&](auto hc) {
    constexpr int H = decltype(hc)::value;
#pragma unroll
    for (int v = 0; v < NP; ++v) {
      const int g = H * NP + v, u = g >> 2, qb = g & 3;
      const int I = tile_row(u, NBT), J = tile_col(u, NBT);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = I * TB + rb * 16 + 4 * kq + r;
        const int j = J * TB + qb * 16 + lj;
        if (i < n && j < n) P[(int64_t)j * n + i] = dacc[v][r];
      }
    }
  };
  if (hf == 0)
    write_half(std::integral_constant<int, 0>{});
  else
    write_half(std::integral_constant<int, 1>{});
}

struct StencilPlan {
  int nreg, zparts, zlen, chunks;
};
// Regions of SP plane points; the planes are cut into parts when there are fewer than 512 regions, and
// beyond 2048 regions a workgroup marches several (so that the partial Gram tiles stay within 2048 x n^2).
constexpr int64_t MAX_REGION_BASES = 2048;
StencilPlan stencil_plan(int64_t sxy, int64_t nz) {
  StencilPlan p;
  const int64_t nreg = (sxy + SP - 1) / SP;
  int64_t zp = (512 + nreg - 1) / nreg;
  if (zp > nz) zp = nz;
  if (zp < 1) zp = 1;
  p.nreg = (int)nreg;
  p.zlen = (int)((nz + zp - 1) / zp);
  p.zparts = (int)((nz + p.zlen - 1) / p.zlen);
  p.chunks = (int)((nreg < MAX_REGION_BASES ? nreg : MAX_REGION_BASES) * p.zparts);
  return p;
}

}  // namespace

size_t gram_partial_bytes(int64_t m, int64_t n) {
  GramPlan p = plan(m, n);
  size_t b = (size_t)p.chunks * n * n * sizeof(double);
  if (n > 2 * TB && n <= NBW * TB) {
    const size_t bw = (size_t)wide_plan(m).chunks * n * n * sizeof(double);
    if (bw > b) b = bw;
  }
  if (n <= 2 * TB) {
    const FullPlan f = full_plan(m, BK), g = full_plan(m, BKS);
    const size_t bf = (size_t)(f.chunks > g.chunks ? f.chunks : g.chunks) * n * n * sizeof(double);
    if (bf > b) b = bf;
  }
  return b;
}

static hipError_t reduce(const double* partial, int64_t n, int chunks, double* G, hipStream_t s) {
  gram_reduce_kernel<<<(unsigned)((n * n + 63) / 64), 512, 0, s>>>(partial, (int)n, chunks, G);
  return hipGetLastError();
}

template <bool SYM>
static hipError_t gram_f64(const double* X, int64_t ldx, const double* Y, int64_t ldy, const double* X2, int64_t ldx2,
                           int64_t m, int64_t n, double* partial, double* G, hipStream_t s) {
  if (n <= 2 * TB) {
    const FullPlan f = full_plan(m, BK);
    if (n <= TB)
      gram_full_f64_kernel<1, SYM><<<f.chunks, NT, 0, s>>>(X, ldx, Y, ldy, X2, ldx2, (int)m, (int)n, f.kc, partial);
    else
      gram_full_f64_kernel<2, SYM><<<f.chunks, NT, 0, s>>>(X, ldx, Y, ldy, X2, ldx2, (int)m, (int)n, f.kc, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce(partial, n, f.chunks, G, s);
  }
  GramPlan p = plan(m, n);
  gram_f64_kernel<SYM><<<dim3(p.tiles, p.chunks), NT, 0, s>>>(X, ldx, Y, ldy, X2, ldx2, (int)m, (int)n, p.nb, p.kc,
                                                              partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return reduce(partial, n, p.chunks, G, s);
}

hipError_t launch_gram_f64(const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t m, int64_t n,
                           double* partial, double* G, hipStream_t s) {
  return gram_f64<false>(X, ldx, Y, ldy, nullptr, 0, m, n, partial, G, s);
}

hipError_t launch_gram_symm(const double* Z, int64_t ldz, const double* Wsym, const double* Woff, int64_t ldw,
                            int64_t m, int64_t n, double* partial, double* G, hipStream_t s) {
  return gram_f64<true>(Z, ldz, Wsym, ldw, Woff, ldw, m, n, partial, G, s);
}

hipError_t launch_gram_symm_layers(const double* Z, int64_t ldz, const double* W, int64_t ldw, int64_t wstride,
                                  int layers, int64_t m, int64_t n, double* partial, double* G, hipStream_t s) {
  if (n <= 2 * TB || n > NBW * TB || layers < 1) return hipErrorInvalidValue;
  const FullPlan f = wide_plan(m);
  gram_wide_symm_kernel<<<f.chunks, NTW, 0, s>>>(Z, ldz, W, ldw, wstride, layers, (int)m, (int)n, f.kc, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return reduce(partial, n, f.chunks, G, s);
}

hipError_t launch_gram_fp32(const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t m, int64_t n,
                            double* partial, double* G, hipStream_t s) {
  GramPlan p = plan(m, n);
  gram_f64_kernel<false, true><<<dim3(p.tiles, p.chunks), NT, 0, s>>>(X, ldx, Y, ldy, nullptr, 0, (int)m, (int)n,
                                                                      p.nb, p.kc, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return reduce(partial, n, p.chunks, G, s);
}

hipError_t launch_gram_split(const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t m, int64_t n,
                             int slices, double* partial, double* G, hipStream_t s) {
  if (n <= 2 * TB) {
    const FullPlan f = full_plan(m, BKS);
    const int M = (int)m, N = (int)n;
    if (n <= TB) {
      if (slices == 2) gram_full_split_kernel<2, 1><<<f.chunks, NT, 0, s>>>(X, ldx, Y, ldy, M, N, f.kc, partial);
      else gram_full_split_kernel<3, 1><<<f.chunks, NT, 0, s>>>(X, ldx, Y, ldy, M, N, f.kc, partial);
    } else {
      if (slices == 2) gram_full_split_kernel<2, 2><<<f.chunks, NT, 0, s>>>(X, ldx, Y, ldy, M, N, f.kc, partial);
      else gram_full_split_kernel<3, 2><<<f.chunks, NT, 0, s>>>(X, ldx, Y, ldy, M, N, f.kc, partial);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce(partial, n, f.chunks, G, s);
  }
  GramPlan p = plan(m, n);
  if (slices == 2)
    gram_split_kernel<2><<<dim3(p.tiles, p.chunks), NT, 0, s>>>(X, ldx, Y, ldy, (int)m, (int)n, p.nb, p.kc, partial);
  else
    gram_split_kernel<3><<<dim3(p.tiles, p.chunks), NT, 0, s>>>(X, ldx, Y, ldy, (int)m, (int)n, p.nb, p.kc, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return reduce(partial, n, p.chunks, G, s);
}

bool stencil_gram_fits(const oqr_op* op, int64_t ldz, int64_t n) {
  if (op->kind != OQR_OP_STENCIL7 || n < 1 || n > 2 * TB) return false;
  const int64_t sxy = (int64_t)op->nx * op->ny, m = sxy * op->nz;
  if (m < 1) return false;
  // 32-bit byte offsets within one 64-column block, 32-bit row indices
  return ((int64_t)(TB - 1) * ldz + m) * 8 < 0x7fffffffll && m < 0x7fffffffll;
}

size_t stencil_gram_partial_bytes(const oqr_op* op, int64_t n) {
  if (op->kind != OQR_OP_STENCIL7 || n < 1 || n > 2 * TB) return 0;
  const int64_t sxy = (int64_t)op->nx * op->ny;
  if (sxy < 1 || op->nz < 1) return 0;
  return (size_t)stencil_plan(sxy, op->nz).chunks * n * n * sizeof(double);
}

hipError_t launch_stencil_gram_split(const oqr_op* op, const double* Z, int64_t ldz, int64_t n, int slices,
                                     double* partial, double* G, hipStream_t s) {
  if (!stencil_gram_fits(op, ldz, n) || (slices != 2 && slices != 3)) return hipErrorInvalidValue;
  const StencilPlan p = stencil_plan((int64_t)op->nx * op->ny, op->nz);
#define OQR_SGS(S_, NBT_)                                                                                    \
  stencil_gram_split_kernel<S_, NBT_><<<p.chunks, NT2, 0, s>>>(Z, ldz, (int)n, op->nx, op->ny, op->nz, op->center, \
                                                              op->off, p.nreg, p.zparts, p.zlen, partial)
  if (slices == 3) {
    if (n <= TB) OQR_SGS(3, 1); else OQR_SGS(3, 2);
  } else {
    if (n <= TB) OQR_SGS(2, 1); else OQR_SGS(2, 2);
  }
#undef OQR_SGS
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return reduce(partial, n, p.chunks, G, s);
}

hipError_t launch_stencil_gram(const oqr_op* op, const double* Z, int64_t ldz, int64_t n, double* partial, double* G,
                               hipStream_t s) {
  if (!stencil_gram_fits(op, ldz, n)) return hipErrorInvalidValue;
  const StencilPlan p = stencil_plan((int64_t)op->nx * op->ny, op->nz);
  if (n <= TB)
    stencil_gram_kernel<1><<<p.chunks, NT, 0, s>>>(Z, ldz, (int)n, op->nx, op->ny, op->nz, op->center, op->off,
                                                   p.nreg, p.zparts, p.zlen, partial);
  else
    stencil_gram_kernel<2><<<p.chunks, NT, 0, s>>>(Z, ldz, (int)n, op->nx, op->ny, op->nz, op->center, op->off,
                                                   p.nreg, p.zparts, p.zlen, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return reduce(partial, n, p.chunks, G, s);
}

}  // namespace oqr
