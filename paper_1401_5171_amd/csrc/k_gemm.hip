// Dense operator product W = A * Z (step 1 of CHOLQR, Algorithm 1), on MFMA.
//
// A is m x m (column-major, lda), Z and W are m x n (column-major).  A is the
// large operand and is streamed from HBM exactly once: a workgroup owns a
// 64-row block of W over the full width of n (up to 256 columns), so that
// each A tile is used for every column.  Z tiles are re-read by every row
// block and are served from L2/MALL.
#include "common.hpp"

namespace oqr {
namespace {

constexpr int BM = 64;       // rows of W per workgroup
constexpr int NT = 256;      // threads per workgroup (4 waves)

// ---------------------------------------------------------------------------------------------
// FP64: v_mfma_f64_16x16x4_f64.  Wave w owns all 64 rows and columns [w*16*CB, (w+1)*16*CB).
// ---------------------------------------------------------------------------------------------
constexpr int BK64 = 16;
// LDS row strides (doubles) against bank conflicts.  As (80 = 16 mod 32): the A-fragment reads (2 K rows x
// 16 rows per half-wave) cover disjoint bank halves; its stores are contiguous.  Bs (270 = 2 x odd): the
// stores (16 K rows x 2 columns per half-wave) hit distinct banks and the B-fragment reads overlap in 2 lanes.
constexpr int APAD = 16, BPAD = 14;

// K ranges of the products.  GEMM_FULL: row tile blockIdx.x, K slice blockIdx.z of width kchunk.
// GEMM_UPPER (A symmetric, strictly upper block triangle): row tile t needs K in [BM (t + 1), m);
// tiles t and R - 1 - t form pair blockIdx.x (their lengths sum to m - BM), the pair's K steps are cut
// into gridDim.z equal parts, and part blockIdx.z goes to layer blockIdx.z of the output (both tiles of
// the pair are written in every layer, zeros where the part has no steps).  GEMM_DIAG: row tile
// blockIdx.x, K in its own diagonal block [BM t, BM (t + 1)); the result is added to Wadd.  GEMM_SYMH: as
// GEMM_UPPER, but row tile t starts at its own diagonal block, whose entries below the diagonal count as
// zero and whose diagonal counts half: the product is W' = (U + D/2) Z with U the strictly upper part of
// A and D the lower-triangle-free diagonal blocks, so that A = (U + D/2) + (U + D/2)^T and
// Z^T A Z = Z^T W' + W'^T Z.  GEMM_DIAGH: row tile blockIdx.x over its own diagonal block only, with
// the masking of GEMM_SYMH (D' Z, D' = the upper triangles of the diagonal blocks with the diagonal
// halved), written as it is: added to U Z (GEMM_UPPER, any precision) it gives W'.
enum GemmMode { GEMM_FULL = 0, GEMM_UPPER = 1, GEMM_DIAG = 2, GEMM_SYMH = 3, GEMM_DIAGH = 4 };

struct Seg {
  int tile, k0, k1;
  bool desc;           // K steps taken from the top of [k0, k1) down
};

// The row-tile segments of workgroup (pair p, part h) in GEMM_UPPER, K steps of ks: a in tile p and,
// unless the pair is one tile (returns false), b in tile R - 1 - p.  With diag, a tile's K range starts
// at its own diagonal block.  A pair's steps form one list, cut into H equal parts (part h takes entries
// [T h / H, T (h + 1) / H)): tile p's steps, then tile R - 1 - p's, each from its start up; or, with
// sync, tile p's from the top of K down and then tile R - 1 - p's from its start up.  With sync the
// list has the same length for every pair (for m a multiple of BM) and its s-th entry lies at the same
// K for every pair (the top step less ks s while in tile p, then ks s plus a fixed offset, BM or -BM
// with diag), so the workgroups of one part walk K together and each K tile of Z is fetched into L2
// once rather than once per workgroup.
__device__ __forceinline__ bool upper_segments(int m, int p, int h, int H, int ks, Seg& a, Seg& b,
                                               bool diag = false, bool sync = false) {
  const int R = (m + BM - 1) / BM;
  const int ta = p, tb = R - 1 - p;
  const int d = diag ? 0 : 1;
  const int sa = min(m, BM * (ta + d)), sb = min(m, BM * (tb + d));
  const int na = (m - sa + ks - 1) / ks, nb = (tb != ta) ? (m - sb + ks - 1) / ks : 0;
  const int T = na + nb;
  const int s0 = (int)((int64_t)T * h / H), s1 = (int)((int64_t)T * (h + 1) / H);
  if (sync)   // entries [s0, min(s1, na)) are tile p's steps na - 1 - s (downward)
    a = {ta, min(m, sa + ks * (na - min(s1, na))), min(m, sa + ks * (na - min(s0, na))), true};
  else
    a = {ta, min(m, sa + ks * min(s0, na)), min(m, sa + ks * min(s1, na)), false};
  b = {tb, min(m, sb + ks * max(s0 - na, 0)), min(m, sb + ks * max(s1 - na, 0)), false};
  return tb != ta;
}

// Start of step s of a K range [kb, ke) cut into steps of ks from kb, taken from the top down if desc;
// past the last step, ke (loads there read nothing and return zeros).
__device__ __forceinline__ int kpos(int kb, int ke, int ks, int s, bool desc) {
  const int ns = (ke - kb + ks - 1) / ks;
  return s >= ns ? ke : (desc ? kb + ks * (ns - 1 - s) : kb + ks * s);
}

// F32: the FP32 operand pass.  A and Z are rounded to FP32 as they leave LDS and multiplied on
// v_mfma_f32_16x16x4_f32 (the same lane layouts as the FP64 instruction), with FP32 sums over at most
// F32_FOLD rows of K folded into the FP64 accumulators.
constexpr int F32_FOLD = 960;

template <int CB, int MODE, bool F32 = false>
__global__ __launch_bounds__(NT, 2) void gemm_f64_kernel(const double* __restrict__ A, int64_t lda,
                                                          const double* __restrict__ Z, int64_t ldz,
                                                          double* __restrict__ W, int64_t ldw, int m, int n,
                                                          int kchunk, int64_t wstride,
                                                          const double* __restrict__ Wadd, int64_t ldadd) {
  constexpr int BN = 64 * CB;                   // columns per workgroup
  __shared__ double As[BK64][BM + APAD];
  __shared__ double Bs[BK64][BN + BPAD];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int j0 = blockIdx.y * BN;
  const int wc = wave * 16 * CB;
  W += blockIdx.z * wstride;
  // row of accumulator element r within a 16 x 16 tile: the FP64 instruction's layout (4 r + l / 16), or
  // the FP32 one's (4 (l / 16) + r); FP32 sums are folded element by element, so they keep theirs
  auto drow = [](int r, int l) { return F32 ? 4 * (l >> 4) + r : 4 * r + (l >> 4); };

  // global -> register staging
  constexpr int AR = BM * BK64 / NT;            // 4
  constexpr int BR = BK64 * BN / NT;            // 4*CB
  const int ai = t % BM, ak = t / BM;           // A: row ai, k = ak + 4r
  const int bk = t % BK64, bj = t / BK64;       // Z: k = bk, col = bj + 16r
  uint32_t boff[BR];
#pragma unroll
  for (int r = 0; r < BR; ++r)
    boff[r] = (j0 + bj + 16 * r < n) ? (uint32_t)(((int64_t)(bj + 16 * r) * ldz + bk) * 8) : kOOB;

  // rows [i0, i0 + BM) of A times Z over K [kb, ke); result (+ Wadd) into W
  auto segment = [&](int i0, int kb, int ke) {
    f64x4 acc[4][CB];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < CB; ++b) acc[a][b] = f64x4{0, 0, 0, 0};
    double ra[AR], rb[BR];
    int ka = kb;                       // K step held in ra
    uint32_t aoff[AR];
#pragma unroll
    for (int r = 0; r < AR; ++r) aoff[r] = (i0 + ai < m) ? (uint32_t)(((int64_t)(ak + 4 * r) * lda + ai) * 8) : kOOB;
    auto load = [&](int k0) {
      // A rows i0.., columns k0..: the size bound cuts k >= ke; Z rows k0.., columns j0..
      const bufrsrc abuf = make_buf(A + (int64_t)min(k0, ke) * lda + i0, (int64_t)(ke - min(k0, ke)) * lda * 8);
      const bufrsrc zbuf = make_buf(Z + (int64_t)j0 * ldz + k0, (int64_t)(n - j0) * ldz * 8);
      const bool kin = k0 + bk < ke;
      ka = k0;
#pragma unroll
      for (int r = 0; r < AR; ++r) ra[r] = buf_f64(abuf, aoff[r]);
#pragma unroll
      for (int r = 0; r < BR; ++r) rb[r] = buf_f64(zbuf, kin ? boff[r] : kOOB);
    };
    auto store = [&]() {
      if ((MODE == GEMM_SYMH || MODE == GEMM_DIAGH) && ka < i0 + BM) {
        // the diagonal block (uniform test): below the diagonal 0, on it half
#pragma unroll
        for (int r = 0; r < AR; ++r) {
          const int d = ka + ak + 4 * r - (i0 + ai);
          ra[r] = d < 0 ? 0.0 : (d == 0 ? 0.5 * ra[r] : ra[r]);
        }
      }
#pragma unroll
      for (int r = 0; r < AR; ++r) As[ak + 4 * r][ai] = ra[r];
#pragma unroll
      for (int r = 0; r < BR; ++r) Bs[bk][bj + 16 * r] = rb[r];
    };

    f32x4 acc32[F32 ? 4 : 1][F32 ? CB : 1];
    auto fold32 = [&]() {
      if constexpr (F32) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < CB; ++b) {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[a][b][r] += (double)acc32[a][b][r];
            acc32[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
          }
      }
    };
    if constexpr (F32) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < CB; ++b) acc32[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    __syncthreads();                   // the previous segment's last reads of As / Bs
    load(kb);
    store();
    __syncthreads();
    int step = 0;
    for (int k0 = kb; k0 < ke; k0 += BK64) {
      load(k0 + BK64);                 // past the end: guarded loads return zeros
#pragma unroll
      for (int kk = 0; kk < BK64; kk += 4) {
        const int kr = kk + (lane >> 4);
        double af[4], bf[CB];
#pragma unroll
        for (int a = 0; a < 4; ++a) af[a] = As[kr][a * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < CB; ++b) bf[b] = Bs[kr][wc + b * 16 + (lane & 15)];
        if constexpr (F32) {
          float af32[4], bf32[CB];
#pragma unroll
          for (int a = 0; a < 4; ++a) af32[a] = (float)af[a];
#pragma unroll
          for (int b = 0; b < CB; ++b) bf32[b] = (float)bf[b];
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < CB; ++b)
              acc32[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(af32[a], bf32[b], acc32[a][b], 0, 0, 0);
        } else {
#pragma unroll
          for (int a = 0; a < 4; ++a)
            // GEMM_DIAGH: rows 16 a .. of D' are zero left of column 16 a, so a K step wholly left of
            // them adds nothing (uniform test)
            if (MODE != GEMM_DIAGH || k0 - i0 >= 16 * a) {
#pragma unroll
              for (int b = 0; b < CB; ++b) acc[a][b] = mfma_f64(af[a], bf[b], acc[a][b]);
            }
        }
      }
      if (F32 && ++step == F32_FOLD / BK64) {
        fold32();
        step = 0;
      }
      __syncthreads();
      store();
      __syncthreads();
    }
    fold32();
    if (MODE == GEMM_DIAG) {
      // W = acc + Wadd: the addends of one row block are loaded together (branch-free buffer loads,
      // lanes outside the matrix masked with kOOB) before any is used, one round trip per row block
      const bufrsrc wb = make_buf(Wadd, ((int64_t)(n - 1) * ldadd + m) * 8);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        double add[CB][4];
#pragma unroll
        for (int b = 0; b < CB; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = i0 + a * 16 + drow(r, lane);
            const int j = j0 + wc + b * 16 + (lane & 15);
            add[b][r] = buf_f64(wb, ((uint32_t)((int64_t)j * ldadd + i) * 8u) | ((i < m && j < n) ? 0u : kOOB));
          }
#pragma unroll
        for (int b = 0; b < CB; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = i0 + a * 16 + drow(r, lane);
            const int j = j0 + wc + b * 16 + (lane & 15);
            if (i < m && j < n) W[(int64_t)j * ldw + i] = acc[a][b][r] + add[b][r];
          }
      }
    } else {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < CB; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = i0 + a * 16 + drow(r, lane);
            const int j = j0 + wc + b * 16 + (lane & 15);
            if (i < m && j < n) W[(int64_t)j * ldw + i] = acc[a][b][r];
          }
    }
  };

  if (MODE == GEMM_UPPER || MODE == GEMM_SYMH) {
    Seg sa, sb;
    const bool two = upper_segments(m, blockIdx.x, blockIdx.z, gridDim.z, BK64, sa, sb, MODE == GEMM_SYMH);
    segment(sa.tile * BM, sa.k0, sa.k1);           // ascending (no sync): sa.desc is false
    if (two) segment(sb.tile * BM, sb.k0, sb.k1);
  } else if (MODE == GEMM_DIAG || MODE == GEMM_DIAGH) {
    const int i0 = blockIdx.x * BM;
    segment(i0, i0, min(m, i0 + BM));
  } else {
    const int kb = blockIdx.z * kchunk;
    segment(blockIdx.x * BM, kb, min(m, kb + kchunk));
  }
}

// ---------------------------------------------------------------------------------------------
// Split bfloat16: v_mfma_f32_16x16x32_bf16 on the S-slice products with slice indices p + q < S.
// A is split on the fly (FP64 -> FP32 -> S bfloat16 slices) into a double-buffered LDS tile; the
// slices of Z are pre-split in HBM and read as MFMA B fragments straight into registers, one
// K step ahead.  FP32 accumulation over at most 960 rows of K, then folded into FP64
// accumulators kept in LDS (each lane owns its slots).  One wave per SIMD, one barrier per step.
// ---------------------------------------------------------------------------------------------
constexpr int BKS = 32;
constexpr int SROW = BKS + 8;   // LDS row stride of an A slice (bf16 elements)

template <int S, int CB, int MODE>
__global__ __launch_bounds__(NT, 1) void gemm_split_kernel(const double* __restrict__ A, int64_t lda,
                                                            const unsigned short* __restrict__ zs,
                                                            double* __restrict__ W, int64_t ldw, int m, int n,
                                                            int kchunk, int64_t wstride) {
  constexpr int BN = 64 * CB;
  __shared__ __attribute__((aligned(16))) unsigned short As[2][S][BM][SROW];
  __shared__ double Dacc[NT / 64][4 * CB * 4][64];     // FP64 accumulators: [wave][slot][lane]
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int j0 = blockIdx.y * BN;
  const int wc = j0 + wave * 16 * CB;
  const int64_t mp = split_ld(m);             // ld of the slices of Z (rows padded with zeros)
  const int64_t slice_stride = mp * n;
  // the current segment: rows [i0, i0 + BM), K [kb, ke) (kb a multiple of BKS)
  int i0 = 0, kb = 0, ke = 0;
  bool kdesc = false;          // K steps taken from the top down
  W += blockIdx.z * wstride;

  f32x4 acc[4][CB];
  // A tile 64 x 32: thread t loads row ai = t % 64, k = 8 ak .. 8 ak + 7 (ak = t / 64).
  // Three register stages keep A two K steps ahead of the MFMAs (HBM latency).
  const int ai = t % BM, ak = t / BM;
  uint32_t aoff[8];
  double ra0[8], ra1[8], ra2[8];
  auto load_a = [&](double (&ra)[8], int st) {      // A tile of K step st
    const int k0 = kpos(kb, ke, BKS, st, kdesc);
    const bufrsrc abuf = make_buf(A + (int64_t)min(k0, ke) * lda + i0, (int64_t)(ke - min(k0, ke)) * lda * 8);
#pragma unroll
    for (int e = 0; e < 8; ++e) ra[e] = buf_f64(abuf, aoff[e]);
  };
  // FP64 -> FP32 -> S bfloat16 slices, two elements per v_cvt_pk_bf16_f32 (round to nearest even);
  // each remainder r - bf16(r) is exact in FP32.
  auto store_a = [&](const double (&ra)[8], int buf) {
    f32x2 r[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = f32x2{(float)ra[2 * q], (float)ra[2 * q + 1]};
#pragma unroll
    for (int s = 0; s < S; ++s) {
      unsigned w[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        w[q] = __builtin_bit_cast(unsigned, __builtin_convertvector(r[q], bf16x2));
        if (s + 1 < S) {
          r[q].x -= __uint_as_float(w[q] << 16);
          r[q].y -= __uint_as_float(w[q] & 0xffff0000u);
        }
      }
      *reinterpret_cast<uint4*>(&As[buf][s][ai][ak * 8]) = make_uint4(w[0], w[1], w[2], w[3]);
    }
  };
  // B fragments: lane holds k = 8 (lane / 16) .. + 7 of column wc + 16 b + lane % 16.
  uint32_t zoff[CB];
#pragma unroll
  for (int b = 0; b < CB; ++b) {
    const int j = wc + 16 * b + (lane & 15);
    zoff[b] = (j < n) ? (uint32_t)(((int64_t)j * mp + 8 * (lane >> 4)) * 2) : kOOB;
  }
  uint4 bf0[S][CB], bf1[S][CB], bf2[S][CB];
  auto load_b = [&](int st, uint4 (&dst)[S][CB]) {
    // rows k0 .. k0 + 31 of every slice (K step st); past the slice (or the padded end) the buffer is empty
    const int k0 = kpos(kb, ke, BKS, st, kdesc);
    const bool live = k0 < ke || (ke == m && k0 < mp);
    const bufrsrc zbuf = make_buf(zs + min((int64_t)k0, mp), live ? (int64_t)(S * slice_stride - k0) * 2 : 0);
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int b = 0; b < CB; ++b)
        dst[s][b] = buf_b128(zbuf, zoff[b] == kOOB ? kOOB : zoff[b] + (uint32_t)(s * slice_stride * 2));
  };

  // K steps are padded to a multiple of 6 (3 A register stages x 2 B fragment buffers); steps past the
  // end of K read empty buffers and contribute zeros, so no load sits under a branch.
  // One K step, a single basic block: request B(st+2) and A(st+3); read the A fragments of buffer
  // st & 1; convert A(st+1) into the other buffer while the MFMAs run; one barrier.  B is requested
  // before A: memory counters retire in order, so the wait for B(st+1) at the next step must not
  // also wait for the HBM loads of A issued after it.
  auto step = [&](int st, const double (&ra_store)[8], double (&ra_fill)[8], const uint4 (&bu)[S][CB],
                  uint4 (&bfill)[S][CB]) __attribute__((always_inline)) {
    const int cur = st & 1;
    load_b(st + 2, bfill);
    load_a(ra_fill, st + 3);
    const int kq = 8 * (lane >> 4);
    bf16x8 af[S][4];
#pragma unroll
    for (int p = 0; p < S; ++p)
#pragma unroll
      for (int a = 0; a < 4; ++a)
        af[p][a] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&As[cur][p][a * 16 + (lane & 15)][kq]));
    store_a(ra_store, cur ^ 1);
#pragma unroll
    for (int p = 0; p < S; ++p)
#pragma unroll
      for (int q = 0; q < S - p; ++q)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < CB; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[p][a], __builtin_bit_cast(bf16x8, bu[q][b]),
                                                                acc[a][b], 0, 0, 0);
    // interleave: one MFMA, then a few VALU / LDS-write instructions of the conversion
#pragma unroll
    for (int i = 0; i < 4 * CB * S * (S + 1) / 2; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);
      __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
    }
    __syncthreads();
  };
  auto fold = [&]() {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < CB; ++b) {
#pragma unroll
        for (int r = 0; r < 4; ++r) Dacc[wave][(a * CB + b) * 4 + r][lane] += (double)acc[a][b][r];
        acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
  };

  auto segment = [&]() {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) Dacc[wave][(a * CB + b) * 4 + r][lane] = 0.0;
    }
#pragma unroll
  for (int e = 0; e < 8; ++e) aoff[e] = (i0 + ai < m) ? (uint32_t)(((int64_t)(ak * 8 + e) * lda + ai) * 8) : kOOB;
  const int nsteps = ((ke - kb + BKS - 1) / BKS + 5) / 6 * 6;
  load_b(0, bf0);
  load_b(1, bf1);
  load_a(ra0, 0);
  load_a(ra1, 1);
  load_a(ra2, 2);
  store_a(ra0, 0);
  __syncthreads();
  for (int st = 0; st < nsteps; st += 6) {
    step(st + 0, ra1, ra0, bf0, bf2);
    step(st + 1, ra2, ra1, bf1, bf0);
    step(st + 2, ra0, ra2, bf2, bf1);
    step(st + 3, ra1, ra0, bf0, bf2);
    step(st + 4, ra2, ra1, bf1, bf0);
    step(st + 5, ra0, ra2, bf2, bf1);
    if ((st / 6) % 5 == 4) fold();      // FP32 accumulation over at most 30 steps (960 rows of K)
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < CB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) Dacc[wave][(a * CB + b) * 4 + r][lane] += (double)acc[a][b][r];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < CB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + a * 16 + 4 * (lane >> 4) + r;
        const int j = wc + b * 16 + (lane & 15);
        if (i < m && j < n) W[(int64_t)j * ldw + i] = Dacc[wave][(a * CB + b) * 4 + r][lane];
      }
  };

  if (MODE == GEMM_UPPER) {
    Seg sa, sb;
    const bool two = upper_segments(m, blockIdx.x, blockIdx.z, gridDim.z, BKS, sa, sb, false, true);
    i0 = sa.tile * BM, kb = sa.k0, ke = sa.k1, kdesc = sa.desc;
    segment();
    if (two) {
      __syncthreads();                  // the last reads of As
      i0 = sb.tile * BM, kb = sb.k0, ke = sb.k1, kdesc = sb.desc;
      segment();
    }
  } else {
    i0 = blockIdx.x * BM, kb = blockIdx.z * kchunk, ke = min(m, kb + kchunk);
    segment();
  }
}

// Split bfloat16 product for n in (128, 256]: 512 threads (two waves per SIMD), a 64-row block of W
// over 256 columns.  Wave w owns all 64 rows and columns 32 w .. 32 w + 31 (4 x 2 tiles).  Per K step
// of 32 the workgroup converts the A tile into S slices in double-buffered LDS (one barrier per step,
// the next two A tiles in flight in registers); every wave reads its B fragments (8 consecutive K of a
// column of a slice: 16 contiguous bytes of the tiled layout) straight from memory into registers,
// three K steps ahead, so that B never passes through LDS and no two waves load the same fragment.
// FP32 accumulation over at most 960 rows of K, folded into FP64 accumulators held in registers.
constexpr int NT2 = 512;
constexpr int BN2 = 256;

template <int S, int MODE>
__global__ __launch_bounds__(NT2, 1) void gemm_split2_kernel(const double* __restrict__ A, int64_t lda,
                                                             const unsigned short* __restrict__ zs,
                                                             double* __restrict__ W, int64_t ldw, int m, int n,
                                                             int kchunk, int64_t wstride) {
  __shared__ __attribute__((aligned(16))) unsigned short As[2][S][BM][SROW];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t mp = split_ld(m);
  constexpr int64_t TILE = (int64_t)S * BN2 * BKS;   // bf16 elements of one K step of the tiled slices
  // the current segment: rows [i0, i0 + BM), K [kb, ke) (kb a multiple of BKS)
  int i0 = 0, kb = 0, ke = 0;
  bool kdesc = false;          // K steps taken from the top down
  W += blockIdx.z * wstride;

  f32x4 acc[4][2];
  double dacc[4][2][4];
  // A tile 64 x 32: thread t loads row ai = t % 64, k = 4 aq .. 4 aq + 3 (aq = t / 64)
  const int ai = t % BM, aq = t / BM;
  uint32_t aoff[4];
  // B fragment (slice q, tile b): lane holds K kq .. kq + 7 of column 32 wave + 16 b + lane % 16
  const int kq = 8 * (lane >> 4);
  uint32_t fb[S][2];
#pragma unroll
  for (int q = 0; q < S; ++q)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = 32 * wave + 16 * b + (lane & 15);
      fb[q][b] = (col < n) ? (uint32_t)((((int64_t)q * BN2 + col) * BKS + kq) * 2) : kOOB;
    }
  double ra0[4], ra1[4];
  uint4 bq0[S][2], bq1[S][2], bq2[S][2];
  auto load_a = [&](int k0, double (&ra)[4]) {
    const bufrsrc abuf = make_buf(A + (int64_t)min(k0, ke) * lda + i0, (int64_t)(ke - min(k0, ke)) * lda * 8);
#pragma unroll
    for (int e = 0; e < 4; ++e) ra[e] = buf_f64(abuf, aoff[e]);
  };
  auto load_b = [&](int k0, uint4 (&bq)[S][2]) {
    // the K step's tile of slices; past the slice (or the padded end) the buffer is empty
    const bool live = k0 < ke || (ke == m && k0 < mp);
    const bufrsrc zbuf = make_buf(zs + (live ? (int64_t)(k0 / BKS) * TILE : 0), live ? TILE * 2 : 0);
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
      for (int b = 0; b < 2; ++b) bq[q][b] = buf_b128(zbuf, fb[q][b]);
  };
  auto store_a = [&](int buf, const double (&ra)[4]) {
    // FP64 -> FP32 -> S bf16 slices (RNE, two per v_cvt_pk_bf16_f32); remainders exact in FP32
    f32x2 r[2] = {f32x2{(float)ra[0], (float)ra[1]}, f32x2{(float)ra[2], (float)ra[3]}};
#pragma unroll
    for (int sl = 0; sl < S; ++sl) {
      unsigned w[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        w[q] = __builtin_bit_cast(unsigned, __builtin_convertvector(r[q], bf16x2));
        if (sl + 1 < S) {
          r[q].x -= __uint_as_float(w[q] << 16);
          r[q].y -= __uint_as_float(w[q] & 0xffff0000u);
        }
      }
      *reinterpret_cast<uint2*>(&As[buf][sl][ai][aq * 4]) = make_uint2(w[0], w[1]);
    }
  };
  auto fold = [&]() {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
#pragma unroll
        for (int r = 0; r < 4; ++r) dacc[a][b][r] += (double)acc[a][b][r];
        acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
  };
  auto compute = [&](int st, const uint4 (&bq)[S][2]) {
    const int cur = st & 1;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      bf16x8 af[S];
#pragma unroll
      for (int p = 0; p < S; ++p)
        af[p] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&As[cur][p][16 * a + (lane & 15)][kq]));
#pragma unroll
      for (int p = 0; p < S; ++p)
#pragma unroll
        for (int q = 0; q < S - p; ++q)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[p], __builtin_bit_cast(bf16x8, bq[q][b]),
                                                                acc[a][b], 0, 0, 0);
    }
    if (st % 30 == 29) fold();                // FP32 accumulation over at most 960 rows of K
  };

  auto segment = [&]() {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < 4; ++r) dacc[a][b][r] = 0.0;
      }
#pragma unroll
    for (int e = 0; e < 4; ++e) aoff[e] = (i0 + ai < m) ? (uint32_t)(((int64_t)(aq * 4 + e) * lda + ai) * 8) : kOOB;
    // K steps padded to a multiple of 6 (2 A buffers x 3 B stages); steps past the end read empty
    // buffers and add zeros
    const int nsteps = ((ke - kb + BKS - 1) / BKS + 5) / 6 * 6;
    load_a(kpos(kb, ke, BKS, 0, kdesc), ra0);
    load_b(kpos(kb, ke, BKS, 0, kdesc), bq0);
    load_b(kpos(kb, ke, BKS, 1, kdesc), bq1);
    load_b(kpos(kb, ke, BKS, 2, kdesc), bq2);
    store_a(0, ra0);
    __syncthreads();
    load_a(kpos(kb, ke, BKS, 1, kdesc), ra0);
    load_a(kpos(kb, ke, BKS, 2, kdesc), ra1);
    // step st: MFMAs on A buffer st & 1 and B stage st % 3; A(st + 1) into the other buffer; A and B of
    // step st + 3 requested
#define OQR_SPLIT2_STEP(st, RA, BQ)       \
  compute(st, BQ);                        \
  store_a(((st) + 1) & 1, RA);            \
  load_a(kpos(kb, ke, BKS, (st) + 3, kdesc), RA); \
  load_b(kpos(kb, ke, BKS, (st) + 3, kdesc), BQ); \
  __syncthreads();
    for (int st = 0; st < nsteps; st += 6) {
      OQR_SPLIT2_STEP(st + 0, ra0, bq0)
      OQR_SPLIT2_STEP(st + 1, ra1, bq1)
      OQR_SPLIT2_STEP(st + 2, ra0, bq2)
      OQR_SPLIT2_STEP(st + 3, ra1, bq0)
      OQR_SPLIT2_STEP(st + 4, ra0, bq1)
      OQR_SPLIT2_STEP(st + 5, ra1, bq2)
    }
#undef OQR_SPLIT2_STEP
    fold();
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + 16 * a + 4 * (lane >> 4) + r;
          const int j = 32 * wave + 16 * b + (lane & 15);
          if (i < m && j < n) W[(int64_t)j * ldw + i] = dacc[a][b][r];
        }
  };

  if (MODE == GEMM_UPPER) {
    Seg sa, sb;
    const bool two = upper_segments(m, blockIdx.x, blockIdx.z, gridDim.z, BKS, sa, sb, false, true);
    i0 = sa.tile * BM, kb = sa.k0, ke = sa.k1, kdesc = sa.desc;
    segment();
    if (two) {
      __syncthreads();                  // the last reads of As
      i0 = sb.tile * BM, kb = sb.k0, ke = sb.k1, kdesc = sb.desc;
      segment();
    }
  } else {
    i0 = blockIdx.x * BM, kb = blockIdx.z * kchunk, ke = min(m, kb + kchunk);
    segment();
  }
}

// Slices of Z, rows m..split_ld(m)-1 zero.  Column layout (n <= 128): zs[s][j][i] (ld split_ld(m)).
// Tiled layout (n > 128, read by gemm_split2_kernel): zs[i / 32][s][j][i % 32] with 256 columns per
// tile, so that the slices of one 32-row K step form one contiguous block.
__global__ void split_z_kernel(const double* __restrict__ Z, int64_t ldz, unsigned short* __restrict__ zs,
                               int64_t m, int64_t n, int slices, int tiled) {
  // four consecutive rows per thread (one 32-row segment in either layout): one 8-byte store per slice
  const int64_t mp = split_ld(m);
  const int64_t idx = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (idx >= mp * n) return;
  const int64_t j = idx / mp, i = idx % mp;
  double r[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) r[e] = (i + e < m) ? Z[j * ldz + i + e] : 0.0;
  for (int s = 0; s < slices; ++s) {
    unsigned short b[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      b[e] = bf16_bits((float)r[e]);
      r[e] -= (double)bf16_to_f32(b[e]);
    }
    const int64_t o = tiled ? (((i / BKS) * slices + s) * BN2 + j) * BKS + i % BKS : (int64_t)s * mp * n + idx;
    *reinterpret_cast<uint2*>(zs + o) = make_uint2((unsigned)b[0] | ((unsigned)b[1] << 16),
                                                   (unsigned)b[2] | ((unsigned)b[3] << 16));
  }
}

int col_blocks(int64_t n) { return n <= 64 ? 1 : (n <= 128 ? 2 : 4); }

// W(i, j) = sum_z P[z](i, j) (ld m), z ascending.
__global__ void ksum_kernel(const double* __restrict__ P, int ks, int64_t m, int64_t n, double* __restrict__ W,
                            int64_t ldw) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * n) return;
  double s = 0.0;
  for (int z = 0; z < ks; ++z) s += P[(int64_t)z * m * n + idx];
  W[(idx / m) * ldw + idx % m] = s;
}

struct KSplit {
  int ks, kchunk;
};
// Split K when the row x column tiles leave CUs idle (fewer than two workgroups per CU).
KSplit ksplit(int64_t m, int64_t n) {
  const int cb = col_blocks(n);
  const int64_t wgs = (int64_t)ceil_div(m, BM) * ceil_div(n, 64 * cb);
  const int64_t target = 2 * (int64_t)device_cu_count();
  KSplit k{1, (int)m};
  if (wgs >= target || m < 2048) return k;
  int ks = (int)((target + wgs - 1) / wgs);
  if (ks > 8) ks = 8;
  if (ks > m / 1024) ks = (int)(m / 1024);
  if (ks < 2) return k;
  int64_t chunk = (m + ks - 1) / ks;
  chunk = (chunk + 95) / 96 * 96;              // a multiple of both K steps
  k.ks = (int)((m + chunk - 1) / chunk);
  k.kchunk = (int)chunk;
  return k;
}

}  // namespace

// Parts per pair of the GEMM_UPPER schedule: enough workgroups for two per CU, at most 8 layers.
static int upper_parts(int64_t m, int64_t n) {
  const int64_t R = ceil_div(m, BM), P = (R + 1) / 2, ycb = ceil_div(n, 64 * col_blocks(n));
  const int64_t target = 2 * (int64_t)device_cu_count();
  int64_t H = (target + P * ycb - 1) / (P * ycb);
  if (H > 8) H = 8;
  if (H < 1) H = 1;
  return (int)H;
}

size_t gemm_kpart_bytes(int64_t m, int64_t n, bool diag_layer) {
  const KSplit k = ksplit(m, n);
  int layers = k.ks > 1 ? k.ks : 0;
  const int h = upper_parts(m, n);
  if (h > 1 && h + (diag_layer ? 1 : 0) > layers) layers = h + (diag_layer ? 1 : 0);
  return (size_t)layers * m * n * sizeof(double);
}

static hipError_t ksum(const double* P, int ks, int64_t m, int64_t n, double* W, int64_t ldw, hipStream_t s) {
  const int64_t total = m * n;
  ksum_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(P, ks, m, n, W, ldw);
  return hipGetLastError();
}

#define OQR_GEMM_T(cb, MODE_, F32_, grid, out, ldo, kchunk, stride, wadd, ldadd)                                \
  do {                                                                                                          \
    const int M_ = (int)m, N_ = (int)n;                                                                         \
    if ((cb) == 1)                                                                                              \
      gemm_f64_kernel<1, MODE_, F32_><<<(grid), NT, 0, s>>>(A, lda, Z, ldz, out, ldo, M_, N_, kchunk, stride, wadd, \
                                                             ldadd);                                            \
    else if ((cb) == 2)                                                                                         \
      gemm_f64_kernel<2, MODE_, F32_><<<(grid), NT, 0, s>>>(A, lda, Z, ldz, out, ldo, M_, N_, kchunk, stride, wadd, \
                                                             ldadd);                                            \
    else                                                                                                        \
      gemm_f64_kernel<4, MODE_, F32_><<<(grid), NT, 0, s>>>(A, lda, Z, ldz, out, ldo, M_, N_, kchunk, stride, wadd, \
                                                             ldadd);                                            \
  } while (0)
#define OQR_GEMM_F64(cb, MODE_, grid, out, ldo, kchunk, stride, wadd, ldadd) \
  OQR_GEMM_T(cb, MODE_, false, grid, out, ldo, kchunk, stride, wadd, ldadd)

hipError_t launch_gemm_f64(const double* A, int64_t lda, const double* Z, int64_t ldz, double* W, int64_t ldw,
                           int64_t m, int64_t n, double* kpart, hipStream_t s) {
  const int cb = col_blocks(n);
  KSplit k = ksplit(m, n);
  if (!kpart) k = KSplit{1, (int)m};
  dim3 grid(ceil_div(m, BM), ceil_div(n, 64 * cb), k.ks);
  double* out = k.ks > 1 ? kpart : W;
  const int64_t ldo = k.ks > 1 ? m : ldw, stride = k.ks > 1 ? m * n : 0;
  OQR_GEMM_F64(cb, GEMM_FULL, grid, out, ldo, k.kchunk, stride, nullptr, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || k.ks == 1) return e;
  return ksum(kpart, k.ks, m, n, W, ldw, s);
}

int symm_layers(int64_t m, int64_t n, const double* kpart) { return kpart ? upper_parts(m, n) : 1; }

hipError_t launch_symm_upper(const double* A, int64_t lda, const double* Z, int64_t ldz, double* Woff, int64_t ldw,
                             int64_t m, int64_t n, double* kpart, hipStream_t s, bool f32) {
  const int cb = col_blocks(n);
  const int R = ceil_div(m, BM), P = (R + 1) / 2, ycb = ceil_div(n, 64 * cb);
  const int H = symm_layers(m, n, kpart);
  double* out = H > 1 ? kpart : Woff;
  const int64_t ldo = H > 1 ? m : ldw, stride = H > 1 ? m * n : 0;
  if (f32)
    OQR_GEMM_T(cb, GEMM_UPPER, true, dim3(P, ycb, H), out, ldo, 0, stride, nullptr, 0);
  else
    OQR_GEMM_F64(cb, GEMM_UPPER, dim3(P, ycb, H), out, ldo, 0, stride, nullptr, 0);
  return hipGetLastError();
}

hipError_t launch_symm_half(const double* A, int64_t lda, const double* Z, int64_t ldz, double* W, int64_t ldw,
                            int64_t m, int64_t n, double* kpart, hipStream_t s) {
  const int cb = col_blocks(n);
  const int R = ceil_div(m, BM), P = (R + 1) / 2, ycb = ceil_div(n, 64 * cb);
  const int H = symm_layers(m, n, kpart);
  double* out = H > 1 ? kpart : W;
  const int64_t ldo = H > 1 ? m : ldw, stride = H > 1 ? m * n : 0;
  OQR_GEMM_F64(cb, GEMM_SYMH, dim3(P, ycb, H), out, ldo, 0, stride, nullptr, 0);
  return hipGetLastError();
}

hipError_t launch_symm_diag_half(const double* A, int64_t lda, const double* Z, int64_t ldz, double* W, int64_t ldw,
                                 int64_t m, int64_t n, hipStream_t s) {
  const int cb = col_blocks(n);
  OQR_GEMM_F64(cb, GEMM_DIAGH, dim3(ceil_div(m, BM), ceil_div(n, 64 * cb), 1), W, ldw, 0, 0, nullptr, 0);
  return hipGetLastError();
}

hipError_t launch_layer_sum(const double* kpart, int layers, int64_t m, int64_t n, double* W, int64_t ldw,
                            hipStream_t s) {
  return layers > 1 ? ksum(kpart, layers, m, n, W, ldw, s) : hipSuccess;
}

hipError_t launch_symm_finish(const double* A, int64_t lda, const double* Z, int64_t ldz, double* Woff, double* Wsym,
                              int64_t ldw, int64_t m, int64_t n, const double* kpart, int layers, hipStream_t s) {
  hipError_t e;
  if (layers > 1 && (e = ksum(kpart, layers, m, n, Woff, ldw, s)) != hipSuccess) return e;
  const int cb = col_blocks(n);
  const double* Wo = Woff;
  OQR_GEMM_F64(cb, GEMM_DIAG, dim3(ceil_div(m, BM), ceil_div(n, 64 * cb), 1), Wsym, ldw, 0, 0, Wo, ldw);
  return hipGetLastError();
}

template <int MODE>
static hipError_t split_launch(const double* A, int64_t lda, const unsigned short* zs, double* out, int64_t ldo,
                               int64_t m, int64_t n, int slices, dim3 grid, int kchunk, int64_t stride, hipStream_t s) {
  const int cb = col_blocks(n), M = (int)m, N = (int)n;
  if (cb == 4) {
    if (slices == 2)
      gemm_split2_kernel<2, MODE><<<grid, NT2, 0, s>>>(A, lda, zs, out, ldo, M, N, kchunk, stride);
    else
      gemm_split2_kernel<3, MODE><<<grid, NT2, 0, s>>>(A, lda, zs, out, ldo, M, N, kchunk, stride);
  } else if (slices == 2) {
    if (cb == 1) gemm_split_kernel<2, 1, MODE><<<grid, NT, 0, s>>>(A, lda, zs, out, ldo, M, N, kchunk, stride);
    else gemm_split_kernel<2, 2, MODE><<<grid, NT, 0, s>>>(A, lda, zs, out, ldo, M, N, kchunk, stride);
  } else {
    if (cb == 1) gemm_split_kernel<3, 1, MODE><<<grid, NT, 0, s>>>(A, lda, zs, out, ldo, M, N, kchunk, stride);
    else gemm_split_kernel<3, 2, MODE><<<grid, NT, 0, s>>>(A, lda, zs, out, ldo, M, N, kchunk, stride);
  }
  return hipGetLastError();
}

hipError_t launch_gemm_split(const double* A, int64_t lda, const unsigned short* zs, double* W, int64_t ldw,
                             int64_t m, int64_t n, int slices, double* kpart, hipStream_t s) {
  const int cb = col_blocks(n);
  KSplit k = ksplit(m, n);
  if (!kpart) k = KSplit{1, (int)m};
  dim3 grid(ceil_div(m, BM), ceil_div(n, 64 * cb), k.ks);
  double* out = k.ks > 1 ? kpart : W;
  const int64_t ldo = k.ks > 1 ? m : ldw, stride = k.ks > 1 ? m * n : 0;
  hipError_t e = split_launch<GEMM_FULL>(A, lda, zs, out, ldo, m, n, slices, grid, k.kchunk, stride, s);
  if (e != hipSuccess || k.ks == 1) return e;
  return ksum(kpart, k.ks, m, n, W, ldw, s);
}

hipError_t launch_symm_split_upper(const double* A, int64_t lda, const unsigned short* zs, double* Woff, int64_t ldw,
                                   int64_t m, int64_t n, int slices, double* kpart, hipStream_t s) {
  const int cb = col_blocks(n);
  const int R = ceil_div(m, BM), P = (R + 1) / 2, ycb = ceil_div(n, 64 * cb);
  const int H = symm_layers(m, n, kpart);
  double* out = H > 1 ? kpart : Woff;
  const int64_t ldo = H > 1 ? m : ldw, stride = H > 1 ? m * n : 0;
  return split_launch<GEMM_UPPER>(A, lda, zs, out, ldo, m, n, slices, dim3(P, ycb, H), 0, stride, s);
}

size_t split_z_elems(int64_t m, int64_t n, int slices) {
  return (size_t)slices * split_ld(m) * (col_blocks(n) == 4 ? BN2 : n);
}

hipError_t launch_split_z(const double* Z, int64_t ldz, unsigned short* zs, int64_t m, int64_t n, int slices,
                          hipStream_t s) {
  const int64_t total = split_ld(m) * n / 4;     // threads: four rows each (split_ld is a multiple of 32)
  split_z_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(Z, ldz, zs, m, n, slices, col_blocks(n) == 4);
  return hipGetLastError();
}

}  // namespace oqr
