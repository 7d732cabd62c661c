// Small dense kernels of the CholQR pass: the n x n Cholesky factorisation of
// the Gram matrix (step 3 of Algorithm 1, R = chol(C)) with the shift-and-retry
// rule, the triangular product R = R2 R1 that combines two passes, and fills.
//
// Cholesky: one workgroup of 512 threads (8 waves), blocked left-looking with
// 32x32 blocks and a one-row lookahead, writing R in place.  For block row K:
//   (a) the diagonal block is factored by wave 0 in registers (lane j holds
//       column j; pivots and pivot rows broadcast by readlane), while waves
//       1..7 form the blocks (K+1, J) of G - sum_{P<K} R_P,K+1^T R_PJ on FP64
//       MFMA, reading the finished rows of R (L2-resident),
//   (b) the rest of block row K is solved column by column,
//       R_KJ = R_KK^{-T} (G_KJ - ...), written to R and kept in LDS,
//   (c) waves 1..7 subtract the term P = K from LDS: block row K+1 is ready.
// A pivot that is not positive (or NaN) restarts the factorisation from G with
// a larger diagonal shift; after the last retry the 1-based pivot index goes
// to info (LAPACK potrf convention).
#include "common.hpp"

#include <math.h>

namespace oqr {
namespace {

constexpr int CB = 32;
constexpr int NTC = 512;
constexpr int NW = NTC / 64;
constexpr int DPT = CB * CB / NTC;   // diagonal-block entries per thread

// v of lane l, in every lane (a register read, no LDS)
__device__ __forceinline__ double bcast_lane(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Factors the diagonal block Dk (CB x CB, upper triangle used) in place on one wave, in registers:
// lane j keeps column j; the pivot and pivot row k's entries are broadcast with readlane, so a pivot
// costs neither an LDS round trip nor a workgroup barrier.  Lanes j <= k keep their lower entries,
// which are never read; lanes 32..63 mirror 0..31 and store nothing.  1 / r_kk goes to rdiag; a pivot
// that is not positive (or NaN) stores its 1-based index plus k0 in *s_fail and leaves Dk unchanged.
// Kept out of line so that its 32 register columns do not add to the pressure of the MFMA update.
__device__ __noinline__ void diag_factor(double (*Dk)[CB + 1], double* rdiag, int* s_fail, int k0, int lane) {
  const int j = lane & (CB - 1);
  double d[CB];
#pragma unroll
  for (int i = 0; i < CB; ++i) d[i] = Dk[i][j];
  int fail = 0;
  // fully unrolled (constant register indices); after a failed pivot the rest is skipped, a
  // uniform branch since the pivot is a broadcast value
#pragma unroll
  for (int k = 0; k < CB; ++k) {
    if (fail == 0) {
      const double piv = bcast_lane(d[k], k);
      if (!(piv > 0.0)) {
        fail = k0 + k + 1;
      } else {
        const double ri = rsqrt_nr(piv), rkk = piv * ri;   // one refined reciprocal square root per pivot
        if (lane == 0) rdiag[k] = ri;
        d[k] = (j == k) ? rkk : ((j > k) ? d[k] * ri : d[k]);      // row k of R
#pragma unroll
        for (int i = k + 1; i < CB; ++i) d[i] = d[i] - bcast_lane(d[k], i) * d[k];   // r_ki r_kj
      }
    }
  }
  if (fail) {
    if (lane == 0) *s_fail = fail;
  } else if (lane < CB) {
#pragma unroll
    for (int i = 0; i < CB; ++i) Dk[i][j] = d[i];
  }
}

// Left-looking with a one-block-row lookahead.  Block row K + 1 is
//   G(K+1, J) - sum_{P <= K} R_{P,K+1}^T R_{P,J},
// and only its last term needs block row K.  So while wave 0 factors the diagonal block of row K,
// waves 1..7 accumulate the terms P < K of row K + 1 (one block each, R rows read from L2); after the
// solve of row K (kept in LDS) they add the term P = K, and row K + 1 is ready.  The terms are added
// in the same order (P ascending) as a plain left-looking sweep, so the factor does not depend on
// the lookahead.
__global__ __launch_bounds__(NTC) void chol_kernel(const double* __restrict__ G, int n, double* __restrict__ R,
                                                    int64_t ldr, double unit, double c_first, double c_retry,
                                                    int max_retries, int32_t* __restrict__ info,
                                                    double* __restrict__ shift_used) {
  __shared__ double Dk[1][CB][CB + 1];         // the diagonal block of block row K
  __shared__ double Dz[CB][CB + 1];            // its factor's strictly upper part, zero elsewhere
  __shared__ double P[CB][OQR_MAX_N + 2];     // block row K: P[p][j] = entry (k0 + p, j), j absolute column;
                                              // after the solve of row K, row K of R
  __shared__ double red[NW];
  __shared__ double rdiag[CB];                // 1 / r_kk of the current diagonal block
  __shared__ double s_dmax;
  __shared__ int s_fail;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  if (info[0] != 0) return;                   // an earlier pass failed
  const int nb = (n + CB - 1) / CB;

  // max_i G_ii (estimator of ||G||_2 for the shift)
  double v = (t < n) ? G[(int64_t)t * n + t] : 0.0;
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  if (lane == 0) red[wave] = v;
  __syncthreads();
  if (t == 0) {
    double mx = 0.0;
    for (int w = 0; w < NW; ++w) mx = fmax(mx, red[w]);
    s_dmax = mx;
  }
  __syncthreads();
  const double dmax = s_dmax;
  const int li = lane >> 4, lj = lane & 15;   // MFMA layouts
  // G (n x n) and R (n columns of ldr) through buffer resources; the host keeps n * ldr * 8 below 2^31
  const bufrsrc gbuf = make_buf(G, (int64_t)n * n * 8);
  const bufrsrc rbuf = make_buf(R, ((int64_t)(n - 1) * ldr + n) * 8);

  // block (KR, J) of G + s I (upper triangle; identity beyond n) into acc.  Branch-free buffer loads,
  // lanes outside the triangle masked with kOOB (they read 0), so that the 16 loads are in flight
  // together.
  auto load_g = [&](int KR, int J, double s, f64x4 (&acc)[2][2]) {
    const int r0 = KR * CB, J0 = J * CB;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = r0 + 16 * x + 4 * r + li, j = J0 + 16 * y + lj;
          const bool in = i < n && j < n && i <= j;
          acc[x][y][r] = buf_f64(gbuf, ((uint32_t)(j * n + i) * 8u) | (in ? 0u : kOOB));
        }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = r0 + 16 * x + 4 * r + li, j = J0 + 16 * y + lj;
          if (i == j) acc[x][y][r] = (i < n) ? acc[x][y][r] + s : 1.0;
        }
  };
  // acc -= sum over the finished block rows P < PEND of R_{P,KR}^T R_{P,J}, rows of R read from L2 in
  // chunks of 32 (8 MFMA k steps), the next chunk loaded during the current one
  auto update_l2 = [&](int KR, int J, int pend, f64x4 (&acc)[2][2]) {
    const int k0 = KR * CB, J0 = J * CB, kend = pend * CB;
    // byte offsets of this lane's entries of R in columns k0 + 16 x + lj (A operand) and
    // J0 + 16 x + lj (B operand), rows li + 4 u of a chunk; columns beyond n read 0
    uint32_t aoff[2], boff[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const int ca = k0 + 16 * x + lj, cb = J0 + 16 * x + lj;
      aoff[x] = ((uint32_t)((int64_t)ca * ldr + li) * 8u) | (ca < n ? 0u : kOOB);
      boff[x] = ((uint32_t)((int64_t)cb * ldr + li) * 8u) | (cb < n ? 0u : kOOB);
    }
    double a[8][2], b[8][2];
    auto load_chunk = [&](int p0, double (&aa)[8][2], double (&bb)[8][2]) {
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          aa[u][x] = buf_f64(rbuf, aoff[x] + (uint32_t)(p0 + 4 * u) * 8u);
          bb[u][x] = buf_f64(rbuf, boff[x] + (uint32_t)(p0 + 4 * u) * 8u);
        }
    };
    if (kend > 0) load_chunk(0, a, b);
    for (int p0 = 0; p0 < kend; p0 += CB) {          // kend is a multiple of 32
      double na[8][2], nbv[8][2];
      if (p0 + CB < kend) load_chunk(p0 + CB, na, nbv);
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) acc[x][y] = mfma_f64(-a[u][x], b[u][y], acc[x][y]);
      if (p0 + CB < kend) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int x = 0; x < 2; ++x) {
            a[u][x] = na[u][x];
            b[u][x] = nbv[u][x];
          }
      }
    }
  };
  // acc -= R_{K,KR}^T R_{K,J} from row K of R held in P (columns beyond n read 0, as from L2)
  auto update_lds = [&](int KR, int J, f64x4 (&acc)[2][2]) {
    const int k0 = KR * CB, J0 = J * CB;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      double a[2], b[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const int ca = k0 + 16 * x + lj, cb = J0 + 16 * x + lj;
        const double va = P[4 * u + li][ca], vb = P[4 * u + li][cb];
        a[x] = ca < n ? va : 0.0;
        b[x] = cb < n ? vb : 0.0;
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = mfma_f64(-a[x], b[y], acc[x][y]);
    }
  };
  auto store_block = [&](int KR, int J, const f64x4 (&acc)[2][2]) {
    const int J0 = J * CB;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * x + 4 * r + li, j = 16 * y + lj;
          if (J == KR) Dk[0][i][j] = acc[x][y][r];
          else P[i][J0 + j] = acc[x][y][r];
        }
  };

  double c = c_first;
  for (int attempt = 0;; ++attempt) {
    const double s = c * unit * dmax;
    if (t == 0) s_fail = 0;
    // block row 0: G itself
    if (wave < nb) {
      f64x4 acc[2][2];
      load_g(0, wave, s, acc);
      store_block(0, wave, acc);
    }
    __syncthreads();
    for (int K = 0; K < nb; ++K) {
      const int k0 = K * CB;
      // (a) wave 0 factors the diagonal block of row K in registers; waves 1..7 start block
      // (K + 1, K + w) of the next row with the terms of the rows before K
      f64x4 nxt[2][2];
      const int Jn = K + wave;                  // the next row's block of wave w (w >= 1)
      const bool has_next = wave >= 1 && K + 1 < nb && Jn < nb;
      if (wave == 0) {
        diag_factor(Dk[0], rdiag, &s_fail, k0, lane);
      } else if (has_next) {
        load_g(K + 1, Jn, s, nxt);
        update_l2(K + 1, Jn, K, nxt);
      }
      __syncthreads();
      if (s_fail) break;
      // (b) write the diagonal block; solve the rest of block row K, four lanes per column (lane `sub`
      // owns rows sub + 4e; pivots are broadcast within the quad); row K of R goes to R and stays in P
#pragma unroll
      for (int e = 0; e < DPT; ++e) {
        const int di = (t + NTC * e) >> 5, dj = (t + NTC * e) & 31;
        Dz[di][dj] = (di < dj) ? Dk[0][di][dj] : 0.0;
        if (k0 + di < n && k0 + dj < n) R[(int64_t)(k0 + dj) * ldr + k0 + di] = (di <= dj) ? Dk[0][di][dj] : 0.0;
      }
      __syncthreads();
      {
        const int sub = t & 3;
        for (int cb = k0 + CB; cb < n; cb += NTC / 4) {
          const int jcol = cb + (t >> 2);
          const bool ok = jcol < n;
          double x[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) x[e] = P[sub + 4 * e][ok ? jcol : 0];
#pragma unroll
          for (int p = 0; p < CB; ++p) {
            const int owner = p & 3, ep = p >> 2;
            // branch-free: every lane scales, the owner's value is broadcast
            const double q = quad_bcast(x[ep] * rdiag[p], owner);
            if (sub == owner) x[ep] = q;
            // entries at or left of the pivot meet a zero of Dz: x - 0 q = x, no select
#pragma unroll
            for (int e = 0; e < 8; ++e)
              if (4 * e + 3 > p) x[e] = x[e] - Dz[p][sub + 4 * e] * q;
            __builtin_amdgcn_sched_barrier(0);   // keep the LDS reads of one pivot row together
          }
          if (ok) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              P[sub + 4 * e][jcol] = x[e];
              if (k0 + sub + 4 * e < n) R[(int64_t)jcol * ldr + k0 + sub + 4 * e] = x[e];
            }
          }
        }
      }
      // strictly lower part of block column K (rows below the diagonal block) is zero
      for (int idx = t; idx < CB * n; idx += NTC) {
        const int j = k0 + idx % CB, i = k0 + CB + idx / CB;
        if (j < n && i < n) R[(int64_t)j * ldr + i] = 0.0;
      }
      __syncthreads();
      // (c) waves 1..7 add the term of row K and leave block row K + 1 in Dk / P.  Each wave reads the
      // columns of block K + 1 (never written here: that block goes to Dk) and of its own block, and
      // writes only its own block after reading it.
      if (has_next) {
        update_lds(K + 1, Jn, nxt);
        store_block(K + 1, Jn, nxt);
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

// R = R2 * R1 for upper triangular n x n factors, one workgroup per 16 x 16 tile of R.  Entry (i, j)
// sums R2(i, k) R1(k, j) over the K blocks of the tile row to the tile column in increasing k; the
// factors' entries with k < i or k > j are read as zero (whatever the lower parts hold), so those terms
// add exact zeros and each entry is the plain sum over k = i .. j.  The next K block is loaded into
// registers while the current one is multiplied from LDS.
__global__ __launch_bounds__(256) void trmm_upper_kernel(const double* __restrict__ R2, int64_t ld2,
                                                         const double* __restrict__ R1, int64_t ld1,
                                                         double* __restrict__ R, int64_t ldr, int n,
                                                         const int32_t* __restrict__ info) {
  __shared__ double As[16][17];               // R2(16 I + ti, 16 K + kk)
  __shared__ double Bs[16][17];               // R1(16 K + kk, 16 J + tj)
  const int I = blockIdx.y, J = blockIdx.x;
  const int ti = threadIdx.x & 15, tj = threadIdx.x >> 4;
  const int i = 16 * I + ti, j = 16 * J + tj;
  if (info && info[0] != 0) return;
  if (I > J) {                                // below the diagonal: zero
    if (i < n && j < n) R[(int64_t)j * ldr + i] = 0.0;
    return;
  }
  auto fetch = [&](int K, double& a, double& b) {
    const int ka = 16 * K + tj, kb = 16 * K + ti;
    a = (i < n && ka < n && ka >= i) ? R2[(int64_t)ka * ld2 + i] : 0.0;
    b = (kb < n && j < n && kb <= j) ? R1[(int64_t)j * ld1 + kb] : 0.0;
  };
  double a, b;
  fetch(I, a, b);
  double s = 0.0;
  for (int K = I; K <= J; ++K) {
    As[ti][tj] = a;
    Bs[ti][tj] = b;
    __syncthreads();
    if (K < J) fetch(K + 1, a, b);
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) s += As[ti][kk] * Bs[kk][tj];
    __syncthreads();
  }
  if (i < n && j < n) R[(int64_t)j * ldr + i] = s;
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

int device_cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cached[dev] = v;
  }
  return cached[dev] > 0 ? cached[dev] : 256;
}

hipError_t launch_chol_small(const double* G, int64_t n, double* R, int64_t ldr, double unit, double c_first,
                             double c_retry, int max_retries, int32_t* info, double* shift_used, hipStream_t s) {
  chol_kernel<<<1, NTC, 0, s>>>(G, (int)n, R, ldr, unit, c_first, c_retry, max_retries, info, shift_used);
  return hipGetLastError();
}

hipError_t launch_trmm_upper(const double* R2, int64_t ld2, const double* R1, int64_t ld1, double* R, int64_t ldr,
                             int64_t n, const int32_t* info, hipStream_t s) {
  const unsigned tiles = (unsigned)((n + 15) / 16);
  trmm_upper_kernel<<<dim3(tiles, tiles), 256, 0, s>>>(R2, ld2, R1, ld1, R, ldr, (int)n, info);
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
