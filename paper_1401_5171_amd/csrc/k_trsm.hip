// Triangular solve Q = Z R^{-1} (step 4 of CHOLQR, Algorithm 1), FP64.
//
// Each row of Q solves q_i R = z_i, the row-wise solve whose backward error
// |dR^i| <= c n u |R| gives the residual bound of Theorem 2.1.  Column blocks
// of 32 are processed left to right:
//   (1) Z_J -= Q_{<J} R_{<J,J}    FP64 MFMA (a blocked form of the same sums)
//   (2) Q_J  = Z_J R_JJ^{-1}       substitution, k ascending, 4 lanes per row;
//       the pivot is applied as a product with 1/r_kk (computed once per
//       workgroup), which perturbs r_kk by one more rounding and keeps the
//       componentwise backward error bound.
// A workgroup owns BMR = 64 rows x all n <= 128 columns, staged once in LDS (Z is
// read from HBM once and Q written once, column-coalesced, at the end).  Q may
// alias Z: the whole row block of Z is in LDS before any of its Q is written.
// For 128 < n <= 256, trsm_wide_kernel (32-row blocks, right-looking updates).
#include "common.hpp"

namespace oqr {
namespace {

constexpr int JB = 32;
constexpr int NT = 256;

template <int NMAX, int BMR>
__global__ __launch_bounds__(NT, 2) void trsm_kernel(const double* Z, int64_t ldz, const double* __restrict__ R,
                                                     int64_t ldr, double* Q, int64_t ldq, int m, int n,
                                                     const int32_t* __restrict__ info) {
  constexpr int LDQ = BMR + 1;               // LDS column stride (doubles)
  __shared__ double Qs[NMAX * LDQ];          // Qs[j * LDQ + i]: row i of the block, column j
  // strictly upper part of R_JJ, per column owner: RZ[c][sub * 8 + e] = R(j0 + c, j0 + sub + 4e)
  // for sub + 4e > c, else 0; rinv[c] = 1 / R(j0 + c, j0 + c).  Staged at the start of block J,
  // after the barrier that ends the previous block's substitution (its last reader).
  __shared__ __attribute__((aligned(16))) double RZ[JB][JB];
  __shared__ double rinv[JB];
  if (info[0] != 0) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int i0 = blockIdx.x * BMR;
  const int nblk = (n + JB - 1) / JB;
  const bufrsrc rb_ = make_buf(R, ((int64_t)(n - 1) * ldr + n) * 8);

  auto stage_r = [&](int J) {
    const int j0 = J * JB;
    for (int idx = t; idx < JB * JB; idx += NT) {
      const int c = idx / JB, q = idx % JB, sub = q >> 3, e = q & 7;
      const int col = sub + 4 * e;
      const int gr = j0 + c, gc = j0 + col;
      RZ[c][q] = (col > c && gc < n) ? R[(int64_t)gc * ldr + gr] : 0.0;
    }
    if (t < JB) {
      const int g = j0 + t;
      rinv[t] = (g < n) ? 1.0 / R[(int64_t)g * ldr + g] : 1.0;
    }
  };

  // load the Z row block (column-major: BMR contiguous rows per column), 16 loads in flight per thread
  {
    constexpr int STRIDE = NT / BMR;
    const int i = t % BMR, jq = t / BMR;
    const bool ok = i0 + i < m;
#pragma unroll
    for (int jb = 0; jb < NMAX; jb += 16 * STRIDE) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int j = jb + jq + STRIDE * u;
        v[u] = sel_load(Z, (int64_t)j * ldz + i0 + i, ok && j < n);
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) Qs[(jb + jq + STRIDE * u) * LDQ + i] = v[u];
    }
  }
  __syncthreads();

  const int li = lane >> 4, lj = lane & 15;
  // MFMA tiles of the update: BMR = 64: wave = 16-row block, both 16-column halves;
  //                           BMR = 32: wave = (16-row block, half)
  constexpr int NH = (BMR == 64) ? 2 : 1;
  const int rb = (BMR == 64) ? wave : (wave >> 1);
  const int h0 = (BMR == 64) ? 0 : (wave & 1);
  const int row = t >> 2, sub = t & 3;      // substitution: 4 lanes per row
  for (int J = 0; J < nblk; ++J) {
    const int j0 = J * JB;
    stage_r(J);
    // (1) block update on MFMA
    if (J > 0) {
      f64x4 acc[NH];
#pragma unroll
      for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[h][r] = Qs[(j0 + 16 * (h0 + h) + lj) * LDQ + rb * 16 + 4 * r + li];
      // byte offsets of this lane's R entries (column jc, rows li + ..); columns beyond n read 0.  R
      // spans less than 2^31 bytes (the host checks n * ldr).
      uint32_t rco[NH], rcm[NH];
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const int jc = j0 + 16 * (h0 + h) + lj;
        rco[h] = (uint32_t)((int64_t)jc * ldr + li) * 8u;
        rcm[h] = jc < n ? 0u : kOOB;
      }
      // R fragments are read from L2 in chunks of 32 k (8 MFMA steps), one chunk ahead; branch-free
      // buffer loads (a chunk past j0 is masked with kOOB), so the loads overlap the products
      double bf[NH][8];
#pragma unroll
      for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int s = 0; s < 8; ++s) bf[h][s] = buf_f64(rb_, (rco[h] + (uint32_t)(4 * s) * 8u) | rcm[h]);
      for (int kc = 0; kc < j0; kc += 32) {
        double nb[NH][8];
        const uint32_t mm = kc + 32 < j0 ? 0u : kOOB;
#pragma unroll
        for (int h = 0; h < NH; ++h)
#pragma unroll
          for (int s = 0; s < 8; ++s)
            nb[h][s] = buf_f64(rb_, (rco[h] + (uint32_t)(kc + 32 + 4 * s) * 8u) | rcm[h] | mm);
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int kr = kc + 4 * s + li;
          const double a = -Qs[kr * LDQ + rb * 16 + lj];
#pragma unroll
          for (int h = 0; h < NH; ++h) acc[h] = mfma_f64(a, bf[h][s], acc[h]);
        }
#pragma unroll
        for (int h = 0; h < NH; ++h)
#pragma unroll
          for (int s = 0; s < 8; ++s) bf[h][s] = nb[h][s];
      }
      // columns j0.. are written, columns < j0 were read: disjoint, no barrier in between
#pragma unroll
      for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) Qs[(j0 + 16 * (h0 + h) + lj) * LDQ + rb * 16 + 4 * r + li] = acc[h][r];
    }
    __syncthreads();
    // (2) substitution on the 32 columns of the block: lane `sub` of a row owns columns sub + 4e
    if (row < BMR) {
      double x[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = Qs[(j0 + sub + 4 * e) * LDQ + row];
      // the operands of step c + 1 are read from LDS during step c (one wave per SIMD hides nothing)
      double rzc[8], rzn[8], ric = rinv[0], rin = 1.0;
      #pragma unroll
      for (int e = 0; e < 8; ++e) rzc[e] = RZ[0][sub * 8 + e];
      #pragma unroll
      for (int c = 0; c < JB; ++c) {
        if (c + 1 < JB) {
      #pragma unroll
          for (int e = 0; e < 8; ++e) rzn[e] = RZ[c + 1][sub * 8 + e];
          rin = rinv[c + 1];
        }
        const int owner = c & 3, ec = c >> 2;
        const double q = quad_bcast(x[ec] * ric, owner);
        // columns sub + 4e <= c are final: e below (c - 3) / 4 is skipped for every lane
      #pragma unroll
        for (int e = 0; e < 8; ++e)
          if (4 * e + 3 > c) x[e] = __builtin_fma(-q, rzc[e], x[e]);
      #pragma unroll
        for (int e = 0; e < 8; ++e) rzc[e] = rzn[e];
        ric = rin;
      }
      // a settled column meets only zeros of RZ, so each x[e] still holds its pivot's numerator: the
      // scale by 1 / r_kk, made where the pivot was broadcast, is made here once more (same product)
#pragma unroll
      for (int e = 0; e < 8; ++e) Qs[(j0 + sub + 4 * e) * LDQ + row] = x[e] * rinv[sub + 4 * e];
    }
    __syncthreads();
  }
  // store Q: column-major, BMR contiguous rows per column
  {
    constexpr int STRIDE = NT / BMR;
    const int i = t % BMR, jq = t / BMR;
    if (i0 + i < m) {
      for (int j = jq; j < n; j += STRIDE) Q[(int64_t)j * ldq + i0 + i] = Qs[j * LDQ + i];
    }
  }
}

// Right-looking variant for 128 < n <= 256 (32-row blocks, two workgroups per CU): after the
// substitution of column block J, every column right of it is updated at once,
//   Z_{>J} -= Q_J R_{J,>J}            FP64 MFMA, one K step of 32 per update,
// so that a wave owns up to four 16-column tiles of both 16-row blocks (eight independent chains,
// each pair sharing its R fragments) instead of one chain over all earlier columns.  The R fragments
// of the update (row block J of R, columns right of it) are requested before the substitution and
// arrive while it runs, and the next diagonal block of R one block ahead.  The substitution itself
// is the one of trsm_kernel (4 lanes per row, FP64, pivots as products with 1/r_kk).
constexpr int WNMAX = 256, WBMR = 32, WLDQ = WBMR + 1;
constexpr int WCT = 4;                       // column tiles per wave (up to 14 right of block 0)
__global__ __launch_bounds__(NT, 2) void trsm_wide_kernel(const double* Z, int64_t ldz, const double* __restrict__ R,
                                                          int64_t ldr, double* Q, int64_t ldq, int m, int n,
                                                          const int32_t* __restrict__ info) {
  __shared__ double Qs[WNMAX * WLDQ];        // Qs[j * WLDQ + i]: row i of the block, column j
  __shared__ __attribute__((aligned(16))) double RZ[JB][JB];
  __shared__ double rinv[JB];
  if (info[0] != 0) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int i0 = blockIdx.x * WBMR;
  const int nblk = (n + JB - 1) / JB;
  const int nct = (n + 15) / 16;             // 16-column tiles of Q
  const bufrsrc rb_ = make_buf(R, ((int64_t)(n - 1) * ldr + n) * 8);

  // load the Z row block (column-major: 32 contiguous rows per column)
  {
    constexpr int STRIDE = NT / WBMR;
    const int i = t % WBMR, jq = t / WBMR;
    const bool ok = i0 + i < m;
#pragma unroll
    for (int jb = 0; jb < WNMAX; jb += 16 * STRIDE) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int j = jb + jq + STRIDE * u;
        v[u] = sel_load(Z, (int64_t)j * ldz + i0 + i, ok && j < n);
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) Qs[(jb + jq + STRIDE * u) * WLDQ + i] = v[u];
    }
  }

  const int li = lane >> 4, lj = lane & 15;
  const int row = t >> 2, sub = t & 3;       // substitution: 4 lanes per row
  // R_JJ entries of this thread (strictly upper part per column owner; zero elsewhere) and, for t < 32,
  // the pivot r_kk: requested one block ahead (branch-free buffer loads, masked entries read zero)
  double rzp[JB * JB / NT], rdp = 1.0;
  auto fetch_diag = [&](int J) {
    const int j0 = J * JB;
#pragma unroll
    for (int w = 0; w < JB * JB / NT; ++w) {
      const int idx = t + NT * w, c = idx / JB, q = idx % JB, sb = q >> 3, e = q & 7;
      const int col = sb + 4 * e, gr = j0 + c, gc = j0 + col;
      const uint32_t msk = (col > c && gc < n) ? 0u : kOOB;
      rzp[w] = buf_f64(rb_, (uint32_t)((int64_t)gc * ldr + gr) * 8u | msk);
    }
    const int g = j0 + (t & (JB - 1));
    rdp = buf_f64(rb_, (uint32_t)((int64_t)g * ldr + g) * 8u | (g < n ? 0u : kOOB));
  };
  fetch_diag(0);
  for (int J = 0; J < nblk; ++J) {
    const int j0 = J * JB;
    // R_JJ into LDS (RZ, rinv); the previous block's update (the last reader of RZ is the previous
    // substitution) ended with a barrier
#pragma unroll
    for (int w = 0; w < JB * JB / NT; ++w) {
      const int idx = t + NT * w;
      RZ[idx / JB][idx % JB] = rzp[w];
    }
    if (t < JB) rinv[t] = (j0 + t < n) ? 1.0 / rdp : 1.0;
    if (J + 1 < nblk) fetch_diag(J + 1);     // in flight during this block's substitution and update
    // R fragments of this block's update: the wave's column tiles are ct0 + wave + 4 v; lane (li, lj)
    // holds R(j0 + 4 s + li, 16 ct + lj), s = 0..7.  Columns past n, or tiles past the last, read zero.
    const int ct0 = (j0 + JB) / 16;
    double bf[WCT][8];
#pragma unroll
    for (int v = 0; v < WCT; ++v) {
      const int ct = ct0 + wave + 4 * v, col = 16 * ct + lj;
      const uint32_t base = (uint32_t)((int64_t)col * ldr + j0 + li) * 8u;
      const uint32_t msk = (ct < nct && col < n) ? 0u : kOOB;
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2) bf[v][s2] = buf_f64(rb_, (base + 32u * s2) | msk);
    }
    __syncthreads();
    // substitution on the 32 columns of block J: lane `sub` of a row owns columns sub + 4e
    if (row < WBMR) {
      double x[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = Qs[(j0 + sub + 4 * e) * WLDQ + row];
      double rzc[8], rzn[8], ric = rinv[0], rin = 1.0;
#pragma unroll
      for (int e = 0; e < 8; ++e) rzc[e] = RZ[0][sub * 8 + e];
#pragma unroll
      for (int c = 0; c < JB; ++c) {
        if (c + 1 < JB) {
#pragma unroll
          for (int e = 0; e < 8; ++e) rzn[e] = RZ[c + 1][sub * 8 + e];
          rin = rinv[c + 1];
        }
        const int owner = c & 3, ec = c >> 2;
        const double q = quad_bcast(x[ec] * ric, owner);
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (4 * e + 3 > c) x[e] = __builtin_fma(-q, rzc[e], x[e]);
#pragma unroll
        for (int e = 0; e < 8; ++e) rzc[e] = rzn[e];
        ric = rin;
      }
      // pivots scaled once more here (settled columns met only zeros of RZ): same products as at the
      // broadcast
#pragma unroll
      for (int e = 0; e < 8; ++e) Qs[(j0 + sub + 4 * e) * WLDQ + row] = x[e] * rinv[sub + 4 * e];
    }
    __syncthreads();
    // right-looking update of the columns right of block J: independent 16 x 16 tiles, K = 32
    if (j0 + JB < n) {
      double a[2][8];                        // -Q(16 rb + lj, j0 + 4 s + li) for both row blocks
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int s2 = 0; s2 < 8; ++s2) a[rb][s2] = -Qs[(j0 + 4 * s2 + li) * WLDQ + 16 * rb + lj];
#pragma unroll
      for (int v = 0; v < WCT; ++v) {
        const int ct = ct0 + wave + 4 * v;
        if (ct < nct) {                      // wave-uniform
          f64x4 acc[2];
#pragma unroll
          for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[rb][r] = Qs[(16 * ct + lj) * WLDQ + 16 * rb + 4 * r + li];
#pragma unroll
          for (int s2 = 0; s2 < 8; ++s2)
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) acc[rb] = mfma_f64(a[rb][s2], bf[v][s2], acc[rb]);
#pragma unroll
          for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) Qs[(16 * ct + lj) * WLDQ + 16 * rb + 4 * r + li] = acc[rb][r];
        }
      }
    }
    __syncthreads();
  }
  // store Q: column-major, 32 contiguous rows per column
  {
    constexpr int STRIDE = NT / WBMR;
    const int i = t % WBMR, jq = t / WBMR;
    if (i0 + i < m) {
      for (int j = jq; j < n; j += STRIDE) Q[(int64_t)j * ldq + i0 + i] = Qs[j * WLDQ + i];
    }
  }
}

// Persistent variant for n <= NMAX <= 128 and many row tiles: one workgroup per CU walks the tiles
// blockIdx.x, + gridDim.x, ...  R is the same for every tile, so each wave keeps the R fragments of
// its MFMA updates in registers and the diagonal blocks stay in LDS for the whole launch; the next
// tile's Z is loaded into registers while the current tile is solved.  Same operations in the same
// order as trsm_kernel<NMAX, 64>, so the results are identical.
template <int NMAX>
__global__ __launch_bounds__(NT, 1) void trsm_persist_kernel(const double* Z, int64_t ldz,
                                                             const double* __restrict__ R, int64_t ldr, double* Q,
                                                             int64_t ldq, int m, int n, int ntiles,
                                                             const int32_t* __restrict__ info) {
  constexpr int BMR = 64, LDQ = BMR + 1, NBLK = NMAX / JB;
  constexpr int NF = 8 * NBLK * (NBLK - 1) / 2;   // R fragments per lane and half: sum over J of 8 J
  __shared__ double Qs[NMAX * LDQ];
  __shared__ __attribute__((aligned(16))) double RZ[NBLK][JB][JB];
  __shared__ double rinv[NBLK][JB];
  if (info[0] != 0) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int li = lane >> 4, lj = lane & 15;
  const int nblk = (n + JB - 1) / JB;
  // diagonal blocks, once
  for (int idx = t; idx < NBLK * JB * JB; idx += NT) {
    const int J = idx / (JB * JB), c = (idx / JB) % JB, q = idx % JB, sub = q >> 3, e = q & 7;
    const int col = sub + 4 * e, gr = J * JB + c, gc = J * JB + col;
    RZ[J][c][q] = (col > c && gc < n) ? R[(int64_t)gc * ldr + gr] : 0.0;
  }
  for (int idx = t; idx < NBLK * JB; idx += NT) {
    const int g = idx;
    rinv[idx / JB][idx % JB] = (g < n) ? 1.0 / R[(int64_t)g * ldr + g] : 1.0;
  }
  // off-diagonal R fragments, once: rf[h][off(J) + s] = R(4 s + li, j0 + 16 h + lj), s < 8 J
  double rf[2][NF > 0 ? NF : 1];
#pragma unroll
  for (int J = 1; J < NBLK; ++J) {
    const int off = 8 * J * (J - 1) / 2;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int jc = J * JB + 16 * h + lj;
#pragma unroll
      for (int s2 = 0; s2 < 8 * J; ++s2) {
        const int k = 4 * s2 + li;
        rf[h][off + s2] = (jc < n && k < n) ? R[(int64_t)jc * ldr + k] : 0.0;
      }
    }
  }
  // Z tile prefetch: thread (row i = t % 64, columns jq + 4u)
  constexpr int PU = NMAX / 4;
  const int pi = t % BMR, pj = t / BMR;
  double zr[PU];
  auto prefetch = [&](int tile) {
    const int row = min(tile * BMR + pi, m - 1);
#pragma unroll
    for (int u = 0; u < PU; ++u) zr[u] = Z[(int64_t)min(pj + 4 * u, n - 1) * ldz + row];
  };
  const int row = t >> 2, sub = t & 3;      // substitution: 4 lanes per row
  int tile = blockIdx.x;
  if (tile < ntiles) prefetch(tile);
  for (; tile < ntiles; tile += gridDim.x) {
    const int i0 = tile * BMR;
#pragma unroll
    for (int u = 0; u < PU; ++u) Qs[(pj + 4 * u) * LDQ + pi] = (pj + 4 * u < n) ? zr[u] : 0.0;
    __syncthreads();
    if (tile + (int)gridDim.x < ntiles) prefetch(tile + gridDim.x);
#pragma unroll
    for (int J = 0; J < NBLK; ++J) {
      if (J >= nblk) break;
      const int j0 = J * JB;
      if (J > 0) {
        const int off = 8 * J * (J - 1) / 2;
        f64x4 acc[2];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[h][r] = Qs[(j0 + 16 * h + lj) * LDQ + wave * 16 + 4 * r + li];
#pragma unroll
        for (int s2 = 0; s2 < 8 * J; ++s2) {
          const double a = -Qs[(4 * s2 + li) * LDQ + wave * 16 + lj];
          acc[0] = mfma_f64(a, rf[0][off + s2], acc[0]);
          acc[1] = mfma_f64(a, rf[1][off + s2], acc[1]);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int r = 0; r < 4; ++r) Qs[(j0 + 16 * h + lj) * LDQ + wave * 16 + 4 * r + li] = acc[h][r];
      }
      __syncthreads();
      {
        double x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = Qs[(j0 + sub + 4 * e) * LDQ + row];
        // the operands of step c + 1 are read from LDS during step c (one wave per SIMD hides nothing)
        double rzc[8], rzn[8], ric = rinv[J][0], rin = 1.0;
        #pragma unroll
        for (int e = 0; e < 8; ++e) rzc[e] = RZ[J][0][sub * 8 + e];
        #pragma unroll
        for (int c = 0; c < JB; ++c) {
          if (c + 1 < JB) {
        #pragma unroll
            for (int e = 0; e < 8; ++e) rzn[e] = RZ[J][c + 1][sub * 8 + e];
            rin = rinv[J][c + 1];
          }
          const int owner = c & 3, ec = c >> 2;
          const double q = quad_bcast(x[ec] * ric, owner);
          // columns sub + 4e <= c are final: e below (c - 3) / 4 is skipped for every lane
        #pragma unroll
          for (int e = 0; e < 8; ++e)
            if (4 * e + 3 > c) x[e] = __builtin_fma(-q, rzc[e], x[e]);
        #pragma unroll
          for (int e = 0; e < 8; ++e) rzc[e] = rzn[e];
          ric = rin;
        }
        // pivots scaled once more here (settled columns met only zeros of RZ): same products as at the
        // broadcast
#pragma unroll
        for (int e = 0; e < 8; ++e) Qs[(j0 + sub + 4 * e) * LDQ + row] = x[e] * rinv[J][sub + 4 * e];
      }
      __syncthreads();
    }
    if (i0 + pi < m) {
      for (int j = pj; j < n; j += 4) Q[(int64_t)j * ldq + i0 + pi] = Qs[j * LDQ + pi];
    }
    __syncthreads();
  }
}

// Persistent variant for 64 < n <= 128 with 128-row tiles: one workgroup (four waves, one per SIMD)
// per CU; every thread carries two rows (t / 4 and t / 4 + 64) through the substitution, so two
// independent chains share each pivot's R row, and every wave updates four 16-row blocks of one
// 16-column half on MFMA (four accumulator chains, half the R fragments of a wave in registers).
// Row c of a diagonal block of R is kept from column 4 floor(c / 4) on (the first column a lane of the
// quad can hold at step c), with zeros in columns <= c, so that the 128-row tile fits in LDS and the
// update of step c needs no per-lane select: a settled column meets a zero and keeps its value.  The
// pivot is scaled by 1 / R(c, c) where it is broadcast, and each lane's own columns once the block is
// done, which gives the same product.  The R fragments take the registers a next-tile prefetch would
// need, so a tile's Z is loaded at its start.  Every entry is formed by the same operations in the same
// order as in trsm_persist_kernel instantiated for 128 columns, so the results are identical (but for
// the sign of an exact zero).
constexpr int NM2 = 128, BM2 = 128, LDQ2 = BM2 + 1, NBLK2 = NM2 / JB;

__host__ __device__ constexpr int rz_row(int c) {        // start of row c: groups of four rows of 32 - 4 g
  return 128 * (c >> 2) - 8 * (c >> 2) * ((c >> 2) - 1) + (c & 3) * (JB - 4 * (c >> 2));
}
constexpr int RZP = rz_row(JB);                          // entries of one diagonal block (576)

__global__ __launch_bounds__(NT, 1) void trsm_persist2_kernel(const double* Z, int64_t ldz,
                                                              const double* __restrict__ R, int64_t ldr,
                                                              double* Q, int64_t ldq, int m, int n, int ntiles,
                                                              const int32_t* __restrict__ info) {
  constexpr int NF = 8 * NBLK2 * (NBLK2 - 1) / 2;
  __shared__ double Qs[NM2 * LDQ2];               // Qs[j * LDQ2 + i]: row i of the tile, column j
  __shared__ double RZ[NBLK2][RZP];               // R(j0 + c, j0 + col), col >= 4 floor(c / 4), by rows
  __shared__ double rinv[NBLK2][JB];
  if (info[0] != 0) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int li = lane >> 4, lj = lane & 15;
  const int nblk = (n + JB - 1) / JB;
  for (int idx = t; idx < NBLK2 * RZP; idx += NT) {
    const int J = idx / RZP, k = idx % RZP;
    int c = 0;
    while (k >= rz_row(c + 1)) ++c;
    const int col = 4 * (c >> 2) + (k - rz_row(c)), gr = J * JB + c, gc = J * JB + col;
    RZ[J][k] = (col > c && gc < n) ? R[(int64_t)gc * ldr + gr] : 0.0;
  }
  for (int idx = t; idx < NBLK2 * JB; idx += NT)
    rinv[idx / JB][idx % JB] = (idx < n) ? 1.0 / R[(int64_t)idx * ldr + idx] : 1.0;
  // MFMA update: wave w owns column half hw = w & 1 of every block and the four 16-row blocks
  // 4 (w >> 1) .. 4 (w >> 1) + 3, so it keeps the R fragments of its half only:
  // rf[off(J) + s] = R(4 s + li, j0 + 16 hw + lj), s < 8 J
  const int hw = wave & 1, rb0 = 4 * (wave >> 1);
  double rf[NF];
#pragma unroll
  for (int J = 1; J < NBLK2; ++J) {
    const int off = 8 * J * (J - 1) / 2;
    const int jc = J * JB + 16 * hw + lj;
#pragma unroll
    for (int s2 = 0; s2 < 8 * J; ++s2) {
      const int kk = 4 * s2 + li;
      rf[off + s2] = (jc < n && kk < n) ? R[(int64_t)jc * ldr + kk] : 0.0;
    }
  }
  // Z tile: thread (row pi = t % 128, columns pj + 2u), in groups of 16 loads (no registers held
  // across the tile: the R fragments fill them)
  constexpr int PU = NM2 / 2;
  const int pi = t % BM2, pj = t / BM2;
  const int row = t >> 2, sub = t & 3;      // substitution rows row and row + 64, 4 lanes per row
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int i0 = tile * BM2;
    {
      const int zrow = min(i0 + pi, m - 1);
#pragma unroll
      for (int u0 = 0; u0 < PU; u0 += 16) {
        double zr[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) zr[u] = Z[(int64_t)min(pj + 2 * (u0 + u), n - 1) * ldz + zrow];
#pragma unroll
        for (int u = 0; u < 16; ++u) Qs[(pj + 2 * (u0 + u)) * LDQ2 + pi] = (pj + 2 * (u0 + u) < n) ? zr[u] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int J = 0; J < NBLK2; ++J) {
      if (J >= nblk) break;
      const int j0 = J * JB;
      if (J > 0) {
        const int off = 8 * J * (J - 1) / 2;
        f64x4 acc[4];                             // row block rb0 + b, column half hw
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[b][r] = Qs[(j0 + 16 * hw + lj) * LDQ2 + (rb0 + b) * 16 + 4 * r + li];
#pragma unroll
        for (int s2 = 0; s2 < 8 * J; ++s2) {
#pragma unroll
          for (int b = 0; b < 4; ++b)
            acc[b] = mfma_f64(-Qs[(4 * s2 + li) * LDQ2 + (rb0 + b) * 16 + lj], rf[off + s2], acc[b]);
          __builtin_amdgcn_sched_barrier(0);    // operand reads of one K step at a time
        }
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) Qs[(j0 + 16 * hw + lj) * LDQ2 + (rb0 + b) * 16 + 4 * r + li] = acc[b][r];
      }
      __syncthreads();
      {
        double x0[8], x1[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          x0[e] = Qs[(j0 + sub + 4 * e) * LDQ2 + row];
          x1[e] = Qs[(j0 + sub + 4 * e) * LDQ2 + row + 64];
        }
        // R row c of the block for this lane's columns sub + 4e, staged one step ahead (columns of
        // groups below c / 4 are settled for every lane and neither read nor updated)
        double rzc[8], rzn[8], ric = rinv[J][0], rin = 1.0;
        const double* rzl = &RZ[J][sub];
        auto stage = [&](double (&v)[8], int c) {
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if (4 * e + 3 > c) v[e] = rzl[rz_row(c) + 4 * (e - (c >> 2))];
        };
        stage(rzc, 0);
#pragma unroll
        for (int c = 0; c < JB; ++c) {
          if (c + 1 < JB) {
            stage(rzn, c + 1);
            rin = rinv[J][c + 1];
          }
          const int owner = c & 3, ec = c >> 2;
          const double q0 = quad_bcast(x0[ec] * ric, owner);
          const double q1 = quad_bcast(x1[ec] * ric, owner);
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if (4 * e + 3 > c) {
              x0[e] = __builtin_fma(-q0, rzc[e], x0[e]);
              x1[e] = __builtin_fma(-q1, rzc[e], x1[e]);
            }
#pragma unroll
          for (int e = 0; e < 8; ++e) rzc[e] = rzn[e];
          ric = rin;
          __builtin_amdgcn_sched_barrier(0);    // the R row of step c + 1 only
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const double ri = rinv[J][sub + 4 * e];
          Qs[(j0 + sub + 4 * e) * LDQ2 + row] = x0[e] * ri;
          Qs[(j0 + sub + 4 * e) * LDQ2 + row + 64] = x1[e] * ri;
        }
      }
      __syncthreads();
    }
    if (i0 + pi < m) {
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        const int j = pj + 2 * u;
        if (j < n) Q[(int64_t)j * ldq + i0 + pi] = Qs[j * LDQ2 + pi];
      }
    }
    __syncthreads();
  }
}

// W = A Z for the 7-point operator (Dirichlet boundary, index p = x + nx (y + ny z)).
// A thread owns one (x, y) point of one column and marches through z: the values at z-1, z and z+1
// stay in registers, so each plane is read from HBM once; the four in-plane neighbours come from
// lines that the same and adjacent waves load (cache hits).  Centres are fetched two planes ahead,
// neighbours one plane ahead, with buffer loads whose out-of-grid offsets read as zero.
__global__ __launch_bounds__(256) void stencil_march_kernel(const double* __restrict__ Z, int64_t ldz,
                                                             double* __restrict__ W, int64_t ldw, int nx, int ny,
                                                             int nz, double center, double off) {
  const int64_t sxy = (int64_t)nx * ny;
  const int64_t m = sxy * nz;
  const int j = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // point of the plane
  if (idx >= sxy) return;
  const int x = (int)(idx % nx), y = (int)(idx / nx);
  const bufrsrc zb = make_buf(Z + (int64_t)j * ldz, m * 8);
  double* w = W + (int64_t)j * ldw + idx;
  const bool xl = x > 0, xr = x < nx - 1, yl = y > 0, yr = y < ny - 1;
  auto at = [&](int zz, int d, bool ok) -> uint32_t {
    return (ok && zz >= 0 && zz < nz) ? (uint32_t)(((int64_t)zz * sxy + idx + d) * 8) : kOOB;
  };
  double cm = 0.0;
  double c0 = buf_f64(zb, at(0, 0, true));
  double cp = buf_f64(zb, at(1, 0, true));
  double n0 = buf_f64(zb, at(0, -1, xl)), n1 = buf_f64(zb, at(0, 1, xr));
  double n2 = buf_f64(zb, at(0, -nx, yl)), n3 = buf_f64(zb, at(0, nx, yr));
  for (int z = 0; z < nz; ++z) {
    const double cpp = buf_f64(zb, at(z + 2, 0, true));
    const double p0 = buf_f64(zb, at(z + 1, -1, xl)), p1 = buf_f64(zb, at(z + 1, 1, xr));
    const double p2 = buf_f64(zb, at(z + 1, -nx, yl)), p3 = buf_f64(zb, at(z + 1, nx, yr));
    w[(int64_t)z * sxy] = center * c0 + off * (((n0 + n1) + (n2 + n3)) + (cm + cp));
    cm = c0;
    c0 = cp;
    cp = cpp;
    n0 = p0;
    n1 = p1;
    n2 = p2;
    n3 = p3;
  }
}

}  // namespace

hipError_t launch_trsm(const double* Z, int64_t ldz, const double* R, int64_t ldr, double* Q, int64_t ldq,
                       int64_t m, int64_t n, const int32_t* info, hipStream_t s) {
  const int64_t ntiles = (m + 63) / 64;
  const int cus = device_cu_count();
  if (n <= 128 && ntiles >= 4 * cus && ntiles < 0x7fffffff) {
    const int grid = (n <= 64) ? 2 * cus : cus;   // 188 / 388 VGPRs: two or one workgroup per CU
    if (n <= 64) {
      trsm_persist_kernel<64><<<grid, NT, 0, s>>>(Z, ldz, R, ldr, Q, ldq, (int)m, (int)n, (int)ntiles, info);
    } else {
      const int64_t nt2 = (m + BM2 - 1) / BM2;
      trsm_persist2_kernel<<<grid, NT, 0, s>>>(Z, ldz, R, ldr, Q, ldq, (int)m, (int)n, (int)nt2, info);
    }
    return hipGetLastError();
  }
  if (n <= 64)
    trsm_kernel<64, 64><<<ceil_div(m, 64), NT, 0, s>>>(Z, ldz, R, ldr, Q, ldq, (int)m, (int)n, info);
  else if (n <= 128)
    trsm_kernel<128, 64><<<ceil_div(m, 64), NT, 0, s>>>(Z, ldz, R, ldr, Q, ldq, (int)m, (int)n, info);
  else
    trsm_wide_kernel<<<ceil_div(m, WBMR), NT, 0, s>>>(Z, ldz, R, ldr, Q, ldq, (int)m, (int)n, info);
  return hipGetLastError();
}

// W = A Z for a symmetric tridiagonal A stored as t = [diagonal (m), off-diagonal (m - 1)].
__global__ void tridiag_apply_kernel(const double* __restrict__ t, int64_t m, const double* __restrict__ Z,
                                     int64_t ldz, double* __restrict__ W, int64_t ldw, int64_t n) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * n) return;
  const int64_t j = idx / m, i = idx % m;
  const double* z = Z + j * ldz;
  double w = t[i] * z[i];
  if (i > 0) w += t[m + i - 1] * z[i - 1];
  if (i + 1 < m) w += t[m + i] * z[i + 1];
  W[j * ldw + i] = w;
}

hipError_t launch_sparse_apply(const oqr_op* op, const double* Z, int64_t ldz, double* W, int64_t ldw, int64_t n,
                               hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (op->kind == OQR_OP_TRIDIAG) {
    const int64_t m = op->lda, total = m * n;
    if (m == 0) return hipSuccess;
    tridiag_apply_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>((const double*)op->a, m, Z, ldz, W, ldw, n);
    return hipGetLastError();
  }
  const int64_t sxy = (int64_t)op->nx * op->ny;
  if (sxy == 0) return hipSuccess;
  if (sxy * op->nz * 8 > 0x7fffffffll) return hipErrorInvalidValue;   // 32-bit buffer offsets per column
  stencil_march_kernel<<<dim3((unsigned)((sxy + 255) / 256), (unsigned)n), 256, 0, s>>>(
      Z, ldz, W, ldw, op->nx, op->ny, op->nz, op->center, op->off);
  return hipGetLastError();
}

}  // namespace oqr
