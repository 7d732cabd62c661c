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
// A workgroup owns BMR rows x all n columns, staged once in LDS (Z is read
// from HBM once and Q written once, column-coalesced, at the end); BMR = 64
// for n <= 128 and 32 above, so that two workgroups fit in one CU's LDS.  Q may
// alias Z: the whole row block of Z is in LDS before any of its Q is written.
#include "common.hpp"

namespace oqr {
namespace {

constexpr int JB = 32;
constexpr int NT = 256;

// Broadcast lane O of every group of four lanes to the whole group (DPP quad_perm).
template <int O>
__device__ __forceinline__ double quad_bcast(double v) {
  constexpr int ctrl = O | (O << 2) | (O << 4) | (O << 6);
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), ctrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), ctrl, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double quad_bcast(double v, int o) {
  switch (o) {
    case 0: return quad_bcast<0>(v);
    case 1: return quad_bcast<1>(v);
    case 2: return quad_bcast<2>(v);
    default: return quad_bcast<3>(v);
  }
}

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
      const double* Rc[NH];
      bool okc[NH];
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const int jc = j0 + 16 * (h0 + h) + lj;
        okc[h] = jc < n;
        Rc[h] = R + (int64_t)min(jc, n - 1) * ldr + li;
      }
      // R fragments are read from L2 in chunks of 32 k (8 MFMA steps), one chunk ahead
      double bf[NH][8];
#pragma unroll
      for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int s = 0; s < 8; ++s) bf[h][s] = sel_load(Rc[h], 4 * s, okc[h]);
      for (int kc = 0; kc < j0; kc += 32) {
        double nb[NH][8];
        const bool more = kc + 32 < j0;
#pragma unroll
        for (int h = 0; h < NH; ++h)
#pragma unroll
          for (int s = 0; s < 8; ++s) nb[h][s] = sel_load(Rc[h], kc + 32 + 4 * s, more && okc[h]);
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
#pragma unroll
      for (int c = 0; c < JB; ++c) {
        const int owner = c & 3, ec = c >> 2;
        const double q = quad_bcast(x[ec] * rinv[c], owner);
        const double* rz = &RZ[c][sub * 8];
        // columns sub + 4e <= c are final: e below (c - 3) / 4 is skipped for every lane
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (4 * e + 3 > c) x[e] = __builtin_fma(-q, rz[e], x[e]);
        x[ec] = (sub == owner) ? q : x[ec];
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) Qs[(j0 + sub + 4 * e) * LDQ + row] = x[e];
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
  if (n <= 64)
    trsm_kernel<64, 64><<<ceil_div(m, 64), NT, 0, s>>>(Z, ldz, R, ldr, Q, ldq, (int)m, (int)n, info);
  else if (n <= 128)
    trsm_kernel<128, 64><<<ceil_div(m, 64), NT, 0, s>>>(Z, ldz, R, ldr, Q, ldq, (int)m, (int)n, info);
  else
    trsm_kernel<256, 32><<<ceil_div(m, 32), NT, 0, s>>>(Z, ldz, R, ldr, Q, ldq, (int)m, (int)n, info);
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
