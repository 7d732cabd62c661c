// Triangular solve Q = Z R^{-1} (step 4 of CHOLQR, Algorithm 1), FP64.
//
// Each row of Q solves q_i R = z_i, the row-wise solve whose backward error
// |dR^i| <= c n u |R| gives the residual bound of Theorem 2.1.  Column blocks
// of 32 are processed left to right:
//   (1) Z_J -= Q_{<J} R_{<J,J}    FP64 MFMA (a blocked form of the same sums)
//   (2) Q_J  = Z_J R_JJ^{-1}       substitution, k ascending, 4 lanes per row
// A workgroup owns 64 rows x all n columns, staged once in LDS (Z is read
// from HBM once and Q written once).  Q may alias Z: the whole row block of Z
// is in LDS before any of its Q columns is written.
#include "common.hpp"

namespace oqr {
namespace {

constexpr int BM = 64;
constexpr int JB = 32;
constexpr int NT = 256;
constexpr int LDQ = BM + 1;   // LDS column stride (doubles)

template <int NMAX>
__global__ __launch_bounds__(NT) void trsm_kernel(const double* Z, int64_t ldz, const double* __restrict__ R,
                                                  int64_t ldr, double* Q, int64_t ldq, int m, int n,
                                                  const int32_t* __restrict__ info) {
  __shared__ double Qs[NMAX * LDQ];          // Qs[j * LDQ + i]: row i of the block, column j
  __shared__ double RJ[JB][JB + 1];          // diagonal block of R
  if (info[0] != 0) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int i0 = blockIdx.x * BM;
  const int nblk = (n + JB - 1) / JB;

  // load the Z row block (column-major: 64 contiguous rows per column), 16 loads in flight per thread
  {
    const int i = t % BM, jq = t / BM;
    const bool ok = i0 + i < m;
    constexpr int STRIDE = NT / BM;
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
  const int row = t >> 2, sub = t & 3;      // substitution: 4 lanes per row
  for (int J = 0; J < nblk; ++J) {
    const int j0 = J * JB;
    // stage R_JJ (upper 32x32; identity beyond n)
    for (int idx = t; idx < JB * JB; idx += NT) {
      const int p = idx % JB, c = idx / JB;
      const int gp = j0 + p, gc = j0 + c;
      double v;
      if (gp < n && gc < n) v = (p <= c) ? R[(int64_t)gc * ldr + gp] : 0.0;
      else v = (p == c) ? 1.0 : 0.0;
      RJ[p][c] = v;
    }
    __syncthreads();
    // (1) block update on MFMA: wave w owns rows 16w..16w+15, two 16-column halves
    if (J > 0) {
      f64x4 acc[2];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[h][r] = Qs[(j0 + 16 * h + (lane & 15)) * LDQ + wave * 16 + 4 * r + (lane >> 4)];
      const int jc0 = j0 + (lane & 15), jc1 = j0 + 16 + (lane & 15);
      const double* R0 = R + (int64_t)min(jc0, n - 1) * ldr + (lane >> 4);
      const double* R1 = R + (int64_t)min(jc1, n - 1) * ldr + (lane >> 4);
      const bool ok0 = jc0 < n, ok1 = jc1 < n;
      // R fragments are read from L2 in chunks of 32 k (8 MFMA steps), one chunk ahead
      double b0[8], b1[8];
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        b0[s] = sel_load(R0, 4 * s, ok0);
        b1[s] = sel_load(R1, 4 * s, ok1);
      }
      for (int kc = 0; kc < j0; kc += 32) {
        double nb0[8], nb1[8];
        const bool more = kc + 32 < j0;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          nb0[s] = sel_load(R0, kc + 32 + 4 * s, more && ok0);
          nb1[s] = sel_load(R1, kc + 32 + 4 * s, more && ok1);
        }
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int kr = kc + 4 * s + (lane >> 4);
          const double a = -Qs[kr * LDQ + wave * 16 + (lane & 15)];
          acc[0] = mfma_f64(a, b0[s], acc[0]);
          acc[1] = mfma_f64(a, b1[s], acc[1]);
        }
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          b0[s] = nb0[s];
          b1[s] = nb1[s];
        }
      }
      __syncthreads();
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) Qs[(j0 + 16 * h + (lane & 15)) * LDQ + wave * 16 + 4 * r + (lane >> 4)] = acc[h][r];
      __syncthreads();
    }
    // (2) substitution on the 32 columns of the block: lane `sub` of a row owns columns sub + 4e
    {
      double x[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = Qs[(j0 + sub + 4 * e) * LDQ + row];
#pragma unroll
      for (int c = 0; c < JB; ++c) {
        const int owner = c & 3, ec = c >> 2;
        // branch-free: every lane divides, the owner's quotient is broadcast
        const double qo = x[ec] / RJ[c][c];
        const double q = __shfl(qo, (lane & ~3) | owner);
        if (sub == owner) x[ec] = q;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const double upd = x[e] - q * RJ[c][sub + 4 * e];
          x[e] = (sub + 4 * e > c) ? upd : x[e];
        }
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int j = j0 + sub + 4 * e;
        Qs[j * LDQ + row] = x[e];
        if (i0 + row < m && j < n) Q[(int64_t)j * ldq + i0 + row] = x[e];
      }
    }
    __syncthreads();
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
  const int grid = ceil_div(m, BM);
  if (n <= 64)
    trsm_kernel<64><<<grid, NT, 0, s>>>(Z, ldz, R, ldr, Q, ldq, (int)m, (int)n, info);
  else if (n <= 128)
    trsm_kernel<128><<<grid, NT, 0, s>>>(Z, ldz, R, ldr, Q, ldq, (int)m, (int)n, info);
  else
    trsm_kernel<256><<<grid, NT, 0, s>>>(Z, ldz, R, ldr, Q, ldq, (int)m, (int)n, info);
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
