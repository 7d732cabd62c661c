// QR factorisation in the Euclidean inner product, Z = Y U with Y^T Y = I: the Euclidean step of
// PRE-CHOLQR (Algorithm 2), CHOL-EQR (Algorithm 3) and EQR-SYEV (Algorithm 4).
//
// For n <= 64 it is a tree of Householder QRs (TSQR).  The rows are cut into blocks of B rows
// (B = 256, 512, 1024 for n <= 64, 32, 16).  One workgroup factors one block with Householder
// reflections (LAPACK convention H = I - tau v v^T, v(j) = 1), the block held in registers: lane c of
// a wave owns column c, each thread 64 rows of it (row r * SEGS + s in register r, s the thread's row
// segment), so that a column's reflector, dot products and updates are register arithmetic plus one
// cross-segment sum through LDS.  The n x n triangles of one level are stacked into the matrix of the
// next (floor(B / n) of them per block) until one block is left.  The explicit factor is then formed
// top-down: the top block applies its reflections to diag(sign R_ii), every lower block to its n rows
// of the parent's factor padded with zeros, the leaves write Y.  All reflections are Householder
// reflections of the Euclidean product, so the factorisation keeps the backward stability of the
// column-by-column Householder QR; the diagonal of U is made positive.  Larger n uses the column-by-
// column kernels.
#include "common.hpp"

namespace oqr {
namespace {

constexpr int TQ_NT = 256;      // four waves
constexpr int TQ_STAGE = 4096;  // doubles in one LDS staging tile (B rows x CH columns)

template <int NC>
struct TQ {
  static constexpr int RS = 64 / NC;                    // row segments per wave
  static constexpr int SEGS = 4 * RS;                   // row segments per workgroup
  static constexpr int B = SEGS * 64;                   // rows per block
  static constexpr int CH = TQ_STAGE / B;               // columns per staging tile
  static constexpr int LDST = B + 1;                    // staging column stride (odd: no bank conflicts)
  static constexpr int RLOW = (64 + SEGS - 1) / SEGS;   // registers that can hold a row < 64
};

// Rows [r0, r0 + nrow) x columns [c0, c0 + CH) of M into st (zero outside the matrix).
template <int NC>
__device__ __forceinline__ void stage_in(const double* __restrict__ M, int64_t ld, int64_t r0, int nrow, int n,
                                         int c0, double* st) {
  using P = TQ<NC>;
  for (int idx = threadIdx.x; idx < P::CH * P::B; idx += TQ_NT) {
    const int cc = idx / P::B, row = idx % P::B, col = c0 + cc;
    double v = 0.0;
    if (row < nrow && col < n) v = M[(int64_t)col * ld + r0 + row];
    st[cc * P::LDST + row] = v;
  }
}

// Factor every block of M (rows x n, ld): reflectors overwrite M, tau[blk * n + j], and the block's
// upper triangle U_blk (n x n, zero below the diagonal) goes to rows [blk n, blk n + n) of Rn (ldr).
template <int NC>
__global__ __launch_bounds__(TQ_NT) void tsqr_factor_kernel(double* __restrict__ M, int64_t ld, int64_t rows,
                                                               int n, int br, double* __restrict__ tau,
                                                               double* __restrict__ Rn, int64_t ldr) {
  using P = TQ<NC>;
  constexpr int SEGS = P::SEGS, CH = P::CH, LDST = P::LDST, RLOW = P::RLOW;
  __shared__ double st[CH * LDST];
  __shared__ double vb[2][P::B];     // the current column below the diagonal (x), double-buffered
  __shared__ double red[SEGS];
  __shared__ double xjj;
  __shared__ double wred[SEGS][NC];
  const int tid = threadIdx.x, l = tid & 63, c = l % NC;
  const int s = (tid >> 6) * P::RS + l / NC;
  const int blk = blockIdx.x;
  const int64_t r0 = (int64_t)blk * br;
  const int nrow = (int)min((int64_t)br, rows - r0);

  double L[64];
#pragma unroll
  for (int r = 0; r < 64; ++r) L[r] = 0.0;
  for (int c0 = 0; c0 < n; c0 += CH) {
    stage_in<NC>(M, ld, r0, nrow, n, c0, st);
    __syncthreads();
    if (c >= c0 && c < c0 + CH) {
#pragma unroll
      for (int r = 0; r < 64; ++r) L[r] = st[(c - c0) * LDST + r * SEGS + s];
    }
    __syncthreads();
  }

  for (int j = 0; j < n; ++j) {
    const int pb = j & 1;
    // the owner of column j: its squared norm below the diagonal (per segment) and the column itself
    if (c == j) {
      double part = 0.0;
#pragma unroll
      for (int r = 0; r < 64; ++r) {
        const int row = r * SEGS + s;
        double x = L[r];
        if (r < RLOW) {
          if (row == j) xjj = x;
          x = (row > j) ? x : 0.0;
        }
        part = fma(x, x, part);
        vb[pb][row] = x;
      }
      red[s] = part;
    }
    __syncthreads();
    double sig = 0.0;
#pragma unroll
    for (int k = 0; k < SEGS; ++k) sig += red[k];
    const double x0 = xjj;
    double beta = x0, tq = 0.0, scale = 0.0;   // sig == 0: H = I
    if (sig != 0.0) {
      const double nrm = sqrt(fma(x0, x0, sig));
      beta = (x0 >= 0.0) ? -nrm : nrm;
      scale = 1.0 / (x0 - beta);
      tq = (beta - x0) / beta;
    }
    const bool upd = c > j && c < n;
    const int sj = j % SEGS, rj = j / SEGS;
    // v = e_j + scale * x: partial v^T a_c over this thread's rows
    if (upd) {
      double acc = 0.0, aj = 0.0;
#pragma unroll
      for (int r = 0; r < 64; ++r) {
        acc = fma(vb[pb][r * SEGS + s], L[r], acc);
        if (r % 16 == 15) __builtin_amdgcn_sched_barrier(0);   // bounds the LDS reads in flight
      }
      if (s == sj) {
#pragma unroll
        for (int r = 0; r < RLOW; ++r) aj = (r == rj) ? L[r] : aj;
      }
      wred[s][c] = fma(scale, acc, aj);
    }
    __syncthreads();
    if (upd) {
      double wsum = 0.0;
#pragma unroll
      for (int k = 0; k < SEGS; ++k) wsum += wred[k][c];
      const double tw = tq * wsum, tws = tw * scale;
#pragma unroll
      for (int r = 0; r < 64; ++r) {
        L[r] = fma(-tws, vb[pb][r * SEGS + s], L[r]);
        if (r % 16 == 15) __builtin_amdgcn_sched_barrier(0);
      }
      if (s == sj) {
#pragma unroll
        for (int r = 0; r < RLOW; ++r) L[r] = (r == rj) ? L[r] - tw : L[r];
      }
    } else if (c == j) {
#pragma unroll
      for (int r = 0; r < 64; ++r) {
        const int row = r * SEGS + s;
        if (r < RLOW)
          L[r] = (row > j) ? L[r] * scale : ((row == j) ? beta : L[r]);
        else
          L[r] *= scale;
      }
      if (s == 0) tau[(int64_t)blk * n + j] = tq;
    }
  }

  for (int c0 = 0; c0 < n; c0 += CH) {
    if (c >= c0 && c < c0 + CH) {
#pragma unroll
      for (int r = 0; r < 64; ++r) st[(c - c0) * LDST + r * SEGS + s] = L[r];
    }
    __syncthreads();
    for (int idx = tid; idx < CH * P::B; idx += TQ_NT) {
      const int cc = idx / P::B, row = idx % P::B, col = c0 + cc;
      if (col >= n) continue;
      const double v = st[cc * LDST + row];
      if (row < nrow) M[(int64_t)col * ld + r0 + row] = v;
      if (row < n) Rn[(int64_t)col * ldr + (int64_t)blk * n + row] = (row <= col) ? v : 0.0;
    }
    __syncthreads();
  }
}

// Form the explicit factor of every block of a level: Out_blk = H_blk [C_blk; 0], C_blk = rows
// [blk n, blk n + n) of Cin (ldc), or diag(sign Rtop_ii) for the top block (Rtop != null).
template <int NC>
__global__ __launch_bounds__(TQ_NT, 2) void tsqr_form_kernel(const double* __restrict__ M, int64_t ld, int64_t rows,
                                                             int n, int br, const double* __restrict__ tau,
                                                             const double* __restrict__ Cin, int64_t ldc,
                                                             const double* __restrict__ Rtop,
                                                             double* __restrict__ Out, int64_t ldo) {
  using P = TQ<NC>;
  constexpr int SEGS = P::SEGS, CH = P::CH, LDST = P::LDST, RLOW = P::RLOW;
  __shared__ double st[CH * LDST];
  __shared__ double wred[2][SEGS][NC];
  const int tid = threadIdx.x, l = tid & 63, c = l % NC;
  const int s = (tid >> 6) * P::RS + l / NC;
  const int blk = blockIdx.x;
  const int64_t r0 = (int64_t)blk * br;
  const int nrow = (int)min((int64_t)br, rows - r0);

  double Y[64];
#pragma unroll
  for (int r = 0; r < 64; ++r) Y[r] = 0.0;
  if (c < n) {
#pragma unroll
    for (int r = 0; r < RLOW; ++r) {
      const int row = r * SEGS + s;
      if (row < n) {
        if (Rtop)
          Y[r] = (row == c) ? ((Rtop[(int64_t)row * n + row] < 0.0) ? -1.0 : 1.0) : 0.0;
        else
          Y[r] = Cin[(int64_t)c * ldc + (int64_t)blk * n + row];
      }
    }
  }

  int ph = 0;
  for (int c0 = ((n - 1) / CH) * CH; c0 >= 0; c0 -= CH) {
    __syncthreads();
    stage_in<NC>(M, ld, r0, nrow, n, c0, st);
    __syncthreads();
    for (int j = min(n, c0 + CH) - 1; j >= c0; --j) {
      const double tq = tau[(int64_t)blk * n + j];
      if (tq == 0.0) continue;   // H_j = I (the same value in every thread)
      const double* vc = st + (j - c0) * LDST;
      if (c < n) {
        double p = 0.0;
#pragma unroll
        for (int r = 0; r < 64; ++r) {
          const int row = r * SEGS + s;
          double v = vc[row];
          if (r < RLOW) v = (row > j) ? v : ((row == j) ? 1.0 : 0.0);
          p = fma(v, Y[r], p);
        }
        wred[ph][s][c] = p;
      }
      __syncthreads();
      if (c < n) {
        double wsum = 0.0;
#pragma unroll
        for (int k = 0; k < SEGS; ++k) wsum += wred[ph][k][c];
        const double tw = tq * wsum;
#pragma unroll
        for (int r = 0; r < 64; ++r) {
          const int row = r * SEGS + s;
          double v = vc[row];
          if (r < RLOW) v = (row > j) ? v : ((row == j) ? 1.0 : 0.0);
          Y[r] = fma(-tw, v, Y[r]);
        }
      }
      ph ^= 1;
    }
  }

  for (int c0 = 0; c0 < n; c0 += CH) {
    __syncthreads();
    if (c >= c0 && c < c0 + CH) {
#pragma unroll
      for (int r = 0; r < 64; ++r) st[(c - c0) * LDST + r * SEGS + s] = Y[r];
    }
    __syncthreads();
    for (int idx = tid; idx < CH * P::B; idx += TQ_NT) {
      const int cc = idx / P::B, row = idx % P::B, col = c0 + cc;
      if (col < n && row < nrow) Out[(int64_t)col * ldo + r0 + row] = st[cc * LDST + row];
    }
  }
}

// U = diag(sign Rtop_ii) Rtop, upper triangle.
__global__ void tsqr_sign_r_kernel(const double* __restrict__ Rtop, int n, double* __restrict__ U, int64_t ldu) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int col = idx / n, i = idx % n;
  const double sg = (Rtop[(int64_t)i * n + i] < 0.0) ? -1.0 : 1.0;
  U[(int64_t)col * ldu + i] = (i <= col) ? sg * Rtop[(int64_t)col * n + i] : 0.0;
}

constexpr int TSQR_MAX_N = 64;
constexpr int TSQR_MAX_LEVELS = 32;

int tsqr_nc(int64_t n) { return n <= 16 ? 16 : (n <= 32 ? 32 : 64); }

struct Level {
  int64_t rows;
  int br, blocks;
};

// The levels of the tree for m x n; returns their count.
int tsqr_levels(int64_t m, int64_t n, Level* lv) {
  const int B = 256 * 64 / tsqr_nc(n);
  int k = 0;
  lv[0] = {m, B, ceil_div(m, B)};
  while (lv[k].blocks > 1 && k + 1 < TSQR_MAX_LEVELS) {
    const int64_t rows = (int64_t)lv[k].blocks * n;
    const int br = (int)((B / n) * n);
    lv[k + 1] = {rows, br, ceil_div(rows, br)};
    ++k;
  }
  return k + 1;
}

struct TsqrWs {
  double* tau[TSQR_MAX_LEVELS];
  double* S[TSQR_MAX_LEVELS];   // level matrices above the leaves (S[0] unused)
  double* P[TSQR_MAX_LEVELS];   // their explicit factors
  double* Rtop;
};

size_t tsqr_ws(int64_t m, int64_t n, const Level* lv, int nl, TsqrWs* w, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return (double*)p;
  };
  for (int k = 0; k < nl; ++k) {
    double* t = take((size_t)lv[k].blocks * n * sizeof(double));
    double* S = k ? take((size_t)lv[k].rows * n * sizeof(double)) : nullptr;
    double* P = k ? take((size_t)lv[k].rows * n * sizeof(double)) : nullptr;
    if (w) {
      w->tau[k] = t;
      w->S[k] = S;
      w->P[k] = P;
    }
  }
  double* rt = take((size_t)n * n * sizeof(double));
  if (w) w->Rtop = rt;
  return off;
}

template <int NC>
hipError_t tsqr_run(double* W, int64_t ldw, int64_t m, int64_t n, const Level* lv, int nl, const TsqrWs& w,
                    double* U, int64_t ldu, double* Y, int64_t ldy, hipStream_t s) {
  for (int k = 0; k < nl; ++k) {
    double* Mk = k ? w.S[k] : W;
    const int64_t ldm = k ? lv[k].rows : ldw;
    double* Rn = (k + 1 < nl) ? w.S[k + 1] : w.Rtop;
    const int64_t ldr = (k + 1 < nl) ? lv[k + 1].rows : n;
    tsqr_factor_kernel<NC><<<lv[k].blocks, TQ_NT, 0, s>>>(Mk, ldm, lv[k].rows, (int)n, lv[k].br, w.tau[k], Rn, ldr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  for (int k = nl - 1; k >= 0; --k) {
    const double* Mk = k ? w.S[k] : W;
    const int64_t ldm = k ? lv[k].rows : ldw;
    const bool top = (k == nl - 1);
    const double* Cin = top ? nullptr : w.P[k + 1];
    const int64_t ldc = top ? 0 : lv[k + 1].rows;
    double* Out = k ? w.P[k] : Y;
    const int64_t ldo = k ? lv[k].rows : ldy;
    tsqr_form_kernel<NC><<<lv[k].blocks, TQ_NT, 0, s>>>(Mk, ldm, lv[k].rows, (int)n, lv[k].br, w.tau[k], Cin, ldc,
                                                        top ? w.Rtop : nullptr, Out, ldo);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  tsqr_sign_r_kernel<<<ceil_div(n * n, 256), 256, 0, s>>>(w.Rtop, (int)n, U, ldu);
  return hipGetLastError();
}

}  // namespace

size_t euclid_qr_ws_bytes(int64_t m, int64_t n) {
  if (n <= 0) return 0;
  if (n > TSQR_MAX_N) return align256((size_t)(n + 8) * sizeof(double));
  Level lv[TSQR_MAX_LEVELS];
  const int nl = tsqr_levels(m, n, lv);
  return tsqr_ws(m, n, lv, nl, nullptr, nullptr);
}

hipError_t launch_euclid_qr(double* W, int64_t ldw, int64_t m, int64_t n, void* ws, double* U, int64_t ldu, double* Y,
                            int64_t ldy, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n > TSQR_MAX_N) return launch_householder_qr(W, ldw, m, n, (double*)ws, U, ldu, Y, ldy, s);
  Level lv[TSQR_MAX_LEVELS];
  const int nl = tsqr_levels(m, n, lv);
  if (lv[nl - 1].blocks != 1) return hipErrorInvalidValue;
  TsqrWs w;
  tsqr_ws(m, n, lv, nl, &w, (char*)ws);
  switch (tsqr_nc(n)) {
    case 16: return tsqr_run<16>(W, ldw, m, n, lv, nl, w, U, ldu, Y, ldy, s);
    case 32: return tsqr_run<32>(W, ldw, m, n, lv, nl, w, U, ldu, Y, ldy, s);
    default: return tsqr_run<64>(W, ldw, m, n, lv, nl, w, U, ldu, Y, ldy, s);
  }
}

}  // namespace oqr
