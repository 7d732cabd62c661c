// QR factorisation in the Euclidean inner product, Z = Y U with Y^T Y = I: the Euclidean step of
// PRE-CHOLQR (Algorithm 2), CHOL-EQR (Algorithm 3) and EQR-SYEV (Algorithm 4).
//
// For n <= 64 it is a tree of Householder QRs (TSQR).  The rows are cut into blocks of B rows
// (B = 256, 512, 1024 for n <= 64, 32, 16).  One workgroup factors one block with Householder
// reflections (LAPACK convention H = I - tau v v^T, v(j) = 1), the block held in registers: lane c of
// a wave owns column c, each thread 32 rows of it (row r * SEGS + s in register r, s the thread's row
// segment; eight waves), so that a column's reflector, dot products and updates are register
// arithmetic plus one cross-segment sum through LDS.  The n x n triangles of one level are stacked into the matrix of the
// next (floor(B / n) of them per block) until one block is left.  The explicit factor is then formed
// top-down: the top block applies its reflections to diag(sign R_ii), every lower block to its n rows
// of the parent's factor padded with zeros, the leaves write Y.  All reflections are Householder
// reflections of the Euclidean product, so the factorisation keeps the backward stability of the
// column-by-column Householder QR; the diagonal of U is made positive.  Larger n uses the column-by-
// column kernels.
#include <type_traits>

#include "common.hpp"

namespace oqr {
namespace {

constexpr int TQ_NT = 512;      // eight waves
constexpr int TQ_RPT = 32;      // rows per thread (registers)
constexpr int TQ_STAGE = 4096;  // doubles in one LDS staging tile (B rows x CH columns)

template <int NC>
struct TQ {
  static constexpr int RS = 64 / NC;                    // row segments per wave
  static constexpr int SEGS = (TQ_NT / 64) * RS;        // row segments per workgroup
  static constexpr int B = SEGS * TQ_RPT;               // rows per block
  static constexpr int CH = TQ_STAGE / B;               // columns per staging tile
  static constexpr int LDST = B + 1;                    // staging column stride (odd: no bank conflicts)
  static constexpr int RLOW = (64 + SEGS - 1) / SEGS;   // registers that can hold a row < 64
};

// f(integral_constant<int, I>) for I = B .. E - 1, expanded at compile time.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Sum of p[0], p[stride], ..., p[(N - 1) stride] (LDS) as a pairwise tree, N a power of two.
template <int N>
__device__ __forceinline__ double lds_tree_sum(const double* p, int stride) {
  if constexpr (N > 16) {
    const double lo = lds_tree_sum<N / 2>(p, stride);
    return lo + lds_tree_sum<N / 2>(p + (N / 2) * stride, stride);
  } else {
    double v[N];
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = p[k * stride];
#pragma unroll
    for (int w = 1; w < N; w <<= 1)
#pragma unroll
      for (int k = 0; k + w < N; k += 2 * w) v[k] += v[k + w];
    return v[0];
  }
}

// 1 / d from the hardware reciprocal refined by two Newton steps (a short dependent chain).
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  return fma(r, fma(-d, r, 1.0), r);
}

// Sum of eight partial sums in a fixed order.
__device__ __forceinline__ double sum8(const double (&a)[8]) {
  return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// Rows [r0, r0 + nrow) x columns [c0, c0 + CH) of M into st (zero outside the matrix).  The loads are
// unconditional (clamped address, value zeroed) and unrolled, so that all of them are in flight before
// the first wait.
// With REFL the block holds Householder vectors: the staged column col is v_col (zero above row col,
// one at row col).
template <int NC, bool REFL>
__device__ __forceinline__ void stage_in(const double* __restrict__ M, int64_t ld, int64_t r0, int nrow, int n,
                                         int c0, double* st) {
  using P = TQ<NC>;
  constexpr int PER = P::CH * P::B / TQ_NT;
  const double* Mb = M + r0;
  double v[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int idx = threadIdx.x + k * TQ_NT;
    const int cc = idx / P::B, row = idx % P::B, col = c0 + cc;
    v[k] = sel_load(Mb, (int64_t)col * ld + row, row < nrow && col < n);
    if (REFL) v[k] = (row > col) ? v[k] : ((row == col) ? 1.0 : 0.0);
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int idx = threadIdx.x + k * TQ_NT;
    st[(idx / P::B) * P::LDST + idx % P::B] = v[k];
  }
}

// Factor every block of M (rows x n, ld): reflectors overwrite M, tau[blk * n + j], and the block's
// upper triangle U_blk (n x n, zero below the diagonal) goes to rows [blk n, blk n + n) of Rn (ldr).
template <int NC>
__global__ __launch_bounds__(TQ_NT, 4) void tsqr_factor_kernel(double* __restrict__ M, int64_t ld, int64_t rows,
                                                               int n, int br, double* __restrict__ tau,
                                                               double* __restrict__ Rn, int64_t ldr) {
  using P = TQ<NC>;
  constexpr int SEGS = P::SEGS, CH = P::CH, LDST = P::LDST, RLOW = P::RLOW;
  __shared__ double st[CH * LDST];
  __shared__ __attribute__((aligned(16))) double vb[2][P::B];   // column j below the diagonal, per segment
  __shared__ double red[SEGS];
  __shared__ double xjj;
  __shared__ double wred[SEGS][NC];
  const int tid = threadIdx.x, l = tid & 63, c = l % NC;
  const int s = (tid >> 6) * P::RS + l / NC;
  const int blk = blockIdx.x;
  const int64_t r0 = (int64_t)blk * br;
  const int nrow = (int)min((int64_t)br, rows - r0);

  double L[TQ_RPT];
#pragma unroll
  for (int r = 0; r < TQ_RPT; ++r) L[r] = 0.0;
  for (int c0 = 0; c0 < n; c0 += CH) {
    stage_in<NC, false>(M, ld, r0, nrow, n, c0, st);
    __syncthreads();
    if (c >= c0 && c < c0 + CH) {
#pragma unroll
      for (int r = 0; r < TQ_RPT; ++r) L[r] = st[(c - c0) * LDST + r * SEGS + s];
    }
    __syncthreads();
  }

  // Column j = rj * SEGS + sj: its diagonal row lives in register rj of segment sj.  The loop over rj
  // is expanded at compile time so that rj indexes the register array directly.
  static_for<0, RLOW>([&](auto rjc) {
    constexpr int rj = decltype(rjc)::value;
    for (int sj = 0; sj < SEGS; ++sj) {
      const int j = rj * SEGS + sj;
      if (j >= n) return;
      const int pb = j & 1;
      double* vs = &vb[pb][s * TQ_RPT];   // this thread's rows of the column, in register order
      // the owner of column j: its squared norm below the diagonal (per segment) and the column
      if (c == j) {
        double pa[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int r = 0; r < TQ_RPT; r += 2) {
          double x[2] = {L[r], L[r + 1]};
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            if (r + h < rj) {
              x[h] = 0.0;
            } else if (r + h == rj) {
              if (s == sj) xjj = x[h];
              x[h] = (s > sj) ? x[h] : 0.0;
            }
            pa[(r + h) & 7] = fma(x[h], x[h], pa[(r + h) & 7]);
          }
          *(double2*)(vs + r) = make_double2(x[0], x[1]);
        }
        red[s] = sum8(pa);
      }
      __syncthreads();
      const double sig = lds_tree_sum<SEGS>(red, 1);
      const double x0 = xjj;
      double beta = x0, tq = 0.0, scale = 0.0;   // sig == 0: H = I
      if (sig != 0.0) {
        const double nrm = sqrt(fma(x0, x0, sig));
        beta = (x0 >= 0.0) ? -nrm : nrm;
        scale = recip(x0 - beta);
        tq = (beta - x0) * recip(beta);
      }
      const bool upd = c > j && c < n;
      // v = e_j + scale * x: partial v^T a_c over this thread's rows
      if (upd) {
        double pa[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int r = 0; r < TQ_RPT; r += 2) {
          const double2 v2 = *(const double2*)(vs + r);
          pa[r & 7] = fma(v2.x, L[r], pa[r & 7]);
          pa[(r + 1) & 7] = fma(v2.y, L[r + 1], pa[(r + 1) & 7]);
          if (r % 16 == 14) __builtin_amdgcn_sched_barrier(0);   // bounds the LDS reads in flight
        }
        wred[s][c] = fma(scale, sum8(pa), (s == sj) ? L[rj] : 0.0);
      }
      __syncthreads();
      if (upd) {
        const double wsum = lds_tree_sum<SEGS>(&wred[0][c], NC);
        const double tw = tq * wsum, tws = tw * scale;
#pragma unroll
        for (int r = 0; r < TQ_RPT; r += 2) {
          const double2 v2 = *(const double2*)(vs + r);
          L[r] = fma(-tws, v2.x, L[r]);
          L[r + 1] = fma(-tws, v2.y, L[r + 1]);
          if (r % 16 == 14) __builtin_amdgcn_sched_barrier(0);
        }
        if (s == sj) L[rj] -= tw;
      } else if (c == j) {
#pragma unroll
        for (int r = 0; r < TQ_RPT; ++r) {
          if (r > rj)
            L[r] *= scale;
          else if (r == rj)
            L[r] = (s > sj) ? L[r] * scale : ((s == sj) ? beta : L[r]);
        }
        if (s == 0) tau[(int64_t)blk * n + j] = tq;
      }
    }
  });

  for (int c0 = 0; c0 < n; c0 += CH) {
    if (c >= c0 && c < c0 + CH) {
#pragma unroll
      for (int r = 0; r < TQ_RPT; ++r) st[(c - c0) * LDST + r * SEGS + s] = L[r];
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
  __shared__ double taus[64];
  const int tid = threadIdx.x, l = tid & 63, c = l % NC;
  const int s = (tid >> 6) * P::RS + l / NC;
  const int blk = blockIdx.x;
  const int64_t r0 = (int64_t)blk * br;
  const int nrow = (int)min((int64_t)br, rows - r0);
  if (tid < n) taus[tid] = tau[(int64_t)blk * n + tid];

  double Y[TQ_RPT];
#pragma unroll
  for (int r = 0; r < TQ_RPT; ++r) Y[r] = 0.0;
  if (c < n) {
#pragma unroll
    for (int r = 0; r < RLOW; ++r) {
      const int row = r * SEGS + s;
      if (Rtop) {
        const double d = sel_load(Rtop, (int64_t)row * n + row, row < n);
        Y[r] = (row == c) ? ((d < 0.0) ? -1.0 : 1.0) : 0.0;
      } else {
        Y[r] = sel_load(Cin, (int64_t)c * ldc + (int64_t)blk * n + row, row < n);
      }
    }
  }

  double vr[TQ_RPT];   // v_j on this thread's rows
  int ph = 0;
  for (int c0 = ((n - 1) / CH) * CH; c0 >= 0; c0 -= CH) {
    __syncthreads();
    stage_in<NC, true>(M, ld, r0, nrow, n, c0, st);
    __syncthreads();
    for (int j = min(n, c0 + CH) - 1; j >= c0; --j) {
      const double tq = taus[j];
      if (tq == 0.0) continue;   // H_j = I (the same value in every thread)
      const double* vc = st + (j - c0) * LDST;
      if (c < n) {
        double pa[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int r = 0; r < TQ_RPT; ++r) {
          vr[r] = vc[r * SEGS + s];
          pa[r & 7] = fma(vr[r], Y[r], pa[r & 7]);
        }
        wred[ph][s][c] = sum8(pa);
      }
      __syncthreads();
      if (c < n) {
        const double wsum = lds_tree_sum<SEGS>(&wred[ph][0][c], NC);
        const double tw = tq * wsum;
#pragma unroll
        for (int r = 0; r < TQ_RPT; ++r) Y[r] = fma(-tw, vr[r], Y[r]);
      }
      ph ^= 1;
    }
  }

  for (int c0 = 0; c0 < n; c0 += CH) {
    __syncthreads();
    if (c >= c0 && c < c0 + CH) {
#pragma unroll
      for (int r = 0; r < TQ_RPT; ++r) st[(c - c0) * LDST + r * SEGS + s] = Y[r];
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
