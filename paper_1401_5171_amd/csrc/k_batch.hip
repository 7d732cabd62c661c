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
constexpr int BR = 128;       // largest row block (rows of A per block of W)
constexpr int BK = 32;        // largest K step of the A X product
constexpr int LD = NB + 1;

// Tile shapes of the Gram phase, chosen per instance from the tuning table: rows per row block and
// K step.  Shape id s: BR_OF[s] x BK_OF[s].
constexpr int NSHAPES = OQR_BATCH_SHAPES;
constexpr int BR_OF[NSHAPES] = {128, 64, 128, 64};
constexpr int BK_OF[NSHAPES] = {32, 32, 16, 16};

constexpr double U64 = 1.1102230246251565e-16;

// Values the whole workgroup shares, moved to scalar registers (a non-inlined callee receives them in
// vector registers; buffer resources must be scalar).
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffff));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return ((int64_t)hi << 32) | (uint32_t)lo;
}
template <class P>
__device__ __forceinline__ P* uni(P* p) { return (P*)(uintptr_t)uni((int64_t)(uintptr_t)p); }

// Bounds-checked buffer load of element e, or 0 where `ok` is false: the byte offset is OR-ed with
// kOOB, which lies beyond every operand's range (items are limited to 2^31 - 1 bytes), so the
// hardware returns zero.  Branch-free on purpose: a select between the load and its use, or a load
// under a branch, makes the compiler wait for the load at once and serialises a prefetch.  The raw
// value is returned so that nothing consumes it before it is needed.
template <class T> struct Raw;
template <> struct Raw<double> {
  typedef double type;
  static __device__ __forceinline__ double load(bufrsrc r, int64_t e, bool ok) {
    return buf_f64(r, ((uint32_t)e * 8u) | (ok ? 0u : kOOB));
  }
};
template <> struct Raw<float> {
  typedef float type;
  static __device__ __forceinline__ float load(bufrsrc r, int64_t e, bool ok) {
    return __builtin_bit_cast(float,
                              __builtin_amdgcn_raw_buffer_load_b32(r, (int)(((uint32_t)e * 4u) | (ok ? 0u : kOOB)), 0, 0));
  }
};

struct Tiles {
  double As[BK * (BR + 1)];   // A tile of the current shape: As[k (BR_ + 1) + i] (odd stride: conflict-free
                              // MFMA operand reads)
  double Xs[BK][LD];          // X tile: Xs[k][j]
};
struct Fact {
  double Gs[NB][LD];          // Gram, then the factor R (upper)
  double Ws[NB][LD];          // R1 at the end of pass 2
};
struct Smem {
  union {
    Tiles tl;                 // streaming phase of G = X^T A X
    double xb[64][LD];        // half of X_b (64 rows) for the products X_b^T W_b
    double red[3][4][4][64];  // partial G of waves in row groups > 0
    Fact f;                   // Cholesky, substitution, R = R2 R1
  };
  double diag[NB];
  int idx;
  int fail;
  double dmax;
};

// G = X^T A X for one instance, A symmetric: row block b (BR rows) streams only its diagonal block and
// the blocks right of it, W_b = A_b,diag X_b + A_b,right X (MFMA, W_b in registers), and
// G = D + H + H^T with D += X_b^T (A_b,diag X_b) and H += X_b^T (A_b,right X), so A is read about half;
// W_b's accumulators serve directly as the B operand of X_b^T W_b (the FP64 MFMA's D layout is its
// B layout, one K step per accumulator element).
// Wave w owns the 16 columns cb = w % CLS of W and G and the row group rg = w / CLS of each row block
// (RG = 4 / CLS groups of 16 * RBW rows).  On return, waves of row group 0 hold G(:, 16 cb ..) in g.
// SITE (0 persistent kernel, 1 split kernels) gives each calling kernel its own copy of these out-of-line
// functions: a copy shared with the split kernels gets a register allocation that spills several hundred
// bytes per lane in the wide shapes and runs the persistent launch 1.6x slower.
template <class T, int CLS, int BR_, int BK_, int SITE>
__device__ __noinline__ void gram_phase(const T* A_, int64_t lda_, const T* X_, int64_t ldx_, int m_, int n_,
                                        int rb_first_, int rb_step_, Smem& S, f64x4 (&g_out)[4]) {
  const T* A = uni(A_);
  const T* X = uni(X_);
  const int64_t lda = uni(lda_), ldx = uni(ldx_);
  const int m = uni(m_), n = uni(n_);
  const int rb_first = uni(rb_first_), rb_step = uni(rb_step_);   // row blocks rb_first, + rb_step, ...
  static_assert(BR_ % 64 == 0 && BR_ <= BR && BK_ <= BK && BK_ % 4 == 0, "tile shape");
  constexpr int RG = 4 / CLS, RBW = BR_ / 16 / RG;
  constexpr int ASTR = BR_ + 1;                // LDS stride of the A tile
  constexpr int KSTR = NT / BR_;               // K rows loaded per pass of the workgroup
  constexpr int XSTR = NT / BK_;               // X columns loaded per pass
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int li = lane >> 4, lj = lane & 15;
  const int cb = wave % CLS, rg = wave / CLS;
  const int nbk = (n + 15) / 16;
  const bool active = cb < nbk;               // wave-uniform
  f64x4 g[4], h[4];                            // D, H (the blocks right of the diagonal); local, so
                                               // that they stay in registers
#pragma unroll
  for (int b = 0; b < 4; ++b) g[b] = h[b] = f64x4{0, 0, 0, 0};
  // tile loads: A BR_ BK_ / NT values per thread (row t % BR_, k = t / BR_ + KSTR q), X BK_ NB / NT values
  // (k = t % BK_, col t / BK_ + XSTR q), unconditional buffer loads (elements outside the matrix read as
  // 0), consumed only at the next LDS store
  const int ai = t % BR_, ak = uni(t / BR_);   // ak is wave-uniform (BR_ >= 64)
  const int xk = t % BK_, xj = t / BK_;
  typedef typename Raw<T>::type RT;
  const bufrsrc abuf = make_buf(A, ((int64_t)(m - 1) * lda + m) * (int64_t)sizeof(T));
  const bufrsrc xbuf = make_buf(X, ((int64_t)(n - 1) * ldx + m) * (int64_t)sizeof(T));
  RT ra[BR_ * BK_ / NT], rx[BK_ * NB / NT];
  for (int r0 = rb_first * BR_; r0 < m; r0 += rb_step * BR_) {
    auto load = [&](int k0) {
      const bool rok = r0 + ai < m;
#pragma unroll
      for (int q = 0; q < BR_ * BK_ / NT; ++q) {
        const int k = k0 + ak + KSTR * q;
        ra[q] = Raw<T>::load(abuf, (int64_t)k * lda + r0 + ai, rok && k < m);
      }
#pragma unroll
      for (int q = 0; q < BK_ * NB / NT; ++q) {
        const int j = xj + XSTR * q, k = k0 + xk;
        rx[q] = Raw<T>::load(xbuf, (int64_t)j * ldx + k, j < n && k < m);
      }
    };
    f64x4 w[RBW];
#pragma unroll
    for (int b = 0; b < RBW; ++b) w[b] = f64x4{0, 0, 0, 0};
    // dst += X_b^T W_b over this wave's rows.  X_b (the row block's rows of X) is staged through LDS
    // in halves of 64 rows, each one coalesced load (a wave per column, 64 rows) and one barrier,
    // so that the products wait for two memory round trips per call rather than one per 16-row block.
    // The tiles of the K loop are dead here (every K step ends with a barrier) and the halves overlay
    // them; the trailing barrier protects the half from the next K step's tile stores.
    auto accum = [&](f64x4 (&dst)[4]) {
#pragma unroll
      for (int hf = 0; hf < BR_ / 64; ++hf) {
        const int xi = t & 63, xw = uni(t >> 6);   // one column per wave
        RT xv[4 * CLS];
#pragma unroll
        for (int q = 0; q < 4 * CLS; ++q) {
          const int j = xw + 4 * q, row = r0 + 64 * hf + xi;
          xv[q] = Raw<T>::load(xbuf, (int64_t)j * ldx + row, j < n && row < m);
        }
#pragma unroll
        for (int q = 0; q < 4 * CLS; ++q) S.xb[xi][xw + 4 * q] = (double)xv[q];
        __syncthreads();
        if (active) {
#pragma unroll
          for (int rb = 0; rb < RBW; ++rb) {
            const int rl = 16 * RBW * rg + 16 * rb - 64 * hf;     // first row of the block in this half
            if (rl >= 0 && rl < 64) {                              // wave-uniform
#pragma unroll
              for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
                for (int gi = 0; gi < CLS; ++gi)
                  if (gi < nbk) dst[gi] = mfma_f64(S.xb[rl + 4 * s4 + li][16 * gi + lj], w[rb][s4], dst[gi]);
            }
          }
        }
        __syncthreads();
      }
    };
    const int dend = min(m, r0 + BR_);         // end of the diagonal block
    auto kstep = [&](int k0) {
#pragma unroll
      for (int q = 0; q < BR_ * BK_ / NT; ++q) S.tl.As[(ak + KSTR * q) * ASTR + ai] = (double)ra[q];
#pragma unroll
      for (int q = 0; q < BK_ * NB / NT; ++q) S.tl.Xs[xk][xj + XSTR * q] = (double)rx[q];
      __syncthreads();
      load(k0 + BK_);                         // in flight during the MFMAs below (past the end: zeros)
      if (active) {
#pragma unroll
        for (int kk = 0; kk < BK_; kk += 4) {
          const double b = S.tl.Xs[kk + li][16 * cb + lj];
#pragma unroll
          for (int rb = 0; rb < RBW; ++rb)
            w[rb] = mfma_f64(S.tl.As[(kk + li) * ASTR + 16 * RBW * rg + 16 * rb + lj], b, w[rb]);
          __builtin_amdgcn_sched_barrier(0);   // operand reads of one K sub-step only: no hoisting
        }
      }
      __syncthreads();
    };
    load(r0);
    for (int k0 = r0; k0 < dend; k0 += BK_) kstep(k0);
    accum(g);                                  // D += X_b^T (A_b,diag X_b)
    if (dend < m) {
#pragma unroll
      for (int b = 0; b < RBW; ++b) w[b] = f64x4{0, 0, 0, 0};
      for (int k0 = dend; k0 < m; k0 += BK_) kstep(k0);
      accum(h);                                // H += X_b^T (A_b,right X)
    }
  }
  // sum the row groups into the waves of group 0
  if (RG > 1) {
    auto reduce_groups = [&](f64x4 (&v)[4]) {
      if (rg > 0 && active) {
#pragma unroll
        for (int gi = 0; gi < 4; ++gi)
#pragma unroll
          for (int r = 0; r < 4; ++r) S.red[wave - CLS][gi][r][lane] = v[gi][r];
      }
      __syncthreads();
      if (rg == 0 && active) {
#pragma unroll
        for (int q = 1; q < RG; ++q)
#pragma unroll
          for (int gi = 0; gi < 4; ++gi)
#pragma unroll
            for (int r = 0; r < 4; ++r) v[gi][r] += S.red[q * CLS + wave - CLS][gi][r][lane];
      }
      __syncthreads();
    };
    reduce_groups(g);
    reduce_groups(h);
  }
  // G = D + H + H^T: H through LDS (Ws is free until the end of the pass)
  const bool own = rg == 0 && active;
  if (own) {
#pragma unroll
    for (int gi = 0; gi < 4; ++gi)
#pragma unroll
      for (int r = 0; r < 4; ++r) S.f.Ws[gi * 16 + 4 * r + li][cb * 16 + lj] = h[gi][r];
  }
  __syncthreads();
  if (own) {
#pragma unroll
    for (int gi = 0; gi < 4; ++gi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = gi * 16 + 4 * r + li, j = cb * 16 + lj;
        g[gi][r] += h[gi][r] + ((i < nbk * 16) ? S.f.Ws[j][i] : 0.0);
      }
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) g_out[b] = g[b];
  __syncthreads();
}

// One CHOLQR pass on instance (A, X) in place: X <- X R^{-1}, R into smem Gs (upper, zero lower).
// Returns 0 or the failing pivot (1-based).
template <class T, int CLS, int SITE>
__device__ __forceinline__ void gram_shape(int shape, const T* A, int64_t lda, const T* X, int64_t ldx, int m, int n,
                                           int rb_first, int rb_step, Smem& S, f64x4 (&g)[4]) {
  switch (shape) {
    case 1: gram_phase<T, CLS, BR_OF[1], BK_OF[1], SITE>(A, lda, X, ldx, m, n, rb_first, rb_step, S, g); break;
    case 2: gram_phase<T, CLS, BR_OF[2], BK_OF[2], SITE>(A, lda, X, ldx, m, n, rb_first, rb_step, S, g); break;
    case 3: gram_phase<T, CLS, BR_OF[3], BK_OF[3], SITE>(A, lda, X, ldx, m, n, rb_first, rb_step, S, g); break;
    default: gram_phase<T, CLS, BR_OF[0], BK_OF[0], SITE>(A, lda, X, ldx, m, n, rb_first, rb_step, S, g); break;
  }
}

// G (or the part of G from the row blocks rb_first, rb_first + rb_step, ...) of instance (A, X) into the
// accumulators g of the waves of row group 0 (column block cb = wave < cls); returns cls.
template <class T, int SITE>
__device__ __forceinline__ int gram_wg(const T* A, int64_t lda, const T* X, int64_t ldx, int m, int n, int shape,
                                       int rb_first, int rb_step, Smem& S, f64x4 (&g)[4]) {
  const int nbk = (n + 15) / 16;
  shape = uni(shape);
  if (nbk <= 1) {
    gram_shape<T, 1, SITE>(shape, A, lda, X, ldx, m, n, rb_first, rb_step, S, g);
    return 1;
  }
  if (nbk == 2) {
    gram_shape<T, 2, SITE>(shape, A, lda, X, ldx, m, n, rb_first, rb_step, S, g);
    return 2;
  }
  gram_shape<T, 4, SITE>(shape, A, lda, X, ldx, m, n, rb_first, rb_step, S, g);
  return 4;
}

// The rest of one CHOLQR pass from G in the accumulators g (waves wave < cls of row group 0):
// R = chol(G + s I) with the shift-and-retry rule, R into smem Gs (upper, zero lower), then
// X <- Xin R^{-1} (X may alias Xin).  Returns 0 or the failing pivot (1-based).
template <class T, int SITE>
__device__ __noinline__ int finish_wg(const f64x4 (&g)[4], int cls, const T* Xin, int64_t ldxin, T* X, int64_t ldx,
                                      int m, int n, double unit, double c_first, double c_retry, int max_retries,
                                      Smem& S) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int li = lane >> 4, lj = lane & 15;
  const int nbk = (n + 15) / 16;
  const bool owner = wave < cls && wave < nbk;   // waves holding a column block of G
  const int cb = wave;
  // ---- R = chol(G + s I), retries from the accumulators ------------------------------------------
  // max diag(G): diagonal entries sit in block b == wave, element r with 4r + li == lj
  if (t < NB) S.diag[t] = 0.0;
  __syncthreads();
  if (owner) {
#pragma unroll
    for (int gi = 0; gi < 4; ++gi)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (gi == cb && 4 * r + li == lj) S.diag[cb * 16 + lj] = g[gi][r];
  }
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
    for (int e = t; e < NB * NB; e += NT) {
      const int i = e / NB, j = e % NB;
      if (i >= n || j >= n) S.f.Gs[i][j] = (i == j) ? 1.0 : 0.0;
    }
    if (owner) {
#pragma unroll
      for (int gi = 0; gi < 4; ++gi)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = gi * 16 + 4 * r + li, j = cb * 16 + lj;
          if (i < n && j < n) S.f.Gs[i][j] = g[gi][r] + (i == j ? s : 0.0);
        }
    }
    if (t == 0) S.fail = 0;
    __syncthreads();
    // right-looking, upper: one entry per thread-slot, two barriers per pivot
    for (int k = 0; k < n; ++k) {
      const double piv = S.f.Gs[k][k];
      if (!(piv > 0.0)) {
        if (t == 0) S.fail = k + 1;
        break;
      }
      const double rkk = sqrt(piv);
      double nv[NB * NB / NT];
#pragma unroll
      for (int q = 0; q < NB * NB / NT; ++q) {
        const int e = t + NT * q, i = e / NB, j = e % NB;
        double v = S.f.Gs[i][j];
        if (i == k && j >= k) v = (j == k) ? rkk : v / rkk;
        else if (i > k && j >= i) v = v - (S.f.Gs[k][i] / rkk) * (S.f.Gs[k][j] / rkk);
        nv[q] = v;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < NB * NB / NT; ++q) {
        const int e = t + NT * q, i = e / NB, j = e % NB;
        S.f.Gs[i][j] = nv[q];
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
    if (i > j) S.f.Gs[i][j] = 0.0;
  }
  __syncthreads();
  // ---- X <- X R^{-1}: four lanes per row (lane `sub` owns columns sub + 4e), the pivot column's
  // value broadcast within the quad; q_ij = (x_ij - sum_{k<j} q_ik r_kj) / r_jj, k ascending ---------
  // The next 64 rows are loaded while the current ones are solved (rows are disjoint, so X may alias
  // Xin); loads past the end read zeros.
  {
    typedef typename Raw<T>::type RT;
    const int sub = t & 3;
    const bufrsrc inb = make_buf(uni(Xin), (uni((int64_t)(n - 1) * ldxin) + uni(m)) * (int64_t)sizeof(T));
    RT xn[NB / 4];
    auto fetch = [&](int r0) {
      const int row = r0 + (t >> 2);
#pragma unroll
      for (int e = 0; e < NB / 4; ++e)
        xn[e] = Raw<T>::load(inb, (int64_t)(sub + 4 * e) * ldxin + row, row < m && sub + 4 * e < n);
    };
    fetch(0);
    for (int r0 = 0; r0 < m; r0 += NT / 4) {
      const int row = r0 + (t >> 2);
      const bool ok = row < m;
      double x[NB / 4];
#pragma unroll
      for (int e = 0; e < NB / 4; ++e) x[e] = (double)xn[e];
      fetch(r0 + NT / 4);
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c < n) {
          const int owner = c & 3, ec = c >> 2;
          const double qo = x[ec] / S.f.Gs[c][c];
          const double qv = __shfl(qo, (lane & ~3) | owner);
          if (sub == owner) x[ec] = qv;
#pragma unroll
          for (int e = 0; e < NB / 4; ++e) {
            const double upd = x[e] - qv * S.f.Gs[c][sub + 4 * e];
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

// One CHOLQR pass on instance (A, Xin) into X: X <- Xin R^{-1}, R into smem Gs (upper, zero lower).
// Returns 0 or the failing pivot (1-based).
template <class T>
__device__ __noinline__ int cholqr_pass_wg(const T* A, int64_t lda, const T* Xin, int64_t ldxin, T* X, int64_t ldx, int m,
                                           int n, int shape, double unit, double c_first, double c_retry,
                                           int max_retries, Smem& S) {
  f64x4 g[4];
  const int cls = gram_wg<T, 0>(A, lda, Xin, ldxin, m, n, shape, 0, 1, S, g);
  return finish_wg<T, 0>(g, cls, Xin, ldxin, X, ldx, m, n, unit, c_first, c_retry, max_retries, S);
}

// An item the kernel can run: the documented shape limits, leading dimensions that hold the matrices,
// and every operand within the byte range of a buffer resource (the streaming loads take 32-bit
// offsets).  Checked before anything of the item is read, so a malformed item only sets its info.
__host__ __device__ inline bool item_ok_size(const oqr_batch_item& it, int max_m, int64_t esize) {
  const int64_t m = it.m, n = it.n, lim = 0x7fffffff / esize;
  if (n < 1 || n > NB || m < n || m > max_m) return false;
  if (!it.a || !it.z || !it.q || !it.r) return false;
  if (it.lda < m || it.ldz < m || it.ldq < m || it.ldr < n) return false;
  if (it.lda > lim || it.ldz > lim || it.ldq > lim || it.ldr > lim) return false;
  return (m - 1) * it.lda + m <= lim && (n - 1) * it.ldz + m <= lim && (n - 1) * it.ldq + m <= lim;
}
template <class T>
__device__ __forceinline__ bool item_ok(const oqr_batch_item& it, int max_m) {
  const int64_t m = it.m, n = it.n, lim = 0x7fffffff / (int64_t)sizeof(T);
  if (n < 1 || n > NB || m < n || m > max_m) return false;
  if (!it.a || !it.z || !it.q || !it.r) return false;
  if (it.lda < m || it.ldz < m || it.ldq < m || it.ldr < n) return false;
  if (it.lda > lim || it.ldz > lim || it.ldq > lim || it.ldr > lim) return false;
  return (m - 1) * it.lda + m <= lim && (n - 1) * it.ldz + m <= lim && (n - 1) * it.ldq + m <= lim;
}

// Tile shape of an instance: the tuning table's entry for its m bucket and n class.
__host__ __device__ inline int m_bucket(int m) {
  int b = 0;
  for (int lim = 512; b < OQR_BATCH_MBUCKETS - 1 && m >= lim; lim <<= 1) ++b;
  return b;
}
__host__ __device__ inline int n_class(int n) { return n <= 8 ? 0 : n <= 16 ? 1 : n <= 32 ? 2 : 3; }

struct ShapeTable {
  uint8_t s[OQR_BATCH_MBUCKETS][OQR_BATCH_NCLASSES];
};

template <class T>
__global__ __launch_bounds__(NT, 2) void batch_kernel(const oqr_batch_item* __restrict__ items,
                                                    const int32_t* __restrict__ order, int batch, int max_m,
                                                    int32_t* __restrict__ counter, int32_t* __restrict__ info,
                                                    double c_retry, int max_retries, ShapeTable shapes,
                                                    const int32_t* __restrict__ big) {
  __shared__ Smem S;
  const int t = threadIdx.x;
  for (;;) {
    if (t == 0) S.idx = atomicAdd(counter, 1);
    __syncthreads();
    const int slot = S.idx;
    __syncthreads();
    if (slot >= batch) break;
    const int id = order[slot];
    if (big && big[id]) continue;            // split over several workgroups by the staged launches
    const oqr_batch_item it = items[id];
    if (!item_ok<T>(it, max_m)) {
      if (t == 0) info[id] = OQR_BATCH_BAD_ITEM;
      __syncthreads();
      continue;
    }
    const T* A = (const T*)it.a;
    const T* Z = (const T*)it.z;
    T* Q = (T*)it.q;
    T* R = (T*)it.r;
    const int m = it.m, n = it.n;
    const int shape = shapes.s[m_bucket(m)][n_class(n)];
    // pass 1 (Z -> Q), pass 2 (Q in place); both FP64 arithmetic
    int f = cholqr_pass_wg<T>(A, it.lda, Z, it.ldz, Q, it.ldq, m, n, shape, U64, 0.0, c_retry, max_retries, S);
    if (f) {
      if (t == 0) info[id] = f;
      __syncthreads();
      continue;
    }
    // R1 waits in the output R (upper n x n) across pass 2
    for (int e = t; e < n * n; e += NT) {
      const int i = e % n, j = e / n;
      R[(int64_t)j * it.ldr + i] = (T)S.f.Gs[i][j];
    }
    __syncthreads();
    f = cholqr_pass_wg<T>(A, it.lda, Q, it.ldq, Q, it.ldq, m, n, shape, U64, 0.0, c_retry, max_retries, S);
    if (f) {
      if (t == 0) info[id] = f;
      __syncthreads();
      continue;
    }
    // R = R2 R1: R2 in Gs, R1 (back from R) into Ws
    for (int e = t; e < NB * NB; e += NT) {
      const int i = e % NB, j = e / NB;
      S.f.Ws[i][j] = (i < n && j < n) ? (double)R[(int64_t)j * it.ldr + i] : 0.0;
    }
    __syncthreads();
    for (int e = t; e < n * n; e += NT) {
      const int i = e % n, j = e / n;
      double s = 0.0;
      if (i <= j)
        for (int k = i; k <= j; ++k) s += S.f.Gs[i][k] * S.f.Ws[k][j];
      R[(int64_t)j * it.ldr + i] = (T)s;
    }
    if (t == 0) info[id] = 0;
    __syncthreads();
  }
}

// Split instances (cooperative workgroups): the largest instances, those with m >= split_m, run each
// pass as `parts` workgroups over interleaved row blocks (part p takes row blocks p, p + parts, ...),
// whose partial Grams go to the workspace, then one workgroup per instance sums the parts in order
// and factors and solves.  Four launches (Gram parts and finish, twice) before the persistent kernel
// takes the rest; nothing waits on another workgroup.  The order kernel lists the split instances in
// large[0 .. ctl[1]) and flags them in big[].
constexpr int MAX_PARTS = 8;
constexpr int SPLIT_SLOTS = 512;
constexpr int PART_DOUBLES = 4 * 4 * 4 * 64;    // waves of row group 0 x accumulators x elements x lanes

template <class T>
__global__ __launch_bounds__(NT, 2) void split_gram_kernel(const oqr_batch_item* __restrict__ items,
                                                         const int32_t* __restrict__ large,
                                                         const int32_t* __restrict__ ctl, int parts, int pass,
                                                         const int32_t* __restrict__ info,
                                                         double* __restrict__ partial, ShapeTable shapes) {
  __shared__ Smem S;
  const int p = blockIdx.x, k = blockIdx.y;
  if (k >= ctl[1] || p >= parts) return;
  const int id = large[k];
  if (pass == 2 && info[id] != 0) return;
  const oqr_batch_item it = items[id];
  const int m = it.m, n = it.n;
  const T* X = (const T*)(pass == 1 ? it.z : it.q);
  const int64_t ldx = pass == 1 ? it.ldz : it.ldq;
  f64x4 g[4];
  const int cls = gram_wg<T, 1>((const T*)it.a, it.lda, X, ldx, m, n, shapes.s[m_bucket(m)][n_class(n)], p, parts, S, g);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  double* P = partial + ((int64_t)k * MAX_PARTS + p) * PART_DOUBLES;
  if (wave < cls) {
#pragma unroll
    for (int gi = 0; gi < 4; ++gi)
#pragma unroll
      for (int r = 0; r < 4; ++r) P[((wave * 4 + gi) * 4 + r) * 64 + lane] = g[gi][r];
  }
}

template <class T>
__global__ __launch_bounds__(NT, 2) void split_finish_kernel(const oqr_batch_item* __restrict__ items,
                                                           const int32_t* __restrict__ large,
                                                           const int32_t* __restrict__ ctl, int parts, int pass,
                                                           int32_t* __restrict__ info,
                                                           const double* __restrict__ partial, double c_retry,
                                                           int max_retries) {
  __shared__ Smem S;
  const int k = blockIdx.x;
  if (k >= ctl[1]) return;
  const int id = large[k];
  if (pass == 2 && info[id] != 0) return;
  const oqr_batch_item it = items[id];
  const int m = it.m, n = it.n;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int nbk = (n + 15) / 16, cls = nbk <= 1 ? 1 : (nbk == 2 ? 2 : 4);
  // G = sum of the parts, in part order
  f64x4 g[4];
#pragma unroll
  for (int gi = 0; gi < 4; ++gi) g[gi] = f64x4{0, 0, 0, 0};
  if (wave < cls) {
    for (int p = 0; p < parts; ++p) {
      const double* P = partial + ((int64_t)k * MAX_PARTS + p) * PART_DOUBLES;
#pragma unroll
      for (int gi = 0; gi < 4; ++gi)
#pragma unroll
        for (int r = 0; r < 4; ++r) g[gi][r] += P[((wave * 4 + gi) * 4 + r) * 64 + lane];
    }
  }
  T* Q = (T*)it.q;
  T* R = (T*)it.r;
  const T* Xin = (const T*)(pass == 1 ? it.z : it.q);
  const int64_t ldxin = pass == 1 ? it.ldz : it.ldq;
  const int f = finish_wg<T, 1>(g, cls, Xin, ldxin, Q, it.ldq, m, n, U64, 0.0, c_retry, max_retries, S);
  if (f) {
    if (t == 0) info[id] = f;
    return;
  }
  if (pass == 1) {
    // R1 waits in the output R (upper n x n) across pass 2
    for (int e = t; e < n * n; e += NT) {
      const int i = e % n, j = e / n;
      R[(int64_t)j * it.ldr + i] = (T)S.f.Gs[i][j];
    }
    return;
  }
  // R = R2 R1: R2 in Gs, R1 (back from R) into Ws
  for (int e = t; e < NB * NB; e += NT) {
    const int i = e % NB, j = e / NB;
    S.f.Ws[i][j] = (i < n && j < n) ? (double)R[(int64_t)j * it.ldr + i] : 0.0;
  }
  __syncthreads();
  for (int e = t; e < n * n; e += NT) {
    const int i = e % n, j = e / n;
    double sum = 0.0;
    if (i <= j)
      for (int kk = i; kk <= j; ++kk) sum += S.f.Gs[i][kk] * S.f.Ws[kk][j];
    R[(int64_t)j * it.ldr + i] = (T)sum;
  }
}

// order[] = instance indices sorted by decreasing cost m^2 n (one workgroup, bitonic sort in LDS).
constexpr int SORT_MAX = 8192;
// With split_m > 0 it also lists the split instances: the first `slots` items of the sorted order with
// m >= split_m that pass the item check go to large[] (count in ctl[1]) and get big[id] = 1.
__global__ __launch_bounds__(1024) void order_kernel(const oqr_batch_item* __restrict__ items, int batch,
                                                     int32_t* __restrict__ order, int32_t* __restrict__ counter,
                                                     int32_t* __restrict__ info, int split_m, int slots,
                                                     int max_m, int esize, int32_t* __restrict__ big,
                                                     int32_t* __restrict__ large) {
  __shared__ unsigned long long key[SORT_MAX];
  __shared__ int cnt[1024];
  const int t = threadIdx.x;
  int p2 = 1;
  while (p2 < batch) p2 <<= 1;
  // key = (2^50 - cost) << 13 | index: ascending keys = descending cost, ties by index
  for (int i = t; i < p2; i += 1024) {
    unsigned long long k = ~0ull;                      // padding sorts last
    if (i < batch) {
      const double cost = fmax(fmin((double)items[i].m * items[i].m * items[i].n, 1125899906842624.0), 0.0);
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
  if (split_m <= 0) {
    if (t == 0) counter[1] = 0;
    return;
  }
  // thread t examines sorted entries t CH .. t CH + CH - 1; an exclusive scan of the counts places them
  constexpr int CH = SORT_MAX / 1024;
  bool cand[CH];
  int c = 0;
#pragma unroll
  for (int u = 0; u < CH; ++u) {
    const int i = t * CH + u;
    bool ok = false;
    if (i < batch) {
      const oqr_batch_item it = items[(int)(key[i] & (SORT_MAX - 1))];
      ok = it.m >= split_m && item_ok_size(it, max_m, esize);
    }
    cand[u] = ok;
    c += ok ? 1 : 0;
  }
  cnt[t] = c;
  __syncthreads();
  if (t == 0) {
    int run = 0;
    for (int q = 0; q < 1024; ++q) {
      const int v = cnt[q];
      cnt[q] = run;
      run += v;
    }
    counter[1] = run < slots ? run : slots;
  }
  __syncthreads();
  int pos = cnt[t];
#pragma unroll
  for (int u = 0; u < CH; ++u) {
    const int i = t * CH + u;
    if (i < batch) {
      const int id = (int)(key[i] & (SORT_MAX - 1));
      const bool take = cand[u] && pos < slots;
      if (take) large[pos] = id;
      big[id] = take ? 1 : 0;
      pos += cand[u] ? 1 : 0;
    }
  }
}

__global__ void identity_order_kernel(int batch, int32_t* order, int32_t* counter, int32_t* info) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < batch) {
    order[i] = i;
    info[i] = 0;
  }
  if (i == 0) counter[0] = 0;
}

// Built-in tuning (used when the caller passes none): two workgroups per compute unit, largest instances
// first, the 128 x 32 shape for every class.
oqr_batch_tuning builtin_tuning() {
  oqr_batch_tuning tu;
  tu.wg_per_cu = 2;
  tu.sort = 1;
  for (int b = 0; b < OQR_BATCH_MBUCKETS; ++b)
    for (int c = 0; c < OQR_BATCH_NCLASSES; ++c) tu.shape[b][c] = 0;
  tu.split_m = 0;
  tu.parts = 1;
  return tu;
}

// Workspace: ctl (counter, split count) | order | big | large | partial Grams of the split instances.
struct BatchWs {
  int32_t* ctl;
  int32_t* order;
  int32_t* big;
  int32_t* large;
  double* partial;
  size_t bytes;
};
BatchWs batch_ws(int64_t batch, void* base) {
  const int64_t slots = batch < SPLIT_SLOTS ? batch : SPLIT_SLOTS;
  char* p = (char*)base;
  BatchWs w;
  size_t off = 0;
  w.ctl = (int32_t*)(p + off);
  off += align256(sizeof(int32_t) * 64);
  w.order = (int32_t*)(p + off);
  off += align256(sizeof(int32_t) * (size_t)batch);
  w.big = (int32_t*)(p + off);
  off += align256(sizeof(int32_t) * (size_t)batch);
  w.large = (int32_t*)(p + off);
  off += align256(sizeof(int32_t) * (size_t)slots);
  w.partial = (double*)(p + off);
  off += align256(sizeof(double) * (size_t)slots * MAX_PARTS * PART_DOUBLES);
  w.bytes = off;
  return w;
}

}  // namespace
}  // namespace oqr

using namespace oqr;

extern "C" {

void oqr_batched_default_tuning(oqr_batch_tuning* tuning) {
  if (tuning) *tuning = builtin_tuning();
}

size_t oqr_batched_workspace_bytes(int64_t batch, int32_t max_m, int32_t max_n, int32_t dtype) {
  (void)max_m;
  (void)max_n;
  (void)dtype;
  if (batch < 0 || batch > (1 << 30)) return 0;
  return batch_ws(batch > 0 ? batch : 1, nullptr).bytes;
}

int oqr_cholqr2_batched(int64_t batch, const oqr_batch_item* items_dev, int32_t dtype, int32_t max_m, int32_t max_n,
                        const oqr_opts* opts, const oqr_batch_tuning* tuning, void* ws, size_t ws_bytes,
                        int32_t* info_dev, void* stream) {
  if (batch < 0 || batch > (1 << 30)) return OQR_E_ARG;
  if (batch == 0) return OQR_OK;
  if (!items_dev || !info_dev || max_m < 1 || max_n < 1 || max_n > NB || max_m < max_n) return OQR_E_ARG;
  if (dtype != OQR_F64 && dtype != OQR_F32) return OQR_E_ARG;
  const oqr_batch_tuning tu = tuning ? *tuning : builtin_tuning();
  if (tu.wg_per_cu < 1 || tu.wg_per_cu > 3 || (tu.sort != 0 && tu.sort != 1)) return OQR_E_ARG;
  if (tu.split_m < 0 || tu.parts < 1 || tu.parts > MAX_PARTS) return OQR_E_ARG;
  ShapeTable shapes;
  for (int b = 0; b < OQR_BATCH_MBUCKETS; ++b)
    for (int c = 0; c < OQR_BATCH_NCLASSES; ++c) {
      if (tu.shape[b][c] >= NSHAPES) return OQR_E_ARG;
      shapes.s[b][c] = tu.shape[b][c];
    }
  oqr_opts o;
  if (opts) o = *opts;
  else oqr_default_opts(&o);
  if (!(o.shift_c >= 0.0) || o.max_retries < 0 || o.max_retries > 16) return OQR_E_ARG;
  if (o.pass1 != OQR_P_FP64 || o.pass2 != OQR_P_FP64) return OQR_E_UNSUPPORTED;
  const size_t need = oqr_batched_workspace_bytes(batch, max_m, max_n, dtype);
  if (!ws || ws_bytes < need || ((uintptr_t)ws & 255u)) return OQR_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const BatchWs w = batch_ws(batch, ws);
  const int slots = (int)(batch < SPLIT_SLOTS ? batch : SPLIT_SLOTS);
  // split instances need the sorted order (they are the largest); a batch that cannot be sorted in one
  // workgroup runs unsplit
  const bool split = tu.split_m > 0 && tu.sort && batch <= SORT_MAX;
  const int esize = dtype == OQR_F64 ? 8 : 4;
  if (tu.sort && batch <= SORT_MAX)
    order_kernel<<<1, 1024, 0, s>>>(items_dev, (int)batch, w.order, w.ctl, info_dev, split ? tu.split_m : 0, slots,
                                    max_m, esize, w.big, w.large);
  else
    identity_order_kernel<<<(unsigned)((batch + 255) / 256), 256, 0, s>>>((int)batch, w.order, w.ctl, info_dev);
  if (hipGetLastError() != hipSuccess) return OQR_E_HIP;
  // compute-unit count, queried once per device (outside any graph capture: the first call)
  const int cus = device_cu_count();
  int64_t grid = (int64_t)cus * tu.wg_per_cu;
  if (grid > batch) grid = batch;
  trace_pre(K_BATCH, s);
  if (split) {
    const dim3 pg(tu.parts, slots);
    for (int pass = 1; pass <= 2; ++pass) {
      if (dtype == OQR_F64) {
        split_gram_kernel<double><<<pg, NT, 0, s>>>(items_dev, w.large, w.ctl, tu.parts, pass, info_dev, w.partial,
                                                    shapes);
        split_finish_kernel<double><<<slots, NT, 0, s>>>(items_dev, w.large, w.ctl, tu.parts, pass, info_dev,
                                                         w.partial, o.shift_c, o.max_retries);
      } else {
        split_gram_kernel<float><<<pg, NT, 0, s>>>(items_dev, w.large, w.ctl, tu.parts, pass, info_dev, w.partial,
                                                   shapes);
        split_finish_kernel<float><<<slots, NT, 0, s>>>(items_dev, w.large, w.ctl, tu.parts, pass, info_dev,
                                                        w.partial, o.shift_c, o.max_retries);
      }
    }
  }
  if (dtype == OQR_F64)
    batch_kernel<double><<<(unsigned)grid, NT, 0, s>>>(items_dev, w.order, (int)batch, max_m, w.ctl, info_dev,
                                                       o.shift_c, o.max_retries, shapes, split ? w.big : nullptr);
  else
    batch_kernel<float><<<(unsigned)grid, NT, 0, s>>>(items_dev, w.order, (int)batch, max_m, w.ctl, info_dev,
                                                      o.shift_c, o.max_retries, shapes, split ? w.big : nullptr);
  const hipError_t e = hipGetLastError();
  trace_post(K_BATCH, s);
  return e == hipSuccess ? OQR_OK : OQR_E_HIP;
}

}  // extern "C"
