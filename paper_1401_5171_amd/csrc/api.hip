// The C ABI of the library (declared in include/oqr.h): argument checks,
// workspace carving and the kernel sequence of each algorithm.  Every step
// runs on the caller's stream; nothing here allocates or synchronises.
#include <math.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "common.hpp"

// Scratch of oqr_cholqr2_noalloc: every device holds its own copy, at its own address, from the load
// of the library's code object until the process ends.  Host code never passes this name to a kernel
// (on the host it is only a handle); it uses the device address looked up by noalloc_scratch().
static __device__ __align__(256) unsigned char scratch[OQR_NOALLOC_SCRATCH_BYTES];

namespace oqr {

// ---- optional per-kernel timing (oqr_trace_start / oqr_trace_stop) ---------------------------
namespace {
struct TraceState {
  int kernel = 0;                       // 0 = off
  std::vector<hipEvent_t> begin, end;   // one pair per traced launch
  size_t used = 0;
  bool failed = false;
};
TraceState g_trace;

const char* const kKernelNames[] = {"",        "gemm_f64", "gemm_split", "gram",  "chol",     "trsm",
                                    "stencil", "split_z",  "batch",      "symm_diag"};
constexpr int kNumKernels = 10;
}  // namespace

void trace_pre(int kid, hipStream_t s) {
  if (g_trace.kernel != kid || g_trace.failed) return;
  if (g_trace.used == g_trace.begin.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      g_trace.failed = true;
      return;
    }
    g_trace.begin.push_back(a);
    g_trace.end.push_back(b);
  }
  if (hipEventRecord(g_trace.begin[g_trace.used], s) != hipSuccess) g_trace.failed = true;
}

void trace_post(int kid, hipStream_t s) {
  if (g_trace.kernel != kid || g_trace.failed) return;
  if (hipEventRecord(g_trace.end[g_trace.used], s) != hipSuccess) g_trace.failed = true;
  ++g_trace.used;
}

#define OQR_TRACED(kid, s, expr)            \
  do {                                      \
    trace_pre((kid), (s));                  \
    hipError_t e_ = (expr);                 \
    trace_post((kid), (s));                 \
    if (e_ != hipSuccess) return OQR_E_HIP; \
  } while (0)

// Implemented in k_check.hip / k_baselines.hip / k_gs.hip / k_batch.hip.
size_t check_workspace_bytes(const oqr_op* A, int64_t m, int64_t n);
int check_run(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n, const double* Q, int64_t ldq,
              const double* R, int64_t ldr, void* ws, size_t ws_bytes, double* out, hipStream_t s);
size_t gs_workspace_bytes(const oqr_op* A, int64_t m, int64_t n);
int gs_run(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n, double* Q, int64_t ldq, double* R,
           int64_t ldr, int variant, void* ws, int32_t* info, hipStream_t s);
size_t gls_workspace_bytes(const oqr_op* A, int64_t m, int64_t n, int64_t k);
int gls_run(const oqr_op* A, const double* Q, int64_t ldq, const double* R, int64_t ldr, int64_t m, int64_t n,
            const double* B, int64_t ldb, int64_t k, double* X, int64_t ldx, void* ws, hipStream_t s);
size_t chol_a_workspace_bytes(int64_t m, int64_t n);
size_t chol_a_tridiag_workspace_bytes(int64_t m, int64_t n);
int chol_a_tridiag_run(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n, double* Q, int64_t ldq,
                       double* R, int64_t ldr, void* ws, int32_t* info, hipStream_t s);
int chol_a_run(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n, double* Q, int64_t ldq,
               double* R, int64_t ldr, void* ws, int32_t* info, hipStream_t s);
size_t eig_a_workspace_bytes(int64_t m, int64_t n);
int eig_a_run(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n, double* Q, int64_t ldq,
              double* R, int64_t ldr, void* ws, int32_t* info, hipStream_t s);

namespace {

constexpr double U64 = 1.1102230246251565e-16;   // 2^-53
constexpr double U32 = 5.9604644775390625e-08;   // 2^-24

#define OQR_TRY(expr)                       \
  do {                                      \
    hipError_t e_ = (expr);                 \
    if (e_ != hipSuccess) return OQR_E_HIP; \
  } while (0)

oqr_opts defaults() {
  oqr_opts o;
  o.pass1 = OQR_P_FP64;
  o.pass2 = OQR_P_FP64;
  o.shift_c = 1.0;
  o.max_retries = 3;
  o.gs_variant = OQR_GS_CGS;
  return o;
}

int64_t op_m(const oqr_op* A) { return (int64_t)A->nx * A->ny * A->nz; }

int slices_of(int prec) { return prec == OQR_P_BF16X3 ? 3 : 2; }

bool prec_ok(int p) { return p == OQR_P_FP64 || p == OQR_P_FP32 || p == OQR_P_BF16X2 || p == OQR_P_BF16X3; }
bool split_prec(int p) { return p == OQR_P_BF16X2 || p == OQR_P_BF16X3; }

int check_op(const oqr_op* A, int64_t m) {
  if (!A) return OQR_E_ARG;
  if (A->kind == OQR_OP_DENSE) {
    if (!A->a || A->lda < m || A->lda < 1) return OQR_E_ARG;
    if (A->dtype != OQR_F64) return OQR_E_UNSUPPORTED;
  } else if (A->kind == OQR_OP_STENCIL7) {
    if (A->nx < 1 || A->ny < 1 || A->nz < 1 || op_m(A) != m) return OQR_E_ARG;
  } else if (A->kind == OQR_OP_TRIDIAG) {
    if (!A->a || A->lda != m || m < 1) return OQR_E_ARG;
    if (A->dtype != OQR_F64) return OQR_E_UNSUPPORTED;
  } else {
    return OQR_E_ARG;
  }
  return OQR_OK;
}

// The kernels address an operand with 32-bit byte offsets from a base that moves with the tile, and
// a tile spans at most min(n, 64) columns (Gram tiles, stencil column groups) or min(n, 256) (the
// right operand of the dense product).  Every leading dimension of an n-column operand, and the
// library's own m x n workspace (leading dimension below m + 32), must keep that many columns within
// 2^31 bytes; larger requests are refused rather than read past the reach of an offset.
bool offsets_fit(const oqr_op* A, int64_t m, int64_t n, int64_t ld) {
  const int64_t span = (A->kind == OQR_OP_DENSE) ? 256 : 64;
  const int64_t cols = n < 1 ? 1 : (n < span ? n : span);
  const int64_t reach = (int64_t)0x7fffffff / 8 / cols;
  return ld <= reach && m + 32 <= reach;
}

int check_common(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n, const double* Q, int64_t ldq,
                 const double* R, int64_t ldr, const int32_t* info) {
  if (m < 0 || n < 0 || m < n) return OQR_E_ARG;
  if (n > OQR_MAX_N) return OQR_E_UNSUPPORTED;
  if (!info) return OQR_E_ARG;
  if (n == 0) return OQR_OK;
  if (!Z || !Q || !R) return OQR_E_ARG;
  if (ldz < m || ldq < m || ldr < n || ldz < 1) return OQR_E_ARG;
  int rc = check_op(A, m);
  if (rc) return rc;
  if (!offsets_fit(A, m, n, ldz > ldq ? ldz : ldq)) return OQR_E_UNSUPPORTED;
  if (n * ldr > (int64_t)0x7fffffff / 8) return OQR_E_UNSUPPORTED;    // R through a buffer resource
  // Q may alias Z exactly; any other overlap is rejected.
  if (Q != Z) {
    const char* zb = (const char*)Z;
    const char* ze = zb + ((n - 1) * ldz + m) * sizeof(double);
    const char* qb = (const char*)Q;
    const char* qe = qb + ((n - 1) * ldq + m) * sizeof(double);
    if (qb < ze && zb < qe) return OQR_E_ARG;
  } else if (ldq != ldz) {
    return OQR_E_ARG;
  }
  return OQR_OK;
}

// Workspace of one CholQR pass sequence.
struct Carve {
  char* base;
  size_t off;
  template <class T>
  T* take(size_t count) {
    T* p = (T*)(base + off);
    off = align256(off + count * sizeof(T));
    return p;
  }
};

struct PassWs {
  double* W;          // m x n, leading dimension ldw (dense: the strictly upper block triangle of A times Z;
                      // stencil: A Z, or the first-pass Q of CholQR2 when the Gram is fused)
  int64_t ldw;
  double* Ws;         // m x n (dense: W + the diagonal blocks of A times Z)
  double* partial;    // Gram partials
  double* G;          // n x n
  double* R1;         // n x n (first pass of CholQR2)
  double* R2;         // n x n (second pass)
  unsigned short* zs; // bf16 slices of Z (dense reduced precision)
  double* kpart;      // split-K partial products of the dense GEMMs (may be empty)
  int kpart_layers;   // m x n layers in kpart
  double* shifts;     // [2] shift used per pass
};

// Leading dimension of the m x n workspace W.  For the stencil it is padded past a multiple of 128 bytes,
// so that the rows of different columns fall in different cache sets (with ld = m = 2^k the same row of
// every column maps to one set, and the neighbour rows that the fused Gram re-reads are evicted).
int64_t w_ld(const oqr_op* A, int64_t m) { return A->kind == OQR_OP_STENCIL7 ? (m + 15) / 16 * 16 + 16 : m; }

size_t pass_ws(const oqr_op* A, int64_t m, int64_t n, const oqr_opts& o, bool two, PassWs* out, void* base) {
  Carve c{(char*)base, 0};
  PassWs w;
  w.ldw = w_ld(A, m);
  w.W = c.take<double>((size_t)w.ldw * n);
  w.Ws = c.take<double>(A->kind == OQR_OP_DENSE ? (size_t)m * n : 0);
  size_t pb = gram_partial_bytes(m, n);
  const size_t spb = stencil_gram_partial_bytes(A, n);
  if (spb > pb) pb = spb;
  w.partial = c.take<double>(pb / sizeof(double));
  w.G = c.take<double>((size_t)n * n);
  w.R1 = c.take<double>((size_t)n * n);
  w.R2 = c.take<double>((size_t)n * n);
  int maxs = 0;
  if (A->kind == OQR_OP_DENSE) {
    if (split_prec(o.pass1)) maxs = slices_of(o.pass1);
    if (two && split_prec(o.pass2) && slices_of(o.pass2) > maxs) maxs = slices_of(o.pass2);
  }
  w.zs = c.take<unsigned short>(maxs ? split_z_elems(m, n, maxs) : 0);
  // a reduced-precision dense pass with 128 < n <= 256 puts D' Z in a layer after the product's parts
  const bool reduced = o.pass1 != OQR_P_FP64 || (two && o.pass2 != OQR_P_FP64);
  const size_t kp = A->kind == OQR_OP_DENSE ? gemm_kpart_bytes(m, n, reduced && n > 128 && n <= 256) : 0;
  w.kpart = kp ? c.take<double>(kp / sizeof(double)) : nullptr;
  w.kpart_layers = (m > 0 && n > 0) ? (int)(kp / ((size_t)m * n * sizeof(double))) : 0;
  w.shifts = c.take<double>(2);
  if (out) *out = w;
  return c.off;
}

// G = Z^T A Z for symmetric A from Woff (strictly upper block triangle of A times Z) and Wsym (Woff plus
// the diagonal blocks): G = Z^T Wsym + Woff^T Z, upper triangle.
hipError_t gram_symm(const double* Z, int64_t ldz, int64_t m, int64_t n, const PassWs& w, hipStream_t s) {
  return launch_gram_symm(Z, ldz, w.Ws, w.W, m, m, n, w.partial, w.G, s);
}

// Whether a pass on the 7-point operator forms A Z inside the Gram kernel (FP64 and split bfloat16 Grams,
// n <= 128); the FP32 Gram runs unfused, on W = A Z.
bool stencil_fused(const oqr_op* A, int64_t ldz, int64_t n, int prec) {
  return A->kind == OQR_OP_STENCIL7 && prec != OQR_P_FP32 && stencil_gram_fits(A, ldz, n);
}

// One CHOLQR pass (Algorithm 1) on the device: W = A Z; G = Z^T W; R = chol(G [+ s I]); Q = Z R^{-1}.
// For the 7-point operator with n <= 128 the first two steps run as one kernel that never stores W.
// Dense A is symmetric: the product reads only its upper block triangle and G is assembled from the
// two halves (gram_symm).
int cholqr_pass(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n, double* Q, int64_t ldq,
                double* R, int64_t ldr, int prec, const oqr_opts& o, const PassWs& w, double* shift_slot,
                int32_t* info, hipStream_t s) {
  if (A->kind == OQR_OP_DENSE) {
    const double* a = (const double*)A->a;
    if (prec == OQR_P_FP64) {
      // W' = (U + D/2) Z, then G = Z^T W' + W'^T Z: the diagonal blocks ride in the product; for
      // 128 < n <= 256 the Gram adds the product's layers as it loads them
      const int H = symm_layers(m, n, w.kpart);
      OQR_TRACED(K_GEMM_F64, s, launch_symm_half(a, A->lda, Z, ldz, w.W, m, m, n, w.kpart, s));
      if (n > 128) {
        OQR_TRACED(K_GRAM, s, launch_gram_symm_layers(Z, ldz, H > 1 ? w.kpart : w.W, m, (int64_t)m * n, H, m, n,
                                                      w.partial, w.G, s));
      } else {
        if (H > 1) OQR_TRACED(K_SYMM_DIAG, s, launch_layer_sum(w.kpart, H, m, n, w.W, m, s));
        OQR_TRACED(K_GRAM, s, launch_gram_symm(Z, ldz, w.W, w.W, m, m, n, w.partial, w.G, s));
      }
    } else {
      // reduced precision: U Z in the pass's precision, the diagonal blocks in FP64.  For 128 < n <= 256
      // with the product in layers, D' Z goes to the next layer and the Gram adds them all as it loads
      // them: G = Z^T W' + W'^T Z as in the FP64 pass.  Otherwise Wsym = Woff + D Z and
      // G = Z^T Wsym + Woff^T Z.
      const int H = symm_layers(m, n, w.kpart);
      const bool layered = n > 128 && n <= 256 && H > 1 && w.kpart_layers > H;
      if (prec == OQR_P_FP32) {
        OQR_TRACED(K_GEMM_SPLIT, s, launch_symm_upper(a, A->lda, Z, ldz, w.W, m, m, n, w.kpart, s, true));
      } else {
        OQR_TRACED(K_SPLIT_Z, s, launch_split_z(Z, ldz, w.zs, m, n, slices_of(prec), s));
        OQR_TRACED(K_GEMM_SPLIT, s,
                   launch_symm_split_upper(a, A->lda, w.zs, w.W, m, m, n, slices_of(prec), w.kpart, s));
      }
      if (layered) {
        const int64_t mn = (int64_t)m * n;
        OQR_TRACED(K_SYMM_DIAG, s, launch_symm_diag_half(a, A->lda, Z, ldz, w.kpart + H * mn, m, m, n, s));
        OQR_TRACED(K_GRAM, s, launch_gram_symm_layers(Z, ldz, w.kpart, m, mn, H + 1, m, n, w.partial, w.G, s));
      } else {
        OQR_TRACED(K_SYMM_DIAG, s,
                   launch_symm_finish(a, A->lda, Z, ldz, w.W, w.Ws, m, m, n, w.kpart, H, s));
        OQR_TRACED(K_GRAM, s, gram_symm(Z, ldz, m, n, w, s));
      }
    }
  } else if (stencil_fused(A, ldz, n, prec)) {
    if (prec == OQR_P_FP64)
      OQR_TRACED(K_GRAM, s, launch_stencil_gram(A, Z, ldz, n, w.partial, w.G, s));
    else
      OQR_TRACED(K_GRAM, s, launch_stencil_gram_split(A, Z, ldz, n, slices_of(prec), w.partial, w.G, s));
  } else {
    OQR_TRACED(K_STENCIL, s, launch_sparse_apply(A, Z, ldz, w.W, w.ldw, n, s));
    if (prec == OQR_P_FP64)
      OQR_TRACED(K_GRAM, s, launch_gram_f64(Z, ldz, w.W, w.ldw, m, n, w.partial, w.G, s));
    else if (prec == OQR_P_FP32)
      OQR_TRACED(K_GRAM, s, launch_gram_fp32(Z, ldz, w.W, w.ldw, m, n, w.partial, w.G, s));
    else
      OQR_TRACED(K_GRAM, s, launch_gram_split(Z, ldz, w.W, w.ldw, m, n, slices_of(prec), w.partial, w.G, s));
  }
  const bool red = prec != OQR_P_FP64;
  OQR_TRACED(K_CHOL, s, launch_chol_small(w.G, n, R, ldr, red ? U32 : U64, red ? o.shift_c : 0.0,
                                          red ? 10.0 * o.shift_c : o.shift_c, o.max_retries, info, shift_slot, s));
  OQR_TRACED(K_TRSM, s, launch_trsm(Z, ldz, R, ldr, Q, ldq, m, n, info, s));
  return OQR_OK;
}

// PRE-CHOLQR workspace: one CholQR pass, then the Householder copy of Z, U and the Euclidean QR's own.
size_t pre_ws(const oqr_op* A, int64_t m, int64_t n, const oqr_opts& o) {
  return align256(pass_ws(A, m, n, o, false, nullptr, nullptr)) + align256((size_t)m * n * sizeof(double)) +
         align256((size_t)n * n * sizeof(double)) + align256(euclid_qr_ws_bytes(m, n));
}

int resolve_opts(const oqr_opts* in, oqr_opts* out) {
  *out = in ? *in : defaults();
  if (!prec_ok(out->pass1) || !prec_ok(out->pass2)) return OQR_E_ARG;
  if (!(out->shift_c >= 0.0) || !isfinite(out->shift_c)) return OQR_E_ARG;
  if (out->max_retries < 0 || out->max_retries > 16) return OQR_E_ARG;
  return OQR_OK;
}

int ws_check(void* ws, size_t ws_bytes, size_t need) {
  if (need == 0) return OQR_OK;
  if (!ws || ws_bytes < need || ((uintptr_t)ws & 255u)) return OQR_E_WORKSPACE;
  return OQR_OK;
}

// Device address of `scratch` on the current device, looked up once per device (with that device
// current) and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

int noalloc_scratch(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return OQR_E_HIP;
  if (dev < 0 || dev >= kMaxDevices) return OQR_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return OQR_E_HIP;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return OQR_OK;
}

}  // namespace
}  // namespace oqr

using namespace oqr;

extern "C" {

void oqr_default_opts(oqr_opts* opts) {
  if (opts) *opts = defaults();
}

int oqr_version(void) { return 100; }

int oqr_trace_start(const char* kernel) {
  if (!kernel) return OQR_E_ARG;
  int kid = 0;
  for (int k = 1; k < kNumKernels; ++k)
    if (strcmp(kernel, kKernelNames[k]) == 0) kid = k;
  if (!kid) return OQR_E_ARG;
  g_trace.kernel = kid;
  g_trace.used = 0;
  g_trace.failed = false;
  return OQR_OK;
}

int oqr_trace_stop(double* total_ms, int32_t* count) {
  if (!total_ms || !count) return OQR_E_ARG;
  const int kid = g_trace.kernel;
  g_trace.kernel = 0;
  *total_ms = 0.0;
  *count = 0;
  if (!kid) return OQR_E_ARG;
  if (g_trace.failed) return OQR_E_HIP;
  for (size_t i = 0; i < g_trace.used; ++i) {
    if (hipEventSynchronize(g_trace.end[i]) != hipSuccess) return OQR_E_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, g_trace.begin[i], g_trace.end[i]) != hipSuccess) return OQR_E_HIP;
    *total_ms += ms;
  }
  *count = (int32_t)g_trace.used;
  g_trace.used = 0;
  return OQR_OK;
}

const char* oqr_status_string(int status) {
  switch (status) {
    case OQR_OK: return "OQR_OK: success";
    case OQR_E_ARG: return "OQR_E_ARG: invalid argument (size, leading dimension, pointer or option)";
    case OQR_E_NOT_SPD: return "OQR_E_NOT_SPD: operator is not symmetric positive definite";
    case OQR_E_HIP: return "OQR_E_HIP: a HIP launch or runtime call failed";
    case OQR_E_WORKSPACE: return "OQR_E_WORKSPACE: workspace too small or not 256-byte aligned";
    case OQR_E_UNSUPPORTED: return "OQR_E_UNSUPPORTED: request not implemented by the library";
    case OQR_E_SCRATCH:
      return "OQR_E_SCRATCH: the request needs more scratch than the fixed OQR_NOALLOC_SCRATCH_BYTES of "
             "oqr_cholqr2_noalloc (use oqr_cholqr2 with a workspace)";
    default: return "unknown oqr status";
  }
}

size_t oqr_workspace_bytes(int32_t alg, const oqr_op* A, int64_t m, int64_t n, const oqr_opts* opts) {
  oqr_opts o;
  if (resolve_opts(opts, &o) != OQR_OK || !A || m < n || n < 0 || n > OQR_MAX_N) return 0;
  if (n == 0) return 0;
  if (check_op(A, m) != OQR_OK) return 0;
  switch (alg) {
    case OQR_ALG_CHOLQR: return pass_ws(A, m, n, o, false, nullptr, nullptr);
    case OQR_ALG_CHOLQR2: return pass_ws(A, m, n, o, true, nullptr, nullptr);
    case OQR_ALG_CHOL_A:
      return A->kind == OQR_OP_DENSE ? chol_a_workspace_bytes(m, n)
                                     : A->kind == OQR_OP_TRIDIAG ? chol_a_tridiag_workspace_bytes(m, n) : 0;
    case OQR_ALG_EIG_A: return A->kind == OQR_OP_DENSE ? eig_a_workspace_bytes(m, n) : 0;
    case OQR_ALG_GS: return gs_workspace_bytes(A, m, n);
    case OQR_ALG_PRE_CHOLQR: return pre_ws(A, m, n, o);
    default: return 0;
  }
}

int oqr_cholqr(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n, double* Q, int64_t ldq,
               double* R, int64_t ldr, const oqr_opts* opts, void* ws, size_t ws_bytes, int32_t* info_dev,
               void* stream) {
  int rc = check_common(A, Z, ldz, m, n, Q, ldq, R, ldr, info_dev);
  if (rc) return rc;
  oqr_opts o;
  if ((rc = resolve_opts(opts, &o))) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (n > 0 && (rc = ws_check(ws, ws_bytes, pass_ws(A, m, n, o, false, nullptr, nullptr)))) return rc;
  if (launch_fill_i32(info_dev, 0, 1, s) != hipSuccess) return OQR_E_HIP;
  if (n == 0) return OQR_OK;
  PassWs w;
  pass_ws(A, m, n, o, false, &w, ws);
  return cholqr_pass(A, Z, ldz, m, n, Q, ldq, R, ldr, o.pass1, o, w, w.shifts, info_dev, s);
}

int oqr_pre_cholqr(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n, double* Q, int64_t ldq,
                   double* R, int64_t ldr, const oqr_opts* opts, void* ws, size_t ws_bytes, int32_t* info_dev,
                   void* stream) {
  int rc = check_common(A, Z, ldz, m, n, Q, ldq, R, ldr, info_dev);
  if (rc) return rc;
  oqr_opts o;
  if ((rc = resolve_opts(opts, &o))) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (n > 0 && (rc = ws_check(ws, ws_bytes, pre_ws(A, m, n, o)))) return rc;
  if (launch_fill_i32(info_dev, 0, 1, s) != hipSuccess) return OQR_E_HIP;
  if (n == 0) return OQR_OK;

  PassWs w;
  char* base = (char*)ws;
  const size_t pw = align256(pass_ws(A, m, n, o, false, &w, base));
  double* Wh = (double*)(base + pw);
  double* U = (double*)(base + pw + align256((size_t)m * n * sizeof(double)));
  void* qr_ws = (char*)U + align256((size_t)n * n * sizeof(double));
  // Z = Y U (Householder, Euclidean product); Y goes to Q (Z has been copied, so Q may alias Z)
  if (launch_copy_matrix(Z, ldz, Wh, m, m, n, s) != hipSuccess) return OQR_E_HIP;
  if (launch_euclid_qr(Wh, m, m, n, qr_ws, U, n, Q, ldq, s) != hipSuccess) return OQR_E_HIP;
  // Y = Q S (CHOLQR-A), R = S U
  if ((rc = cholqr_pass(A, Q, ldq, m, n, Q, ldq, w.R1, n, o.pass1, o, w, w.shifts, info_dev, s))) return rc;
  if (launch_trmm_upper(w.R1, n, U, n, R, ldr, n, info_dev, s) != hipSuccess) return OQR_E_HIP;
  return OQR_OK;
}

int oqr_cholqr2(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n, double* Q, int64_t ldq,
                double* R, int64_t ldr, const oqr_opts* opts, void* ws, size_t ws_bytes, int32_t* info_dev,
                void* stream) {
  int rc = check_common(A, Z, ldz, m, n, Q, ldq, R, ldr, info_dev);
  if (rc) return rc;
  oqr_opts o;
  if ((rc = resolve_opts(opts, &o))) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (n > 0 && (rc = ws_check(ws, ws_bytes, pass_ws(A, m, n, o, true, nullptr, nullptr)))) return rc;
  if (launch_fill_i32(info_dev, 0, 1, s) != hipSuccess) return OQR_E_HIP;
  if (n == 0) return OQR_OK;
  PassWs w;
  pass_ws(A, m, n, o, true, &w, ws);
  // pass 1: Z -> (Q1, R1);  pass 2: Q1 -> (Q, R2);  R = R2 R1.  Q1 is kept in Q (pass 2 in place), or, for
  // the stencil with the fused Gram, in the padded workspace W, whose A Q1 the second pass never stores.
  const bool q1_in_w = stencil_fused(A, w.ldw, n, o.pass2);
  double* q1 = q1_in_w ? w.W : Q;
  const int64_t ldq1 = q1_in_w ? w.ldw : ldq;
  if ((rc = cholqr_pass(A, Z, ldz, m, n, q1, ldq1, w.R1, n, o.pass1, o, w, w.shifts, info_dev, s))) return rc;
  if ((rc = cholqr_pass(A, q1, ldq1, m, n, Q, ldq, w.R2, n, o.pass2, o, w, w.shifts + 1, info_dev, s))) return rc;
  if (launch_trmm_upper(w.R2, n, w.R1, n, R, ldr, n, info_dev, s) != hipSuccess) return OQR_E_HIP;
  return OQR_OK;
}

size_t oqr_noalloc_scratch_bytes(void) { return OQR_NOALLOC_SCRATCH_BYTES; }

int oqr_cholqr2_noalloc(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n, double* Q, int64_t ldq,
                        double* R, int64_t ldr, const oqr_opts* opts, int32_t* info_dev, void* stream) {
  int rc = check_common(A, Z, ldz, m, n, Q, ldq, R, ldr, info_dev);
  if (rc) return rc;
  oqr_opts o;
  if ((rc = resolve_opts(opts, &o))) return rc;
  if (n > 0 && pass_ws(A, m, n, o, true, nullptr, nullptr) > OQR_NOALLOC_SCRATCH_BYTES) return OQR_E_SCRATCH;
  void* ws = nullptr;
  if (n > 0 && (rc = noalloc_scratch(&ws))) return rc;
  // the same kernel sequence as oqr_cholqr2, on the library's scratch instead of a caller's workspace
  return oqr_cholqr2(A, Z, ldz, m, n, Q, ldq, R, ldr, opts, ws, OQR_NOALLOC_SCRATCH_BYTES, info_dev, stream);
}

int oqr_gs(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n, double* Q, int64_t ldq, double* R,
           int64_t ldr, const oqr_opts* opts, void* ws, size_t ws_bytes, int32_t* info_dev, void* stream) {
  int rc = check_common(A, Z, ldz, m, n, Q, ldq, R, ldr, info_dev);
  if (rc) return rc;
  oqr_opts o;
  if ((rc = resolve_opts(opts, &o))) return rc;
  if (o.gs_variant < OQR_GS_CGS || o.gs_variant > OQR_GS_CGS2) return OQR_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (n > 0 && (rc = ws_check(ws, ws_bytes, gs_workspace_bytes(A, m, n)))) return rc;
  if (launch_fill_i32(info_dev, 0, 1, s) != hipSuccess) return OQR_E_HIP;
  if (n == 0) return OQR_OK;

  return gs_run(A, Z, ldz, m, n, Q, ldq, R, ldr, o.gs_variant, ws, info_dev, s);
}

int oqr_chol_a(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n, double* Q, int64_t ldq,
               double* R, int64_t ldr, const oqr_opts* opts, void* ws, size_t ws_bytes, int32_t* info_dev,
               void* stream) {
  int rc = check_common(A, Z, ldz, m, n, Q, ldq, R, ldr, info_dev);
  if (rc) return rc;
  if (A->kind == OQR_OP_STENCIL7) return OQR_E_UNSUPPORTED;
  oqr_opts o;
  if ((rc = resolve_opts(opts, &o))) return rc;
  hipStream_t s = (hipStream_t)stream;
  const size_t need = A->kind == OQR_OP_TRIDIAG ? chol_a_tridiag_workspace_bytes(m, n) : chol_a_workspace_bytes(m, n);
  if (n > 0 && (rc = ws_check(ws, ws_bytes, need))) return rc;
  if (launch_fill_i32(info_dev, 0, 1, s) != hipSuccess) return OQR_E_HIP;
  if (n == 0) return OQR_OK;
  if (A->kind == OQR_OP_TRIDIAG) return chol_a_tridiag_run(A, Z, ldz, m, n, Q, ldq, R, ldr, ws, info_dev, s);
  return chol_a_run(A, Z, ldz, m, n, Q, ldq, R, ldr, ws, info_dev, s);
}

int oqr_eig_a(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n, double* Q, int64_t ldq,
              double* R, int64_t ldr, const oqr_opts* opts, void* ws, size_t ws_bytes, int32_t* info_dev,
              void* stream) {
  int rc = check_common(A, Z, ldz, m, n, Q, ldq, R, ldr, info_dev);
  if (rc) return rc;
  if (A->kind != OQR_OP_DENSE) return OQR_E_UNSUPPORTED;
  oqr_opts o;
  if ((rc = resolve_opts(opts, &o))) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (n > 0 && (rc = ws_check(ws, ws_bytes, eig_a_workspace_bytes(m, n)))) return rc;
  if (launch_fill_i32(info_dev, 0, 1, s) != hipSuccess) return OQR_E_HIP;
  if (n == 0) return OQR_OK;

  return eig_a_run(A, Z, ldz, m, n, Q, ldq, R, ldr, ws, info_dev, s);
}

size_t oqr_gls_workspace_bytes(const oqr_op* A, int64_t m, int64_t n, int64_t k) {
  if (!A || m < n || n < 1 || n > OQR_MAX_N || k < 0 || check_op(A, m) != OQR_OK) return 0;
  return gls_workspace_bytes(A, m, n, k > 0 ? k : 1);
}

int oqr_gls(const oqr_op* A, const double* Q, int64_t ldq, const double* R, int64_t ldr, int64_t m, int64_t n,
            const double* B, int64_t ldb, int64_t k, double* X, int64_t ldx, void* ws, size_t ws_bytes, void* stream) {
  if (!A || !Q || !R || !B || !X) return OQR_E_ARG;
  if (m < n || n < 1 || n > OQR_MAX_N || k < 0) return OQR_E_ARG;
  if (ldq < m || ldr < n || ldb < m || ldx < n) return OQR_E_ARG;
  if (check_op(A, m) != OQR_OK) return OQR_E_ARG;
  if (!offsets_fit(A, m, n, ldq) || !offsets_fit(A, m, k, ldb) || k > 0x7fffffff) return OQR_E_UNSUPPORTED;
  if (k == 0) return OQR_OK;
  int rc;
  if ((rc = ws_check(ws, ws_bytes, gls_workspace_bytes(A, m, n, k)))) return rc;
  return gls_run(A, Q, ldq, R, ldr, m, n, B, ldb, k, X, ldx, ws, (hipStream_t)stream);
}

int oqr_check(const oqr_op* A, const double* Z, int64_t ldz, int64_t m, int64_t n, const double* Q, int64_t ldq,
              const double* R, int64_t ldr, void* ws, size_t ws_bytes, double* out_dev, void* stream) {
  if (!out_dev) return OQR_E_ARG;
  if (m < n || n < 1 || n > OQR_MAX_N || !Z || !Q || !R || ldz < m || ldq < m || ldr < n) return OQR_E_ARG;
  int rc = check_op(A, m);
  if (rc) return rc;
  if (!offsets_fit(A, m, n, ldz > ldq ? ldz : ldq)) return OQR_E_UNSUPPORTED;
  if ((rc = ws_check(ws, ws_bytes, check_workspace_bytes(A, m, n)))) return rc;
  return check_run(A, Z, ldz, m, n, Q, ldq, R, ldr, ws, ws_bytes, out_dev, (hipStream_t)stream);
}

}  // extern "C"
