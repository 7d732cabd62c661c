// Shared device/host helpers of the oblique-QR library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "oqr.h"

namespace oqr {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Lane layouts of the MFMA instructions used here (wave64; verified on gfx950):
//  v_mfma_f64_16x16x4_f64   A[i][k]: lane l holds (i = l%16, k = l/16); B[k][j]: (k = l/16, j = l%16);
//                           D[i][j]: lane l, element r holds (i = 4r + l/16, j = l%16).
//  v_mfma_f32_16x16x4_f32   A and B as the FP64 instruction; D: lane l, element r holds (i = 4(l/16) + r, j = l%16).
//  v_mfma_f32_16x16x32_bf16 A[i][k]: lane l holds i = l%16, k = 8(l/16)+e; B[k][j]: k = 8(l/16)+e, j = l%16;
//                           D: lane l, element r holds (i = 4(l/16) + r, j = l%16).
//  v_mfma_f32_32x32x16_bf16 A[i][k]: i = l%32, k = 8(l/32)+e; B[k][j]: k = 8(l/32)+e, j = l%32;
//                           D: element r holds (i = 8(r/4) + 4(l/32) + r%4, j = l%32).

__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Round an FP32 value to bfloat16, nearest-even, returned as its 16 bits.
// (Inputs here are finite; a NaN input maps to a quiet NaN.)
__device__ __forceinline__ unsigned short bf16_bits(float f) {
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short b) { return __uint_as_float(((unsigned int)b) << 16); }

// Split x (FP64) into k bfloat16 slices s_0 = bf16(x), s_j = bf16(x - s_0 - ... - s_{j-1}),
// rounding through FP32 at each step.
template <int K>
__device__ __forceinline__ void split_bf16(double x, unsigned short (&s)[K]) {
  double r = x;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    s[j] = bf16_bits((float)r);
    r -= (double)bf16_to_f32(s[j]);
  }
}

// Branch-free guarded load: the element is always read from a valid address (index 0 when the
// guard fails) and replaced by zero afterwards, so no divergent branch or wait is generated.
template <class T>
__device__ __forceinline__ T sel_load(const T* base, int64_t idx, bool valid) {
  const T v = base[valid ? idx : 0];
  return valid ? v : T(0);
}

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

// Raw buffer loads: a buffer resource (base, size in bytes) and 32-bit byte offsets.  An offset
// at or beyond the size returns zero, which gives bounds-checked tile loads without branches or
// selects; kOOB marks a lane whose element lies outside the matrix.
typedef __amdgpu_buffer_rsrc_t bufrsrc;
constexpr uint32_t kOOB = 0x80000000u;
__device__ __forceinline__ bufrsrc make_buf(const void* base, int64_t bytes) {
  const int64_t lim = 0x7fffffff;
  const int nb = (int)(bytes <= 0 ? 0 : (bytes > lim ? lim : bytes));
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, nb, 0x00020000);
}
__device__ __forceinline__ double buf_f64(bufrsrc r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ __forceinline__ uint4 buf_b128(bufrsrc r, uint32_t off) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 v = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
  return make_uint4(v.x, v.y, v.z, v.w);
}

// 1 / sqrt(x) for finite x > 0: the hardware estimate refined by two Newton steps (a dependent chain
// of seven operations instead of a correctly rounded square root and a division; the result is within
// about one unit in the last place).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = fma(0.5 * r, fma(-x * r, r, 1.0), r);
  return fma(0.5 * r, fma(-x * r, r, 1.0), r);
}

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
// Leading dimension of the bfloat16 slices of Z: m rounded up to a multiple of 32.
__host__ __device__ inline int64_t split_ld(int64_t m) { return (m + 31) & ~(int64_t)31; }
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Kernel ids for oqr_trace_start (names in api.hip).
enum KernelId { K_GEMM_F64 = 1, K_GEMM_SPLIT = 2, K_GRAM = 3, K_CHOL = 4, K_TRSM = 5, K_STENCIL = 6, K_SPLIT_Z = 7,
               K_BATCH = 8, K_SYMM_DIAG = 9 };
void trace_pre(int kid, hipStream_t s);
void trace_post(int kid, hipStream_t s);

// ---- launchers implemented in the kernel translation units --------------------------------------

// Compute units of the current device (queried once per device).
int device_cu_count();

// W (m x n, ldw) = A (m x m, lda) * Z (m x n, ldz), FP64 MFMA.  When the tile grid is too small for
// the device, K is split over workgroups into FP64 partial products in kpart (gemm_kpart_bytes; null
// disables the split) that are then summed in a fixed order.  diag_layer: one more layer than the
// symmetric product's parts, for the diagonal blocks of a reduced-precision pass (launch_symm_diag_half).
size_t gemm_kpart_bytes(int64_t m, int64_t n, bool diag_layer = false);
hipError_t launch_gemm_f64(const double* A, int64_t lda, const double* Z, int64_t ldz, double* W, int64_t ldw,
                           int64_t m, int64_t n, double* kpart, hipStream_t s);
// A symmetric, only its upper block triangle read (blocks of 64 rows): Woff = (strictly upper block
// triangle of A) Z, then Wsym = Woff + blockdiag(A) Z, so that Z^T A Z = Z^T Wsym + Woff^T Z.  The
// strictly upper part is balanced over workgroups: row tiles t and R - 1 - t are paired and a pair is
// cut into symm_layers parts whose partial products go to the layers of kpart (summed by
// launch_symm_finish; with one layer the product goes to Woff directly).
int symm_layers(int64_t m, int64_t n, const double* kpart);
// f32: the FP32 operand pass (A and Z rounded to FP32, FP32 MFMA, FP32 sums over at most 960 rows of K
// folded into FP64).
hipError_t launch_symm_upper(const double* A, int64_t lda, const double* Z, int64_t ldz, double* Woff, int64_t ldw,
                             int64_t m, int64_t n, double* kpart, hipStream_t s, bool f32 = false);
// Woff of launch_symm_upper with A split on the fly into bfloat16 slices (Z pre-split, as for
// launch_gemm_split); the diagonal blocks are then added in FP64 by launch_symm_finish.
hipError_t launch_symm_split_upper(const double* A, int64_t lda, const unsigned short* zs, double* Woff, int64_t ldw,
                                   int64_t m, int64_t n, int slices, double* kpart, hipStream_t s);
// W' = (U + D/2) Z for symmetric A (U the strictly upper block triangle, D the diagonal blocks with
// their lower triangles dropped), FP64: Z^T A Z = Z^T W' + W'^T Z.  With more than one layer the
// partial products go to kpart and launch_layer_sum adds them into W.
hipError_t launch_symm_half(const double* A, int64_t lda, const double* Z, int64_t ldz, double* W, int64_t ldw,
                            int64_t m, int64_t n, double* kpart, hipStream_t s);
hipError_t launch_layer_sum(const double* kpart, int layers, int64_t m, int64_t n, double* W, int64_t ldw,
                            hipStream_t s);
// W = D' Z, FP64, D' the diagonal blocks of A with their lower triangles dropped and their diagonal
// halved; with the layers of launch_symm_upper / launch_symm_split_upper (U Z) it sums to W' of
// launch_symm_half, so that a reduced-precision pass can form Z^T A Z = Z^T W' + W'^T Z.
hipError_t launch_symm_diag_half(const double* A, int64_t lda, const double* Z, int64_t ldz, double* W, int64_t ldw,
                                 int64_t m, int64_t n, hipStream_t s);
hipError_t launch_symm_finish(const double* A, int64_t lda, const double* Z, int64_t ldz, double* Woff, double* Wsym,
                              int64_t ldw, int64_t m, int64_t n, const double* kpart, int layers, hipStream_t s);
// W = A * Z with A split on the fly into `slices` bfloat16 slices and Z pre-split (zs: slices x n
// columns of split_ld(m) bf16 each); FP32 MFMA accumulation over K tiles of 256, FP64 across tiles.
hipError_t launch_gemm_split(const double* A, int64_t lda, const unsigned short* zs, double* W, int64_t ldw,
                             int64_t m, int64_t n, int slices, double* kpart, hipStream_t s);
// Slices of Z for launch_gemm_split (layout chosen by n; split_z_elems bf16 elements).
size_t split_z_elems(int64_t m, int64_t n, int slices);
hipError_t launch_split_z(const double* Z, int64_t ldz, unsigned short* zs, int64_t m, int64_t n, int slices,
                          hipStream_t s);
// W = A Z for a matrix-free operator (7-point stencil or tridiagonal), FP64.
hipError_t launch_sparse_apply(const oqr_op* op, const double* Z, int64_t ldz, double* W, int64_t ldw,
                                int64_t n, hipStream_t s);

// Gram: partial[c] = (X^T Y) restricted to row chunk c, upper 64x64 tiles; then G = sum_c partial[c].
size_t gram_partial_bytes(int64_t m, int64_t n);
// G = Z^T W + W^T Z (upper triangle, both triangles written) for 128 < n <= 256, W the sum of `layers`
// m x n layers W + h wstride (leading dimension ldw), added in layer order as they are loaded.
hipError_t launch_gram_symm_layers(const double* Z, int64_t ldz, const double* W, int64_t ldw, int64_t wstride,
                                  int layers, int64_t m, int64_t n, double* partial, double* G, hipStream_t s);
// G = Z^T Wsym + Woff^T Z (upper triangle; both products accumulated in the same tiles, one pass).
hipError_t launch_gram_symm(const double* Z, int64_t ldz, const double* Wsym, const double* Woff, int64_t ldw,
                            int64_t m, int64_t n, double* partial, double* G, hipStream_t s);
// G = Z^T (A Z) for the 7-point operator (OQR_OP_STENCIL7) in one pass, A Z formed in registers and never
// stored; fits: n <= 128 and 32-bit offsets inside a 64-column block of Z.
bool stencil_gram_fits(const oqr_op* op, int64_t ldz, int64_t n);
size_t stencil_gram_partial_bytes(const oqr_op* op, int64_t n);
hipError_t launch_stencil_gram(const oqr_op* op, const double* Z, int64_t ldz, int64_t n, double* partial, double* G,
                               hipStream_t s);
// The same in split bfloat16 (slices 2 or 3): products p + q < slices on MFMA, FP32 over 256 rows, FP64 beyond.
hipError_t launch_stencil_gram_split(const oqr_op* op, const double* Z, int64_t ldz, int64_t n, int slices,
                                     double* partial, double* G, hipStream_t s);
hipError_t launch_gram_f64(const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t m, int64_t n,
                           double* partial, double* G, hipStream_t s);
hipError_t launch_gram_split(const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t m, int64_t n,
                             int slices, double* partial, double* G, hipStream_t s);
// The same in FP32 operands: X, Y rounded to FP32, FP32 MFMA, FP32 sums over 256 rows, FP64 beyond.
hipError_t launch_gram_fp32(const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t m, int64_t n,
                            double* partial, double* G, hipStream_t s);

// Shifted Cholesky of G (n x n, ld n, FP64, upper triangle read) into R (ldr), info on device.
// Shift s = c * unit * max_i G_ii with c = c_first on the first attempt; on a failed pivot the
// constant becomes c_retry (if it was 0) or 10c, at most max_retries times.  Skipped if *info != 0.
hipError_t launch_chol_small(const double* G, int64_t n, double* R, int64_t ldr, double unit, double c_first,
                             double c_retry, int max_retries, int32_t* info, double* shift_used, hipStream_t s);
// Q = Z R^{-1} (row-wise substitution), Q may alias Z.  Skipped when *info != 0.
hipError_t launch_trsm(const double* Z, int64_t ldz, const double* R, int64_t ldr, double* Q, int64_t ldq,
                       int64_t m, int64_t n, const int32_t* info, hipStream_t s);
// R = R2 * R1 (upper x upper).
hipError_t launch_trmm_upper(const double* R2, int64_t ld2, const double* R1, int64_t ld1, double* R, int64_t ldr,
                             int64_t n, const int32_t* info, hipStream_t s);
// Householder QR of W (m x n, overwritten by the reflectors): R (n x n, positive diagonal) and the
// explicit orthonormal factor Y (m x n).  tau: n doubles.
hipError_t launch_householder_qr(double* W, int64_t ldw, int64_t m, int64_t n, double* tau, double* R, int64_t ldr,
                                 double* Y, int64_t ldy, hipStream_t s);
// Euclidean QR of W (m x n, m >= n, overwritten): U (n x n, positive diagonal) and the explicit
// orthonormal factor Y (m x n).  A Householder TSQR tree for n <= 64, the column-by-column kernels
// above; ws: euclid_qr_ws_bytes(m, n).
size_t euclid_qr_ws_bytes(int64_t m, int64_t n);
hipError_t launch_euclid_qr(double* W, int64_t ldw, int64_t m, int64_t n, void* ws, double* U, int64_t ldu, double* Y,
                            int64_t ldy, hipStream_t s);
hipError_t launch_copy_matrix(const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t m, int64_t n,
                              hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t s);

}  // namespace oqr
