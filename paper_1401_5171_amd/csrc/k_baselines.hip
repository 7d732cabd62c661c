// Baseline algorithms of the paper behind the same ABI (placeholders until built).
#include "common.hpp"

namespace oqr {

size_t gs_workspace_bytes(const oqr_op*, int64_t, int64_t) { return 0; }
int gs_run(const oqr_op*, const double*, int64_t, int64_t, int64_t, double*, int64_t, double*, int64_t, int, void*,
           int32_t*, hipStream_t) {
  return OQR_E_UNSUPPORTED;
}
size_t chol_a_workspace_bytes(int64_t, int64_t) { return 0; }
int chol_a_run(const oqr_op*, const double*, int64_t, int64_t, int64_t, double*, int64_t, double*, int64_t, void*,
               int32_t*, hipStream_t) {
  return OQR_E_UNSUPPORTED;
}
size_t eig_a_workspace_bytes(int64_t, int64_t) { return 0; }
int eig_a_run(const oqr_op*, const double*, int64_t, int64_t, int64_t, double*, int64_t, double*, int64_t, void*,
              int32_t*, hipStream_t) {
  return OQR_E_UNSUPPORTED;
}

}  // namespace oqr

