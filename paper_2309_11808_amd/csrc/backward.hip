// Adjoint of the SPOD path (not part of the paper): filled in by the
// differentiation kernels.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace spod {

size_t backward_workspace(const Plan& p) {
  (void)p;
  return 0;
}

spod_status launch_backward(const Plan& p, const void* q, spod_dtype dtype, const double* lam,
                            const void* psi, const double* g_lam, const void* g_phi, int n_modes,
                            void* g_q, void* ws, hipStream_t st) {
  (void)p; (void)q; (void)dtype; (void)lam; (void)psi; (void)g_lam; (void)g_phi;
  (void)n_modes; (void)g_q; (void)ws; (void)st;
  return fail(SPOD_ERR_UNSUPPORTED, "spod_backward is not built yet");
}

}  // namespace spod
