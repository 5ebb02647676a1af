// Learned coarse correction (z += P0 MLP(R0 r)): placeholder entry points.
#include "fmp_common.h"

struct fmp_ctx;
fmp_status fmp_coarse_forward(fmp_ctx*, const double*, hipStream_t, const double** out) {
  *out = nullptr;
  return FMP_ERR_UNSUPPORTED;
}
size_t fmp_coarse_workspace(int, int) { return 256; }
void fmp_coarse_bind(fmp_ctx*, void*) {}

extern "C" {
fmp_status fmp_coarse_size(fmp_handle, int32_t*) { return FMP_ERR_UNSUPPORTED; }
fmp_status fmp_set_coarse_model(fmp_handle, int32_t, const float*, size_t) { return FMP_ERR_UNSUPPORTED; }
fmp_status fmp_coarse_restrict(fmp_handle, const double*, double*, void*) { return FMP_ERR_UNSUPPORTED; }
fmp_status fmp_mlp_loss_grad(int32_t, int32_t, int32_t, const float*, const float*, const float*,
                             float*, float*, void*, size_t, void*) { return FMP_ERR_UNSUPPORTED; }
size_t fmp_mlp_scratch_bytes(int32_t, int32_t, int32_t) { return 0; }
fmp_status fmp_mlp_adam(int32_t, float*, const float*, float*, float*, int32_t, float, void*) {
  return FMP_ERR_UNSUPPORTED;
}
}
