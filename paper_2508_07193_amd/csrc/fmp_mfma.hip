// BF16 MFMA transform passes: placeholder.
#include "fmp_common.h"
namespace fmp {
int mfma_zslab(int cls) { return 256 / kClasses[cls]; }
hipError_t launch_mfma_pass_a(int, const double*, float*, const BoxDev*, const DomainDev*,
                              const int4*, int, const __hip_bfloat16*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_mfma_pass_b(int, float*, const BoxDev*, const int4*, int,
                              const __hip_bfloat16*, const float*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_mfma_pass_c(int, const float*, double*, const BoxDev*, const DomainDev*,
                              const int4*, int, const __hip_bfloat16*, const double*, int,
                              hipStream_t) {
  return hipErrorNotSupported;
}
}  // namespace fmp
