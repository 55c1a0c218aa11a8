// Entry points of forms not built yet; the ABI refuses those options.
#include "internal.hpp"

namespace ivf {

hipError_t launch_coarse_mfma(const Tables&, const float*, int32_t, int, const Workspace&,
                              hipStream_t) {
  return hipErrorNotSupported;
}

hipError_t launch_scan_batched(const Tables&, const float*, int32_t, int32_t, int32_t, int32_t,
                               const Workspace&, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace ivf
