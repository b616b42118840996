// placeholder: generic workgroup-per-instance kernels (filled in next)
#include "device_common.h"
namespace irk {
bool wg_class_supported(int, int, int) { return false; }
hipError_t launch_wg_class(int, int, int, const LaunchArgs&, int, int, hipStream_t) {
  return hipErrorInvalidValue;
}
}  // namespace irk
