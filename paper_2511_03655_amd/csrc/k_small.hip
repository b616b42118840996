// Launchers of the small-system kernel (device code in small_kernel.h).
#include "small_kernel.h"

namespace irk {

// ------------------------------------------------------------------ launchers

template <int KIND, int NB, int D>
hipError_t launch_small(const LaunchArgs& a, int n_items, int num_cus, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  auto kern = a.exact ? small_kernel<KIND, NB, D, true> : small_kernel<KIND, NB, D, false>;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  const int want = (n_items + 7) / 8;
  const int cap = class_blocks_per_cu(per_cu, 1) * num_cus;
  const int grid = want < cap ? want : cap;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64), 0, st, a);
  return hipGetLastError();
}

// Small classes compiled in: (kind, bodies, dimension).
hipError_t launch_small_class(int kind, int nb, int d, const LaunchArgs& a, int n_items,
                              int num_cus, hipStream_t st) {
  if (kind == kKepler) {
    if (d == 2) return launch_small<kKepler, 1, 2>(a, n_items, num_cus, st);
    if (d == 3) return launch_small<kKepler, 1, 3>(a, n_items, num_cus, st);
  } else if (kind == kGravity && d == 3) {
    switch (nb) {
      case 2: return launch_small<kGravity, 2, 3>(a, n_items, num_cus, st);
      case 3: return launch_small<kGravity, 3, 3>(a, n_items, num_cus, st);
      case 4: return launch_small<kGravity, 4, 3>(a, n_items, num_cus, st);
      case 5: return launch_small<kGravity, 5, 3>(a, n_items, num_cus, st);
      case 6: return launch_small<kGravity, 6, 3>(a, n_items, num_cus, st);
      case 7: return launch_small<kGravity, 7, 3>(a, n_items, num_cus, st);
      case 8: return launch_small<kGravity, 8, 3>(a, n_items, num_cus, st);
      default: break;
    }
  } else if (kind == kGravity && d == 2) {
    switch (nb) {
      case 2: return launch_small<kGravity, 2, 2>(a, n_items, num_cus, st);
      case 3: return launch_small<kGravity, 3, 2>(a, n_items, num_cus, st);
      case 4: return launch_small<kGravity, 4, 2>(a, n_items, num_cus, st);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

bool small_class_supported(int kind, int nb, int d) {
  if (kind == kKepler) return nb == 1 && (d == 2 || d == 3);
  if (kind == kGravity && d == 3) return nb >= 2 && nb <= 8;
  if (kind == kGravity && d == 2) return nb >= 2 && nb <= 4;
  return false;
}

}  // namespace irk
