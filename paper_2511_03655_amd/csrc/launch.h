// Host-side entry points of the kernels (shared by the context runtime and the
// serving loop).
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.h"

namespace irk {
hipError_t launch_prepare(const InstDesc* desc, InstStat* stat, double* state,
                          const double* params, const double* q0, const double* p0, double* qout,
                          double* pout, uint8_t* step_iters, int32_t* heads, int n_heads,
                          int n_inst, hipStream_t st, const int32_t* ids = nullptr);
hipError_t launch_small_class(int kind, int nb, int d, const LaunchArgs& a, int n_items,
                              int num_cus, hipStream_t st);
bool small_class_supported(int kind, int nb, int d);
hipError_t launch_wg_class(int kind, int d, int S, const LaunchArgs& a, int n_items, int num_cus,
                           hipStream_t st);
bool wg_class_supported(int kind, int n, int d);
int wg_slot_size(int n);
bool large_class_supported(int kind, int n, int d);
size_t large_scratch_bytes(int n, int nchunks);
int large_chunks(int n, bool exact, int num_cus);
hipError_t launch_large(const LaunchArgs& a, int inst, int n, void* scratch, int nchunks,
                        int num_cus, hipStream_t st);

// Kernel class of a problem: 0 small-system kernel, 1 workgroup kernel,
// 2 whole-GPU kernel, -1 unsupported.  S: slot width for class 1.
inline int kernel_class(int kind, int n, int d, int* S) {
  *S = 0;
  if (small_class_supported(kind, n, d)) return 0;
  if (wg_class_supported(kind, n, d)) {
    *S = wg_slot_size(n);
    return 1;
  }
  if (large_class_supported(kind, n, d)) return 2;
  return -1;
}
}  // namespace irk
