// Host-side entry points of the kernels (shared by the context runtime and the
// serving loop).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>

#include "device_common.h"

namespace irk {

// Launch shapes picked by the autotuner (tuning.cpp); 0 = built-in default.
struct LaunchTune {
  int wg_block = 0;    // workgroup kernel: lanes per workgroup (systems per workgroup = block / slot)
  int large_tile = 0;  // whole-GPU kernel: sources per LDS tile (128 or 256)
};
struct TuneTable {
  std::map<std::string, int> values;
  int get(const std::string& key, int dflt) const;
};
TuneTable load_tune_table();
std::string wg_tune_key(int kind, int d, int S);
std::string large_tune_key(int n);
hipError_t launch_prepare(const InstDesc* desc, InstStat* stat, double* state,
                          const double* params, const double* q0, const double* p0, double* qout,
                          double* pout, uint8_t* step_iters, int32_t* heads, int n_heads,
                          int n_inst, hipStream_t st, const int32_t* ids = nullptr,
                          int64_t* prev = nullptr, uint8_t* evicted = nullptr);
hipError_t launch_nan_fill(const InstDesc* desc, const InstStat* stat, double* qout, double* pout,
                           int n_inst, hipStream_t st);
hipError_t launch_order(const int32_t* qin, int32_t* qout, int32_t count, const InstDesc* desc,
                        const InstStat* stat, int64_t* prev, int32_t* head, int32_t* qprom,
                        int32_t* counts, int32_t* head_prom, double promote_k,
                        uint8_t* evicted, hipStream_t st);
hipError_t launch_small_class(int kind, int nb, int d, const LaunchArgs& a, int n_items,
                              int num_cus, hipStream_t st);
bool small_class_supported(int kind, int nb, int d);
// Latency kernel for a few Kepler orbits (one 8-lane wavefront per orbit;
// bit-identical to the small-system kernel): whether a launch qualifies, and
// the launch.
bool kepler_lane_supported(int d, int n_items, const LaunchArgs& a);
hipError_t launch_kepler_lanes(int d, const LaunchArgs& a, int n_items, hipStream_t st);
hipError_t launch_wg_class(int kind, int d, int S, const LaunchArgs& a, int n_items, int num_cus,
                           hipStream_t st, int block = 0);
bool wg_class_supported(int kind, int n, int d);
int wg_slot_size(int n);
bool large_class_supported(int kind, int n, int d);
size_t large_scratch_bytes(int n, int nchunks);
size_t large_control_bytes();  // leading bytes of the scratch to zero once at allocation
int large_chunks(int n, bool exact, int num_cus);
hipError_t launch_large(const LaunchArgs& a, int inst, int n, void* scratch, int nchunks,
                        int num_cus, hipStream_t st, int tile = 0);
bool stage_class_supported(int kind, int n, int d);
int stage_np(int n);
hipError_t launch_stage_class(int d, int np, const LaunchArgs& a, int n_items, int num_cus,
                              hipStream_t st);

// User-supplied force compiled at run time (user_force.cpp): instances of
// Dq = dq components (unit masses) on the one-instance-per-lane kernel for
// dq <= kLaneMaxDqHost, else on the small-system kernel (one per 8-lane slot).
constexpr int kUserMaxDq = 64;
constexpr int kLaneMaxDqHost = 4;  // = kLaneMaxDq of lane_kernel.h
struct UserKernel {
  hipModule_t mod = nullptr;
  hipFunction_t fn = nullptr;
  int dq = 0;
  int per_cu = 1;          // occupancy: workgroups per CU
  int lanes_per_inst = 8;  // 1: lane kernel, 8: small-system kernel
  bool exact = false;
  bool ode = false;        // first-order form (irkgl16_user_rhs)
  int stages = 8;          // s of the s-stage member (2, 4, 6, 8)
  int method = 0;          // 0: IRKGL; 1: Strang; 2: SUZ90 (explicit baselines)
};
bool user_dq_supported(int dq);
bool stages_supported(int s);  // 2, 4, 6, 8
// 0 on success; -1 compile error (log filled); -3 HIP error.
int user_compile_check(const char* src, int dq, bool ode, std::string* log);
int user_kernel_create(const char* src, int dq, bool exact, bool ode, int stages, int method,
                       UserKernel** out, std::string* log);
void user_kernel_free(UserKernel* k);
hipError_t launch_user(const UserKernel& k, const LaunchArgs& a, int n_items, int num_cus,
                       hipStream_t st);

// Kernel classes.
constexpr int kClassSmall = 0;  // several systems per wavefront (few bodies)
constexpr int kClassWg = 1;     // one lane per body or site, systems in workgroup slots
constexpr int kClassLarge = 2;  // one system on the whole GPU (cooperative launch)
constexpr int kClassStage = 3;  // one lane per (body, stage), one system per workgroup
constexpr int kClassUser = 4;   // user force compiled at run time (small-system kernel)

// Kernel class of a problem, or -1 if unsupported.  *size: the class's size
// parameter (bodies for the small kernel, slot width for the workgroup kernel,
// padded body count for the stage-parallel kernel).
inline int kernel_class(int kind, int n, int d, int* size) {
  *size = 0;
  if (small_class_supported(kind, n, d)) {
    *size = n;
    return kClassSmall;
  }
  if (stage_class_supported(kind, n, d)) {
    *size = stage_np(n);
    return kClassStage;
  }
  if (wg_class_supported(kind, n, d)) {
    *size = wg_slot_size(n);
    return kClassWg;
  }
  if (large_class_supported(kind, n, d)) return kClassLarge;
  return -1;
}

// Launches the persistent kernel of a batched class over the queue in `a`.
inline hipError_t launch_batched(int cls, int kind, int size, int d, const LaunchArgs& a,
                                 int n_items, int num_cus, hipStream_t st,
                                 const LaunchTune& tune = LaunchTune()) {
  switch (cls) {
    case kClassSmall:
      // a few Kepler orbits: one 8-lane wavefront each (the same arithmetic
      // as the slot kernel, a shorter iteration)
      if (kind == kKepler && kepler_lane_supported(d, n_items, a))
        return launch_kepler_lanes(d, a, n_items, st);
      return launch_small_class(kind, size, d, a, n_items, num_cus, st);
    case kClassWg: return launch_wg_class(kind, d, size, a, n_items, num_cus, st, tune.wg_block);
    case kClassStage: return launch_stage_class(d, size, a, n_items, num_cus, st);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace irk
