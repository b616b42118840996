// Run-time compilation of a user-supplied force (paper section 3.3: the
// user's right-hand side is a generic function that the method evaluates at
// all 8 stages at once; here the caller's device function is compiled with
// hiprtc into one of the batched kernels).
//
// The program handed to hiprtc is
//
//     #define IRKGL16_USER_FORCE 1       (or IRKGL16_USER_ODE: first-order form)
//     #define IRKGL16_DQ <dq>
//     <caller's source, which defines irkgl16_user_force (or irkgl16_user_rhs)>
//     #include "lane_kernel.h"     (dq <= kLaneMaxDq: one instance per lane)
//     #include "small_kernel.h"    (otherwise: one instance per 8-lane slot)
//     #include "split_kernel.h"    (explicit baselines: one instance per lane)
//
// with the device headers served from copies embedded in this library at
// build time, so the run-time kernel is the same code as the ahead-of-time
// one.  The kernels are instantiated for the context's stage count (8, or 2,
// 4, 6 for the lower-order members of the family).  Compiled code objects are
// cached per process by (source, dq, form, arithmetic mode, stage count).
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "lane_kernel.h"
#include "launch.h"
#include "rtc_headers.inc"

namespace irk {

namespace {

static_assert(kLaneMaxDqHost == kLaneMaxDq, "lane kernel size limit out of sync");

constexpr int kNumRtcHeaders = (int)(sizeof(kRtcHeaderNames) / sizeof(kRtcHeaderNames[0]));

bool use_lane_kernel(int dq) { return dq <= kLaneMaxDqHost; }

// Kicks per step of an explicit method (0: not explicit).
int split_kicks(int method) { return method == 1 ? 1 : method == 2 ? 5 : 0; }

std::string kernel_expr(int dq, bool exact, bool ode, int stages, int method) {
  if (split_kicks(method))
    return "&irk::split_kernel<" + std::to_string(kUser) + ", " + std::to_string(dq) + ", " +
           std::to_string(split_kicks(method)) + ">";
  const std::string mode = exact ? "true" : "false";
  const std::string kind = std::to_string(ode ? kUserOde : kUser);
  const std::string st = std::to_string(stages);
  if (use_lane_kernel(dq))
    return "&irk::lane_kernel<" + kind + ", " + std::to_string(dq) + ", " + mode + ", " + st + ">";
  return "&irk::small_kernel<" + kind + ", 1, " + std::to_string(dq) + ", " + mode + ", " + st +
         ">";
}

struct Compiled {
  std::vector<char> code;
  std::string lowered;
};

std::mutex g_cache_mu;
std::map<std::tuple<std::string, int, bool, bool, int, int>, Compiled> g_cache;

// Compiles the program for one (source, dq, form, mode, stage count); on
// failure returns false and the compiler log in *log.
bool compile(const char* src, int dq, bool exact, bool ode, int stages, int method,
             Compiled* out, std::string* log) {
  std::string prog = std::string(ode ? "#define IRKGL16_USER_ODE 1" : "#define IRKGL16_USER_FORCE 1") +
                     "\n#define IRKGL16_DQ " + std::to_string(dq) +
                     "\n#line 1 \"user_force\"\n" + src + "\n#line 1 \"irkgl16_rtc\"\n" +
                     (split_kicks(method)   ? "#include \"split_kernel.h\"\n"
                      : use_lane_kernel(dq) ? "#include \"lane_kernel.h\"\n"
                                            : "#include \"small_kernel.h\"\n");
  hiprtcProgram p;
  if (hiprtcCreateProgram(&p, prog.c_str(), "irkgl16_user.hip", kNumRtcHeaders, kRtcHeaderTexts,
                          kRtcHeaderNames) != HIPRTC_SUCCESS) {
    *log = "hiprtcCreateProgram failed";
    return false;
  }
  const std::string expr = kernel_expr(dq, exact, ode, stages, method);
  bool ok = hiprtcAddNameExpression(p, expr.c_str()) == HIPRTC_SUCCESS;
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
  const hiprtcResult rc = ok ? hiprtcCompileProgram(p, (int)(sizeof(opts) / sizeof(opts[0])), opts)
                             : HIPRTC_ERROR_INVALID_INPUT;
  size_t log_size = 0;
  if (hiprtcGetProgramLogSize(p, &log_size) == HIPRTC_SUCCESS && log_size > 1) {
    std::string l(log_size, '\0');
    if (hiprtcGetProgramLog(p, &l[0]) == HIPRTC_SUCCESS) {
      l.resize(std::strlen(l.c_str()));
      *log = l;
    }
  }
  ok = ok && rc == HIPRTC_SUCCESS;
  if (ok) {
    const char* lowered = nullptr;
    size_t code_size = 0;
    ok = hiprtcGetLoweredName(p, expr.c_str(), &lowered) == HIPRTC_SUCCESS && lowered &&
         hiprtcGetCodeSize(p, &code_size) == HIPRTC_SUCCESS && code_size > 0;
    if (ok) {
      out->lowered = lowered;
      out->code.resize(code_size);
      ok = hiprtcGetCode(p, out->code.data()) == HIPRTC_SUCCESS;
    }
    if (!ok && log->empty()) *log = "hiprtc produced no code object for the kernel";
  }
  (void)hiprtcDestroyProgram(&p);
  return ok;
}

bool compile_cached(const char* src, int dq, bool exact, bool ode, int stages, int method,
                    Compiled* out, std::string* log) {
  const auto key = std::make_tuple(std::string(src), dq, exact, ode, stages, method);
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      *out = it->second;
      return true;
    }
  }
  if (!compile(src, dq, exact, ode, stages, method, out, log)) return false;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_cache[key] = *out;
  return true;
}

}  // namespace

bool user_dq_supported(int dq) { return dq >= 1 && dq <= kUserMaxDq; }

bool stages_supported(int s) { return s == 2 || s == 4 || s == 6 || s == 8; }

int user_compile_check(const char* src, int dq, bool ode, std::string* log) {
  log->clear();
  if (!src || !user_dq_supported(dq)) {
    *log = "invalid source pointer or dimension";
    return -1;
  }
  Compiled c;
  return compile_cached(src, dq, false, ode, kS, 0, &c, log) ? 0 : -1;
}

int user_kernel_create(const char* src, int dq, bool exact, bool ode, int stages, int method,
                       UserKernel** out, std::string* log) {
  *out = nullptr;
  log->clear();
  if (!src || !user_dq_supported(dq) || !stages_supported(stages)) return -1;
  if (method != 0 && (ode || !split_kicks(method))) return -1;
  Compiled c;
  if (!compile_cached(src, dq, exact, ode, stages, method, &c, log)) return -1;
  UserKernel* k = new UserKernel();
  k->dq = dq;
  k->exact = exact;
  k->ode = ode;
  k->stages = stages;
  k->method = method;
  k->lanes_per_inst = (split_kicks(method) || use_lane_kernel(dq)) ? 1 : 8;
  if (hipModuleLoadData(&k->mod, c.code.data()) != hipSuccess ||
      hipModuleGetFunction(&k->fn, k->mod, c.lowered.c_str()) != hipSuccess) {
    user_kernel_free(k);
    *log = "loading the compiled code object failed";
    return -3;
  }
  int per_cu = 0;
  if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k->fn, 64, 0) != hipSuccess) {
    user_kernel_free(k);
    return -3;
  }
  k->per_cu = per_cu < 1 ? 1 : per_cu;
  *out = k;
  return 0;
}

void user_kernel_free(UserKernel* k) {
  if (!k) return;
  if (k->mod) (void)hipModuleUnload(k->mod);
  delete k;
}

hipError_t launch_user(const UserKernel& k, const LaunchArgs& a, int n_items, int num_cus,
                       hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  if (a.exact != (k.exact ? 1 : 0)) return hipErrorInvalidValue;
  const int per_wg = 64 / k.lanes_per_inst;  // instances per 64-lane workgroup
  const int want = (n_items + per_wg - 1) / per_wg;
  const int cap = class_blocks_per_cu(k.per_cu, 1) * num_cus;
  const int grid = want < cap ? want : cap;
  LaunchArgs arg = a;
  void* params[] = {&arg};
  return hipModuleLaunchKernel(k.fn, (unsigned)grid, 1, 1, 64, 1, 1, 0, st, params, nullptr);
}

}  // namespace irk
