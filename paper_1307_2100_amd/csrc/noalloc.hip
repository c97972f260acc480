// tc_execute_noalloc: tc_execute with the workspace taken from a fixed
// device array instead of the caller, for callers that cannot allocate
// device memory (code under graph capture, serving loops).  Nothing here
// calls hipMalloc, hipFree or an allocating library routine.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/tc.h"
#include "kernels.hpp"

namespace {

// The workspace of every tc_execute_noalloc call on a device.  Each device
// holds its own copy from the library's load until the process ends.  In
// host code this name is not a device address: host code reaches the array
// only through the per-device pointer from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[TC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices];   // device address of `scratch` per device id (null until looked up)

// The array's device address on the current device, looked up once per
// device with that device current.
tc_status scratch_on_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return tc::set_error(TC_ERR_HIP, (std::string("hipGetDevice: ") + hipGetErrorString(e)).c_str());
  if (dev < 0 || dev >= kMaxDevices) return tc::set_error(TC_ERR_UNSUPPORTED, "device id beyond 63");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return tc::set_error(TC_ERR_HIP, (std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)).c_str());
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return TC_OK;
}

}  // namespace

extern "C" tc_status tc_execute_noalloc(tc_plan_t plan, const double* A, const double* B, double* C, double alpha,
                                        double beta, void* stream) {
  if (!plan) return tc::set_error(TC_ERR_INVALID_ARG, "plan is null");
  tc_plan_info info;
  tc_status s = tc_plan_query(plan, &info);
  if (s != TC_OK) return s;
  if (info.workspace_bytes > (size_t)TC_NOALLOC_SCRATCH_BYTES)
    return tc::set_error(TC_ERR_WORKSPACE,
                         ("plan needs a workspace of " + std::to_string(info.workspace_bytes) +
                          " bytes; tc_execute_noalloc holds at most " + std::to_string(TC_NOALLOC_SCRATCH_BYTES))
                             .c_str());
  void* ws = nullptr;
  if (info.workspace_bytes > 0) {
    s = scratch_on_current_device(&ws);
    if (s != TC_OK) return s;
  }
  // every kernel writes the workspace bytes it later reads (no counter or
  // accumulator there starts from zero), so the previous call's contents need
  // no clearing
  return tc_execute(plan, A, B, C, alpha, beta, ws, info.workspace_bytes ? (size_t)TC_NOALLOC_SCRATCH_BYTES : 0,
                    stream);
}
