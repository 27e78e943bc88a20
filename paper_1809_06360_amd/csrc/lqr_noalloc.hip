// lqr_solve_noalloc: lqr_solve with the library's own scratch array in place
// of a caller-owned workspace, for callers that cannot allocate device memory.
//
// The array `scratch` below is a file-scope device variable: the runtime
// places one copy on each device when it loads the library's code there, and
// that copy lives until the process ends. In host code the name `scratch` is
// only a stand-in for the variable (handing it to a kernel would fault), so
// every use goes through the device address that hipGetSymbolAddress returns
// for the current device, looked up once per device and kept in g_scratch.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "lqr_kernels.h"
#include "mi355lqr.h"

static __device__ __align__(256) char scratch[LQR_NOALLOC_SCRATCH_BYTES];

namespace lqr {
namespace {

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch;  // device ordinal -> that device's copy of `scratch`

// Device address of the current device's copy of `scratch` (first call on a
// device: looked up with that device current).
lqr_status_t scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return LQR_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch.find(dev);
  if (it == g_scratch.end()) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr)
      return LQR_ERR_HIP;
    it = g_scratch.emplace(dev, ptr).first;
  }
  *out = it->second;
  return LQR_SUCCESS;
}

}  // namespace
}  // namespace lqr

extern "C" lqr_status_t lqr_solve_noalloc(const lqr_problem_t* prob, const lqr_options_t* opts,
                                          void* stream) {
  try {
    size_t need = 0;
    lqr_status_t st = lqr::solve_bytes(prob, opts, &need);
    if (st != LQR_SUCCESS) return st;
    if (need > (size_t)LQR_NOALLOC_SCRATCH_BYTES) return LQR_ERR_WORKSPACE;
    void* ws = nullptr;
    if ((st = lqr::scratch_address(&ws)) != LQR_SUCCESS) return st;
    return lqr::solve_single(prob, opts, ws, (size_t)LQR_NOALLOC_SCRATCH_BYTES, stream);
  } catch (...) {
    return LQR_ERR_INVALID_ARG;
  }
}
