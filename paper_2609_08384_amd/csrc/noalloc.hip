// brahms_propagate_noalloc: brahms_propagate for callers that cannot
// allocate device memory (see include/brahms.h).
//
// The plan's workspace (per-step propagator and twiddle tables, RK4
// coefficients, the finite flag and the diagnostics' partial sums) is taken
// from `scratch`, a fixed array in the library's device code object.  Each
// GPU holds its own copy at its own address; host code must never use the
// array's name as a device address (on the host it names a stand-in
// object), only the address hipGetSymbolAddress returns for the current
// device, looked up once per device and kept in g_scratch.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "../../include/brahms.h"
#include "plan.hpp"

using brahms::detail::fail;

namespace {

constexpr int kMaxDevices = 64;

// Device scratch of the no-allocation entry point (BRAHMS_NOALLOC_SCRATCH_BYTES).
static __device__ __align__(256) char scratch[BRAHMS_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of the current device's scratch (looked up on its first use
// on that device).
brahms_status scratch_address(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(BRAHMS_E_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[dev] == nullptr) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (ptr == nullptr || reinterpret_cast<uintptr_t>(ptr) % brahms::detail::kAlign != 0)
      return fail(BRAHMS_E_DEVICE, "scratch symbol has no usable device address");
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return BRAHMS_OK;
}

}  // namespace

extern "C" {

brahms_status brahms_propagate_noalloc(brahms_plan plan, void* const* fields, double z_end) {
  if (brahms_status st = brahms::detail::check_plan(plan)) return st;
  if (fields == nullptr) return fail(BRAHMS_E_INVALID_ARG, "fields is NULL");
  if (plan->use_graph)
    return fail(BRAHMS_E_STATE, "a plan with the graph schedule (capturing and releasing graphs "
                                "allocates and frees device memory)");
  if (plan->ws_size > size_t(BRAHMS_NOALLOC_SCRATCH_BYTES))
    return fail(BRAHMS_E_INVALID_ARG,
                "the plan needs " + std::to_string(plan->ws_size) +
                    " bytes of workspace, more than the static scratch of " +
                    std::to_string(size_t(BRAHMS_NOALLOC_SCRATCH_BYTES)) + " bytes");
  void* ws = nullptr;
  if (brahms_status st = scratch_address(&ws)) return st;
  // no timing events are created in this call
  const bool timing = plan->timing;
  plan->timing = false;
  brahms_status st = brahms_plan_bind(plan, fields, ws);
  if (st == BRAHMS_OK) st = brahms_propagate(plan, z_end);
  plan->timing = timing;
  return st;
}

}  // extern "C"
