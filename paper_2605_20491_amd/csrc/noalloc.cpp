// The separable inverse apply for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc): the apply's only scratch -- the ping-pong workspace of the
// MFMA passes, or the diagonal tables of the grouped small-extent passes --
// comes from one file-scope device array instead of the plan's lazily grown
// buffers.
//
// Each device holds its own copy of the array from the moment the library's
// code object is loaded on it until the process ends.  Its device address is
// looked up once per device (with that device current) and cached; host code
// uses only that address, never the array's name.  Every call on a device
// shares its array: calls that overlap on one device (two streams, two host
// threads) race on it and must be ordered by the caller.  Nothing in the
// array has to start at zero: the passes overwrite every scratch value they
// read.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/ts.h"
#include "ts_apply.h"
#include "ts_internal.h"

namespace ts {
namespace {

constexpr size_t kScratchBytes = TS_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (the current device).
int scratch_ptr(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) { set_error("device id out of range"); return TS_ERR_DEVICE; }
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("hipGetSymbolAddress of the no-alloc scratch failed: ") + hipGetErrorString(e));
      return TS_ERR_DEVICE;
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return TS_OK;
}

}  // namespace
}  // namespace ts

using namespace ts;

int ts_apply_inverse_noalloc(ts_plan* plan, const void* b, void* u, int dtype, int prec, void* hip_stream) {
  if (!plan) { set_error("null plan"); return TS_ERR_INVALID; }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) { set_error("hipGetDevice failed"); return TS_ERR_DEVICE; }
  if (dev != plan->device) {
    set_error("the plan lives on device " + std::to_string(plan->device) + " but device " + std::to_string(dev) +
              " is current");
    return TS_ERR_INVALID;
  }
  // carve the slots the inverse apply uses out of the array
  size_t off[kSlots] = {}, need[kSlots] = {};
  size_t total = 0;
  for (int i = 0; i < kSlots; ++i) {
    need[i] = need_inverse(plan, i);
    off[i] = total;
    total += (size_t)round_up((int64_t)need[i], 256);
  }
  if (total > kScratchBytes) {
    set_error("the apply needs " + std::to_string(total) + " bytes of scratch; the no-alloc entry point holds " +
              std::to_string(kScratchBytes) + " (use ts_apply_inverse)");
    return TS_ERR_INVALID;
  }
  void* base = nullptr;
  int rc = scratch_ptr(dev, &base);
  if (rc) return rc;
  ExecCtx c;
  c.growable = false;
  for (int i = 0; i < kSlots; ++i) {
    c.buf[i] = need[i] ? (char*)base + off[i] : nullptr;
    c.bytes[i] = need[i] ? (size_t)round_up((int64_t)need[i], 256) : 0;
  }
  return apply_inverse_impl(plan, plan->sigma, b, u, dtype, prec, (hipStream_t)hip_stream, c, nullptr);
}
