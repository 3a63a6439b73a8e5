// Execution of a plan without allocation: the plan's intermediates live in
// a fixed device array instead of a caller-provided workspace.
//
// For callers that cannot allocate device memory while they run (code under
// stream capture, tight serving loops, harnesses that forbid allocation):
// hexla_execute_static runs the same steps and kernels as hexla_execute,
// with `scratch` as the workspace. The array is a file-scope device
// variable of kStaticScratchBytes; every device the library runs on holds
// its own copy until the process ends. Its device address is looked up once
// per device (hipGetSymbolAddress, with that device current) and only that
// address is handed to kernels and copies: the array's name is a host-side
// stand-in on the host.
//
// Every call on one device shares that device's array and leaves its
// contents behind; the plans' kernels never read a workspace byte they have
// not written in the same execution. Calls that overlap on one device (two
// streams, two threads) race on the array.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.h"

namespace {

constexpr size_t kStaticScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_lock;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's copy of `scratch` (the device must be
// current). Looked up on the first call on each device.
hipError_t scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> hold(g_lock);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace

extern "C" {

hexla_status hexla_execute_static(hexla_plan* plan, void* out, int64_t ld_out) {
  if (!plan) return HEXLA_E_INVALID_ARG;
  hexla_ctx* ctx = plan->ctx;
  if (!ctx) return HEXLA_E_INVALID_ARG;
  if (ctx->device < 0) return hexla::set_err(ctx, HEXLA_E_UNSUPPORTED, "dry-run context cannot execute");
  if (ctx->device >= kMaxDevices)
    return hexla::set_err(ctx, HEXLA_E_UNSUPPORTED, "execute_static: device index above 63");
  if (plan->ws_bytes > kStaticScratchBytes)
    return hexla::set_err(ctx, HEXLA_E_INVALID_ARG,
                          "execute_static: the plan needs " + std::to_string(plan->ws_bytes) +
                              " workspace bytes; the static scratch holds " +
                              std::to_string(kStaticScratchBytes));
  hipError_t e = hexla::enter_device(ctx->device);
  void* ws = nullptr;
  if (e == hipSuccess) e = scratch_address(ctx->device, &ws);
  if (e != hipSuccess) {
    ctx->err = std::string("execute_static: scratch address: ") + hipGetErrorString(e);
    return HEXLA_E_DEVICE;
  }
  const hexla_status st = hexla::check_buffers(plan, out, ld_out, ws, kStaticScratchBytes);
  if (st != HEXLA_OK) return st;
  return hexla::run_steps(plan, out, ld_out, ws, ctx->stream);
}

hexla_status hexla_static_scratch_bytes(size_t* bytes) {
  if (!bytes) return HEXLA_E_INVALID_ARG;
  *bytes = kStaticScratchBytes;
  return HEXLA_OK;
}

}  // extern "C"
