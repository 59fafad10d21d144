// Solve entry point that allocates nothing: the workspace lives in a
// file-scope device array instead of the context's allocation.
//
// In host code `scratch` names the host-side shadow of the array, not device
// memory; the device address of each GPU's copy is resolved once per device
// with hipGetSymbolAddress (that device current) and only that address is
// passed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pinmpc.h"
#include "pinmpc_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[PINMPC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_scratch[kMaxDevices] = {};   // device address of `scratch` per device

// Device address of this device's copy of `scratch` (resolved on the first
// call per device; the device must be current).  Null on failure.
void* scratch_on(int device) {
  std::lock_guard<std::mutex> lk(g_mutex);
  if (!g_scratch[device]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch[device] = ptr;
  }
  return g_scratch[device];
}

}  // namespace

extern "C" int pinmpc_solve_noalloc(pinmpc_ctx c, const pinmpc_batch* in, pinmpc_out* out,
                                    void* hip_stream) {
  const int device = pinmpc::context_device(c);
  if (device < 0 || device >= kMaxDevices || !out) return PINMPC_EINVAL;
  const int rc = pinmpc::check_batch(in);
  if (rc) return rc;
  size_t need = 0;
  pinmpc_workspace_bytes_contacts(nullptr, in->batch, in->n_max, pinmpc::contacts_of(in), &need);
  if (need > PINMPC_NOALLOC_SCRATCH_BYTES) return PINMPC_ETOOBIG;
  if (hipSetDevice(device) != hipSuccess) return PINMPC_EDEVICE;
  void* base = scratch_on(device);
  if (!base) return PINMPC_EDEVICE;
  return pinmpc::solve_in_buffer(c, in, out, (hipStream_t)hip_stream, base,
                                 PINMPC_NOALLOC_SCRATCH_BYTES);
}
