// Fixed device workspace for callers that cannot allocate device memory
// (code under stream capture, tight serving loops, harnesses that forbid
// allocation): one file-scope array per GPU, of kStaticWorkspaceBytes,
// used by opf_load_network_static as the workspace of a single instance.
//
// In host code the array's name is only a host-side stand-in; its device
// address is taken once per device with hipGetSymbolAddress (with that
// device current) and kept in a table, and only that address is ever
// passed to kernels, copies or fills.
#include <hip/hip_runtime.h>

#include <mutex>

#include "opf_internal.h"

namespace opf {

namespace {

__device__ __align__(256) char scratch[kStaticWorkspaceBytes];

constexpr int kMaxDevices = 64;

struct StaticSlot {
  void* ptr = nullptr;     // device address of this device's array
  const void* owner = nullptr;  // context whose iterate lives in it
};

std::mutex g_mu;
StaticSlot g_slots[kMaxDevices];

}  // namespace

hipError_t static_workspace_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_slots[device].ptr != nullptr) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) {
    e = hipSetDevice(device);
    if (e != hipSuccess) return e;
  }
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return e;
  g_slots[device].ptr = p;
  return hipSuccess;
}

void* static_workspace(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  return g_slots[device].ptr;
}

const void* static_workspace_claim(int device, const void* owner) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  const void* prev = g_slots[device].owner;
  g_slots[device].owner = owner;
  return prev;
}

void static_workspace_release(int device, const void* owner) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_slots[device].owner == owner) g_slots[device].owner = nullptr;
}

}  // namespace opf
