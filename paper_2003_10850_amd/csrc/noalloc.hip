// The device region of the allocation-free calls: one file-scope array per
// GPU (each device that loads the library holds its own copy until the
// process ends). Host code never uses the array's name as an address: the
// device address is looked up once per device, with that device current,
// and kept.
#include <mutex>

#include "g3_device.h"
#include "g3_internal.h"

static __device__ __align__(256) unsigned char scratch[g3::kNoAllocBytes];

// At global scope, so that `scratch` names the array above and not the ctx
// scratch function of namespace g3.
static hipError_t lookup_region(void **ptr) {
  return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

namespace g3 {
namespace {

constexpr int kMaxDevices = 64;
std::mutex region_mu;
void *region_ptr[kMaxDevices] = {};

}  // namespace

int noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(region_mu);
  if (region_ptr[device]) return (int)hipSuccess;
  void *ptr = nullptr;
  const hipError_t e = lookup_region(&ptr);
  if (e != hipSuccess) return (int)e;
  region_ptr[device] = ptr;
  return (int)hipSuccess;
}

void *noalloc_region(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(region_mu);
  return region_ptr[device];
}

}  // namespace g3
