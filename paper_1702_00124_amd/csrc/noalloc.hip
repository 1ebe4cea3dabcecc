// Fixed device scratch for the allocation-free operator entry point
// (apply_K_noalloc): the intermediates of M-hat, J = K-hat + mu2 and the
// full-lattice K live in one file-scope device array instead of the
// context's workspace, so a call makes no device allocation.
//
// The array's name is a host-side stand-in in host code: its device address
// is read once per device with hipGetSymbolAddress (with that device current,
// from wl_create) and only that address is handed to kernels.  Every call on
// one device shares that device's array; calls that overlap on one device
// race.  No part of it needs to start at zero: each operator writes every
// intermediate site before it reads it.
#include <mutex>

#include "wl_ops.h"

namespace wl {

constexpr size_t kScratchBytes = size_t(256) << 20;  // 256 MiB per device
constexpr int kScratchDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};
}  // namespace

size_t scratch_limit() { return kScratchBytes; }

// the array's device address on `device` (the current device), looked up once
void scratch_register(int device) {
  WL_REQUIRE(device >= 0 && device < kScratchDevices, WL_EUNSUPPORTED, "scratch: device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  WL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  WL_REQUIRE(p != nullptr, WL_EHIP, "scratch: hipGetSymbolAddress returned a null address");
  g_scratch_ptr[device] = p;
}

void* scratch_ptr(int device) {
  WL_REQUIRE(device >= 0 && device < kScratchDevices, WL_EUNSUPPORTED, "scratch: device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  void* p = g_scratch_ptr[device];
  WL_REQUIRE(p != nullptr, WL_EINVAL, "scratch: not registered for this device (no context created on it)");
  return p;
}

}  // namespace wl
