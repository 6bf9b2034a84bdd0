// The position-resolved local energies for callers that cannot allocate
// device memory (code under graph capture, tight serving loops, harnesses
// that forbid allocation): the same computation as ttn_local_energies, with
// its work buffer in a static device array of this library instead of a
// buffer the caller brings.
//
// The array (NOALLOC_SCRATCH_BYTES) exists once per GPU the library runs on
// and lives until the process ends.  In host code its name is only a
// host-side stand-in; the device address comes from hipGetSymbolAddress,
// taken once per device with that device current and kept per device, and
// only that address is handed to the kernels.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "ttn.h"

static __device__ __align__(256) unsigned char scratch[TTN_NOALLOC_SCRATCH_BYTES];

namespace ttn {
hipStream_t handle_stream(ttn_handle h);
ttn_status set_error(ttn_status st, const char* msg);
}  // namespace ttn

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_scratch[MAX_DEVICES] = {};

// The device address of `scratch` on device dev, looked up on the first call
// for that device with the device current (the caller's current device is
// restored afterwards).
ttn_status scratch_on(int dev, void** out) {
  char msg[256];
  if (dev < 0 || dev >= MAX_DEVICES) {
    std::snprintf(msg, sizeof msg, "device %d outside [0, %d)", dev, MAX_DEVICES);
    return ttn::set_error(TTN_EINVAL, msg);
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != dev) {
      hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess || !p) {
      std::snprintf(msg, sizeof msg, "hipGetSymbolAddress of the static scratch on device %d: %s", dev,
                    hipGetErrorString(e));
      return ttn::set_error(TTN_EHIP, msg);
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return TTN_OK;
}

}  // namespace

extern "C" ttn_status ttn_local_energies_noalloc(ttn_handle h, int b, double* site, double* bond) {
  if (!h || !site || !bond) return ttn::set_error(TTN_EINVAL, "bad arguments");
  size_t need = 0;
  ttn_status st = ttn_positions_bytes(h, b, &need);
  if (st) return st;
  if (need > (size_t)TTN_NOALLOC_SCRATCH_BYTES) {
    char msg[256];
    std::snprintf(msg, sizeof msg, "member %d needs %zu bytes of work, above the %zu bytes of the static scratch", b,
                  need, (size_t)TTN_NOALLOC_SCRATCH_BYTES);
    return ttn::set_error(TTN_ENOMEM, msg);
  }
  // the device of the handle's stream (the null stream: the current device)
  int dev = -1;
  hipStream_t s = ttn::handle_stream(h);
  hipError_t e = s ? hipStreamGetDevice(s, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess) {
    char msg[256];
    std::snprintf(msg, sizeof msg, "device of the handle's stream: %s", hipGetErrorString(e));
    return ttn::set_error(TTN_EHIP, msg);
  }
  void* p = nullptr;
  if ((st = scratch_on(dev, &p))) return st;
  return ttn_local_energies(h, b, p, (size_t)TTN_NOALLOC_SCRATCH_BYTES, site, bond);
}
