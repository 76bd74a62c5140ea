// Fixed device workspace of the allocation-free entry points.
//
// `scratch` is a file-scope device array: every device the library runs on holds
// its own copy, at its own address, from the first use until the process ends.
// Host code never passes the array's name to a kernel (on the host it names a
// stand-in, not device memory); noalloc_init resolves the device address once
// per device with hipGetSymbolAddress and every later use goes through that
// pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

namespace tnfem {

static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_ptr[MAX_DEVICES] = {};
hipError_t g_status[MAX_DEVICES] = {};
bool g_tried[MAX_DEVICES] = {};
}  // namespace

void noalloc_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_tried[device]) return;
  g_tried[device] = true;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e == hipSuccess && cur != device) e = hipSetDevice(device);
  void* p = nullptr;
  if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_status[device] = e;
  g_ptr[device] = e == hipSuccess ? static_cast<double*>(p) : nullptr;
  if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
}

double* noalloc_scratch(int device) {
  if (device < 0 || device >= MAX_DEVICES) fail(TNFEM_EINVAL, "device %d out of range", device);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_tried[device]) fail(TNFEM_EDEVICE, "no context was created on device %d", device);
  if (!g_ptr[device])
    fail(TNFEM_EDEVICE, "hipGetSymbolAddress of the fixed workspace failed on device %d: %s", device,
         hipGetErrorString(g_status[device]));
  return g_ptr[device];
}

}  // namespace tnfem
