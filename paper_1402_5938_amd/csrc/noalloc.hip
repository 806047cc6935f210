// Static device scratch for the allocation-free operator product (gllmg_apply_noalloc).
//
// The two-kernel product writes every element's vector y_e into an element-vector buffer that the
// gather then sums in node order. gllmg_apply takes that buffer from the problem's workspace;
// gllmg_apply_noalloc takes it from the file-scope array below instead, so a caller that must
// not allocate (graph capture, a serving loop, a harness that forbids it) runs the same kernels
// on memory that exists from the moment the library's code is loaded on a device.
//
// In host code the array's name is only a host-side stand-in: its device address, which differs
// from device to device, is looked up once per device with hipGetSymbolAddress (with that
// device current) and kept in a per-device table; only that address is ever passed to kernels.
#include <mutex>

#include "internal.h"

namespace gllmg {

namespace {

__device__ __align__(256) char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

void* static_scratch(int dev) {
  GLLMG_CHECK(dev >= 0 && dev < kMaxDevices, GLLMG_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return g_scratch_ptr[dev];
  int cur = -1;
  GLLMG_HIP(hipGetDevice(&cur));
  if (cur != dev) GLLMG_HIP(hipSetDevice(dev));
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != dev) (void)hipSetDevice(cur);
  if (e != hipSuccess || p == nullptr)
    throw Error(GLLMG_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[dev] = p;
  return p;
}

}  // namespace gllmg
