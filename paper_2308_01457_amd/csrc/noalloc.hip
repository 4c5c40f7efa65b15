// Work memory of the allocation-free entry point (fosb_far_field_moments_noalloc):
// a file-scope device array, one copy per GPU, whose address each device
// reports once through hipGetSymbolAddress.  Host code uses only that address.
#include "common.h"

namespace fosb {

static_assert(kNoAllocScratchBytes == (size_t)FOSB_NOALLOC_SCRATCH_BYTES, "scratch size");

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
}  // namespace

void noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) fail(FOSB_E_UNSUPPORTED, "device %d: at most %d devices", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_ptr[device]) return;
  int cur = -1;
  FOSB_HIP(hipGetDevice(&cur));
  if (cur != device) fail(FOSB_E_DEVICE, "scratch set-up: device %d is not current (%d is)", device, cur);
  void* p = nullptr;
  FOSB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) fail(FOSB_E_DEVICE, "scratch set-up: no address for device %d", device);
  g_ptr[device] = p;
}

void* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (device < 0 || device >= kMaxDevices || !g_ptr[device])
    fail(FOSB_E_DEVICE, "scratch of device %d was not set up (create a context on it first)", device);
  return g_ptr[device];
}

__global__ void k_zero_f64(double* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

void zero_f64(hipStream_t s, double* p, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  FOSB_LAUNCH_CHECK();
}

}  // namespace fosb
