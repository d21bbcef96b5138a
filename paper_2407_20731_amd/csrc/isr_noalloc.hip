// Allocation-free compression (isr_compress_noalloc in include/isr.h) for
// callers that cannot allocate device memory: code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc.  Its scratch (the
// exponent histograms, selection state, candidate lists and per-element
// counts of one compression) is a fixed device array of this file, and the
// blob goes to the caller's buffer.
//
// Host code never passes the array's name to a kernel: on the host that name
// is only a stand-in for the device symbol.  Its device address is looked up
// once per GPU with hipGetSymbolAddress (each GPU holds its own copy of the
// array at its own address) and only that address is used afterwards.
#include <hip/hip_runtime.h>

#include <mutex>

#include "isr.h"
#include "isr_internal.h"
#include "isr_sched.h"

namespace isr {

static __device__ __align__(256) unsigned char scratch[ISR_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEV = 64;
static std::mutex g_mu[MAX_DEV];   // one compression at a time per GPU
static void* g_ptr[MAX_DEV];       // device address of `scratch` on each GPU, once looked up
static std::mutex g_init_mu;

// Look up the array's device address on `device`, which must be current.
// Called by isr_create; the entry point repeats it for a device not yet seen.
int noalloc_init(int device) {
  if (device < 0 || device >= MAX_DEV) return set_error(ISR_EINVAL, "device %d beyond the supported %d", device, MAX_DEV);
  std::lock_guard<std::mutex> g(g_init_mu);
  if (g_ptr[device]) return ISR_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return set_error(ISR_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
  g_ptr[device] = p;
  return ISR_OK;
}

// Header bytes of the serialized blob, written by a kernel from its
// arguments so that the entry point needs no staging memory.
struct HdrBytes {
  unsigned char b[ISR_NOALLOC_HDR_MAX];
  int n;
};

__global__ __launch_bounds__(64) void k_put_bytes(HdrBytes h, unsigned char* dst) {
  for (int i = threadIdx.x; i < h.n; i += 64) dst[i] = h.b[i];
}

hipError_t launch_put_bytes(const void* src, int n, void* dst, hipStream_t s) {
  HdrBytes h;
  if (n < 0 || n > ISR_NOALLOC_HDR_MAX) return hipErrorInvalidValue;
  for (int i = 0; i < n; ++i) h.b[i] = ((const unsigned char*)src)[i];
  h.n = n;
  hipLaunchKernelGGL(k_put_bytes, dim3(1), dim3(64), 0, s, h, (unsigned char*)dst);
  return hipGetLastError();
}

}  // namespace isr

extern "C" int isr_compress_noalloc(isr_ctx* ctx, const isr_field* f, void* d_out, uint64_t out_cap,
                                    uint64_t* out_bytes, isr_stats* st) {
  using namespace isr;
  if (!ctx) return set_error(ISR_EINVAL, "ctx is NULL");
  if (st) *st = isr_stats{};
  const int dev = ctx_device(ctx);
  if (dev < 0 || dev >= MAX_DEV) return set_error(ISR_EINVAL, "device %d beyond the supported %d", dev, MAX_DEV);
  if (hipSetDevice(dev) != hipSuccess) return set_error(ISR_EDEVICE, "hipSetDevice(%d) failed", dev);
  if (!g_ptr[dev]) {
    const int rc = noalloc_init(dev);
    if (rc) return rc;
  }
  std::lock_guard<std::mutex> g(g_mu[dev]);
  return run_compress_noalloc(ctx, f, (char*)g_ptr[dev], (size_t)ISR_NOALLOC_SCRATCH_BYTES, d_out, out_cap, out_bytes,
                              st);
}
