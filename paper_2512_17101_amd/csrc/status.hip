// Device-side failure flags and the synchronising status call.
//
// Kernels that can meet a failure they cannot return (a Newton solve that
// does not converge, a non-finite state) OR a bit into one word per device;
// dg_synchronize waits for a stream, reads the word, clears it and turns the
// bits into a status code.  The word is a file-scope device variable: each
// GPU holds its own copy, whose address is looked up once per device.
#include <mutex>
#include <string>

#include "internal.hpp"

namespace {

__device__ unsigned int g_status_flags;

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned* g_addr[kMaxDevices] = {};

}  // namespace

namespace dg {

unsigned* device_flags() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_status_flags)) != hipSuccess) return nullptr;
    g_addr[dev] = static_cast<unsigned*>(p);
  }
  return g_addr[dev];
}

}  // namespace dg

using namespace dg;

extern "C" dg_status dg_synchronize(int device, hipStream_t stream) {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(DG_ERR_ARG, "dg_synchronize: invalid device");
  DeviceGuard g(device);
  if (!g.ok) return fail(DG_ERR_HIP, "dg_synchronize: hipSetDevice failed");
  DG_HIP(hipStreamSynchronize(stream));
  unsigned* f = device_flags();
  if (!f) return fail(DG_ERR_HIP, "dg_synchronize: status word not found");
  unsigned h = 0;
  DG_HIP(hipMemcpy(&h, f, sizeof(h), hipMemcpyDeviceToHost));
  if (h == 0) return DG_OK;
  const unsigned z = 0;
  DG_HIP(hipMemcpy(f, &z, sizeof(z), hipMemcpyHostToDevice));
  if (h & kFlagNonFinite)
    return fail(DG_ERR_NONFINITE, std::string("dg_synchronize: a kernel produced a non-finite value") +
                                      ((h & kFlagNoConv) ? "; a Newton solve did not converge" : ""));
  return fail(DG_ERR_NOCONV, "dg_synchronize: a Newton solve did not converge (iteration count -1)");
}
