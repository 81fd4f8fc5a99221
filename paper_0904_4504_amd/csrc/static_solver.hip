// lbm_create_static: a solver whose device memory is the library's own
// static scratch array, for callers that cannot allocate device memory.
//
// The array is a file-scope __device__ variable, one copy per device.  Host
// code never passes the array's name to a kernel or a copy (in host code it
// is a host-side stand-in, not a device address): the first use on a device
// asks the runtime for that device's address of the array
// (hipGetSymbolAddress, with the device current) and keeps it; the solver is
// then created in that memory exactly as lbm_create_in would create it in a
// caller's buffer, so it runs the same kernels on the same layout.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"

namespace {

constexpr uint64_t kScratchBytes = LBM_STATIC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};   // device address of `scratch`, per device
bool g_busy[kMaxDevices] = {};   // a live solver occupies the array

}  // namespace

void lbm::release_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (device >= 0 && device < kMaxDevices) g_busy[device] = false;
}

extern "C" int lbm_create_static(const lbm_params* p, void* hip_stream, lbm_solver** out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  uint64_t need = 0;
  int rc = lbm_required_bytes(p, &need);
  if (rc) return rc;
  if (need > kScratchBytes) return LBM_ESCRATCH;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return LBM_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return LBM_EINVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_busy[dev]) return LBM_ESCRATCH;
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
      (void)hipGetLastError();
      return LBM_EHIP;
    }
    g_ptr[dev] = ptr;
  }
  rc = lbm::create_solver(p, hip_stream, g_ptr[dev], kScratchBytes, false, out);
  if (rc) return rc;
  (*out)->in_scratch = true;
  g_busy[dev] = true;
  return LBM_OK;
}
