// fobf_filter_ws_static: the workspace form of the filter with its N/D
// workspace in a library-held device array instead of a caller buffer, for
// callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The array lives in this translation unit's code object: every GPU the
// library runs on holds its own copy, at its own address, from the first
// call on that GPU until the process ends.  Host code never passes the
// array's name to a kernel (on the host that name is only a stand-in for
// the symbol): the address hipGetSymbolAddress returns for the current
// device is what the kernels receive, exactly as they receive a caller's
// workspace pointer.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>

#include "fobf_internal.h"

namespace fobf {
namespace {

constexpr size_t kScratchBytes = FOBF_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::atomic<void*> g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// The device address of this device's copy of `scratch`, looked up once
// per device (with that device current) and kept.
fobf_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(FOBF_EHIP, "fobf_filter_ws_static: no current HIP device");
  void* p = g_scratch[dev].load(std::memory_order_acquire);
  if (!p) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    p = g_scratch[dev].load(std::memory_order_relaxed);
    if (!p) {
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return fail(FOBF_EHIP, std::string("fobf_filter_ws_static: hipGetSymbolAddress: ") +
                                   hipGetErrorString(e));
      g_scratch[dev].store(p, std::memory_order_release);
    }
  }
  *out = p;
  return FOBF_OK;
}

}  // namespace
}  // namespace fobf

using namespace fobf;

extern "C" fobf_status fobf_filter_ws_static(const float* d_in, float* d_out, int H, int W,
                                             int ld_in, int ld_out, double theta, int K, int T,
                                             const double* c, int prec, int algo,
                                             void* hip_stream) {
  fobf_status st = validate_filter(d_in, d_out, H, W, ld_in, ld_out, theta, K, T, c, prec, algo);
  if (st != FOBF_OK) return st;
  if (H == 0 || W == 0) return FOBF_OK;
  size_t need = 0;
  st = fobf_filter_workspace_size(H, W, theta, prec, &need);
  if (st != FOBF_OK) return st;
  if (need > kScratchBytes)
    return fail(FOBF_EINVAL, "fobf_filter_ws_static: the image needs " + std::to_string(need) +
                                 " workspace bytes, above the " +
                                 std::to_string(kScratchBytes) + " of the static scratch");
  // no workspace form for this image: the plain kernels need no scratch
  if (need == 0 || algo == FOBF_ALGO_VALU)
    return fobf_filter(d_in, d_out, H, W, ld_in, ld_out, theta, K, T, c, prec, algo,
                       hip_stream);
  void* ptr = nullptr;
  st = scratch_address(&ptr);
  if (st != FOBF_OK) return st;
  return fobf_filter_ws(d_in, d_out, H, W, ld_in, ld_out, theta, K, T, c, prec, algo, ptr,
                        kScratchBytes, hip_stream);
}
