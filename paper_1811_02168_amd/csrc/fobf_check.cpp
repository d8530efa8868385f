// Violation word of the debug-check build (FOBF_CHECKS=1): one device word
// per GPU that the kernels OR their violation bits into (FOBF_CHECK_* in
// fobf.h), and fobf_check_take, which reads and clears it.  The release
// build has no word: its kernels carry a null pointer and never look at it.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>

#include "fobf_internal.h"

#ifndef FOBF_CHECKS
#define FOBF_CHECKS 0
#endif

namespace fobf {
namespace {
constexpr int kMaxDevices = 64;
std::atomic<unsigned int*> g_word[kMaxDevices];
std::mutex g_word_mu;
}  // namespace

unsigned int* check_word() {
#if FOBF_CHECKS
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  unsigned int* w = g_word[dev].load(std::memory_order_acquire);
  if (!w) {
    std::lock_guard<std::mutex> lk(g_word_mu);
    w = g_word[dev].load(std::memory_order_relaxed);
    if (!w) {
      void* p = nullptr;
      if (hipMalloc(&p, 256) != hipSuccess) return nullptr;
      if (hipMemset(p, 0, 256) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(p);
        return nullptr;
      }
      w = static_cast<unsigned int*>(p);
      g_word[dev].store(w, std::memory_order_release);
    }
  }
  return w;
#else
  return nullptr;
#endif
}

}  // namespace fobf

using namespace fobf;

extern "C" fobf_status fobf_check_take(unsigned int* bits) {
  if (!bits) return fail(FOBF_EINVAL, "fobf_check_take: bits is NULL");
#if FOBF_CHECKS
  unsigned int* w = check_word();
  if (!w) return fail(FOBF_EHIP, "fobf_check_take: no violation word on this device");
  if (hipDeviceSynchronize() != hipSuccess)
    return fail(FOBF_EHIP, "fobf_check_take: hipDeviceSynchronize failed");
  unsigned int v = 0;
  if (hipMemcpy(&v, w, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemset(w, 0, sizeof(v)) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
    return fail(FOBF_EHIP, "fobf_check_take: reading the violation word failed");
  *bits = v;
  return FOBF_OK;
#else
  *bits = 0;
  return fail(FOBF_EINVAL, "fobf_check_take: this library was built without FOBF_CHECKS");
#endif
}
