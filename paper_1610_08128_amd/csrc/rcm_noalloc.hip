// The allocation-free entry point (rcm_order_noalloc in rcm.h): an ordering
// whose workspace is a file-scope device array instead of caller memory or
// a library allocation, for callers that cannot allocate device memory.
//
// The array's name in host code is only a host-side stand-in: its device
// address is looked up once per device with hipGetSymbolAddress (with that
// device current) and only that address is handed to the library.  Every
// call on a device shares the device's copy of the array; a per-device
// mutex serialises the calls of this process, and each call initialises
// the parts of the workspace it relies on, so the contents a previous call
// left behind never matter.

#include <mutex>

#include "rcm_common.hpp"

namespace {

constexpr size_t kScratchBytes = RCM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_device_mutex[kMaxDevices];
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

extern "C" rcm_status rcm_order_noalloc(int32_t n, const int32_t* rowptr, const int32_t* colidx,
                                        int32_t* perm_out, int32_t* iperm_out, rcm_stats* stats,
                                        const rcm_options* opts, void* stream) {
  // argument and option errors, and the empty graph, need no device
  const rcm_status st = rcm::check_call(n, opts);
  if (st != RCM_OK || n == 0)
    return rcm::order_single(n, rowptr, colidx, perm_out, iperm_out, stats, opts, nullptr, 0,
                             stream, false);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return RCM_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_device_mutex[dev]);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
      return RCM_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  return rcm::order_single(n, rowptr, colidx, perm_out, iperm_out, stats, opts,
                           g_scratch_ptr[dev], kScratchBytes, stream, false);
}
