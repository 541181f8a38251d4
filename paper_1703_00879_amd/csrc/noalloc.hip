// The library's own scratch array: the work area of cola_step_static, the step for
// callers that cannot allocate device memory.
//
// The array is a file-scope device variable, so every GPU the library is loaded on holds
// its own copy for the life of the process.  Host code never passes the array's name to a
// kernel (on the host that name is only a stand-in, not a device address): the first call
// on each device looks the device address up with hipGetSymbolAddress, with that device
// current, and keeps it per device.  All calls on one device share the array; the step
// writes every byte it reads from it (the deposit clears its counters with a fill kernel,
// every mesh is written before it is read), so nothing from an earlier call leaks into a
// later one, and calls that overlap on one device race.

#include <mutex>

#include "internal.h"

namespace cola {

static __device__ __align__(256) unsigned char scratch[kStaticWorkBytes];

void* static_work(size_t need) {
  if (need > kStaticWorkBytes)
    throw Error{COLA_E_SIZE, "the run's work area (" + std::to_string(need) +
                                 " bytes) exceeds the library's scratch array (" +
                                 std::to_string(kStaticWorkBytes) + " bytes)"};
  int dev = 0;
  COLA_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error{COLA_E_UNSUPPORTED, "device index out of range"};
  static std::mutex mu;
  static void* ptr[kMaxDevices] = {};
  std::lock_guard<std::mutex> lk(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    COLA_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error{COLA_E_HIP, "hipGetSymbolAddress returned a null address"};
    ptr[dev] = p;
  }
  return ptr[dev];
}

}  // namespace cola
