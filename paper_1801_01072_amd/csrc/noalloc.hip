// noalloc.hip -- the fixed device scratch behind ent_entropy_estimate_noalloc:
// a file-scope device array that holds the estimate's workspace, so that the
// call needs no device allocation.  Each GPU the library runs on has its own
// copy of the array (allocated with the code object, held until the process
// ends); host code reaches it only through the address hipGetSymbolAddress
// returns for the current device, never through the array's name.
#include <map>
#include <mutex>

#include "kernels.hpp"

namespace ent {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

struct ScratchSlot {
  std::mutex use;       // held for the whole of one call on this device
  void *ptr = nullptr;  // this device's copy of the array
};

std::mutex g_slots_mu;
std::map<int, ScratchSlot *> g_slots;

}  // namespace

hipError_t noalloc_scratch(int dev, void **ptr, std::mutex **use) {
  ScratchSlot *slot = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_slots_mu);
    auto it = g_slots.find(dev);
    if (it == g_slots.end()) {
      // first call on this device (which is current): look the address up once
      void *p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || p == nullptr) return e != hipSuccess ? e : hipErrorInvalidSymbol;
      slot = new ScratchSlot();
      slot->ptr = p;
      g_slots[dev] = slot;
    } else {
      slot = it->second;
    }
  }
  *ptr = slot->ptr;
  *use = &slot->use;
  return hipSuccess;
}

}  // namespace ent
