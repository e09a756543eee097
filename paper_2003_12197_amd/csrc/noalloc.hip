// noalloc.hip -- hers_search_noalloc: the search with its workspace in a
// static device array, for callers that cannot allocate device memory.
//
// The array lives in this library's code object, so each GPU the library
// runs on holds its own copy (HERS_SCRATCH_BYTES) until the process ends.  In
// host code its name stands for a host-side shadow, not a device address: the
// device address is resolved once per device with hipGetSymbolAddress (the
// context creation calls scratch_setup with the device current) and only that
// pointer is handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/hers.h"
#include "internal.h"

#define HERS_SCRATCH_MAX_DEVICES 64

static __device__ __align__(256) unsigned char scratch[HERS_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[HERS_SCRATCH_MAX_DEVICES] = {};
}  // namespace

int hers::scratch_setup(int device) {
  if (device < 0 || device >= HERS_SCRATCH_MAX_DEVICES) {
    hers::set_last_error("device index beyond the scratch table");
    return HERS_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return HERS_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    hers::set_last_error(std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(e));
    return HERS_EDEVICE;
  }
  g_scratch_ptr[device] = p;
  return HERS_OK;
}

extern "C" int hers_search_noalloc(hers_ctx* ctx, const uint32_t* gallery_dev, uint64_t gallery_words, int64_t m,
                                   int32_t d, const uint32_t* probe_dev, uint64_t probe_words, uint64_t* scores_dev,
                                   void* stream) {
  if (!ctx) {
    hers::set_last_error("null context");
    return HERS_EINVAL;
  }
  const int dev = hers::ctx_device(ctx);
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    ws = dev >= 0 && dev < HERS_SCRATCH_MAX_DEVICES ? g_scratch_ptr[dev] : nullptr;
  }
  if (!ws) {
    hers::set_last_error("the scratch array of this device is not set up");
    return HERS_EDEVICE;
  }
  if (hers::search_ws_block_bytes(ctx) > HERS_SCRATCH_BYTES) {
    hers::set_last_error("one block's search workspace exceeds the scratch array (HERS_SCRATCH_BYTES)");
    return HERS_ESPACE;
  }
  // blocks in chunks of the scratch; every word the kernels read there is
  // written first in the same call, so nothing is cleared
  return hers::search_impl(ctx, gallery_dev, gallery_words, m, d, probe_dev, probe_words, scores_dev, ws,
                           HERS_SCRATCH_BYTES, stream, false);
}
