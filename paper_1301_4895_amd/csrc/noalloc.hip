// mb_make_blocks_noalloc: the blocks call for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).  The site-chunk partial sums that
// mb_make_blocks keeps in the caller's workspace live here in a file-scope
// device array of fixed size, one per GPU for the life of the process.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace {

// Every byte of the partial sums is written by the site-sum kernel before the
// finish kernel reads it, so nothing here needs to start at zero.
__device__ __align__(256) unsigned char scratch[MB_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mutex;
void *g_scratch[MAX_DEVICES] = {};   // device address of `scratch`, per device

// The device address of this device's copy of `scratch` (looked up once per
// device, with that device current).  The host-side name of the array is not
// a device address and is never passed to a kernel or a copy.
int scratch_of_current_device(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return mb::fail(MB_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= MAX_DEVICES) return mb::fail(MB_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return mb::fail(MB_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return MB_OK;
}

}  // namespace

extern "C" int mb_make_blocks_noalloc(const mb_term_list *tl, const mb_problem *p, void *blocks,
                                      size_t blocks_bytes, void *stream) {
  int rc = mb::check_blocks_problem(tl, p);
  if (rc) return rc;
  const size_t need = mb::blocks_workspace_bytes(tl, p);
  if (need > size_t(MB_NOALLOC_SCRATCH_BYTES))
    return mb::fail(MB_ENOWORKSPACE, "mb_make_blocks_noalloc: the site-chunk partial sums of this problem need " +
                                         std::to_string(need) + " bytes, above the fixed scratch of " +
                                         std::to_string(size_t(MB_NOALLOC_SCRATCH_BYTES)) +
                                         " bytes (use mb_make_blocks with a workspace, or fewer lanes)");
  void *ws = nullptr;
  if ((rc = scratch_of_current_device(&ws))) return rc;
  return mb::make_blocks_with(tl, p, blocks, blocks_bytes, ws, size_t(MB_NOALLOC_SCRATCH_BYTES), stream);
}
