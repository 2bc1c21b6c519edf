// lopc_static.hip -- the library-held scratch of lopc_decompress_static: a
// file-scope device array (one copy per GPU, alive until the process ends)
// whose device address is looked up once per device when a context is made.
#include <hip/hip_runtime.h>

#include "lopc_host.h"

namespace lopc {

// Params of the call, then one 64-bit record offset per chunk.
__device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

hipError_t static_scratch_address(void** ptr) {
  *ptr = nullptr;
  return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

}  // namespace lopc
