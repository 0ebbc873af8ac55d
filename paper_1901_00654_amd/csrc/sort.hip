// Radix sort of the finest-cell keys (setup step of the point binning), by
// rocPRIM's device radix sort: LSD passes over the key bits that can be set,
// the original point index carried along as the value.
#include <rocprim/device/device_radix_sort.hpp>

#include "launch.h"

namespace tsmg {

// Stable sort of (key, original index) pairs on bits [0, bits). With
// tmp == nullptr only *tmp_bytes is computed. key_in and val_in are left as
// they are; the sorted pairs go to key_out, val_out.
hipError_t sort_pairs(uint32_t* key_in, uint32_t* key_out, uint32_t* val_in, uint32_t* val_out, int64_t n,
                      int bits, void* tmp, size_t* tmp_bytes, hipStream_t st) {
  const unsigned end_bit = unsigned(bits < 1 ? 1 : (bits > 32 ? 32 : bits));
  return rocprim::radix_sort_pairs(tmp, *tmp_bytes, key_in, key_out, val_in, val_out, size_t(n), 0u, end_bit, st);
}

}  // namespace tsmg
