// Radix sort of the finest-cell Morton keys (setup step of the point binning).
#include <hipcub/hipcub.hpp>
#include "launch.h"

namespace tsmg {

// Stable LSD radix sort of (key, original index) pairs on bits [0, bits).
// With tmp == nullptr only *tmp_bytes is computed.
hipError_t sort_pairs(uint32_t* key_in, uint32_t* key_out, uint32_t* val_in, uint32_t* val_out, int64_t n,
                      int bits, void* tmp, size_t* tmp_bytes, hipStream_t st) {
  return hipcub::DeviceRadixSort::SortPairs(tmp, *tmp_bytes, key_in, key_out, val_in, val_out, int(n), 0,
                                            bits < 1 ? 1 : bits, st);
}

}  // namespace tsmg
