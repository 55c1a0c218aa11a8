// Small-set ordering for the top-nprobe and top-k outputs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ivf {

// Ascending order of n keys by rank: key i goes to the slot equal to the
// number of keys below it plus the equal keys before it (all lanes of a wave
// read the same src[j], a broadcast). One pass and one barrier; src and dst
// must not overlap.
__device__ inline void block_rank_sort(const uint64_t* src, uint32_t n, uint64_t* dst) {
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    const uint64_t k = src[i];
    uint32_t r = 0;
    for (uint32_t j = 0; j < n; ++j) {
      const uint64_t o = src[j];
      r += (o < k || (o == k && j < i)) ? 1u : 0u;
    }
    dst[r] = k;
  }
  __syncthreads();
}

}  // namespace ivf
