// Small device helpers shared by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

namespace sbm {

// Blocks are dispatched round-robin over the 8 XCDs; this gives XCD x a
// contiguous range of block indices (so neighbouring cells hit that XCD's L2).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    int x = b & 7, q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// The threads of one cell always sit in one wave, so data exchanged through
// LDS between them needs no block barrier: LDS instructions of a wave complete
// in order, and this only keeps the compiler from moving memory operations
// across the exchange point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace sbm
