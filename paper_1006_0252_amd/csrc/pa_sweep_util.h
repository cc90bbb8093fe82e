// Device helpers shared by the sweep kernels.
#pragma once

#include "pa_common.h"

namespace pa {

// ---------------------------------------------------------------- small helpers
// LDS writes of one wave made visible to its other lanes (each wave owns its LDS rows, so no
// block barrier is needed once the block-shared tables are built)
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t field16(const uint4v& v, int f)
{
    const uint32_t w = (f >> 1) == 0 ? v.x : ((f >> 1) == 1 ? v.y : ((f >> 1) == 2 ? v.z : v.w));
    return (f & 1) ? (w >> 16) : (w & 0xFFFFu);
}

// full 64-bit acceptance test on a first-look tie: U = (u16 << 48) | u48 < T64
static __device__ __noinline__ bool tie_accept(uint32_t u16, uint64_t T64, uint32_t site, uint32_t r, uint32_t ctr2,
                                        uint32_t k0, uint32_t k1)
{
    const uint4v v = philox10(site, r, ctr2, kTagTie, k0, k1);
    const uint64_t U = ((uint64_t)u16 << 48) | (uint64_t)v.x | ((uint64_t)(v.y & 0xFFFFu) << 32);
    return U < T64;
}

// pack 4 bytes of 0/1 into 4 bits (byte k -> bit k)
__device__ __forceinline__ uint32_t pack4(uint32_t d) { return ((d & 0x01010101u) * 0x01020408u) >> 24; }
// unpack 4 bits into 4 bytes of 0/1
__device__ __forceinline__ uint32_t unpack4(uint32_t b) { return ((b & 0xFu) * 0x00204081u) & 0x01010101u; }

}  // namespace pa
