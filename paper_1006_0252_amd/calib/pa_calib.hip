// Vector-ALU issue rate and engine clock of the device, for the ALU roofline of the sweep.
//
// Each wave runs `iters` iterations of 16 independent dependency chains of one instruction kind
// (written as inline assembly, so the count per iteration is exact), with enough waves per SIMD
// that issue, not latency, limits the rate.  Wave 0 of every block records the shader clock
// counter and the constant-rate wall clock at its start and end, so that the host can turn the
// cycle count of the loop into a clock frequency.  Nothing here touches the library's state.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

enum Kind { kXor = 0, kBitop3 = 1, kMad64 = 2, kPkSub = 3, kPkMin = 4, kMix = 5, kKinds = 6 };

template <int KIND>
__device__ __forceinline__ void body(uint32_t (&a)[16], uint64_t (&w)[8], uint32_t b, uint32_t c)
{
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if constexpr (KIND == kXor) {
            asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a[i]) : "v"(b));
        } else if constexpr (KIND == kBitop3) {
            asm volatile("v_bitop3_b32 %0, %1, %2, %0 bitop3:0x96" : "+v"(a[i]) : "v"(b), "v"(c));
        } else if constexpr (KIND == kMad64) {
            if (i < 8) asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(w[i]) : "v"(b), "v"(c) : "vcc");
            else asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(w[i - 8]) : "v"(c), "v"(b) : "vcc");
        } else if constexpr (KIND == kPkSub) {
            asm volatile("v_pk_sub_u16 %0, %1, %0 clamp" : "+v"(a[i]) : "v"(b));
        } else if constexpr (KIND == kPkMin) {
            asm volatile("v_pk_min_u16 %0, %1, %0" : "+v"(a[i]) : "v"(b));
        } else {
            // the Philox round's pair, alternating: one 64-bit product, one three-input xor
            if (i % 2 == 0) asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(w[i / 2]) : "v"(b), "v"(c) : "vcc");
            else asm volatile("v_bitop3_b32 %0, %1, %2, %0 bitop3:0x96" : "+v"(a[i]) : "v"(b), "v"(c));
        }
    }
}

template <int KIND>
__global__ void __launch_bounds__(256) k_valu(int iters, uint32_t seed, uint64_t* __restrict__ clocks,
                                              uint32_t* __restrict__ sink)
{
    uint32_t a[16];
    uint64_t w[8];
    const uint32_t b = seed * 2654435761u + threadIdx.x, c = b ^ 0x9E3779B9u;
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = b + (uint32_t)i;
#pragma unroll
    for (int i = 0; i < 8; ++i) w[i] = (uint64_t)(c + (uint32_t)i) << 7;
    __syncthreads();
    const uint64_t t0 = clock64(), r0 = wall_clock64();
    for (int it = 0; it < iters; ++it) body<KIND>(a, w, b, c);
    const uint64_t t1 = clock64(), r1 = wall_clock64();
    uint32_t acc = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc ^= a[i];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc ^= (uint32_t)w[i] ^ (uint32_t)(w[i] >> 32);
    sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
    if (threadIdx.x == 0) {
        uint64_t* o = clocks + 4 * (size_t)blockIdx.x;
        o[0] = t0;
        o[1] = t1;
        o[2] = r0;
        o[3] = r1;
    }
}

}  // namespace

extern "C" {

// VALU instructions per wave and loop iteration of each kind
int pa_calib_instructions_per_iteration(int kind) { return (kind >= 0 && kind < kKinds) ? 16 : -1; }

// One timed launch of `kind`: n_blocks blocks of 256 threads, iters iterations each.  clocks_dev
// (device, uint64 [n_blocks][4]) receives (clock start, clock end, wall clock start, wall clock
// end) of wave 0 of each block; sink_dev (device, uint32 [n_blocks * 256]) keeps the chains live.
// Returns 0, 1 for a bad argument, 5 for a launch error.
int pa_calib_valu(int kind, int n_blocks, int iters, uint64_t* clocks_dev, uint32_t* sink_dev, void* stream)
{
    if (kind < 0 || kind >= kKinds || n_blocks <= 0 || iters <= 0 || !clocks_dev || !sink_dev) return 1;
    hipStream_t s = (hipStream_t)stream;
    const dim3 g((unsigned)n_blocks), blk(256);
    switch (kind) {
        case kXor: hipLaunchKernelGGL(k_valu<kXor>, g, blk, 0, s, iters, 1u, clocks_dev, sink_dev); break;
        case kBitop3: hipLaunchKernelGGL(k_valu<kBitop3>, g, blk, 0, s, iters, 2u, clocks_dev, sink_dev); break;
        case kMad64: hipLaunchKernelGGL(k_valu<kMad64>, g, blk, 0, s, iters, 3u, clocks_dev, sink_dev); break;
        case kPkSub: hipLaunchKernelGGL(k_valu<kPkSub>, g, blk, 0, s, iters, 4u, clocks_dev, sink_dev); break;
        case kPkMin: hipLaunchKernelGGL(k_valu<kPkMin>, g, blk, 0, s, iters, 5u, clocks_dev, sink_dev); break;
        default: hipLaunchKernelGGL(k_valu<kMix>, g, blk, 0, s, iters, 6u, clocks_dev, sink_dev); break;
    }
    return hipGetLastError() == hipSuccess ? 0 : 5;
}

// rate of the constant wall clock that wall_clock64() counts, in kHz
int pa_calib_wall_clock_khz(int* khz)
{
    int dev = 0;
    if (!khz || hipGetDevice(&dev) != hipSuccess) return 5;
    return hipDeviceGetAttribute(khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess ? 0 : 5;
}

}  // extern "C"
