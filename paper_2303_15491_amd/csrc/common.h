// Device helpers shared by the segmentation kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace plmss {

constexpr int kWave = 64;
constexpr int kBlock = 256;       // threads per block in every kernel
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr uint32_t kNumXcd = 8;   // MI355X: 8 accelerator complex dies, 32 CUs each

// Workgroups are dispatched round-robin over the XCDs (block b runs on XCD
// b % 8).  Each XCD has its own L2, so hand every XCD one contiguous range of
// the logical block space instead of every 8th block: neighbouring tiles then
// share an L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nblocks) {
    const uint32_t q = nblocks / kNumXcd, r = nblocks % kNumXcd;
    const uint32_t xcd = b % kNumXcd, k = b / kNumXcd;
    return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + k;
}

// Pointers that reach a kernel inside a descriptor (not as a kernel argument)
// are generic to the compiler, which then emits flat memory instructions; flat
// accesses also count against the LDS wait counter, so every LDS wait would
// wait for them too.  Device data lives in global memory: say so.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}

// Element i of a global array.  With O32 the address is the array's base plus
// a 32-bit byte offset (valid while i * sizeof(T) < 2^32): the base stays in
// scalar registers and each address costs one vector register, not a pair.
template <bool O32, typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gelem(T* base, uint32_t i) {
    if constexpr (O32)
        return (__attribute__((address_space(1))) T*)((__attribute__((address_space(1))) char*)base +
                                                       i * uint32_t(sizeof(T)));
    else
        return gmem(base) + i;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / kWave; }

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (uint64_t(1) << lane_id()) - 1;
}

// Order-preserving integer keys of IEEE values: unsigned comparison of keys is
// the IEEE order, with -0 mapped to +0 so that the two compare equal (ties are
// then decided by vertex id).  NaNs are reported separately.  The keys of all
// non-NaN values lie strictly between 0 and the all-ones pattern.
__device__ __forceinline__ uint32_t sos_key(float f) {
    uint32_t u = __float_as_uint(f);
    u = (u == 0x80000000u) ? 0u : u;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ uint64_t sos_key(double f) {
    uint64_t u = static_cast<uint64_t>(__double_as_longlong(f));
    u = (u == 0x8000000000000000ull) ? 0ull : u;
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
// NaN from the key alone: the transform maps +NaNs above key(+inf) and -NaNs
// below key(-inf), and nothing else lies there.
__device__ __forceinline__ bool key_is_nan(uint32_t k) { return k > 0xFF800000u || k < 0x007FFFFFu; }
__device__ __forceinline__ bool key_is_nan(uint64_t k) {
    return k > 0xFFF0000000000000ull || k < 0x000FFFFFFFFFFFFFull;
}
__device__ __forceinline__ bool is_nan(float f) {
    return (__float_as_uint(f) & 0x7fffffffu) > 0x7f800000u;
}
__device__ __forceinline__ bool is_nan(double f) {
    return (static_cast<uint64_t>(__double_as_longlong(f)) & 0x7fffffffffffffffull) >
           0x7ff0000000000000ull;
}

// Exclusive prefix sum over one block of kBlock threads.  tmp: kWavesPerBlock
// words of LDS.  Returns the thread's exclusive prefix; *total receives the
// block sum.  Must be called by all threads of the block.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t* tmp,
                                                         uint32_t* total) {
    // the thread index is opaque to the compiler here, so that the shuffle
    // addresses derived from it are recomputed at each call instead of being
    // held in registers (or spilled) across a kernel's loop
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = int(tid) & (kWave - 1), w = int(tid) / kWave;
    uint32_t inc = x;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t y = uint32_t(__builtin_amdgcn_ds_bpermute((lane - d) << 2, int(inc)));
        if (lane >= d) inc += y;
    }
    if (lane == kWave - 1) tmp[w] = inc;
    __syncthreads();
    uint32_t base = 0, sum = 0;
#pragma unroll
    for (int i = 0; i < kWavesPerBlock; ++i) {
        uint32_t t = tmp[i];
        base += (i < w) ? t : 0u;
        sum += t;
    }
    __syncthreads();
    *total = sum;
    return base + inc - x;
}

}  // namespace plmss
