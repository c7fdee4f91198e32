// Device helpers shared by the gfx950 decode kernels (arXiv:1903.10107, Secs. 2-3).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "decoder.hpp"
#include "rcbp.hpp"

namespace qkdldpc {

template <typename ET>
struct AccLim;
template <>
struct AccLim<int8_t> {
    static constexpr int value = 127;
};
template <>
struct AccLim<int16_t> {
    static constexpr int value = 32767;
};

// Read-only table entry through the constant address space, so that uniform
// indices become scalar loads (the kernels never write the code tables).
template <typename T>
__device__ __forceinline__ T ldc(const T *p, int i)
{
    return ((const __attribute__((address_space(4))) T *)p)[i];
}

// (r + s) mod Z for r, s in [0, Z)
__device__ __forceinline__ int rot(int r, int s, int z)
{
    const unsigned t = (unsigned)(r + s);
    const unsigned u = t - (unsigned)z;
    return (int)(t < u ? t : u);
}

// Stage the frame's LLRs into E, clamped to [-lim, lim] (lim = min(E_max, 127)).
// With int8 E, lim = 127 and 16-byte aligned rows, 16 bytes move per lane and
// the only value to fix, -128, is found with an exact packed-byte zero test.
// Sixteen int8 LLRs with every -128 replaced by -127.
__device__ __forceinline__ uint4 llr_no_m128(uint4 v)
{
    unsigned *w = reinterpret_cast<unsigned *>(&v);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const unsigned x = w[k] ^ 0x80808080u;  // bytes equal to 0x80 become 0
        // exact per-byte zero test (no carry crosses a byte): 0x80 where x's byte is 0
        const unsigned z = ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u;
        w[k] += z >> 7;  // 0x80 (-128) -> 0x81 (-127)
    }
    return v;
}

// Hard decisions [E_j < 0] of four int8 soft values (byte k of x is E_{4i+k})
// as the low four bits, LSB first: the sign bits, moved to bits 0, 8, 16, 24,
// are gathered into bits 24..27 by one multiplication (no carries: the partial
// products occupy distinct bits).
__device__ __forceinline__ unsigned sign_nibble(unsigned x)
{
    return (((x >> 7) & 0x01010101u) * 0x01020408u) >> 24;
}

template <typename ET>
__device__ __forceinline__ void stage_llr(ET *E, const int8_t *__restrict__ llr, int n, int lim, int tid, int nthr)
{
    if constexpr (sizeof(ET) == 1) {
        if (lim == 127 && (n & 15) == 0 && (((uintptr_t)llr) & 15) == 0) {
            const uint4 *src = reinterpret_cast<const uint4 *>(llr);
            uint4 *dst = reinterpret_cast<uint4 *>(E);
            for (int q = tid; q < (n >> 4); q += nthr)
                dst[q] = llr_no_m128(src[q]);
            return;
        }
    }
    for (int j = tid; j < n; j += nthr)
        E[j] = (ET)clampi(llr[j], -lim, lim);
}

template <typename ET>
__device__ __forceinline__ s16x2 load_pair(const ET *__restrict__ p, int a0, int a1)
{
    s16x2 v;
    v.x = (short)p[a0];
    v.y = (short)p[a1];
    return v;
}

__device__ __forceinline__ u16x2 as_u(s16x2 v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ s16x2 as_s(u16x2 v) { return __builtin_bit_cast(s16x2, v); }

// packed syndrome bits of rows i and i + Z/2, as sign bits of the halves
__device__ __forceinline__ s16x2 syn_pair(const uint8_t *__restrict__ s_syn, int i0, int i1)
{
    s16x2 s;
    s.x = (short)-(int)((s_syn[i0 >> 3] >> (i0 & 7)) & 1);
    s.y = (short)-(int)((s_syn[i1 >> 3] >> (i1 & 7)) & 1);
    return s;
}

// Workgroup-wide OR of pred. Two flag words alternate between successive votes:
// a vote writes flags[ph] (every writer stores 1), waits at the barrier, reads
// it, and thread 0 clears the other word, whose last readers all passed this
// barrier and whose next writers come after at least one more barrier.
__device__ __forceinline__ int block_any(int pred, int *flags, int ph)
{
    if (pred)
        flags[ph] = 1;
    __syncthreads();
    const int any = flags[ph];
    if (threadIdx.x == 0)
        flags[ph ^ 1] = 0;
    return any;
}

// Allow a kernel the device's largest dynamic LDS, once per kernel instance and
// process (not a stream operation, so decode launches can be graph-captured).
template <auto KERN>
inline hipError_t allow_max_lds()
{
    static const hipError_t once = []() {
        int dev = 0, lim = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        // static LDS of the kernel (e.g. block reductions) counts against the same limit
        hipFuncAttributes fa{};
        if (e == hipSuccess)
            e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(KERN));
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(KERN), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    lim - (int)fa.sharedSizeBytes);
        return e;
    }();
    return once;
}

} // namespace qkdldpc
