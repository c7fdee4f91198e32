// LDS read-bandwidth probe: the measured peak that the decoder's LDS traffic is
// compared against. Every workgroup fills 64 KB of LDS, then each lane reads
// it in a rotating pattern (consecutive lanes hit consecutive addresses, so the
// reads are free of bank conflicts) and folds the values into a register that
// is written out at the end, so no read can be dropped.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "decoder.hpp"

namespace qkdldpc {

namespace {

constexpr int kProbeWords = 4096;  // 64 KB of uint4

// MODE 0: 16-byte reads (ds_read_b128); MODE 1: byte reads (ds_read_u8), the
// width of the decoder's soft-value and message accesses.
template <int MODE>
__global__ __launch_bounds__(1024) void k_probe_lds(int reps, uint32_t *out)
{
    __shared__ uint4 buf[kProbeWords];
    const int tid = threadIdx.x;
    for (int i = tid; i < kProbeWords; i += blockDim.x)
        buf[i] = uint4{(unsigned)i, (unsigned)i * 3u, (unsigned)i * 5u, (unsigned)i * 7u};
    __syncthreads();
    uint32_t acc = 0;
    // eight reads per step, one per 8 KB eighth of the buffer, at a rotating
    // position inside it (constant offsets between the eight)
    if constexpr (MODE == 0) {
        for (int r = 0; r < reps; ++r) {
            const uint4 *p = buf + ((tid + r) & 511);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const uint4 v = p[512 * k];
                // three-input XORs (truth table 0x96) keep the VALU work below the reads
                acc = __builtin_amdgcn_bitop3_b32(acc, v.x, v.y, 0x96);
                acc = __builtin_amdgcn_bitop3_b32(acc, v.z, v.w, 0x96);
            }
        }
    } else {
        const uint8_t *b8 = reinterpret_cast<const uint8_t *>(buf);
        for (int r = 0; r < reps; ++r) {
            const uint8_t *p = b8 + ((tid + r) & 8191);
#pragma unroll
            for (int k = 0; k < 8; ++k)
                acc += p[8192 * k];
        }
    }
    out[(size_t)blockIdx.x * blockDim.x + tid] = acc;
}

} // namespace

hipError_t launch_probe_lds(int mode, int n_workgroups, int reps, uint32_t *out, hipStream_t s)
{
    if (mode == 0)
        hipLaunchKernelGGL(k_probe_lds<0>, dim3(n_workgroups), dim3(1024), 0, s, reps, out);
    else
        hipLaunchKernelGGL(k_probe_lds<1>, dim3(n_workgroups), dim3(1024), 0, s, reps, out);
    return hipGetLastError();
}

} // namespace qkdldpc
