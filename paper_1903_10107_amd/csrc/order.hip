// Decode order for persistent schedules: frames whose hard decision violates
// more checks first. Before decoding, Bob's hard decision y^ = [llr < 0] fails
// the check rows i with (H y^)_i != s_i (Sec. 2, the stopping rule applied to
// the channel values); the number of such rows grows with the number of channel
// errors and predicts the iterations a frame needs, so handing the queue's
// frames out in decreasing order of that count starts the long decodes first
// and shortens the batch's tail. The order affects only when a frame is
// decoded, never its result.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "decoder.hpp"
#include "kernels.hpp"

namespace qkdldpc {

namespace {

constexpr int kWeightThreads = 256;
constexpr int kOrderThreads = 1024, kOrderBins = 1024;

// Sign bit j of the frame's channel values, from LDS words (LDS) or read from
// the channel values themselves.
template <bool LDS>
__device__ __forceinline__ unsigned sign_bit(const uint32_t *bits, const int8_t *y, int j)
{
    if constexpr (LDS)
        return (bits[j >> 5] >> (j & 31)) & 1u;
    else
        return y[j] < 0;
}

// out_w[f] = number of check rows i with (H y^)_i != s_i. One workgroup per
// frame; with LDS the hard decision is first packed into words with wavefront
// ballots (64 consecutive positions per ballot).
template <bool LDS>
__global__ __launch_bounds__(kWeightThreads) void k_unsat_weight(DevCode C, const uint8_t *__restrict__ syn,
                                                                 int syn_bytes, const int8_t *__restrict__ llr,
                                                                 int32_t *__restrict__ out_w)
{
    extern __shared__ __align__(16) uint32_t s_bits[];
    __shared__ int s_red[kWeightThreads / 64];
    const int f = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    const int8_t *y = llr + (size_t)f * C.n;
    if constexpr (LDS) {
        const int nwords = (C.n + 31) >> 5;
        for (int j0 = wave * 64; j0 < C.n; j0 += nw * 64) {
            const int j = j0 + lane;
            const unsigned long long m = __ballot(j < C.n && y[j] < 0);
            if (lane == 0) {
                s_bits[j0 >> 5] = (uint32_t)m;
                if ((j0 >> 5) + 1 < nwords)
                    s_bits[(j0 >> 5) + 1] = (uint32_t)(m >> 32);
            }
        }
        __syncthreads();
    }
    const uint8_t *s = syn + (size_t)f * syn_bytes;
    int cnt = 0;
    for (int i = tid; i < C.m; i += blockDim.x) {
        const int b = i / C.z, r = i - b * C.z;
        const int d = ldc(C.deg, b), o = ldc(C.blk_off, b);
        unsigned par = (s[i >> 3] >> (i & 7)) & 1u;
        for (int k = 0; k < d; ++k)
            par ^= sign_bit<LDS>(s_bits, y, ldc(C.colbase, o + k) + rot(r, ldc(C.shift, o + k), C.z));
        cnt += (int)par;
    }
    // fixed-order sum: the lanes of a wave, then the waves
#pragma unroll
    for (int d = 32; d > 0; d >>= 1)
        cnt += __shfl_xor(cnt, d, 64);
    if (lane == 0)
        s_red[wave] = cnt;
    __syncthreads();
    if (tid == 0) {
        int t = 0;
        for (int k = 0; k < nw; ++k)
            t += s_red[k];
        out_w[f] = t;
    }
}

// Bucket sort of the frames by decreasing weight in one workgroup: bucket
// kOrderBins - 1 - min(w >> shift, kOrderBins - 1), counted and placed with LDS
// atomics (the order inside a bucket is whatever the atomics give).
__global__ __launch_bounds__(kOrderThreads) void k_order_desc(const int32_t *__restrict__ w, int n_frames, int shift,
                                                              int32_t *__restrict__ order)
{
    __shared__ int hist[kOrderBins];
    __shared__ int wsum[kOrderThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    hist[tid] = 0;
    __syncthreads();
    auto bucket = [&](int f) {
        const int key = min(max(w[f], 0) >> shift, kOrderBins - 1);
        return kOrderBins - 1 - key;
    };
    for (int f = tid; f < n_frames; f += kOrderThreads)
        atomicAdd(&hist[bucket(f)], 1);
    __syncthreads();
    // exclusive prefix sum of the bucket counts (one bucket per thread)
    const int v = hist[tid];
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d)
            x += y;
    }
    if (lane == 63)
        wsum[wave] = x;
    __syncthreads();
    int before = 0;
    for (int k = 0; k < wave; ++k)
        before += wsum[k];
    __syncthreads();
    hist[tid] = before + x - v;  // first position of bucket tid
    __syncthreads();
    for (int f = tid; f < n_frames; f += kOrderThreads)
        order[atomicAdd(&hist[bucket(f)], 1)] = f;
}

} // namespace

hipError_t launch_order_by_unsat(const DevCode &C, const uint8_t *syn, const int8_t *llr, int n_frames,
                                 int32_t *out_w, int32_t *out_order, hipStream_t s)
{
    int dev = 0, lds_limit = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess)
        return e;
    const int syn_bytes = (C.m + 7) / 8;
    const size_t bit_bytes = (((size_t)C.n + 63) / 64) * 8;  // whole ballots
    if (bit_bytes + 64 <= (size_t)lds_limit) {
        if (bit_bytes > 65536) {
            e = allow_max_lds<k_unsat_weight<true>>();
            if (e != hipSuccess)
                return e;
        }
        hipLaunchKernelGGL(k_unsat_weight<true>, dim3(n_frames), dim3(kWeightThreads), bit_bytes, s, C, syn, syn_bytes,
                           llr, out_w);
    } else {
        hipLaunchKernelGGL(k_unsat_weight<false>, dim3(n_frames), dim3(kWeightThreads), 0, s, C, syn, syn_bytes, llr,
                           out_w);
    }
    e = hipGetLastError();
    if (e != hipSuccess || !out_order)
        return e;
    // buckets of 2^shift weights, so that every weight up to m has a bucket
    int shift = 0;
    while (((long long)C.m >> shift) >= kOrderBins)
        ++shift;
    hipLaunchKernelGGL(k_order_desc, dim3(1), dim3(kOrderThreads), 0, s, out_w, n_frames, shift, out_order);
    return hipGetLastError();
}

} // namespace qkdldpc
