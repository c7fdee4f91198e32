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
#include "syndrome_words.hpp"

namespace qkdldpc {

namespace {

constexpr int kWeightThreads = 512;
constexpr int kOrderThreads = 1024, kOrderBins = 1024;
constexpr int kBallotsInFlight = 8;

// Sign bits of the four int8 values of a dword (byte k -> bit k): the top bit
// of each byte moved to bit 0 of its byte, then one multiply collects the four
// bits in the top byte (no carries: every partial sum stays below 16).
__device__ __forceinline__ uint32_t sign_nibble(uint32_t x)
{
    return (((x >> 7) & 0x01010101u) * 0x01020408u) >> 24;
}

// The sign bits of a frame's n channel values (n a multiple of 32, y 16-byte
// aligned) into LDS words, bit j of the frame at bit j & 31 of word j >> 5: 16
// values per lane and load, four loads in flight; the 16 bits of a load come
// from one multiply per dword, and two neighbouring lanes' halves make a word.
__device__ __forceinline__ void stage_signs16(const int8_t *y, int n, uint32_t *bits, int tid, int nthr)
{
    const uint4 *y4 = reinterpret_cast<const uint4 *>(y);
    const int n16 = n >> 4;
    for (int q0 = tid; q0 < n16; q0 += 4 * nthr) {
        uint4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = q0 + u * nthr;
            v[u] = q < n16 ? y4[q] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = q0 + u * nthr;
            const uint32_t h = sign_nibble(v[u].x) | sign_nibble(v[u].y) << 4 | sign_nibble(v[u].z) << 8 |
                               sign_nibble(v[u].w) << 12;
            // q and q ^ 1 are neighbouring lanes (nthr is even), both in range or
            // both not (n16 is even)
            const uint32_t other = (uint32_t)__shfl_xor((int)h, 1, 64);
            if (q < n16 && (q & 1) == 0)
                bits[q >> 1] = h | other << 16;
        }
    }
}

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
// frame. The code's tables go to LDS first (per nonzero block {column start,
// shift}, per base row {first block, degree}), then the frame's syndrome; with
// LDS the hard decision is packed into words with wavefront ballots (64
// consecutive positions per ballot, kBallotsInFlight loads in flight per lane).
// Rows are taken layer by layer, so every lane of a wave uses the same blocks.
template <bool LDS>
__global__ __launch_bounds__(kWeightThreads) void k_unsat_weight(DevCode C, const uint8_t *__restrict__ syn,
                                                                 int syn_bytes, const int8_t *__restrict__ llr,
                                                                 int vec16, int32_t *__restrict__ out_w)
{
    extern __shared__ __align__(16) int2 s_tab[];
    __shared__ int s_red[kWeightThreads / 64];
    int2 *s_rows = s_tab + C.n_blocks;
    uint8_t *s_syn = reinterpret_cast<uint8_t *>(s_rows + C.mb);
    uint32_t *s_bits = reinterpret_cast<uint32_t *>(s_syn + ((syn_bytes + 15) & ~15));
    const int f = blockIdx.x, tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nw = nthr >> 6;
    const int8_t *y = llr + (size_t)f * C.n;
    for (int e = tid; e < C.n_blocks; e += nthr)
        s_tab[e] = make_int2(C.colbase[e], C.shift[e]);
    for (int b = tid; b < C.mb; b += nthr)
        s_rows[b] = make_int2(C.blk_off[b], C.deg[b]);
    const uint8_t *sg = syn + (size_t)f * syn_bytes;
    for (int i = tid; i < syn_bytes; i += nthr)
        s_syn[i] = sg[i];
    if constexpr (LDS) {
        const int nwords = (C.n + 31) >> 5;
        constexpr int U = kBallotsInFlight;
        if (vec16)
            stage_signs16(y, C.n, s_bits, tid, nthr);
        else
        for (int j0 = wave * 64 * U; j0 < C.n; j0 += nw * 64 * U) {
            bool neg[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = j0 + u * 64 + lane;
                neg[u] = j < C.n && y[j] < 0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const unsigned long long m = __ballot(neg[u]);
                const int w0 = (j0 + u * 64) >> 5;
                if (lane == 0 && w0 < nwords) {
                    s_bits[w0] = (uint32_t)m;
                    if (w0 + 1 < nwords)
                        s_bits[w0 + 1] = (uint32_t)(m >> 32);
                }
            }
        }
    }
    __syncthreads();
    int cnt = 0;
    for (int b = 0; b < C.mb; ++b) {
        const int2 row = s_rows[b];
        for (int r = tid; r < C.z; r += nthr) {
            const int i = b * C.z + r;
            unsigned par = (s_syn[i >> 3] >> (i & 7)) & 1u;
#pragma unroll 4
            for (int k = 0; k < row.y; ++k) {
                const int2 cs = s_tab[row.x + k];
                par ^= sign_bit<LDS>(s_bits, y, cs.x + rot(r, cs.y, C.z));
            }
            cnt += (int)par;
        }
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

// The same count for Z a multiple of 32, word-parallel: 32 rows of a layer at a
// time, each block one funnel shift of the packed signs (the syndrome
// encoder's form), XOR the syndrome word, then a population count.
__global__ __launch_bounds__(kWeightThreads) void k_unsat_weight_words(DevCode C, const uint32_t *__restrict__ syn,
                                                                       const int8_t *__restrict__ llr,
                                                                       int32_t *__restrict__ out_w)
{
    extern __shared__ __align__(16) int2 s_tab[];
    __shared__ int s_red[kWeightThreads / 64];
    int2 *s_rows = s_tab + C.n_blocks;
    uint32_t *s_bits = reinterpret_cast<uint32_t *>(s_rows + C.mb);
    const int f = blockIdx.x, tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nw = nthr >> 6;
    const int wz = C.z >> 5, sw = C.m >> 5;
    stage_syndrome_tables(C, s_tab, s_rows, tid, nthr);
    stage_signs16(llr + (size_t)f * C.n, C.n, s_bits, tid, nthr);
    __syncthreads();
    const uint32_t *sf = syn + (size_t)f * sw;
    int cnt = 0;
    for (int w = tid; w < sw; w += nthr)
        cnt += __popc(syndrome_word(s_tab, s_rows, wz, s_bits, w) ^ sf[w]);
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

namespace {

// The per-frame counts: word-parallel when Z is a multiple of 32 (and the
// buffers allow word loads), else one lane per row with the signs in LDS words
// (or read from the channel values when those words do not fit in LDS).
hipError_t launch_unsat(const DevCode &C, const uint8_t *syn, const int8_t *llr, int n_frames, int32_t *out_w,
                        int lds_limit, hipStream_t s)
{
    const size_t word_lds = ((size_t)C.n_blocks + C.mb) * sizeof(int2) + (size_t)C.n / 8;
    if (C.z % 32 == 0 && reinterpret_cast<uintptr_t>(llr) % 16 == 0 && reinterpret_cast<uintptr_t>(syn) % 4 == 0 &&
        word_lds <= (size_t)lds_limit) {
        if (word_lds > 65536) {
            hipError_t e = allow_max_lds<k_unsat_weight_words>();
            if (e != hipSuccess)
                return e;
        }
        hipLaunchKernelGGL(k_unsat_weight_words, dim3(n_frames), dim3(kWeightThreads), word_lds, s, C,
                           reinterpret_cast<const uint32_t *>(syn), llr, out_w);
        return hipGetLastError();
    }
    // tables, then the packed syndrome (16-byte padded), then the sign bits
    const int syn_bytes = (C.m + 7) / 8;
    const size_t tab_bytes = ((size_t)C.n_blocks + C.mb) * sizeof(int2) + (((size_t)syn_bytes + 15) & ~(size_t)15);
    const size_t bit_bytes = (((size_t)C.n + 31) / 32) * 4;
    if (tab_bytes + bit_bytes + 64 <= (size_t)lds_limit) {
        if (tab_bytes + bit_bytes > 65536) {
            hipError_t e = allow_max_lds<k_unsat_weight<true>>();
            if (e != hipSuccess)
                return e;
        }
        // 16-byte loads when every frame's channel values start at a 16-byte boundary
        const int vec16 = C.n % 32 == 0 && reinterpret_cast<uintptr_t>(llr) % 16 == 0;
        hipLaunchKernelGGL(k_unsat_weight<true>, dim3(n_frames), dim3(kWeightThreads), tab_bytes + bit_bytes, s, C,
                           syn, syn_bytes, llr, vec16, out_w);
    } else {
        if (tab_bytes > 65536) {
            hipError_t e = allow_max_lds<k_unsat_weight<false>>();
            if (e != hipSuccess)
                return e;
        }
        hipLaunchKernelGGL(k_unsat_weight<false>, dim3(n_frames), dim3(kWeightThreads), tab_bytes, s, C, syn,
                           syn_bytes, llr, 0, out_w);
    }
    return hipGetLastError();
}

} // namespace

hipError_t launch_order_by_unsat(const DevCode &C, const uint8_t *syn, const int8_t *llr, int n_frames,
                                 int32_t *out_w, int32_t *out_order, hipStream_t s)
{
    int dev = 0, lds_limit = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e == hipSuccess)
        e = launch_unsat(C, syn, llr, n_frames, out_w, lds_limit, s);
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
