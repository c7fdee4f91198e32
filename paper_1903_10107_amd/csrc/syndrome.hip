// Alice's side of the syndrome exchange (s = H x) and small utility kernels.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "kernels.hpp"
#include "syndrome_words.hpp"

namespace qkdldpc {

// Alice's side: s = H x for packed x, one thread per check row, packed with a ballot.
__global__ __launch_bounds__(256) void k_syndrome(DevCode C, const uint8_t *__restrict__ bits, int bit_bytes,
                                                  uint8_t *__restrict__ out_syn, int syn_bytes)
{
    const int f = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int par = 0;
    if (i < C.m) {
        const int b = i / C.z, r = i - b * C.z;
        const int d = ldc(C.deg, b), o = ldc(C.blk_off, b);
        const uint8_t *x = bits + (size_t)f * bit_bytes;
        for (int k = 0; k < d; ++k) {
            const int j = ldc(C.colbase, o + k) + rot(r, ldc(C.shift, o + k), C.z);
            par ^= (x[j >> 3] >> (j & 7)) & 1;
        }
    }
    const unsigned long long mask = __ballot(par);
    const int lane = threadIdx.x & 63;
    const int w0 = i - lane;  // first row of this wave, a multiple of 64
    if (lane < 8) {
        const int byte = (w0 >> 3) + lane;
        if (byte < syn_bytes)
            out_syn[(size_t)f * syn_bytes + byte] = (uint8_t)(mask >> (8 * lane));
    }
}

// The same with the frame's packed bits staged in LDS first (one workgroup of
// 1024 threads per frame; every check row then reads its d bits from LDS), for
// batches of many frames whose packed frame (n / 8 bytes) fits in LDS.
__global__ __launch_bounds__(1024) void k_syndrome_lds(DevCode C, const uint8_t *__restrict__ bits, int bit_bytes,
                                                       uint8_t *__restrict__ out_syn, int syn_bytes)
{
    extern __shared__ __align__(16) uint8_t s_x[];
    const int f = blockIdx.x, tid = threadIdx.x, nthr = blockDim.x;
    const uint8_t *x = bits + (size_t)f * bit_bytes;
    for (int i = tid; i < bit_bytes; i += nthr)
        s_x[i] = x[i];
    __syncthreads();
    const int lane = tid & 63;
    // rows in whole waves, so that every ballot covers 64 consecutive rows
    for (int i0 = tid - lane; i0 < C.m; i0 += nthr) {
        const int i = i0 + lane;
        int par = 0;
        if (i < C.m) {
            const int b = i / C.z, r = i - b * C.z;
            const int d = ldc(C.deg, b), o = ldc(C.blk_off, b);
            for (int k = 0; k < d; ++k) {
                const int j = ldc(C.colbase, o + k) + rot(r, ldc(C.shift, o + k), C.z);
                par ^= (s_x[j >> 3] >> (j & 7)) & 1;
            }
        }
        const unsigned long long mask = __ballot(par);
        if (lane < 8) {
            const int byte = (i0 >> 3) + lane;
            if (byte < syn_bytes)
                out_syn[(size_t)f * syn_bytes + byte] = (uint8_t)(mask >> (8 * lane));
        }
    }
}

// One thread per (frame, syndrome word), grid-stride; x is read through the
// caches (each word of x serves about six alignbits), the code's tables from LDS.
__global__ __launch_bounds__(256) void k_syndrome_words(DevCode C, const uint32_t *__restrict__ bits, int n_frames,
                                                        uint32_t *__restrict__ out_syn)
{
    extern __shared__ __align__(16) int2 s_tab[];
    int2 *s_rows = s_tab + C.n_blocks;
    const int wz = C.z >> 5, xw = C.n >> 5, sw = C.m >> 5;
    stage_syndrome_tables(C, s_tab, s_rows, threadIdx.x, blockDim.x);
    __syncthreads();
    const long long total = (long long)n_frames * sw;
    for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (long long)gridDim.x * blockDim.x) {
        const int f = (int)(g / sw), w = (int)(g - (long long)f * sw);
        out_syn[g] = syndrome_word(s_tab, s_rows, wz, bits + (size_t)f * xw, w);
    }
}

// kSynFpw frames per workgroup, their packed bits staged in LDS with every
// column block written twice in a row (2 Z/32 words), so that the two words an
// entry funnel-shifts, (k + s/32) and (k + s/32 + 1), never wrap: an entry costs
// one add, one paired LDS read, one alignbit and one XOR. x is read from memory
// once, in 16-byte loads when the frames are 16-byte aligned and Z/32 is a
// multiple of 4, every load of a thread issued before its stores. Threads map
// to (frame, block row, word) pairs with no per-word division.
// Dynamic LDS: int2 {doubled-block word index + s/32, s mod 32} per nonzero
// block, int2 {first block, degree} per base row, then (16-byte aligned at
// x_off) the frames.
constexpr int kSynFpw = 4;

// i / d for 0 <= i < 2^22 and d >= 1, from rd = 1/d in float: the product is
// within 1 of i / d there, and one step each way corrects it
__device__ __forceinline__ int div_small(int i, int d, float rd)
{
    int q = (int)((float)i * rd);
    q -= q * d > i;
    q += (q + 1) * d <= i;
    return q;
}

__global__ __launch_bounds__(256) void k_syndrome_words_lds(DevCode C, const uint32_t *__restrict__ bits, int n_frames,
                                                           int x_off, uint32_t *__restrict__ out_syn)
{
    extern __shared__ __align__(16) int2 s_tab[];
    int2 *s_rows = s_tab + C.n_blocks;
    uint32_t *s_x = reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(s_tab) + x_off);
    const int wz = C.z >> 5, xw = C.n >> 5, sw = C.m >> 5, mb = C.mb;
    const int f0 = blockIdx.x * kSynFpw, tid = threadIdx.x, nthr = blockDim.x;
    const int nf = n_frames - f0 < kSynFpw ? n_frames - f0 : kSynFpw;
    const uint32_t *x = bits + (size_t)f0 * xw;
    for (int e = tid; e < C.n_blocks; e += nthr) {
        const int sh = C.shift[e];
        s_tab[e] = make_int2(2 * (C.colbase[e] >> 5) + (sh >> 5), sh & 31);
    }
    for (int r = tid; r < mb; r += nthr)
        s_rows[r] = make_int2(C.blk_off[r], C.deg[r]);
    // frame word i = c wz + k goes to 2 c wz + k and 2 c wz + wz + k; loads and
    // stores are unconditional (an index past the end takes the last word,
    // which is then stored again with its own value), so no load waits behind
    // a branch
    constexpr int U = 4;
    auto stage = [&](const auto *src, auto *dst, int total, int bw) {  // bw: block width in elements
        const float rbw = 1.0f / (float)bw;
        std::remove_const_t<std::remove_pointer_t<decltype(src)>> v[U];
        for (int i0 = tid; i0 < total; i0 += U * nthr) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                v[u] = src[i0 + u * nthr < total ? i0 + u * nthr : total - 1];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * nthr < total ? i0 + u * nthr : total - 1;
                const int c = div_small(i, bw, rbw), d = i + c * bw;  // 2 c bw + (i - c bw)
                dst[d] = v[u];
                dst[d + bw] = v[u];
            }
        }
    };
    if (((uintptr_t)x & 15) == 0 && (wz & 3) == 0)
        stage(reinterpret_cast<const uint4 *>(x), reinterpret_cast<uint4 *>(s_x), nf * (xw >> 2), wz >> 2);
    else
        stage(x, s_x, nf * xw, wz);
    __syncthreads();
    // kl lanes take the words of one (frame, block row) pair, the workgroup
    // slots / pairs at a time
    const int kl = wz < nthr ? wz : nthr, slots = nthr / kl;
    const int slot = tid / kl, k0 = tid - slot * kl;
    if (slot >= slots)
        return;
    int j = slot / mb, b = slot - j * mb;  // pair p = j mb + b, advanced by slots
    for (int p = slot; p < nf * mb; p += slots) {
        const int2 r = s_rows[b];
        const uint32_t *xj = s_x + (size_t)j * 2 * xw;
        for (int k = k0; k < wz; k += kl) {
            uint32_t acc = 0;
#pragma unroll 4
            for (int e = r.x; e < r.x + r.y; ++e) {
                const int2 t = s_tab[e];
                const uint32_t *q = xj + t.x + k;
                acc ^= __builtin_amdgcn_alignbit(q[1], q[0], (uint32_t)t.y);
            }
            out_syn[(size_t)(f0 + j) * sw + b * wz + k] = acc;
        }
        for (b += slots; b >= mb; b -= mb)
            ++j;
    }
}

// The same words with the frames grouped by XCD: the hardware hands workgroup
// p to XCD p mod 8, so workgroup p takes frame (p mod 8) + 8 j, where j counts
// that XCD's frames, and the j-th frame's words are split over bpf workgroups.
// Every workgroup of a frame then runs on one XCD and the three block rows that
// read each word of x find it in that XCD's L2 after the first, instead of
// every XCD fetching the frame from memory.
__global__ __launch_bounds__(256) void k_syndrome_words_xcd(DevCode C, const uint32_t *__restrict__ bits,
                                                            int n_frames, int bpf, uint32_t *__restrict__ out_syn)
{
    extern __shared__ __align__(16) int2 s_tab[];
    int2 *s_rows = s_tab + C.n_blocks;
    const int wz = C.z >> 5, xw = C.n >> 5, sw = C.m >> 5;
    const int p = blockIdx.x, slot = p >> 3;
    const int f = (p & 7) + 8 * (slot / bpf);
    const int w = (slot % bpf) * blockDim.x + threadIdx.x;
    if (f >= n_frames)
        return;  // the whole workgroup: f is uniform
    stage_syndrome_tables(C, s_tab, s_rows, threadIdx.x, blockDim.x);
    __syncthreads();
    if (w < sw)
        out_syn[(size_t)f * sw + w] = syndrome_word(s_tab, s_rows, wz, bits + (size_t)f * xw, w);
}

hipError_t launch_syndrome(const DevCode &C, const uint8_t *bits, int n_frames, uint8_t *out_syn, hipStream_t s)
{
    const int bit_bytes = (C.n + 7) / 8, syn_bytes = (C.m + 7) / 8;
    int dev = 0, lds_limit = 0;
    hipError_t e0 = hipGetDevice(&dev);
    if (e0 == hipSuccess)
        e0 = hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e0 != hipSuccess)
        return e0;
    // Z a multiple of 32 makes every block, frame row and syndrome row whole
    // 32-bit words; the word kernels also need 4-byte aligned buffers
    if (C.z % 32 == 0 && ((uintptr_t)bits | (uintptr_t)out_syn) % 4 == 0) {
        const uint32_t *xw = reinterpret_cast<const uint32_t *>(bits);
        uint32_t *sw = reinterpret_cast<uint32_t *>(out_syn);
        const int words = C.m >> 5;
        const size_t tab_bytes = ((size_t)C.n_blocks + C.mb) * sizeof(int2);
        if (tab_bytes <= (size_t)lds_limit) {
            if (tab_bytes > 65536) {
                hipError_t e = allow_max_lds<k_syndrome_words>();
                if (e != hipSuccess)
                    return e;
            }
            const long long total = (long long)n_frames * words;
            const long long bpf = (words + 255) / 256;
            const long long xcd_blocks = 8 * ((n_frames + 7) / 8) * bpf;
            // grouped by XCD for frames of at least 8 workgroups (m >= 2^16): there a
            // frame's words are read by many workgroups and the L2 reuse pays; small
            // frames keep the plain order, which measured faster for n = 32768
            if (n_frames >= 8 && bpf >= 8 && xcd_blocks < (1ll << 31)) {
                if (tab_bytes > 65536) {
                    hipError_t e = allow_max_lds<k_syndrome_words_xcd>();
                    if (e != hipSuccess)
                        return e;
                }
                hipLaunchKernelGGL(k_syndrome_words_xcd, dim3((unsigned)xcd_blocks), dim3(256), tab_bytes, s, C, xw,
                                   n_frames, (int)bpf, sw);
                return hipGetLastError();
            }
            // a workgroup per frame with the frame in LDS, where the batch fills
            // the chip and a frame has at least a wave of syndrome words
            const size_t x_off = (tab_bytes + 15) & ~(size_t)15;
            const size_t lds_bytes = x_off + (size_t)kSynFpw * (C.n >> 5) * 8;  // every block twice
            if (n_frames >= 256 * kSynFpw && words >= 64 && lds_bytes <= (size_t)lds_limit) {
                if (lds_bytes > 65536) {
                    hipError_t e = allow_max_lds<k_syndrome_words_lds>();
                    if (e != hipSuccess)
                        return e;
                }
                hipLaunchKernelGGL(k_syndrome_words_lds, dim3((unsigned)((n_frames + kSynFpw - 1) / kSynFpw)),
                                   dim3(256), lds_bytes, s, C, xw, n_frames, (int)x_off, sw);
                return hipGetLastError();
            }
            const long long blocks = (total + 255) / 256;
            hipLaunchKernelGGL(k_syndrome_words, dim3((unsigned)(blocks < (1 << 20) ? blocks : (1 << 20))),
                               dim3(256), tab_bytes, s, C, xw, n_frames, sw);
            return hipGetLastError();
        }
    }
    // one workgroup per frame fills the chip only with many frames; a few long
    // frames go row-parallel instead
    if (bit_bytes <= lds_limit && n_frames >= 128) {
        if (bit_bytes > 65536) {
            hipError_t e = allow_max_lds<k_syndrome_lds>();
            if (e != hipSuccess)
                return e;
        }
        hipLaunchKernelGGL(k_syndrome_lds, dim3(n_frames), dim3(1024), bit_bytes, s, C, bits, bit_bytes, out_syn,
                           syn_bytes);
        return hipGetLastError();
    }
    const int threads = 256;
    dim3 grid((C.m + threads - 1) / threads, n_frames);
    hipLaunchKernelGGL(k_syndrome, grid, dim3(threads), 0, s, C, bits, bit_bytes, out_syn, syn_bytes);
    return hipGetLastError();
}

// Interactive rate adaptation (Sec. 4.1): Alice reveals the values of some
// positions of listed frames; Bob's LLRs there become the shortened value,
// +-127 with the sign of the revealed bit. Positions outside [0, n) and frame
// ids outside [0, n_frames) are skipped.
__global__ __launch_bounds__(256) void k_reveal(int8_t *__restrict__ llr, int n, int n_frames,
                                                const int32_t *__restrict__ frame_ids, int k,
                                                const int32_t *__restrict__ positions,
                                                const uint8_t *__restrict__ values, int r)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long long)k * r)
        return;
    const int i = (int)(q / r);
    const int f = frame_ids[i];
    const int j = positions[q];
    if ((unsigned)f < (unsigned)n_frames && (unsigned)j < (unsigned)n)
        llr[(size_t)f * n + j] = values[q] ? (int8_t)-127 : (int8_t)127;
}

hipError_t launch_reveal(int8_t *llr, int n, int n_frames, const int32_t *frame_ids, int k, const int32_t *positions,
                         const uint8_t *values, int r, hipStream_t s)
{
    const long long total = (long long)k * r;
    const int threads = 256;
    hipLaunchKernelGGL(k_reveal, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads), 0, s, llr, n,
                       n_frames, frame_ids, k, positions, values, r);
    return hipGetLastError();
}

// Reset the frame queue of a persistent launch (a kernel, not a memset, so that
// the pair can be captured in a graph and replayed).
__global__ void k_queue_reset(int *queue)
{
    if (threadIdx.x == 0)
        *queue = 0;
}

hipError_t launch_queue_reset(int *queue, hipStream_t s)
{
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, queue);
    return hipGetLastError();
}

hipError_t launch_decode(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s)
{
    if (P.layer_sync)
        return launch_decode_multi(P, C, A, s);
    if (P.split_reg)
        return launch_decode_reg(P, C, A, s);
    if (P.split_dmax)
        return launch_decode_split(P, C, A, s);
    if (P.pairs)
        return launch_decode_pairs(P, C, A, s);
    return launch_decode_scalar(P, C, A, s);
}

} // namespace qkdldpc
