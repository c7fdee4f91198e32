// gfx950 decode kernel with the CN->VN messages in registers: the path of
// codes with five base rows (the 5 x Nb family), a power-of-two lift Z <= 1024,
// rows of 19 or 20 edges, 8-bit soft values with E_max > MSG_max and no offset
// table
// (arXiv:1903.10107, Secs. 2-3: Eqs. 1, 4, 8, 9, Alg. 1 and Alg. 2).
//
// The row-pair arithmetic is the split family's (two lanes per row pair
// (r, r + Z/2), both rows as the 16-bit halves of each register, lane A holding
// edges 0 .. DH-1 and lane B edges DMAX-1 .. DH, one lane swap for the
// forward-backward fold). What differs is where the state lives:
//
// * L: a lane owns the same row pair and slots in every layer, so the messages
//   of all layers stay in its registers from the first iteration to the last
//   (MB x DH registers, two rows each). Nothing of L is read or written in
//   LDS, and no byte packing is needed for it.
// * E: int8 in LDS at offset 0, plus a dummy block column for padding slots.
// * Addresses: the E byte address of row r's edge in slot i of layer b does not
//   depend on the frame, so every lane computes its MB x DH addresses once per
//   workgroup into an LDS table of 16-bit entries laid out [lane][layer][slot]:
//   a lane reads its entries at immediate offsets from one base, and the lane
//   stride of MB x DH entries (25 dwords for MB x DH = 50) is odd in dwords, so
//   a wave's reads fall in distinct banks. Row r + Z/2 is at the address XOR Z/2.
// * Padding: rows shorter than DMAX fill their last slots with the dummy
//   column; a per-lane bit mask marks the real slots, and padding operands are
//   masked to the fold's neutral value.
//
// The syndrome test of the state after iteration t-1 is folded into layer 0 of
// iteration t, as in the split family: layer 0 loads exactly that state, and
// the other layers are tested only when all of layer 0's rows hold.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "split_common.hpp"

namespace qkdldpc {

namespace {

constexpr int kRegLayers = 5;

struct RegLds {
    int8_t *E;        // [n + Z] soft values plus the dummy block column, at LDS offset 0
    uint8_t *syn;     // packed syndrome of the current frame
    uint16_t *addr;   // [threads][MB][DH] E byte address of each lane's slot
    int *flags;       // three vote words and one queue slot
};

__device__ __forceinline__ RegLds reg_lds(const DecodeArgs &A)
{
    extern __shared__ __align__(16) uint8_t smem[];
    RegLds M;
    M.E = reinterpret_cast<int8_t *>(smem);
    M.syn = smem + A.lds_syn_off;
    M.addr = reinterpret_cast<uint16_t *>(smem + A.lds_tab_off);
    M.flags = reinterpret_cast<int *>(smem + A.lds_flag_off);
    return M;
}

// Per-lane constants of a workgroup: the row pair, the real-slot mask.
struct RegLane {
    int tid, nthr, h, r;
    bool active;          // the lane pair owns a row pair (r < Z/2)
    uint64_t real;        // bit b * DH + i: slot i of layer b holds an edge
};

// Address table and real-slot mask, once per workgroup. A lane of an idle pair
// points every slot at the dummy column and marks none real, so its operands
// are neutral and its E writes land in the dummy column.
template <int MB, int DH>
__device__ __forceinline__ RegLane reg_setup(const DevCode &C, const DecodeArgs &A, const RegLds &M)
{
    RegLane G;
    G.tid = threadIdx.x;
    G.nthr = blockDim.x;
    G.h = G.tid & 1;
    G.r = G.tid >> 1;
    const int hz = C.z >> 1;
    G.active = G.r < hz;
    G.real = 0;
    const unsigned zm = (unsigned)(C.z - 1), dummy = (unsigned)(C.nb * C.z);
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
        for (int i = 0; i < DH; ++i) {
            const int4 te = A.lane_tab[(b * DH + i) * 2 + G.h];
            const bool real = G.active && te.z != 0;
            const unsigned a0 = G.active ? (((unsigned)G.r + (unsigned)te.x) & zm) | (unsigned)te.y : dummy;
            M.addr[G.tid * (MB * DH) + b * DH + i] = (uint16_t)a0;
            if (real)
                G.real |= 1ull << (b * DH + i);
        }
    return G;
}

// 0xffffffff when slot i of layer b holds an edge, else 0
template <int DH>
__device__ __forceinline__ int real_mask(const RegLane &G, int b, int i)
{
    return -(int)((G.real >> (b * DH + i)) & 1u);
}

// E of both rows of the pair at the slot addresses of layer b
template <int DH>
__device__ __forceinline__ void reg_fetch(const RegLds &M, const unsigned (&a0)[DH], unsigned hzb, s16x2 (&e)[DH])
{
#pragma unroll
    for (int i = 0; i < DH; ++i)
        e[i] = pack_halves(lds_ld<int8_t>(a0[i]), lds_ld<int8_t>(a0[i] ^ hzb));
}

template <int MB, int DH>
__device__ __forceinline__ void reg_addr(const RegLds &M, const RegLane &G, int b, unsigned (&a0)[DH])
{
    // one 16-bit load per slot: merged wider loads would need a mask or shift
    // per entry to split them, so an empty asm statement that may touch memory
    // keeps the loads apart
    const uint16_t *row = M.addr + G.tid * (MB * DH) + b * DH;
#pragma unroll
    for (int i = 0; i < DH; ++i) {
        a0[i] = row[i];
        __asm__ volatile("" ::: "memory");
    }
}

// XOR over this lane's real slots of the soft values' sign bits
template <int DMIN, int DMAX>
__device__ __forceinline__ s16x2 reg_parity(const RegLane &G, int b, const s16x2 (&e)[DMAX / 2])
{
    constexpr int DH = DMAX / 2;
    s16x2 own = splat2(0);
#pragma unroll
    for (int i = 0; i < DH; ++i)
        own ^= split_pad_slot<DMIN, DMAX>(i) ? (e[i] & __builtin_bit_cast(s16x2, real_mask<DH>(G, b, i))) : e[i];
    return own;
}

// layer b's pair of syndrome bits as the sign bits of two 16-bit halves (bit b:
// row b*Z + r, bit 16 + b: row b*Z + r + Z/2)
__device__ __forceinline__ s16x2 reg_syn(unsigned synm, int b)
{
    return __builtin_bit_cast(s16x2, (synm << (15 - b)) & 0x80008000u);
}

// 1 when some check row of layers [b0, b1) owned by this lane pair fails
template <int DMIN, int DMAX, int MB>
__device__ __forceinline__ int reg_unsat(const RegLds &M, const RegLane &G, unsigned synm, unsigned hzb, int b0,
                                         int b1)
{
    constexpr int DH = DMAX / 2;
    s16x2 any = splat2(0);
    // one layer at a time (not unrolled), so that the loads of several layers
    // do not compete with the message registers
#pragma unroll 1
    for (int b = b0; b < b1; ++b) {
        unsigned a0[DH];
        s16x2 e[DH];
        reg_addr<MB, DH>(M, G, b, a0);
        reg_fetch<DH>(M, a0, hzb, e);
        const s16x2 own = reg_parity<DMIN, DMAX>(G, b, e);
        any |= reg_syn(synm, b) ^ own ^ swap_pair(own);
    }
    return G.active && (any.x | any.y) < 0;
}

// Eq. 8, the check node (Eqs. 1 and 4 by Alg. 1 in forward-backward order, or
// min-sum) and Eq. 9 under Alg. 2 for one lane's slots of a row pair in layer
// b; lk holds the row pair's messages of that layer and receives the new ones.
template <int DMIN, int DMAX, int RULE>
__device__ __forceinline__ void reg_finish(const DevCode &C, const RegLane &G, int b, const s16x2 (&e)[DMAX / 2],
                                           const unsigned (&a0)[DMAX / 2], s16x2 (&lk)[DMAX / 2], s16x2 syn,
                                           unsigned hzb)
{
    constexpr int DH = DMAX / 2;
    const s16x2 em = splat2(C.e_max);
    const u16x2 mm = usplat2(C.msg_max), kf = usplat2(16384 - C.e_max * C.e_max);
    s16x2 vg[DH];
    u16x2 p[DH];
    s16x2 own = splat2(0);
#pragma unroll
    for (int i = 0; i < DH; ++i) {
        // Eq. 8, saturated to the 8-bit soft-value range
        const s16x2 v = vmin2(vmax2(e[i] - lk[i], splat2(-127)), splat2(127));
        u16x2 pi = as_u(vmin2(vmax2(v, -v), as_s(mm)));
        // Alg. 2: E is frozen where |E| = E_max, that is where E^2 = E_max^2.
        // With kf = 2^14 - E_max^2, E^2 + kf has bit 14 set exactly there (below
        // E_max it is at most 2^14 - 2 E_max + 1). Flipping bit 14 of v there
        // moves it 2^14 away from 0 without changing its sign, so the sum with
        // the new message stays beyond +-E_max and the clamp below returns E
        // (v has the sign of E there because E_max > MSG_max >= |L|); no 16-bit
        // overflow: |v| + 2^14 + MSG_max < 2^15.
        const u16x2 sq = as_u(e[i]) * as_u(e[i]) + kf;
        s16x2 x = v ^ (as_s(sq) & splat2(0x4000));
        if (split_pad_slot<DMIN, DMAX>(i)) {
            const int rm = real_mask<DH>(G, b, i);
            const u16x2 mk = __builtin_bit_cast(u16x2, rm);
            x = x & __builtin_bit_cast(s16x2, rm);
            pi = (pi & mk) | (usplat2(kPad) & ~mk);
        }
        vg[i] = x;
        own ^= x;
        p[i] = pi;
    }
    // sign product of Eq. 1 over the whole row, times the syndrome bit
    const s16x2 par = syn ^ own ^ swap_pair(own);
    u16x2 out[DH];
    pair_fold<DH, RULE>(p, out);
#pragma unroll
    for (int i = 0; i < DH; ++i) {
        const s16x2 sg = (par ^ vg[i]) >> (short)15;  // -1 in a half whose message is negative
        const s16x2 ln = (as_s(out[i]) ^ sg) - sg;
        // Eq. 9 under Alg. 2 (frozen halves keep E, see above), clamped to +-E_max
        const s16x2 o = vmin2(vmax2(vg[i] + ln, -em), em);
        lds_st<int8_t>(a0[i], (int8_t)o.x);
        lds_st<int8_t>(a0[i] ^ hzb, (int8_t)o.y);
        lk[i] = ln;
    }
}

// Decode frame f with one workgroup (address table already built).
template <int DMIN, int DMAX, int MB, int RULE>
__device__ __forceinline__ void reg_decode_frame(const DevCode &C, const DecodeArgs &A, const RegLds &M,
                                                 const RegLane &G, int f)
{
    constexpr int DH = DMAX / 2;
    const int z = C.z, n = C.n, hz = z >> 1;
    const unsigned hzb = (unsigned)hz;
    const int tid = G.tid, nthr = G.nthr;

    // stage in: syndrome, E = llr (-128 read as -127), vote words
    const uint8_t *syn = A.syn + (size_t)f * A.syn_bytes;
    for (int i = tid; i < A.syn_bytes; i += nthr)
        M.syn[i] = syn[i];
    stage_llr<int8_t>(M.E, A.llr + (size_t)f * n, n, C.e_max < 127 ? C.e_max : 127, tid, nthr);
    if (tid < 3)
        M.flags[tid] = 0;
    __syncthreads();

    // the lane's syndrome bits: bit b for row b*Z + r, bit 16 + b for row b*Z + r + Z/2
    unsigned synm = 0;
    if (G.active)
#pragma unroll 1
        for (int b = 0; b < MB; ++b) {
            const int i0 = b * z + G.r, i1 = i0 + hz;
            synm |= (unsigned)((M.syn[i0 >> 3] >> (i0 & 7)) & 1) << b |
                    (unsigned)((M.syn[i1 >> 3] >> (i1 & 7)) & 1) << (16 + b);
        }

    int vk = 0, iters = 0;
    // layer 0 first: a frame that fails there skips testing the other layers
    int conv = !block_vote(reg_unsat<DMIN, DMAX, MB>(M, G, synm, hzb, 0, 1), M.flags, vk) &&
               !block_vote(reg_unsat<DMIN, DMAX, MB>(M, G, synm, hzb, 1, MB), M.flags, vk);

    s16x2 Lr[MB][DH];
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
        for (int i = 0; i < DH; ++i)
            Lr[b][i] = splat2(0);

    for (int t = 1; t <= A.max_iter && !conv; ++t) {
        bool stop = false;
#pragma unroll
        for (int b = 0; b < MB; ++b) {
            // the slot addresses before the barrier that orders the previous
            // layer's E writes; after it only the E reads remain
            unsigned a0[DH];
            reg_addr<MB, DH>(M, G, b, a0);
            __syncthreads();
            s16x2 e[DH];
            reg_fetch<DH>(M, a0, hzb, e);
            if (b == 0 && t >= 2) {
                const s16x2 own = reg_parity<DMIN, DMAX>(G, 0, e);
                const s16x2 pe = reg_syn(synm, 0) ^ own ^ swap_pair(own);
                const int fail0 = G.active && (pe.x | pe.y) < 0;
                if (!block_vote(fail0, M.flags, vk) &&
                    !block_vote(reg_unsat<DMIN, DMAX, MB>(M, G, synm, hzb, 1, MB), M.flags, vk)) {
                    conv = 1;
                    iters = t - 1;
                    stop = true;
                    break;
                }
            }
            reg_finish<DMIN, DMAX, RULE>(C, G, b, e, a0, Lr[b], reg_syn(synm, b), hzb);
        }
        if (stop)
            break;
        iters = t;
    }
    // the last layer's E writes before the final test and the stage-out reads
    __syncthreads();
    if (!conv && A.max_iter > 0)
        conv = !block_vote(reg_unsat<DMIN, DMAX, MB>(M, G, synm, hzb, 0, 1), M.flags, vk) &&
               !block_vote(reg_unsat<DMIN, DMAX, MB>(M, G, synm, hzb, 1, MB), M.flags, vk);
    if (!conv)
        iters = A.max_iter;

    // stage out: hard decisions (wavefront ballot), flag, count, optional state
    const int lane = tid & 63, wv = tid >> 6, nwv = nthr >> 6;
    const int nwords = (n + 63) >> 6;
    uint8_t *ob = A.out_bits + (size_t)f * A.bit_bytes;
    for (int w = wv; w < nwords; w += nwv) {
        const int j = (w << 6) + lane;
        const bool neg = j < n && M.E[j] < 0;
        const unsigned long long mask = __ballot(neg);
        if (lane < 8) {
            const int byte = (w << 3) + lane;
            if (byte < A.bit_bytes)
                ob[byte] = (uint8_t)(mask >> (8 * lane));
        }
    }
    if (tid == 0) {
        A.out_conv[f] = (uint8_t)conv;
        if (A.out_iters)
            A.out_iters[f] = iters;
    }
    if (A.out_L && G.active) {
        // canonical [block][row] layout: each lane writes its slots of every layer
        // (zero when no iteration ran, which the registers then still hold)
        int8_t *oL = A.out_L + (size_t)f * C.n_blocks * z;
        // (the asm statement keeps the table reads below inside the frame loop of
        // the persistent kernel, rather than held in registers across frames)
        __asm__ volatile("" ::: "memory");
#pragma unroll
        for (int b = 0; b < MB; ++b)
#pragma unroll
            for (int i = 0; i < DH; ++i) {
                const int blk = A.lane_tab[(b * DH + i) * 2 + G.h].w;
                if (blk >= 0) {
                    oL[(size_t)blk * z + G.r] = (int8_t)Lr[b][i].x;
                    oL[(size_t)blk * z + G.r + hz] = (int8_t)Lr[b][i].y;
                }
            }
    }
    if (A.out_E)
        for (int j = tid; j < n; j += nthr)
            A.out_E[(size_t)f * n + j] = (int16_t)M.E[j];
}

// One workgroup per frame (grid = frames).
template <int DMIN, int DMAX, int MB, int RULE>
__global__ __launch_bounds__(1024) void k_decode_frame_reg(DevCode C, DecodeArgs A)
{
    const RegLds M = reg_lds(A);
    const RegLane G = reg_setup<MB, DMAX / 2>(C, A, M);
    reg_decode_frame<DMIN, DMAX, MB, RULE>(C, A, M, G, blockIdx.x);
}

// Persistent workgroups: each takes the next position of a device queue (reset
// to 0 by k_queue_reset before the launch), decodes frame order[position] (or
// position), and stops once the queue is past the last frame, which every wave
// of every workgroup reaches.
template <int DMIN, int DMAX, int MB, int RULE>
__global__ __launch_bounds__(1024) void k_decode_reg_persistent(DevCode C, DecodeArgs A)
{
    const RegLds M = reg_lds(A);
    const RegLane G = reg_setup<MB, DMAX / 2>(C, A, M);
    for (;;) {
        __syncthreads();  // the previous frame's stage-out is done with E and the queue slot
        if (threadIdx.x == 0)
            M.flags[3] = atomicAdd(A.queue, 1);
        __syncthreads();
        const int q = M.flags[3];
        if (q >= A.n_frames)
            break;
        const int f = A.order ? A.order[q] : q;
        if ((unsigned)f < (unsigned)A.n_frames)
            reg_decode_frame<DMIN, DMAX, MB, RULE>(C, A, M, G, f);
    }
}

template <int DMIN, int DMAX, int MB, int RULE>
hipError_t launch_one_reg(const DevCode &C, const DecodeArgs &A, int threads, size_t lds, hipStream_t s)
{
    const bool persistent = A.persistent_wgs > 0;
    auto kern = persistent ? k_decode_reg_persistent<DMIN, DMAX, MB, RULE> : k_decode_frame_reg<DMIN, DMAX, MB, RULE>;
    if (lds > 65536) {
        hipError_t e = persistent ? allow_max_lds<k_decode_reg_persistent<DMIN, DMAX, MB, RULE>>()
                                  : allow_max_lds<k_decode_frame_reg<DMIN, DMAX, MB, RULE>>();
        if (e != hipSuccess)
            return e;
    }
    if (persistent) {
        hipError_t e = launch_queue_reset(A.queue, s);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(kern, dim3(persistent ? A.persistent_wgs : A.n_frames), dim3(threads), lds, s, C, A);
    return hipGetLastError();
}

template <int DMIN>
hipError_t launch_rule_reg(int rule, const DevCode &C, const DecodeArgs &A, int threads, size_t lds, hipStream_t s)
{
    if (rule == LDPC_RULE_MINSUM)
        return launch_one_reg<DMIN, 20, kRegLayers, kRuleMinSum>(C, A, threads, lds, s);
    return launch_one_reg<DMIN, 20, kRegLayers, kRuleRcbpFB>(C, A, threads, lds, s);
}

} // namespace

hipError_t launch_decode_reg(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s)
{
    if (C.mb != kRegLayers || P.split_dmax != 20 || P.min_deg < 19 || P.acc_bits != 8 || C.offsets ||
        C.e_max <= C.msg_max)
        return hipErrorInvalidValue;
    return launch_rule_reg<19>(P.cn_rule, C, A, P.threads, P.lds_bytes, s);
}

} // namespace qkdldpc
