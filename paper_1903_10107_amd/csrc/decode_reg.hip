// gfx950 decode kernel with the CN->VN messages in registers: the path of
// codes with five base rows (the 5 x Nb family), a power-of-two lift Z <= 1024,
// rows of 19 or 20 edges, 8-bit soft values with E_max > MSG_max, with or without
// an offset table
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
    int *flags;       // three vote words, the queue slot, two last-layer test words
    int *offs;        // offset tables: [offset_iters][MB][DH][2] the slot's offset in both halves
};

__device__ __forceinline__ RegLds reg_lds(const DecodeArgs &A)
{
    extern __shared__ __align__(16) uint8_t smem[];
    RegLds M;
    M.E = reinterpret_cast<int8_t *>(smem);
    M.syn = smem + A.lds_syn_off;
    M.addr = reinterpret_cast<uint16_t *>(smem + A.lds_tab_off);
    M.flags = reinterpret_cast<int *>(smem + A.lds_flag_off);
    M.offs = reinterpret_cast<int *>(smem + A.lds_flag_off + 32);
    return M;
}

// The offset table, once per workgroup: for each of its rows, layer b, slot i
// and lane half h, the offset of the slot's block in both 16-bit halves (both
// rows of a pair share the block), 0 for padding slots. Read after the
// stage-in barrier.
template <int MB, int DH>
__device__ __forceinline__ void reg_stage_offsets(const DevCode &C, const DecodeArgs &A, const RegLds &M)
{
    const int total = C.offset_iters * MB * DH * 2;
    for (int q = threadIdx.x; q < total; q += blockDim.x) {
        const int slot = q % (MB * DH * 2), row = q / (MB * DH * 2);
        const int blk = A.lane_tab[slot].w;
        const unsigned o = (unsigned)(blk >= 0 ? C.offsets[(size_t)row * C.n_blocks + blk] : 0) & 0xffffu;
        M.offs[q] = (int)(o | o << 16);
    }
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
    // Every lane reads its entries (the table has both halves of every slot),
    // so that the loads do not sit in a branch that waits for each in turn; one
    // layer's entries at a time (an empty asm statement that may touch memory
    // keeps the layers' loads apart), so that they are in flight together
    // without holding all layers' entries in registers.
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        __asm__ volatile("" ::: "memory");
#pragma unroll
        for (int i = 0; i < DH; ++i) {
            const int4 te = A.lane_tab[(b * DH + i) * 2 + G.h];
            const bool real = G.active && te.z != 0;
            const unsigned a1 = (((unsigned)G.r + (unsigned)te.x) & zm) | (unsigned)te.y;
            M.addr[G.tid * (MB * DH) + b * DH + i] = (uint16_t)(G.active ? a1 : dummy);
            G.real |= (uint64_t)real << (b * DH + i);
        }
    }
    // the mask is complete here (otherwise its bits are formed where it is first
    // used, and the table entries stay live, in scratch, until then)
    __asm__ volatile("" : "+v"(G.real));
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

// Hands the zero-extended 32-bit addresses to an empty asm statement, so that
// a use in a later basic block (after a layer barrier) does not mask them to 16
// bits again. The statement waits for the loads: place it where they are
// complete anyway (at a barrier, after the E writes).
template <int DH>
__device__ __forceinline__ void reg_pin(unsigned (&a0)[DH])
{
#pragma unroll
    for (int i = 0; i < DH; ++i)
        __asm__ volatile("" : "+v"(a0[i]));
}

// a ^ b ^ c in one instruction (v_bitop3_b32 with truth table 0x96; the
// compiler keeps a chain of two-input XORs otherwise)
__device__ __forceinline__ s16x2 xor3(s16x2 a, s16x2 b, s16x2 c)
{
    return __builtin_bit_cast(s16x2, __builtin_amdgcn_bitop3_b32(__builtin_bit_cast(unsigned, a),
                                                                 __builtin_bit_cast(unsigned, b),
                                                                 __builtin_bit_cast(unsigned, c), 0x96));
}

// XOR of x[0 .. N-1], two operands per instruction
template <int N>
__device__ __forceinline__ s16x2 xor_all(const s16x2 (&x)[N])
{
    s16x2 acc = x[0];
    int i = 1;
#pragma unroll
    for (; i + 1 < N; i += 2)
        acc = xor3(acc, x[i], x[i + 1]);
    if (i < N)
        acc ^= x[i];
    return acc;
}

// XOR over this lane's real slots of the soft values' sign bits
template <int DMIN, int DMAX>
__device__ __forceinline__ s16x2 reg_parity(const RegLane &G, int b, const s16x2 (&e)[DMAX / 2])
{
    constexpr int DH = DMAX / 2;
    s16x2 t[DH];
#pragma unroll
    for (int i = 0; i < DH; ++i)
        t[i] = split_pad_slot<DMIN, DMAX>(i) ? (e[i] & __builtin_bit_cast(s16x2, real_mask<DH>(G, b, i))) : e[i];
    return xor_all<DH>(t);
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
        any |= xor3(reg_syn(synm, b), own, swap_pair(own));
    }
    return G.active && (any.x | any.y) < 0;
}

// Eq. 8, the check node (Eqs. 1 and 4 by Alg. 1 in forward-backward order, or
// min-sum) and Eq. 9 under Alg. 2 for one lane's slots of a row pair in layer
// b; lk holds the row pair's messages of that layer and receives the new ones.
// With PAR, also the syndrome test of the row pair on the new soft values: 1 when
// a row fails. (Used on the last layer, whose variable nodes take their final
// value of the iteration there.) With OFF, the magnitudes lose the offsets of the
// slots' blocks (orow[2 i] for slot i) and are clamped to [0, MSG_max].
template <int DMIN, int DMAX, int RULE, bool PAR = false, bool OFF = false>
__device__ __forceinline__ int reg_finish(const DevCode &C, const RegLane &G, int b, const s16x2 (&e)[DMAX / 2],
                                          const unsigned (&a0)[DMAX / 2], s16x2 (&lk)[DMAX / 2], s16x2 syn,
                                          unsigned hzb, const int *orow = nullptr)
{
    constexpr int DH = DMAX / 2;
    const s16x2 em = splat2(C.e_max);
    const u16x2 mm = usplat2(C.msg_max), kf = usplat2(16384 - C.e_max * C.e_max);
    s16x2 vg[DH];
    u16x2 p[DH];
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
        p[i] = pi;
    }
    // sign product of Eq. 1 over the whole row, times the syndrome bit (x has
    // the sign of v)
    const s16x2 own = xor_all<DH>(vg);
    const s16x2 par = xor3(syn, own, swap_pair(own));
    u16x2 out[DH];
    pair_fold<DH, RULE>(p, out);
    if constexpr (OFF) {
#pragma unroll
        for (int i = 0; i < DH; ++i) {
            const s16x2 oi = __builtin_bit_cast(s16x2, orow[2 * i]);
            out[i] = as_u(vmin2(vmax2(as_s(out[i]) - oi, splat2(0)), as_s(mm)));
        }
    }
    s16x2 ot[DH];
#pragma unroll
    for (int i = 0; i < DH; ++i) {
        const s16x2 sg = (par ^ vg[i]) >> (short)15;  // -1 in a half whose message is negative
        const s16x2 ln = (as_s(out[i]) ^ sg) - sg;
        // Eq. 9 under Alg. 2 (frozen halves keep E, see above), clamped to +-E_max
        const s16x2 o = vmin2(vmax2(vg[i] + ln, -em), em);
        lds_st<int8_t>(a0[i], (int8_t)o.x);
        lds_st<int8_t>(a0[i] ^ hzb, (int8_t)o.y);
        lk[i] = ln;
        if constexpr (PAR)
            ot[i] = split_pad_slot<DMIN, DMAX>(i) ? (o & __builtin_bit_cast(s16x2, real_mask<DH>(G, b, i))) : o;
    }
    if constexpr (PAR) {
        const s16x2 own_o = xor_all<DH>(ot);
        const s16x2 pe = xor3(syn, own_o, swap_pair(own_o));
        return G.active && (pe.x | pe.y) < 0;
    }
    return 0;
}

// Decode frame f with one workgroup (address table, and with OFF the offsets,
// already staged).
template <int DMIN, int DMAX, int MB, int RULE, bool OFF>
__device__ __forceinline__ void reg_decode_frame(const DevCode &C, const DecodeArgs &A, const RegLds &M,
                                                 const RegLane &G, int f)
{
    constexpr int DH = DMAX / 2;
    const int z = C.z, n = C.n, hz = z >> 1;
    const unsigned hzb = (unsigned)hz;
    const int tid = G.tid, nthr = G.nthr;

    // stage in: syndrome, E = llr (-128 read as -127), vote words
    const uint8_t *syn = A.syn + (size_t)f * A.syn_bytes;
    const int8_t *llr = A.llr + (size_t)f * n;
    const int n16 = n >> 4;
    if (C.e_max >= 127 && (n & 15) == 0 && ((uintptr_t)llr & 15) == 0 && n16 <= 2 * nthr &&
        A.syn_bytes <= nthr) {
        // at most two 16-byte LLR chunks and one syndrome byte per thread: all
        // loads issued (at clamped, always valid indices) before any LDS write
        const uint4 *src = reinterpret_cast<const uint4 *>(llr);
        const int q0 = tid, q1 = tid + nthr;
        const uint4 v0 = src[q0 < n16 ? q0 : n16 - 1];
        const uint4 v1 = src[q1 < n16 ? q1 : n16 - 1];
        const uint8_t sb = syn[tid < A.syn_bytes ? tid : A.syn_bytes - 1];
        uint4 *dst = reinterpret_cast<uint4 *>(M.E);
        if (q0 < n16)
            dst[q0] = llr_no_m128(v0);
        if (q1 < n16)
            dst[q1] = llr_no_m128(v1);
        if (tid < A.syn_bytes)
            M.syn[tid] = sb;
    } else {
        for (int i = tid; i < A.syn_bytes; i += nthr)
            M.syn[i] = syn[i];
        stage_llr<int8_t>(M.E, llr, n, C.e_max < 127 ? C.e_max : 127, tid, nthr);
    }
    if (tid < 6 && tid != 3)  // vote words 0-2 and the last-layer test words 4-5 (3 is the queue slot)
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

    // The syndrome test of the state after iteration t-1 starts from its last
    // layer: that layer's variable nodes take their final value of the
    // iteration in it, so its rows are tested on the values it writes, and a
    // failing lane sets word 4 + (t-1) % 2 before the barrier that opens
    // iteration t. Only when no last-layer row failed (rare before convergence)
    // are the other layers tested, layer 0 on the values it loads anyway,
    // and voted on; otherwise the test costs no barrier of its own. Thread 0
    // clears the word after the next barrier, which every reader has passed.
    for (int t = 1; t <= A.max_iter && !conv; ++t) {
        bool stop = false;
        // this lane's offsets of iteration t: row min(t - 1, offset_iters - 1)
        const int *orow_t = nullptr;
        if constexpr (OFF)
            orow_t = M.offs + (size_t)(t - 1 < C.offset_iters - 1 ? t - 1 : C.offset_iters - 1) * (MB * DH * 2) + G.h;
#pragma unroll
        for (int b = 0; b < MB; ++b) {
            // the slot addresses before the barrier that orders the previous
            // layer's E writes; after it only the E reads remain
            unsigned a0[DH];
            reg_addr<MB, DH>(M, G, b, a0);
            reg_pin<DH>(a0);
            __syncthreads();
            if (b == 1 && t >= 2 && tid == 0)
                M.flags[4 + ((t - 1) & 1)] = 0;
            s16x2 e[DH];
            reg_fetch<DH>(M, a0, hzb, e);
            if (b == 0 && t >= 2 && !M.flags[4 + ((t - 1) & 1)]) {
                const s16x2 own = reg_parity<DMIN, DMAX>(G, 0, e);
                const s16x2 pe = xor3(reg_syn(synm, 0), own, swap_pair(own));
                const int fail = (G.active && (pe.x | pe.y) < 0) |
                                 reg_unsat<DMIN, DMAX, MB>(M, G, synm, hzb, 1, MB - 1);
                if (!block_vote(fail, M.flags, vk)) {
                    conv = 1;
                    iters = t - 1;
                    stop = true;
                    break;
                }
            }
            const int *orow = OFF ? orow_t + b * DH * 2 : nullptr;
            if (b == MB - 1) {
                if (reg_finish<DMIN, DMAX, RULE, true, OFF>(C, G, b, e, a0, Lr[b], reg_syn(synm, b), hzb, orow))
                    M.flags[4 + (t & 1)] = 1;
            } else {
                reg_finish<DMIN, DMAX, RULE, false, OFF>(C, G, b, e, a0, Lr[b], reg_syn(synm, b), hzb, orow);
            }
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

    // stage out: hard decisions, flag, count, optional state
    uint8_t *ob = A.out_bits + (size_t)f * A.bit_bytes;
    if ((n & 7) == 0) {
        // one output byte per thread and step from an 8-byte LDS read
        const uint2 *e8 = reinterpret_cast<const uint2 *>(M.E);
#pragma unroll 4
        for (int q = tid; q < (n >> 3); q += nthr) {
            const uint2 w = e8[q];
            ob[q] = (uint8_t)(sign_nibble(w.x) | sign_nibble(w.y) << 4);
        }
    } else {
        // wavefront ballots over 64 soft values
        const int lane = tid & 63, wv = tid >> 6, nwv = nthr >> 6;
        const int nwords = (n + 63) >> 6;
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
template <int DMIN, int DMAX, int MB, int RULE, bool OFF>
__global__ __launch_bounds__(1024) void k_decode_frame_reg(DevCode C, DecodeArgs A)
{
    const RegLds M = reg_lds(A);
    if constexpr (OFF)
        reg_stage_offsets<MB, DMAX / 2>(C, A, M);
    const RegLane G = reg_setup<MB, DMAX / 2>(C, A, M);
    reg_decode_frame<DMIN, DMAX, MB, RULE, OFF>(C, A, M, G, blockIdx.x);
}

// Persistent workgroups: each takes the next position of a device queue (reset
// to 0 by k_queue_reset before the launch), decodes frame order[position] (or
// position), and stops once the queue is past the last frame, which every wave
// of every workgroup reaches.
template <int DMIN, int DMAX, int MB, int RULE, bool OFF>
__global__ __launch_bounds__(1024) void k_decode_reg_persistent(DevCode C, DecodeArgs A)
{
    const RegLds M = reg_lds(A);
    if constexpr (OFF)
        reg_stage_offsets<MB, DMAX / 2>(C, A, M);
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
            reg_decode_frame<DMIN, DMAX, MB, RULE, OFF>(C, A, M, G, f);
    }
}

// ---------------------------------------------------------------------------
// Several frames per workgroup for lifts of at most 64 (frames_per_workgroup in
// the schedule): a frame's Z lanes (two per row pair) lie in one wave, so a wave
// decodes 64 / Z frames on its own and a workgroup of W waves decodes
// W x 64 / Z frames with no workgroup barrier in the decode (one at the start,
// after an offset table is staged, is the only one). Within a wave the LDS
// instructions execute in program order, so a layer's E reads follow the
// previous layer's E writes without a barrier; the syndrome tests are wave
// ballots over each frame's lanes. Frames of one wave run in lockstep: a frame
// that has converged stops updating its state (its lanes are masked off) while
// the other frames of the wave go on.
// ---------------------------------------------------------------------------

// LDS of the wave kernel: frame slot k's E (plus dummy column) at k * esz, its
// syndrome at syn_off + k * syn_bytes, then the per-lane address table and,
// with an offset table, its rows as in the one-frame kernels.
struct WaveGeom {
    int fpw;        // frames per workgroup
    int esz;        // bytes per frame slot's E region (n + Z rounded up to 16)
    int syn_off;    // LDS offset of the syndromes
    int tab_off;    // LDS offset of the address table
    int off_off;    // LDS offset of the staged offsets
};

__host__ __device__ inline WaveGeom wave_geom(int n, int z, int syn_bytes, int fpw, int threads, int mb, int dh)
{
    WaveGeom g;
    g.fpw = fpw;
    g.esz = (n + z + 15) & ~15;
    g.syn_off = fpw * g.esz;
    g.tab_off = (g.syn_off + fpw * syn_bytes + 15) & ~15;
    g.off_off = (g.tab_off + threads * mb * dh * 2 + 15) & ~15;
    return g;
}

__host__ __device__ inline size_t wave_lds_bytes(int n, int z, int syn_bytes, int fpw, int threads, int mb, int dh,
                                                 int offset_iters)
{
    const WaveGeom g = wave_geom(n, z, syn_bytes, fpw, threads, mb, dh);
    return (size_t)g.off_off + (size_t)offset_iters * mb * dh * 2 * 4;
}

template <int DMIN, int DMAX, int MB, int RULE, bool OFF>
__global__ __launch_bounds__(1024) void k_decode_wave_reg(DevCode C, DecodeArgs A)
{
    constexpr int DH = DMAX / 2;
    extern __shared__ __align__(16) uint8_t smem[];
    const int z = C.z, n = C.n, hz = z >> 1;
    const unsigned hzb = (unsigned)hz, zm = (unsigned)(z - 1);
    const WaveGeom W = wave_geom(n, z, A.syn_bytes, A.frames_per_wg, blockDim.x, MB, DH);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int fw = 64 / z;                       // frames per wave
    const int sub = lane / z;                    // frame of this lane within the wave
    const int slot = wave * fw + sub;            // frame slot within the workgroup
    const int lane0 = sub * z;                   // first lane of the frame in the wave
    const int f = blockIdx.x * W.fpw + slot;
    const bool valid = f < A.n_frames;
    const unsigned long long fmask = z == 64 ? ~0ull : ((1ull << z) - 1ull);
    int8_t *E = reinterpret_cast<int8_t *>(smem) + slot * W.esz;
    uint8_t *syn_s = smem + W.syn_off + slot * A.syn_bytes;

    RegLds M;
    M.E = E;
    M.syn = syn_s;
    M.addr = reinterpret_cast<uint16_t *>(smem + W.tab_off);
    M.flags = nullptr;
    M.offs = reinterpret_cast<int *>(smem + W.off_off);
    if constexpr (OFF) {
        // the offsets every frame of the workgroup uses: the kernel's one
        // workgroup barrier, before any wave's control flow depends on its frames
        reg_stage_offsets<MB, DH>(C, A, M);
        __syncthreads();
    }
    RegLane G;
    G.tid = tid;
    G.nthr = blockDim.x;
    G.h = tid & 1;
    G.r = (lane - lane0) >> 1;
    G.active = valid;
    G.real = 0;
    {
        const unsigned ebase = (unsigned)(slot * W.esz), dummy = ebase + (unsigned)(C.nb * z);
        // as in reg_setup: unconditional loads, one layer at a time
#pragma unroll
        for (int b = 0; b < MB; ++b) {
            __asm__ volatile("" ::: "memory");
#pragma unroll
            for (int i = 0; i < DH; ++i) {
                const int4 te = A.lane_tab[(b * DH + i) * 2 + G.h];
                const unsigned a1 = ebase + ((((unsigned)G.r + (unsigned)te.x) & zm) | (unsigned)te.y);
                M.addr[tid * (MB * DH) + b * DH + i] = (uint16_t)(valid ? a1 : dummy);
                G.real |= (uint64_t)(valid && te.z != 0) << (b * DH + i);
            }
        }
        __asm__ volatile("" : "+v"(G.real));
    }
    // 1 when some lane of this lane's frame has pred (a wave ballot)
    auto frame_any = [&](bool pred) -> bool { return ((__ballot(pred) >> lane0) & fmask) != 0; };

    // stage in, by the frame's own lanes
    const int lf = lane - lane0;
    if (valid) {
        const uint8_t *sg = A.syn + (size_t)f * A.syn_bytes;
        for (int i = lf; i < A.syn_bytes; i += z)
            syn_s[i] = sg[i];
        stage_llr<int8_t>(E, A.llr + (size_t)f * n, n, C.e_max < 127 ? C.e_max : 127, lf, z);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    unsigned synm = 0;
    if (valid)
#pragma unroll 1
        for (int b = 0; b < MB; ++b) {
            const int i0 = b * z + G.r, i1 = i0 + hz;
            synm |= (unsigned)((syn_s[i0 >> 3] >> (i0 & 7)) & 1) << b |
                    (unsigned)((syn_s[i1 >> 3] >> (i1 & 7)) & 1) << (16 + b);
        }

    const bool u0 = frame_any(reg_unsat<DMIN, DMAX, MB>(M, G, synm, hzb, 0, 1));
    const bool u1 = frame_any(reg_unsat<DMIN, DMAX, MB>(M, G, synm, hzb, 1, MB));
    bool conv = valid && !u0 && !u1;
    bool done = conv || !valid;
    int iters = 0;

    s16x2 Lr[MB][DH];
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
        for (int i = 0; i < DH; ++i)
            Lr[b][i] = splat2(0);

    for (int t = 1; t <= A.max_iter; ++t) {
        if (__ballot(!done) == 0)
            break;
        // this lane's offsets of iteration t: row min(t - 1, offset_iters - 1)
        const int *orow_t = nullptr;
        if constexpr (OFF)
            orow_t = M.offs + (size_t)(t - 1 < C.offset_iters - 1 ? t - 1 : C.offset_iters - 1) * (MB * DH * 2) + G.h;
#pragma unroll
        for (int b = 0; b < MB; ++b) {
            unsigned a0[DH];
            reg_addr<MB, DH>(M, G, b, a0);
            s16x2 e[DH];
            reg_fetch<DH>(M, a0, hzb, e);
            if (b == 0 && t >= 2) {
                // the state after iteration t-1: layer 0 from the values just read,
                // the other layers only for frames whose layer 0 holds
                const s16x2 own = reg_parity<DMIN, DMAX>(G, 0, e);
                const s16x2 pe = xor3(reg_syn(synm, 0), own, swap_pair(own));
                const bool pass0 = !frame_any(valid && (pe.x | pe.y) < 0);
                const bool need = !done && pass0;
                if (__ballot(need) != 0) {
                    const bool rest = frame_any(reg_unsat<DMIN, DMAX, MB>(M, G, synm, hzb, 1, MB));
                    if (need && !rest) {
                        done = true;
                        conv = true;
                        iters = t - 1;
                    }
                }
            }
            if (!done)
                reg_finish<DMIN, DMAX, RULE, false, OFF>(C, G, b, e, a0, Lr[b], reg_syn(synm, b), hzb,
                                                         OFF ? orow_t + b * DH * 2 : nullptr);
            // the next layer's reads come after these writes in program order
            __builtin_amdgcn_wave_barrier();
        }
        if (!done)
            iters = t;
    }
    {
        // frames that ran out of iterations: the test after the last one
        const bool a = frame_any(reg_unsat<DMIN, DMAX, MB>(M, G, synm, hzb, 0, 1));
        const bool c = frame_any(reg_unsat<DMIN, DMAX, MB>(M, G, synm, hzb, 1, MB));
        if (valid && !conv && A.max_iter > 0)
            conv = !a && !c;
    }
    if (!conv)
        iters = A.max_iter;

    // stage out: every frame of the wave in turn, 64 hard decisions per ballot
    const int nwords = (n + 63) >> 6;
    for (int k = 0; k < fw; ++k) {
        const int fk = blockIdx.x * W.fpw + wave * fw + k;
        if (fk >= A.n_frames)
            break;  // uniform: fk depends on k only
        const int8_t *Ek = reinterpret_cast<const int8_t *>(smem) + (wave * fw + k) * W.esz;
        uint8_t *ob = A.out_bits + (size_t)fk * A.bit_bytes;
        for (int w = 0; w < nwords; ++w) {
            const int j = (w << 6) + lane;
            const unsigned long long mask = __ballot(j < n && Ek[j] < 0);
            if (lane < 8) {
                const int byte = (w << 3) + lane;
                if (byte < A.bit_bytes)
                    ob[byte] = (uint8_t)(mask >> (8 * lane));
            }
        }
    }
    if (valid && lane == lane0) {
        A.out_conv[f] = (uint8_t)conv;
        if (A.out_iters)
            A.out_iters[f] = iters;
    }
    if (A.out_L && valid) {
        int8_t *oL = A.out_L + (size_t)f * C.n_blocks * z;
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
    if (A.out_E && valid)
        for (int j = lf; j < n; j += z)
            A.out_E[(size_t)f * n + j] = (int16_t)E[j];
}

template <int DMIN, int DMAX, int MB, int RULE, bool OFF>
hipError_t launch_one_reg(const DevCode &C, const DecodeArgs &A, int threads, size_t lds, hipStream_t s)
{
    if (A.frames_per_wg > 0) {
        const int fw = 64 / C.z, wthreads = 64 * (A.frames_per_wg / fw);
        const size_t wlds = wave_lds_bytes(C.n, C.z, A.syn_bytes, A.frames_per_wg, wthreads, MB, DMAX / 2,
                                           OFF ? C.offset_iters : 0);
        if (wlds > 65536) {
            hipError_t e = allow_max_lds<k_decode_wave_reg<DMIN, DMAX, MB, RULE, OFF>>();
            if (e != hipSuccess)
                return e;
        }
        const int grid = (A.n_frames + A.frames_per_wg - 1) / A.frames_per_wg;
        auto wkern = k_decode_wave_reg<DMIN, DMAX, MB, RULE, OFF>;
        hipLaunchKernelGGL(wkern, dim3(grid), dim3(wthreads), wlds, s, C, A);
        return hipGetLastError();
    }
    const bool persistent = A.persistent_wgs > 0;
    auto kern = persistent ? k_decode_reg_persistent<DMIN, DMAX, MB, RULE, OFF>
                           : k_decode_frame_reg<DMIN, DMAX, MB, RULE, OFF>;
    if (lds > 65536) {
        hipError_t e = persistent ? allow_max_lds<k_decode_reg_persistent<DMIN, DMAX, MB, RULE, OFF>>()
                                  : allow_max_lds<k_decode_frame_reg<DMIN, DMAX, MB, RULE, OFF>>();
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
    if (C.offsets) {
        if (rule == LDPC_RULE_MINSUM)
            return launch_one_reg<DMIN, 20, kRegLayers, kRuleMinSum, true>(C, A, threads, lds, s);
        return launch_one_reg<DMIN, 20, kRegLayers, kRuleRcbpFB, true>(C, A, threads, lds, s);
    }
    if (rule == LDPC_RULE_MINSUM)
        return launch_one_reg<DMIN, 20, kRegLayers, kRuleMinSum, false>(C, A, threads, lds, s);
    return launch_one_reg<DMIN, 20, kRegLayers, kRuleRcbpFB, false>(C, A, threads, lds, s);
}

} // namespace

size_t wave_reg_lds_bytes(int n, int z, int syn_bytes, int fpw, int offset_iters)
{
    const int fw = 64 / z;
    return wave_lds_bytes(n, z, syn_bytes, fpw, 64 * (fpw / fw), kRegLayers, 10, offset_iters);
}

hipError_t launch_decode_reg(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s)
{
    if (C.mb != kRegLayers || P.split_dmax != 20 || P.min_deg < 19 || P.acc_bits != 8 || C.e_max <= C.msg_max)
        return hipErrorInvalidValue;
    return launch_rule_reg<19>(P.cn_rule, C, A, P.threads, P.lds_bytes, s);
}

} // namespace qkdldpc
