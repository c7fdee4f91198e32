// Row-pair machinery shared by the split decode kernels (two lanes per row
// pair, both rows as the 16-bit halves of each register; arXiv:1903.10107,
// Eqs. 1, 4, 8, 9, Alg. 1 and Alg. 2). See decode_split.hip for the layouts.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace qkdldpc {

typedef int8_t __attribute__((address_space(3))) lds_i8;
typedef int16_t __attribute__((address_space(3))) lds_i16;
template <typename ET>
struct LdsPtr;
template <>
struct LdsPtr<int8_t> {
    typedef lds_i8 *type;
};
template <>
struct LdsPtr<int16_t> {
    typedef lds_i16 *type;
};

// element at an absolute LDS byte address
template <typename ET>
__device__ __forceinline__ ET lds_ld(unsigned addr)
{
    return *(typename LdsPtr<ET>::type)(uintptr_t)addr;
}
template <typename ET>
__device__ __forceinline__ void lds_st(unsigned addr, ET v)
{
    *(typename LdsPtr<ET>::type)(uintptr_t)addr = v;
}

// two sign-extended values as the halves of one register: the low 16 bits of
// lo and of hi (one v_perm; the loads stay sign-extending byte loads)
__device__ __forceinline__ s16x2 pack_halves(int lo, int hi)
{
    return __builtin_bit_cast(s16x2, __builtin_amdgcn_perm((unsigned)hi, (unsigned)lo, 0x05040100u));
}

// exchange a 32-bit value with the other lane of the pair (DPP quad_perm [1,0,3,2])
__device__ __forceinline__ int swap_pair(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);
}
__device__ __forceinline__ s16x2 swap_pair(s16x2 x) { return __builtin_bit_cast(s16x2, swap_pair(__builtin_bit_cast(int, x))); }
__device__ __forceinline__ u16x2 swap_pair(u16x2 x) { return __builtin_bit_cast(u16x2, swap_pair(__builtin_bit_cast(int, x))); }

template <int DMIN, int DMAX>
__host__ __device__ constexpr bool split_pad_slot(int i)
{
    // lane A's slot i is edge i; lane B's slot i is edge DMAX-1-i
    return i >= DMIN || DMAX - 1 - i >= DMIN;
}

// Workgroup-wide OR of pred over three rotating LDS flag words: vote k writes
// word k % 3, waits, reads it, and thread 0 clears word (k + 2) % 3, whose last
// readers passed this barrier and whose next writers come after the next one.
__device__ __forceinline__ int block_vote(int pred, int *flags, int &k)
{
    const int w = k;
    if (pred)
        flags[w] = 1;
    __syncthreads();
    const int any = flags[w];
    if (threadIdx.x == 0)
        flags[w == 0 ? 2 : w - 1] = 0;
    k = w == 2 ? 0 : w + 1;
    return any;
}

// E byte addresses of a row pair for its slot: a0 = ((r + shift) mod Z) + column
// start, a1 = a0 with the Z/2 bit flipped (Z a power of two, column starts Z-aligned).
__device__ __forceinline__ unsigned slot_addr(int4 te, int r, unsigned zm, unsigned esh)
{
    // (t & mask) | start in one bitop3 (truth table 0xEA); the second row's
    // address is then one XOR
    return __builtin_amdgcn_bitop3_b32(((unsigned)r + (unsigned)te.x) << esh, zm << esh, (unsigned)te.y, 0xEA);
}

// L slots of one lane for one row pair and layer.
template <int DH, bool LG>
struct LRef;

// LDS, lane-interleaved: slot i of the lower half at p[2i], of the upper half at p[2DH + 2i]
template <int DH>
struct LRef<DH, false> {
    int8_t *p;
    __device__ __forceinline__ void load(s16x2 (&lk)[DH], bool) const
    {
#pragma unroll
        for (int i = 0; i < DH; ++i) {
            lk[i] = pack_halves(p[2 * i], p[2 * DH + 2 * i]);
        }
    }
    __device__ __forceinline__ void store(const s16x2 (&ln)[DH]) const
    {
#pragma unroll
        for (int i = 0; i < DH; ++i) {
            p[2 * i] = (int8_t)ln[i].x;
            p[2 * DH + 2 * i] = (int8_t)ln[i].y;
        }
    }
};

// Global: the chunk of one row pair and layer is 4 DH bytes, a 16-bit slot
// (lower half, upper half) per byte pair, nothing unused. Slots 2k and 2k+1 of a
// lane share a dword. DH even: lane 0's DH/2 dwords, then lane 1's. DH odd: lane
// 0's (DH-1)/2 dwords, one dword holding the last slot of lane 0 (low half) and
// of lane 1 (high half), then lane 1's dwords; each lane then reads its
// (DH+1)/2 dwords in one aligned load (lane 1's start at the shared dword) and
// writes its dwords and its 16-bit half of the shared one. Addresses are a base
// uniform over the workgroup plus a 32-bit per-lane offset. zero: take L = 0
// unread.
template <int DH>
struct LRef<DH, true> {
    static constexpr int NW = (DH + 1) / 2;  // dwords one lane reads
    static constexpr int ND = DH / 2;        // dwords one lane writes whole
    static constexpr bool ODD = DH & 1;
    static constexpr int PAIR_BYTES = 4 * DH;
    uint8_t *base;
    unsigned off;  // byte offset of the row pair's chunk
    int h;         // lane of the pair
    static __host__ __device__ __forceinline__ unsigned read_off(int h) { return (unsigned)h * 4u * ND; }
    static __host__ __device__ __forceinline__ unsigned dword_off(int h) { return (unsigned)h * 4u * NW; }
    static __host__ __device__ __forceinline__ unsigned short_off(int h) { return 4u * ND + 2u * (unsigned)h; }
    // byte of slot s's lower half in the chunk (for a readback of L)
    static __host__ __device__ __forceinline__ unsigned slot_byte(int h, int s)
    {
        return ODD && s == DH - 1 ? short_off(h) : dword_off(h) + 2u * (unsigned)s;
    }
    static __device__ __forceinline__ void fetch(const uint8_t *base, unsigned off, int h, uint32_t (&w)[NW])
    {
        const uint32_t *d = reinterpret_cast<const uint32_t *>(base + (off + read_off(h)));
#pragma unroll
        for (int k = 0; k < NW; ++k)
            w[k] = d[k];
    }
    // slot registers from the words fetch() read: bytes (x, x+1) of the word
    // pair move to the top of the two 16-bit halves, then an arithmetic shift.
    // DH odd: lane 1's slot words start one dword later, and the last slots
    // sit in the shared dword (lane 0: word ND, bytes 0-1; lane 1: word 0,
    // bytes 2-3).
    static __device__ __forceinline__ void unpack(const uint32_t (&w)[NW], int h, s16x2 (&lk)[DH])
    {
        if constexpr (ODD) {
            const unsigned sl = h ? 0x050c040cu : 0x010c000cu, sh = h ? 0x070c060cu : 0x030c020cu;
            const unsigned st = h ? 0x030c020cu : 0x050c040cu;
#pragma unroll
            for (int k = 0; k < ND; ++k) {
                lk[2 * k] = cell(__builtin_amdgcn_perm(w[k + 1], w[k], sl));
                lk[2 * k + 1] = cell(__builtin_amdgcn_perm(w[k + 1], w[k], sh));
            }
            lk[DH - 1] = cell(__builtin_amdgcn_perm(w[ND], w[0], st));
        } else {
#pragma unroll
            for (int k = 0; k < ND; ++k) {
                lk[2 * k] = cell(__builtin_amdgcn_perm(w[k], w[k], 0x010c000cu));
                lk[2 * k + 1] = cell(__builtin_amdgcn_perm(w[k], w[k], 0x030c020cu));
            }
        }
    }
    static __device__ __forceinline__ s16x2 cell(unsigned x) { return __builtin_bit_cast(s16x2, x) >> (short)8; }
    __device__ __forceinline__ void load(s16x2 (&lk)[DH], bool zero) const
    {
        if (zero) {
#pragma unroll
            for (int i = 0; i < DH; ++i)
                lk[i] = splat2(0);
            return;
        }
        uint32_t w[NW];
        fetch(base, off, h, w);
        unpack(w, h, lk);
    }
    // low bytes of the two 16-bit halves of a and of b, in that order
    static __device__ __forceinline__ uint32_t pack(s16x2 a, s16x2 b)
    {
        return __builtin_amdgcn_perm(__builtin_bit_cast(uint32_t, b), __builtin_bit_cast(uint32_t, a), 0x06040200u);
    }
    __device__ __forceinline__ void store(const s16x2 (&ln)[DH]) const
    {
        uint32_t *d = reinterpret_cast<uint32_t *>(base + (off + dword_off(h)));
#pragma unroll
        for (int k = 0; k < ND; ++k)
            d[k] = pack(ln[2 * k], ln[2 * k + 1]);
        if constexpr (ODD)
            *reinterpret_cast<uint16_t *>(base + (off + short_off(h))) = (uint16_t)pack(ln[DH - 1], ln[DH - 1]);
    }
};

template <int DH>
struct SplitRow {
    s16x2 e[DH], lk[DH];
    unsigned a0[DH];
    int pm[DH];
    unsigned off[(DH + 1) / 2];  // magnitude offsets of the slots' blocks, 16 bits each (offset tables only)
};

// Slot addresses, padding masks and (OFF) offsets of one lane's slots.
// off_row: the offset table's row of the current iteration; padding slots
// (block -1) take offset 0.
template <int DMIN, int DMAX, typename ET, bool OFF = false>
__device__ __forceinline__ void split_addr(SplitRow<DMAX / 2> &R, const int4 *__restrict__ tab, int r, unsigned zm,
                                           const int32_t *__restrict__ off_row = nullptr)
{
    constexpr int DH = DMAX / 2;
    constexpr unsigned esh = sizeof(ET) == 2 ? 1 : 0;
#pragma unroll
    for (int i = 0; i < DH; ++i) {
        const int4 te = tab[2 * i];
        R.a0[i] = slot_addr(te, r, zm, esh);
        R.pm[i] = te.z;
        if constexpr (OFF) {
            const unsigned o = (unsigned)(te.w >= 0 ? off_row[te.w] : 0) & 0xffffu;
            R.off[i / 2] = i % 2 ? R.off[i / 2] | (o << 16) : o;
        }
    }
}

// E of both rows at the slot addresses
template <typename ET, int DH>
__device__ __forceinline__ void split_fetch_e(SplitRow<DH> &R, unsigned hzb)
{
#pragma unroll
    for (int i = 0; i < DH; ++i)
        R.e[i] = pack_halves(lds_ld<ET>(R.a0[i]), lds_ld<ET>(R.a0[i] ^ hzb));
}

template <int DMIN, int DMAX, typename ET, bool OFF = false>
__device__ __forceinline__ void split_load_e(SplitRow<DMAX / 2> &R, const int4 *__restrict__ tab, int r, unsigned zm,
                                             unsigned hzb, const int32_t *__restrict__ off_row = nullptr)
{
    split_addr<DMIN, DMAX, ET, OFF>(R, tab, r, zm, off_row);
    split_fetch_e<ET>(R, hzb);
}

template <int DMIN, int DMAX, typename ET, bool LG, bool OFF = false>
__device__ __forceinline__ void split_load(SplitRow<DMAX / 2> &R, const LRef<DMAX / 2, LG> &Lr,
                                           const int4 *__restrict__ tab, int r, unsigned zm, unsigned hzb,
                                           bool first, const int32_t *__restrict__ off_row = nullptr)
{
    split_load_e<DMIN, DMAX, ET, OFF>(R, tab, r, zm, hzb, off_row);
    Lr.load(R.lk, first);
}

// XOR of the hard-decision sign bits of the row pair's slots held by this lane
template <int DMIN, int DMAX>
__device__ __forceinline__ s16x2 split_e_parity(const SplitRow<DMAX / 2> &R)
{
    constexpr int DH = DMAX / 2;
    s16x2 own = splat2(0);
#pragma unroll
    for (int i = 0; i < DH; ++i)
        own ^= split_pad_slot<DMIN, DMAX>(i) ? (R.e[i] & __builtin_bit_cast(s16x2, R.pm[i])) : R.e[i];
    return own;
}

// E stores of the LDS kernels: both rows of the pair at absolute LDS addresses.
template <typename ET>
struct LdsESink {
    unsigned hzb;  // the Z/2 bit of the byte address
    __device__ __forceinline__ void operator()(unsigned a0, s16x2 o) const
    {
        lds_st<ET>(a0, (ET)o.x);
        lds_st<ET>(a0 ^ hzb, (ET)o.y);
    }
};

// Check-node magnitudes of a row pair whose DMAX = 2 DH operands are split over
// the two lanes of a pair (lane A: edges 0 .. DH-1, lane B: edges DMAX-1 .. DH):
// min-sum, or Eq. 4 by Alg. 1 in forward-backward order. Lane A's left fold over
// its slots gives the forward partials, lane B's the backward ones; one lane
// swap hands each lane the other's last partial, and each lane's outputs are
// out_i = tau(X_{i-1}, W_{DH-1-i}) with out_0 = W_{DH-1}.
template <int DH, int RULE>
__device__ __forceinline__ void pair_fold(const u16x2 (&p)[DH], u16x2 (&out)[DH])
{
    if constexpr (RULE == kRuleMinSum) {
        u16x2 m1 = usplat2(0x7fff), m2 = usplat2(0x7fff);
#pragma unroll
        for (int i = 0; i < DH; ++i) {
            m2 = umin2(m2, umax2(m1, p[i]));
            m1 = umin2(m1, p[i]);
        }
        const u16x2 o1 = swap_pair(m1), o2 = swap_pair(m2);
        m2 = umin2(umin2(m2, o2), umax2(m1, o1));
        m1 = umin2(m1, o1);
        const u16x2 diff = m2 - m1;
#pragma unroll
        for (int i = 0; i < DH; ++i)
            out[i] = m2 - umin2(p[i] - m1, usplat2(1)) * diff;
    } else {
        u16x2 X[DH], W[DH];
        X[0] = p[0];
#pragma unroll
        for (int i = 1; i < DH; ++i)
            X[i] = tau2(X[i - 1], p[i]);
        W[0] = swap_pair(X[DH - 1]);
#pragma unroll
        for (int k = 1; k < DH; ++k)
            W[k] = tau2(W[k - 1], p[DH - k]);
        out[0] = W[DH - 1];
#pragma unroll
        for (int i = 1; i < DH; ++i)
            out[i] = tau2(X[i - 1], W[DH - 1 - i]);
    }
}

// Eq. 8, the check node (Eqs. 1, 4 by Alg. 1, or min-sum) and Eq. 9 under Alg. 2
// for one lane's slots of a row pair; the new soft values go to es(a0, value),
// the new messages to Lr.
template <int DMIN, int DMAX, typename ET, int RULE, bool LG, bool OFF = false, class ES>
__device__ __forceinline__ void split_finish(const DevCode &C, const SplitRow<DMAX / 2> &R,
                                             const LRef<DMAX / 2, LG> &Lr, s16x2 syn, const ES &es)
{
    constexpr int DH = DMAX / 2;
    constexpr int ACC = AccLim<ET>::value;
    const s16x2 em = splat2(C.e_max), em1 = splat2(C.e_max - 1);
    const u16x2 mm = usplat2(C.msg_max);
    s16x2 v[DH];
    u16x2 p[DH];
    s16x2 own = splat2(0);
#pragma unroll
    for (int i = 0; i < DH; ++i) {
        // Eq. 8, saturated to the soft-value range
        s16x2 vi = vmin2(vmax2(__builtin_elementwise_sub_sat(R.e[i], R.lk[i]), splat2(-ACC)), splat2(ACC));
        u16x2 pi = as_u(vmin2(vmax2(vi, -vi), as_s(mm)));
        if (split_pad_slot<DMIN, DMAX>(i)) {
            const u16x2 mk = __builtin_bit_cast(u16x2, R.pm[i]);
            vi = vi & __builtin_bit_cast(s16x2, R.pm[i]);
            pi = (pi & mk) | (usplat2(kPad) & ~mk);
        }
        v[i] = vi;
        own ^= vi;
        p[i] = pi;
    }
    // sign product of Eq. 1 over the whole row, times the syndrome bit
    const s16x2 par = syn ^ own ^ swap_pair(own);
    u16x2 out[DH];
    pair_fold<DH, RULE>(p, out);
    if constexpr (OFF) {
        // offset table: magnitude = clamp(mag - offset, 0, MSG_max) (both halves share the block)
#pragma unroll
        for (int i = 0; i < DH; ++i) {
            const unsigned sel = i % 2 ? 0x03020302u : 0x01000100u;  // splat the slot's 16-bit half
            const s16x2 oi = __builtin_bit_cast(s16x2, __builtin_amdgcn_perm(R.off[i / 2], R.off[i / 2], sel));
            out[i] = as_u(vmin2(vmax2(as_s(out[i]) - oi, splat2(0)), as_s(mm)));
        }
    }
    s16x2 ln[DH];
#pragma unroll
    for (int i = 0; i < DH; ++i) {
        const s16x2 sg = (par ^ v[i]) >> (short)15;  // -1 in a half whose message is negative
        const s16x2 mg = as_s(out[i]);
        ln[i] = (mg ^ sg) - sg;
        // Eq. 9 under Alg. 2: halves whose stored |E| is E_max keep E
        s16x2 o;
        if constexpr (sizeof(ET) == 1) {
            // g = E - clamp(E, +-(E_max - 1)) is +-1 exactly where |E| = E_max and 0
            // elsewhere; 511 g (odd, so one multiply-add) drives the sum past
            // +-E_max there, and the clamp returns E itself (no 16-bit overflow:
            // |v + ln + 511 g| <= 127 + 127 + 511)
            const s16x2 g = R.e[i] - vmin2(vmax2(R.e[i], -em1), em1);
            o = vmin2(vmax2(v[i] + (g * splat2(511) + ln[i]), -em), em);
        } else {
            // 16-bit E: the same g, scaled to +-32767 and added with saturation
            // after the update. A frozen E = E_max gives v >= E_max - MSG_max, so
            // v + ln >= E_max - 2 MSG_max and the saturating sum reaches at least
            // min(32767, E_max + 32513) >= E_max; symmetrically for -E_max.
            const s16x2 g = R.e[i] - vmin2(vmax2(R.e[i], -em1), em1);
            const s16x2 x = __builtin_elementwise_add_sat(v[i], ln[i]);
            o = vmin2(vmax2(__builtin_elementwise_add_sat(x, g * splat2(32767)), -em), em);
        }
        es(R.a0[i], o);
    }
    Lr.store(ln);
}

// 1 when some check row of layers [b0, b1) owned by this lane pair fails
template <int DMIN, int DMAX, typename ET>
__device__ __forceinline__ int split_rows_unsat(const DevCode &C, const uint8_t *__restrict__ s_syn,
                                                const int4 *__restrict__ s_tab, int h, int r, int b0, int b1)
{
    constexpr int DH = DMAX / 2;
    constexpr unsigned esh = sizeof(ET) == 2 ? 1 : 0;
    const int z = C.z, hz = z >> 1;
    const unsigned zm = (unsigned)(z - 1), hzb = (unsigned)hz << esh;
    s16x2 any = splat2(0);
    for (int b = b0; b < b1; ++b) {
        const int4 *tab = s_tab + b * DH * 2 + h;
        s16x2 x[DH];
#pragma unroll
        for (int i = 0; i < DH; ++i) {
            const int4 te = tab[2 * i];
            const unsigned a0 = slot_addr(te, r, zm, esh);
            x[i] = pack_halves(lds_ld<ET>(a0), lds_ld<ET>(a0 ^ hzb));
            if (split_pad_slot<DMIN, DMAX>(i))
                x[i] = x[i] & __builtin_bit_cast(s16x2, te.z);
        }
        s16x2 own = splat2(0);
#pragma unroll
        for (int i = 0; i < DH; ++i)
            own ^= x[i];
        any |= syn_pair(s_syn, b * z + r, b * z + r + hz) ^ own ^ swap_pair(own);
    }
    return (any.x | any.y) < 0;
}


} // namespace qkdldpc
