// gfx950 kernels of the quantized layered decoder (arXiv:1903.10107, Secs. 2-3).
//
// One workgroup decodes one frame from start to finish: stage in, pre-check,
// every iteration (all layers, then the syndrome test), stage out. Thread t
// owns rows t, t + T, ... of every layer; the rows of one layer touch disjoint
// variable nodes (one circulant per base entry), so a layer needs no atomics,
// only a workgroup barrier before the next layer reads what it wrote.
//
// Decoder state: soft values E (int8 or int16, one per variable node) and
// CN->VN messages L (int8, one per edge, laid out [block][row]). When both fit
// in the workgroup's LDS (n = 32768 takes 32 KB + 96 KB) they live there for the
// whole decode and HBM sees only the inputs and outputs; otherwise they live in
// a global-memory workspace, one slice per frame.
//
// Per edge the work is integer VALU arithmetic (saturating subtract, clip,
// three tau evaluations of Alg. 1 for the forward-backward fold, sign, the
// saturating update of Alg. 2); there is no dense contraction, so no MFMA.
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

// Magnitudes of the CN->VN messages of one row (Eq. 4 over all operands but k).
// p[k]: clipped input magnitudes, k < d. m[k]: output magnitudes.
template <int DMAX, int RULE>
__device__ __forceinline__ void cn_fold(const int (&p)[DMAX], int (&m)[DMAX], int d)
{
    if constexpr (RULE == kRuleMinSum) {
        // min1 / min2 / argmin
        int m1 = 0x7fff, m2 = 0x7fff, am = -1;
#pragma unroll
        for (int k = 0; k < DMAX; ++k) {
            if (k < d) {
                const int x = p[k];
                const bool lt = x < m1;
                m2 = lt ? m1 : (x < m2 ? x : m2);
                am = lt ? k : am;
                m1 = lt ? x : m1;
            }
        }
#pragma unroll
        for (int k = 0; k < DMAX; ++k)
            if (k < d)
                m[k] = k == am ? m2 : m1;
    } else if constexpr (RULE == kRuleRcbpEq7) {
        // Right folds in ascending edge order: S_k = tau(p_k, S_{k+1}), S_{d-1} = p_{d-1}.
        // Output k < d-1: tau(p_0, tau(p_1, ... tau(p_{k-1}, S_{k+1})));
        // output d-1: the right fold of p_0 .. p_{d-2}.
        int S[DMAX];
#pragma unroll
        for (int k = DMAX - 1; k >= 0; --k) {
            if (k < d) {
                if (k == d - 1)
                    S[k] = p[k];
                else
                    S[k] = tau(p[k], S[k + 1 < DMAX ? k + 1 : k]);
            }
        }
#pragma unroll
        for (int k = 0; k < DMAX; ++k) {
            if (k < d) {
                int acc, i0;
                if (k < d - 1) {
                    acc = S[k + 1 < DMAX ? k + 1 : k];
                    i0 = k - 1;
                } else {
                    acc = p[k >= 1 ? k - 1 : 0];
                    i0 = k - 2;
                }
#pragma unroll
                for (int i = DMAX - 1; i >= 0; --i)
                    if (i <= i0)
                        acc = tau(p[i], acc);
                m[k] = acc;
            }
        }
    } else {
        // Forward-backward: F_0 = p_0, F_k = tau(F_{k-1}, p_k); B_{d-1} = p_{d-1},
        // B_k = tau(p_k, B_{k+1}); out_0 = B_1, out_{d-1} = F_{d-2},
        // out_k = tau(F_{k-1}, B_{k+1}). F is kept in m[] and overwritten from the
        // top down by the outputs once it has been consumed.
        m[0] = p[0];
#pragma unroll
        for (int k = 1; k < DMAX - 1; ++k)
            if (k <= d - 2)
                m[k] = tau(m[k - 1], p[k]);
        int B = 0;
#pragma unroll
        for (int k = DMAX - 1; k >= 1; --k) {
            if (k < d) {
                if (k == d - 1) {
                    m[k] = m[k - 1];
                    B = p[k];
                } else {
                    m[k] = tau(m[k - 1], B);
                    B = tau(p[k], B);
                }
            }
        }
        m[0] = B;
    }
}

// One check row r of layer (o, d): Eq. 8, Eq. 1 times the syndrome bit, the
// fold, Eq. 9 under the saturation rule of Alg. 2.
template <int DMAX, typename ET, int RULE>
__device__ __forceinline__ void row_update(const DevCode &C, ET *__restrict__ E, int8_t *__restrict__ L,
                                           int o, int d, int r, int synbit, const int32_t *off_row)
{
    constexpr int ACC = AccLim<ET>::value;
    const int z = C.z;
    int v[DMAX], p[DMAX], m[DMAX];
    unsigned frozen = 0;
    int par = -synbit;
#pragma unroll
    for (int k = 0; k < DMAX; ++k) {
        if (k < d) {
            const int e = E[ldc(C.colbase, o + k) + rot(r, ldc(C.shift, o + k), z)];
            const int lo = L[(o + k) * z + r];
            const int vk = clampi(e - lo, -ACC, ACC);
            v[k] = vk;
            par ^= vk;
            const int a = vk < 0 ? -vk : vk;
            p[k] = a < C.msg_max ? a : C.msg_max;
            frozen |= (unsigned)(e == C.e_max || e == -C.e_max) << k;
        }
    }
    cn_fold<DMAX, RULE>(p, m, d);
#pragma unroll
    for (int k = 0; k < DMAX; ++k) {
        if (k < d) {
            int mg = m[k];
            if (off_row)
                mg = clampi(mg - ldc(off_row, o + k), 0, C.msg_max);
            const int s = (par ^ v[k]) >> 31;  // -1 when the message is negative
            const int ln = (mg ^ s) - s;
            if (!((frozen >> k) & 1u))
                E[ldc(C.colbase, o + k) + rot(r, ldc(C.shift, o + k), z)] = (ET)clampi(v[k] + ln, -C.e_max, C.e_max);
            L[(o + k) * z + r] = (int8_t)ln;
        }
    }
}

// 1 when some check row owned by this thread fails H x^ = s, x^_j = [E_j < 0].
template <int DMAX, typename ET>
__device__ __forceinline__ int rows_unsat(const DevCode &C, const ET *__restrict__ E,
                                          const uint8_t *__restrict__ s_syn, int tid, int nthr)
{
    int any = 0;
    for (int b = 0; b < C.mb; ++b) {
        const int d = ldc(C.deg, b), o = ldc(C.blk_off, b);
        for (int r = tid; r < C.z; r += nthr) {
            const int i = b * C.z + r;
            int acc = -(int)((s_syn[i >> 3] >> (i & 7)) & 1);
#pragma unroll
            for (int k = 0; k < DMAX; ++k)
                if (k < d)
                    acc ^= (int)E[ldc(C.colbase, o + k) + rot(r, ldc(C.shift, o + k), C.z)];
            any |= acc;
        }
    }
    return any < 0;
}

// Stage in: packed syndrome to LDS; E = llr clamped symmetrically; L = 0.
template <typename ET>
__device__ __forceinline__ void stage_in(const DevCode &C, const DecodeArgs &A, uint8_t *s_syn, ET *E, int8_t *L,
                                         int f, int tid, int nthr)
{
    const int n = C.n, ne = C.n_blocks * C.z;
    const uint8_t *syn = A.syn + (size_t)f * A.syn_bytes;
    for (int i = tid; i < A.syn_bytes; i += nthr)
        s_syn[i] = syn[i];
    const int8_t *llr = A.llr + (size_t)f * n;
    const int lim0 = C.e_max < 127 ? C.e_max : 127;
    for (int j = tid; j < n; j += nthr)
        E[j] = (ET)clampi(llr[j], -lim0, lim0);
    for (int e = tid; e < ne; e += nthr)
        L[e] = 0;
    __syncthreads();
}

// Stage out: hard decisions packed with a wavefront ballot (64 bits per wave
// step), flags, iteration count and, when asked, the final state.
template <typename ET>
__device__ __forceinline__ void stage_out(const DevCode &C, const DecodeArgs &A, const ET *E, const int8_t *L,
                                          int f, int tid, int nthr, int conv, int iters)
{
    const int n = C.n, ne = C.n_blocks * C.z;
    const int lane = tid & 63, wv = tid >> 6, nwv = nthr >> 6;
    const int nwords = (n + 63) >> 6;
    uint8_t *ob = A.out_bits + (size_t)f * A.bit_bytes;
    for (int w = wv; w < nwords; w += nwv) {
        const int j = (w << 6) + lane;
        const bool neg = j < n && E[j] < 0;
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
    if (A.out_L)
        for (int e = tid; e < ne; e += nthr)
            A.out_L[(size_t)f * ne + e] = L[e];
    if (A.out_E)
        for (int j = tid; j < n; j += nthr)
            A.out_E[(size_t)f * n + j] = (int16_t)E[j];
}

template <int DMAX, typename ET, int RULE, bool LDS_STATE>
__global__ __launch_bounds__(1024) void k_decode_frame(DevCode C, DecodeArgs A)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const int f = blockIdx.x;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int z = C.z, n = C.n;
    const int ne = C.n_blocks * z;
    uint8_t *s_syn = smem + A.lds_syn_off;
    ET *E;
    int8_t *L;
    if constexpr (LDS_STATE) {
        E = reinterpret_cast<ET *>(smem + A.lds_e_off);
        L = reinterpret_cast<int8_t *>(smem + A.lds_l_off);
    } else {
        uint8_t *w = A.ws + (size_t)f * A.ws_frame_bytes;
        E = reinterpret_cast<ET *>(w);
        L = reinterpret_cast<int8_t *>(w + A.ws_l_off);
    }

    stage_in<ET>(C, A, s_syn, E, L, f, tid, nthr);
    int conv = !__syncthreads_or(rows_unsat<DMAX, ET>(C, E, s_syn, tid, nthr));
    int iters = 0;
    for (int t = 1; t <= A.max_iter && !conv; ++t) {
        const int32_t *off_row = nullptr;
        if (C.offsets)
            off_row = C.offsets + (size_t)(t - 1 < C.offset_iters - 1 ? t - 1 : C.offset_iters - 1) * C.n_blocks;
        for (int b = 0; b < C.mb; ++b) {
            const int d = ldc(C.deg, b), o = ldc(C.blk_off, b);
            for (int r = tid; r < z; r += nthr) {
                const int i = b * z + r;
                const int sb = (s_syn[i >> 3] >> (i & 7)) & 1;
                row_update<DMAX, ET, RULE>(C, E, L, o, d, r, sb, off_row);
            }
            __syncthreads();
        }
        iters = t;
        conv = !__syncthreads_or(rows_unsat<DMAX, ET>(C, E, s_syn, tid, nthr));
    }
    if (!conv)
        iters = A.max_iter;

    stage_out<ET>(C, A, E, L, f, tid, nthr, conv, iters);
}

// ---------------------------------------------------------------------------
// Packed variant: a lane owns the row pair (r, r + Z/2) of every layer and
// keeps both rows in the two 16-bit halves of each register, so that every
// VN/CN step is one v_pk_* instruction for two rows. For even Z the two rows'
// variable nodes in a block are x = (r + s) mod Z and (x + Z/2) mod Z; for a
// power-of-two Z the second address is the first with bit Z/2 flipped.
//
// LDS layout (all offsets from the host): E [n] at offset 0, so that a variable
// node index is its LDS address; L transposed as [pair r][block][half] with a
// per-pair stride of an odd number of dwords (one ds_read_i8 per half at an
// immediate offset, no bank conflicts across lanes); the packed syndrome; two
// flag words for the workgroup-wide "some check fails" vote.
// ---------------------------------------------------------------------------

template <bool POW2>
__device__ __forceinline__ int pair_first(const DevCode &C, int blk, int r)
{
    if constexpr (POW2) {
        const unsigned cs = (unsigned)ldc(C.colshift, blk);  // c * Z | shift
        const unsigned zm = (unsigned)(C.z - 1);
        return (int)((((unsigned)r + cs) & zm) | (cs & ~zm));
    } else {
        return ldc(C.colbase, blk) + rot(r, ldc(C.shift, blk), C.z);
    }
}

template <bool POW2>
__device__ __forceinline__ int pair_second(const DevCode &C, int blk, int a0)
{
    const int h = C.z >> 1;
    if constexpr (POW2) {
        return a0 ^ h;
    } else {
        const int cb = ldc(C.colbase, blk);
        return cb + rot(a0 - cb, h, C.z);
    }
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

// One row pair (r, r + Z/2) of layer (o, d), d in [DMIN, DMAX]: Eq. 8, the sign
// of Eq. 1 times the syndrome bits, the fold, Eq. 9 under Alg. 2.
// Lt: this pair's L slice at the layer's first block ([block][half]).
template <int DMIN, int DMAX, typename ET, int RULE, bool POW2>
__device__ __forceinline__ void row_update_x2(const DevCode &C, ET *__restrict__ E, int8_t *__restrict__ Lt,
                                              int o, int d, int r, s16x2 par, const int32_t *off_row)
{
    constexpr int ACC = AccLim<ET>::value;
    const s16x2 em = splat2(C.e_max);
    const u16x2 mm = usplat2(C.msg_max);
    s16x2 v[DMAX], e[DMAX], lk[DMAX];
    u16x2 p[DMAX], m[DMAX];
    int a0s[DMAX];
    // all loads first (padding slots re-read the row's last edge), so they batch
#pragma unroll
    for (int k = 0; k < DMAX; ++k) {
        const int kk = k < DMIN ? k : (k < d ? k : d - 1);
        const int a0 = pair_first<POW2>(C, o + kk, r);
        a0s[k] = a0;
        e[k] = load_pair(E, a0, pair_second<POW2>(C, o + kk, a0));
        lk[k] = load_pair(Lt, 2 * kk, 2 * kk + 1);
    }
#pragma unroll
    for (int k = 0; k < DMAX; ++k) {
        // Eq. 8, saturated to the soft-value range
        s16x2 vk = vmin2(vmax2(__builtin_elementwise_sub_sat(e[k], lk[k]), splat2(-ACC)), splat2(ACC));
        u16x2 pk = as_u(vmin2(vmax2(vk, -vk), as_s(mm)));
        if (k >= DMIN && k >= d) {
            vk = splat2(0);
            pk = usplat2(kPad);
        }
        v[k] = vk;
        par ^= vk;
        p[k] = pk;
    }
    cn_fold_x2<DMAX, RULE>(p, m);
#pragma unroll
    for (int k = 0; k < DMAX; ++k) {
        if (k < DMIN || k < d) {
            s16x2 mg = as_s(m[k]);
            if (off_row)
                mg = vmin2(vmax2(mg - splat2(ldc(off_row, o + k)), splat2(0)), as_s(mm));
            const s16x2 sg = (par ^ v[k]) >> (short)15;  // -1 in a half whose message is negative
            const s16x2 ln = (mg ^ sg) - sg;
            // Eq. 9 under Alg. 2: halves whose stored |E| is E_max keep E
            const s16x2 ne = vmin2(vmax2(__builtin_elementwise_add_sat(v[k], ln), -em), em);
            const s16x2 ae = vmax2(e[k], -e[k]);
            const s16x2 frozen = vmin2(em - ae, splat2(1)) - splat2(1);  // -1 where |E| == E_max
            const s16x2 out = (frozen & e[k]) | (~frozen & ne);
            const int a0 = a0s[k];
            E[a0] = (ET)out.x;
            E[pair_second<POW2>(C, o + k, a0)] = (ET)out.y;
            Lt[2 * k] = (int8_t)ln.x;
            Lt[2 * k + 1] = (int8_t)ln.y;
        }
    }
}

// packed syndrome bits of rows i and i + Z/2, as sign bits of the halves
__device__ __forceinline__ s16x2 syn_pair(const uint8_t *__restrict__ s_syn, int i0, int i1)
{
    s16x2 s;
    s.x = (short)-(int)((s_syn[i0 >> 3] >> (i0 & 7)) & 1);
    s.y = (short)-(int)((s_syn[i1 >> 3] >> (i1 & 7)) & 1);
    return s;
}

template <int DMIN, int DMAX, typename ET, bool POW2>
__device__ __forceinline__ int rows_unsat_x2(const DevCode &C, const ET *__restrict__ E,
                                             const uint8_t *__restrict__ s_syn, int tid, int nthr)
{
    const int z = C.z, h = z >> 1;
    s16x2 any = splat2(0);
    for (int b = 0; b < C.mb; ++b) {
        const int d = ldc(C.deg, b), o = ldc(C.blk_off, b);
        for (int r = tid; r < h; r += nthr) {
            s16x2 acc = syn_pair(s_syn, b * z + r, b * z + r + h);
            s16x2 x[DMAX];
#pragma unroll
            for (int k = 0; k < DMAX; ++k) {
                const int kk = k < DMIN ? k : (k < d ? k : d - 1);
                const int a0 = pair_first<POW2>(C, o + kk, r);
                x[k] = load_pair(E, a0, pair_second<POW2>(C, o + kk, a0));
            }
#pragma unroll
            for (int k = 0; k < DMAX; ++k)
                if (k < DMIN || k < d)
                    acc ^= x[k];
            any |= acc;
        }
    }
    return (any.x | any.y) < 0;
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

template <int DMIN, int DMAX, typename ET, int RULE, bool POW2>
__global__ __launch_bounds__(512) void k_decode_frame_x2(DevCode C, DecodeArgs A)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const int f = blockIdx.x;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int z = C.z, n = C.n, h = z >> 1, nb2 = 2 * C.n_blocks;
    ET *E = reinterpret_cast<ET *>(smem);  // the host places E at offset 0
    int8_t *L = reinterpret_cast<int8_t *>(smem + A.lds_l_off);
    uint8_t *s_syn = smem + A.lds_syn_off;
    int *flags = reinterpret_cast<int *>(smem + A.lds_flag_off);
    const int S = A.l_stride;

    // stage in
    const uint8_t *syn = A.syn + (size_t)f * A.syn_bytes;
    for (int i = tid; i < A.syn_bytes; i += nthr)
        s_syn[i] = syn[i];
    const int8_t *llr = A.llr + (size_t)f * n;
    const int lim0 = C.e_max < 127 ? C.e_max : 127;
    for (int j = tid; j < n; j += nthr)
        E[j] = (ET)clampi(llr[j], -lim0, lim0);
    for (int r = tid; r < h; r += nthr)
        for (int q = 0; q < nb2; ++q)
            L[r * S + q] = 0;
    if (tid < 2)
        flags[tid] = 0;
    __syncthreads();

    int conv = !block_any(rows_unsat_x2<DMIN, DMAX, ET, POW2>(C, E, s_syn, tid, nthr), flags, 0);
    int iters = 0;
    for (int t = 1; t <= A.max_iter && !conv; ++t) {
        const int32_t *off_row = nullptr;
        if (C.offsets)
            off_row = C.offsets + (size_t)(t - 1 < C.offset_iters - 1 ? t - 1 : C.offset_iters - 1) * C.n_blocks;
        for (int b = 0; b < C.mb; ++b) {
            const int d = ldc(C.deg, b), o = ldc(C.blk_off, b);
            for (int r = tid; r < h; r += nthr)
                row_update_x2<DMIN, DMAX, ET, RULE, POW2>(C, E, L + r * S + 2 * o, o, d, r,
                                                          syn_pair(s_syn, b * z + r, b * z + r + h), off_row);
            __syncthreads();
        }
        iters = t;
        conv = !block_any(rows_unsat_x2<DMIN, DMAX, ET, POW2>(C, E, s_syn, tid, nthr), flags, t & 1);
    }
    if (!conv)
        iters = A.max_iter;

    // stage out: hard decisions (wavefront ballot), flags, optional state
    const int lane = tid & 63, wv = tid >> 6, nwv = nthr >> 6;
    const int nwords = (n + 63) >> 6;
    uint8_t *ob = A.out_bits + (size_t)f * A.bit_bytes;
    for (int w = wv; w < nwords; w += nwv) {
        const int j = (w << 6) + lane;
        const bool neg = j < n && E[j] < 0;
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
    if (A.out_L) {
        // canonical [block][row] layout
        const int ne = C.n_blocks * z;
        for (int e = tid; e < ne; e += nthr) {
            const int blk = e / z, row = e - blk * z;
            const int half = row >= h, r = row - half * h;
            A.out_L[(size_t)f * ne + e] = L[r * S + 2 * blk + half];
        }
    }
    if (A.out_E)
        for (int j = tid; j < n; j += nthr)
            A.out_E[(size_t)f * n + j] = (int16_t)E[j];
}

// ---------------------------------------------------------------------------
// Split variant: two adjacent lanes share a row pair, so a frame of Z = 1024
// runs 16 waves per CU instead of 8. Both lanes execute the same code. Lane A
// (even) holds edges 0 .. DH-1 of the row pair in order, lane B (odd) holds
// edges DMAX-1 down to DH, so a left fold over a lane's own slots is the
// forward partial F for A and the backward partial B for B. One lane swap
// hands A the value B_DH and B the value F_{DH-1}; each lane then folds its
// slots the other way, W_k, and its outputs are out_i = tau(X_{i-1}, W_{DH-1-i})
// with out_0 = W_{DH-1}, which is the forward-backward fold edge by edge.
//
// Per-lane slot entries {c*Z | shift, LDS address of block column c, pad mask,
// block} sit in LDS; padding slots point at a dummy block column past E, so
// they need no store guards, and their operands are masked to 0 / kPad. E is
// addressed with absolute LDS addresses (the table holds them), so no base is
// added per access. L of a row pair is laid out [layer][half][slot][lane].
//
// When every row pair has its own lane pair (Z/2 <= threads/2), the syndrome
// test of the state after iteration t-1 is folded into layer 0 of iteration t:
// layer 0 reads exactly that state, so its rows' parities come from the
// loaded values; only when all of them hold are the other layers tested,
// before layer 0 writes anything.
// ---------------------------------------------------------------------------

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
    return ((((unsigned)r + (unsigned)te.x) & zm) << esh) | (unsigned)te.y;
}

template <int DH>
struct SplitRow {
    s16x2 e[DH], lk[DH];
    unsigned a0[DH];
    int pm[DH];
};

template <int DMIN, int DMAX, typename ET>
__device__ __forceinline__ void split_load(SplitRow<DMAX / 2> &R, const int8_t *__restrict__ Lp,
                                           const int4 *__restrict__ tab, int r, unsigned zm, unsigned hzb)
{
    constexpr int DH = DMAX / 2;
    constexpr unsigned esh = sizeof(ET) == 2 ? 1 : 0;
#pragma unroll
    for (int i = 0; i < DH; ++i) {
        const int4 te = tab[2 * i];
        const unsigned a0 = slot_addr(te, r, zm, esh);
        R.a0[i] = a0;
        R.pm[i] = te.z;
        s16x2 ev;
        ev.x = (short)lds_ld<ET>(a0);
        ev.y = (short)lds_ld<ET>(a0 ^ hzb);
        R.e[i] = ev;
        s16x2 lv;
        lv.x = (short)Lp[2 * i];
        lv.y = (short)Lp[2 * DH + 2 * i];
        R.lk[i] = lv;
    }
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

template <int DMIN, int DMAX, typename ET, int RULE>
__device__ __forceinline__ void split_finish(const DevCode &C, const SplitRow<DMAX / 2> &R, int8_t *__restrict__ Lp,
                                             s16x2 syn, unsigned hzb)
{
    constexpr int DH = DMAX / 2;
    constexpr int ACC = AccLim<ET>::value;
    const s16x2 em = splat2(C.e_max);
    const u16x2 mm = usplat2(C.msg_max);
    s16x2 v[DH];
    u16x2 p[DH], X[DH], W[DH];
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
#pragma unroll
    for (int i = 0; i < DH; ++i) {
        const s16x2 sg = (par ^ v[i]) >> (short)15;  // -1 in a half whose message is negative
        const s16x2 mg = as_s(out[i]);
        const s16x2 ln = (mg ^ sg) - sg;
        // Eq. 9 under Alg. 2: halves whose stored |E| is E_max keep E
        const s16x2 ne = vmin2(vmax2(__builtin_elementwise_add_sat(v[i], ln), -em), em);
        const s16x2 ae = vmax2(R.e[i], -R.e[i]);
        const s16x2 frozen = vmin2(em - ae, splat2(1)) - splat2(1);
        const s16x2 o = (frozen & R.e[i]) | (~frozen & ne);
        lds_st<ET>(R.a0[i], (ET)o.x);
        lds_st<ET>(R.a0[i] ^ hzb, (ET)o.y);
        Lp[2 * i] = (int8_t)ln.x;
        Lp[2 * DH + 2 * i] = (int8_t)ln.y;
    }
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
            x[i].x = (short)lds_ld<ET>(a0);
            x[i].y = (short)lds_ld<ET>(a0 ^ hzb);
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

template <int DMIN, int DMAX, typename ET, int RULE>
__global__ __launch_bounds__(1024) void k_decode_frame_split(DevCode C, DecodeArgs A)
{
    constexpr int DH = DMAX / 2;
    constexpr unsigned esh = sizeof(ET) == 2 ? 1 : 0;
    extern __shared__ __align__(16) uint8_t smem[];
    const int f = blockIdx.x;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int z = C.z, n = C.n, hz = z >> 1, h = tid & 1;
    const unsigned zm = (unsigned)(z - 1), hzb = (unsigned)hz << esh;
    ET *E = reinterpret_cast<ET *>(smem);  // E (plus one dummy block column) at offset 0
    int8_t *L = reinterpret_cast<int8_t *>(smem + A.lds_l_off);
    uint8_t *s_syn = smem + A.lds_syn_off;
    int4 *s_tab = reinterpret_cast<int4 *>(smem + A.lds_tab_off);
    int *flags = reinterpret_cast<int *>(smem + A.lds_flag_off);
    const int S = A.l_stride;
    const unsigned ebase = (unsigned)(uintptr_t)E;
    // The slot addresses OR a column start into a row offset, which needs E to
    // start at a multiple of Z elements; this kernel uses no static LDS, so the
    // dynamic area starts at 0. Report a frame as not decoded otherwise.
    if (ebase & ((unsigned)(z << esh) - 1)) {
        if (tid == 0) {
            A.out_conv[f] = 0;
            if (A.out_iters)
                A.out_iters[f] = -1;
        }
        return;
    }

    // stage in: syndrome, E, L = 0, lane table with absolute column addresses, vote words
    const uint8_t *syn = A.syn + (size_t)f * A.syn_bytes;
    for (int i = tid; i < A.syn_bytes; i += nthr)
        s_syn[i] = syn[i];
    const int8_t *llr = A.llr + (size_t)f * n;
    const int lim0 = C.e_max < 127 ? C.e_max : 127;
    for (int j = tid; j < n; j += nthr)
        E[j] = (ET)clampi(llr[j], -lim0, lim0);
    int *L32 = reinterpret_cast<int *>(L);
    for (int w = tid; w < (hz * S) >> 2; w += nthr)
        L32[w] = 0;
    for (int q = tid; q < C.mb * DH * 2; q += nthr) {
        int4 te = A.lane_tab[q];
        te.y = (int)(((unsigned)te.y << esh) + ebase);
        s_tab[q] = te;
    }
    if (tid < 3)
        flags[tid] = 0;
    __syncthreads();

    int vk = 0;
    int conv, iters = 0;
    if (hz <= (nthr >> 1)) {
        // one row pair per lane pair: the check is folded into layer 0
        const int r = tid >> 1;
        const bool act = r < hz;
        int8_t *Lr = L + r * S + h;
        conv = !block_vote(act ? split_rows_unsat<DMIN, DMAX, ET>(C, s_syn, s_tab, h, r, 0, C.mb) : 0, flags, vk);
        for (int t = 1; t <= A.max_iter && !conv; ++t) {
            {
                SplitRow<DH> R;
                const s16x2 syn0 = act ? syn_pair(s_syn, r, r + hz) : splat2(0);
                if (act)
                    split_load<DMIN, DMAX, ET>(R, Lr, s_tab + h, r, zm, hzb);
                if (t >= 2) {
                    int fail0 = 0;
                    if (act) {
                        const s16x2 own = split_e_parity<DMIN, DMAX>(R);
                        const s16x2 pe = syn0 ^ own ^ swap_pair(own);
                        fail0 = (pe.x | pe.y) < 0;
                    }
                    if (!block_vote(fail0, flags, vk)) {
                        const int failr = act ? split_rows_unsat<DMIN, DMAX, ET>(C, s_syn, s_tab, h, r, 1, C.mb) : 0;
                        if (!block_vote(failr, flags, vk)) {
                            conv = 1;
                            iters = t - 1;
                            break;
                        }
                    }
                }
                if (act)
                    split_finish<DMIN, DMAX, ET, RULE>(C, R, Lr, syn0, hzb);
                __syncthreads();
            }
            for (int b = 1; b < C.mb; ++b) {
                if (act) {
                    SplitRow<DH> R;
                    int8_t *Lb = Lr + b * 4 * DH;
                    split_load<DMIN, DMAX, ET>(R, Lb, s_tab + b * DH * 2 + h, r, zm, hzb);
                    split_finish<DMIN, DMAX, ET, RULE>(C, R, Lb, syn_pair(s_syn, b * z + r, b * z + r + hz), hzb);
                }
                __syncthreads();
            }
            iters = t;
        }
        if (!conv && A.max_iter > 0)
            conv = !block_vote(act ? split_rows_unsat<DMIN, DMAX, ET>(C, s_syn, s_tab, h, r, 0, C.mb) : 0, flags,
                               vk);
    } else {
        // several row pairs per lane pair: separate check after every iteration
        auto unsat_all = [&]() {
            int u = 0;
            for (int r = tid >> 1; r < hz; r += nthr >> 1)
                u |= split_rows_unsat<DMIN, DMAX, ET>(C, s_syn, s_tab, h, r, 0, C.mb);
            return u;
        };
        conv = !block_vote(unsat_all(), flags, vk);
        for (int t = 1; t <= A.max_iter && !conv; ++t) {
            for (int b = 0; b < C.mb; ++b) {
                for (int r = tid >> 1; r < hz; r += nthr >> 1) {
                    SplitRow<DH> R;
                    int8_t *Lb = L + r * S + h + b * 4 * DH;
                    split_load<DMIN, DMAX, ET>(R, Lb, s_tab + b * DH * 2 + h, r, zm, hzb);
                    split_finish<DMIN, DMAX, ET, RULE>(C, R, Lb, syn_pair(s_syn, b * z + r, b * z + r + hz), hzb);
                }
                __syncthreads();
            }
            iters = t;
            conv = !block_vote(unsat_all(), flags, vk);
        }
    }
    if (!conv)
        iters = A.max_iter;

    // stage out: hard decisions (wavefront ballot), flags, optional state
    const int lane = tid & 63, wv = tid >> 6, nwv = nthr >> 6;
    const int nwords = (n + 63) >> 6;
    uint8_t *ob = A.out_bits + (size_t)f * A.bit_bytes;
    for (int w = wv; w < nwords; w += nwv) {
        const int j = (w << 6) + lane;
        const bool neg = j < n && E[j] < 0;
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
    if (A.out_L) {
        // canonical [block][row] layout
        const int ne = C.n_blocks * z;
        for (int e = tid; e < ne; e += nthr) {
            const int blk = e / z, row = e - blk * z;
            const int half = row >= hz, r = row - half * hz;
            A.out_L[(size_t)f * ne + e] = L[r * S + A.blk2slot[blk] + half * 2 * DH];
        }
    }
    if (A.out_E)
        for (int j = tid; j < n; j += nthr)
            A.out_E[(size_t)f * n + j] = (int16_t)E[j];
}

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

namespace {

template <int DMAX, typename ET, int RULE, bool LDS>
hipError_t launch_one(const DevCode &C, const DecodeArgs &A, int threads, size_t lds, hipStream_t s)
{
    auto kern = k_decode_frame<DMAX, ET, RULE, LDS>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(kern, dim3(A.n_frames), dim3(threads), lds, s, C, A);
    return hipGetLastError();
}

template <int DMIN, int DMAX, typename ET, int RULE, bool POW2>
hipError_t launch_one_x2(const DevCode &C, const DecodeArgs &A, int threads, size_t lds, hipStream_t s)
{
    auto kern = k_decode_frame_x2<DMIN, DMAX, ET, RULE, POW2>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(kern, dim3(A.n_frames), dim3(threads), lds, s, C, A);
    return hipGetLastError();
}

template <int DMIN, int DMAX, typename ET, bool POW2>
hipError_t launch_rule_x2(int rule, const DevCode &C, const DecodeArgs &A, int threads, size_t lds, hipStream_t s)
{
    switch (rule) {
    case LDPC_RULE_RCBP_EQ7:
        return launch_one_x2<DMIN, DMAX, ET, LDPC_RULE_RCBP_EQ7, POW2>(C, A, threads, lds, s);
    case LDPC_RULE_MINSUM:
        return launch_one_x2<DMIN, DMAX, ET, LDPC_RULE_MINSUM, POW2>(C, A, threads, lds, s);
    default:
        return launch_one_x2<DMIN, DMAX, ET, LDPC_RULE_RCBP_FB, POW2>(C, A, threads, lds, s);
    }
}

// Degree variants: DMAX bounds the row degree; rows shorter than DMIN... DMAX are
// padded, rows of degree >= DMIN need no per-slot test below DMIN.
template <typename ET, bool POW2>
hipError_t launch_deg_x2(int min_deg, int max_deg, int rule, const DevCode &C, const DecodeArgs &A, int threads,
                         size_t lds, hipStream_t s)
{
    if (max_deg <= 8)
        return min_deg >= 6 ? launch_rule_x2<6, 8, ET, POW2>(rule, C, A, threads, lds, s)
                            : launch_rule_x2<2, 8, ET, POW2>(rule, C, A, threads, lds, s);
    if (max_deg <= 20)
        return min_deg >= 19 ? launch_rule_x2<19, 20, ET, POW2>(rule, C, A, threads, lds, s)
                             : launch_rule_x2<2, 20, ET, POW2>(rule, C, A, threads, lds, s);
    return launch_rule_x2<2, 32, ET, POW2>(rule, C, A, threads, lds, s);
}

template <typename ET>
hipError_t launch_x2(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s)
{
    if (P.pow2)
        return launch_deg_x2<ET, true>(P.min_deg, P.max_deg, P.cn_rule, C, A, P.threads, P.lds_bytes, s);
    return launch_deg_x2<ET, false>(P.min_deg, P.max_deg, P.cn_rule, C, A, P.threads, P.lds_bytes, s);
}

template <int DMIN, int DMAX, typename ET, int RULE>
hipError_t launch_one_split(const DevCode &C, const DecodeArgs &A, int threads, size_t lds, hipStream_t s)
{
    auto kern = k_decode_frame_split<DMIN, DMAX, ET, RULE>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(kern, dim3(A.n_frames), dim3(threads), lds, s, C, A);
    return hipGetLastError();
}

template <int DMIN, int DMAX, typename ET>
hipError_t launch_rule_split(int rule, const DevCode &C, const DecodeArgs &A, int threads, size_t lds,
                             hipStream_t s)
{
    if (rule == LDPC_RULE_MINSUM)
        return launch_one_split<DMIN, DMAX, ET, kRuleMinSum>(C, A, threads, lds, s);
    return launch_one_split<DMIN, DMAX, ET, kRuleRcbpFB>(C, A, threads, lds, s);
}

template <typename ET>
hipError_t launch_split(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s)
{
    switch (P.split_dmax) {
    case 8:
        return P.min_deg >= 6 ? launch_rule_split<6, 8, ET>(P.cn_rule, C, A, P.threads, P.lds_bytes, s)
                              : launch_rule_split<2, 8, ET>(P.cn_rule, C, A, P.threads, P.lds_bytes, s);
    default:
        return P.min_deg >= 19 ? launch_rule_split<19, 20, ET>(P.cn_rule, C, A, P.threads, P.lds_bytes, s)
                               : launch_rule_split<2, 20, ET>(P.cn_rule, C, A, P.threads, P.lds_bytes, s);
    }
}

template <int DMAX, typename ET, bool LDS>
hipError_t launch_rule(int rule, const DevCode &C, const DecodeArgs &A, int threads, size_t lds, hipStream_t s)
{
    switch (rule) {
    case LDPC_RULE_RCBP_EQ7:
        return launch_one<DMAX, ET, LDPC_RULE_RCBP_EQ7, LDS>(C, A, threads, lds, s);
    case LDPC_RULE_MINSUM:
        return launch_one<DMAX, ET, LDPC_RULE_MINSUM, LDS>(C, A, threads, lds, s);
    default:
        return launch_one<DMAX, ET, LDPC_RULE_RCBP_FB, LDS>(C, A, threads, lds, s);
    }
}

template <typename ET, bool LDS>
hipError_t launch_deg(int max_deg, int rule, const DevCode &C, const DecodeArgs &A, int threads, size_t lds,
                      hipStream_t s)
{
    if (max_deg <= 8)
        return launch_rule<8, ET, LDS>(rule, C, A, threads, lds, s);
    if (max_deg <= 20)
        return launch_rule<20, ET, LDS>(rule, C, A, threads, lds, s);
    return launch_rule<32, ET, LDS>(rule, C, A, threads, lds, s);
}

} // namespace

hipError_t launch_decode(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s)
{
    if (P.split_dmax)
        return P.acc_bits == 16 ? launch_split<int16_t>(P, C, A, s) : launch_split<int8_t>(P, C, A, s);
    if (P.pairs)
        return P.acc_bits == 16 ? launch_x2<int16_t>(P, C, A, s) : launch_x2<int8_t>(P, C, A, s);
    if (P.acc_bits == 16) {
        if (P.lds_state)
            return launch_deg<int16_t, true>(P.max_deg, P.cn_rule, C, A, P.threads, P.lds_bytes, s);
        return launch_deg<int16_t, false>(P.max_deg, P.cn_rule, C, A, P.threads, P.lds_bytes, s);
    }
    if (P.lds_state)
        return launch_deg<int8_t, true>(P.max_deg, P.cn_rule, C, A, P.threads, P.lds_bytes, s);
    return launch_deg<int8_t, false>(P.max_deg, P.cn_rule, C, A, P.threads, P.lds_bytes, s);
}

hipError_t launch_syndrome(const DevCode &C, const uint8_t *bits, int n_frames, uint8_t *out_syn, hipStream_t s)
{
    const int bit_bytes = (C.n + 7) / 8, syn_bytes = (C.m + 7) / 8;
    const int threads = 256;
    dim3 grid((C.m + threads - 1) / threads, n_frames);
    hipLaunchKernelGGL(k_syndrome, grid, dim3(threads), 0, s, C, bits, bit_bytes, out_syn, syn_bytes);
    return hipGetLastError();
}

} // namespace qkdldpc
