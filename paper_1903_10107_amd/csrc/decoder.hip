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
