// gfx950 decode kernel, one lane per row pair (r, r + Z/2), 16-bit packed
// arithmetic, state in LDS. Used for even Z that is not a power of two, row
// degrees above 20, the literal Eq. 7 fold order, and per-iteration offsets.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace qkdldpc {

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
    stage_llr<ET>(E, A.llr + (size_t)f * n, n, C.e_max < 127 ? C.e_max : 127, tid, nthr);
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

namespace {

template <int DMIN, int DMAX, typename ET, int RULE, bool POW2>
hipError_t launch_one_x2(const DevCode &C, const DecodeArgs &A, int threads, size_t lds, hipStream_t s)
{
    auto kern = k_decode_frame_x2<DMIN, DMAX, ET, RULE, POW2>;
    if (lds > 65536) {
        hipError_t e = allow_max_lds<k_decode_frame_x2<DMIN, DMAX, ET, RULE, POW2>>();
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

} // namespace

hipError_t launch_decode_pairs(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s)
{
    return P.acc_bits == 16 ? launch_x2<int16_t>(P, C, A, s) : launch_x2<int8_t>(P, C, A, s);
}

} // namespace qkdldpc
