// gfx950 decode kernels, one lane per row (32-bit arithmetic): state in LDS or,
// when it does not fit, in a global-memory workspace slice per frame.
//
// One workgroup decodes one frame from start to finish: stage in, pre-check,
// every iteration (all layers, then the syndrome test), stage out. Thread t
// owns rows t, t + T, ... of every layer; the rows of one layer touch disjoint
// variable nodes (one circulant per base entry), so a layer needs no atomics,
// only a workgroup barrier before the next layer reads what it wrote.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace qkdldpc {

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
    stage_llr<ET>(E, A.llr + (size_t)f * n, n, C.e_max < 127 ? C.e_max : 127, tid, nthr);
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
    const int z = C.z;
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

namespace {

template <int DMAX, typename ET, int RULE, bool LDS>
hipError_t launch_one(const DevCode &C, const DecodeArgs &A, int threads, size_t lds, hipStream_t s)
{
    auto kern = k_decode_frame<DMAX, ET, RULE, LDS>;
    if (lds > 65536) {
        hipError_t e = allow_max_lds<k_decode_frame<DMAX, ET, RULE, LDS>>();
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(kern, dim3(A.n_frames), dim3(threads), lds, s, C, A);
    return hipGetLastError();
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

hipError_t launch_decode_scalar(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s)
{
    if (P.acc_bits == 16) {
        if (P.lds_state)
            return launch_deg<int16_t, true>(P.max_deg, P.cn_rule, C, A, P.threads, P.lds_bytes, s);
        return launch_deg<int16_t, false>(P.max_deg, P.cn_rule, C, A, P.threads, P.lds_bytes, s);
    }
    if (P.lds_state)
        return launch_deg<int8_t, true>(P.max_deg, P.cn_rule, C, A, P.threads, P.lds_bytes, s);
    return launch_deg<int8_t, false>(P.max_deg, P.cn_rule, C, A, P.threads, P.lds_bytes, s);
}

} // namespace qkdldpc
