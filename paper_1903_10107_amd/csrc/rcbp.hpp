// Check-node and variable-node arithmetic of the quantized layered decoder,
// shared by the gfx950 kernels and by the host self-description export.
//
// All magnitudes handed to tau are already clipped to MSG_max (the VN->CN
// magnitudes are min(|L_ji|, MSG_max), and tau never exceeds the smaller of its
// operands), so the MSG_max clip at the top of Alg. 1 (Sec. 3.2) is a no-op here.
#pragma once

#include <hip/hip_runtime.h>

namespace qkdldpc {

// Alg. 1 in branch-free form. With l = min(a, b), g = max(a, b), d = g - l:
//   l > 2 :  tau = l - [d < 2] - [d < 6]
//   l <= 2:  tau = max(l - [d < 4], 0)
// Both corrections are max((K - d) >> 2, 0) with K = 9 (l > 2) or K = 7 (l <= 2):
// (9 - d) >> 2 is 2 for d in {0, 1}, 1 for d in 2..5, <= 0 from d = 6 on;
// (7 - d) >> 2 is 1 for d in 0..3 and <= 0 from d = 4 on. The result is then
// clamp(l - y, 0, l), which is max(l - max(y, 0), 0).
__host__ __device__ __forceinline__ int tau(int a, int b)
{
    const int g = a > b ? a : b;
    const int l = a < b ? a : b;
    const int k = l > 2 ? 9 : 7;
    const int y = (l - g + k) >> 2;
    int t = l - y;
    t = t < 0 ? 0 : t;
    return t > l ? l : t;
}

// Two 16-bit lanes per 32-bit register (v_pk_* instructions on gfx950).
typedef short s16x2 __attribute__((ext_vector_type(2)));

__host__ __device__ __forceinline__ s16x2 vmin2(s16x2 a, s16x2 b) { return __builtin_elementwise_min(a, b); }
__host__ __device__ __forceinline__ s16x2 vmax2(s16x2 a, s16x2 b) { return __builtin_elementwise_max(a, b); }
__host__ __device__ __forceinline__ s16x2 splat2(int v) { return (s16x2)((short)v); }

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__host__ __device__ __forceinline__ u16x2 umin2(u16x2 a, u16x2 b) { return __builtin_elementwise_min(a, b); }
__host__ __device__ __forceinline__ u16x2 umax2(u16x2 a, u16x2 b) { return __builtin_elementwise_max(a, b); }
__host__ __device__ __forceinline__ u16x2 usat_sub2(u16x2 a, u16x2 b) { return __builtin_elementwise_sub_sat(a, b); }
__host__ __device__ __forceinline__ u16x2 usplat2(int v) { return (u16x2)((unsigned short)v); }

// Alg. 1 on two operand pairs at once, with unsigned saturating arithmetic.
// With l = min, d = max - min: K = med3(3l, 7, 9) is 7 for l in {1, 2} and 9 for
// l >= 3 (for l = 0 the result is 0 whatever K is); the correction is
// c = max(K - d, 0) >> 2 and tau = max(l - c, 0). Equal to tau() above on
// [0, 63]^2; with one operand >= the other + 6 (for instance the padding value
// 8191) the result is exactly the smaller operand.
__host__ __device__ __forceinline__ u16x2 tau2(u16x2 a, u16x2 b)
{
    const u16x2 l = umin2(a, b);
    const u16x2 d = umax2(a, b) - l;
    const u16x2 k = umax2(umin2(l * (unsigned short)3, usplat2(9)), usplat2(7));
    return usat_sub2(l, usat_sub2(k, d) >> (unsigned short)2);
}

// Operand used to pad a row of degree d < DMAX up to DMAX. It is neutral for
// every rule below when the real operands are at most 127: tau(x, PAD) = x,
// min(x, PAD) = x, and right folds over padding stay above PAD - 2 * 32.
constexpr unsigned short kPad = 8191;

enum { kRuleRcbpFB = 0, kRuleRcbpEq7 = 1, kRuleMinSum = 2 };

// Magnitudes of the CN->VN messages of a row pair, over DMAX operands (real
// ones first, then padding): for every k, the box-plus of Eq. 4 over all
// operands but k, under the rule's fold order.
template <int DMAX, int RULE>
__host__ __device__ __forceinline__ void cn_fold_x2(const u16x2 (&p)[DMAX], u16x2 (&m)[DMAX])
{
    if constexpr (RULE == kRuleMinSum) {
        // min1 / min2; the output to edge k is min2 where p_k equals min1, else min1
        u16x2 m1 = usplat2(0x7fff), m2 = usplat2(0x7fff);
#pragma unroll
        for (int k = 0; k < DMAX; ++k) {
            m2 = umin2(m2, umax2(m1, p[k]));
            m1 = umin2(m1, p[k]);
        }
        const u16x2 diff = m2 - m1;
#pragma unroll
        for (int k = 0; k < DMAX; ++k) {
            const u16x2 u = umin2(p[k] - m1, usplat2(1));  // 0 where p_k is the minimum
            m[k] = m2 - u * diff;
        }
    } else if constexpr (RULE == kRuleRcbpEq7) {
        // literal Eq. 7: S_k = tau(p_k, S_{k+1});
        // output k = tau(p_0, tau(p_1, ... tau(p_{k-1}, S_{k+1})))
        u16x2 S[DMAX];
        S[DMAX - 1] = p[DMAX - 1];
#pragma unroll
        for (int k = DMAX - 2; k >= 0; --k)
            S[k] = tau2(p[k], S[k + 1]);
#pragma unroll
        for (int k = 0; k < DMAX - 1; ++k) {
            u16x2 acc = S[k + 1];
#pragma unroll
            for (int i = k - 1; i >= 0; --i)
                acc = tau2(p[i], acc);
            m[k] = acc;
        }
        u16x2 acc = p[DMAX - 2];
#pragma unroll
        for (int i = DMAX - 3; i >= 0; --i)
            acc = tau2(p[i], acc);
        m[DMAX - 1] = acc;
    } else {
        // forward-backward: F_0 = p_0, F_k = tau(F_{k-1}, p_k); B_{D-1} = p_{D-1},
        // B_k = tau(p_k, B_{k+1}); out_0 = B_1, out_{D-1} = F_{D-2},
        // out_k = tau(F_{k-1}, B_{k+1}). F lives in m[] and is overwritten from the
        // top down by the outputs once consumed.
        m[0] = p[0];
#pragma unroll
        for (int k = 1; k < DMAX - 1; ++k)
            m[k] = tau2(m[k - 1], p[k]);
        u16x2 B = p[DMAX - 1];
        m[DMAX - 1] = m[DMAX - 2];
#pragma unroll
        for (int k = DMAX - 2; k >= 1; --k) {
            const u16x2 out = tau2(m[k - 1], B);
            B = tau2(p[k], B);
            m[k] = out;
        }
        m[0] = B;
    }
}

__host__ __device__ __forceinline__ int clampi(int v, int lo, int hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

} // namespace qkdldpc
