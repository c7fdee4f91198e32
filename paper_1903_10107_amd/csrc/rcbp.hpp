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

__host__ __device__ __forceinline__ int clampi(int v, int lo, int hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

} // namespace qkdldpc
