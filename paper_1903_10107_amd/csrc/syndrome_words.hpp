// Word-parallel syndrome rows for codes with Z a multiple of 32 (shared by
// Alice's syndrome encoder and the decode-order kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace qkdldpc {

// Word-parallel form for Z a multiple of 32. Block b of s is the XOR over its
// nonzero base entries of the column block x_c cyclically rotated by the shift:
// s[bZ + r] ^= x[cZ + (r + s) mod Z]. With Z = 32 W, output word k of a block
// takes bits 32 k + s .. 32 k + s + 31 (mod Z) of x_c, i.e. words (k + s/32) and
// (k + s/32 + 1) mod W funnel-shifted right by s mod 32: one alignbit and one XOR
// per block and 32 syndrome bits, instead of 32 single-bit gathers.
//
// The code's tables are staged in LDS first, per workgroup: for every nonzero
// block, int2{word index of its column block in x, (s mod 32) | (s / 32) << 5},
// and for every base row int2{first block, degree}.
__device__ __forceinline__ void stage_syndrome_tables(const DevCode &C, int2 *tab, int2 *rows, int tid, int nthr)
{
    for (int e = tid; e < C.n_blocks; e += nthr) {
        const int sh = C.shift[e];
        tab[e] = make_int2(C.colbase[e] >> 5, (sh & 31) | (sh >> 5) << 5);
    }
    for (int b = tid; b < C.mb; b += nthr)
        rows[b] = make_int2(C.blk_off[b], C.deg[b]);
}

// Syndrome word w of one frame.
__device__ __forceinline__ uint32_t syndrome_word(const int2 *tab, const int2 *rows, int wz, const uint32_t *x, int w)
{
    const int b = w / wz, k = w - b * wz;
    const int2 r = rows[b];
    uint32_t acc = 0;
#pragma unroll 4
    for (int e = r.x; e < r.x + r.y; ++e) {
        const int2 t = tab[e];
        int u = k + (t.y >> 5);
        u = u >= wz ? u - wz : u;
        const int u1 = u + 1 == wz ? 0 : u + 1;
        acc ^= __builtin_amdgcn_alignbit(x[t.x + u1], x[t.x + u], (uint32_t)(t.y & 31));
    }
    return acc;
}

} // namespace qkdldpc
