// Host-side model of a quasi-cyclic LDPC code (Sec. 4.1 of arXiv:1903.10107:
// an Mb x Nb base matrix whose entries are Z x Z cyclically shifted identities
// or zero blocks) and the device tables the kernels read.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qkdldpc.h"

namespace qkdldpc {

constexpr int kMaxRowDegree = 32;

// Device-side view of a code, passed by value to the kernels. Per-layer and
// per-block entries are uniform across a workgroup, so the kernels read them
// with scalar loads.
struct DevCode {
    const int32_t *deg;      // [mb] nonzero blocks of base row b
    const int32_t *blk_off;  // [mb] index of base row b's first block
    const int32_t *colbase;  // [n_blocks] c * Z of each block, row-major block order
    const int32_t *shift;    // [n_blocks] circulant shift of each block
    const int32_t *colshift; // [n_blocks] c * Z | shift (meaningful when Z is a power of two)
    const int32_t *offsets;  // [offset_iters][n_blocks] or nullptr (int32 so that reads are scalar loads)
    int32_t offset_iters;
    int32_t mb, nb, z, n, m, n_blocks;
    int32_t msg_max, e_max;
};

struct HostCode {
    int32_t mb = 0, nb = 0, z = 0, n = 0, m = 0, n_blocks = 0, min_deg = 0, max_deg = 0;
    int64_t n_edges = 0;
    int32_t has_4cycles = 0;
    int32_t msg_max = 63, e_max = 127, acc_bits = 8, cn_rule = 0, offset_iters = 0, kernel_hint = 0;
    std::vector<int32_t> deg, blk_off, colbase, shift;
    std::vector<int8_t> offsets;
};

// Validates the arguments of ldpc_code_create and fills `out`. Returns an LDPC_*
// code and a message in `err` on failure. Touches no device.
int build_host_code(const int32_t *base, int32_t mb, int32_t nb, int32_t z, const ldpc_params *p,
                    HostCode &out, std::string &err);

} // namespace qkdldpc
