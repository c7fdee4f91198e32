// Launch interface between the C ABI and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "qc_code.hpp"

namespace qkdldpc {

struct DecodeArgs {
    const uint8_t *syn;   // [F][syn_bytes]
    const int8_t *llr;    // [F][n]
    int n_frames;
    int max_iter;
    uint8_t *out_bits;    // [F][bit_bytes]
    uint8_t *out_conv;    // [F]
    int32_t *out_iters;   // [F] or nullptr
    int8_t *out_L;        // [F][n_blocks][z] or nullptr
    int16_t *out_E;       // [F][n] or nullptr
    uint8_t *ws;          // global-memory state when it does not fit in LDS
    size_t ws_frame_bytes;
    size_t ws_l_off;      // offset of L inside a frame's workspace slice
    int syn_bytes, bit_bytes;
    int lds_e_off, lds_l_off;
};

struct LaunchPlan {
    int acc_bits;
    int cn_rule;
    int max_deg;
    int threads;      // workgroup size, a multiple of 64, <= 1024
    bool lds_state;   // E and L in LDS
    size_t lds_bytes; // dynamic LDS per workgroup
};

hipError_t launch_decode(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s);
hipError_t launch_syndrome(const DevCode &C, const uint8_t *bits, int n_frames, uint8_t *out_syn, hipStream_t s);

} // namespace qkdldpc
