// Launch interface between the C ABI and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

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
    size_t ws_frame_bytes; // bytes of one slice: per frame, or per workgroup (split kernel)
    size_t ws_l_off;      // offset of L inside a frame's workspace slice
    int syn_bytes, bit_bytes;
    int lds_e_off, lds_l_off, lds_syn_off, lds_flag_off;
    int l_stride;         // packed kernels: bytes between two row pairs' L slices
    int lds_tab_off;      // split kernel: per-lane slot table in LDS
    const int4 *lane_tab; // split kernel: [mb][DMAX/2][2] {c*Z | shift, c*Z, pad mask, block}
    const int32_t *blk2slot; // split kernel: block -> byte offset of its slot in a row pair's L slice
    int persistent_wgs;   // > 0: that many persistent workgroups pull frames from a queue
    int frames_per_wg;    // > 0 (split_reg, Z <= 64): frames per workgroup, one wave per 64 / Z frames
    int *queue;           // persistent: device counter (reset by k_queue_reset)
    const int32_t *order; // persistent: decode order, a permutation of the frames, or nullptr
    int *mflags;          // layer-synchronous family: per frame {active, unsat, iterations, -}
    int *mcount;          // layer-synchronous family: number of frames not yet retired
};

struct LaunchPlan {
    int acc_bits;
    int cn_rule;
    int min_deg, max_deg;
    int threads;      // workgroup size, a multiple of 64, <= 1024
    bool lds_state;   // E and L in LDS
    bool pairs;       // packed kernel: one lane per row pair (r, r + Z/2); needs even Z and LDS state
    bool pow2;        // Z is a power of two
    int split_dmax;   // split kernel (two lanes per row pair) with this slot count, or 0
    bool split_global_l; // split kernel with L in a global slice per workgroup (E stays in LDS)
    bool layer_sync;  // one launch per layer over all frames, E and L in global slices per frame
    bool split_reg;   // split arithmetic with L in registers (five base rows, 8-bit E)
    size_t lds_bytes; // dynamic LDS per workgroup
};

// Set the thread's ldpc_last_error message; returns code.
int set_error(int code, const std::string &msg);

hipError_t launch_decode(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s);
hipError_t launch_decode_scalar(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s);
hipError_t launch_decode_pairs(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s);
hipError_t launch_decode_split(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s);
hipError_t launch_decode_reg(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s);
// LDS bytes of the split_reg decode with fpw frames per workgroup (Z <= 64)
size_t wave_reg_lds_bytes(int n, int z, int syn_bytes, int fpw, int offset_iters);
hipError_t launch_decode_multi(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s);
// The layer-synchronous decode in three phases, for callers that stop early:
// stage-in and the iteration-0 check; iterations t0..t1; stage-out.
hipError_t launch_multi_head(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s);
hipError_t launch_multi_iters(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, int t0, int t1,
                              hipStream_t s);
hipError_t launch_multi_tail(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s);
// LDS read-bandwidth probe (mode 0: 16-byte reads, 1: byte reads), 1024 threads
// per workgroup, out[n_workgroups * 1024]
hipError_t launch_probe_lds(int mode, int n_workgroups, int reps, uint32_t *out, hipStream_t s);
hipError_t launch_syndrome(const DevCode &C, const uint8_t *bits, int n_frames, uint8_t *out_syn, hipStream_t s);
// per-frame count of check rows the channel hard decision fails, and (when
// out_order is not null) the frames by decreasing count
hipError_t launch_order_by_unsat(const DevCode &C, const uint8_t *syn, const int8_t *llr, int n_frames,
                                 int32_t *out_w, int32_t *out_order, hipStream_t s);
hipError_t launch_queue_reset(int *queue, hipStream_t s);
hipError_t launch_reveal(int8_t *llr, int n, int n_frames, const int32_t *frame_ids, int k, const int32_t *positions,
                         const uint8_t *values, int r, hipStream_t s);

} // namespace qkdldpc
