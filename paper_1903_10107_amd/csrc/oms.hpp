// Launch interface of the differentiable FP32 offset min-sum kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "qc_code.hpp"

namespace qkdldpc {

struct OmsArgs {
    const uint8_t *syn;     // [F][syn_bytes] packed syndromes
    const float *llr;       // [F][n] channel LLRs (forward)
    const uint8_t *xbits;   // [F][bit_bytes] packed target words, or nullptr (forward: no loss)
    const float *beta;      // [T][n_blocks] offsets
    const float *weights;   // [T] loss weights, or nullptr (all ones)
    const float *dloss;     // backward: [F] gradient of the objective with respect to each frame's loss
    int n_frames, n_iter;
    int syn_bytes, bit_bytes;
    float *out_loss;        // forward: [F] or nullptr
    float *out_E;           // forward: [F][n] soft values after the last iteration, or nullptr
    float *tape;            // [F][T][4m + n4]: a four-word record per check row, then E after the iteration
    float *state;           // per-frame global slices of the state that does not fit in LDS, else nullptr
                            // (forward: E [n4] and the row records [4m]; backward: the adjoints of E [n4]
                            // and L [n_blocks * Z, padded to four]); n4 = n padded to four
    float *dbeta_frames;    // backward: [F][T][n_blocks] per-frame offset gradients
    float *dbeta;           // backward: [T][n_blocks] their sum over frames (in frame order)
    float *dllr;            // backward: [F][n] gradient with respect to the channel LLRs, or nullptr
};

struct OmsPlan {
    int dmax;              // register slots per row: 8, 20 or 32
    int threads;           // workgroup size
    bool lds_state;        // backward: the adjoints of E and L in LDS
    size_t lds_bytes;      // backward: dynamic LDS per workgroup
    bool fwd_lds_state;    // forward: E and the row records in LDS
    size_t fwd_lds_bytes;  // forward: dynamic LDS per workgroup
};

hipError_t launch_oms_forward(const OmsPlan &P, const DevCode &C, const OmsArgs &A, hipStream_t s);
hipError_t launch_oms_backward(const OmsPlan &P, const DevCode &C, const OmsArgs &A, hipStream_t s);

} // namespace qkdldpc
