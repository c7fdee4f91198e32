/*
 * qkdldpc: C ABI of an MI355X (gfx950) decoder for quantized layered
 * belief-propagation decoding of LDPC syndromes, as used in QKD information
 * reconciliation (Mao, Li, Han, Guo, "High Throughput and Low Cost LDPC
 * Reconciliation for Quantum Key Distribution", arXiv:1903.10107).
 *
 * Bob holds soft values for his sifted key y and receives Alice's syndrome
 * s = Hx; the decoder returns x^ with H x^ = s when it converges (Sec. 2 of the
 * paper: layered schedule, Eqs. 1, 7, 8, 9, stopping rule; Sec. 3: 8-bit
 * messages, improved-RCBP check node of Alg. 1, saturation-oriented variable
 * node of Alg. 2).
 *
 * Memory: every array argument of the decode calls is a DEVICE pointer (for
 * instance from a torch tensor on the GPU); the base matrix and the parameter
 * block of ldpc_code_create are HOST pointers and are copied. The caller owns
 * every buffer it passes; the library owns the code handle and the device
 * tables behind it. All decode calls are asynchronous with respect to the host
 * and ordered on the given stream (a hipStream_t; NULL is the null stream).
 *
 * Errors: every int-returning call returns LDPC_OK (0) or a negative code and
 * then sets a thread-local message readable with ldpc_last_error(). Arguments
 * are checked on the host before anything reaches the device, so invalid
 * arguments never launch a kernel. Non-convergence of a frame is not an error.
 *
 * Bit packing (syndromes and decoded bits): bit i lives in byte i >> 3 at bit
 * position i & 7 (LSB first).
 *
 * Circulant convention: block (b, c) of the base matrix with shift s joins
 * check row b*Z + r to variable column c*Z + (r + s) mod Z; -1 is a zero block.
 */
#ifndef QKDLDPC_H
#define QKDLDPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ldpc_code ldpc_code;

enum {
    LDPC_OK = 0,
    LDPC_EINVAL = -1,      /* invalid argument */
    LDPC_ENOMEM = -2,      /* host or device allocation failed */
    LDPC_EDEVICE = -3,     /* a HIP call or kernel launch failed, or no GPU */
    LDPC_EUNSUPPORTED = -4 /* valid, but outside what the kernels implement */
};

/* Check-node rules. The degree-d box-plus of Eq. 4 evaluated with the integer
 * tau of Alg. 1 (Sec. 3.2) depends on the fold order because tau is not
 * associative. */
enum {
    LDPC_RULE_RCBP_FB = 0,  /* forward-backward order (default) */
    LDPC_RULE_RCBP_EQ7 = 1, /* literal right fold of Eq. 7 in ascending edge order */
    LDPC_RULE_MINSUM = 2    /* min-sum: min1/min2/argmin of the magnitudes (Sec. 2 cites it) */
};

/* Decoder parameters. A zero-initialised block selects the paper's decoder. */
typedef struct {
    int32_t msg_max;        /* MSG_max of Alg. 1: largest CN message magnitude; 0 -> 63; range 1..127 */
    int32_t e_max;          /* E_max of Alg. 2: saturation of the soft values; 0 -> 127 (8-bit)
                               or 32767 (16-bit); range 1..127 (8-bit), 1..32767 (16-bit) */
    int32_t acc_bits;       /* width of the soft values E: 0 or 8 -> int8, 16 -> int16 */
    int32_t cn_rule;        /* LDPC_RULE_* */
    const int8_t *offsets;  /* HOST pointer or NULL: [offset_iters][n_blocks] magnitude offsets,
                               subtracted from every CN message magnitude at iteration t using
                               row min(t-1, offset_iters-1), result clamped to [0, msg_max];
                               copied at create. NULL = no offsets (the paper's decoder).
                               Every kernel family serves them (LDPC_KERNEL_SPLIT_REG while
                               its LDS holds the table). */
    int32_t offset_iters;   /* rows of offsets; must be >= 1 when offsets != NULL */
    int32_t kernel_hint;    /* 0: pick the kernel family automatically; LDPC_HINT_*: use that
                               family, or fail with LDPC_EUNSUPPORTED when it does not apply
                               (for tuning and testing; results do not depend on it) */
} ldpc_params;

enum {
    LDPC_HINT_AUTO = 0,
    LDPC_HINT_GLOBAL = 1,
    LDPC_HINT_LDS = 2,
    LDPC_HINT_PAIRS = 3,
    LDPC_HINT_SPLIT = 4,
    LDPC_HINT_SPLIT_GLOBAL_L = 5,
    LDPC_HINT_LAYER_SYNC = 6,
    LDPC_HINT_SPLIT_REG = 7
};

/* Build a code from a quasi-cyclic base matrix (Sec. 4.1).
 * base: HOST, int32 [mb][nb] row-major; -1 = zero block, 0..z-1 = circulant shift.
 * Requirements: 1 <= mb < nb; z >= 1; nb * z < 2^31; every base row has
 * between 2 and 32 nonzero blocks; every base column has at least one.
 * Base matrices with 4-cycles are accepted and reported by ldpc_code_dims.
 * params: HOST or NULL (defaults). On success *out receives the handle; the
 * device tables live on the device current at this call.
 * Returns LDPC_EINVAL on a bad argument, LDPC_EUNSUPPORTED for a row degree
 * above 32, LDPC_ENOMEM / LDPC_EDEVICE when the device tables cannot be made. */
int ldpc_code_create(const int32_t *base, int32_t mb, int32_t nb, int32_t z,
                     const ldpc_params *params, ldpc_code **out);

/* Release a handle (NULL is ignored). No decode may be in flight on it. */
void ldpc_code_destroy(ldpc_code *code);

/* Sizes of a code (Sec. 4.1: a QC code of an mb x nb base lifted by z):
 * n = nb*z variable nodes, m = mb*z checks, n_edges = n_blocks*z;
 * has_4cycles = 1 if two base rows and two base columns close a length-4 cycle
 * after lifting. Any output pointer may be NULL. */
int ldpc_code_dims(const ldpc_code *code, int32_t *n, int32_t *m, int64_t *n_edges,
                   int32_t *n_blocks, int32_t *has_4cycles);

/* Decode a batch of frames: the layered decoder of Sec. 2 (layers in ascending
 * base-row order; per check row the VN->CN messages of Eq. 8, the check node of
 * Eqs. 1 and 4 by the integer tau of Alg. 1 (Sec. 3.2) in the rule's fold order,
 * the soft-value update of Eq. 9 under the saturation rule of Alg. 2 (Sec. 3.3);
 * the syndrome test H x^ = s before the first iteration and after each one,
 * stopping a frame as soon as it holds). One frame's result does not depend on
 * the other frames of the batch, on the kernel family or on the schedule.
 * syndromes: DEVICE uint8 [n_frames][ceil(m/8)], Alice's s = Hx, packed.
 * llr_in:    DEVICE int8 [n_frames][n], Bob's channel soft values, positive =
 *            bit 0; -128 is read as -127.
 * max_iter:  iteration limit (>= 0). The syndrome is tested before the first
 *            iteration and after each one; 0 runs the test only.
 * out_bits:  DEVICE uint8 [n_frames][ceil(n/8)], hard decisions [E_j < 0], packed.
 * out_converged: DEVICE uint8 [n_frames], 1 iff H x^ = s.
 * n_frames = 0 is a no-op. May allocate a stream-ordered workspace for codes
 * whose state does not fit on chip (see ldpc_workspace_bytes). Returns
 * LDPC_EINVAL for a NULL code or buffer, n_frames < 0, max_iter < 0, more than
 * 65535 frames on the layer-synchronous family, or a code created on another
 * device than the current one; LDPC_EDEVICE when the workspace allocation or a
 * launch fails. */
int ldpc_decode_batch(const ldpc_code *code, const uint8_t *syndromes, const int8_t *llr_in,
                      int32_t n_frames, int32_t max_iter, uint8_t *out_bits,
                      uint8_t *out_converged, void *stream);

/* As ldpc_decode_batch (Secs. 2 and 3), plus the decoder state the paper keeps
 * (Sec. 2: only the soft values E and the CN->VN messages L are stored) and
 * optional outputs (each may be NULL):
 * out_iters: DEVICE int32 [n_frames]: iterations run (0 = converged at the
 *            pre-check; max_iter when not converged).
 * out_L:     DEVICE int8 [n_frames][n_blocks][z]: final CN->VN messages, blocks
 *            in row-major base order, row r of the block at index r.
 * out_E:     DEVICE int16 [n_frames][n]: final soft values.
 * workspace: DEVICE buffer of at least ldpc_workspace_bytes(code, n_frames)
 *            bytes, or NULL (the call then allocates it stream-ordered when
 *            that size is not 0); no allocation happens when it is given, and
 *            a smaller workspace_bytes is LDPC_EINVAL.
 * Other errors as for ldpc_decode_batch. */
int ldpc_decode_batch_ex(const ldpc_code *code, const uint8_t *syndromes, const int8_t *llr_in,
                         int32_t n_frames, int32_t max_iter, uint8_t *out_bits,
                         uint8_t *out_converged, int32_t *out_iters, int8_t *out_L,
                         int16_t *out_E, void *workspace, size_t workspace_bytes, void *stream);

/* Kernel family the decode calls of a code launch (one workgroup per frame):
 * LDPC_KERNEL_GLOBAL   state in a global-memory workspace, one lane per row;
 * LDPC_KERNEL_LDS      state in LDS, one lane per row;
 * LDPC_KERNEL_PAIRS    state in LDS, one lane per row pair (r, r + z/2), 16-bit packed;
 * LDPC_KERNEL_SPLIT    state in LDS, two lanes per row pair, 16-bit packed;
 * LDPC_KERNEL_SPLIT_GLOBAL_L  as LDPC_KERNEL_SPLIT with E in LDS and the CN
 *                      messages L in a global-memory slice per workgroup (codes
 *                      whose L does not fit in LDS beside E).
 * LDPC_KERNEL_SPLIT_REG  as LDPC_KERNEL_SPLIT with the CN messages L of every
 *                      layer held in registers for the whole decode and E in
 *                      LDS (codes of five base rows, power-of-two z <= 1024,
 *                      rows of 19 or 20 edges, 8-bit soft values with
 *                      e_max > msg_max).
 * LDPC_KERNEL_LAYER_SYNC  one launch per layer over all frames, several
 *                      workgroups per frame, E and L in global slices per frame
 *                      (codes whose soft values do not fit in LDS, e.g. n = 2^20);
 *                      the decode is a sequence of launches on the stream; at
 *                      most 65535 frames per decode call (LDPC_EINVAL above).
 * Automatic selection prefers them in the order SPLIT_REG, SPLIT,
 * SPLIT_GLOBAL_L, LAYER_SYNC, PAIRS, LDS, GLOBAL, taking the first that applies. Also the
 * workgroup size and the dynamic LDS bytes per workgroup. Any output pointer may
 * be NULL. */
enum {
    LDPC_KERNEL_GLOBAL = 0,
    LDPC_KERNEL_LDS = 1,
    LDPC_KERNEL_PAIRS = 2,
    LDPC_KERNEL_SPLIT = 3,
    LDPC_KERNEL_SPLIT_GLOBAL_L = 4,
    LDPC_KERNEL_LAYER_SYNC = 5,
    LDPC_KERNEL_SPLIT_REG = 6
};
int ldpc_code_plan(const ldpc_code *code, int32_t *kernel, int32_t *threads, int32_t *lds_bytes);

/* Device workspace needed by a decode of n_frames frames (0 when the whole
 * decoder state stays in on-chip memory). Returns 0 for invalid arguments. */
size_t ldpc_workspace_bytes(const ldpc_code *code, int32_t n_frames);

/* Batch schedule. A zero-initialised block is one workgroup per frame, placed by
 * the hardware dispatcher (what ldpc_decode_batch does). */
typedef struct {
    int32_t persistent_workgroups; /* > 0: launch that many workgroups; each takes the next
                                      frame from a device queue until none is left, so a CU that
                                      finishes a frame starts another at once. Needs the
                                      LDPC_KERNEL_SPLIT_REG, LDPC_KERNEL_SPLIT or LDPC_KERNEL_SPLIT_GLOBAL_L kernel
                                      family (ldpc_code_plan); the latter's workspace then
                                      holds one L slice per workgroup instead of per frame. */
    const int32_t *order;          /* DEVICE int32 [n_frames] or NULL: the order in which the
                                      queue hands out frames, a permutation of 0..n_frames-1
                                      (for instance hardest first); out-of-range entries are
                                      skipped. Only with persistent_workgroups > 0. */
    int32_t check_every;           /* Layer-synchronous family (LDPC_KERNEL_LAYER_SYNC) only;
                                      ignored by the others, whose decode is one launch that
                                      ends with its frames. 0: every iteration up to max_iter
                                      is enqueued and the call returns at once (launches after
                                      a frame's retirement return immediately for it). k > 0:
                                      after every k iterations the host waits for the stream
                                      and reads the number of frames not yet retired; at 0 it
                                      launches no further iterations. The call (or
                                      ldpc_batch_launch) then returns only when the decode
                                      has finished; results are the same. */
    int32_t frames_per_workgroup;  /* 0: one frame per workgroup. > 0: that many frames per
                                      workgroup, each frame's z lanes inside one wave (64 / z
                                      frames per wave, no workgroup barrier in the decode);
                                      needs the LDPC_KERNEL_SPLIT_REG family with z <= 64, a
                                      multiple of 64 / z, at most 16 waves per workgroup, all
                                      frames' soft values within 64 KB of LDS, and no
                                      persistent schedule (LDPC_EUNSUPPORTED / LDPC_EINVAL
                                      otherwise). */
} ldpc_schedule;

/* ldpc_decode_batch_ex with a schedule (NULL = default): frames are independent
 * (the paper's inter-frame parallel scheme, Sec. 4.2), so the schedule only
 * places them on the GPU. The decoded results do
 * not depend on the schedule. The workspace must hold
 * ldpc_workspace_bytes_sched(code, n_frames, sched) bytes (a persistent schedule
 * needs 256 bytes for its queue); NULL allocates it stream-ordered.
 * Returns LDPC_EUNSUPPORTED for a persistent schedule on other kernel families. */
int ldpc_decode_batch_sched(const ldpc_code *code, const uint8_t *syndromes, const int8_t *llr_in,
                            int32_t n_frames, int32_t max_iter, uint8_t *out_bits,
                            uint8_t *out_converged, int32_t *out_iters, const ldpc_schedule *sched,
                            void *workspace, size_t workspace_bytes, void *stream);
size_t ldpc_workspace_bytes_sched(const ldpc_code *code, int32_t n_frames, const ldpc_schedule *sched);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * decode as ldpc_decode_batch_sched, with the workspace taken from a static
 * device buffer of LDPC_STATIC_WORKSPACE_BYTES that the library holds on every
 * device it runs on until the process ends. No call allocates or frees device
 * memory. Arguments and results are those of ldpc_decode_batch_sched without
 * the workspace arguments.
 * Errors: LDPC_EINVAL when ldpc_workspace_bytes_sched(code, n_frames, sched)
 * exceeds LDPC_STATIC_WORKSPACE_BYTES (decode fewer frames per call, or use a
 * persistent schedule, whose workspace does not grow with the frames);
 * LDPC_EUNSUPPORTED for sched->check_every > 0 (that schedule reads a count back
 * to the host). All calls on one device share its buffer, which keeps the last
 * call's contents: two calls that overlap on one device (different streams, or
 * different host threads) race and must be ordered by the caller. */
#define LDPC_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int ldpc_decode_batch_static(const ldpc_code *code, const uint8_t *syndromes, const int8_t *llr_in,
                             int32_t n_frames, int32_t max_iter, uint8_t *out_bits,
                             uint8_t *out_converged, int32_t *out_iters, const ldpc_schedule *sched,
                             void *stream);

/* A decode of fixed buffers captured once as a HIP graph (the queue reset and the
 * decode kernel), replayed by ldpc_batch_launch with one graph launch. With
 * sched->check_every = k > 0 on the layer-synchronous family the batch holds a
 * graph for the stage-in, one per block of k iterations and one for the
 * stage-out, and ldpc_batch_launch replays the blocks until every frame has
 * retired (it waits for the stream after each block). All
 * pointers are DEVICE pointers that must stay valid for the life of the batch;
 * the workspace, when one is needed and not given, is allocated at create and
 * freed at destroy. The code handle must outlive the batch. A batch owns fixed
 * output and workspace buffers, so two launches of the same batch must not
 * overlap (launch it on one stream, or order the streams). */
typedef struct ldpc_batch ldpc_batch;
int ldpc_batch_create(const ldpc_code *code, const uint8_t *syndromes, const int8_t *llr_in,
                      int32_t n_frames, int32_t max_iter, uint8_t *out_bits, uint8_t *out_converged,
                      int32_t *out_iters, const ldpc_schedule *sched, void *workspace,
                      size_t workspace_bytes, ldpc_batch **out);
int ldpc_batch_launch(ldpc_batch *batch, void *stream);
void ldpc_batch_destroy(ldpc_batch *batch);

/* Decode order for a persistent schedule (ldpc_schedule.order): frames whose
 * channel hard decision y^ = [llr < 0] fails more check rows first. Sec. 2
 * tests H x^ = s to stop; applied to y^ before any iteration, the number of
 * failing rows grows with the number of channel errors and predicts how many
 * iterations a frame needs, so decoding those frames first shortens a batch's
 * tail. The order never changes a frame's result.
 * syndromes: DEVICE uint8 [n_frames][ceil(m/8)]; llr_in: DEVICE int8 [n_frames][n].
 * out_unsat: DEVICE int32 [n_frames]: the number of rows i with (H y^)_i != s_i.
 * out_order: DEVICE int32 [n_frames] or NULL: a permutation of 0..n_frames-1 by
 *            decreasing out_unsat, in buckets of 2^k counts (k the smallest with
 *            m >> k < 1024); the order inside a bucket is unspecified.
 * Uses no workspace and allocates nothing; asynchronous on stream. Returns
 * LDPC_EINVAL for NULL arguments or n_frames < 0 (0 is a no-op), LDPC_EDEVICE
 * for launch failures. */
int ldpc_order_by_unsat(const ldpc_code *code, const uint8_t *syndromes, const int8_t *llr_in,
                        int32_t n_frames, int32_t *out_unsat, int32_t *out_order, void *stream);

/* Alice's side of the syndrome exchange (Sec. 2: she sends s = H x over the
 * public channel): out_syn = H bits over GF(2) for a batch, with the code's QC
 * structure (check row b Z + r reads bit c Z + ((r + shift) mod Z) of every
 * nonzero block (b, c)).
 *   bits     DEVICE uint8 [n_frames][ceil(n/8)], bit j -> byte j>>3, bit (j&7)
 *   out_syn  DEVICE uint8 [n_frames][ceil(m/8)], the same packing (the syndromes
 *            ldpc_decode_batch takes)
 * The caller owns both buffers; any alignment is accepted (4-byte aligned
 * buffers take the word-parallel kernels). Uses no workspace and allocates
 * nothing; asynchronous on stream. Returns LDPC_EINVAL for a NULL code or
 * buffer, n_frames < 0 (0 is a no-op) or a code created on another device than
 * the current one, LDPC_EDEVICE when a launch fails. */
int ldpc_syndrome_batch(const ldpc_code *code, const uint8_t *bits, int32_t n_frames,
                        uint8_t *out_syn, void *stream);

/* Interactive rate adaptation (Sec. 4.1): after a failed decode Alice reveals
 * the values of further positions of a frame (typically punctured ones, which
 * then count as shortened), and Bob decodes again. For each listed frame
 * frame_ids[i] (i < k) and each of its r positions positions[i * r + q], the
 * LLR becomes the shortened value: -127 if values[i * r + q] != 0 (bit 1), else
 * +127. Ids outside [0, n_frames) and positions outside [0, n) are skipped, so
 * rows can be padded with -1.
 *   llr        DEVICE int8 [n_frames][n], updated in place
 *   frame_ids  DEVICE int32 [k]
 *   positions  DEVICE int32 [k][r]
 *   values     DEVICE uint8 [k][r], the revealed bits (0 or 1)
 * Returns LDPC_EINVAL for NULL pointers (when k * r > 0), negative counts or
 * k * r >= 2^31.
 * Asynchronous on stream. */
int ldpc_reveal_batch(const ldpc_code *code, int8_t *llr, int32_t n_frames, const int32_t *frame_ids,
                      int32_t k, const int32_t *positions, const uint8_t *values, int32_t r,
                      void *stream);

/* ------------------------------------------------------------------------
 * Differentiable FP32 offset min-sum with learned offsets.
 *
 * The layered schedule of Sec. 2 (Eqs. 8 and 9) with the check node simplified
 * to offset min-sum (the usual simplification of BP that the paper cites,
 * Sec. 2) and one offset per iteration and base-matrix edge:
 *   v_k = E_j - L_k;  L_k = sigma_k * max(min_{k' != k} |v_k'| - beta[t][blk_k], 0);  E_j = v_k + L_k
 * with sigma_k the row's sign product times (-1)^{s_i} times sgn(v_k)
 * (sgn(0) = +1). n_iter iterations run without early stopping. The training
 * loss of a frame is sum_t w_t * sum_j softplus(-(1 - 2 x_j) E_j^(t)) / n, the
 * binary cross-entropy of the soft values after every iteration t against the
 * transmitted word x. The backward pass gives the gradient of
 * sum_f dloss_f * loss_f with respect to the offsets (summed over frames) and,
 * optionally, the channel LLRs. Ties between minima go to the lowest edge index;
 * d|v|/dv = 0 at v = 0; the clamp at 0 passes gradient only where
 * min - beta > 0. Results are deterministic (fixed-order reductions).
 *
 * The code's own decoder parameters (msg_max, e_max, rule, offsets) play no
 * part here; only its base matrix and lifting do.
 *
 * Buffers (all DEVICE, caller-owned):
 *   syndromes     uint8 [F][ceil(m/8)] packed LSB-first
 *   llr           float [F][n], positive = bit 0
 *   target_bits   uint8 [F][ceil(n/8)] the transmitted words x, packed LSB-first
 *   beta          float [n_iter][n_blocks] (blocks in row-major base-matrix order)
 *   loss_weights  float [n_iter], or NULL for all ones
 *   tape          ldpc_oms_tape_bytes(code, F, n_iter) bytes, 16-byte aligned:
 *                 written by the forward pass, read by the backward pass (per
 *                 check row and iteration the two smallest |VN->CN| values, their
 *                 edge indices and the signs; soft values after every iteration)
 *   workspace     ldpc_oms_workspace_bytes(code, F, n_iter) bytes: FP32 state of
 *                 codes whose state does not fit in LDS, and per-frame offset
 *                 gradients. The forward pass keeps E and one record per check
 *                 row (not a value per edge), so it reads the workspace only when
 *                 that smaller state does not fit in LDS; otherwise it may be NULL.
 * Returns LDPC_EINVAL for bad arguments (n_iter < 1, NULL pointers, short or
 * misaligned tape, short workspace), LDPC_EUNSUPPORTED when the offset table (n_iter x n_blocks
 * floats) does not fit in on-chip memory, LDPC_EDEVICE for launch failures.
 * Asynchronous on stream.
 * ------------------------------------------------------------------------ */
size_t ldpc_oms_tape_bytes(const ldpc_code *code, int32_t n_frames, int32_t n_iter);
size_t ldpc_oms_workspace_bytes(const ldpc_code *code, int32_t n_frames, int32_t n_iter);

/* Forward pass. out_loss: float [F] per-frame loss, or NULL (then target_bits
 * may be NULL); out_E: float [F][n] soft values after the last iteration, or NULL. */
int ldpc_oms_forward(const ldpc_code *code, const uint8_t *syndromes, const float *llr,
                     const uint8_t *target_bits, int32_t n_frames, int32_t n_iter, const float *beta,
                     const float *loss_weights, float *out_loss, float *out_E, void *tape,
                     size_t tape_bytes, void *workspace, size_t workspace_bytes, void *stream);

/* Backward pass over the tape of the forward pass with the same arguments.
 * dloss: float [F]; out_dbeta: float [n_iter][n_blocks] (overwritten);
 * out_dllr: float [F][n] or NULL. */
int ldpc_oms_backward(const ldpc_code *code, const uint8_t *syndromes, const uint8_t *target_bits,
                      int32_t n_frames, int32_t n_iter, const float *beta, const float *loss_weights,
                      const float *dloss, const void *tape, size_t tape_bytes, float *out_dbeta,
                      float *out_dllr, void *workspace, size_t workspace_bytes, void *stream);

/* Diagnostics: LDS read-bandwidth probe, the measured on-chip peak that the
 * decoder's LDS traffic is reported against (its state lives in LDS). Launches
 * n_workgroups workgroups of 1024 threads on the stream; each fills 64 KB of
 * LDS and every thread then makes reps * 8 conflict-free reads of 16 bytes
 * (mode 0) or of one byte (mode 1, the width of the decoder's accesses),
 * folding them into out[workgroup * 1024 + thread] (DEVICE uint32). Bytes read
 * = n_workgroups * 1024 * reps * 8 * (16 or 1). LDPC_EINVAL for a mode other
 * than 0 or 1, n_workgroups or reps below 1, or a NULL out. */
int ldpc_probe_lds_bandwidth(int32_t mode, int32_t n_workgroups, int32_t reps, uint32_t *out, void *stream);

/* Message describing the last error on this thread ("" if none). */
const char *ldpc_last_error(void);

/* Library version, major * 10000 + minor * 100 + patch. */
int ldpc_version(void);

/* Host-side self description of the kernels' check-node arithmetic: writes
 * tau(p, q) of Alg. 1 for p, q in [0, 63] (MSG_max = 63) into out[64 * 64],
 * computed by the same inline function the GPU kernels use, compiled for the
 * host. HOST pointer. For testing the kernels' arithmetic without a GPU. */
int ldpc_host_tau_table(int32_t *out);

/* Host-side self description of the packed check-node fold of the GPU kernels
 * (two rows per 32-bit register, rows shorter than 32 padded with a neutral
 * operand): for a row of degree d in 2..32 and clipped input magnitudes in
 * 0..127, writes the output magnitude for every edge under the given rule, for
 * the two rows held in the low and high halves. HOST pointers, length d. */
int ldpc_host_fold_pair(int32_t rule, const int32_t *p_lo, const int32_t *p_hi, int32_t d,
                        int32_t *out_lo, int32_t *out_hi);

#ifdef __cplusplus
}
#endif

#endif /* QKDLDPC_H */
