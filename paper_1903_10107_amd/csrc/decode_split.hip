// gfx950 decode kernel, two lanes per row pair, 16-bit packed arithmetic,
// state in LDS: the path of power-of-two Z with row degree up to 20.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "split_common.hpp"

namespace qkdldpc {

// ---------------------------------------------------------------------------
// Split variant: two adjacent lanes share a row pair, so a frame of Z = 1024
// runs 16 waves per CU instead of 8. Both lanes execute the same code. Lane A
// (even) holds edges 0 .. DH-1 of the row pair in order, lane B (odd) holds
// edges DMAX-1 down to DH, so a left fold over a lane's own slots is the
// forward partial F for A and the backward partial B for B. One lane swap
// hands A the value B_DH and B the value F_{DH-1}; each lane then folds its
// slots the other way, W_k, and its outputs are out_i = tau(X_{i-1}, W_{DH-1-i})
// with out_0 = W_{DH-1}, which is the forward-backward fold edge by edge.
//
// Per-lane slot entries {c*Z | shift, LDS address of block column c, pad mask,
// block} sit in LDS; padding slots point at a dummy block column past E, so
// they need no store guards, and their operands are masked to 0 / kPad. E is
// addressed with absolute LDS addresses (the table holds them), so no base is
// added per access. L of a row pair is laid out [layer][half][slot][lane].
//
// L lives in LDS when it fits beside E; otherwise (LG) it streams from a
// global workspace slice per workgroup laid out [layer][row pair][4 DH bytes]
// (a 16-bit slot per byte pair, the two lanes' slots side by side, see LRef),
// so a wave touches one contiguous run and no byte goes unused. The first iteration takes L = 0 without
// reading it, so the slice needs no clearing between frames.
//
// When every row pair has a lane pair (Z/2 <= RPL x threads/2, with RPL row
// pairs per lane pair), the syndrome test of the state after iteration t-1 is
// folded into layer 0 of iteration t: layer 0 reads exactly that state, so its
// rows' parities come from the loaded values; only when all of them hold are
// the other layers tested, before layer 0 writes anything.
// ---------------------------------------------------------------------------

// LDS regions of the split kernel, set up once per workgroup.
template <typename ET>
struct SplitLds {
    ET *E;          // E plus one dummy block column, at offset 0
    int8_t *L;      // [row pair][layer][half][slot][lane]
    uint8_t *syn;   // packed syndrome of the current frame
    int4 *tab;      // per-lane slot table with absolute column addresses
    int *flags;     // three vote words and one queue slot
};

// Row pairs per lane pair on the folded-check path: two for the short rows of
// DMAX = 8 (Z up to 4096 with 1024 threads), one otherwise.
template <int DMAX>
constexpr int split_rpl() { return DMAX <= 8 ? 2 : 1; }
// (DMAX = 6 serves rows of degree exactly 6, DMAX = 8 degrees up to 8, DMAX = 20 up to 20.)

// Layers of prefetch distance for L in global memory (folded-check path).
template <int DMAX>
constexpr int split_pd() { return DMAX <= 8 ? 3 : 2; }

// Decode frame f with one workgroup (the LDS table must already be staged).
// LG: L in the global slice Lg of this workgroup, else in LDS.
template <int DMIN, int DMAX, typename ET, int RULE, bool LG, bool OFF>
__device__ __forceinline__ void split_decode_frame(const DevCode &C, const DecodeArgs &A, const SplitLds<ET> &M,
                                                   uint8_t *Lg, int f)
{
    // the offset table's row of iteration t (OFF): min(t - 1, offset_iters - 1)
    auto off_row = [&](int t) -> const int32_t * {
        if constexpr (OFF)
            return C.offsets + (size_t)(t - 1 < C.offset_iters - 1 ? t - 1 : C.offset_iters - 1) * C.n_blocks;
        else
            return nullptr;
    };
    constexpr int DH = DMAX / 2;
    constexpr int RPL = split_rpl<DMAX>();
    constexpr unsigned esh = sizeof(ET) == 2 ? 1 : 0;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int z = C.z, n = C.n, hz = z >> 1, h = tid & 1;
    const unsigned zm = (unsigned)(z - 1), hzb = (unsigned)hz << esh;
    ET *E = M.E;
    int8_t *L = M.L;
    uint8_t *s_syn = M.syn;
    const int4 *s_tab = M.tab;
    int *flags = M.flags;
    const int S = A.l_stride;
    const LdsESink<ET> es{hzb};
    auto lref = [&](int b, int r) {
        if constexpr (LG)
            return LRef<DH, true>{Lg + (size_t)b * hz * LRef<DH, true>::PAIR_BYTES,
                                  (unsigned)r * LRef<DH, true>::PAIR_BYTES, h};
        else
            return LRef<DH, false>{L + r * S + h + b * 4 * DH};
    };

    // stage in: syndrome, E, L = 0 (LDS only), vote words
    const uint8_t *syn = A.syn + (size_t)f * A.syn_bytes;
    for (int i = tid; i < A.syn_bytes; i += nthr)
        s_syn[i] = syn[i];
    stage_llr<ET>(E, A.llr + (size_t)f * n, n, C.e_max < 127 ? C.e_max : 127, tid, nthr);
    if constexpr (!LG) {
        uint4 *L128 = reinterpret_cast<uint4 *>(L);
        for (int w = tid; w < (hz * S) >> 4; w += nthr)
            L128[w] = uint4{0, 0, 0, 0};
        for (int w = ((hz * S) & ~15) + tid; w < hz * S; w += nthr)
            L[w] = 0;
    }
    if (tid < 3)
        flags[tid] = 0;
    __syncthreads();
    int vk = 0;
    int conv, iters = 0;
    const int lp = tid >> 1, np = nthr >> 1;
    // At most 32 layers (the syndrome bits of a lane's rows fit two registers);
    // global L on this path: every lane pair owns RPL row pairs, and there are
    // more layers than the prefetch distance
    if (C.mb <= 32 && (LG ? hz == RPL * np && C.mb > split_pd<DMAX>() : hz <= RPL * np)) {
        // every row pair has a lane pair: the check is folded into layer 0
        auto unsat_range = [&](int b0, int b1) {
            int u = 0;
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                const int r = lp + k * np;
                if (r < hz)
                    u |= split_rows_unsat<DMIN, DMAX, ET>(C, s_syn, s_tab, h, r, b0, b1);
            }
            return u;
        };
        // layer 0 first: a frame that fails there (nearly every frame before its
        // first iteration) skips testing the other layers
        conv = !block_vote(unsat_range(0, 1), flags, vk) && !block_vote(unsat_range(1, C.mb), flags, vk);
        // Each lane keeps its row pairs' syndrome bits in registers (this path
        // takes at most 32 layers): word b / 16, bit b % 16 for row b*Z + r and
        // bit 16 + b % 16 for row b*Z + r + Z/2; layer b's pair (the sign bits
        // of two 16-bit halves) is then (word << (15 - b % 16)) & 0x80008000.
        unsigned synm[RPL][2];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const int r = lp + k * np;
            synm[k][0] = synm[k][1] = 0;
            if (r < hz)
                for (int b = 0; b < C.mb; ++b) {
                    const int i0 = b * z + r, i1 = i0 + hz;
                    const unsigned bits = (unsigned)((s_syn[i0 >> 3] >> (i0 & 7)) & 1) << (b & 15) |
                                          (unsigned)((s_syn[i1 >> 3] >> (i1 & 7)) & 1) << (16 + (b & 15));
                    synm[k][b >> 4] |= bits;
                }
        }
        auto syn_of = [&](int k, int b) {
            const unsigned w = b < 16 ? synm[k][0] : synm[k][1];
            return __builtin_bit_cast(s16x2, (w << (15 - (b & 15))) & 0x80008000u);
        };
        if constexpr (!LG) {
            // Each layer step reads its slot addresses and L (private to the lane,
            // written by it one iteration earlier) before the barrier that orders
            // the previous step's E writes, so that after it only E is waited for.
            auto prepare = [&](SplitRow<DH> (&R)[RPL], int t, int b) {
#pragma unroll
                for (int k = 0; k < RPL; ++k) {
                    const int r = lp + k * np;
                    if (r < hz) {
                        split_addr<DMIN, DMAX, ET, OFF>(R[k], s_tab + b * DH * 2 + h, r, zm, off_row(t));
                        lref(b, r).load(R[k].lk, t == 1);
                    }
                }
            };
            for (int t = 1; t <= A.max_iter && !conv; ++t) {
                {
                    SplitRow<DH> R[RPL];
                    prepare(R, t, 0);
                    __syncthreads();
#pragma unroll
                    for (int k = 0; k < RPL; ++k)
                        if (lp + k * np < hz)
                            split_fetch_e<ET>(R[k], hzb);
                    if (t >= 2) {
                        int fail0 = 0;
#pragma unroll
                        for (int k = 0; k < RPL; ++k)
                            if (lp + k * np < hz) {
                                const s16x2 own = split_e_parity<DMIN, DMAX>(R[k]);
                                const s16x2 pe = syn_of(k, 0) ^ own ^ swap_pair(own);
                                fail0 |= (pe.x | pe.y) < 0;
                            }
                        if (!block_vote(fail0, flags, vk)) {
                            if (!block_vote(unsat_range(1, C.mb), flags, vk)) {
                                conv = 1;
                                iters = t - 1;
                                break;
                            }
                        }
                    }
#pragma unroll
                    for (int k = 0; k < RPL; ++k) {
                        const int r = lp + k * np;
                        if (r < hz)
                            split_finish<DMIN, DMAX, ET, RULE, LG, OFF>(C, R[k], lref(0, r), syn_of(k, 0), es);
                    }
                }
                for (int b = 1; b < C.mb; ++b) {
                    SplitRow<DH> R[RPL];
                    prepare(R, t, b);
                    __syncthreads();
#pragma unroll
                    for (int k = 0; k < RPL; ++k) {
                        const int r = lp + k * np;
                        if (r < hz) {
                            split_fetch_e<ET>(R[k], hzb);
                            split_finish<DMIN, DMAX, ET, RULE, LG, OFF>(C, R[k], lref(b, r), syn_of(k, b), es);
                        }
                    }
                }
                iters = t;
            }
            // the last step's E writes before the stage-out reads
            __syncthreads();
        } else {
            // Global L, software-pipelined: one flat loop over the layer steps g
            // of all iterations, unrolled by PD so that register slot j always
            // serves the steps g = j (mod PD). After step g has unpacked its words
            // from slot j, the slot is refilled with the words of step g + PD,
            // whose latency then overlaps PD layers of work. That layer was last
            // written at step g + PD - mb < g, before an earlier barrier, as
            // mb > PD here. The first iteration takes L = 0 without reading it.
            constexpr int NW = LRef<DH, true>::NW;
            constexpr int PD = split_pd<DMAX>();
            // Every lane pair owns RPL row pairs here, so every memory access of
            // the loop is issued by every lane: the number in flight is the same
            // on all paths and the wait for a slot leaves the younger requests
            // outstanding. 32-bit byte offsets into the slice (a few hundred KB)
            // keep the slice base uniform, so the loads fill the slot registers
            // in place.
            int rr[RPL];
            unsigned ro[RPL];  // chunk offsets of the lane's row pairs within a layer
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                rr[k] = lp + k * np;
                ro[k] = (unsigned)rr[k] * LRef<DH, true>::PAIR_BYTES;
            }
            auto layer_l = [&](int b) { return Lg + (size_t)b * hz * LRef<DH, true>::PAIR_BYTES; };
            uint32_t pf[PD][RPL][NW] = {};
            auto fetch = [&](uint32_t (&dst)[RPL][NW], int b) {
#pragma unroll
                for (int k = 0; k < RPL; ++k)
                    LRef<DH, true>::fetch(layer_l(b), ro[k], h, dst[k]);
            };
            int t = 1, b = 0;
            bool done = conv || A.max_iter == 0;
            while (!done) {
#pragma unroll
                for (int j = 0; j < PD; ++j) {
                    if (done)
                        break;
                    SplitRow<DH> R[RPL];
                    const s16x2 zero = splat2(0);
                    // slot addresses before the barrier that orders the previous
                    // step's E writes; after it the E reads
#pragma unroll
                    for (int k = 0; k < RPL; ++k)
                        split_addr<DMIN, DMAX, ET, OFF>(R[k], s_tab + b * DH * 2 + h, rr[k], zm, off_row(t));
                    __syncthreads();
#pragma unroll
                    for (int k = 0; k < RPL; ++k) {
                        split_fetch_e<ET>(R[k], hzb);
                        s16x2 lw[DH];
                        LRef<DH, true>::unpack(pf[j][k], h, lw);
#pragma unroll
                        for (int i = 0; i < DH; ++i)
                            R[k].lk[i] = t >= 2 ? lw[i] : zero;
                    }
                    if (b == 0 && t >= 2) {
                        int fail0 = 0;
#pragma unroll
                        for (int k = 0; k < RPL; ++k) {
                            const s16x2 own = split_e_parity<DMIN, DMAX>(R[k]);
                            const s16x2 pe = syn_of(k, 0) ^ own ^ swap_pair(own);
                            fail0 |= (pe.x | pe.y) < 0;
                        }
                        if (!block_vote(fail0, flags, vk) && !block_vote(unsat_range(1, C.mb), flags, vk)) {
                            conv = 1;
                            iters = t - 1;
                            done = true;
                            break;
                        }
                    }
                    // refill the slot with step g + PD (loaded every time; unused data
                    // of the first iteration or past the last one is ignored)
                    fetch(pf[j], b + PD >= C.mb ? b + PD - C.mb : b + PD);
#pragma unroll
                    for (int k = 0; k < RPL; ++k)
                        split_finish<DMIN, DMAX, ET, RULE, true, OFF>(C, R[k], LRef<DH, true>{layer_l(b), ro[k], h},
                                                                      syn_of(k, b), es);
                    if (++b == C.mb) {
                        b = 0;
                        iters = t;
                        if (++t > A.max_iter)
                            done = true;
                    }
                }
            }
            // the last step's E writes before the final check and the stage-out
            __syncthreads();
        }
        if (!conv && A.max_iter > 0)
            conv = !block_vote(unsat_range(0, 1), flags, vk) && !block_vote(unsat_range(1, C.mb), flags, vk);
    } else {
        // more row pairs than that: separate check after every iteration
        auto unsat_all = [&]() {
            int u = 0;
            for (int r = lp; r < hz; r += np)
                u |= split_rows_unsat<DMIN, DMAX, ET>(C, s_syn, s_tab, h, r, 0, C.mb);
            return u;
        };
        conv = !block_vote(unsat_all(), flags, vk);
        for (int t = 1; t <= A.max_iter && !conv; ++t) {
            for (int b = 0; b < C.mb; ++b) {
                for (int r = lp; r < hz; r += np) {
                    SplitRow<DH> R;
                    const auto Lr = lref(b, r);
                    split_load<DMIN, DMAX, ET, LG, OFF>(R, Lr, s_tab + b * DH * 2 + h, r, zm, hzb, t == 1,
                                                        off_row(t));
                    split_finish<DMIN, DMAX, ET, RULE, LG, OFF>(C, R, Lr,
                                                                syn_pair(s_syn, b * z + r, b * z + r + hz), es);
                }
                __syncthreads();
            }
            iters = t;
            conv = !block_vote(unsat_all(), flags, vk);
        }
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
        // canonical [block][row] layout; L was never written when no iteration ran
        const int ne = C.n_blocks * z;
        for (int e = tid; e < ne; e += nthr) {
            const int blk = e / z, row = e - blk * z;
            const int half = row >= hz, r = row - half * hz;
            const int v = A.blk2slot[blk];  // b * 4DH + 2 * slot + lane
            int8_t x;
            if constexpr (LG) {
                const int b = v / (4 * DH), rem = v - b * 4 * DH;
                x = iters == 0 ? (int8_t)0
                               : (int8_t)Lg[((size_t)b * hz + r) * LRef<DH, true>::PAIR_BYTES +
                                            LRef<DH, true>::slot_byte(rem & 1, rem >> 1) + half];
            } else {
                x = L[r * S + v + half * 2 * DH];
            }
            A.out_L[(size_t)f * ne + e] = x;
        }
    }
    if (A.out_E)
        for (int j = tid; j < n; j += nthr)
            A.out_E[(size_t)f * n + j] = (int16_t)E[j];
}

// Split LDS layout and the ebase invariant: the slot addresses OR a column
// start into a row offset, which needs E to start at a multiple of Z elements;
// these kernels use no static LDS, so the dynamic area starts at 0.
template <typename ET>
__device__ __forceinline__ bool split_setup(const DevCode &C, const DecodeArgs &A, SplitLds<ET> &M)
{
    constexpr int DH_UNUSED = 0;
    (void)DH_UNUSED;
    constexpr unsigned esh = sizeof(ET) == 2 ? 1 : 0;
    extern __shared__ __align__(16) uint8_t smem[];
    M.E = reinterpret_cast<ET *>(smem);
    M.L = reinterpret_cast<int8_t *>(smem + A.lds_l_off);
    M.syn = smem + A.lds_syn_off;
    M.tab = reinterpret_cast<int4 *>(smem + A.lds_tab_off);
    M.flags = reinterpret_cast<int *>(smem + A.lds_flag_off);
    const unsigned ebase = (unsigned)(uintptr_t)M.E;
    return (ebase & ((unsigned)(C.z << esh) - 1)) == 0;
}

template <typename ET>
__device__ __forceinline__ void split_stage_table(const DevCode &C, const DecodeArgs &A, const SplitLds<ET> &M,
                                                  int dh)
{
    constexpr unsigned esh = sizeof(ET) == 2 ? 1 : 0;
    const unsigned ebase = (unsigned)(uintptr_t)M.E;
    for (int q = threadIdx.x; q < C.mb * dh * 2; q += blockDim.x) {
        int4 te = A.lane_tab[q];
        te.y = (int)(((unsigned)te.y << esh) + ebase);
        M.tab[q] = te;
    }
}

// Global L slice of this workgroup (LG), indexed by workgroup so that
// persistent workgroups reuse theirs from frame to frame.
template <bool LG>
__device__ __forceinline__ uint8_t *split_l_slice(const DecodeArgs &A)
{
    return LG ? A.ws + (size_t)blockIdx.x * A.ws_frame_bytes : nullptr;
}

// One workgroup per frame (grid = frames).
template <int DMIN, int DMAX, typename ET, int RULE, bool LG, bool OFF>
__global__ __launch_bounds__(1024) void k_decode_frame_split(DevCode C, DecodeArgs A)
{
    SplitLds<ET> M;
    const int f = blockIdx.x;
    if (!split_setup<ET>(C, A, M)) {
        if (threadIdx.x == 0) {
            A.out_conv[f] = 0;
            if (A.out_iters)
                A.out_iters[f] = -1;
        }
        return;
    }
    split_stage_table<ET>(C, A, M, DMAX / 2);
    split_decode_frame<DMIN, DMAX, ET, RULE, LG, OFF>(C, A, M, split_l_slice<LG>(A), f);
}

// Persistent workgroups: each one takes the next position of a device queue
// (atomic counter, reset to 0 by k_queue_reset before the launch), decodes
// frame order[position] (or position), and stops once the queue is past the
// last frame, which every wave of every workgroup reaches.
template <int DMIN, int DMAX, typename ET, int RULE, bool LG, bool OFF>
__global__ __launch_bounds__(1024) void k_decode_split_persistent(DevCode C, DecodeArgs A)
{
    SplitLds<ET> M;
    if (!split_setup<ET>(C, A, M))
        return;
    split_stage_table<ET>(C, A, M, DMAX / 2);
    uint8_t *Lg = split_l_slice<LG>(A);
    for (;;) {
        __syncthreads();  // the previous frame's stage-out is done with E and the queue slot
        if (threadIdx.x == 0)
            M.flags[3] = atomicAdd(A.queue, 1);
        __syncthreads();
        const int q = M.flags[3];
        if (q >= A.n_frames)
            break;
        const int f = A.order ? A.order[q] : q;
        if ((unsigned)f < (unsigned)A.n_frames)
            split_decode_frame<DMIN, DMAX, ET, RULE, LG, OFF>(C, A, M, Lg, f);
    }
}

namespace {

template <int DMIN, int DMAX, typename ET, int RULE, bool LG, bool OFF>
hipError_t launch_one_split(const DevCode &C, const DecodeArgs &A, int threads, size_t lds, hipStream_t s)
{
    const bool persistent = A.persistent_wgs > 0;
    auto kern = persistent ? k_decode_split_persistent<DMIN, DMAX, ET, RULE, LG, OFF>
                           : k_decode_frame_split<DMIN, DMAX, ET, RULE, LG, OFF>;
    if (lds > 65536) {
        hipError_t e = persistent ? allow_max_lds<k_decode_split_persistent<DMIN, DMAX, ET, RULE, LG, OFF>>()
                                  : allow_max_lds<k_decode_frame_split<DMIN, DMAX, ET, RULE, LG, OFF>>();
        if (e != hipSuccess)
            return e;
    }
    if (persistent) {
        hipError_t e = launch_queue_reset(A.queue, s);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(kern, dim3(persistent ? A.persistent_wgs : A.n_frames), dim3(threads), lds, s, C, A);
    return hipGetLastError();
}

template <int DMIN, int DMAX, typename ET, bool LG, bool OFF>
hipError_t launch_rule_split(int rule, const DevCode &C, const DecodeArgs &A, int threads, size_t lds,
                             hipStream_t s)
{
    if (rule == LDPC_RULE_MINSUM)
        return launch_one_split<DMIN, DMAX, ET, kRuleMinSum, LG, OFF>(C, A, threads, lds, s);
    return launch_one_split<DMIN, DMAX, ET, kRuleRcbpFB, LG, OFF>(C, A, threads, lds, s);
}

template <typename ET, bool LG, bool OFF>
hipError_t launch_split(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s)
{
    switch (P.split_dmax) {
    case 6:
        return launch_rule_split<6, 6, ET, LG, OFF>(P.cn_rule, C, A, P.threads, P.lds_bytes, s);
    case 8:
        return P.min_deg >= 6 ? launch_rule_split<6, 8, ET, LG, OFF>(P.cn_rule, C, A, P.threads, P.lds_bytes, s)
                              : launch_rule_split<2, 8, ET, LG, OFF>(P.cn_rule, C, A, P.threads, P.lds_bytes, s);
    default:
        return P.min_deg >= 19 ? launch_rule_split<19, 20, ET, LG, OFF>(P.cn_rule, C, A, P.threads, P.lds_bytes, s)
                               : launch_rule_split<2, 20, ET, LG, OFF>(P.cn_rule, C, A, P.threads, P.lds_bytes, s);
    }
}

} // namespace

hipError_t launch_decode_split(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s)
{
    if (P.split_global_l && C.offsets)
        return P.acc_bits == 16 ? launch_split<int16_t, true, true>(P, C, A, s)
                                : launch_split<int8_t, true, true>(P, C, A, s);
    if (P.split_global_l)
        return P.acc_bits == 16 ? launch_split<int16_t, true, false>(P, C, A, s)
                                : launch_split<int8_t, true, false>(P, C, A, s);
    if (C.offsets)
        return P.acc_bits == 16 ? launch_split<int16_t, false, true>(P, C, A, s)
                                : launch_split<int8_t, false, true>(P, C, A, s);
    return P.acc_bits == 16 ? launch_split<int16_t, false, false>(P, C, A, s)
                            : launch_split<int8_t, false, false>(P, C, A, s);
}

} // namespace qkdldpc
