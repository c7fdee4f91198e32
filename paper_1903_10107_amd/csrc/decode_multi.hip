// Layer-synchronous decoding for frames whose soft values do not fit in one
// CU's LDS (n = 1048576 with 16-bit E): every layer is one launch over all
// frames with several workgroups per frame, so a frame spreads over many CUs and
// the kernel boundary orders layer b before layer b + 1 (Sec. 2: the rows of a
// QC layer are independent, consecutive layers are not). Per decode:
//   stage in; check(0); finalize(0);
//   for t = 1 .. max_iter: layer(0, t) ... layer(mb - 1, t); check(t); finalize(t)
//   stage out
// A frame that has converged (or reached max_iter) is retired by finalize and
// every later launch exits at once for it, so its state stays as it was at
// that point, as in the one-workgroup kernels.
//
// Row pairs and arithmetic are those of the split kernels (two lanes per row
// pair, both rows in the 16-bit halves, Alg. 1 in forward-backward order, Eq. 9
// under Alg. 2); E lives in a global slice per frame and is read and written at
// the QC-shifted positions, L in the global-L chunk layout
// [layer][row pair][4 DH bytes]. Iteration 1 takes L = 0 unread.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "split_common.hpp"

namespace qkdldpc {

namespace {

// E stores into a frame's global slice: both rows of the pair.
template <typename ET>
struct GlobalESink {
    ET *E;
    unsigned hz;  // Z/2: flips between the two rows' columns
    __device__ __forceinline__ void operator()(unsigned a0, s16x2 o) const
    {
        at(a0) = (ET)o.x;
        at(a0 ^ hz) = (ET)o.y;
    }
    // element i through a 32-bit byte offset from the frame's (uniform) base, so
    // the access takes the scalar-base plus vector-offset form
    __device__ __forceinline__ ET &at(unsigned i) const
    {
        return *reinterpret_cast<ET *>(reinterpret_cast<uint8_t *>(E) + (i * (unsigned)sizeof(ET)));
    }
};

// Element indices and values of E for a lane's slots: a0 = ((r + shift) mod Z)
// + c Z from the lane-table entry {c Z | shift, c Z, pad mask, block}.
// OFF: also the slots' offsets from the offset table's row off_row (padding
// slots, block -1, take 0), two 16-bit offsets per register.
template <int DMIN, int DMAX, typename ET, bool OFF = false>
__device__ __forceinline__ void load_e_global(SplitRow<DMAX / 2> &R, const int4 *tab, int r, unsigned zm, unsigned hz,
                                              const ET *__restrict__ E, const int32_t *__restrict__ off_row = nullptr)
{
    constexpr int DH = DMAX / 2;
#pragma unroll
    for (int i = 0; i < DH; ++i) {
        const int4 te = tab[2 * i];
        const unsigned a0 = (((unsigned)r + (unsigned)te.x) & zm) | (unsigned)te.y;
        R.a0[i] = a0;
        R.pm[i] = te.z;
        const uint8_t *eb = reinterpret_cast<const uint8_t *>(E);  // 32-bit byte offsets, uniform base
        R.e[i] = pack_halves(*reinterpret_cast<const ET *>(eb + a0 * (unsigned)sizeof(ET)),
                             *reinterpret_cast<const ET *>(eb + (a0 ^ hz) * (unsigned)sizeof(ET)));
        if constexpr (OFF) {
            const unsigned o = (unsigned)(te.w >= 0 ? off_row[te.w] : 0) & 0xffffu;
            R.off[i / 2] = i % 2 ? R.off[i / 2] | (o << 16) : o;
        }
    }
}

// per frame: active, unsat (a failing row was seen), iterations when retired
__device__ __forceinline__ int *frame_flags(const DecodeArgs &A, int f) { return A.mflags + 4 * f; }

template <typename ET>
__device__ __forceinline__ ET *frame_e(const DecodeArgs &A, int f)
{
    return reinterpret_cast<ET *>(A.ws + (size_t)f * A.ws_frame_bytes);
}

__device__ __forceinline__ uint8_t *frame_l(const DecodeArgs &A, int f)
{
    return A.ws + (size_t)f * A.ws_frame_bytes + A.ws_l_off;
}

} // namespace

// E = clamp(llr), frame flags: active, no failed row seen yet.
template <typename ET>
__global__ __launch_bounds__(256) void k_multi_stage_in(DevCode C, DecodeArgs A)
{
    const int f = blockIdx.y;
    const int lim = C.e_max < 127 ? C.e_max : 127;
    ET *E = frame_e<ET>(A, f);
    const int8_t *llr = A.llr + (size_t)f * C.n;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < C.n; j += gridDim.x * blockDim.x)
        E[j] = (ET)clampi(llr[j], -lim, lim);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        frame_flags(A, f)[0] = 1;
        frame_flags(A, f)[1] = 0;
        frame_flags(A, f)[2] = 0;
        if (f == 0)
            *A.mcount = A.n_frames;
    }
}

// Syndrome test of the current state: any failing row of an active frame sets
// its unsat flag (one atomic per workgroup). Layers are tested one at a time and
// a workgroup stops at the first layer with a failing row, or as soon as
// another workgroup has flagged the frame: a frame that has not converged
// almost always fails in layer 0, so the test costs a fraction of a pass.
template <int DMIN, int DMAX, typename ET>
__global__ __launch_bounds__(1024) void k_multi_check(DevCode C, DecodeArgs A)
{
    constexpr int DH = DMAX / 2;
    const int f = blockIdx.y;
    int *fl = frame_flags(A, f);
    if (!fl[0] || __atomic_load_n(&fl[1], __ATOMIC_RELAXED))
        return;
    const int tid = threadIdx.x, h = tid & 1, z = C.z, hz = z >> 1;
    const int r = blockIdx.x * (blockDim.x >> 1) + (tid >> 1);
    const bool act = r < hz;
    const unsigned zm = (unsigned)(z - 1);
    const ET *E = frame_e<ET>(A, f);
    const uint8_t *syn = A.syn + (size_t)f * A.syn_bytes;
    for (int b = 0; b < C.mb; ++b) {
        int fail = 0;
        if (act) {
            const int4 *tab = A.lane_tab + b * DH * 2 + h;
            s16x2 own = splat2(0);
#pragma unroll
            for (int i = 0; i < DH; ++i) {
                const int4 te = tab[2 * i];
                const unsigned a0 = (((unsigned)r + (unsigned)te.x) & zm) | (unsigned)te.y;
                s16x2 x;
                x.x = (short)E[a0];
                x.y = (short)E[a0 ^ (unsigned)hz];
                if (split_pad_slot<DMIN, DMAX>(i))
                    x = x & __builtin_bit_cast(s16x2, te.z);
                own ^= x;
            }
            const int i0 = b * z + r, i1 = i0 + hz;
            s16x2 sp;
            sp.x = (short)(((syn[i0 >> 3] >> (i0 & 7)) & 1) ? -1 : 0);
            sp.y = (short)(((syn[i1 >> 3] >> (i1 & 7)) & 1) ? -1 : 0);
            const s16x2 pe = sp ^ own ^ swap_pair(own);
            fail = (pe.x | pe.y) < 0;
        }
        if (__syncthreads_or(fail)) {
            if (tid == 0)
                atomicOr(&fl[1], 1);
            return;
        }
    }
}

// Retire frames: converged at iteration t (no failing row), or out of iterations.
__global__ __launch_bounds__(256) void k_multi_finalize(DecodeArgs A, int t)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= A.n_frames)
        return;
    int *fl = frame_flags(A, f);
    if (fl[0]) {
        if (!fl[1]) {
            fl[0] = 0;
            fl[2] = t;
            A.out_conv[f] = 1;
            if (A.out_iters)
                A.out_iters[f] = t;
            atomicSub(A.mcount, 1);
        } else if (t >= A.max_iter) {
            fl[0] = 0;
            fl[2] = A.max_iter;
            A.out_conv[f] = 0;
            if (A.out_iters)
                A.out_iters[f] = A.max_iter;
            atomicSub(A.mcount, 1);
        }
    }
    fl[1] = 0;
}

// Layer b of iteration t for every active frame.
template <int DMIN, int DMAX, typename ET, int RULE, bool OFF>
__global__ __launch_bounds__(1024) void k_multi_layer(DevCode C, DecodeArgs A, int b, int t)
{
    constexpr int DH = DMAX / 2;
    __shared__ int4 s_tab[2 * DH];
    const int tid = threadIdx.x, h = tid & 1, z = C.z, hz = z >> 1;
    // One workgroup per chunk of np row pairs of a frame, on a 1-D grid padded to
    // a multiple of 8. Workgroup p runs on XCD p mod 8, and XCD k takes the k-th
    // eighth of the (frame, chunk) pairs in order: neighbouring chunks of a frame,
    // whose QC-shifted E windows share their boundary lines, then meet in one L2.
    const int np = blockDim.x >> 1, ch = (hz + np - 1) / np;
    const int q = (int)(blockIdx.x & 7) * (int)(gridDim.x >> 3) + (int)(blockIdx.x >> 3);
    const int f = q / ch, chunk = q - f * ch;
    if (f >= A.n_frames || !frame_flags(A, f)[0])
        return;  // uniform over the workgroup
    if (tid < 2 * DH)
        s_tab[tid] = A.lane_tab[b * DH * 2 + tid];
    __syncthreads();
    const int r = chunk * np + (tid >> 1);
    if (r >= hz)
        return;
    const unsigned zm = (unsigned)(z - 1);
    ET *E = frame_e<ET>(A, f);
    const LRef<DH, true> Lr{frame_l(A, f) + (size_t)b * hz * LRef<DH, true>::PAIR_BYTES,
                            (unsigned)r * LRef<DH, true>::PAIR_BYTES, h};
    SplitRow<DH> R;
    const int32_t *off_row = nullptr;
    if constexpr (OFF)  // row min(t - 1, offset_iters - 1) of the offset table
        off_row = C.offsets + (size_t)(t - 1 < C.offset_iters - 1 ? t - 1 : C.offset_iters - 1) * C.n_blocks;
    load_e_global<DMIN, DMAX, ET, OFF>(R, s_tab + h, r, zm, (unsigned)hz, E, off_row);
    Lr.load(R.lk, t == 1);
    const uint8_t *syn = A.syn + (size_t)f * A.syn_bytes;
    const int i0 = b * z + r, i1 = i0 + hz;
    s16x2 sp;
    sp.x = (short)(((syn[i0 >> 3] >> (i0 & 7)) & 1) ? -1 : 0);
    sp.y = (short)(((syn[i1 >> 3] >> (i1 & 7)) & 1) ? -1 : 0);
    split_finish<DMIN, DMAX, ET, RULE, true, OFF>(C, R, Lr, sp, GlobalESink<ET>{E, (unsigned)hz});
}

// Hard decisions (wavefront ballots) and, on request, the final state.
template <int DMAX, typename ET>
__global__ __launch_bounds__(256) void k_multi_stage_out(DevCode C, DecodeArgs A)
{
    constexpr int DH = DMAX / 2;
    const int f = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const ET *E = frame_e<ET>(A, f);
    const int nwords = (C.n + 63) >> 6;
    uint8_t *ob = A.out_bits + (size_t)f * A.bit_bytes;
    const int wpb = blockDim.x >> 6;
    for (int w = blockIdx.x * wpb + (threadIdx.x >> 6); w < nwords; w += gridDim.x * wpb) {
        const int j = (w << 6) + lane;
        const bool neg = j < C.n && E[j] < 0;
        const unsigned long long mask = __ballot(neg);
        if (lane < 8) {
            const int byte = (w << 3) + lane;
            if (byte < A.bit_bytes)
                ob[byte] = (uint8_t)(mask >> (8 * lane));
        }
    }
    const int gtid = blockIdx.x * blockDim.x + threadIdx.x, gn = gridDim.x * blockDim.x;
    if (A.out_E)
        for (int j = gtid; j < C.n; j += gn)
            A.out_E[(size_t)f * C.n + j] = (int16_t)E[j];
    if (A.out_L) {
        // canonical [block][row]; L was never written when no iteration ran
        const int z = C.z, hz = z >> 1, ne = C.n_blocks * z;
        const bool none = frame_flags(A, f)[2] == 0;
        const uint8_t *Lg = frame_l(A, f);
        for (int e = gtid; e < ne; e += gn) {
            const int blk = e / z, row = e - blk * z;
            const int half = row >= hz, r = row - half * hz;
            const int v = A.blk2slot[blk];  // b * 4DH + 2 * slot + lane
            const int b = v / (4 * DH), rem = v - b * 4 * DH;
            A.out_L[(size_t)f * ne + e] =
                none ? (int8_t)0
                     : (int8_t)Lg[((size_t)b * hz + r) * LRef<DH, true>::PAIR_BYTES +
                                  LRef<DH, true>::slot_byte(rem & 1, rem >> 1) + half];
        }
    }
}

namespace {

// Launch phases: stage-in and the iteration-0 check and retirement (0),
// iterations t0..t1 (1), stage-out (2).
constexpr int kLayerThreads = 512;

template <int DMIN, int DMAX, typename ET, int RULE, bool OFF>
hipError_t run_multi(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, int phase, int t0, int t1,
                     hipStream_t s)
{
    const int F = A.n_frames, hz = C.z / 2;
    const int np = P.threads / 2;
    const dim3 rows((hz + np - 1) / np, F);
    // layer launches in smaller workgroups than the check: at the layer
    // kernel's register count a CU then holds several, and one's loads overlap
    // another's arithmetic
    const int lt = P.threads < kLayerThreads ? P.threads : kLayerThreads;
    const unsigned lch = (unsigned)((hz + lt / 2 - 1) / (lt / 2));
    const dim3 layer_grid(8 * (((unsigned)F * lch + 7) / 8));
    const dim3 elems((C.n + 1023) / 1024 < 64 ? (C.n + 1023) / 1024 : 64, F);
    const dim3 fin((F + 255) / 256);
    if (phase == 0) {
        hipLaunchKernelGGL((k_multi_stage_in<ET>), elems, dim3(256), 0, s, C, A);
        hipLaunchKernelGGL((k_multi_check<DMIN, DMAX, ET>), rows, dim3(P.threads), 0, s, C, A);
        hipLaunchKernelGGL(k_multi_finalize, fin, dim3(256), 0, s, A, 0);
        return hipGetLastError();
    }
    if (phase == 2) {
        hipLaunchKernelGGL((k_multi_stage_out<DMAX, ET>), elems, dim3(256), 0, s, C, A);
        return hipGetLastError();
    }
    hipError_t e = hipSuccess;
    for (int t = t0; t <= t1 && e == hipSuccess; ++t) {
        for (int b = 0; b < C.mb; ++b)
            hipLaunchKernelGGL((k_multi_layer<DMIN, DMAX, ET, RULE, OFF>), layer_grid, dim3(lt), 0, s, C, A, b, t);
        hipLaunchKernelGGL((k_multi_check<DMIN, DMAX, ET>), rows, dim3(P.threads), 0, s, C, A);
        hipLaunchKernelGGL(k_multi_finalize, fin, dim3(256), 0, s, A, t);
        e = hipGetLastError();
    }
    return e;
}

template <int DMIN, int DMAX, typename ET>
hipError_t run_rule(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, int phase, int t0, int t1,
                    hipStream_t s)
{
    if (C.offsets)
        return P.cn_rule == LDPC_RULE_MINSUM ? run_multi<DMIN, DMAX, ET, kRuleMinSum, true>(P, C, A, phase, t0, t1, s)
                                             : run_multi<DMIN, DMAX, ET, kRuleRcbpFB, true>(P, C, A, phase, t0, t1, s);
    if (P.cn_rule == LDPC_RULE_MINSUM)
        return run_multi<DMIN, DMAX, ET, kRuleMinSum, false>(P, C, A, phase, t0, t1, s);
    return run_multi<DMIN, DMAX, ET, kRuleRcbpFB, false>(P, C, A, phase, t0, t1, s);
}

template <typename ET>
hipError_t run_et(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, int phase, int t0, int t1,
                  hipStream_t s)
{
    switch (P.split_dmax) {
    case 6:
        return run_rule<6, 6, ET>(P, C, A, phase, t0, t1, s);
    case 8:
        return P.min_deg >= 6 ? run_rule<6, 8, ET>(P, C, A, phase, t0, t1, s)
                              : run_rule<2, 8, ET>(P, C, A, phase, t0, t1, s);
    default:
        return P.min_deg >= 19 ? run_rule<19, 20, ET>(P, C, A, phase, t0, t1, s)
                               : run_rule<2, 20, ET>(P, C, A, phase, t0, t1, s);
    }
}

hipError_t run_phase(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, int phase, int t0, int t1,
                     hipStream_t s)
{
    return P.acc_bits == 16 ? run_et<int16_t>(P, C, A, phase, t0, t1, s)
                            : run_et<int8_t>(P, C, A, phase, t0, t1, s);
}

} // namespace

hipError_t launch_multi_head(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s)
{
    return run_phase(P, C, A, 0, 0, 0, s);
}

hipError_t launch_multi_iters(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, int t0, int t1,
                              hipStream_t s)
{
    return run_phase(P, C, A, 1, t0, t1, s);
}

hipError_t launch_multi_tail(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s)
{
    return run_phase(P, C, A, 2, 0, 0, s);
}

// The whole decode, every iteration enqueued (retired frames make the later
// launches return at once).
hipError_t launch_decode_multi(const LaunchPlan &P, const DevCode &C, const DecodeArgs &A, hipStream_t s)
{
    hipError_t e = launch_multi_head(P, C, A, s);
    if (e == hipSuccess && A.max_iter > 0)
        e = launch_multi_iters(P, C, A, 1, A.max_iter, s);
    if (e == hipSuccess)
        e = launch_multi_tail(P, C, A, s);
    return e;
}

} // namespace qkdldpc
