// Differentiable FP32 offset min-sum with learned offsets (per iteration and
// per base-matrix edge): forward pass with the training loss, and its backward
// pass. The schedule is the layered one of Sec. 2 (Eqs. 8 and 9) with the check
// node simplified to offset min-sum and the syndrome sign of syndrome decoding;
// T iterations run without early stopping so the decode is a fixed function of
// the offsets.
//
// Forward, per row i of layer b with edges k to columns j_k:
//   v_k = E_{j_k} - L_k
//   sigma_k = (-1)^{s_i} prod_k' sgn(v_k') sgn(v_k), sgn(0) = +1
//   L_k = sigma_k max(min_{k' != k} |v_k'| - beta_{t, blk_k}, 0),  E_{j_k} = v_k + L_k
// and after iteration t the loss gains w_t / n * sum_j softplus(-(1 - 2 x_j) E_j).
// The backward pass needs, of every row's v, only its minimum and second minimum
// (values and edge indices) and the signs: the tape keeps that record per check
// row and iteration (four words: m1, m2, the sign bits of v by edge, i1 | i2 << 8)
// and E after every iteration. The same record and the offsets of its iteration
// give every L_k of the row, so the forward pass keeps E and one record per row
// on chip instead of a value per edge (for n = 8192 that is 53 KB instead of
// 128 KB, and two frames share a CU). The backward pass walks layers and iterations in
// reverse and propagates the adjoints of E and L. Ties go to the lowest edge
// index, d|v|/dv is 0 at v = 0 and the offset's clamp passes gradient only where
// min - beta > 0. Reductions run in a fixed order, so results are deterministic.
//
// Four lanes (a quad) share a row: lane q holds the row's edges
// k in [q * S, (q + 1) * S), S = DMAX / 4, in registers. The row's sign parity,
// minimum (with its edge index), second minimum (with its index) are combined
// across the quad with two xor-shuffles; ties compare (value, index), so the
// lowest index wins as in the sequential definition. The adjoint of L is laid
// out per layer as [row][edge] (layer b starts at blk_off[b] * Z), so a quad
// reads and writes contiguous words; lane q of a quad writes word q of the row's
// record.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "oms.hpp"

namespace qkdldpc {

namespace {

constexpr int kQuad = 4;

__device__ __forceinline__ float wave_sum(float x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        x += __shfl_xor(x, o, 64);
    return x;
}

// softplus(u) = max(u, 0) + log(1 + exp(-|u|)) and the logistic function, on
// the hardware exp2/log2/reciprocal approximations (about one ulp each): the
// loss is a sum of positive terms, so the absolute error of log(1 + t) when
// 1 + t rounds (at most half an ulp of 1 per term) is far below the loss's
// own rounding; the logistic function feeds gradients only.
__device__ __forceinline__ float softplus(float u) { return fmaxf(u, 0.f) + __logf(1.f + __expf(-fabsf(u))); }

__device__ __forceinline__ float sigmoid(float u) { return __builtin_amdgcn_rcpf(1.f + __expf(-u)); }

// +1 for a target bit 0, -1 for 1
__device__ __forceinline__ float target_sign(const uint8_t *xb, int j) { return (xb[j >> 3] >> (j & 7)) & 1 ? -1.f : 1.f; }

// Sum over the workgroup in a fixed order; red holds one float per wave. The
// result is valid in thread 0.
__device__ __forceinline__ float block_sum(float x, float *red)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    x = wave_sum(x);
    if (lane == 0)
        red[w] = x;
    __syncthreads();
    float s = 0.f;
    if (threadIdx.x == 0)
        for (int i = 0; i < nw; ++i)
            s += red[i];
    __syncthreads();
    return s;
}

// (m1, i1): smallest |v| and its edge index; (m2, i2): smallest among the other
// edges and its index; par: xor of the sign bits and the syndrome bit.
struct RowMin {
    float m1, m2;
    int i1, i2, par;
};

__device__ __forceinline__ bool lex_less(float a, int ia, float b, int ib) { return a < b || (a == b && ia < ib); }

// Value of the quad partner at xor distance O (1 or 2): a DPP quad permutation,
// [1,0,3,2] or [2,3,0,1]; every lane of the wave takes part.
template <int O>
__device__ __forceinline__ int quad_xor(int x)
{
    static_assert(O == 1 || O == 2, "quad partner");
    return __builtin_amdgcn_update_dpp(0, x, O == 1 ? 0xB1 : 0x4E, 0xF, 0xF, false);
}
template <int O>
__device__ __forceinline__ float quad_xor(float x)
{
    return __builtin_bit_cast(float, quad_xor<O>(__builtin_bit_cast(int, x)));
}

// Combine with the quad partner at xor distance O.
template <int O>
__device__ __forceinline__ RowMin quad_combine(RowMin a)
{
    RowMin b;
    b.m1 = quad_xor<O>(a.m1);
    b.m2 = quad_xor<O>(a.m2);
    b.i1 = quad_xor<O>(a.i1);
    b.i2 = quad_xor<O>(a.i2);
    b.par = quad_xor<O>(a.par);
    RowMin r;
    r.par = a.par ^ b.par;
    const bool aw = lex_less(a.m1, a.i1, b.m1, b.i1);
    const RowMin &w = aw ? a : b, &l = aw ? b : a;
    r.m1 = w.m1;
    r.i1 = w.i1;
    // second: the better of the winner's second and the loser's first
    const bool s2 = lex_less(w.m2, w.i2, l.m1, l.i1);
    r.m2 = s2 ? w.m2 : l.m1;
    r.i2 = s2 ? w.i2 : l.i1;
    return r;
}

struct OmsState {
    float *E, *L;      // forward: E [n] and the row records [m][4] (at a 16-byte
                       // boundary); backward: the adjoints of E [n] and L [n_blocks * Z]
    int2 *blk;         // per block {column start c*Z, circulant shift}, staged in LDS
    float *beta;       // offsets [T][n_blocks] staged in LDS
    float *red;        // reduction scratch
    uint8_t *syn;      // packed syndrome of the frame
    uint8_t *xb;       // packed target bits of the frame (when given)
};

// LDS: [state if LDS] [block table, 16-byte aligned] [beta T * n_blocks] [red] [syndrome,
// 16-byte padded] [target bits]
// second: floats of the second state array (4m forward, n_blocks * Z backward).
// Both arrays start at 16-byte boundaries (each is padded to a multiple of four
// floats), in LDS and in the per-frame global slices alike.
__device__ __forceinline__ OmsState oms_state(const DevCode &C, const OmsArgs &A, bool lds, int red_floats,
                                              size_t second)
{
    extern __shared__ __align__(16) uint8_t smem[];
    OmsState S;
    const size_t n4 = ((size_t)C.n + 3) & ~(size_t)3, st = n4 + ((second + 3) & ~(size_t)3);
    uint8_t *p = smem;
    if (lds) {
        S.E = reinterpret_cast<float *>(p);
        S.L = S.E + n4;
        p += st * sizeof(float);
    } else {
        S.E = A.state + (size_t)blockIdx.x * st;
        S.L = S.E + n4;
    }
    S.blk = reinterpret_cast<int2 *>(p);
    p += (size_t)C.n_blocks * sizeof(int2);
    S.beta = reinterpret_cast<float *>(p);
    p += (size_t)A.n_iter * C.n_blocks * sizeof(float);
    S.red = reinterpret_cast<float *>(p);
    p += (size_t)red_floats * sizeof(float);
    S.syn = p;
    p += ((size_t)A.syn_bytes + 15) & ~(size_t)15;
    S.xb = p;
    return S;
}

__device__ __forceinline__ void stage_common(const DevCode &C, const OmsArgs &A, const OmsState &S)
{
    const int tid = threadIdx.x, nthr = blockDim.x;
    const uint8_t *syn = A.syn + (size_t)blockIdx.x * A.syn_bytes;
    for (int i = tid; i < A.syn_bytes; i += nthr)
        S.syn[i] = syn[i];
    if (A.xbits) {
        const uint8_t *xb = A.xbits + (size_t)blockIdx.x * A.bit_bytes;
        for (int i = tid; i < A.bit_bytes; i += nthr)
            S.xb[i] = xb[i];
    }
    for (int i = tid; i < A.n_iter * C.n_blocks; i += nthr)
        S.beta[i] = A.beta[i];
    for (int i = tid; i < C.n_blocks; i += nthr)
        S.blk[i] = int2{ldc(C.colbase, i), ldc(C.shift, i)};
}

} // namespace

// Two workgroups per CU for rows of up to 20 edges with the state in LDS (64
// VGPRs, and the forward state E + row records is small enough for two in LDS).
template <int DMAX, bool LDS>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(DMAX <= 20 && LDS ? 8 : 1)))
void k_oms_forward(DevCode C, OmsArgs A)
{
    constexpr int SL = DMAX / kQuad;  // edges per lane
    const int f = blockIdx.x, tid = threadIdx.x, nthr = blockDim.x;
    const int z = C.z, n = C.n, T = A.n_iter;
    const int q = tid & (kQuad - 1), rq = tid / kQuad, nq = nthr / kQuad;
    OmsState S = oms_state(C, A, LDS, 16, (size_t)4 * C.m);
    float *E = S.E;
    // The row's CN->VN values of the last iteration are a function of its record
    // (m1, m2, sign bits, i1 | i2 << 8) and that iteration's offsets, so the
    // forward keeps one record per row instead of a value per edge.
    float4 *Rec = reinterpret_cast<float4 *>(S.L);
    stage_common(C, A, S);
    const float *llr = A.llr + (size_t)f * n;
    for (int j = tid; j < n; j += nthr)
        E[j] = llr[j];
    __syncthreads();
    const size_t per_iter = (size_t)4 * C.m + ((n + 3) & ~3);  // row records, then E (16-byte rows)
    float *tape = A.tape + (size_t)f * T * per_iter;
    const uint8_t *xb = A.xbits ? S.xb : nullptr;
    float loss = 0.f;
    for (int t = 0; t < T; ++t) {
        const float *bt = S.beta + t * C.n_blocks;
        const float *bp = S.beta + (t > 0 ? t - 1 : 0) * C.n_blocks;  // offsets of the record's iteration
        float *tv = tape + (size_t)t * per_iter;
        for (int b = 0; b < C.mb; ++b) {
            const int d = ldc(C.deg, b), o = ldc(C.blk_off, b);
            // all lanes of a quad take part in the shuffles, so the row loop is
            // uniform across the quad (rows past Z are masked per lane)
            for (int r0 = 0; r0 < z; r0 += nq) {
                const int r = r0 + rq;
                const bool act = r < z;
                const int i = b * z + r;
                const int sbit = act ? (S.syn[i >> 3] >> (i & 7)) & 1 : 0;
                // the row's record of iteration t - 1 (all four lanes read the same 16 bytes)
                float4 rp = make_float4(0.f, 0.f, 0.f, 0.f);
                if (act && t > 0)
                    rp = Rec[i];
                const unsigned psb = __builtin_bit_cast(unsigned, rp.z);
                const int pi1 = __builtin_bit_cast(int, rp.w) & 0xff;
                const unsigned ppar = (unsigned)sbit ^ (__builtin_popcount(psb) & 1);
                float v[SL];
                int col[SL];
                RowMin M;
                M.m1 = M.m2 = INFINITY;
                M.i1 = M.i2 = DMAX;
                M.par = q == 0 ? sbit : 0;
#pragma unroll
                for (int s = 0; s < SL; ++s) {
                    const int k = q * SL + s;
                    v[s] = 0.f;
                    col[s] = 0;
                    if (act && k < d) {
                        const int2 cs = S.blk[o + k];
                        const int j = cs.x + rot(r, cs.y, z);
                        // L of this edge from iteration t - 1 (0 before the first)
                        float lo = 0.f;
                        if (t > 0) {
                            const float mag = fmaxf((k == pi1 ? rp.y : rp.x) - bp[o + k], 0.f);
                            lo = (ppar ^ ((psb >> k) & 1)) ? -mag : mag;
                        }
                        const float vk = E[j] - lo;
                        v[s] = vk;
                        col[s] = j;
                        M.par ^= vk < 0.f;
                        const float a = fabsf(vk);
                        if (a < M.m1) {
                            M.m2 = M.m1;
                            M.i2 = M.i1;
                            M.m1 = a;
                            M.i1 = k;
                        } else if (a < M.m2) {
                            M.m2 = a;
                            M.i2 = k;
                        }
                    }
                }
                M = quad_combine<1>(M);
                M = quad_combine<2>(M);
                // the row's record: sign bits of v by edge index, combined over the quad;
                // lane q writes word q, to LDS (read back in iteration t + 1) and to the tape
                unsigned sb = 0;
#pragma unroll
                for (int s = 0; s < SL; ++s)
                    sb |= (unsigned)(v[s] < 0.f) << (q * SL + s);
                sb |= (unsigned)quad_xor<1>((int)sb);
                sb |= (unsigned)quad_xor<2>((int)sb);
                if (act) {
                    const float rec = q == 0   ? M.m1
                                      : q == 1 ? M.m2
                                      : q == 2 ? __builtin_bit_cast(float, sb)
                                               : __builtin_bit_cast(float, M.i1 | M.i2 << 8);
                    S.L[(size_t)i * 4 + q] = rec;
                    tv[(size_t)i * 4 + q] = rec;
                }
#pragma unroll
                for (int s = 0; s < SL; ++s) {
                    const int k = q * SL + s;
                    if (act && k < d) {
                        const float mag = fmaxf((k == M.i1 ? M.m2 : M.m1) - bt[o + k], 0.f);
                        const float ln = (M.par ^ (v[s] < 0.f)) ? -mag : mag;
                        E[col[s]] = v[s] + ln;
                    }
                }
            }
            __syncthreads();
        }
        // E after iteration t: to the tape, and into the loss
        float *te = tv + (size_t)4 * C.m;
        float part = 0.f;
        for (int j = tid; j < n; j += nthr) {
            const float e = E[j];
            te[j] = e;
            if (xb)
                part += softplus(-target_sign(xb, j) * e);
        }
        const float s = block_sum(part, S.red);
        if (tid == 0)
            loss += (A.weights ? A.weights[t] : 1.f) * s / (float)n;
    }
    if (tid == 0 && A.out_loss)
        A.out_loss[f] = loss;
    if (A.out_E)
        for (int j = tid; j < n; j += nthr)
            A.out_E[(size_t)f * n + j] = E[j];
}

// MBR > 0: the adjoint of L lives in registers, MBR layers of SL slots per lane.
// That needs every row of a layer handled by one quad in one pass (4 Z <= the
// workgroup) and at most MBR layers; each lane then owns the same row and edge
// slots in every layer and iteration, so the adjoint it reads is the one it
// wrote. Otherwise (MBR = 0) the adjoint of L is laid out [layer][row][edge] in
// the state.
template <int DMAX, bool LDS, int MBR>
__global__ __launch_bounds__(1024) void k_oms_backward(DevCode C, OmsArgs A)
{
    constexpr int SL = DMAX / kQuad;
    const int f = blockIdx.x, tid = threadIdx.x, nthr = blockDim.x;
    const int z = C.z, n = C.n, T = A.n_iter;
    const int q = tid & (kQuad - 1), rq = tid / kQuad, nq = nthr / kQuad;
    const int lane = tid & 63, w = tid >> 6, nw = nthr >> 6;
    const size_t ne = (size_t)C.n_blocks * z;
    OmsState S = oms_state(C, A, LDS, 16 * DMAX, ne);
    float *Eb = S.E, *Lb = S.L;  // adjoints of E and L
    stage_common(C, A, S);
    for (int j = tid; j < n; j += nthr)
        Eb[j] = 0.f;
    if constexpr (MBR == 0)
        for (size_t e = tid; e < ne; e += nthr)
            Lb[e] = 0.f;
    float lreg[MBR > 0 ? MBR : 1][SL];
#pragma unroll
    for (int b = 0; b < (MBR > 0 ? MBR : 1); ++b)
#pragma unroll
        for (int s = 0; s < SL; ++s)
            lreg[b][s] = 0.f;
    __syncthreads();
    const size_t per_iter = (size_t)4 * C.m + ((n + 3) & ~3);  // row records, then E (16-byte rows)
    const float *tape = A.tape + (size_t)f * T * per_iter;
    const uint8_t *xb = S.xb;
    const float g = A.dloss[f] / (float)n;
    // The tape record of the next row chunk in walk order (layers and iterations
    // in reverse) is requested while the current chunk is processed, so its
    // global latency overlaps that work and the layer barriers.
    float4 rnext;
    auto fetch_rec = [&](int t, int b, int r0) {
        const int r = r0 + rq;
        rnext = r < z ? reinterpret_cast<const float4 *>(tape + (size_t)t * per_iter)[(size_t)b * z + r]
                      : make_float4(0.f, 0.f, 0.f, 0.f);
    };
    fetch_rec(T - 1, C.mb - 1, 0);
    for (int t = T - 1; t >= 0; --t) {
        const float *bt = S.beta + t * C.n_blocks;
        const float *tv = tape + (size_t)t * per_iter;
        // the loss term of iteration t
        const float wt = (A.weights ? A.weights[t] : 1.f) * g;
        // four tape reads in flight per thread
        for (int j0 = tid; j0 < n; j0 += 4 * nthr) {
            float e4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = j0 + u * nthr;
                e4[u] = j < n ? tv[(size_t)4 * C.m + j] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = j0 + u * nthr;
                if (j < n) {
                    const float y = target_sign(xb, j);
                    Eb[j] += wt * sigmoid(-y * e4[u]) * -y;
                }
            }
        }
        __syncthreads();
        // layer b; lr: this lane's register adjoints of L for the layer (MBR > 0)
        auto layer = [&](int b, float(&lr)[SL]) {
            const int d = ldc(C.deg, b), o = ldc(C.blk_off, b);
            const size_t lb = (size_t)o * z;
            float acc[SL];
#pragma unroll
            for (int s = 0; s < SL; ++s)
                acc[s] = 0.f;
            for (int r0 = 0; r0 < z; r0 += nq) {
                const int r = r0 + rq;
                const bool act = r < z;
                float vb[SL];
                int col[SL];
                const float4 rec = rnext;
                if (r0 + nq < z)
                    fetch_rec(t, b, r0 + nq);
                else if (b > 0)
                    fetch_rec(t, b - 1, 0);
                else if (t > 0)
                    fetch_rec(t - 1, C.mb - 1, 0);
                // the forward pass's minima, indices and signs of this row
                RowMin M;
                M.m1 = rec.x;
                M.m2 = rec.y;
                const unsigned sb = __builtin_bit_cast(unsigned, rec.z);
                const int ii = __builtin_bit_cast(int, rec.w);
                M.i1 = ii & 0xff;
                M.i2 = ii >> 8;
                M.par = __builtin_popcount(sb) & 1;
                if (act) {
                    const int i = b * z + r;
                    M.par ^= (S.syn[i >> 3] >> (i & 7)) & 1;
                }
#pragma unroll
                for (int s = 0; s < SL; ++s) {
                    const int k = q * SL + s;
                    col[s] = 0;
                    if (act && k < d) {
                        const int2 cs = S.blk[o + k];
                        col[s] = cs.x + rot(r, cs.y, z);
                    }
                }
                // adjoint of L_k (new) = its own adjoint + that of E_{j_k} (E = v + L)
                float g_rest = 0.f, g_i1 = 0.f;
#pragma unroll
                for (int s = 0; s < SL; ++s) {
                    const int k = q * SL + s;
                    vb[s] = 0.f;
                    if (act && k < d) {
                        const int blk = o + k;
                        const float eb = Eb[col[s]];
                        const float a = (MBR > 0 ? lr[s] : Lb[lb + (size_t)r * d + k]) + eb;
                        const float sig = (M.par ^ ((sb >> k) & 1)) ? -1.f : 1.f;
                        const bool live = (k == M.i1 ? M.m2 : M.m1) - bt[blk] > 0.f;
                        const float gg = live ? a * sig : 0.f;
                        acc[s] -= gg;
                        vb[s] = eb;
                        if (k == M.i1)
                            g_i1 = gg;
                        else
                            g_rest += gg;
                    }
                }
                // every k != i1 read |v_i1|, k = i1 read |v_i2|: sum over the quad
                g_rest += quad_xor<1>(g_rest);
                g_rest += quad_xor<2>(g_rest);
                g_i1 += quad_xor<1>(g_i1);
                g_i1 += quad_xor<2>(g_i1);
#pragma unroll
                for (int s = 0; s < SL; ++s) {
                    const int k = q * SL + s;
                    if (act && k < d) {
                        // sgn(v_k): |v_i1| = m1, |v_i2| = m2, and the sign bit
                        const float sgn = (sb >> k) & 1 ? -1.f : 1.f;
                        if (k == M.i1 && M.m1 != 0.f)
                            vb[s] += sgn * g_rest;
                        if (k == M.i2 && M.m2 != 0.f)
                            vb[s] += sgn * g_i1;
                        Eb[col[s]] = vb[s];
                        if constexpr (MBR > 0)
                            lr[s] = -vb[s];
                        else
                            Lb[lb + (size_t)r * d + k] = -vb[s];
                    }
                }
            }
            // offset gradients of this layer: fixed-order reduction over the
            // workgroup (per edge slot: the quads of a wave, then the waves)
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                float x = acc[s];
#pragma unroll
                for (int o2 = 32; o2 >= kQuad; o2 >>= 1)
                    x += __shfl_xor(x, o2, 64);
                if (lane < kQuad && lane * SL + s < d)
                    S.red[w * DMAX + lane * SL + s] = x;
            }
            __syncthreads();
            if (tid < d) {
                float s = 0.f;
                for (int qq = 0; qq < nw; ++qq)
                    s += S.red[qq * DMAX + tid];
                A.dbeta_frames[((size_t)f * T + t) * C.n_blocks + o + tid] = s;
            }
            __syncthreads();
        };
        if constexpr (MBR > 0) {
#pragma unroll
            for (int b = MBR - 1; b >= 0; --b)
                if (b < C.mb)
                    layer(b, lreg[b]);
        } else {
            for (int b = C.mb - 1; b >= 0; --b)
                layer(b, lreg[0]);
        }
    }
    if (A.dllr)
        for (int j = tid; j < n; j += nthr)
            A.dllr[(size_t)f * n + j] = Eb[j];
}

// dbeta[q] = sum over frames of dbeta_frames[f][q] in a fixed order: the
// frames split into kSumGroups contiguous groups, each summed in frame order by
// its own lane (loads eight at a time), then the group sums in group order, so
// the result is the same on every run.
constexpr int kSumGroups = 8, kSumCols = 32;
__global__ __launch_bounds__(kSumGroups * kSumCols) void k_oms_sum_frames(const float *__restrict__ part, int n_frames,
                                                                        int per_frame, float *__restrict__ out)
{
    __shared__ float partial[kSumGroups][kSumCols];
    const int c = threadIdx.x % kSumCols, g = threadIdx.x / kSumCols;
    const int q = blockIdx.x * kSumCols + c;
    const int per_group = (n_frames + kSumGroups - 1) / kSumGroups;
    const int f0 = g * per_group, f1 = min(n_frames, f0 + per_group);
    float s = 0.f;
    if (q < per_frame) {
        int f = f0;
        for (; f + 8 <= f1; f += 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                v[u] = part[(size_t)(f + u) * per_frame + q];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                s += v[u];
        }
        for (; f < f1; ++f)
            s += part[(size_t)f * per_frame + q];
    }
    partial[g][c] = s;
    __syncthreads();
    if (g == 0 && q < per_frame) {
        float t = 0.f;
        for (int i = 0; i < kSumGroups; ++i)
            t += partial[i][c];
        out[q] = t;
    }
}

namespace {

template <int DMAX>
hipError_t fwd(const OmsPlan &P, const DevCode &C, const OmsArgs &A, hipStream_t s)
{
    if (P.fwd_lds_state) {
        if (P.fwd_lds_bytes > 65536) {
            hipError_t e = allow_max_lds<k_oms_forward<DMAX, true>>();
            if (e != hipSuccess)
                return e;
        }
        hipLaunchKernelGGL((k_oms_forward<DMAX, true>), dim3(A.n_frames), dim3(P.threads), P.fwd_lds_bytes, s, C,
                           A);
    } else {
        if (P.fwd_lds_bytes > 65536) {
            hipError_t e = allow_max_lds<k_oms_forward<DMAX, false>>();
            if (e != hipSuccess)
                return e;
        }
        hipLaunchKernelGGL((k_oms_forward<DMAX, false>), dim3(A.n_frames), dim3(P.threads), P.fwd_lds_bytes, s, C,
                           A);
    }
    return hipGetLastError();
}

template <int DMAX, bool LDS, int MBR>
hipError_t bwd_launch(const OmsPlan &P, const DevCode &C, const OmsArgs &A, hipStream_t s)
{
    if (P.lds_bytes > 65536) {
        hipError_t e = allow_max_lds<k_oms_backward<DMAX, LDS, MBR>>();
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL((k_oms_backward<DMAX, LDS, MBR>), dim3(A.n_frames), dim3(P.threads), P.lds_bytes, s, C, A);
    return hipGetLastError();
}

// layers whose adjoint of L the backward keeps in registers (row degrees up to 20)
constexpr int kBwdRegLayers = 8;

template <int DMAX>
hipError_t bwd(const OmsPlan &P, const DevCode &C, const OmsArgs &A, hipStream_t s)
{
    // one pass of the quads covers a layer's rows, and few enough layers
    const bool regs = DMAX <= 20 && P.threads / kQuad >= C.z && C.mb <= kBwdRegLayers;
    hipError_t e0 = hipSuccess;
    if (A.n_frames == 0) {
        // nothing to differentiate: the frame sum writes zeros
    } else if (P.lds_state) {
        e0 = regs ? bwd_launch<DMAX, true, DMAX <= 20 ? kBwdRegLayers : 0>(P, C, A, s)
                  : bwd_launch<DMAX, true, 0>(P, C, A, s);
    } else {
        e0 = regs ? bwd_launch<DMAX, false, DMAX <= 20 ? kBwdRegLayers : 0>(P, C, A, s)
                  : bwd_launch<DMAX, false, 0>(P, C, A, s);
    }
    if (e0 != hipSuccess)
        return e0;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const int per = A.n_iter * C.n_blocks;
    hipLaunchKernelGGL(k_oms_sum_frames, dim3((per + kSumCols - 1) / kSumCols), dim3(kSumGroups * kSumCols), 0, s,
                       A.dbeta_frames, A.n_frames, per,
                       A.dbeta);
    return hipGetLastError();
}

} // namespace

hipError_t launch_oms_forward(const OmsPlan &P, const DevCode &C, const OmsArgs &A, hipStream_t s)
{
    switch (P.dmax) {
    case 8:
        return fwd<8>(P, C, A, s);
    case 20:
        return fwd<20>(P, C, A, s);
    default:
        return fwd<32>(P, C, A, s);
    }
}

hipError_t launch_oms_backward(const OmsPlan &P, const DevCode &C, const OmsArgs &A, hipStream_t s)
{
    switch (P.dmax) {
    case 8:
        return bwd<8>(P, C, A, s);
    case 20:
        return bwd<20>(P, C, A, s);
    default:
        return bwd<32>(P, C, A, s);
    }
}

} // namespace qkdldpc
