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
// The tape keeps every v_k and E after every iteration; the backward pass walks
// layers and iterations in reverse, recomputes the minima and their indices from
// v, and propagates the adjoints of E and L. Ties go to the lowest edge index,
// d|v|/dv is 0 at v = 0 and the offset's clamp passes gradient only where
// min - beta > 0. Reductions run in a fixed order, so results are deterministic.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "oms.hpp"

namespace qkdldpc {

namespace {

__device__ __forceinline__ float wave_sum(float x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        x += __shfl_xor(x, o, 64);
    return x;
}

__device__ __forceinline__ float softplus(float u) { return fmaxf(u, 0.f) + log1pf(expf(-fabsf(u))); }

__device__ __forceinline__ float sigmoid(float u) { return 1.f / (1.f + expf(-u)); }

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

struct OmsState {
    float *E, *L;      // E [n], L [n_blocks * Z] (forward) or their adjoints (backward)
    uint8_t *syn;      // packed syndrome of the frame
    float *red;        // reduction scratch
};

__device__ __forceinline__ OmsState oms_state(const DevCode &C, const OmsArgs &A, bool lds, int red_floats)
{
    extern __shared__ __align__(16) uint8_t smem[];
    OmsState S;
    const size_t ne = (size_t)C.n_blocks * C.z;
    uint8_t *p = smem;
    if (lds) {
        S.E = reinterpret_cast<float *>(p);
        S.L = S.E + C.n;
        p += (C.n + ne) * sizeof(float);
    } else {
        S.E = A.state + (size_t)blockIdx.x * (C.n + ne);
        S.L = S.E + C.n;
    }
    S.red = reinterpret_cast<float *>(p);
    p += (size_t)red_floats * sizeof(float);
    S.syn = p;
    return S;
}

} // namespace

template <int DMAX, bool LDS>
__global__ __launch_bounds__(512) void k_oms_forward(DevCode C, OmsArgs A)
{
    const int f = blockIdx.x, tid = threadIdx.x, nthr = blockDim.x;
    const int z = C.z, n = C.n, T = A.n_iter;
    const size_t ne = (size_t)C.n_blocks * z;
    OmsState S = oms_state(C, A, LDS, 16);
    float *E = S.E, *L = S.L;
    const uint8_t *syn = A.syn + (size_t)f * A.syn_bytes;
    for (int i = tid; i < A.syn_bytes; i += nthr)
        S.syn[i] = syn[i];
    const float *llr = A.llr + (size_t)f * n;
    for (int j = tid; j < n; j += nthr)
        E[j] = llr[j];
    for (size_t e = tid; e < ne; e += nthr)
        L[e] = 0.f;
    __syncthreads();
    float *tape = A.tape + (size_t)f * T * (ne + n);
    const uint8_t *xb = A.xbits ? A.xbits + (size_t)f * A.bit_bytes : nullptr;
    float loss = 0.f;
    for (int t = 0; t < T; ++t) {
        const float *bt = A.beta + (size_t)t * C.n_blocks;
        float *tv = tape + (size_t)t * (ne + n);
        for (int b = 0; b < C.mb; ++b) {
            const int d = ldc(C.deg, b), o = ldc(C.blk_off, b);
            for (int r = tid; r < z; r += nthr) {
                float v[DMAX];
                int col[DMAX];
                const int i = b * z + r;
                int par = (S.syn[i >> 3] >> (i & 7)) & 1;
                float m1 = INFINITY, m2 = INFINITY;
                int i1 = 0;
#pragma unroll
                for (int k = 0; k < DMAX; ++k) {
                    if (k < d) {
                        const int blk = o + k;
                        const int j = ldc(C.colbase, blk) + rot(r, ldc(C.shift, blk), z);
                        const float vk = E[j] - L[(size_t)blk * z + r];
                        tv[(size_t)blk * z + r] = vk;
                        v[k] = vk;
                        col[k] = j;
                        par ^= vk < 0.f;
                        const float a = fabsf(vk);
                        if (a < m1) {
                            m2 = m1;
                            m1 = a;
                            i1 = k;
                        } else if (a < m2) {
                            m2 = a;
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < DMAX; ++k) {
                    if (k < d) {
                        const int blk = o + k;
                        const float mag = fmaxf((k == i1 ? m2 : m1) - bt[blk], 0.f);
                        const float ln = (par ^ (v[k] < 0.f)) ? -mag : mag;
                        L[(size_t)blk * z + r] = ln;
                        E[col[k]] = v[k] + ln;
                    }
                }
            }
            __syncthreads();
        }
        // E after iteration t: to the tape, and into the loss
        float *te = tv + ne;
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

template <int DMAX, bool LDS>
__global__ __launch_bounds__(512) void k_oms_backward(DevCode C, OmsArgs A)
{
    const int f = blockIdx.x, tid = threadIdx.x, nthr = blockDim.x;
    const int z = C.z, n = C.n, T = A.n_iter;
    const int lane = tid & 63, w = tid >> 6, nw = nthr >> 6;
    const size_t ne = (size_t)C.n_blocks * z;
    OmsState S = oms_state(C, A, LDS, 16 * DMAX);
    float *Eb = S.E, *Lb = S.L;  // adjoints of E and L
    const uint8_t *syn = A.syn + (size_t)f * A.syn_bytes;
    for (int i = tid; i < A.syn_bytes; i += nthr)
        S.syn[i] = syn[i];
    for (int j = tid; j < n; j += nthr)
        Eb[j] = 0.f;
    for (size_t e = tid; e < ne; e += nthr)
        Lb[e] = 0.f;
    __syncthreads();
    const float *tape = A.tape + (size_t)f * T * (ne + n);
    const uint8_t *xb = A.xbits + (size_t)f * A.bit_bytes;
    const float g = A.dloss[f] / (float)n;
    for (int t = T - 1; t >= 0; --t) {
        const float *bt = A.beta + (size_t)t * C.n_blocks;
        const float *tv = tape + (size_t)t * (ne + n);
        // the loss term of iteration t
        const float wt = (A.weights ? A.weights[t] : 1.f) * g;
        for (int j = tid; j < n; j += nthr) {
            const float y = target_sign(xb, j);
            Eb[j] += wt * sigmoid(-y * tv[ne + j]) * -y;
        }
        __syncthreads();
        for (int b = C.mb - 1; b >= 0; --b) {
            const int d = ldc(C.deg, b), o = ldc(C.blk_off, b);
            float acc[DMAX];
#pragma unroll
            for (int k = 0; k < DMAX; ++k)
                acc[k] = 0.f;
            for (int r = tid; r < z; r += nthr) {
                float v[DMAX], vb[DMAX], gk[DMAX];
                int col[DMAX];
                const int i = b * z + r;
                int par = (S.syn[i >> 3] >> (i & 7)) & 1;
                float m1 = INFINITY, m2 = INFINITY;
                int i1 = 0, i2 = 0;
#pragma unroll
                for (int k = 0; k < DMAX; ++k) {
                    if (k < d) {
                        const int blk = o + k;
                        col[k] = ldc(C.colbase, blk) + rot(r, ldc(C.shift, blk), z);
                        const float vk = tv[(size_t)blk * z + r];
                        v[k] = vk;
                        par ^= vk < 0.f;
                        const float a = fabsf(vk);
                        if (a < m1) {
                            m2 = m1;
                            i2 = i1;
                            m1 = a;
                            i1 = k;
                        } else if (a < m2) {
                            m2 = a;
                            i2 = k;
                        }
                    }
                }
                // adjoint of L_k (new) = its own adjoint + that of E_{j_k} (E = v + L)
                float g_rest = 0.f, g_i1 = 0.f;
#pragma unroll
                for (int k = 0; k < DMAX; ++k) {
                    gk[k] = 0.f;
                    if (k < d) {
                        const int blk = o + k;
                        const float eb = Eb[col[k]];
                        const float a = Lb[(size_t)blk * z + r] + eb;
                        const float sig = (par ^ (v[k] < 0.f)) ? -1.f : 1.f;
                        const bool live = (k == i1 ? m2 : m1) - bt[blk] > 0.f;
                        const float gg = live ? a * sig : 0.f;
                        gk[k] = gg;
                        acc[k] -= gg;
                        vb[k] = eb;
                        if (k == i1)
                            g_i1 = gg;
                        else
                            g_rest += gg;
                    }
                }
                // through the minima: every k != i1 read |v_i1|, k = i1 read |v_i2|
#pragma unroll
                for (int k = 0; k < DMAX; ++k) {
                    if (k < d) {
                        const float sg = v[k] > 0.f ? 1.f : v[k] < 0.f ? -1.f : 0.f;
                        if (k == i1)
                            vb[k] += sg * g_rest;
                        if (k == i2 && d > 1)
                            vb[k] += sg * g_i1;
                    }
                }
#pragma unroll
                for (int k = 0; k < DMAX; ++k) {
                    if (k < d) {
                        Eb[col[k]] = vb[k];
                        Lb[(size_t)(o + k) * z + r] = -vb[k];
                    }
                }
                (void)gk;
            }
            // offset gradients of this layer: fixed-order reduction over the workgroup
#pragma unroll
            for (int k = 0; k < DMAX; ++k) {
                if (k < d) {
                    const float s = wave_sum(acc[k]);
                    if (lane == 0)
                        S.red[w * DMAX + k] = s;
                }
            }
            __syncthreads();
            if (tid < d) {
                float s = 0.f;
                for (int q = 0; q < nw; ++q)
                    s += S.red[q * DMAX + tid];
                A.dbeta_frames[((size_t)f * T + t) * C.n_blocks + o + tid] = s;
            }
            __syncthreads();
        }
    }
    if (A.dllr)
        for (int j = tid; j < n; j += nthr)
            A.dllr[(size_t)f * n + j] = Eb[j];
}

// dbeta[q] = sum over frames of dbeta_frames[f][q], in frame order
__global__ void k_oms_sum_frames(const float *__restrict__ part, int n_frames, int per_frame, float *__restrict__ out)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= per_frame)
        return;
    float s = 0.f;
    for (int f = 0; f < n_frames; ++f)
        s += part[(size_t)f * per_frame + q];
    out[q] = s;
}

namespace {

template <int DMAX>
hipError_t fwd(const OmsPlan &P, const DevCode &C, const OmsArgs &A, hipStream_t s)
{
    if (P.lds_state) {
        if (P.lds_bytes > 65536) {
            hipError_t e = allow_max_lds<k_oms_forward<DMAX, true>>();
            if (e != hipSuccess)
                return e;
        }
        hipLaunchKernelGGL((k_oms_forward<DMAX, true>), dim3(A.n_frames), dim3(P.threads), P.lds_bytes, s, C, A);
    } else {
        hipLaunchKernelGGL((k_oms_forward<DMAX, false>), dim3(A.n_frames), dim3(P.threads), P.lds_bytes, s, C, A);
    }
    return hipGetLastError();
}

template <int DMAX>
hipError_t bwd(const OmsPlan &P, const DevCode &C, const OmsArgs &A, hipStream_t s)
{
    if (A.n_frames == 0) {
        // nothing to differentiate: the frame sum writes zeros
    } else if (P.lds_state) {
        if (P.lds_bytes > 65536) {
            hipError_t e = allow_max_lds<k_oms_backward<DMAX, true>>();
            if (e != hipSuccess)
                return e;
        }
        hipLaunchKernelGGL((k_oms_backward<DMAX, true>), dim3(A.n_frames), dim3(P.threads), P.lds_bytes, s, C, A);
    } else {
        hipLaunchKernelGGL((k_oms_backward<DMAX, false>), dim3(A.n_frames), dim3(P.threads), P.lds_bytes, s, C, A);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const int per = A.n_iter * C.n_blocks;
    hipLaunchKernelGGL(k_oms_sum_frames, dim3((per + 255) / 256), dim3(256), 0, s, A.dbeta_frames, A.n_frames, per,
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
