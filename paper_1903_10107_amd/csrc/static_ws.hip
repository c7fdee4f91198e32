// ldpc_decode_batch_static: ldpc_decode_batch_sched with its workspace in a
// file-scope device array instead of memory the library or the caller
// allocates, for callers that cannot allocate device memory.
//
// The array is a host-side stand-in in host code: its device address comes from
// hipGetSymbolAddress, taken once per device with that device current and kept
// per device (each device holds its own copy of the array at its own address).
// Only that address is ever passed to kernels.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "../../include/qkdldpc.h"
#include "decoder.hpp"

namespace {

static __device__ __align__(256) uint8_t scratch[LDPC_STATIC_WORKSPACE_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void *g_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (nullptr and an error message
// when it cannot be had).
int scratch_ptr(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return qkdldpc::set_error(LDPC_EDEVICE, std::string("ldpc_decode_batch_static: hipGetDevice: ") +
                                                    hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return qkdldpc::set_error(LDPC_EUNSUPPORTED, "ldpc_decode_batch_static: device index out of range");
    std::lock_guard<std::mutex> g(g_lock);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return qkdldpc::set_error(LDPC_EDEVICE, std::string("ldpc_decode_batch_static: hipGetSymbolAddress: ") +
                                                        hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return LDPC_OK;
}

} // namespace

extern "C" int ldpc_decode_batch_static(const ldpc_code *code, const uint8_t *syndromes, const int8_t *llr_in,
                                        int32_t n_frames, int32_t max_iter, uint8_t *out_bits,
                                        uint8_t *out_converged, int32_t *out_iters, const ldpc_schedule *sched,
                                        void *stream)
{
    if (!code)
        return qkdldpc::set_error(LDPC_EINVAL, "ldpc_decode_batch_static: code is NULL");
    if (sched && sched->check_every > 0)
        return qkdldpc::set_error(LDPC_EUNSUPPORTED,
                                  "ldpc_decode_batch_static: check_every > 0 reads back to the host; use 0");
    const size_t need = ldpc_workspace_bytes_sched(code, n_frames, sched);
    if (need > (size_t)LDPC_STATIC_WORKSPACE_BYTES)
        return qkdldpc::set_error(LDPC_EINVAL, "ldpc_decode_batch_static: the decode needs " + std::to_string(need) +
                                                   " workspace bytes, above the static limit of " +
                                                   std::to_string((size_t)LDPC_STATIC_WORKSPACE_BYTES));
    void *ws = nullptr;
    if (need > 0) {
        const int rc = scratch_ptr(&ws);
        if (rc != LDPC_OK)
            return rc;
    }
    // with a workspace of the queried size the decode allocates nothing; the
    // kernels initialise every part of it they read (queue reset kernel, stage-in)
    return ldpc_decode_batch_sched(code, syndromes, llr_in, n_frames, max_iter, out_bits, out_converged, out_iters,
                                   sched, ws, need, stream);
}
