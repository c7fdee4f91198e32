// C ABI of the decoder library (declarations and contracts in include/qkdldpc.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/qkdldpc.h"
#include "decoder.hpp"
#include "oms.hpp"
#include "qc_code.hpp"
#include "rcbp.hpp"

using qkdldpc::DecodeArgs;
using qkdldpc::DevCode;
using qkdldpc::HostCode;
using qkdldpc::LaunchPlan;

struct ldpc_code {
    HostCode h;
    int device = -1;
    int32_t *d_tables = nullptr; // deg[mb] | blk_off[mb] | colbase | shift | colshift [n_blocks each]
    int32_t *d_offsets = nullptr;
    void *d_split = nullptr;     // split kernel: lane table [mb][DMAX/2][2] int4, then blk2slot [n_blocks]
    size_t lane_tab_bytes = 0;
    int lds_tab_off = 0;
    DevCode dev{};
    LaunchPlan plan{};
    size_t ws_frame_bytes = 0, ws_l_off = 0;
    int lds_e_off = 0, lds_l_off = 0, lds_syn_off = 0, lds_flag_off = 0, l_stride = 0;
    int lds_limit = 0;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

} // namespace

// Error reporting for the library's other source files.
int qkdldpc::set_error(int code, const std::string &msg) { return fail(code, msg); }

namespace {

int hip_fail(const char *what, hipError_t e)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return LDPC_EDEVICE;
}

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Per-lane slot table of the split kernel: lane A's slot i is edge i of the
// layer, lane B's slot i is edge DMAX-1-i; edges past the row degree are
// padding and point at the dummy block column nb.
std::vector<int32_t> split_tables(const HostCode &h, int dmax)
{
    const int dh = dmax / 2;
    std::vector<int32_t> t((size_t)h.mb * dh * 2 * 4 + h.n_blocks, 0);
    int32_t *b2s = t.data() + (size_t)h.mb * dh * 2 * 4;
    for (int b = 0; b < h.mb; ++b)
        for (int i = 0; i < dh; ++i)
            for (int lane = 0; lane < 2; ++lane) {
                const int g = lane ? dmax - 1 - i : i;
                int32_t *e = t.data() + (((size_t)b * dh + i) * 2 + lane) * 4;
                if (g < h.deg[b]) {
                    const int blk = h.blk_off[b] + g;
                    e[0] = h.colbase[blk] | h.shift[blk];
                    e[1] = h.colbase[blk];
                    e[2] = -1;
                    e[3] = blk;
                    b2s[blk] = b * 4 * dh + 2 * i + lane;
                } else {
                    e[0] = 0;
                    e[1] = h.nb * h.z;
                    e[2] = 0;
                    e[3] = -1;
                }
            }
    return t;
}

// Kernel families in order of preference; each applies under its own conditions.
// Returns false when the requested family (hint > 0) does not apply.
bool make_plan(ldpc_code *c, int lds_limit, int hint)
{
    const HostCode &h = c->h;
    const size_t esize = h.acc_bits == 16 ? 2 : 1;
    LaunchPlan &P = c->plan;
    P.acc_bits = h.acc_bits;
    P.cn_rule = h.cn_rule;
    P.min_deg = h.min_deg;
    P.max_deg = h.max_deg;
    P.pow2 = (h.z & (h.z - 1)) == 0;
    P.pairs = false;
    P.split_dmax = 0;
    const size_t syn_bytes = (size_t)(h.m + 7) / 8;
    const size_t e_al = round_up((size_t)h.n * esize, 16);

    // Split (two lanes per row pair): power-of-two Z, forward-backward or min-sum
    // rule, row degree <= 20. LDS: E plus a dummy block column, L as
    // [pair][layer][half][slot][lane] with an odd-dword pair stride, the
    // syndrome, the lane table, three vote words and the queue slot. When L does
    // not fit, it moves to a global slice per workgroup (mb * Z * DMAX bytes)
    // and only E, the syndrome, the table and the vote words stay in LDS.
    P.split_global_l = false;
    P.layer_sync = false;
    const bool split_hint = hint == LDPC_HINT_SPLIT || hint == LDPC_HINT_SPLIT_GLOBAL_L;
    const bool split_ok = P.pow2 && h.z >= 2 && h.max_deg <= 20 &&
                          (h.cn_rule == LDPC_RULE_RCBP_FB || h.cn_rule == LDPC_RULE_MINSUM);
    const int dmax = (h.min_deg == 6 && h.max_deg == 6) ? 6 : h.max_deg <= 8 ? 8 : 20, dh = dmax / 2;
    P.split_reg = false;
    // Split arithmetic with L in registers: five base rows, rows of 19 or 20 edges
    // (DMAX = 20), 8-bit soft values with E_max > MSG_max (the frozen test
    // relies on a frozen E and its Eq. 8 value sharing a sign), one lane pair per
    // row pair (Z <= 1024), E byte addresses below 2^16. LDS: E plus the dummy
    // block column, the syndrome, the per-lane address table [threads][mb][dh] of
    // 16-bit entries, three vote words, the queue slot and two last-layer test
    // words (32 bytes), then with an offset table its rows per layer, slot and
    // lane half (4 bytes each).
    if ((hint == 0 || hint == LDPC_HINT_SPLIT_REG) && split_ok && h.mb == 5 && dmax == 20 && h.min_deg >= 19 &&
        h.acc_bits == 8 && h.e_max > h.msg_max && h.z <= 1024 && (size_t)h.n + h.z <= 65536) {
        const int threads = (int)std::min<size_t>(1024, 2 * round_up((size_t)h.z / 2, 32));
        const size_t e_sp = round_up((size_t)h.n + h.z, 16);
        const size_t tab = round_up((size_t)h.mb * dh * threads * 2, 16);
        const size_t offs = h.offsets.empty() ? 0 : (size_t)h.offset_iters * h.mb * dh * 2 * 4;
        const size_t total = e_sp + round_up(syn_bytes, 16) + tab + 32 + offs;
        if (total <= (size_t)lds_limit) {
            P.split_reg = true;
            P.split_dmax = dmax;
            P.split_global_l = false;
            P.layer_sync = false;
            P.lds_state = true;
            P.lds_bytes = total;
            P.threads = threads;
            c->l_stride = 0;
            c->lds_l_off = 0;
            c->lds_syn_off = (int)e_sp;
            c->lds_tab_off = (int)(e_sp + round_up(syn_bytes, 16));
            c->lds_flag_off = (int)(c->lds_tab_off + tab);
            c->ws_l_off = 0;
            c->ws_frame_bytes = 0;
            c->lane_tab_bytes = (size_t)h.mb * dh * 2 * 16;
            return true;
        }
    }
    if (hint == LDPC_HINT_SPLIT_REG)
        return false;
    if ((hint == 0 || split_hint) && split_ok) {
        const size_t e_sp = round_up(((size_t)h.n + h.z) * esize, 16);
        const size_t stride = (((size_t)h.mb * dh) | 1) * 4;
        const size_t l_sp = round_up((size_t)(h.z / 2) * stride, 16);
        const size_t tab = (size_t)h.mb * dh * 2 * 16;
        const size_t total_sp = e_sp + l_sp + round_up(syn_bytes, 16) + tab + 16;
        const size_t total_gl = e_sp + round_up(syn_bytes, 16) + tab + 16;
        const bool lds_l = hint != LDPC_HINT_SPLIT_GLOBAL_L && total_sp <= (size_t)lds_limit;
        const bool glob_l = !lds_l && hint != LDPC_HINT_SPLIT && total_gl <= (size_t)lds_limit;
        if (lds_l || glob_l) {
            const size_t l_len = lds_l ? l_sp : 0;
            P.split_dmax = dmax;
            P.split_global_l = glob_l;
            P.lds_state = lds_l;
            P.lds_bytes = lds_l ? total_sp : total_gl;
            P.threads = (int)std::min<size_t>(1024, 2 * round_up((size_t)h.z / 2, 32));
            c->l_stride = (int)stride;
            c->lds_l_off = (int)e_sp;
            c->lds_syn_off = (int)(e_sp + l_len);
            c->lds_tab_off = (int)(e_sp + l_len + round_up(syn_bytes, 16));
            c->lds_flag_off = (int)(c->lds_tab_off + tab);
            c->ws_l_off = 0;
            // L of all layers: a chunk of 4 dh bytes per row pair and layer
            c->ws_frame_bytes = glob_l ? round_up((size_t)h.mb * (h.z / 2) * 4 * dh, 256) : 0;
            c->lane_tab_bytes = tab;
            return true;
        }
    }
    if (split_hint)
        return false;
    // Layer-synchronous (frames whose E does not fit in LDS beside the split
    // kernel's tables): a global slice per frame holds E (plus the dummy block
    // column) and L in the global-L chunk layout; the frame flags follow the
    // slices in the workspace.
    if ((hint == 0 || hint == LDPC_HINT_LAYER_SYNC) && split_ok) {
        P.split_dmax = dmax;
        P.layer_sync = true;
        P.lds_state = false;
        P.lds_bytes = 0;
        P.threads = (int)std::min<size_t>(1024, 2 * round_up((size_t)h.z / 2, 32));
        c->ws_l_off = round_up(((size_t)h.n + h.z) * esize, 256);
        c->ws_frame_bytes = c->ws_l_off + round_up((size_t)h.mb * (h.z / 2) * 4 * dh, 256);
        c->lane_tab_bytes = (size_t)h.mb * dh * 2 * 16;
        return true;
    }
    if (hint == LDPC_HINT_LAYER_SYNC)
        return false;
    // Pairs (one lane per row pair): even Z. LDS: E at offset 0, L as
    // [pair][block][half] with an odd-dword stride per pair, the syndrome, two
    // vote words.
    const size_t stride = (((2 * (size_t)h.n_blocks + 3) / 4) | 1) * 4;
    const size_t lp_al = round_up((size_t)(h.z / 2) * stride, 16);
    const size_t total_x2 = e_al + lp_al + round_up(syn_bytes, 16) + 16;
    if ((hint == 0 || hint == LDPC_HINT_PAIRS) && h.z % 2 == 0 && total_x2 <= (size_t)lds_limit) {
        P.pairs = true;
        P.lds_state = true;
        P.lds_bytes = total_x2;
        P.threads = (int)std::min<size_t>(512, round_up((size_t)h.z / 2, 64));
        c->l_stride = (int)stride;
        c->lds_l_off = (int)e_al;
        c->lds_syn_off = (int)(e_al + lp_al);
        c->lds_flag_off = (int)(e_al + lp_al + round_up(syn_bytes, 16));
        c->ws_frame_bytes = 0;
        return true;
    }
    if (hint == LDPC_HINT_PAIRS)
        return false;
    // One lane per row: E at offset 0, L [block][row], the syndrome (LDS), or
    // E and L in a global workspace slice per frame.
    P.threads = (int)std::min<size_t>(1024, round_up((size_t)h.z, 64));
    const size_t l_al = round_up((size_t)h.n_edges, 16);
    const size_t total = e_al + l_al + syn_bytes;
    c->lds_e_off = 0;
    c->lds_l_off = (int)e_al;
    c->lds_syn_off = (int)(e_al + l_al);
    if ((hint == 0 || hint == LDPC_HINT_LDS) && total <= (size_t)lds_limit) {
        P.lds_state = true;
        P.lds_bytes = total;
        c->ws_frame_bytes = 0;
        return true;
    }
    if (hint == LDPC_HINT_LDS)
        return false;
    P.lds_state = false;
    P.lds_bytes = syn_bytes;
    c->lds_syn_off = 0;
    c->ws_l_off = round_up((size_t)h.n * esize, 256);
    c->ws_frame_bytes = c->ws_l_off + round_up((size_t)h.n_edges, 256);
    return true;
}

int check_device(const ldpc_code *code)
{
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess)
        return hip_fail("hipGetDevice", e);
    if (cur != code->device) {
        char buf[160];
        std::snprintf(buf, sizeof(buf), "code was created on device %d but device %d is current", code->device, cur);
        return fail(LDPC_EINVAL, buf);
    }
    return LDPC_OK;
}

constexpr size_t kQueueBytes = 256;

bool is_persistent(const ldpc_schedule *sched) { return sched && sched->persistent_workgroups > 0; }

// Queue slot (persistent) plus one state slice per frame, or per persistent
// workgroup for the split kernel, whose slices belong to workgroups.
// Layer-synchronous family: per-frame flags, then the count of frames not yet retired.
size_t layer_sync_flag_bytes(int32_t n_frames) { return round_up((size_t)n_frames * 16, 256) + 256; }

size_t workspace_need(const ldpc_code *code, int32_t n_frames, const ldpc_schedule *sched)
{
    if (is_persistent(sched))
        return kQueueBytes + code->ws_frame_bytes * (size_t)sched->persistent_workgroups;
    if (code->plan.layer_sync)
        return code->ws_frame_bytes * (size_t)n_frames + layer_sync_flag_bytes(n_frames);
    return code->ws_frame_bytes * (size_t)n_frames;
}

int check_decode_args(const ldpc_code *code, const uint8_t *syndromes, const int8_t *llr_in, int32_t n_frames,
                      int32_t max_iter, uint8_t *out_bits, uint8_t *out_converged, const ldpc_schedule *sched)
{
    if (!code)
        return fail(LDPC_EINVAL, "ldpc_decode_batch: code is NULL");
    if (n_frames < 0)
        return fail(LDPC_EINVAL, "ldpc_decode_batch: n_frames < 0");
    if (max_iter < 0)
        return fail(LDPC_EINVAL, "ldpc_decode_batch: max_iter < 0");
    if (n_frames > 0 && (!syndromes || !llr_in || !out_bits || !out_converged))
        return fail(LDPC_EINVAL, "ldpc_decode_batch: syndromes, llr_in, out_bits and out_converged must be non-NULL");
    // the layer-synchronous launches put the frame index in the second grid dimension
    if (code->plan.layer_sync && n_frames > 65535)
        return fail(LDPC_EINVAL, "ldpc_decode_batch: the layer-synchronous family takes at most 65535 frames per call");
    if (sched) {
        if (sched->persistent_workgroups < 0)
            return fail(LDPC_EINVAL, "ldpc_schedule: persistent_workgroups < 0");
        if (sched->order && sched->persistent_workgroups == 0)
            return fail(LDPC_EINVAL, "ldpc_schedule: order needs persistent_workgroups > 0");
        if (sched->persistent_workgroups > 0 && (!code->plan.split_dmax || code->plan.layer_sync))
            return fail(LDPC_EUNSUPPORTED, "ldpc_schedule: persistent workgroups need the split kernel family");
        if (sched->check_every < 0)
            return fail(LDPC_EINVAL, "ldpc_schedule: check_every < 0");
        const int fpw = sched->frames_per_workgroup;
        if (fpw < 0)
            return fail(LDPC_EINVAL, "ldpc_schedule: frames_per_workgroup < 0");
        if (fpw > 0) {
            const int z = code->h.z;
            if (!code->plan.split_reg || z > 64)
                return fail(LDPC_EUNSUPPORTED,
                            "ldpc_schedule: frames_per_workgroup needs the split_reg family with z <= 64");
            const int fw = 64 / z;
            if (fpw % fw != 0 || fpw / fw > 16)
                return fail(LDPC_EINVAL, "ldpc_schedule: frames_per_workgroup must be a multiple of 64 / z, "
                                         "at most 16 waves");
            if (sched->persistent_workgroups > 0)
                return fail(LDPC_EINVAL, "ldpc_schedule: frames_per_workgroup and persistent workgroups exclude "
                                         "each other");
            const size_t esz = ((size_t)code->h.n + z + 15) & ~(size_t)15;
            if ((size_t)fpw * esz > 65536)
                return fail(LDPC_EINVAL, "ldpc_schedule: frames_per_workgroup frames' soft values exceed 64 KB");
            const size_t lds = qkdldpc::wave_reg_lds_bytes(code->h.n, z, (code->h.m + 7) / 8, fpw,
                                                           code->h.offsets.empty() ? 0 : code->h.offset_iters);
            if (lds > (size_t)code->lds_limit)
                return fail(LDPC_EINVAL, "ldpc_schedule: frames_per_workgroup needs more LDS than a workgroup has");
        }
    }
    return LDPC_OK;
}

DecodeArgs make_args(const ldpc_code *code, const uint8_t *syndromes, const int8_t *llr_in, int32_t n_frames,
                     int32_t max_iter, uint8_t *out_bits, uint8_t *out_converged, int32_t *out_iters, int8_t *out_L,
                     int16_t *out_E, const ldpc_schedule *sched, void *ws)
{
    DecodeArgs A{};
    uint8_t *w = static_cast<uint8_t *>(ws);
    A.syn = syndromes;
    A.llr = llr_in;
    A.n_frames = n_frames;
    A.max_iter = max_iter;
    A.out_bits = out_bits;
    A.out_conv = out_converged;
    A.out_iters = out_iters;
    A.out_L = out_L;
    A.out_E = out_E;
    A.frames_per_wg = sched ? sched->frames_per_workgroup : 0;
    if (is_persistent(sched)) {
        A.persistent_wgs = sched->persistent_workgroups;
        A.queue = reinterpret_cast<int *>(w);
        A.order = sched->order;
        w += kQueueBytes;
    }
    A.ws = code->ws_frame_bytes ? w : nullptr;
    if (code->plan.layer_sync) {
        A.mflags = reinterpret_cast<int *>(w + code->ws_frame_bytes * (size_t)n_frames);
        A.mcount = reinterpret_cast<int *>(reinterpret_cast<uint8_t *>(A.mflags) +
                                           round_up((size_t)n_frames * 16, 256));
    }
    A.ws_frame_bytes = code->ws_frame_bytes;
    A.ws_l_off = code->ws_l_off;
    A.syn_bytes = (code->h.m + 7) / 8;
    A.bit_bytes = (code->h.n + 7) / 8;
    A.lds_e_off = code->lds_e_off;
    A.lds_l_off = code->lds_l_off;
    A.lds_syn_off = code->lds_syn_off;
    A.lds_flag_off = code->lds_flag_off;
    A.l_stride = code->l_stride;
    A.lds_tab_off = code->lds_tab_off;
    A.lane_tab = static_cast<const int4 *>(code->d_split);
    A.blk2slot = code->d_split ? reinterpret_cast<const int32_t *>(static_cast<const uint8_t *>(code->d_split) +
                                                                    code->lane_tab_bytes)
                               : nullptr;
    return A;
}

bool early_stop(const ldpc_code *code, const ldpc_schedule *sched)
{
    return code->plan.layer_sync && sched && sched->check_every > 0;
}

// Frames of a layer-synchronous decode not yet retired, read after the stream
// has drained (host is pinned memory or, with nullptr, a stack variable).
hipError_t active_frames(const DecodeArgs &A, int *host, hipStream_t s, int *out)
{
    int local = 0;
    int *dst = host ? host : &local;
    hipError_t e = hipMemcpyAsync(dst, A.mcount, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    *out = *dst;
    return e;
}

// Layer-synchronous decode that stops launching once every frame has retired:
// the active count is read after the iteration-0 check and after every k
// iterations.
hipError_t decode_early_stop(const ldpc_code *code, const DecodeArgs &A, int k, hipStream_t s)
{
    const LaunchPlan &P = code->plan;
    hipError_t e = qkdldpc::launch_multi_head(P, code->dev, A, s);
    int active = 0;
    if (e == hipSuccess)
        e = active_frames(A, nullptr, s, &active);
    for (int t = 1; e == hipSuccess && active > 0 && t <= A.max_iter; t += k) {
        const int t1 = std::min(A.max_iter, t + k - 1);
        e = qkdldpc::launch_multi_iters(P, code->dev, A, t, t1, s);
        if (e == hipSuccess)
            e = active_frames(A, nullptr, s, &active);
    }
    if (e == hipSuccess)
        e = qkdldpc::launch_multi_tail(P, code->dev, A, s);
    return e;
}

int decode_impl(const ldpc_code *code, const uint8_t *syndromes, const int8_t *llr_in, int32_t n_frames,
                int32_t max_iter, uint8_t *out_bits, uint8_t *out_converged, int32_t *out_iters, int8_t *out_L,
                int16_t *out_E, const ldpc_schedule *sched, void *workspace, size_t workspace_bytes, void *stream)
{
    int rc = check_decode_args(code, syndromes, llr_in, n_frames, max_iter, out_bits, out_converged, sched);
    if (rc != LDPC_OK || n_frames == 0)
        return rc;
    rc = check_device(code);
    if (rc != LDPC_OK)
        return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const size_t need = workspace_need(code, n_frames, sched);
    void *ws = workspace;
    bool owned = false;
    if (need > 0) {
        if (ws && workspace_bytes < need)
            return fail(LDPC_EINVAL, "ldpc_decode_batch: workspace smaller than the workspace size query");
        if (!ws) {
            hipError_t e = hipMallocAsync(&ws, need, s);
            if (e != hipSuccess)
                return hip_fail("ldpc_decode_batch: hipMallocAsync workspace", e);
            owned = true;
        }
    }
    const DecodeArgs A = make_args(code, syndromes, llr_in, n_frames, max_iter, out_bits, out_converged, out_iters,
                                   out_L, out_E, sched, ws);
    hipError_t e = early_stop(code, sched) ? decode_early_stop(code, A, sched->check_every, s)
                                           : qkdldpc::launch_decode(code->plan, code->dev, A, s);
    if (owned) {
        hipError_t e2 = hipFreeAsync(ws, s);
        if (e == hipSuccess)
            e = e2;
    }
    if (e != hipSuccess)
        return hip_fail("ldpc_decode_batch: kernel launch", e);
    return LDPC_OK;
}

// Differentiable offset min-sum: register slots, workgroup size (four lanes per
// row, up to 1024 threads) and whether the FP32 state (E and L, or their
// adjoints) fits in LDS beside the offset table, the reduction scratch and the
// syndrome. fits is false when even the offset table does not fit.
qkdldpc::OmsPlan oms_plan(const ldpc_code *c, int32_t n_iter, bool *fits = nullptr)
{
    const HostCode &h = c->h;
    qkdldpc::OmsPlan P{};
    P.dmax = h.max_deg <= 8 ? 8 : h.max_deg <= 20 ? 20 : 32;
    P.threads = (int)std::min<size_t>(1024, round_up(4 * (size_t)h.z, 64));
    const size_t ne = (size_t)h.n_blocks * h.z;
    // reduction scratch, offsets, the block table {column start, shift} with its
    // alignment, the syndrome, the target bits
    const size_t fixed = (size_t)16 * P.dmax * sizeof(float) + (size_t)std::max(n_iter, 0) * h.n_blocks * sizeof(float) +
                         (size_t)h.n_blocks * 8 + 16 + round_up((size_t)(h.m + 7) / 8, 16) +
                         round_up((size_t)(h.n + 7) / 8, 16);
    // state: backward the adjoints of E and L, forward E and a four-word record
    // per check row; each array padded to a multiple of four floats
    const size_t n4 = round_up((size_t)h.n, 4);
    const size_t st = (n4 + round_up(ne, 4)) * sizeof(float);
    const size_t st_f = (n4 + (size_t)4 * h.m) * sizeof(float);
    const size_t limit = (size_t)(c->lds_limit - 1024);
    P.lds_state = st + fixed <= limit;
    P.lds_bytes = (P.lds_state ? st : 0) + fixed;
    P.fwd_lds_state = st_f + fixed <= limit;
    P.fwd_lds_bytes = (P.fwd_lds_state ? st_f : 0) + fixed;
    if (fits)
        *fits = fixed <= limit;
    return P;
}

size_t oms_tape_floats(const HostCode &h, int32_t n_iter)
{
    // per iteration: a four-word record per check row, then E
    return (size_t)n_iter * ((size_t)4 * h.m + (((size_t)h.n + 3) & ~(size_t)3));
}

// Global slices (per frame) for whichever pass's state does not fit in LDS; the
// two passes never run at once, so they share the slices.
size_t oms_state_bytes(const ldpc_code *c, const qkdldpc::OmsPlan &P, int32_t n_frames)
{
    const size_t n4 = round_up((size_t)c->h.n, 4);
    const size_t bwd = P.lds_state ? 0 : n4 + round_up((size_t)c->h.n_blocks * c->h.z, 4);
    const size_t fwd = P.fwd_lds_state ? 0 : n4 + (size_t)4 * c->h.m;
    const size_t per = std::max(bwd, fwd);
    return per ? round_up(per * sizeof(float) * n_frames, 256) : 0;
}

int oms_check(const ldpc_code *code, const char *who, const uint8_t *syndromes, int32_t n_frames, int32_t n_iter,
              const float *beta, const void *tape, size_t tape_bytes)
{
    const std::string w(who);
    if (!code)
        return fail(LDPC_EINVAL, w + ": code is NULL");
    if (n_frames < 0)
        return fail(LDPC_EINVAL, w + ": n_frames < 0");
    if (n_iter < 1)
        return fail(LDPC_EINVAL, w + ": n_iter < 1");
    if (!beta)
        return fail(LDPC_EINVAL, w + ": beta is NULL");
    if (n_frames > 0 && (!syndromes || !tape))
        return fail(LDPC_EINVAL, w + ": syndromes and tape must be non-NULL");
    if (tape_bytes < oms_tape_floats(code->h, n_iter) * sizeof(float) * (size_t)n_frames)
        return fail(LDPC_EINVAL, w + ": tape smaller than ldpc_oms_tape_bytes");
    if (n_frames > 0 && reinterpret_cast<uintptr_t>(tape) % 16 != 0)
        return fail(LDPC_EINVAL, w + ": tape must be 16-byte aligned");
    bool fits = false;
    (void)oms_plan(code, n_iter, &fits);
    if (!fits)
        return fail(LDPC_EUNSUPPORTED, w + ": the offset table (n_iter x n_blocks floats) does not fit in LDS");
    return check_device(code);
}

qkdldpc::OmsArgs oms_args(const ldpc_code *code, const uint8_t *syndromes, const uint8_t *target_bits,
                          int32_t n_frames, int32_t n_iter, const float *beta, const float *loss_weights, void *tape,
                          void *workspace, const qkdldpc::OmsPlan &P)
{
    qkdldpc::OmsArgs A{};
    A.syn = syndromes;
    A.xbits = target_bits;
    A.beta = beta;
    A.weights = loss_weights;
    A.n_frames = n_frames;
    A.n_iter = n_iter;
    A.syn_bytes = (code->h.m + 7) / 8;
    A.bit_bytes = (code->h.n + 7) / 8;
    A.tape = static_cast<float *>(tape);
    A.state = P.lds_state && P.fwd_lds_state ? nullptr : static_cast<float *>(workspace);
    return A;
}

} // namespace

struct ldpc_batch {
    // one graph for the whole decode, or (early stop) stage-in, blocks of
    // iterations and stage-out
    std::vector<hipGraph_t> graphs;
    std::vector<hipGraphExec_t> execs;
    bool early_stop = false;
    DecodeArgs args{};
    int *host_count = nullptr;  // pinned: frames not yet retired (early stop)
    void *owned_ws = nullptr;
    int device = -1;
};

extern "C" {

int ldpc_code_create(const int32_t *base, int32_t mb, int32_t nb, int32_t z, const ldpc_params *params,
                     ldpc_code **out)
{
    if (!out)
        return fail(LDPC_EINVAL, "ldpc_code_create: out is NULL");
    *out = nullptr;
    HostCode h;
    std::string err;
    int rc = qkdldpc::build_host_code(base, mb, nb, z, params, h, err);
    if (rc != LDPC_OK)
        return fail(rc, err);
    if (h.n_edges >= (int64_t(1) << 31))
        return fail(LDPC_EINVAL, "ldpc_code_create: n_blocks * z must be below 2^31");

    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail("ldpc_code_create: no usable GPU (hipGetDevice)", e);
    int lds_limit = 0;
    e = hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess)
        return hip_fail("ldpc_code_create: hipDeviceGetAttribute", e);

    ldpc_code *c = new (std::nothrow) ldpc_code;
    if (!c)
        return fail(LDPC_ENOMEM, "ldpc_code_create: out of host memory");
    c->h = std::move(h);
    c->device = dev;
    c->lds_limit = lds_limit;
    const HostCode &hc = c->h;
    const size_t nt = 2 * (size_t)hc.mb + 3 * (size_t)hc.n_blocks;
    e = hipMalloc(&c->d_tables, nt * sizeof(int32_t));
    if (e != hipSuccess) {
        delete c;
        return hip_fail("ldpc_code_create: hipMalloc", e);
    }
    std::vector<int32_t> tab;
    tab.reserve(nt);
    tab.insert(tab.end(), hc.deg.begin(), hc.deg.end());
    tab.insert(tab.end(), hc.blk_off.begin(), hc.blk_off.end());
    tab.insert(tab.end(), hc.colbase.begin(), hc.colbase.end());
    tab.insert(tab.end(), hc.shift.begin(), hc.shift.end());
    for (int i = 0; i < hc.n_blocks; ++i)
        tab.push_back(hc.colbase[i] | hc.shift[i]);
    e = hipMemcpy(c->d_tables, tab.data(), nt * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && !hc.offsets.empty()) {
        std::vector<int32_t> off32(hc.offsets.begin(), hc.offsets.end());
        e = hipMalloc(&c->d_offsets, off32.size() * sizeof(int32_t));
        if (e == hipSuccess)
            e = hipMemcpy(c->d_offsets, off32.data(), off32.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        ldpc_code_destroy(c);
        return hip_fail("ldpc_code_create: uploading tables", e);
    }
    DevCode &d = c->dev;
    d.deg = c->d_tables;
    d.blk_off = c->d_tables + hc.mb;
    d.colbase = c->d_tables + 2 * hc.mb;
    d.shift = c->d_tables + 2 * hc.mb + hc.n_blocks;
    d.colshift = c->d_tables + 2 * hc.mb + 2 * hc.n_blocks;
    d.offsets = c->d_offsets;
    d.offset_iters = hc.offset_iters;
    d.mb = hc.mb;
    d.nb = hc.nb;
    d.z = hc.z;
    d.n = hc.n;
    d.m = hc.m;
    d.n_blocks = hc.n_blocks;
    d.msg_max = hc.msg_max;
    d.e_max = hc.e_max;
    // leave room for the few bytes of static LDS the barrier reductions use
    if (!make_plan(c, lds_limit - 1024, hc.kernel_hint)) {
        ldpc_code_destroy(c);
        return fail(LDPC_EUNSUPPORTED, "ldpc_code_create: the requested kernel family does not apply to this code");
    }
    if (c->plan.split_dmax) {
        const std::vector<int32_t> st = split_tables(hc, c->plan.split_dmax);
        e = hipMalloc(&c->d_split, st.size() * sizeof(int32_t));
        if (e == hipSuccess)
            e = hipMemcpy(c->d_split, st.data(), st.size() * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            ldpc_code_destroy(c);
            return hip_fail("ldpc_code_create: uploading lane tables", e);
        }
    }
    *out = c;
    return LDPC_OK;
}

void ldpc_code_destroy(ldpc_code *code)
{
    if (!code)
        return;
    if (code->d_tables)
        (void)hipFree(code->d_tables);
    if (code->d_offsets)
        (void)hipFree(code->d_offsets);
    if (code->d_split)
        (void)hipFree(code->d_split);
    delete code;
}

int ldpc_code_dims(const ldpc_code *code, int32_t *n, int32_t *m, int64_t *n_edges, int32_t *n_blocks,
                   int32_t *has_4cycles)
{
    if (!code)
        return fail(LDPC_EINVAL, "ldpc_code_dims: code is NULL");
    if (n)
        *n = code->h.n;
    if (m)
        *m = code->h.m;
    if (n_edges)
        *n_edges = code->h.n_edges;
    if (n_blocks)
        *n_blocks = code->h.n_blocks;
    if (has_4cycles)
        *has_4cycles = code->h.has_4cycles;
    return LDPC_OK;
}

int ldpc_code_plan(const ldpc_code *code, int32_t *kernel, int32_t *threads, int32_t *lds_bytes)
{
    if (!code)
        return fail(LDPC_EINVAL, "ldpc_code_plan: code is NULL");
    const LaunchPlan &P = code->plan;
    if (kernel)
        *kernel = P.layer_sync  ? LDPC_KERNEL_LAYER_SYNC
                  : P.split_reg  ? LDPC_KERNEL_SPLIT_REG
                  : P.split_dmax ? (P.split_global_l ? LDPC_KERNEL_SPLIT_GLOBAL_L : LDPC_KERNEL_SPLIT)
                  : P.pairs    ? LDPC_KERNEL_PAIRS
                  : P.lds_state ? LDPC_KERNEL_LDS
                                : LDPC_KERNEL_GLOBAL;
    if (threads)
        *threads = P.threads;
    if (lds_bytes)
        *lds_bytes = (int32_t)P.lds_bytes;
    return LDPC_OK;
}

size_t ldpc_workspace_bytes(const ldpc_code *code, int32_t n_frames)
{
    if (!code || n_frames < 0)
        return 0;
    return workspace_need(code, n_frames, nullptr);
}

int ldpc_decode_batch_ex(const ldpc_code *code, const uint8_t *syndromes, const int8_t *llr_in, int32_t n_frames,
                         int32_t max_iter, uint8_t *out_bits, uint8_t *out_converged, int32_t *out_iters,
                         int8_t *out_L, int16_t *out_E, void *workspace, size_t workspace_bytes, void *stream)
{
    return decode_impl(code, syndromes, llr_in, n_frames, max_iter, out_bits, out_converged, out_iters, out_L, out_E,
                       nullptr, workspace, workspace_bytes, stream);
}

int ldpc_decode_batch_sched(const ldpc_code *code, const uint8_t *syndromes, const int8_t *llr_in, int32_t n_frames,
                            int32_t max_iter, uint8_t *out_bits, uint8_t *out_converged, int32_t *out_iters,
                            const ldpc_schedule *sched, void *workspace, size_t workspace_bytes, void *stream)
{
    return decode_impl(code, syndromes, llr_in, n_frames, max_iter, out_bits, out_converged, out_iters, nullptr,
                       nullptr, sched, workspace, workspace_bytes, stream);
}

size_t ldpc_workspace_bytes_sched(const ldpc_code *code, int32_t n_frames, const ldpc_schedule *sched)
{
    if (!code || n_frames < 0)
        return 0;
    return workspace_need(code, n_frames, sched);
}

int ldpc_decode_batch(const ldpc_code *code, const uint8_t *syndromes, const int8_t *llr_in, int32_t n_frames,
                      int32_t max_iter, uint8_t *out_bits, uint8_t *out_converged, void *stream)
{
    return ldpc_decode_batch_ex(code, syndromes, llr_in, n_frames, max_iter, out_bits, out_converged, nullptr,
                                nullptr, nullptr, nullptr, 0, stream);
}

int ldpc_batch_create(const ldpc_code *code, const uint8_t *syndromes, const int8_t *llr_in, int32_t n_frames,
                      int32_t max_iter, uint8_t *out_bits, uint8_t *out_converged, int32_t *out_iters,
                      const ldpc_schedule *sched, void *workspace, size_t workspace_bytes, ldpc_batch **out)
{
    if (!out)
        return fail(LDPC_EINVAL, "ldpc_batch_create: out is NULL");
    *out = nullptr;
    int rc = check_decode_args(code, syndromes, llr_in, n_frames, max_iter, out_bits, out_converged, sched);
    if (rc != LDPC_OK)
        return rc;
    if (n_frames == 0)
        return fail(LDPC_EINVAL, "ldpc_batch_create: n_frames must be positive");
    rc = check_device(code);
    if (rc != LDPC_OK)
        return rc;
    ldpc_batch *b = new (std::nothrow) ldpc_batch;
    if (!b)
        return fail(LDPC_ENOMEM, "ldpc_batch_create: out of host memory");
    b->device = code->device;
    const size_t need = workspace_need(code, n_frames, sched);
    void *ws = workspace;
    hipError_t e = hipSuccess;
    if (need > 0) {
        if (ws && workspace_bytes < need) {
            delete b;
            return fail(LDPC_EINVAL, "ldpc_batch_create: workspace smaller than the workspace size query");
        }
        if (!ws) {
            e = hipMalloc(&b->owned_ws, need);
            if (e != hipSuccess) {
                delete b;
                return hip_fail("ldpc_batch_create: hipMalloc workspace", e);
            }
            ws = b->owned_ws;
        }
    }
    const DecodeArgs A = make_args(code, syndromes, llr_in, n_frames, max_iter, out_bits, out_converged, out_iters,
                                   nullptr, nullptr, sched, ws);
    b->args = A;
    b->early_stop = early_stop(code, sched);
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    // capture one launch sequence into the next graph of the batch
    auto capture = [&](auto &&enqueue) {
        hipGraph_t g = nullptr;
        hipError_t ee = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (ee != hipSuccess)
            return ee;
        hipError_t el = enqueue();
        hipError_t ec = hipStreamEndCapture(cs, &g);
        if (g)
            b->graphs.push_back(g);
        ee = el != hipSuccess ? el : ec;
        hipGraphExec_t x = nullptr;
        if (ee == hipSuccess)
            ee = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (x)
            b->execs.push_back(x);
        return ee;
    };
    const LaunchPlan &P = code->plan;
    if (e == hipSuccess && !b->early_stop) {
        e = capture([&] { return qkdldpc::launch_decode(P, code->dev, A, cs); });
    } else if (e == hipSuccess) {
        const int k = sched->check_every;
        e = hipHostMalloc(reinterpret_cast<void **>(&b->host_count), sizeof(int), hipHostMallocDefault);
        if (e == hipSuccess)
            e = capture([&] { return qkdldpc::launch_multi_head(P, code->dev, A, cs); });
        for (int t = 1; e == hipSuccess && t <= max_iter; t += k) {
            const int t1 = std::min(max_iter, t + k - 1);
            e = capture([&] { return qkdldpc::launch_multi_iters(P, code->dev, A, t, t1, cs); });
        }
        if (e == hipSuccess)
            e = capture([&] { return qkdldpc::launch_multi_tail(P, code->dev, A, cs); });
    }
    if (cs)
        (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        ldpc_batch_destroy(b);
        return hip_fail("ldpc_batch_create: graph capture", e);
    }
    *out = b;
    return LDPC_OK;
}

int ldpc_batch_launch(ldpc_batch *batch, void *stream)
{
    if (!batch)
        return fail(LDPC_EINVAL, "ldpc_batch_launch: batch is NULL");
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess)
        return hip_fail("hipGetDevice", e);
    if (cur != batch->device)
        return fail(LDPC_EINVAL, "ldpc_batch_launch: batch was created on another device");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (!batch->early_stop) {
        e = hipGraphLaunch(batch->execs[0], s);
        if (e != hipSuccess)
            return hip_fail("ldpc_batch_launch: hipGraphLaunch", e);
        return LDPC_OK;
    }
    // stage-in, then blocks of iterations while frames remain, then stage-out
    const size_t nx = batch->execs.size();
    int active = 0;
    e = hipGraphLaunch(batch->execs[0], s);
    if (e == hipSuccess)
        e = active_frames(batch->args, batch->host_count, s, &active);
    for (size_t i = 1; e == hipSuccess && active > 0 && i + 1 < nx; ++i) {
        e = hipGraphLaunch(batch->execs[i], s);
        if (e == hipSuccess)
            e = active_frames(batch->args, batch->host_count, s, &active);
    }
    if (e == hipSuccess)
        e = hipGraphLaunch(batch->execs[nx - 1], s);
    if (e != hipSuccess)
        return hip_fail("ldpc_batch_launch: hipGraphLaunch", e);
    return LDPC_OK;
}

void ldpc_batch_destroy(ldpc_batch *batch)
{
    if (!batch)
        return;
    for (hipGraphExec_t x : batch->execs)
        (void)hipGraphExecDestroy(x);
    for (hipGraph_t g : batch->graphs)
        (void)hipGraphDestroy(g);
    if (batch->host_count)
        (void)hipHostFree(batch->host_count);
    if (batch->owned_ws)
        (void)hipFree(batch->owned_ws);
    delete batch;
}

int ldpc_order_by_unsat(const ldpc_code *code, const uint8_t *syndromes, const int8_t *llr_in, int32_t n_frames,
                        int32_t *out_unsat, int32_t *out_order, void *stream)
{
    if (!code)
        return fail(LDPC_EINVAL, "ldpc_order_by_unsat: code is NULL");
    if (n_frames < 0)
        return fail(LDPC_EINVAL, "ldpc_order_by_unsat: n_frames < 0");
    if (n_frames == 0)
        return LDPC_OK;
    if (!syndromes || !llr_in || !out_unsat)
        return fail(LDPC_EINVAL, "ldpc_order_by_unsat: syndromes, llr_in and out_unsat must be non-NULL");
    int rc = check_device(code);
    if (rc != LDPC_OK)
        return rc;
    hipError_t e = qkdldpc::launch_order_by_unsat(code->dev, syndromes, llr_in, n_frames, out_unsat, out_order,
                                                  reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return hip_fail("ldpc_order_by_unsat: kernel launch", e);
    return LDPC_OK;
}

int ldpc_syndrome_batch(const ldpc_code *code, const uint8_t *bits, int32_t n_frames, uint8_t *out_syn,
                        void *stream)
{
    if (!code)
        return fail(LDPC_EINVAL, "ldpc_syndrome_batch: code is NULL");
    if (n_frames < 0)
        return fail(LDPC_EINVAL, "ldpc_syndrome_batch: n_frames < 0");
    if (n_frames == 0)
        return LDPC_OK;
    if (!bits || !out_syn)
        return fail(LDPC_EINVAL, "ldpc_syndrome_batch: bits and out_syn must be non-NULL");
    int rc = check_device(code);
    if (rc != LDPC_OK)
        return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const size_t bb = (code->h.n + 7) / 8, sb = (code->h.m + 7) / 8;
    for (int32_t f0 = 0; f0 < n_frames; f0 += 65535) {
        const int nf = std::min<int32_t>(65535, n_frames - f0);
        hipError_t e = qkdldpc::launch_syndrome(code->dev, bits + (size_t)f0 * bb, nf, out_syn + (size_t)f0 * sb, s);
        if (e != hipSuccess)
            return hip_fail("ldpc_syndrome_batch: kernel launch", e);
    }
    return LDPC_OK;
}

int ldpc_reveal_batch(const ldpc_code *code, int8_t *llr, int32_t n_frames, const int32_t *frame_ids, int32_t k,
                      const int32_t *positions, const uint8_t *values, int32_t r, void *stream)
{
    if (!code)
        return fail(LDPC_EINVAL, "ldpc_reveal_batch: code is NULL");
    if (n_frames < 0 || k < 0 || r < 0)
        return fail(LDPC_EINVAL, "ldpc_reveal_batch: n_frames, k and r must be >= 0");
    if ((long long)k * r >= (1LL << 31))
        return fail(LDPC_EINVAL, "ldpc_reveal_batch: k * r must be below 2^31");
    if ((long long)k * r == 0)
        return LDPC_OK;
    if (!llr || !frame_ids || !positions || !values)
        return fail(LDPC_EINVAL, "ldpc_reveal_batch: llr, frame_ids, positions and values must be non-NULL");
    int rc = check_device(code);
    if (rc != LDPC_OK)
        return rc;
    hipError_t e = qkdldpc::launch_reveal(llr, code->h.n, n_frames, frame_ids, k, positions, values, r,
                                          reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return hip_fail("ldpc_reveal_batch: kernel launch", e);
    return LDPC_OK;
}

size_t ldpc_oms_tape_bytes(const ldpc_code *code, int32_t n_frames, int32_t n_iter)
{
    if (!code || n_frames < 0 || n_iter < 0)
        return 0;
    return oms_tape_floats(code->h, n_iter) * sizeof(float) * (size_t)n_frames;
}

size_t ldpc_oms_workspace_bytes(const ldpc_code *code, int32_t n_frames, int32_t n_iter)
{
    if (!code || n_frames < 0 || n_iter < 0)
        return 0;
    const qkdldpc::OmsPlan P = oms_plan(code, n_iter);
    return oms_state_bytes(code, P, n_frames) + (size_t)n_frames * n_iter * code->h.n_blocks * sizeof(float);
}

int ldpc_oms_forward(const ldpc_code *code, const uint8_t *syndromes, const float *llr, const uint8_t *target_bits,
                     int32_t n_frames, int32_t n_iter, const float *beta, const float *loss_weights, float *out_loss,
                     float *out_E, void *tape, size_t tape_bytes, void *workspace, size_t workspace_bytes,
                     void *stream)
{
    int rc = oms_check(code, "ldpc_oms_forward", syndromes, n_frames, n_iter, beta, tape, tape_bytes);
    if (rc != LDPC_OK || n_frames == 0)
        return rc;
    if (!llr)
        return fail(LDPC_EINVAL, "ldpc_oms_forward: llr is NULL");
    if (out_loss && !target_bits)
        return fail(LDPC_EINVAL, "ldpc_oms_forward: out_loss needs target_bits");
    const qkdldpc::OmsPlan P = oms_plan(code, n_iter);
    // the forward reads the workspace only when its own state does not fit in LDS
    const size_t need = P.fwd_lds_state ? 0 : oms_state_bytes(code, P, n_frames);
    if (need && (!workspace || workspace_bytes < need))
        return fail(LDPC_EINVAL, "ldpc_oms_forward: workspace smaller than ldpc_oms_workspace_bytes");
    qkdldpc::OmsArgs A = oms_args(code, syndromes, target_bits, n_frames, n_iter, beta, loss_weights, tape,
                                  workspace, P);
    A.llr = llr;
    A.out_loss = out_loss;
    A.out_E = out_E;
    hipError_t e = qkdldpc::launch_oms_forward(P, code->dev, A, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return hip_fail("ldpc_oms_forward: kernel launch", e);
    return LDPC_OK;
}

int ldpc_oms_backward(const ldpc_code *code, const uint8_t *syndromes, const uint8_t *target_bits, int32_t n_frames,
                      int32_t n_iter, const float *beta, const float *loss_weights, const float *dloss,
                      const void *tape, size_t tape_bytes, float *out_dbeta, float *out_dllr, void *workspace,
                      size_t workspace_bytes, void *stream)
{
    int rc = oms_check(code, "ldpc_oms_backward", syndromes, n_frames, n_iter, beta, tape, tape_bytes);
    if (rc != LDPC_OK)
        return rc;
    if (!out_dbeta)
        return fail(LDPC_EINVAL, "ldpc_oms_backward: out_dbeta is NULL");
    if (n_frames > 0 && (!target_bits || !dloss))
        return fail(LDPC_EINVAL, "ldpc_oms_backward: target_bits and dloss must be non-NULL");
    const qkdldpc::OmsPlan P = oms_plan(code, n_iter);
    const size_t need = ldpc_oms_workspace_bytes(code, n_frames, n_iter);
    if (need && (!workspace || workspace_bytes < need))
        return fail(LDPC_EINVAL, "ldpc_oms_backward: workspace smaller than ldpc_oms_workspace_bytes");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    qkdldpc::OmsArgs A = oms_args(code, syndromes, target_bits, n_frames, n_iter, beta, loss_weights,
                                  const_cast<void *>(tape), workspace, P);
    A.dloss = dloss;
    A.dbeta_frames = reinterpret_cast<float *>(static_cast<uint8_t *>(workspace) + oms_state_bytes(code, P, n_frames));
    A.dbeta = out_dbeta;
    A.dllr = out_dllr;
    // with no frames only the frame sum runs, writing a zero gradient
    hipError_t e = qkdldpc::launch_oms_backward(P, code->dev, A, s);
    if (e != hipSuccess)
        return hip_fail("ldpc_oms_backward: kernel launch", e);
    return LDPC_OK;
}

int ldpc_probe_lds_bandwidth(int32_t mode, int32_t n_workgroups, int32_t reps, uint32_t *out, void *stream)
{
    if (mode != 0 && mode != 1)
        return fail(LDPC_EINVAL, "ldpc_probe_lds_bandwidth: mode must be 0 or 1");
    if (n_workgroups < 1 || reps < 1 || !out)
        return fail(LDPC_EINVAL, "ldpc_probe_lds_bandwidth: n_workgroups and reps must be >= 1, out non-NULL");
    hipError_t e = qkdldpc::launch_probe_lds(mode, n_workgroups, reps, out, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return hip_fail("ldpc_probe_lds_bandwidth: kernel launch", e);
    return LDPC_OK;
}

const char *ldpc_last_error(void) { return g_err.c_str(); }

int ldpc_version(void) { return 100; }

int ldpc_host_fold_pair(int32_t rule, const int32_t *p_lo, const int32_t *p_hi, int32_t d, int32_t *out_lo,
                        int32_t *out_hi)
{
    using qkdldpc::u16x2;
    constexpr int D = qkdldpc::kMaxRowDegree;
    if (!p_lo || !p_hi || !out_lo || !out_hi)
        return fail(LDPC_EINVAL, "ldpc_host_fold_pair: NULL pointer");
    if (d < 2 || d > D)
        return fail(LDPC_EINVAL, "ldpc_host_fold_pair: d must be in 2..32");
    if (rule < LDPC_RULE_RCBP_FB || rule > LDPC_RULE_MINSUM)
        return fail(LDPC_EINVAL, "ldpc_host_fold_pair: unknown rule");
    u16x2 p[D], m[D];
    for (int k = 0; k < D; ++k) {
        if (k < d) {
            if (p_lo[k] < 0 || p_lo[k] > 127 || p_hi[k] < 0 || p_hi[k] > 127)
                return fail(LDPC_EINVAL, "ldpc_host_fold_pair: magnitudes must be in 0..127");
            p[k] = u16x2{(unsigned short)p_lo[k], (unsigned short)p_hi[k]};
        } else {
            p[k] = u16x2{qkdldpc::kPad, qkdldpc::kPad};
        }
    }
    if (rule == LDPC_RULE_MINSUM)
        qkdldpc::cn_fold_x2<D, qkdldpc::kRuleMinSum>(p, m);
    else if (rule == LDPC_RULE_RCBP_EQ7)
        qkdldpc::cn_fold_x2<D, qkdldpc::kRuleRcbpEq7>(p, m);
    else
        qkdldpc::cn_fold_x2<D, qkdldpc::kRuleRcbpFB>(p, m);
    for (int k = 0; k < d; ++k) {
        out_lo[k] = m[k].x;
        out_hi[k] = m[k].y;
    }
    return LDPC_OK;
}

int ldpc_host_tau_table(int32_t *out)
{
    if (!out)
        return fail(LDPC_EINVAL, "ldpc_host_tau_table: out is NULL");
    for (int p = 0; p < 64; ++p)
        for (int q = 0; q < 64; ++q)
            out[p * 64 + q] = qkdldpc::tau(p, q);
    return LDPC_OK;
}

} // extern "C"
