// Host-side QC code model: validation of the base matrix and parameters, the
// per-layer block tables in the order the decoder visits them (base rows
// ascending, blocks of a row in ascending base column), and the 4-cycle test.
#include "qc_code.hpp"

#include <algorithm>
#include <cstdio>

namespace qkdldpc {

namespace {

std::string fmt(const char *f, long a = 0, long b = 0, long c = 0)
{
    char buf[256];
    std::snprintf(buf, sizeof(buf), f, a, b, c);
    return buf;
}

// Two base rows r1, r2 and two columns c1, c2, all four blocks nonzero, close a
// 4-cycle in the lifted graph iff s[r1,c1] - s[r2,c1] == s[r1,c2] - s[r2,c2] (mod Z).
int detect_4cycles(const int32_t *base, int32_t mb, int32_t nb, int32_t z)
{
    std::vector<int64_t> diffs;
    for (int r1 = 0; r1 < mb; ++r1)
        for (int r2 = r1 + 1; r2 < mb; ++r2) {
            diffs.clear();
            for (int c = 0; c < nb; ++c) {
                const int32_t a = base[r1 * nb + c], b = base[r2 * nb + c];
                if (a >= 0 && b >= 0)
                    diffs.push_back(((int64_t)a - b + z) % z);
            }
            std::sort(diffs.begin(), diffs.end());
            if (std::adjacent_find(diffs.begin(), diffs.end()) != diffs.end())
                return 1;
        }
    return 0;
}

} // namespace

int build_host_code(const int32_t *base, int32_t mb, int32_t nb, int32_t z, const ldpc_params *p,
                    HostCode &out, std::string &err)
{
    if (!base) {
        err = "ldpc_code_create: base is NULL";
        return LDPC_EINVAL;
    }
    if (mb < 1 || nb < 1 || z < 1) {
        err = fmt("ldpc_code_create: need mb >= 1, nb >= 1, z >= 1 (got %ld, %ld, %ld)", mb, nb, z);
        return LDPC_EINVAL;
    }
    if (mb >= nb) {
        err = fmt("ldpc_code_create: need mb < nb for a positive rate (got %ld x %ld)", mb, nb);
        return LDPC_EINVAL;
    }
    if ((int64_t)nb * z >= (int64_t(1) << 31)) {
        err = "ldpc_code_create: nb * z must be below 2^31";
        return LDPC_EINVAL;
    }
    HostCode h;
    h.mb = mb;
    h.nb = nb;
    h.z = z;
    h.n = nb * z;
    h.m = mb * z;
    for (int i = 0; i < mb * nb; ++i)
        if (base[i] < -1 || base[i] >= z) {
            err = fmt("ldpc_code_create: base[%ld][%ld] = %ld is outside [-1, z)", i / nb, i % nb, base[i]);
            return LDPC_EINVAL;
        }
    for (int c = 0; c < nb; ++c) {
        int w = 0;
        for (int b = 0; b < mb; ++b)
            w += base[b * nb + c] >= 0;
        if (w == 0) {
            err = fmt("ldpc_code_create: base column %ld has no nonzero block", c);
            return LDPC_EINVAL;
        }
    }
    h.deg.resize(mb);
    h.blk_off.resize(mb);
    for (int b = 0; b < mb; ++b) {
        h.blk_off[b] = (int32_t)h.colbase.size();
        for (int c = 0; c < nb; ++c) {
            const int32_t s = base[b * nb + c];
            if (s >= 0) {
                h.colbase.push_back(c * z);
                h.shift.push_back(s);
            }
        }
        h.deg[b] = (int32_t)h.colbase.size() - h.blk_off[b];
        if (h.deg[b] < 2) {
            err = fmt("ldpc_code_create: base row %ld has %ld nonzero blocks (need >= 2)", b, h.deg[b]);
            return LDPC_EINVAL;
        }
        if (h.deg[b] > kMaxRowDegree) {
            err = fmt("ldpc_code_create: base row %ld has degree %ld; the kernels support up to %ld", b,
                      h.deg[b], kMaxRowDegree);
            return LDPC_EUNSUPPORTED;
        }
        h.max_deg = std::max(h.max_deg, h.deg[b]);
        h.min_deg = b == 0 ? h.deg[b] : std::min(h.min_deg, h.deg[b]);
    }
    h.n_blocks = (int32_t)h.colbase.size();
    h.n_edges = (int64_t)h.n_blocks * z;
    h.has_4cycles = detect_4cycles(base, mb, nb, z);

    ldpc_params prm{};
    if (p)
        prm = *p;
    h.acc_bits = prm.acc_bits == 0 ? 8 : prm.acc_bits;
    if (h.acc_bits != 8 && h.acc_bits != 16) {
        err = fmt("ldpc_code_create: acc_bits must be 8 or 16 (got %ld)", prm.acc_bits);
        return LDPC_EINVAL;
    }
    h.msg_max = prm.msg_max == 0 ? 63 : prm.msg_max;
    if (h.msg_max < 1 || h.msg_max > 127) {
        err = fmt("ldpc_code_create: msg_max must be in 1..127 (got %ld)", prm.msg_max);
        return LDPC_EINVAL;
    }
    const int lim = h.acc_bits == 16 ? 32767 : 127;
    h.e_max = prm.e_max == 0 ? lim : prm.e_max;
    if (h.e_max < 1 || h.e_max > lim) {
        err = fmt("ldpc_code_create: e_max must be in 1..%ld (got %ld)", lim, prm.e_max);
        return LDPC_EINVAL;
    }
    if (prm.cn_rule < LDPC_RULE_RCBP_FB || prm.cn_rule > LDPC_RULE_MINSUM) {
        err = fmt("ldpc_code_create: unknown cn_rule %ld", prm.cn_rule);
        return LDPC_EINVAL;
    }
    h.cn_rule = prm.cn_rule;
    if (prm.offsets) {
        if (prm.offset_iters < 1) {
            err = "ldpc_code_create: offsets given with offset_iters < 1";
            return LDPC_EINVAL;
        }
        h.offset_iters = prm.offset_iters;
        h.offsets.assign(prm.offsets, prm.offsets + (size_t)prm.offset_iters * h.n_blocks);
    } else if (prm.offset_iters != 0) {
        err = "ldpc_code_create: offset_iters given without offsets";
        return LDPC_EINVAL;
    }
    if (prm.kernel_hint < 0 || prm.kernel_hint > LDPC_HINT_SPLIT_REG) {
        err = fmt("ldpc_code_create: unknown kernel_hint %ld", prm.kernel_hint);
        return LDPC_EINVAL;
    }
    h.kernel_hint = prm.kernel_hint;
    out = std::move(h);
    return LDPC_OK;
}

} // namespace qkdldpc
