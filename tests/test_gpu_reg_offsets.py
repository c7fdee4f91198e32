"""Offset tables on the register-resident family (split_reg): the magnitudes of
the check-node messages lose a per-iteration, per-base-edge offset and are
clamped to [0, MSG_max] (the offset form of the check node, with the offsets the
learned decoder quantizes), on the one-frame-per-workgroup, the persistent and
the several-frames-per-workgroup kernels, for both check-node rules; compared
with the oracle bit for bit."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1903_10107_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1903_10107_amd import binding
    binding.lib()
    return binding


# (z, frames, qber, shortened fraction, offset rows, max_iter): fewer offset
# rows than iterations (the last row repeats), one row, and more rows than
# iterations
CASES = {
    "n1024_rows4": (32, 24, 0.01, 0.0, 4, 40),
    "n8192_rows1": (256, 8, 0.02, 0.25, 1, 30),
    "n32768_rows60": (1024, 4, 0.02, 0.33, 60, 40),
}


@pytest.mark.parametrize("rule", ["rcbp", "minsum"])
@pytest.mark.parametrize("name", list(CASES))
def test_split_reg_offsets_match_oracle(B, name, rule):
    z, F, q, short, rows, T = CASES[name]
    code = I.Code(I.make_base(5, 32, z), z)
    fr = I.make_frames(code, F, q, 55 + z, n_short=int(short * code.n))
    off = np.random.default_rng(z + rows).integers(-1, 3, size=(rows, code.n_blocks)).astype(np.int8)
    cn = B.LDPC_RULE_RCBP_FB if rule == "rcbp" else B.LDPC_RULE_MINSUM
    gc = B.Code(code.base, z, cn_rule=cn, offsets=off)
    assert gc.plan()["kernel"] == "split_reg"
    _say(f"[gpu split_reg offsets] {name} {rule} {gc.plan()}")
    got = B.decode(gc, fr.syn, fr.llr, T, want_state=True)
    ref = O.decode(code.base, z, fr.syn, fr.llr, T, want_state=True,
                   cn_rule=O.RULE_RCBP_FB if rule == "rcbp" else O.RULE_MINSUM, offsets=off)
    for k in ("bits", "conv", "iters", "L", "E"):
        assert np.array_equal(got[k], ref[k]), (name, rule, k)


@pytest.mark.parametrize("rule", ["rcbp", "minsum"])
@pytest.mark.parametrize("fpw", [2, 8])
def test_frames_per_workgroup_with_offsets_matches_oracle(B, fpw, rule):
    """The several-frames-per-workgroup kernel (Z = 32: two frames per wave) with
    an offset table: the staged offsets are shared by the workgroup's frames."""
    import torch
    z, F, T = 32, 20, 40
    code = I.Code(I.make_base(5, 32, z), z)
    fr = I.make_frames(code, F, 0.01, 91 + fpw, n_short=0)
    off = np.random.default_rng(fpw).integers(-1, 3, size=(3, code.n_blocks)).astype(np.int8)
    cn = B.LDPC_RULE_RCBP_FB if rule == "rcbp" else B.LDPC_RULE_MINSUM
    gc = B.Code(code.base, z, cn_rule=cn, offsets=off)
    assert gc.plan()["kernel"] == "split_reg"
    _say(f"[gpu split_reg offsets] fpw={fpw} {rule}")
    bits = torch.zeros((F, code.n // 8), dtype=torch.uint8, device="cuda")
    conv = torch.zeros(F, dtype=torch.uint8, device="cuda")
    iters = torch.zeros(F, dtype=torch.int32, device="cuda")
    B.ldpc_decode_batch_sched(gc, torch.from_numpy(fr.syn).cuda(), torch.from_numpy(fr.llr).cuda(), F, T,
                              bits, conv, iters, frames_per_workgroup=fpw)
    torch.cuda.synchronize()
    ref = O.decode(code.base, z, fr.syn, fr.llr, T,
                   cn_rule=O.RULE_RCBP_FB if rule == "rcbp" else O.RULE_MINSUM, offsets=off)
    assert np.array_equal(bits.cpu().numpy(), ref["bits"])
    assert np.array_equal(conv.cpu().numpy(), ref["conv"])
    assert np.array_equal(iters.cpu().numpy(), ref["iters"])
