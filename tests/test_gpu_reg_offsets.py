"""Offset tables on the register-resident family (split_reg): the magnitudes of
the check-node messages lose a per-iteration, per-base-edge offset and are
clamped to [0, MSG_max] (the offset form of the check node, with the offsets the
learned decoder quantizes), on the one-frame-per-workgroup and the persistent
kernels, for both check-node rules; compared with the oracle bit for bit."""
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


def test_frames_per_workgroup_refuses_offset_tables(B):
    import torch
    code = I.Code(I.make_base(5, 32, 32), 32)
    off = np.zeros((2, code.n_blocks), dtype=np.int8)
    gc = B.Code(code.base, 32, cn_rule=B.LDPC_RULE_MINSUM, offsets=off)
    assert gc.plan()["kernel"] == "split_reg"
    fr = I.make_frames(code, 4, 0.02, 9)
    bits = torch.zeros((4, code.n // 8), dtype=torch.uint8, device="cuda")
    conv = torch.zeros(4, dtype=torch.uint8, device="cuda")
    iters = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(B.LdpcError) as ei:
        B.ldpc_decode_batch_sched(gc, torch.from_numpy(fr.syn).cuda(), torch.from_numpy(fr.llr).cuda(), 4, 10,
                                  bits, conv, iters, frames_per_workgroup=2)
    assert ei.value.code == B.LDPC_EUNSUPPORTED
