"""Interactive reveal-and-retry on the GPU against the same protocol run with
the CPU oracle: each round the oracle decodes the frames that have not
converged, with the LLRs that puncturing p - k and shortening s + k gives
(the generator's own layout), and the GPU's reveal kernel must reproduce those
LLRs exactly; per frame the rounds used, the convergence flags and the decided
words must agree."""
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


def _oracle_protocol(code, fr0, p0, s0, max_iter, step, max_rounds):
    F = fr0.n_frames
    p, s = p0.copy(), s0.copy()
    rounds = np.zeros(F, dtype=np.int64)
    fr = I.adapt_rate(fr0, p, s)
    out = O.decode(code.base, code.z, fr.syn, fr.llr, max_iter)
    bits, conv = out["bits"].copy(), out["conv"].copy()
    for _ in range(max_rounds):
        ids = np.nonzero((conv == 0) & (p > 0))[0]
        if len(ids) == 0:
            break
        k = np.minimum(step, p[ids])
        p[ids] -= k
        s[ids] += k
        rounds[ids] += 1
        fr = I.adapt_rate(fr0, p, s)
        o = O.decode(code.base, code.z, fr.syn[ids], fr.llr[ids], max_iter)
        bits[ids], conv[ids] = o["bits"], o["conv"]
    return rounds, conv, bits, p, s


@pytest.mark.parametrize("name,shape,q,p0,s0,step", [
    ("n1024_split", (5, 32, 32), 0.02, 300, 100, 40),
    ("n6144_deg6_split", (12, 24, 256), 0.04, 1400, 0, 256),
    ("odd_z_global_batch", (4, 12, 37), 0.03, 60, 30, 16),
])
def test_retry_matches_oracle_protocol(B, name, shape, q, p0, s0, step):
    from paper_1903_10107_amd import retry
    mb, nb, z = shape
    code = I.Code(I.make_base(mb, nb, z), z)
    F = 24
    fr0 = I.make_frames(code, F, q, 31)
    pv = np.full(F, p0, dtype=np.int64)
    sv = np.full(F, s0, dtype=np.int64)
    fr = I.adapt_rate(fr0, pv, sv)
    _say(f"[gpu retry] {name}: n={code.n} p0={p0} s0={s0} step={step}")
    res = retry.reconcile(code, fr, 30, reveal_step=step, max_rounds=6, workgroups=7)
    rounds, conv, bits, p, s = _oracle_protocol(code, fr0, pv, sv, 30, step, 6)
    assert rounds.max() > 0, "the case must exercise at least one reveal round"
    assert np.array_equal(res.rounds, rounds)
    assert np.array_equal(res.converged, conv.astype(bool))
    assert np.array_equal(res.bits, bits)
    assert np.array_equal(res.n_punct, p) and np.array_equal(res.n_short, s)


def test_reveal_kernel_writes_shortened_llrs_and_skips_padding(B):
    import torch
    code = I.Code(I.make_base(5, 32, 32), 32)
    gc = B.Code(code.base, code.z)
    F = 5
    llr = torch.zeros((F, code.n), dtype=torch.int8, device="cuda")
    ids = torch.tensor([3, 0, 9, -1], dtype=torch.int32, device="cuda")
    pos = torch.tensor([[1, 2, -1], [code.n - 1, 5000, 0], [4, 4, 4], [7, 7, 7]], dtype=torch.int32, device="cuda")
    val = torch.tensor([[1, 0, 1], [0, 1, 1], [1, 1, 1], [1, 1, 1]], dtype=torch.uint8, device="cuda")
    B.ldpc_reveal_batch(gc, llr, F, ids, pos, val)
    torch.cuda.synchronize()
    got = llr.cpu().numpy()
    want = np.zeros((F, code.n), dtype=np.int8)
    want[3, 1], want[3, 2] = -127, 127
    want[0, code.n - 1], want[0, 0] = 127, -127
    assert np.array_equal(got, want)
