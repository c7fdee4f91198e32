"""Ragged batches of the rate-adaptive mother code (24x48 base, Z = 2048,
n = 98304): per-frame QBER, puncturing and shortening. The GPU decoder matches
the oracle bit for bit on a small batch (whole state) and, on the full
2048-frame batch in the persistent launch the benchmark tunes among, on sampled
frames plus H x^ = s for every converged frame."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1903_10107_amd import inputs as I

pytestmark = pytest.mark.gpu

MAX_ITER = 60


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


@pytest.fixture(scope="module")
def code():
    return I.Code(I.make_base(24, 48, 2048), 2048)


def test_ragged_small_batch_whole_state(B, code):
    fr = I.make_ragged_frames(code, 6, 4242)
    gc = B.Code(code.base, code.z)
    _say(f"[gpu ragged] small: qber={fr.qber.tolist()} {gc.plan()}")
    got = B.decode(gc, fr.syn, fr.llr, MAX_ITER, want_state=True)
    ref = O.decode(code.base, code.z, fr.syn, fr.llr, MAX_ITER, want_state=True)
    for k in ("bits", "conv", "iters", "L", "E"):
        assert np.array_equal(got[k], ref[k]), k


def test_ragged_with_shortening_whole_state(B, code):
    pts = {0.02: (20000, 3000), 0.05: (0, 5000), 0.07: (4000, 1000)}
    fr = I.make_ragged_frames(code, 4, 77, pts)
    gc = B.Code(code.base, code.z)
    got = B.decode(gc, fr.syn, fr.llr, MAX_ITER, want_state=True)
    ref = O.decode(code.base, code.z, fr.syn, fr.llr, MAX_ITER, want_state=True)
    for k in ("bits", "conv", "iters", "L", "E"):
        assert np.array_equal(got[k], ref[k]), k


@pytest.mark.parametrize("wgs", [0, 512])
def test_ragged_full_batch_sampled(B, code, wgs):
    import torch
    F = 2048
    fr = I.make_ragged_frames(code, F, 10107)
    gc = B.Code(code.base, code.z)
    _say(f"[gpu ragged] full F={F} wgs={wgs} {gc.plan()}")
    d_syn, d_llr = torch.from_numpy(fr.syn).cuda(), torch.from_numpy(fr.llr).cuda()
    bits = torch.zeros((F, code.n // 8), dtype=torch.uint8, device="cuda")
    conv = torch.zeros(F, dtype=torch.uint8, device="cuda")
    iters = torch.zeros(F, dtype=torch.int32, device="cuda")
    order = None
    if wgs:
        order = torch.from_numpy(np.argsort(-fr.qber, kind="stable").astype(np.int32)).cuda()
    B.ldpc_decode_batch_sched(gc, d_syn, d_llr, F, MAX_ITER, bits, conv, iters, persistent_workgroups=wgs,
                              order=order)
    torch.cuda.synchronize()
    b, c, it = bits.cpu().numpy(), conv.cpu().numpy(), iters.cpu().numpy()
    _say(f"[gpu ragged] full: conv={c.mean():.4f} mean iters={it.mean():.2f}")
    xh = I.unpack_bits(b, code.n)
    s_ok = (I.pack_bits(I.syndrome_bits(code, xh)) == fr.syn).all(1)
    assert np.array_equal(s_ok, c.astype(bool))
    assert c.mean() > 0.98
    sample = np.unique(np.array([0, 1, 777, F - 1, int(np.argmax(it)), int(np.argmin(it))]))
    ref = O.decode(code.base, code.z, fr.syn[sample], fr.llr[sample], MAX_ITER)
    assert np.array_equal(b[sample], ref["bits"])
    assert np.array_equal(c[sample], ref["conv"])
    assert np.array_equal(it[sample], ref["iters"])
