"""ldpc_decode_batch_static (workspace in the library's static device buffer)
against ldpc_decode_batch_sched (workspace allocated per call) on the kernel
families that use a workspace: two calls in a row, the second with fewer
frames, must give the same bits, flags and iteration counts bit for bit."""
import sys

import numpy as np
import pytest

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


def _outs(code, F):
    import torch
    return (torch.zeros((F, (code.n + 7) // 8), dtype=torch.uint8, device="cuda"),
            torch.zeros(F, dtype=torch.uint8, device="cuda"),
            torch.full((F,), -7, dtype=torch.int32, device="cuda"))


# name: (mb, nb, z, frames of the first call, of the second, qber, shortened fraction,
#        max_iter, kernel hint, persistent workgroups, acc bits)
CASES = {
    "n98304_global_l": (24, 48, 2048, 12, 5, 0.04, 0.1, 20, "auto", 0, 0),
    "n98304_global_l_persistent": (24, 48, 2048, 12, 7, 0.04, 0.1, 20, "auto", 9, 0),
    "n32768_reg_persistent": (5, 32, 1024, 40, 17, 0.02, 0.33, 50, "auto", 13, 0),
    "n8192_global": (5, 32, 256, 24, 9, 0.02, 0.3, 30, "global", 0, 0),
    "n1048576_layer_sync": (10, 64, 16384, 3, 1, 0.02, 0.33, 12, "auto", 0, 16),
}


@pytest.mark.parametrize("name", list(CASES))
def test_static_workspace_matches_allocating_call(B, name):
    import torch
    mb, nb, z, F1, F2, q, short, it, kernel, wgs, acc = CASES[name]
    code = I.Code(I.make_base(mb, nb, z), z)
    gc = B.Code(code.base, z, kernel=kernel, acc_bits=acc)
    need = B.ldpc_workspace_bytes_sched(gc, F1, wgs)
    assert 0 < need <= B.STATIC_WORKSPACE_BYTES, (name, need)
    for F, seed in ((F1, 11), (F2, 12)):
        fr = I.make_frames(code, F, q, seed, n_short=int(short * code.n))
        syn, llr = torch.from_numpy(fr.syn).cuda(), torch.from_numpy(fr.llr).cuda()
        order = torch.from_numpy(np.arange(F)[::-1].astype(np.int32).copy()).cuda() if wgs else None
        _say(f"[gpu no-alloc] {name} F={F} {gc.plan()} persistent={wgs}")
        ref = _outs(code, F)
        B.ldpc_decode_batch_sched(gc, syn, llr, F, it, *ref, persistent_workgroups=wgs, order=order)
        got = _outs(code, F)
        B.ldpc_decode_batch_static(gc, syn, llr, F, it, *got, persistent_workgroups=wgs, order=order)
        torch.cuda.synchronize()
        for a, b, what in zip(got, ref, ("bits", "conv", "iters")):
            assert torch.equal(a, b), (name, F, what)
        assert int(ref[2].min()) >= 0


def test_static_workspace_refuses_what_it_cannot_hold(B):
    import torch
    code = I.Code(I.make_base(10, 64, 16384), 16384)
    gc = B.Code(code.base, code.z, acc_bits=16)
    F = 32
    assert B.ldpc_workspace_bytes_sched(gc, F) > B.STATIC_WORKSPACE_BYTES
    syn = torch.zeros((F, (code.m + 7) // 8), dtype=torch.uint8, device="cuda")
    llr = torch.zeros((F, code.n), dtype=torch.int8, device="cuda")
    outs = _outs(code, F)
    with pytest.raises(B.LdpcError) as ei:
        B.ldpc_decode_batch_static(gc, syn, llr, F, 5, *outs)
    assert ei.value.code == B.LDPC_EINVAL and "static limit" in str(ei.value)
    with pytest.raises(B.LdpcError) as ei:
        B.ldpc_decode_batch_static(gc, syn[:1], llr[:1], 1, 5, *(o[:1] for o in outs), check_every=1)
    assert ei.value.code == B.LDPC_EUNSUPPORTED
