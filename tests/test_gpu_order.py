"""ldpc_order_by_unsat: the per-frame count of check rows the channel hard
decision fails equals the count written out from the circulant definition, the
order is a permutation sorted by decreasing count (in buckets of 2^k), and a
persistent decode that takes frames in that order (in a graph replayed several
times, with the order recomputed on the device before every replay) gives the
oracle's results."""
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


def _unsat_reference(base, z, syn_packed, llr):
    """Rows whose parity over the hard decision [llr < 0] differs from the
    syndrome bit, block by block: block (b, c) with shift s joins row b*Z + r to
    column c*Z + (r + s) mod Z."""
    F, n = llr.shape
    mb, nb = base.shape
    yb = (llr < 0).astype(np.uint8)
    par = np.zeros((F, mb * z), dtype=np.uint8)
    r = np.arange(z)
    for b in range(mb):
        for c in range(nb):
            s = int(base[b, c])
            if s >= 0:
                par[:, b * z + r] ^= yb[:, c * z + (r + s) % z]
    s_bits = I.unpack_bits(syn_packed, mb * z)
    return (par != s_bits).sum(1).astype(np.int32)


def _bucket_shift(m):
    k = 0
    while (m >> k) >= 1024:
        k += 1
    return k


@pytest.mark.parametrize("mb,nb,z,F,q,short", [
    (5, 32, 1024, 300, 0.02, 0.33),    # the headline code (word-parallel counts), several buckets
    (4, 12, 37, 64, 0.05, 0.0),        # odd Z, n not a multiple of 64
    (10, 64, 16384, 4, 0.02, 0.0),     # n = 2^20: 128 KB of sign bits in LDS
    (5, 32, 32, 2500, 0.03, 0.0),      # more frames than the order kernel's threads
    (5, 32, 48, 40, 0.03, 0.0),        # Z not a multiple of 32, n is: one lane per row, 16-byte sign loads
    (10, 64, 32768, 2, 0.02, 0.0),     # n = 2^21: the sign words do not fit in LDS
])
def test_unsat_counts_and_order(B, mb, nb, z, F, q, short):
    import torch
    base = I.make_base(mb, nb, z) if z != 37 else I.make_base(mb, nb, z, 3, 5)
    code = I.Code(base, z)
    fr = I.make_frames(code, F, q, 90 + z, n_short=int(short * code.n))
    gc = B.Code(code.base, code.z)
    _say(f"[gpu order] n={code.n} F={F}")
    syn, llr = torch.from_numpy(fr.syn).cuda(), torch.from_numpy(fr.llr).cuda()
    w = torch.full((F,), -1, dtype=torch.int32, device="cuda")
    order = torch.full((F,), -1, dtype=torch.int32, device="cuda")
    B.ldpc_order_by_unsat(gc, syn, llr, F, w, order)
    torch.cuda.synchronize()
    w, order = w.cpu().numpy(), order.cpu().numpy()
    assert np.array_equal(w, _unsat_reference(code.base, z, fr.syn, fr.llr))
    assert np.array_equal(np.sort(order), np.arange(F))              # a permutation
    key = np.minimum(w[order] >> _bucket_shift(code.m), 1023)
    assert (np.diff(key) <= 0).all()                                  # decreasing buckets
    # counts alone
    w2 = torch.zeros(F, dtype=torch.int32, device="cuda")
    B.ldpc_order_by_unsat(gc, syn, llr, F, w2)
    torch.cuda.synchronize()
    assert np.array_equal(w2.cpu().numpy(), w)


def test_zero_error_frames_count_zero_and_arguments(B):
    import ctypes as C
    import torch
    code = I.Code(I.make_base(5, 32, 32), 32)
    fr = I.make_frames(code, 8, 1e-9, 3)
    gc = B.Code(code.base, code.z)
    syn, llr = torch.from_numpy(fr.syn).cuda(), torch.from_numpy(fr.llr).cuda()
    w = torch.full((8,), -1, dtype=torch.int32, device="cuda")
    B.ldpc_order_by_unsat(gc, syn, llr, 8, w)
    torch.cuda.synchronize()
    assert (w.cpu().numpy() == 0).all()
    lib = B.lib()
    p = C.c_void_p(w.data_ptr())
    assert lib.ldpc_order_by_unsat(gc.handle, None, llr.data_ptr(), 8, p, None, None) == B.LDPC_EINVAL
    assert b"non-NULL" in lib.ldpc_last_error()
    assert lib.ldpc_order_by_unsat(gc.handle, syn.data_ptr(), llr.data_ptr(), -1, p, None, None) == B.LDPC_EINVAL
    assert lib.ldpc_order_by_unsat(None, syn.data_ptr(), llr.data_ptr(), 8, p, None, None) == B.LDPC_EINVAL
    assert lib.ldpc_order_by_unsat(gc.handle, None, None, 0, None, None, None) == B.LDPC_OK


@pytest.mark.parametrize("graph", [False, True])
def test_persistent_decode_in_unsat_order_matches_oracle(B, graph):
    import torch
    from paper_1903_10107_amd import tune
    code = I.Code(I.make_base(5, 32, 1024), 1024)
    F = 600
    fr = I.make_frames(code, F, 0.02, 4321, n_short=int(0.31 * code.n))
    ref = O.decode(code.base, code.z, fr.syn, fr.llr, 50)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    run = tune.Runner(code.base, code.z, fr.syn, fr.llr, 50, tune.Schedule("split", n_cu, "unsat_first", graph))
    _say(f"[gpu order] persistent unsat-first decode, graph={graph}")
    for rep in range(3):
        run.bits.zero_()
        run.iters.fill_(-1)
        run()
        torch.cuda.synchronize()
        bits, conv, iters = run.outputs()
        assert np.array_equal(bits, ref["bits"]) and np.array_equal(conv, ref["conv"]) \
            and np.array_equal(iters, ref["iters"]), f"replay {rep}"
