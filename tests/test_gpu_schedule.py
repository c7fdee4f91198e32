"""Batch schedules and graph-captured batches: the decoded results do not depend
on the schedule. Persistent workgroups with and without a decode order, and a
graph replayed several times with eager work and synchronizations between the
replays, are compared with the one-workgroup-per-frame decode and the oracle."""
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


def _setup(B, z=1024, F=40, q=0.02, short=0.30, seed=31):
    import torch
    code = I.Code(I.make_base(5, 32, z), z)
    fr = I.make_frames(code, F, q, seed, n_short=int(short * code.n))
    gc = B.Code(code.base, code.z)
    dev = dict(syn=torch.from_numpy(fr.syn).cuda(), llr=torch.from_numpy(fr.llr).cuda())
    return code, fr, gc, dev


def _outs(code, F):
    import torch
    return (torch.zeros((F, (code.n + 7) // 8), dtype=torch.uint8, device="cuda"),
            torch.zeros(F, dtype=torch.uint8, device="cuda"),
            torch.zeros(F, dtype=torch.int32, device="cuda"))


@pytest.mark.parametrize("wgs,ordered", [(1, False), (7, True), (64, False), (300, True)])
def test_persistent_schedule_matches_oracle(B, wgs, ordered):
    import torch
    code, fr, gc, dev = _setup(B)
    F = fr.n_frames
    _say(f"[gpu schedule] persistent wgs={wgs} ordered={ordered} {gc.plan()}")
    order = None
    if ordered:
        order = torch.from_numpy(np.random.default_rng(wgs).permutation(F).astype(np.int32)).cuda()
    bits, conv, iters = _outs(code, F)
    B.ldpc_decode_batch_sched(gc, dev["syn"], dev["llr"], F, 50, bits, conv, iters, persistent_workgroups=wgs,
                              order=order)
    torch.cuda.synchronize()
    ref = O.decode(code.base, code.z, fr.syn, fr.llr, 50)
    assert np.array_equal(bits.cpu().numpy(), ref["bits"])
    assert np.array_equal(conv.cpu().numpy(), ref["conv"])
    assert np.array_equal(iters.cpu().numpy(), ref["iters"])


@pytest.mark.parametrize("family", ["split_reg", "split"])
def test_persistent_schedule_with_offset_table(B, family):
    import torch
    code = I.Code(I.make_base(5, 32, 256), 256)
    fr = I.make_frames(code, 24, 0.02, 8, n_short=int(0.2 * code.n))
    off = np.random.default_rng(3).integers(-2, 6, size=(5, code.n_blocks)).astype(np.int8)
    kw = {} if family == "split_reg" else {"kernel": family}   # automatic selection picks split_reg
    gc = B.Code(code.base, code.z, cn_rule=B.LDPC_RULE_MINSUM, offsets=off, **kw)
    assert gc.plan()["kernel"] == family
    _say(f"[gpu schedule] persistent with offsets {gc.plan()}")
    F = fr.n_frames
    bits, conv, iters = _outs(code, F)
    B.ldpc_decode_batch_sched(gc, torch.from_numpy(fr.syn).cuda(), torch.from_numpy(fr.llr).cuda(), F, 40,
                              bits, conv, iters, persistent_workgroups=5)
    torch.cuda.synchronize()
    ref = O.decode(code.base, code.z, fr.syn, fr.llr, 40, cn_rule=O.RULE_MINSUM, offsets=off)
    assert np.array_equal(bits.cpu().numpy(), ref["bits"])
    assert np.array_equal(conv.cpu().numpy(), ref["conv"])
    assert np.array_equal(iters.cpu().numpy(), ref["iters"])


def test_order_with_out_of_range_entries_skips_them(B):
    import torch
    code, fr, gc, dev = _setup(B, F=12)
    F = fr.n_frames
    order = torch.tensor([3, 99, -1, 5] + list(range(6, 12)) + [0, 1], dtype=torch.int32, device="cuda")
    bits, conv, iters = _outs(code, F)
    iters.fill_(-7)
    B.ldpc_decode_batch_sched(gc, dev["syn"], dev["llr"], F, 50, bits, conv, iters, persistent_workgroups=3,
                              order=order)
    torch.cuda.synchronize()
    ref = O.decode(code.base, code.z, fr.syn, fr.llr, 50)
    it = iters.cpu().numpy()
    done = [0, 1, 3, 5] + list(range(6, 12))
    assert np.array_equal(it[done], ref["iters"][done])
    assert it[2] == -7 and it[4] == -7


def test_schedule_argument_errors(B):
    import torch
    code, fr, gc, dev = _setup(B, F=4)
    bits, conv, iters = _outs(code, 4)
    order = torch.arange(4, dtype=torch.int32, device="cuda")
    with pytest.raises(B.LdpcError):
        B.ldpc_decode_batch_sched(gc, dev["syn"], dev["llr"], 4, 10, bits, conv, iters, persistent_workgroups=0,
                                  order=order)
    odd = B.Code(I.make_base(4, 12, 37, 3, 5), 37)          # odd Z: not the split family
    fr2 = I.make_frames(I.Code(odd.base, 37), 2, 0.02, 1)
    b2, c2, i2 = _outs(I.Code(odd.base, 37), 2)
    with pytest.raises(B.LdpcError) as ei:
        B.ldpc_decode_batch_sched(odd, torch.from_numpy(fr2.syn).cuda(), torch.from_numpy(fr2.llr).cuda(), 2, 10,
                                  b2, c2, i2, persistent_workgroups=4)
    assert ei.value.code == B.LDPC_EUNSUPPORTED
    ls = B.Code(I.make_base(5, 32, 64), 64, kernel="layer_sync")   # several launches per decode: no queue
    fr3 = I.make_frames(I.Code(ls.base, 64), 2, 0.02, 1)
    b3, c3, i3 = _outs(I.Code(ls.base, 64), 2)
    with pytest.raises(B.LdpcError) as ei:
        B.ldpc_decode_batch_sched(ls, torch.from_numpy(fr3.syn).cuda(), torch.from_numpy(fr3.llr).cuda(), 2, 10,
                                  b3, c3, i3, persistent_workgroups=4)
    assert ei.value.code == B.LDPC_EUNSUPPORTED


@pytest.mark.parametrize("wgs", [0, 256])
def test_graph_batch_replays_match_eager(B, wgs):
    import torch
    code, fr, gc, dev = _setup(B, F=64, seed=41)
    F = fr.n_frames
    _say(f"[gpu graph] wgs={wgs}")
    eb, ec, ei = _outs(code, F)
    B.ldpc_decode_batch_sched(gc, dev["syn"], dev["llr"], F, 50, eb, ec, ei, persistent_workgroups=wgs)
    torch.cuda.synchronize()
    eager = (eb.cpu().numpy(), ec.cpu().numpy(), ei.cpu().numpy())
    gb, gcv, gi = _outs(code, F)
    batch = B.Batch(gc, dev["syn"], dev["llr"], F, 50, gb, gcv, gi, persistent_workgroups=wgs)
    for rep in range(4):
        gb.zero_()
        gcv.zero_()
        gi.fill_(-1)
        scratch = torch.randn(1 << 16, device="cuda").sum()    # eager work between replays
        batch.launch()
        torch.cuda.synchronize()
        assert float(scratch) == float(scratch)
        assert np.array_equal(gb.cpu().numpy(), eager[0]), rep
        assert np.array_equal(gcv.cpu().numpy(), eager[1]), rep
        assert np.array_equal(gi.cpu().numpy(), eager[2]), rep
    del batch


def test_graph_of_a_layer_synchronous_decode_replays(B):
    """The layer-synchronous family is a sequence of launches; captured as one
    graph it replays to the eager result (with eager work between replays)."""
    import torch
    code = I.Code(I.make_base(5, 32, 256), 256)
    fr = I.make_frames(code, 12, 0.02, 43, n_short=int(0.3 * code.n))
    gc = B.Code(code.base, code.z, kernel="layer_sync")
    syn, llr = torch.from_numpy(fr.syn).cuda(), torch.from_numpy(fr.llr).cuda()
    F = fr.n_frames
    eb, ec, ei = _outs(code, F)
    B.ldpc_decode_batch_sched(gc, syn, llr, F, 30, eb, ec, ei)
    torch.cuda.synchronize()
    ref = O.decode(code.base, code.z, fr.syn, fr.llr, 30)
    assert np.array_equal(eb.cpu().numpy(), ref["bits"]) and np.array_equal(ei.cpu().numpy(), ref["iters"])
    gb, gcv, gi = _outs(code, F)
    batch = B.Batch(gc, syn, llr, F, 30, gb, gcv, gi)
    for rep in range(3):
        gb.zero_()
        gi.fill_(-1)
        scratch = torch.randn(1 << 14, device="cuda").sum()
        batch.launch()
        torch.cuda.synchronize()
        assert float(scratch) == float(scratch)
        assert np.array_equal(gb.cpu().numpy(), ref["bits"]), rep
        assert np.array_equal(gi.cpu().numpy(), ref["iters"]), rep
    del batch


@pytest.mark.parametrize("check_every,graph", [(1, False), (3, False), (1, True), (4, True)])
def test_layer_sync_early_stop_matches_oracle(B, check_every, graph):
    """check_every > 0: the host stops launching iterations once every frame has
    retired; the results are those of the full decode (frames converge at
    different iterations, one frame runs out of iterations, and max_iter is not
    a multiple of check_every)."""
    import torch
    code = I.Code(I.make_base(5, 32, 256), 256)
    q = np.full(10, 0.02)
    q[3] = 0.2                                   # cannot converge: runs all max_iter iterations
    fr = I.make_frames(code, 10, q, 71, n_short=int(0.3 * code.n))
    gc = B.Code(code.base, code.z, kernel="layer_sync")
    syn, llr = torch.from_numpy(fr.syn).cuda(), torch.from_numpy(fr.llr).cuda()
    F, T = fr.n_frames, 13
    ref = O.decode(code.base, code.z, fr.syn, fr.llr, T)
    assert ref["conv"][3] == 0 and ref["iters"].min() < T
    _say(f"[gpu early stop] check_every={check_every} graph={graph} iters={ref['iters'].tolist()}")
    bits, conv, iters = _outs(code, F)
    if graph:
        batch = B.Batch(gc, syn, llr, F, T, bits, conv, iters, check_every=check_every)
        for rep in range(2):
            bits.zero_()
            iters.fill_(-1)
            batch.launch()
            torch.cuda.synchronize()
            assert np.array_equal(bits.cpu().numpy(), ref["bits"]), rep
            assert np.array_equal(conv.cpu().numpy(), ref["conv"]), rep
            assert np.array_equal(iters.cpu().numpy(), ref["iters"]), rep
        del batch
    else:
        B.ldpc_decode_batch_sched(gc, syn, llr, F, T, bits, conv, iters, check_every=check_every)
        torch.cuda.synchronize()
        assert np.array_equal(bits.cpu().numpy(), ref["bits"])
        assert np.array_equal(conv.cpu().numpy(), ref["conv"])
        assert np.array_equal(iters.cpu().numpy(), ref["iters"])


def test_early_stop_all_converged_at_iteration_0_and_argument_errors(B):
    import torch
    code = I.Code(I.make_base(5, 32, 64), 64)
    fr = I.make_frames(code, 4, 1e-9, 5)         # no errors: every frame satisfies the syndrome at once
    gc = B.Code(code.base, code.z, kernel="layer_sync")
    syn, llr = torch.from_numpy(fr.syn).cuda(), torch.from_numpy(fr.llr).cuda()
    bits, conv, iters = _outs(code, 4)
    B.ldpc_decode_batch_sched(gc, syn, llr, 4, 20, bits, conv, iters, check_every=2)
    torch.cuda.synchronize()
    ref = O.decode(code.base, code.z, fr.syn, fr.llr, 20)
    assert np.array_equal(iters.cpu().numpy(), ref["iters"]) and ref["iters"].max() == 0
    assert np.array_equal(bits.cpu().numpy(), ref["bits"])
    with pytest.raises(B.LdpcError) as ei:
        B.ldpc_decode_batch_sched(gc, syn, llr, 4, 20, bits, conv, iters, check_every=-1)
    assert ei.value.code == B.LDPC_EINVAL
    sp = B.Code(code.base, code.z)                # single-launch family: check_every is ignored
    assert sp.plan()["kernel"] in ("split_reg", "split")
    B.ldpc_decode_batch_sched(sp, syn, llr, 4, 20, bits, conv, iters, check_every=2)
    torch.cuda.synchronize()
    assert np.array_equal(bits.cpu().numpy(), ref["bits"])


def test_layer_sync_frame_limit_is_an_argument_error(B):
    """The layer-synchronous launches index frames in the second grid dimension:
    more than 65535 frames per call is refused before anything is launched."""
    import torch
    code = I.Code(I.make_base(5, 32, 32), 32)
    gc = B.Code(code.base, code.z, kernel="layer_sync")
    F = 65536
    syn = torch.zeros((F, (code.m + 7) // 8), dtype=torch.uint8, device="cuda")
    llr = torch.zeros((F, code.n), dtype=torch.int8, device="cuda")
    bits, conv, iters = _outs(code, F)
    with pytest.raises(B.LdpcError) as ei:
        B.ldpc_decode_batch_sched(gc, syn, llr, F, 10, bits, conv, iters)
    assert ei.value.code == B.LDPC_EINVAL


@pytest.mark.parametrize("z,fpw", [(32, 2), (32, 8), (32, 32), (64, 1), (64, 16)])
def test_frames_per_workgroup_matches_oracle(B, z, fpw):
    """Several frames per workgroup (a frame's lanes inside one wave, no
    workgroup barrier) give the oracle's results; frames of one wave converge at
    different iterations, one cannot converge, and the frame count is not a
    multiple of the frames per workgroup."""
    import torch
    code = I.Code(I.make_base(5, 32, z), z)
    F = 37
    q = np.where(np.arange(F) % 4 == 0, 0.03, 0.01)
    q[5] = 0.3
    fr = I.make_frames(code, F, q, 4040 + z)
    gc = B.Code(code.base, code.z)
    assert gc.plan()["kernel"] == "split_reg"
    ref = O.decode(code.base, code.z, fr.syn, fr.llr, 30)
    assert ref["conv"][5] == 0 and len(set(ref["iters"].tolist())) > 3
    _say(f"[gpu fpw] z={z} frames_per_workgroup={fpw}")
    syn, llr = torch.from_numpy(fr.syn).cuda(), torch.from_numpy(fr.llr).cuda()
    bits, conv, iters = _outs(code, F)
    B.ldpc_decode_batch_sched(gc, syn, llr, F, 30, bits, conv, iters, frames_per_workgroup=fpw)
    torch.cuda.synchronize()
    assert np.array_equal(bits.cpu().numpy(), ref["bits"])
    assert np.array_equal(conv.cpu().numpy(), ref["conv"])
    assert np.array_equal(iters.cpu().numpy(), ref["iters"])
    # the same schedule as a replayed graph, and with no iteration at all
    batch = B.Batch(gc, syn, llr, F, 30, bits, conv, iters, frames_per_workgroup=fpw)
    for rep in range(2):
        bits.zero_()
        iters.fill_(-1)
        batch.launch()
        torch.cuda.synchronize()
        assert np.array_equal(bits.cpu().numpy(), ref["bits"]), rep
        assert np.array_equal(iters.cpu().numpy(), ref["iters"]), rep
    del batch
    ref0 = O.decode(code.base, code.z, fr.syn, fr.llr, 0)
    B.ldpc_decode_batch_sched(gc, syn, llr, F, 0, bits, conv, iters, frames_per_workgroup=fpw)
    torch.cuda.synchronize()
    assert np.array_equal(bits.cpu().numpy(), ref0["bits"])
    assert np.array_equal(conv.cpu().numpy(), ref0["conv"])


def test_frames_per_workgroup_argument_errors(B):
    import torch
    code = I.Code(I.make_base(5, 32, 32), 32)
    fr = I.make_frames(code, 4, 0.01, 3)
    syn, llr = torch.from_numpy(fr.syn).cuda(), torch.from_numpy(fr.llr).cuda()
    bits, conv, iters = _outs(code, 4)
    gc = B.Code(code.base, code.z)
    for kw, rc in (({"frames_per_workgroup": 3}, B.LDPC_EINVAL),            # not a multiple of 64 / z
                   ({"frames_per_workgroup": 34}, B.LDPC_EINVAL),           # 17 waves
                   ({"frames_per_workgroup": -2}, B.LDPC_EINVAL),
                   ({"frames_per_workgroup": 2, "persistent_workgroups": 4}, B.LDPC_EINVAL)):
        with pytest.raises(B.LdpcError) as ei:
            B.ldpc_decode_batch_sched(gc, syn, llr, 4, 10, bits, conv, iters, **kw)
        assert ei.value.code == rc, kw
    big = I.Code(I.make_base(5, 32, 256), 256)
    gb = B.Code(big.base, big.z)
    frb = I.make_frames(big, 2, 0.01, 3)
    bb, cb, ib = _outs(big, 2)
    with pytest.raises(B.LdpcError) as ei:
        B.ldpc_decode_batch_sched(gb, torch.from_numpy(frb.syn).cuda(), torch.from_numpy(frb.llr).cuda(), 2, 10,
                                  bb, cb, ib, frames_per_workgroup=2)
    assert ei.value.code == B.LDPC_EUNSUPPORTED
