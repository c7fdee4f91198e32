"""GPU decoder vs the CPU oracle, element by element, through the C ABI.

Every case compares the packed hard decisions, the converged flags, the
iteration counts, the final CN->VN messages L and the final soft values E,
bit-exactly. Small cases decode every frame on both sides; the full-size
workloads decode the whole batch on the GPU in the benchmark's launch
configuration and compare a sample of frames with the oracle, plus H x^ = s
on every converged frame.
"""
import sys
import zlib

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


def _rand_base(mb, nb, z, seed, col_weight=3):
    return I.make_base(mb, nb, z, col_weight, seed)


_HAMMING = np.array([[0, 0, 0, -1, 0, -1, -1],
                     [0, 0, -1, 0, -1, 0, -1],
                     [0, -1, 0, 0, -1, -1, 0]], dtype=np.int32)

CASES = {
    # name: (base factory, z, frames, qber, max_iter, kwargs for code, frame kwargs)
    "n1024_q1": (lambda: I.make_base(5, 32, 32), 32, 64, 0.01, 50, {}, {}),
    "n1024_q3": (lambda: I.make_base(5, 32, 32), 32, 32, 0.03, 50, {}, {}),
    "array_n20": (lambda: I.array_code_base(5, 3, 4), 5, 16, 0.05, 30, {}, {}),
    "odd_z37": (lambda: _rand_base(4, 12, 37, 5), 37, 16, 0.03, 40, {}, {}),
    "n8192_q2": (lambda: I.make_base(5, 32, 256), 256, 16, 0.02, 20, {}, {}),
    "n32768_short": (lambda: I.make_base(5, 32, 1024), 1024, 6, 0.02, 50, {}, {"short_frac": 0.3}),
    "z1500_rows_per_thread_2": (lambda: _rand_base(3, 8, 1500, 6), 1500, 4, 0.03, 30, {}, {}),
    "acc16": (lambda: I.make_base(5, 32, 256), 256, 8, 0.02, 30, {"acc_bits": 16}, {}),
    "acc8_emax100": (lambda: I.make_base(5, 32, 64), 64, 8, 0.02, 30, {"e_max": 100}, {}),
    # 16-bit soft values with a low E_max: the Alg. 2 freeze fires often
    "acc16_emax80": (lambda: I.make_base(5, 32, 64), 64, 8, 0.02, 30, {"acc_bits": 16, "e_max": 80},
                     {"short_frac": 0.2}),
    "layer_sync_acc16_emax80": (lambda: I.make_base(5, 32, 64), 64, 8, 0.02, 30,
                                {"kernel": "layer_sync", "acc_bits": 16, "e_max": 80}, {"short_frac": 0.2}),
    "acc8_emax40_frozen": (lambda: I.make_base(5, 32, 64), 64, 8, 0.02, 30, {"e_max": 40}, {"short_frac": 0.2}),
    "acc16_emax1": (lambda: I.make_base(5, 32, 32), 32, 8, 0.02, 10, {"acc_bits": 16, "e_max": 1}, {}),
    "msgmax31": (lambda: I.make_base(5, 32, 64), 64, 8, 0.02, 30, {"msg_max": 31}, {}),
    "rule_eq7": (lambda: I.make_base(5, 32, 32), 32, 16, 0.02, 30, {"cn_rule": 1}, {}),
    "rule_minsum": (lambda: I.make_base(5, 32, 32), 32, 16, 0.01, 30, {"cn_rule": 2}, {}),
    "minsum_offsets": (lambda: I.make_base(5, 32, 32), 32, 16, 0.01, 30, {"cn_rule": 2, "offsets": "rand"}, {}),
    "rcbp_offsets": (lambda: I.make_base(5, 32, 32), 32, 16, 0.01, 30, {"offsets": "rand"}, {}),
    "minsum_signed_offsets_acc16": (lambda: I.make_base(5, 32, 64), 64, 8, 0.02, 30,
                                    {"cn_rule": 2, "offsets": "rand_signed", "acc_bits": 16}, {}),
    "eq7_offsets": (lambda: I.make_base(5, 32, 32), 32, 8, 0.02, 30, {"cn_rule": 1, "offsets": "rand_signed"}, {}),
    "deg6_offsets": (lambda: I.make_base(12, 24, 256), 256, 6, 0.04, 30, {"offsets": "rand_signed"},
                     {"short_frac": 0.1}),
    "deg6_n98304_global_state": (lambda: I.make_base(24, 48, 2048), 2048, 2, 0.04, 8, {"kernel": "global"},
                                 {"short_frac": 0.1, "punct_frac": 0.1}),
    "deg6_n98304_global_l": (lambda: I.make_base(24, 48, 2048), 2048, 3, 0.04, 12, {},
                             {"short_frac": 0.1, "punct_frac": 0.1}),
    "deg6_z2048_lds_rows_per_pair_2": (lambda: _rand_base(4, 8, 2048, 9), 2048, 4, 0.03, 20, {}, {}),
    "deg6_z4096_global_l_rows_per_pair_4": (lambda: _rand_base(6, 12, 4096, 8), 4096, 2, 0.04, 10, {}, {}),
    "n65536_deg20_global_l": (lambda: I.make_base(5, 32, 2048), 2048, 3, 0.02, 20, {}, {"short_frac": 0.33}),
    "layer_sync_n32768": (lambda: I.make_base(5, 32, 1024), 1024, 5, 0.02, 40, {"kernel": "layer_sync"},
                          {"short_frac": 0.3}),
    "layer_sync_max_iter0": (lambda: I.make_base(5, 32, 64), 64, 6, 0.01, 0, {"kernel": "layer_sync"}, {}),
    "layer_sync_minsum_acc16": (lambda: I.make_base(5, 32, 64), 64, 8, 0.01, 30,
                                {"kernel": "layer_sync", "cn_rule": 2, "acc_bits": 16}, {}),
    "layer_sync_deg6_ragged": (lambda: I.make_base(24, 48, 256), 256, 6, 0.04, 30, {"kernel": "layer_sync"},
                               {"short_frac": 0.05, "punct_frac": 0.1}),
    "deg6_n98304_global_l_offsets": (lambda: I.make_base(24, 48, 2048), 2048, 2, 0.04, 12,
                                     {"cn_rule": 2, "offsets": "rand_signed"}, {"short_frac": 0.1, "punct_frac": 0.1}),
    "layer_sync_offsets": (lambda: I.make_base(5, 32, 64), 64, 6, 0.02, 30,
                           {"kernel": "layer_sync", "offsets": "rand_signed"}, {}),
    "max_iter0": (lambda: I.make_base(5, 32, 32), 32, 16, 0.01, 0, {}, {}),
    "zero_error": (lambda: I.make_base(5, 32, 32), 32, 8, 1e-9, 50, {}, {}),
    "row_deg_24": (lambda: _rand_base(2, 24, 64, 7, 2), 64, 8, 0.01, 30, {}, {}),
    # Z = 1: a plain (Hamming (7,4)) parity-check matrix written as a base matrix,
    # and its Z = 2 lift
    "z1_hamming": (lambda: _HAMMING, 1, 16, 0.1, 10, {}, {}),
    "z2_hamming_lift": (lambda: _HAMMING, 2, 16, 0.1, 10, {}, {}),
}


def _frames(base, z, F, q, fkw, seed):
    code = I.Code(base, z)
    ns = int(fkw.get("short_frac", 0) * code.n)
    npn = int(fkw.get("punct_frac", 0) * code.n)
    return code, I.make_frames(code, F, q, seed, n_short=ns, n_punct=npn)


def _compare(got, ref, frames=None):
    for k in ("bits", "conv", "iters", "L", "E"):
        if k not in ref:
            continue
        g = got[k] if frames is None else got[k][frames]
        assert g.shape == ref[k].shape, k
        if not np.array_equal(g, ref[k]):
            bad = np.argwhere(g != ref[k])
            raise AssertionError(f"{k} differs at {len(bad)} places, first {bad[:5].tolist()}")


@pytest.mark.parametrize("name", list(CASES))
def test_parity_small(B, name):
    mk, z, F, q, it, ckw, fkw = CASES[name]
    base = mk()
    code, fr = _frames(base, z, F, q, fkw, seed=zlib.crc32(name.encode()) & 0xFFFF)
    ckw = dict(ckw)
    okw = {}
    if ckw.get("offsets") in ("rand", "rand_signed"):
        # three iterations' rows; later iterations reuse the last one
        rng = np.random.default_rng(1)
        lo, hi = (0, 4) if ckw["offsets"] == "rand" else (-4, 8)
        ckw["offsets"] = rng.integers(lo, hi, size=(3, code.n_blocks)).astype(np.int8)
    if "offsets" in ckw:
        okw["offsets"] = ckw["offsets"]
    for k in ("acc_bits", "e_max", "msg_max", "cn_rule"):
        if k in ckw:
            okw[k] = ckw[k]
    gc = B.Code(base, z, **ckw)
    _say(f"[gpu parity] {name}: n={code.n} F={F} q={q} max_iter={it} {sorted(okw)} {gc.plan()}")
    got = B.decode(gc, fr.syn, fr.llr, it, want_state=True)
    ref = O.decode(base, z, fr.syn, fr.llr, it, want_state=True, **okw)
    _compare(got, ref)


def test_cases_cover_every_kernel_family(B):
    seen = set()
    for name, (mk, z, F, q, it, ckw, fkw) in CASES.items():
        ckw = dict(ckw)
        if ckw.get("offsets") in ("rand", "rand_signed"):
            ckw["offsets"] = np.zeros((1, int((mk() >= 0).sum())), np.int8)
        seen.add(B.Code(mk(), z, **ckw).plan()["kernel"])
    assert seen == {"global", "lds", "pairs", "split", "split_global_l", "layer_sync", "split_reg"}, seen


def test_llr_minus_128_is_read_as_minus_127(B):
    """-128 anywhere in a row (the vectorized stage-in fixes it byte by byte)."""
    code = I.Code(I.make_base(5, 32, 1024), 1024)
    fr = I.make_frames(code, 4, 0.02, 77, n_short=int(0.33 * code.n))
    llr = fr.llr.copy()
    rng = np.random.default_rng(5)
    llr[rng.random(llr.shape) < 0.05] = -128
    llr[:, 1:9] = np.array([-128, -127, -128, 1, -128, 0, -128, -128], dtype=np.int8)
    gc = B.Code(code.base, code.z)
    _say(f"[gpu parity] llr -128: {gc.plan()}")
    got = B.decode(gc, fr.syn, llr, 30, want_state=True)
    ref = O.decode(code.base, code.z, fr.syn, llr, 30, want_state=True)
    _compare(got, ref)


def test_n_frames_zero_is_a_noop(B):
    import torch
    code = B.Code(I.make_base(5, 32, 32), 32)
    e = torch.empty(0, dtype=torch.uint8, device="cuda")
    B.ldpc_decode_batch(code, e, e.to(torch.int8), 0, 10, e, e)
    torch.cuda.synchronize()


def test_binding_rejects_short_buffers(B):
    import torch
    code = B.Code(I.make_base(5, 32, 32), 32)
    syn = torch.zeros((4, code.m // 8), dtype=torch.uint8, device="cuda")
    llr = torch.zeros((3, code.n), dtype=torch.int8, device="cuda")
    bits = torch.zeros((4, code.n // 8), dtype=torch.uint8, device="cuda")
    conv = torch.zeros(4, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        B.ldpc_decode_batch(code, syn, llr, 4, 10, bits, conv)


@pytest.mark.parametrize("mb,nb,z,frames,misalign", [
    (5, 32, 32, 5, 0),       # word kernel (Z a multiple of 32, fewer than 8 frames), one partial workgroup
    (4, 12, 37, 5, 0),       # Z not a multiple of 32: bit kernel
    (5, 32, 1024, 5, 0),     # word kernel, the n = 32768 code
    (5, 32, 1024, 300, 0),   # word kernel, many frames (workgroups span frames)
    (5, 32, 1024, 1030, 0),  # >= 1024 frames: four frames per workgroup staged in LDS (16-byte loads), last one 2
    (5, 32, 1024, 1027, 4),  # the same with buffers 4- but not 16-byte aligned (dword loads), last workgroup 3
    (5, 32, 256, 1100, 0),   # Z = 256: 40 syndrome words per frame, too few for the LDS kernel
    (10, 64, 16384, 11, 0),  # word kernel grouped by XCD (the n = 2^20 code), frames not a multiple of 8
    (4, 32, 16384, 8, 0),    # grouped by XCD, exactly 8 workgroups per frame
    (3, 8, 96, 130, 0),      # Z = 3 x 32, not a power of two: 3 words per block
    (5, 32, 1024, 130, 1),   # buffers not 4-byte aligned: bit kernel with the frame in LDS
    (5, 32, 1024, 5, 1),     # the same with few frames: row-parallel bit kernel
    (3, 7, 45, 200, 0),      # odd Z with many frames: bit kernel with LDS
])
def test_syndrome_encoder_matches_generator(B, mb, nb, z, frames, misalign):
    import torch
    base = I.make_base(mb, nb, z, 3, 11)
    code = I.Code(base, z)
    rng = np.random.default_rng(12 + frames)
    x = rng.integers(0, 2, size=(frames, code.n), dtype=np.uint8)
    ref = I.pack_bits(I.syndrome_bits(code, x))
    gc = B.Code(base, z)
    _say(f"[gpu syndrome] n={code.n} frames={frames} misalign={misalign}")
    bb, sb = (code.n + 7) // 8, (code.m + 7) // 8
    xflat = torch.zeros(misalign + frames * bb, dtype=torch.uint8, device="cuda")
    xb = xflat[misalign:].view(frames, bb)
    xb.copy_(torch.from_numpy(I.pack_bits(x)))
    oflat = torch.zeros(misalign + frames * sb, dtype=torch.uint8, device="cuda")
    out = oflat[misalign:].view(frames, sb)
    B.ldpc_syndrome_batch(gc, xb, frames, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref)
    assert int(oflat[:misalign].sum()) == 0


def _full_size(B, wl_name, sample, seed=10107):
    wl = I.WORKLOADS[wl_name]
    code = wl.code()
    fr = I.make_frames(code, wl.frames, wl.qber, seed, n_short=int(wl.short_frac * code.n))
    gc = B.Code(code.base, code.z, acc_bits=wl.acc_bits)
    _say(f"[gpu parity full] {wl_name}: n={code.n} F={wl.frames} max_iter={wl.max_iter} {gc.plan()}")
    got = B.decode(gc, fr.syn, fr.llr, wl.max_iter, want_state=True)
    _say(f"[gpu parity full] {wl_name}: gpu done, conv={got['conv'].mean():.3f}")
    # every converged frame satisfies H x^ = s (H applied by the generator, not the decoder)
    xh = I.unpack_bits(got["bits"], code.n)
    s_ok = (I.pack_bits(I.syndrome_bits(code, xh)) == fr.syn).all(1)
    assert np.array_equal(s_ok, got["conv"].astype(bool))
    ref = O.decode(code.base, code.z, fr.syn[sample], fr.llr[sample], wl.max_iter, want_state=True,
                   acc_bits=wl.acc_bits)
    _compare(got, ref, frames=sample)
    return got


def test_parity_full_n32768_every_frame(B):
    # the headline batch in the launch configuration the benchmark times: every
    # one of its 256 frames against the oracle
    got = _full_size(B, "n32768_q2", sample=np.arange(I.WORKLOADS["n32768_q2"].frames))
    assert got["conv"].mean() > 0.9


def test_parity_full_n1048576_sampled(B):
    _full_size(B, "n1048576_q2", sample=np.array([0, 5, 9, 14, 17, 22, 27, 31]))


def test_parity_n1048576_shortened_early_stop(B):
    """The shortened n = 2^20 decode as the benchmark runs it: 16-bit soft values,
    the layer-synchronous family, the host stopping the launches once every frame
    has retired (check_every = 1); every frame against the oracle."""
    import torch
    wl = I.WORKLOADS["n1048576_q2"]
    code = wl.code()
    F = 6
    fr = I.make_frames(code, F, wl.qber, 10107, n_short=int(0.33 * code.n))
    gc = B.Code(code.base, code.z, acc_bits=wl.acc_bits)
    assert gc.plan()["kernel"] == "layer_sync"
    _say(f"[gpu parity] n1048576 shortened, check_every=1, F={F}")
    syn, llr = torch.from_numpy(fr.syn).cuda(), torch.from_numpy(fr.llr).cuda()
    bits = torch.zeros((F, (code.n + 7) // 8), dtype=torch.uint8, device="cuda")
    conv = torch.zeros(F, dtype=torch.uint8, device="cuda")
    iters = torch.full((F,), -1, dtype=torch.int32, device="cuda")
    B.ldpc_decode_batch_sched(gc, syn, llr, F, wl.max_iter, bits, conv, iters, check_every=1)
    torch.cuda.synchronize()
    ref = O.decode(code.base, code.z, fr.syn, fr.llr, wl.max_iter, acc_bits=wl.acc_bits)
    assert ref["conv"].all() and ref["iters"].max() < wl.max_iter
    assert np.array_equal(bits.cpu().numpy(), ref["bits"])
    assert np.array_equal(conv.cpu().numpy(), ref["conv"])
    assert np.array_equal(iters.cpu().numpy(), ref["iters"])


@pytest.mark.parametrize("kernel", ["split_reg", "split", "pairs", "global", "layer_sync"])
@pytest.mark.parametrize("mode", ["saturated", "zero", "small"])
def test_degenerate_channel_values(B, mode, kernel):
    """Soft inputs at the edges of the method: every |E| = E_max from the start
    (Alg. 2 freezes every variable, so the state never moves), all zero (every
    sign is +, every check-node input magnitude 0), and all of magnitude 1 (the
    check node's small-value branch of Alg. 1 everywhere)."""
    code = I.Code(I.make_base(5, 32, 64), 64)
    fr = I.make_frames(code, 8, 0.03, 4242)
    sign = np.where(fr.llr < 0, -1, 1).astype(np.int16)
    llr = {"saturated": 127 * sign, "zero": 0 * sign, "small": 3 * sign}[mode].astype(np.int8)
    gc = B.Code(code.base, code.z, kernel=kernel)
    _say(f"[gpu parity] degenerate {mode} on {gc.plan()}")
    got = B.decode(gc, fr.syn, llr, 20, want_state=True)
    ref = O.decode(code.base, code.z, fr.syn, llr, 20, want_state=True)
    _compare(got, ref)
    if mode == "saturated":
        assert np.array_equal(ref["E"], llr.astype(np.int16)), "frozen state moved"
