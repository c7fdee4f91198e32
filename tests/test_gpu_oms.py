"""Differentiable FP32 offset min-sum on the GPU against the FP64 oracle
(oracle/oms.py) and the integer oracle, through the C ABI.

FP32 against FP64: with LLRs on a 1/64 grid and offsets on odd multiples of
1/128 every soft value and message is a small multiple of 1/128, exact in both
precisions, so the soft values after every iteration agree exactly and so does
every min/argmin/clamp decision; the loss (softplus) and the gradients
(sigmoid, products, sums) differ by rounding only: relative 1e-4 for the loss,
1e-3 of the largest component for the gradients. With integer LLRs and integer
offsets the soft values also equal the integer min-sum oracle's bit for bit.
"""
import sys

import numpy as np
import pytest

import oracle as O
from oracle import oms
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


def _gpu_loss_grad(B, base, z, fr, llr, beta, weights, dloss, T):
    import torch
    dec = B.OmsDecoder(base, z, T, weights)
    syn = torch.from_numpy(fr.syn).cuda()
    xb = torch.from_numpy(I.pack_bits(fr.x)).cuda()
    bt = torch.tensor(beta, dtype=torch.float32, device="cuda", requires_grad=True)
    ll = torch.tensor(llr, dtype=torch.float32, device="cuda", requires_grad=True)
    loss, E = dec.loss(syn, ll, xb, bt, want_E=True)
    (loss * torch.tensor(dloss, dtype=torch.float32, device="cuda")).sum().backward()
    torch.cuda.synchronize()
    return loss.detach().cpu().numpy(), E.cpu().numpy(), bt.grad.cpu().numpy(), ll.grad.cpu().numpy()


def _case(mb, nb, z, cw, F, q, T, seed, dyadic=True):
    """Frames with noisy LLRs and random offsets. dyadic: LLRs on a 1/64 grid and
    offsets on odd multiples of 1/128, so every soft value and message is a small
    multiple of 1/128, exact in FP32 and FP64 alike: the forward passes then agree
    exactly and so do all min/argmin/clamp decisions."""
    code = I.Code(I.make_base(mb, nb, z, cw), z)
    fr = I.make_frames(code, F, q, seed, n_punct=code.n // 20)
    rng = np.random.default_rng(seed)
    llr = fr.llr_f + rng.normal(0, 0.25, size=fr.llr_f.shape) * (fr.llr_f != 0)
    beta = rng.uniform(0.0, 0.5, size=(T, code.n_blocks))
    if dyadic:
        llr = np.round(llr * 64) / 64
        beta = (2 * np.floor(beta * 64) + 1) / 128
    weights = rng.uniform(0.5, 1.5, size=T)
    dloss = rng.uniform(0.5, 1.5, size=F)
    return code, fr, llr, beta, weights, dloss


@pytest.mark.parametrize("shape", [(5, 32, 32, 3), (5, 32, 1024, 3), (5, 32, 512, 3), (8, 16, 64, 2),
                                   (2, 24, 64, 2), (3, 7, 45, 2)],
                         ids=["n1024_dmax20_lds", "n32768_global_state", "n16384_fwd_lds_bwd_global", "n1024_dmax8",
                              "n1536_deg24_dmax32", "n315_odd_n_dmax8"])
def test_forward_and_gradients_match_fp64(B, shape):
    mb, nb, z, cw = shape
    F, T = (2, 3) if z >= 512 else (6, 5)
    code, fr, llr, beta, weights, dloss = _case(mb, nb, z, cw, F, 0.04, T, 11 + z)
    _say(f"[gpu oms] n={code.n} F={F} T={T}")
    loss, E, db, dl = _gpu_loss_grad(B, code.base, z, fr, llr, beta, weights, dloss, T)
    syn = oms.unpack_syndrome(fr.syn, code.m)
    ref = oms.oms_grad(code.base, z, syn, llr.astype(np.float32).astype(np.float64),
                       beta.astype(np.float32).astype(np.float64), fr.x, weights.astype(np.float32), dloss.astype(np.float32))
    _, Eref, _ = oms.oms_forward(code.base, z, syn, llr.astype(np.float32).astype(np.float64),
                                 beta.astype(np.float32).astype(np.float64), fr.x, weights.astype(np.float32))
    Eref = Eref.numpy()
    assert np.array_equal(E, Eref.astype(np.float32)), "dyadic inputs: the forward pass is exact"
    assert np.allclose(loss, ref["loss"], rtol=1e-4, atol=1e-6)
    assert np.allclose(db, ref["dbeta"], rtol=1e-3, atol=1e-3 * np.abs(ref["dbeta"]).max())
    assert np.allclose(dl, ref["dllr"], rtol=1e-3, atol=1e-3 * np.abs(ref["dllr"]).max())


def test_integer_inputs_match_integer_minsum_exactly(B):
    import torch
    code = I.Code(I.make_base(5, 32, 32), 32)
    fr = I.make_frames(code, 6, 0.12, 5)
    rng = np.random.default_rng(3)
    llr = np.where(fr.y == 0, 3, -3).astype(np.int8)
    llr[:, rng.random(code.n) < 0.1] = 0
    T = 3
    off = rng.integers(0, 2, size=(T, code.n_blocks)).astype(np.int8)
    ref = O.decode(code.base, code.z, fr.syn, llr, T, cn_rule=O.RULE_MINSUM, offsets=off, acc_bits=16,
                   msg_max=127, e_max=32767, want_state=True)
    assert (ref["conv"] == 0).all()
    dec = B.OmsDecoder(code.base, code.z, T)
    _, E = dec.loss(torch.from_numpy(fr.syn).cuda(), torch.tensor(llr, dtype=torch.float32, device="cuda"),
                    torch.from_numpy(I.pack_bits(fr.x)).cuda(),
                    torch.tensor(off, dtype=torch.float32, device="cuda"), want_E=True)
    assert np.array_equal(E.cpu().numpy(), ref["E"].astype(np.float32))


def test_gpu_gradient_matches_central_differences(B):
    """The GPU backward pass against central differences of the forward pass,
    taken on the FP64 forward (free of the FP32 rounding noise of the loss sum)
    at generic inputs: off the dyadic grid no minimum sits exactly at its offset,
    where a central difference would average the two one-sided slopes."""
    code, fr, llr, beta, weights, dloss = _case(5, 32, 32, 3, 4, 0.04, 4, 77, dyadic=False)
    _, _, db, dl = _gpu_loss_grad(B, code.base, code.z, fr, llr, beta, weights, dloss, 4)
    syn = oms.unpack_syndrome(fr.syn, code.m)
    w32, g32 = weights.astype(np.float32).astype(np.float64), dloss.astype(np.float32).astype(np.float64)

    def f(bt, ll):
        loss, _, _ = oms.oms_forward(code.base, code.z, syn, ll, bt, fr.x, w32)
        return float((loss.numpy() * g32).sum())

    h = 1e-6
    rng = np.random.default_rng(0)
    picks = list(np.argsort(-np.abs(db).ravel())[:6]) + list(rng.integers(0, db.size, 4))
    for idx in picks:
        t, e = np.unravel_index(idx, db.shape)
        bp, bm = beta.copy(), beta.copy()
        bp[t, e] += h
        bm[t, e] -= h
        fd = (f(bp, llr) - f(bm, llr)) / (2 * h)
        assert fd == pytest.approx(db[t, e], rel=1e-3, abs=1e-4 * np.abs(db).max())
    for (fi, j) in [(0, 3), (1, 500), (3, 1000)]:
        lp, lm = llr.copy(), llr.copy()
        lp[fi, j] += h
        lm[fi, j] -= h
        fd = (f(beta, lp) - f(beta, lm)) / (2 * h)
        assert fd == pytest.approx(dl[fi, j], rel=1e-3, abs=1e-4 * np.abs(dl).max())


def test_backward_is_deterministic_and_zero_frames_give_zero(B):
    import torch
    code, fr, llr, beta, weights, dloss = _case(5, 32, 32, 3, 8, 0.04, 3, 5)
    a = _gpu_loss_grad(B, code.base, code.z, fr, llr, beta, weights, dloss, 3)
    b = _gpu_loss_grad(B, code.base, code.z, fr, llr, beta, weights, dloss, 3)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    dec = B.OmsDecoder(code.base, code.z, 3)
    out = torch.full((3, code.n_blocks), 7.0, device="cuda")
    e8 = torch.empty(0, dtype=torch.uint8, device="cuda")
    B.ldpc_oms_backward(dec.code, e8, e8, 0, 3, torch.zeros((3, code.n_blocks), device="cuda"), None,
                        torch.empty(0, device="cuda"), e8, out, None, None)
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == 0).all()


def test_oms_argument_errors(B):
    import torch
    code = B.Code(I.make_base(5, 32, 32), 32)
    t = torch.empty(16, dtype=torch.uint8, device="cuda")
    lib = B.lib()
    assert lib.ldpc_oms_forward(code.handle, t.data_ptr(), t.data_ptr(), None, 1, 0, t.data_ptr(), None, None, None,
                                t.data_ptr(), 16, None, 0, None) == B.LDPC_EINVAL          # n_iter < 1
    assert lib.ldpc_oms_forward(code.handle, t.data_ptr(), t.data_ptr(), None, 1, 2, t.data_ptr(), None, None, None,
                                t.data_ptr(), 16, None, 0, None) == B.LDPC_EINVAL          # short tape
    assert b"tape" in lib.ldpc_last_error()
    # the tape's row records are read 16 bytes at a time: a misaligned tape is
    # refused before anything is launched
    assert lib.ldpc_oms_forward(code.handle, t.data_ptr(), t.data_ptr(), None, 1, 2, t.data_ptr(), None, None, None,
                                t.data_ptr() + 4, 1 << 30, None, 0, None) == B.LDPC_EINVAL  # misaligned tape
    assert b"aligned" in lib.ldpc_last_error()
    assert lib.ldpc_oms_forward(code.handle, t.data_ptr(), t.data_ptr(), None, 1, 2, None, None, None, None,
                                t.data_ptr(), 1 << 30, None, 0, None) == B.LDPC_EINVAL     # beta NULL
    assert lib.ldpc_oms_backward(code.handle, t.data_ptr(), None, 1, 2, t.data_ptr(), None, t.data_ptr(),
                                 t.data_ptr(), 1 << 30, t.data_ptr(), None, t.data_ptr(), 1 << 30,
                                 None) == B.LDPC_EINVAL                                      # target NULL


def test_full_training_configuration_sampled(B):
    """The training workload as the benchmark runs it (n = 8192, 5x32 base with
    Z = 256, 512 frames per launch, 20 iterations, 36% shortened, the integer
    decoder's LLR grid): frames 0 and 511 against the FP64 oracle. Only those
    two frames carry a loss weight, so the summed offset gradient is theirs.
    Without saturation the soft values of a converging frame grow by orders of
    magnitude over 20 iterations (frame 511 reaches about 6e6), past the range
    where FP32 holds every multiple of 1/128, so E is compared to a relative
    1e-6 (frame 0 stays small and matches exactly)."""
    from paper_1903_10107_amd import learn
    code = I.Code(I.make_base(5, 32, 256), 256)
    F, T = 512, 20
    fr = I.make_frames(code, F, 0.02, 4242, n_short=int(0.36 * code.n))
    llr = learn.training_llr(fr).astype(np.float64)           # integer LLRs x 5/16: exact in FP32
    rng = np.random.default_rng(9)
    beta = (2 * np.floor(rng.uniform(0.0, 0.6, size=(T, code.n_blocks)) * 64) + 1) / 128
    weights = np.linspace(0.5, 1.5, T)
    dloss = np.zeros(F)
    dloss[[0, F - 1]] = [1.0, 0.75]
    _say(f"[gpu oms] full training configuration n={code.n} F={F} T={T}")
    loss, E, db, dl = _gpu_loss_grad(B, code.base, code.z, fr, llr, beta, weights, dloss, T)
    sel = [0, F - 1]
    syn = oms.unpack_syndrome(fr.syn[sel], code.m)
    w32 = weights.astype(np.float32)
    ref = oms.oms_grad(code.base, code.z, syn, llr[sel], beta, fr.x[sel], w32, dloss[sel].astype(np.float32))
    _, Eref, _ = oms.oms_forward(code.base, code.z, syn, llr[sel], beta, fr.x[sel], w32)
    Eref = Eref.numpy()
    assert np.array_equal(E[0], Eref[0].astype(np.float32)), "small soft values: the forward pass is exact"
    assert np.allclose(E[sel], Eref, rtol=1e-6, atol=0)
    assert np.allclose(loss[sel], ref["loss"], rtol=1e-4, atol=1e-6)
    assert np.allclose(db, ref["dbeta"], rtol=1e-3, atol=1e-3 * np.abs(ref["dbeta"]).max())
    assert np.allclose(dl[sel], ref["dllr"], rtol=1e-3, atol=1e-3 * np.abs(ref["dllr"]).max())
    assert not np.any(dl[1:F - 1]), "frames without a loss weight get no gradient"
