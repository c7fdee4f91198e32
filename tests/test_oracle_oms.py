"""Pins of the FP64 offset min-sum oracle (oracle/oms.py), independent of its
own code:

* integer inputs and integer offsets: its forward pass equals the integer
  layered oracle with the min-sum rule and that offset table (16-bit soft
  values, message cap above every magnitude reached), frame by frame;
* offsets above every magnitude: all messages vanish, so E stays the channel
  LLRs and the loss has a closed form with zero offset gradient;
* one check row of degree 3, one iteration: loss and offset gradient written
  out by hand, also with two tied minima (the tie goes to the lower index);
* gradients equal FP64 central differences at generic (non-tied) points.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import oms
from paper_1903_10107_amd import inputs as I


def _frames(code, F, q, seed):
    fr = I.make_frames(code, F, q, seed)
    syn = oms.unpack_syndrome(fr.syn, code.m)
    return fr, syn


def test_forward_equals_integer_minsum_with_offsets():
    code = I.Code(I.make_base(5, 32, 32), 32)
    fr, syn = _frames(code, 6, 0.12, 5)
    rng = np.random.default_rng(3)
    llr = np.where(fr.y == 0, 3, -3).astype(np.int8)
    llr[:, rng.random(code.n) < 0.1] = 0                     # some punctured positions
    T = 3
    off = rng.integers(0, 2, size=(T, code.n_blocks)).astype(np.int8)
    ref = O.decode(code.base, code.z, fr.syn, llr, T, cn_rule=O.RULE_MINSUM, offsets=off, acc_bits=16,
                   msg_max=127, e_max=32767, want_state=True)
    assert (ref["conv"] == 0).all() and (ref["iters"] == T).all(), "frames must run all T iterations"
    assert np.abs(ref["L"]).max() < 127
    _, E, _ = oms.oms_forward(code.base, code.z, syn, llr.astype(np.float64), off.astype(np.float64), fr.x)
    assert np.array_equal(E.numpy(), ref["E"].astype(np.float64))


def test_offsets_above_every_magnitude_silence_the_check_nodes():
    code = I.Code(I.make_base(5, 32, 16), 16)
    fr, syn = _frames(code, 3, 0.05, 9)
    llr = fr.llr_f
    beta = np.full((4, code.n_blocks), 1e6)
    out = oms.oms_grad(code.base, code.z, syn, llr, beta, fr.x)
    y = 1.0 - 2.0 * fr.x
    sp = np.logaddexp(0.0, -y * llr)                          # softplus
    assert np.allclose(out["loss"], 4 * sp.sum(1) / code.n, rtol=1e-13, atol=0)
    assert np.abs(out["dbeta"]).max() == 0.0


def test_single_row_by_hand():
    # one layer, one row, three columns (Z = 1, shifts 0): v = llr
    base = np.array([[0, 0, 0]], dtype=np.int32)
    llr = np.array([[1.5, -0.4, 2.0]])
    x = np.array([[0, 1, 1]])
    syn = np.array([[1]])
    beta = np.array([[0.1, 0.25, 0.05]])
    out = oms.oms_grad(base, 1, syn, llr, beta, x)
    # by hand: sgn = (+, -, +); total sign = (-1)^1 * (-1) = +1; sigma_k = sgn(v_k)
    v = llr[0]
    sig = np.where(v < 0, -1.0, 1.0)
    a = np.abs(v)
    mex = [min(a[1], a[2]), min(a[0], a[2]), min(a[0], a[1])]
    L = [sig[k] * max(mex[k] - beta[0, k], 0.0) for k in range(3)]
    E = v + np.array(L)
    y = 1.0 - 2.0 * x[0]
    loss = sum(math.log1p(math.exp(-y[j] * E[j])) for j in range(3)) / 3
    assert out["loss"][0] == pytest.approx(loss, rel=1e-14)
    # d loss / d beta_k = dsoftplus(-y_k E_k) * (-y_k) * dE_k/dbeta_k / n, dE_k/dbeta_k = -sigma_k [mex_k > beta_k]
    dsp = [1.0 / (1.0 + math.exp(y[j] * E[j])) for j in range(3)]
    db = [dsp[k] * (-y[k]) * (-sig[k] * (mex[k] > beta[0, k])) / 3 for k in range(3)]
    assert np.allclose(out["dbeta"][0], db, rtol=1e-13, atol=1e-16)


def test_gradients_equal_central_differences():
    code = I.Code(I.make_base(5, 32, 8), 8)
    fr, syn = _frames(code, 2, 0.06, 21)
    rng = np.random.default_rng(8)
    llr = fr.llr_f + rng.normal(0, 0.3, size=fr.llr_f.shape)  # generic values, no ties
    T = 3
    beta = rng.uniform(0.0, 0.6, size=(T, code.n_blocks))
    w = np.array([0.5, 1.0, 2.0])
    g = np.array([1.0, -0.7])
    out = oms.oms_grad(code.base, code.z, syn, llr, beta, fr.x, w, g)

    def f(bt, ll):
        loss, _, _ = oms.oms_forward(code.base, code.z, syn, ll, bt, fr.x, w)
        return float((loss.numpy() * g).sum())

    h = 1e-6
    for (t, e) in [(0, 0), (1, 17), (2, 95), (0, 50), (2, 3)]:
        bp, bm = beta.copy(), beta.copy()
        bp[t, e] += h
        bm[t, e] -= h
        fd = (f(bp, llr) - f(bm, llr)) / (2 * h)
        assert fd == pytest.approx(out["dbeta"][t, e], rel=1e-6, abs=1e-9)
    for (fi, j) in [(0, 0), (1, 100), (0, 255)]:
        lp, lm = llr.copy(), llr.copy()
        lp[fi, j] += h
        lm[fi, j] -= h
        fd = (f(beta, lp) - f(beta, lm)) / (2 * h)
        assert fd == pytest.approx(out["dllr"][fi, j], rel=1e-6, abs=1e-9)


def test_tied_minima_send_the_gradient_to_the_lowest_edge():
    base = np.array([[0, 0, 0]], dtype=np.int32)
    llr = np.array([[1.0, -1.0, 2.0]])                       # |v| = 1, 1, 2: minima tied at edges 0, 1
    x = np.array([[0, 0, 0]])
    syn = np.array([[0]])
    beta = np.array([[0.25, 0.25, 0.25]])
    out = oms.oms_grad(base, 1, syn, llr, beta, x)
    # sign product (+)(-)(+) = -1; sigma_k = -sgn(v_k) = (-, +, -)
    # i1 = 0, i2 = 1: L_0 = -(|v_1| - b) = -0.75, L_1 = +(|v_0| - b) = 0.75, L_2 = -(|v_0| - b) = -0.75
    E = np.array([1.0 - 0.75, -1.0 + 0.75, 2.0 - 0.75])
    dsp = 1.0 / (1.0 + np.exp(E))                             # d softplus(-E)/d(-E), target bits 0
    dE = -dsp / 3                                             # d loss / d E_j
    # dE_k/dllr_j: identity, plus through the minima: L_0 reads |v_1|, L_1 and L_2 read |v_0|
    # dL_0/dv_1 = sigma_0 * sgn(v_1) = (-1)(-1) = 1; dL_1/dv_0 = (+1)(+1) = 1; dL_2/dv_0 = (-1)(+1) = -1
    dllr = dE.copy()
    dllr[1] += dE[0] * 1.0
    dllr[0] += dE[1] * 1.0 + dE[2] * -1.0
    assert np.allclose(out["dllr"][0], dllr, rtol=1e-13, atol=1e-16)
