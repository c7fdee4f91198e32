"""Where the decoders stop working (Sec. 3: the quantized decoder is meant to
keep the efficiency of the floating-point one). The FP64 BP oracle's frame error
rate on the rate-27/32 code (5x32 base, Z = 1024, column weight 3) turns from
near 0 to near 1 over a narrow QBER range, the waterfall; its 50% point lies
inside the belief-propagation threshold bracket that density evolution of the
code's degree distribution gives (computed here by population dynamics,
independently of both decoders), and the 8-bit integer decoder's 50% point lies
within 0.1% QBER of the floating-point one."""
import numpy as np
import pytest

import oracle as O
from paper_1903_10107_amd import inputs as I
from paper_1903_10107_amd import metrics as M


def de_converges(q: float, n: int = 20000, iters: int = 300, seed: int = 1) -> bool:
    """Population-dynamics density evolution of BP on a BSC(q) for the ensemble
    of the 5x32 base: variable nodes of degree 3, check nodes of degree 19 (on
    76 of every 96 edges) or 20 (all-zero word, messages as LLRs)."""
    rng = np.random.default_rng(seed)
    l0 = np.log((1 - q) / q)

    def channel(k):
        return np.where(rng.random(k) < q, -l0, l0)

    v = channel(n)
    for _ in range(iters):
        deg20 = rng.random(n) >= 76 / 96
        t = np.tanh(np.clip(v[rng.integers(0, n, size=(n, 19))], -40, 40) / 2)
        t[:, 18] = np.where(deg20, t[:, 18], 1.0)
        c = 2 * np.arctanh(np.clip(np.prod(t, axis=1), -1 + 1e-15, 1 - 1e-15))
        j = rng.integers(0, n, size=(n, 3))
        v = channel(n) + c[j[:, 0]] + c[j[:, 1]]
        post = v + c[j[:, 2]]
        if not (post < 0).any() and np.abs(post).mean() > 30:
            return True
    return False


def _fifty(qs, fer):
    """QBER where the frame error rate crosses 1/2 (linear between neighbours)."""
    for k in range(len(qs) - 1):
        if fer[k] <= 0.5 <= fer[k + 1] and fer[k + 1] > fer[k]:
            return qs[k] + (0.5 - fer[k]) * (qs[k + 1] - qs[k]) / (fer[k + 1] - fer[k])
    raise AssertionError(f"no 50% crossing in {list(zip(qs, fer))}")


def test_waterfall_sits_at_the_bp_threshold_and_integer_tracks_float():
    lo, hi = 0.0130, 0.0155
    assert de_converges(lo), "density evolution should converge below the threshold"
    assert not de_converges(hi), "density evolution should fail above the threshold"
    code = I.Code(I.make_base(5, 32, 1024), 1024)
    qs = [0.0125, 0.0135, 0.0145, 0.0155]
    fer_f, fer_i = [], []
    for q in qs:
        fr = I.make_frames(code, 48, q, 1313)
        fl = O.bp_fp64_decode(code.base, code.z, fr.syn, fr.llr_f, 50)
        it = O.decode(code.base, code.z, fr.syn, fr.llr, 50)
        ok_f, _ = M.frame_outcomes(fr.x, I.unpack_bits(fl["bits"], code.n), fl["conv"])
        ok_i, _ = M.frame_outcomes(fr.x, I.unpack_bits(it["bits"], code.n), it["conv"])
        fer_f.append(1 - ok_f.mean())
        fer_i.append(1 - ok_i.mean())
    assert fer_f[0] < 0.2 and fer_f[-1] > 0.8, fer_f
    q50_f, q50_i = _fifty(qs, fer_f), _fifty(qs, fer_i)
    # a finite-length waterfall sits at or a little below the asymptotic threshold
    assert lo - 0.001 <= q50_f <= hi, (q50_f, fer_f)
    assert abs(q50_i - q50_f) <= 0.001, (q50_i, q50_f, fer_i, fer_f)
