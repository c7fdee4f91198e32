"""Every kernel family forced on the same codes (ldpc_params.kernel_hint) gives
the oracle's results bit for bit, and the schedule autotuner picks among
candidates that all agree."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1903_10107_amd import inputs as I

pytestmark = pytest.mark.gpu

FAMILIES = ("global", "lds", "pairs", "split", "split_global_l", "layer_sync", "split_reg")


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


# (mb, nb, z, frames, qber, shortened fraction, column weight): the split
# kernel's slot variants (min, max row degree) are (19, 20), (2, 20), (6, 8),
# (2, 8) and (6, 6).
CODES = {
    "n1024": (5, 32, 32, 24, 0.02, 0.0, 3),
    "n32768_short": (5, 32, 1024, 4, 0.02, 0.33, 3),
    "n6144_deg6": (12, 24, 256, 6, 0.04, 0.1, 3),
    "n16384_mb4_deg6": (4, 8, 2048, 4, 0.03, 0.0, 3),
    "n6144_mb3_deg6": (3, 6, 1024, 4, 0.03, 0.0, 3),
    "n3840_deg10_w2": (3, 15, 256, 6, 0.03, 0.0, 2),
    "n2048_deg4_w2": (4, 8, 256, 6, 0.05, 0.0, 2),
    "n18432_deg6to7": (4, 9, 2048, 4, 0.03, 0.0, 3),
}


@pytest.mark.parametrize("family", FAMILIES)
@pytest.mark.parametrize("name", list(CODES))
def test_forced_family_matches_oracle(B, name, family):
    mb, nb, z, F, q, short, cw = CODES[name]
    code = I.Code(I.make_base(mb, nb, z, cw), z)
    fr = I.make_frames(code, F, q, 1234 + z, n_short=int(short * code.n))
    try:
        gc = B.Code(code.base, z, kernel=family)
    except B.LdpcError as e:
        assert e.code == B.LDPC_EUNSUPPORTED
        pytest.skip(f"{family} does not apply to {name}: {e}")
    assert gc.plan()["kernel"] == family
    _say(f"[gpu family] {name} {family} {gc.plan()}")
    got = B.decode(gc, fr.syn, fr.llr, 40, want_state=True)
    ref = O.decode(code.base, z, fr.syn, fr.llr, 40, want_state=True)
    for k in ("bits", "conv", "iters", "L", "E"):
        assert np.array_equal(got[k], ref[k]), (name, family, k)


@pytest.mark.parametrize("family", FAMILIES)
@pytest.mark.parametrize("name", ["n1024", "n6144_deg6", "n3840_deg10_w2", "n2048_deg4_w2"])
def test_offset_tables_on_every_family(B, name, family):
    """Per-iteration offsets (signed, fewer rows than iterations) on every kernel
    family that applies to the code."""
    mb, nb, z, F, q, short, cw = CODES[name]
    code = I.Code(I.make_base(mb, nb, z, cw), z)
    fr = I.make_frames(code, F, q, 4321 + z, n_short=int(short * code.n))
    off = np.random.default_rng(z).integers(-3, 8, size=(4, code.n_blocks)).astype(np.int8)
    try:
        B.Code(code.base, z, kernel=family, cn_rule=2)
    except B.LdpcError as e:
        assert e.code == B.LDPC_EUNSUPPORTED
        pytest.skip(f"{family} does not apply to {name}: {e}")
    gc = B.Code(code.base, z, kernel=family, cn_rule=2, offsets=off)   # offsets narrow no family
    assert gc.plan()["kernel"] == family
    _say(f"[gpu family offsets] {name} {family} {gc.plan()}")
    got = B.decode(gc, fr.syn, fr.llr, 40, want_state=True)
    ref = O.decode(code.base, z, fr.syn, fr.llr, 40, want_state=True, cn_rule=O.RULE_MINSUM, offsets=off)
    for k in ("bits", "conv", "iters", "L", "E"):
        assert np.array_equal(got[k], ref[k]), (name, family, k)


def test_global_family_applies_to_every_code(B):
    for name, (mb, nb, z, *_rest, cw) in CODES.items():
        assert B.Code(I.make_base(mb, nb, z, cw), z, kernel="global").plan()["kernel"] == "global"


def test_tuner_picks_an_agreeing_schedule(B, tmp_path):
    from paper_1903_10107_amd import tune
    code = I.Code(I.make_base(5, 32, 1024), 1024)
    F = 48
    qber = np.where(np.arange(F) % 3 == 0, 0.03, 0.015)
    fr = I.make_frames(code, F, qber, 99, n_short=int(0.33 * code.n))
    cache = str(tmp_path / "tune.json")
    _say("[gpu tune] n32768 F=48")
    res = tune.tune(code.base, code.z, fr.syn, fr.llr, 50, difficulty=qber, cache_path=cache, reps=2)
    kinds = {c["schedule"]["kernel"] for c in res["candidates"]}
    assert {"split", "pairs", "global"} <= kinds
    assert any(c["schedule"]["persistent_workgroups"] for c in res["candidates"])
    assert any(c["schedule"]["order"] == "hardest_first" for c in res["candidates"])
    assert res["ms"] == min(c["ms"] for c in res["candidates"])
    again = tune.tune(code.base, code.z, fr.syn, fr.llr, 50, difficulty=qber, cache_path=cache)
    assert again["schedule"] == res["schedule"]
    best = tune.Runner(code.base, code.z, fr.syn, fr.llr, 50, tune.Schedule(**res["schedule"]), qber)
    best()
    bits, conv, iters = best.outputs()
    ref = O.decode(code.base, code.z, fr.syn, fr.llr, 50)
    assert np.array_equal(bits, ref["bits"]) and np.array_equal(conv, ref["conv"])
    assert np.array_equal(iters, ref["iters"])
