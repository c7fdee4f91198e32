"""The register-resident family (split_reg) on frame lengths that take its
general stage-in and stage-out paths: n not a multiple of 16 (the LLRs are not
read as 16-byte chunks), not a multiple of 8 (hard decisions by wavefront
ballots instead of one output byte per thread), and more 16-byte LLR chunks than
two per thread. Each is compared with the oracle bit for bit (hard decisions,
convergence flags, iteration counts, final messages and soft values)."""
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


def five_row_base(nb: int, z: int, seed: int) -> np.ndarray:
    """5 x nb base with rows of 19 or 20 nonzero blocks (every column covered),
    random circulant shifts."""
    rng = np.random.default_rng(seed)
    while True:
        base = np.full((5, nb), -1, dtype=np.int32)
        for b in range(5):
            deg = int(rng.integers(19, 21))
            cols = rng.choice(nb, size=deg, replace=False)
            base[b, cols] = rng.integers(0, z, size=deg)
        if ((base >= 0).sum(axis=0) > 0).all():
            return base


# (nb, z, qber, shortened fraction): n = nb * z
CASES = {
    "n42": (21, 2, 0.03, 0.25),          # n % 8 == 2: both general paths
    "n84": (21, 4, 0.03, 0.25),          # n % 16 == 4, n % 8 == 4
    "n40": (20, 2, 0.03, 0.25),          # n % 16 == 8: general stage-in, byte stage-out
    "n20480": (40, 512, 0.01, 0.35),     # 1280 LLR chunks for 512 threads
}


@pytest.mark.parametrize("name", list(CASES))
def test_split_reg_general_stage_paths_match_oracle(B, name):
    nb, z, q, short = CASES[name]
    base = five_row_base(nb, z, 100 + nb * z)
    code = I.Code(base, z)
    gc = B.Code(base, z, kernel="split_reg")
    assert gc.plan()["kernel"] == "split_reg"
    fr = I.make_frames(code, 6, q, 777 + z, n_short=int(short * code.n))
    _say(f"[gpu split_reg lengths] {name} n={code.n} plan={gc.plan()}")
    got = B.decode(gc, fr.syn, fr.llr, 30, want_state=True)
    ref = O.decode(base, z, fr.syn, fr.llr, 30, want_state=True)
    for k in ("bits", "conv", "iters", "L", "E"):
        assert np.array_equal(got[k], ref[k]), (name, k)
