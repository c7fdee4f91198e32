"""Pins of the oracle's check node against what the paper fixes.

* tau (Alg. 1) against the exact box-plus table it stands for (Sec. 3.2: the
  integer representation of beta((p + 1/2) Delta, (q + 1/2) Delta), Eq. 6).
* tau's closed-form properties (commutative, monotone, within two steps below
  the minimum, equal to the minimum far from it).
* the degree-d fold (Eq. 4 / Eq. 7) against closed forms: min-sum where tau is
  exactly min, identity at degree 2, a single tau at degree 3.
* FP64: Eqs. 2, 3 and 7 agree ("mathematically there is no difference", Sec. 2),
  and the stable form of Eq. 6 equals its tanh statement.
"""
import math
import random

import numpy as np
import pytest

import oracle as O

DELTA = 5.0 / 16.0


def _beta_exact(a, b):
    # Eq. 6 written out
    return 2.0 * math.atanh(math.tanh(a / 2.0) * math.tanh(b / 2.0))


def test_tau_matches_exact_boxplus_table_at_delta_5_16():
    """Floor (bin-index) representation of beta at bin midpoints; Alg. 1 agrees
    with it everywhere on 6-bit inputs except at (2, 2) and (2, 6)."""
    mism = set()
    for p in range(64):
        for q in range(64):
            exact = math.floor(_beta_exact((p + 0.5) * DELTA, (q + 0.5) * DELTA) / DELTA)
            if exact != O.tau(p, q):
                mism.add((p, q, O.tau(p, q), exact))
    assert mism == {(2, 2, 1, 0), (2, 6, 2, 1), (6, 2, 2, 1)}


def test_tau_table_is_far_from_exact_at_other_steps():
    """The fit above is specific: a coarser or finer step disagrees widely."""
    for delta, at_least in ((0.25, 300), (0.5, 300)):
        bad = 0
        for p in range(64):
            for q in range(64):
                exact = math.floor(_beta_exact((p + 0.5) * delta, (q + 0.5) * delta) / delta)
                bad += exact != O.tau(p, q)
        assert bad >= at_least


def test_tau_closed_form_properties():
    t = O.tau_table(64)
    assert np.array_equal(t, t.T)                              # commutative
    assert np.all(np.diff(t, axis=0) >= 0)                     # monotone in p
    assert np.all(np.diff(t, axis=1) >= 0)                     # monotone in q
    p, q = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")
    mn = np.minimum(p, q)
    assert np.all(t <= mn)
    assert np.all(t >= np.maximum(mn - 2, 0))
    far = (mn > 2) & (np.abs(p - q) >= 6)
    assert np.array_equal(t[far], mn[far])                     # exact min far from the minimum
    assert np.all(t[0, :] == 0)
    assert O.tau(63, 63) == 61


def test_tau_clips_inputs_to_msg_max():
    for p in range(0, 128, 3):
        for q in range(0, 128, 5):
            assert O.tau(p, q, 63) == O.tau(min(p, 63), min(q, 63), 63)


def test_tau_is_not_associative():
    """Why the fold order must be fixed: tau(tau(a, b), c) != tau(a, tau(b, c))
    for some triples."""
    t = O.tau_table(64)
    a, b, c = np.meshgrid(np.arange(64), np.arange(64), np.arange(64), indexing="ij")
    left = t[t[a, b], c]
    right = t[a, t[b, c]]
    assert int((left != right).sum()) == 3448


@pytest.mark.parametrize("rule", [O.RULE_RCBP_FB, O.RULE_RCBP_EQ7])
def test_fold_equals_minsum_when_operands_are_far_apart(rule):
    rng = random.Random(5)
    for _ in range(200):
        d = rng.randint(2, 20)
        start = rng.randint(3, 8)
        vals = [start + 6 * i + rng.randint(0, 2) for i in range(d)]
        vals = [min(v, 63) for v in vals]
        # keep pairwise gaps >= 6 after the clip
        if len(set(vals)) != d or any(abs(a - b) < 6 for i, a in enumerate(vals) for b in vals[i + 1:]):
            continue
        rng.shuffle(vals)
        mag = O.cn_magnitudes(vals, rule)
        expect = [min(vals[:k] + vals[k + 1:]) for k in range(d)]
        assert list(mag) == expect


@pytest.mark.parametrize("rule", [O.RULE_RCBP_FB, O.RULE_RCBP_EQ7, O.RULE_MINSUM])
def test_fold_degree_two_passes_the_other_operand(rule):
    for a in range(0, 64, 7):
        for b in range(0, 64, 5):
            assert list(O.cn_magnitudes([a, b], rule)) == [b, a]


@pytest.mark.parametrize("rule", [O.RULE_RCBP_FB, O.RULE_RCBP_EQ7])
def test_fold_degree_three_is_one_tau(rule):
    rng = random.Random(7)
    for _ in range(500):
        p = [rng.randint(0, 63) for _ in range(3)]
        mag = O.cn_magnitudes(p, rule)
        assert mag[0] == O.tau(p[1], p[2])
        assert mag[1] == O.tau(p[0], p[2])
        assert mag[2] == O.tau(p[0], p[1])


def test_forward_backward_and_literal_eq7_orders_differ_somewhere():
    """The two fold orders give different integers on some rows (tau is not
    associative), so the decoder's choice is visible."""
    rng = random.Random(11)
    found = False
    for _ in range(20000):
        p = [rng.randint(0, 12) for _ in range(5)]
        if list(O.cn_magnitudes(p, O.RULE_RCBP_FB)) != list(O.cn_magnitudes(p, O.RULE_RCBP_EQ7)):
            found = True
            break
    assert found
    # the first output is the same right fold under both orders
    for _ in range(300):
        p = [rng.randint(0, 63) for _ in range(rng.randint(2, 20))]
        assert O.cn_magnitudes(p, O.RULE_RCBP_FB)[0] == O.cn_magnitudes(p, O.RULE_RCBP_EQ7)[0]


def test_minsum_rule_is_min_of_others():
    rng = random.Random(3)
    for _ in range(200):
        p = [rng.randint(0, 63) for _ in range(rng.randint(2, 20))]
        assert list(O.cn_magnitudes(p, O.RULE_MINSUM)) == [min(p[:k] + p[k + 1:]) for k in range(len(p))]


def test_fp64_beta_stable_form_equals_eq6():
    rng = random.Random(1)
    for _ in range(1000):
        a, b = rng.uniform(0, 12), rng.uniform(0, 12)
        assert O.beta(a, b) == pytest.approx(_beta_exact(a, b), rel=1e-10, abs=1e-12)
    assert O.beta(0.0, 5.0) == 0.0
    assert O.beta(40.0, 3.0) == pytest.approx(3.0, rel=1e-12)


def test_fp64_eq2_eq3_eq7_agree():
    rng = random.Random(2)
    for _ in range(300):
        d = rng.randint(2, 20)
        a = [rng.uniform(0.2, 8.0) * rng.choice((-1, 1)) for _ in range(d)]
        for k in range(d):
            t, p, f = O.mag_tanh(a, k), O.mag_phi(a, k), O.mag_fold(a, k)
            assert p == pytest.approx(t, rel=1e-9)
            assert f == pytest.approx(t, rel=1e-9)
