"""The seeded input generator: code shapes, syndrome = H x for an
independently written H, LLR quantization, rate-adaptation positions."""
import numpy as np
import pytest

from paper_1903_10107_amd import inputs as I
from tests.dense_h import dense_h, gf2_matvec


def test_base_is_regular_balanced_and_girth_6():
    for mb, nb, z in ((5, 32, 32), (5, 32, 1024), (10, 64, 16384), (24, 48, 2048)):
        b = I.make_base(mb, nb, z)
        assert b.shape == (mb, nb) and b.dtype == np.int32
        assert ((b >= 0).sum(0) == 3).all()
        rw = (b >= 0).sum(1)
        assert rw.max() - rw.min() <= 1
        assert b.max() < z and b.min() >= -1
        assert not I.has_4cycle(b, z)
        assert np.array_equal(b, I.make_base(mb, nb, z))            # seeded


def test_4cycle_detector_finds_a_planted_cycle():
    b = np.array([[0, 1, -1], [2, 3, 0]], dtype=np.int32)
    assert I.has_4cycle(b, 8)          # 0 - 2 == 1 - 3 (mod 8)
    b[1, 1] = 4
    assert not I.has_4cycle(b, 8)


def test_syndrome_matches_dense_h():
    code = I.Code(I.make_base(5, 32, 32), 32)
    fr = I.make_frames(code, 6, 0.05, 1)
    H = dense_h(code.base, code.z)
    assert np.array_equal(gf2_matvec(H, fr.x), I.unpack_bits(fr.syn, code.m))


def test_llr_quantization_steps():
    assert [I.quantize_llr_mag(q) for q in (0.01, 0.02, 0.04, 0.06, 0.08)] == [14, 12, 10, 8, 7]
    code = I.Code(I.make_base(5, 32, 32), 32)
    fr = I.make_frames(code, 4, 0.02, 2)
    assert set(np.unique(fr.llr)) <= {12, -12}
    assert np.array_equal(fr.llr < 0, fr.y == 1)


def test_bit_packing_is_lsb_first():
    bits = np.zeros((1, 16), np.uint8)
    bits[0, 0] = 1
    bits[0, 9] = 1
    assert list(I.pack_bits(bits)[0]) == [1, 2]
    assert np.array_equal(I.unpack_bits(I.pack_bits(bits), 16), bits)


def test_shortened_and_punctured_positions():
    code = I.Code(I.make_base(5, 32, 32), 32)
    fr = I.make_frames(code, 3, 0.04, 3, n_short=100, n_punct=50)
    order = I.position_order(code)
    assert sorted(order.tolist()) == list(range(code.n))
    pun, sh = order[:50], order[50:150]
    assert (fr.llr[:, pun] == 0).all()
    assert np.array_equal(fr.llr[:, sh], np.where(fr.x[:, sh] == 0, 127, -127))
    assert (fr.key_bits() == code.n - 150).all()
    assert (~fr.key_mask[:, sh]).all() and fr.key_mask.sum(1).tolist() == [code.n - 150] * 3


def test_frame_f_does_not_depend_on_batch_size():
    code = I.Code(I.make_base(5, 32, 32), 32)
    a = I.make_frames(code, 5, 0.03, 9)
    b = I.make_frames(code, 2, 0.03, 9, frame_offset=3)
    assert np.array_equal(a.llr[3:], b.llr) and np.array_equal(a.syn[3:], b.syn)


def test_per_frame_qber_and_fixed_weight():
    code = I.Code(I.make_base(5, 32, 32), 32)
    fr = I.make_frames(code, 4, [0.01, 0.02, 0.04, 0.08], 4, fixed_weight=True)
    assert [(fr.x[f] ^ fr.y[f]).sum() for f in range(4)] == [10, 20, 41, 82]


def test_adapt_rate_equals_generating_with_that_split():
    code = I.Code(I.make_base(5, 32, 32), 32)
    qv = np.array([0.01, 0.02, 0.04, 0.06, 0.08, 0.02])
    pv = np.array([100, 0, 40, 0, 0, 100])
    sv = np.array([0, 60, 10, 0, 200, 0])
    ref = I.make_frames(code, 6, qv, 17, n_short=sv, n_punct=pv)
    got = I.adapt_rate(I.make_frames(code, 6, qv, 17), pv, sv)
    for k in ("x", "y", "syn", "llr", "llr_f", "n_punct", "n_short", "key_mask"):
        assert np.array_equal(getattr(got, k), getattr(ref, k)), k
    with pytest.raises(ValueError):
        I.adapt_rate(ref, 0, 0)


def test_ragged_frames_use_the_bucket_points():
    code = I.Code(I.make_base(24, 48, 64), 64)
    pts = {0.01: (900, 0), 0.04: (300, 0), 0.08: (0, 40)}
    fr = I.make_ragged_frames(code, 40, 3, pts)
    assert set(np.unique(fr.qber)) == set(pts)
    for f in range(fr.n_frames):
        assert (fr.n_punct[f], fr.n_short[f]) == pts[float(fr.qber[f])]
        assert (fr.llr[f] == 0).sum() >= fr.n_punct[f]
    small = I.make_ragged_frames(code, 10, 3, pts)
    assert np.array_equal(small.qber, fr.qber[:10]) and np.array_equal(small.llr, fr.llr[:10])


def test_learned_offsets_quantize_to_the_llr_step():
    from paper_1903_10107_amd import learn
    d = I.DELTA
    beta = np.array([[0.0, 0.49 * d, 0.51 * d, 1.5 * d + 1e-9, 100.0, -0.3]])
    assert learn.int_offsets(beta).tolist() == [[0, 0, 1, 2, 63, 0]]
    assert learn.int_offsets(beta, msg_max=31)[0, 4] == 31


def test_committed_traffic_summary_is_readable():
    """The headline workload's rocprofv3 counter summary carries the two fields
    the benchmark reads (the source hash it was taken on and the HBM bytes per
    launch); roofline.traffic is null whenever they are missing or stale."""
    import bench
    kv = bench.traffic_summary("n32768_q2")
    assert len(kv.get("kernel_source_sha256", "")) == 16
    assert float(kv["hbm_bytes_per_dispatch"]) > 0
