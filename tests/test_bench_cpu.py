"""bench.py's own arithmetic and bookkeeping, without a GPU: the algorithmic
operation count behind the ALU roofline, and that the committed headline
profiles were taken on the kernel sources of this tree (bench.py reports the
measured HBM traffic only then)."""
import os
import re

import bench


def test_algorithmic_ops_match_a_hand_count():
    # z = 1, rows of degree 3 and 4: 7 edges x 14 ops, 3 x ((3-2) + (4-2)) Alg. 1
    # evaluations x 9 ops, over 2 frame-iterations
    assert bench.algorithmic_int_ops((1, [3, 4]), 2) == 2 * (14 * 7 + 27 * (1 + 2))
    # scales with the lift and with the iterations
    assert bench.algorithmic_int_ops((8, [3, 4]), 5) == 8 * 5 / 2 * bench.algorithmic_int_ops((1, [3, 4]), 2)


def test_ops_per_edge_iteration_of_the_five_row_code():
    # rows of 19, 19, 19, 19 and 20 edges: 38.19 operations per edge-iteration
    degs = [19, 19, 19, 19, 20]
    per_edge = bench.algorithmic_int_ops((1, degs), 1) / sum(degs)
    assert abs(per_edge - 38.1875) < 1e-9


def _sha_in(path):
    m = re.search(r"kernel_source_sha256: ([0-9a-f]+)", open(path).read())
    return m.group(1) if m else None


def test_committed_headline_profiles_match_the_kernel_sources():
    h = bench.kernel_source_hash()
    for name in ("decode_n32768_q2_traffic.txt", "decode_n32768_q2_kernel_trace.txt"):
        assert _sha_in(os.path.join(bench.PROFILES, name)) == h, (name, h)
    kv = bench.traffic_summary("n32768_q2")
    # at least the frame I/O (LLRs, syndromes, packed bits) of a 256-frame launch
    assert float(kv["hbm_bytes_per_dispatch"]) >= 256 * (32768 + 640 + 4096)
    assert bench.measured_traffic("n32768_q2") == float(kv["hbm_bytes_per_dispatch"])
