"""The C ABI from a plain C program (tests/c_client/decode_client.c: HIP runtime
for device memory, no Python or torch in the process): its decode equals the
oracle's bit for bit. The binary is built by build() beside its source."""
import os
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_1903_10107_amd import inputs as I

pytestmark = pytest.mark.gpu

CLIENT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_client", "decode_client")


@pytest.mark.parametrize("mb,nb,z,frames,q,short_frac,max_iter,acc_bits", [
    (5, 32, 32, 64, 0.01, 0.0, 50, 0),       # n = 1024, the paper's 8-bit decoder
    (5, 32, 1024, 16, 0.02, 0.33, 50, 0),    # n = 32768, shortened to its operating point
    (5, 32, 256, 8, 0.02, 0.2, 30, 16),      # 16-bit soft values
])
def test_c_client_decode_matches_oracle(tmp_path, mb, nb, z, frames, q, short_frac, max_iter, acc_bits):
    assert os.path.exists(CLIENT), f"{CLIENT} is not built; run build() from __graft_entry__"
    code = I.Code(I.make_base(mb, nb, z), z)
    fr = I.make_frames(code, frames, q, 31 + z, n_short=int(short_frac * code.n))
    src, dst = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(src, "wb") as f:
        f.write(np.array([mb, nb, z, frames, max_iter, acc_bits], dtype="<i4").tobytes())
        f.write(np.ascontiguousarray(code.base, dtype="<i4").tobytes())
        f.write(np.ascontiguousarray(fr.syn, dtype=np.uint8).tobytes())
        f.write(np.ascontiguousarray(fr.llr, dtype=np.int8).tobytes())
    print(f"[gpu c client] n={code.n} frames={frames} acc_bits={acc_bits}", flush=True)
    r = subprocess.run([CLIENT, str(src), str(dst)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    raw = np.fromfile(dst, dtype=np.uint8)
    bb = (code.n + 7) // 8
    bits = raw[:frames * bb].reshape(frames, bb)
    conv = raw[frames * bb:frames * bb + frames]
    iters = raw[frames * bb + frames:].view("<i4")
    ref = O.decode(code.base, code.z, fr.syn, fr.llr, max_iter, **({"acc_bits": 16} if acc_bits == 16 else {}))
    assert np.array_equal(bits, ref["bits"])
    assert np.array_equal(conv, ref["conv"])
    assert np.array_equal(iters, ref["iters"])
