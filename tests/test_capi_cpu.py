"""The C ABI without a GPU: the library loads, exports every function the
header declares, rejects invalid arguments on the host (before any device
work), and its check-node arithmetic (compiled for the host from the same
inline function the kernels use) equals the oracle's Alg. 1 table."""
import ctypes as C
import os

import numpy as np
import pytest

import oracle as O
from paper_1903_10107_amd import binding as B
from paper_1903_10107_amd import inputs as I


def test_library_exports_every_declared_function():
    names = B.header_functions()
    assert "ldpc_code_create" in names and "ldpc_decode_batch" in names
    lib = B.lib()
    for n in names:
        assert hasattr(lib, n), n


def test_host_tau_table_equals_oracle_alg1():
    assert np.array_equal(B.ldpc_host_tau_table(), O.tau_table(64))


def test_version():
    assert B.ldpc_version() >= 100


def _create(base, mb, nb, z, prm=None):
    h = C.c_void_p()
    base = np.ascontiguousarray(base, dtype=np.int32)
    rc = B.lib().ldpc_code_create(base.ctypes.data, mb, nb, z, C.byref(prm) if prm else None, C.byref(h))
    return rc, h


GOOD = I.make_base(5, 32, 32)


@pytest.mark.parametrize("case", [
    "null_base", "z0", "mb_ge_nb", "shift_high", "shift_low", "zero_col", "row_deg1", "bad_acc",
    "bad_msg", "bad_emax", "bad_rule", "off_iters0", "iters_no_off", "bad_hint",
])
def test_create_rejects_invalid_arguments(case):
    base = GOOD.copy()
    mb, nb, z = 5, 32, 32
    prm = None
    if case == "null_base":
        h = C.c_void_p()
        assert B.lib().ldpc_code_create(None, mb, nb, z, None, C.byref(h)) == B.LDPC_EINVAL
        return
    if case == "z0":
        z = 0
    elif case == "mb_ge_nb":
        base, mb, nb = GOOD[:, :5].copy(), 5, 5
    elif case == "shift_high":
        base[0, 0] = 32
    elif case == "shift_low":
        base[0, 0] = -2
    elif case == "zero_col":
        base[:, 3] = -1
    elif case == "row_deg1":
        base = np.full((2, 4), -1, np.int32)
        base[0, :] = 0
        base[1, 0] = 1
        mb, nb = 2, 4
    elif case == "bad_acc":
        prm = B.ldpc_params(0, 0, 12, 0, None, 0, 0)
    elif case == "bad_msg":
        prm = B.ldpc_params(200, 0, 0, 0, None, 0, 0)
    elif case == "bad_emax":
        prm = B.ldpc_params(0, 300, 8, 0, None, 0, 0)
    elif case == "bad_rule":
        prm = B.ldpc_params(0, 0, 0, 7, None, 0, 0)
    elif case == "off_iters0":
        off = np.zeros(96, np.int8)
        prm = B.ldpc_params(0, 0, 0, 0, off.ctypes.data, 0, 0)
    elif case == "bad_hint":
        prm = B.ldpc_params(0, 0, 0, 0, None, 0, 9)
    elif case == "iters_no_off":
        prm = B.ldpc_params(0, 0, 0, 0, None, 3, 0)
    rc, h = _create(base, mb, nb, z, prm)
    assert rc == B.LDPC_EINVAL
    assert not h.value
    assert B.ldpc_last_error()


def test_create_rejects_too_high_row_degree_as_unsupported():
    base = np.zeros((2, 40), np.int32)
    rc, _ = _create(base, 2, 40, 7)
    assert rc == B.LDPC_EUNSUPPORTED
    assert "32" in B.ldpc_last_error()


def test_null_out_and_null_code_are_rejected():
    base = np.ascontiguousarray(GOOD)
    assert B.lib().ldpc_code_create(base.ctypes.data, 5, 32, 32, None, None) == B.LDPC_EINVAL
    assert B.lib().ldpc_decode_batch(None, None, None, 1, 1, None, None, None) == B.LDPC_EINVAL
    assert B.lib().ldpc_decode_batch_ex(None, None, None, 1, 1, None, None, None, None, None, None, 0,
                                        None) == B.LDPC_EINVAL
    assert B.lib().ldpc_code_dims(None, None, None, None, None, None) == B.LDPC_EINVAL
    assert B.lib().ldpc_syndrome_batch(None, None, 1, None, None) == B.LDPC_EINVAL
    assert B.lib().ldpc_order_by_unsat(None, None, None, 1, None, None, None) == B.LDPC_EINVAL
    assert b"code is NULL" in B.lib().ldpc_last_error()
    assert B.lib().ldpc_workspace_bytes(None, 4) == 0
    B.lib().ldpc_code_destroy(None)


def test_valid_code_without_a_gpu_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, h = _create(GOOD, 5, 32, 32)
    assert rc == B.LDPC_EDEVICE
    assert not h.value
    with pytest.raises(B.LdpcError):
        B.Code(GOOD, 32)


@pytest.mark.parametrize("rule", [O.RULE_RCBP_FB, O.RULE_RCBP_EQ7, O.RULE_MINSUM])
def test_host_packed_fold_equals_oracle(rule):
    """The kernels' packed fold (two rows per register, padded to 32 operands)
    computes the oracle's magnitudes for every degree and rule."""
    rng = np.random.default_rng(rule + 10)
    lib = B.lib()
    for trial in range(400):
        d = int(rng.integers(2, 33))
        hi_cap = 127 if trial % 4 == 0 else 63
        lo = rng.integers(0, 64 if trial % 3 else 8, size=d).astype(np.int32)
        hi = rng.integers(0, hi_cap + 1, size=d).astype(np.int32)
        olo = np.zeros(d, np.int32)
        ohi = np.zeros(d, np.int32)
        assert lib.ldpc_host_fold_pair(rule, lo.ctypes.data, hi.ctypes.data, d, olo.ctypes.data,
                                       ohi.ctypes.data) == 0
        assert np.array_equal(olo, O.cn_magnitudes(lo, rule, msg_max=127))
        assert np.array_equal(ohi, O.cn_magnitudes(hi, rule, msg_max=127))


def test_one_hip_runtime_in_the_process():
    """The library binds to the HIP runtime torch loads, whatever the import order."""
    import subprocess
    import sys
    code = ("from paper_1903_10107_amd import binding as B; B.lib(); import torch; "
            "m = open('/proc/self/maps').read(); "
            "print(len({l.split()[-1] for l in m.splitlines() if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_c_client_links_and_loads_without_a_gpu():
    """The plain C client of the ABI is built, and its loader finds libqkdldpc and
    the HIP runtime (run without arguments it prints its usage before any HIP call)."""
    import subprocess
    client = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_client", "decode_client")
    assert os.path.exists(client), "build() builds tests/c_client/decode_client"
    out = subprocess.run([client], capture_output=True, text=True, timeout=60)
    assert out.returncode == 1 and "usage" in out.stderr, out.stderr


def test_static_decode_rejects_a_null_code_without_a_gpu():
    rc = B.lib().ldpc_decode_batch_static(None, None, None, 1, 5, None, None, None, None, None)
    assert rc == B.LDPC_EINVAL
    assert b"code is NULL" in B.lib().ldpc_last_error()
