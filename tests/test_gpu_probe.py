"""The LDS bandwidth probe reads what it wrote: its per-thread fold equals the
same fold computed on the host from the fill pattern (so no read was dropped),
and invalid arguments are refused before any launch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1903_10107_amd import binding
    binding.lib()
    return binding


def _expected(mode, reps):
    i = np.arange(4096, dtype=np.uint64)
    words = np.stack([i, 3 * i, 5 * i, 7 * i], axis=1).astype(np.uint32)      # buf[i] = (i, 3i, 5i, 7i)
    tid = np.arange(1024)
    acc = np.zeros(1024, dtype=np.uint32)
    if mode == 0:
        x = words[:, 0] ^ words[:, 1] ^ words[:, 2] ^ words[:, 3]
        for r in range(reps):
            for k in range(8):
                acc ^= x[((tid + r) & 511) + 512 * k]
    else:
        b8 = words.reshape(-1).view(np.uint8)
        for r in range(reps):
            for k in range(8):
                acc += b8[((tid + r) & 8191) + 8192 * k].astype(np.uint32)
    return acc


@pytest.mark.parametrize("mode", [0, 1])
def test_probe_fold_matches_host(B, mode):
    import torch
    n_wg, reps = 3, 5
    out = torch.zeros(n_wg * 1024, dtype=torch.int32, device="cuda")
    B.ldpc_probe_lds_bandwidth(mode, n_wg, reps, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32).reshape(n_wg, 1024)
    exp = _expected(mode, reps)
    for w in range(n_wg):
        assert np.array_equal(got[w], exp), (mode, w)


def test_probe_argument_errors(B):
    import torch
    out = torch.zeros(1024, dtype=torch.int32, device="cuda")
    for args in ((2, 1, 1), (0, 0, 1), (1, 1, 0)):
        with pytest.raises(B.LdpcError) as ei:
            B.ldpc_probe_lds_bandwidth(*args, out)
        assert ei.value.code == B.LDPC_EINVAL
