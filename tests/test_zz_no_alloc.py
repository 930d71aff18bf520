"""The allocation-free sort entry point (static scratch array) against the workspace sort, through the C ABI."""
import numpy as np
import pytest
import torch

from paper_2411_02703_amd import binding as B

pytestmark = pytest.mark.gpu


def _keys(rng, n, bits):
    hi = rng.integers(0, max(1, 1 << (bits - 32)), n, dtype=np.uint64)
    lo = rng.integers(0, 1 << 12, n, dtype=np.uint64) << np.uint64(18)
    return (hi << np.uint64(32)) | lo


def test_static_sort_matches_workspace_sort_on_two_calls(gpu_lib):
    """Two calls in a row, the second smaller (the array keeps the first call's contents); both must equal the
    workspace sort and the stable argsort bit for bit."""
    rng = np.random.default_rng(77)
    nmax = B.gs_sort_static_max()
    assert nmax == 1 << 20
    for n, bits in ((nmax, 45), (300_001, 41), (1, 33)):
        keys = _keys(rng, n, bits)
        vals = rng.permutation(n).astype(np.int32)
        ka = torch.as_tensor(keys.view(np.int64)).cuda()
        va = torch.as_tensor(vals).cuda()
        kb, vb = ka.clone(), va.clone()
        print("static sort", n, bits, flush=True)
        B.gs_sort_pairs_static(ka, va, bits)
        B.gs_sort_pairs(kb, vb, bits)
        torch.cuda.synchronize()
        assert torch.equal(ka, kb) and torch.equal(va, vb)
        order = np.argsort(keys, kind="stable")
        assert np.array_equal(ka.cpu().numpy().view(np.uint64), keys[order])
        assert np.array_equal(va.cpu().numpy(), vals[order])


def test_static_sort_rejects_more_than_its_capacity(gpu_lib):
    n = B.gs_sort_static_max() + 1
    k = torch.zeros(n, dtype=torch.int64, device="cuda")
    v = torch.zeros(n, dtype=torch.int32, device="cuda")
    with pytest.raises(RuntimeError, match="static scratch"):
        B.gs_sort_pairs_static(k, v, 40)
