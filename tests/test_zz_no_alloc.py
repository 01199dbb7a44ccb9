"""nmf_gram_noalloc, the Gram entry point that allocates nothing (its block
partials live in the library's static device scratch), against nmf_gram on
the same inputs: bit-identical results, since both run the same kernels in the
same order, and within the FP64 bound of the oracle.  Two calls in a row, the
second on a smaller input, so the second reads a scratch the first filled;
and no device memory is taken by the calls after the first."""
import numpy as np
import pytest
import torch

import oracle
from paper_1509_09313_amd import binding as L

pytestmark = pytest.mark.gpu


def _case(rows, k, pad, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.0, 1.0, (rows, k)).astype(np.float32)
    t = torch.zeros((rows, k + pad), dtype=torch.float32, device="cuda")
    t[:, :k] = torch.from_numpy(X).cuda()
    return X, t[:, :k]


def _check(X, Xd):
    rows, k = X.shape
    G_ws = L.nmf_gram(Xd)
    G_na = torch.full((k, k), float("nan"), dtype=torch.float64, device="cuda")
    L.nmf_gram_noalloc(Xd, G_na)
    torch.cuda.synchronize()
    a, b = G_ws.cpu().numpy(), G_na.cpu().numpy()
    assert np.array_equal(a, b), np.nanmax(np.abs(a - b))
    X64 = X.astype(np.float64)
    bound = rows * 2.0 ** -52 * (np.abs(X64).T @ np.abs(X64))
    assert np.all(np.abs(b - oracle.gram(X64)) <= bound)
    assert np.array_equal(b, b.T)


def test_noalloc_gram_two_calls_second_smaller():
    # first call: the largest partial footprint (1024 blocks at k = 64)
    X1, X1d = _case(300_001, 64, 3, 11)
    print("nmf_gram_noalloc: rows 300001, k 64", flush=True)
    _check(X1, X1d)
    # second call: fewer blocks and a smaller k, over the partials of the first
    X2, X2d = _case(1_000, 7, 0, 12)
    G = torch.empty((7, 7), dtype=torch.float64, device="cuda")
    free1 = torch.cuda.mem_get_info()[0]
    print("nmf_gram_noalloc: rows 1000, k 7", flush=True)
    L.nmf_gram_noalloc(X2d, G)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free1, "nmf_gram_noalloc took device memory"
    _check(X2, X2d)


def test_noalloc_gram_empty_and_bad_arguments():
    G = torch.full((5, 5), 7.0, dtype=torch.float64, device="cuda")
    X = torch.empty((0, 5), dtype=torch.float32, device="cuda")
    L.nmf_gram_noalloc(X, G)
    torch.cuda.synchronize()
    assert torch.count_nonzero(G).item() == 0
    lib = L.lib()
    p = G.data_ptr()
    assert lib.nmf_gram_noalloc(10, 65, p, 65, p, None) == L.NMF_EINVAL
    assert lib.nmf_gram_noalloc(10, 8, p, 4, p, None) == L.NMF_EINVAL
    assert lib.nmf_gram_noalloc(10, 8, None, 8, p, None) == L.NMF_EINVAL
