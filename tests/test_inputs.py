"""Input generators: Philox against its published known-answer vectors, and the
workload recipes' structural properties (host side; no GPU)."""
import math

import numpy as np
import pytest

from nmf_inputs import configs as C
from nmf_inputs import philox


# Known-answer vectors published with the Random123 library for
# philox4x32-10: (counter, key) -> output.
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,expect", KAT)
def test_philox_known_answers(ctr, key, expect):
    out = philox.philox4x32_10(*ctr, *key)
    assert tuple(int(x) for x in out) == expect


def test_uniform_exact_float32_and_range():
    u = philox.uniform(123, 4, 0, 64, 0, 64)
    assert u.dtype == np.float32
    assert u.min() >= 0.0 and u.max() < 1.0
    # every value is a multiple of 2^-24
    assert np.all((u.astype(np.float64) * 2 ** 24) % 1 == 0)
    assert abs(u.mean() - 0.5) < 0.02


def test_uniform_is_addressable():
    blk = philox.uniform(7, 3, 100, 5, 200, 6)
    pts = philox.uniform_at(7, 3, np.arange(100, 105)[:, None], np.arange(200, 206)[None, :])
    assert np.array_equal(blk, pts)


def test_planted_rows_addressable_and_bounds():
    seed = C.seed_for(2)
    full = C.planted_rows(seed, 40, 6, np.arange(10))
    some = C.planted_rows(seed, 40, 6, np.array([3, 7]), cols=np.array([0, 5, 39]))
    assert np.array_equal(some, full[[3, 7]][:, [0, 5, 39]])
    assert full.min() >= 0.0 and full.max() < 6 + 0.01


def test_video_rows_structure():
    a = C.video_rows(C.seed_for(5), 300, np.arange(400))
    assert a.min() >= 0.0 and a.max() < 1.0
    fg = philox.uniform(C.seed_for(5), C.MID_FGMASK, 0, 400, 0, 300) < np.float32(0.02)
    assert abs(fg.mean() - 0.02) < 0.004


def test_sparse_csr_properties():
    m, n, p = 3000, 2500, 2e-3
    rp, ci, va = C.sparse_csr(C.seed_for(3), m, n, p, inst=7)
    assert rp[0] == 0 and rp[-1] == ci.size == va.size
    assert np.all(np.diff(rp) >= 0)
    for i in range(0, m, 97):
        row = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0) and (row.size == 0 or (row[0] >= 0 and row[-1] < n))
    assert va.min() > 0.0 and va.max() <= 1.0
    dens = ci.size / (m * n)
    assert abs(dens - p) < 5 * math.sqrt(p / (m * n))
    # transpose is a re-indexing of the same entries
    rpt, cit, vat = C.csr_transpose(m, n, rp, ci, va)
    d = C.csr_to_dense(m, n, rp, ci, va)
    dt = C.csr_to_dense(n, m, rpt, cit, vat)
    assert np.array_equal(d.T, dt)


def test_batched_shapes_ranges():
    shapes = C.batched_shapes()
    assert len(shapes) == 256
    ms, ns, ks = zip(*shapes)
    assert 500 <= min(ms) and max(ms) <= 8000
    assert 500 <= min(ns) and max(ns) <= 4000
    assert set(ks) <= {10, 20, 50} and len(set(ks)) == 3


def test_mlp_init_layout():
    k = 30
    lay = C.mlp_layout(k)
    p = C.mlp_init(k, C.seed_for(5))
    assert p.size == lay["total"][1] == 2 * k * 128 + 128 + 128 * 128 + 128 + 128 * k + k
    off, sz = lay["W2"]
    w2 = p[off:off + sz].astype(np.float64)
    assert abs(w2.std() - math.sqrt(2.0 / 128)) < 0.01
    assert np.all(p[lay["b1"][0]:lay["b1"][0] + 128] == 0)
