"""Pins of the oracle's local products (Gram, dense and sparse right-hand
sides) and objective: exact integer arithmetic (Python ints, no rounding) on
small integer-valued inputs, closed forms, and identities.  CPU only."""
import numpy as np

import oracle
from nmf_inputs import configs as C


def int_matrix(rng, shape, lo=-4, hi=5):
    return rng.integers(lo, hi, size=shape).astype(np.int64)


def exact_matmul(a, b):
    """Integer matrix product with Python ints (exact)."""
    a = [[int(v) for v in row] for row in a]
    b = [[int(v) for v in row] for row in b]
    n, k, m = len(a), len(b), len(b[0])
    return np.array([[sum(a[i][t] * b[t][j] for t in range(k)) for j in range(m)] for i in range(n)],
                    dtype=np.float64)


def test_gram_exact_integers(oracle_lib):
    rng = np.random.default_rng(1)
    X = int_matrix(rng, (37, 9))
    G = oracle.gram(X.astype(np.float64))
    assert np.array_equal(G, exact_matmul(X.T, X))
    assert np.array_equal(G, G.T)


def test_gram_closed_form():
    n = 1000
    X = np.stack([np.arange(1, n + 1), np.ones(n)], axis=1).astype(np.float64)
    G = oracle.gram(X)
    assert G[0, 0] == n * (n + 1) * (2 * n + 1) // 6
    assert G[0, 1] == G[1, 0] == n * (n + 1) // 2
    assert G[1, 1] == n


def test_rhs_dense_exact_integers(oracle_lib):
    rng = np.random.default_rng(2)
    A = int_matrix(rng, (23, 31), 0, 7)
    Y = int_matrix(rng, (31, 6))
    W = int_matrix(rng, (23, 6))
    Rw = oracle.rhs_dense_w(A.astype(np.float32), Y.astype(np.float64))
    Rh = oracle.rhs_dense_h(A.astype(np.float32), W.astype(np.float64))
    assert np.array_equal(Rw, exact_matmul(A, Y))
    assert np.array_equal(Rh, exact_matmul(A.T, W))


def test_rhs_dense_rank_one_closed_form(oracle_lib):
    u = np.arange(1, 8, dtype=np.float64)
    v = np.arange(1, 6, dtype=np.float64)
    A = np.outer(u, v).astype(np.float32)
    Y = np.ones((5, 3))
    R = oracle.rhs_dense_w(A, Y)
    assert np.array_equal(R, np.outer(u, np.full(3, v.sum())))


def test_rhs_csr_equals_dense(oracle_lib):
    m, n = 300, 200
    rp, ci, va = C.sparse_csr(11, m, n, 0.05)
    va = np.round(va * 8).astype(np.float32)     # small integers: exact sums
    A = C.csr_to_dense(m, n, rp, ci, va)
    rng = np.random.default_rng(3)
    Y = int_matrix(rng, (n, 7)).astype(np.float64)
    W = int_matrix(rng, (m, 7)).astype(np.float64)
    assert np.array_equal(oracle.rhs_csr(rp, ci, va, Y), exact_matmul(A.astype(np.int64), Y))
    rpt, cit, vat = C.csr_transpose(m, n, rp, ci, va)
    assert np.array_equal(oracle.rhs_csr(rpt, cit, vat, W), exact_matmul(A.T.astype(np.int64), W))


def test_objective_dense_exact(oracle_lib):
    rng = np.random.default_rng(4)
    W = int_matrix(rng, (12, 3), 0, 4)
    Ht = int_matrix(rng, (9, 3), 0, 4)
    A = exact_matmul(W, Ht.T)
    fa, fr = oracle.objective_dense(A.astype(np.float32), W, Ht)
    assert fr == 0.0 and fa == float((A ** 2).sum())
    A2 = A.copy()
    A2[3, 4] += 5
    A2[0, 0] -= 2
    _, fr2 = oracle.objective_dense(A2.astype(np.float32), W, Ht)
    assert fr2 == 25.0 + 4.0


def test_objective_csr_matches_all_entries(oracle_lib):
    m, n, k = 60, 45, 4
    rp, ci, va = C.sparse_csr(13, m, n, 0.1)
    va = np.round(va * 8).astype(np.float32)
    A = C.csr_to_dense(m, n, rp, ci, va).astype(np.int64)
    rng = np.random.default_rng(5)
    W = int_matrix(rng, (m, k), 0, 3)
    Ht = int_matrix(rng, (n, k), 0, 3)
    res = A - exact_matmul(W, Ht.T)
    fa, fr = oracle.objective_csr(m, n, rp, ci, va, W.astype(np.float64), Ht.astype(np.float64))
    assert fa == float((A ** 2).sum())
    assert fr == float((res ** 2).sum())
