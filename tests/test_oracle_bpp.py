"""Pins of the oracle's NNLS solver (block principal pivoting) against facts
that do not depend on it: exhaustive search over all 2^k passive sets, the KKT
conditions of Eq. KKT, closed forms, and SciPy's independent Lawson-Hanson
NNLS.  CPU only."""
import numpy as np
import pytest
from scipy.optimize import nnls

import oracle


def brute_force(G, f):
    """Minimise 1/2 x'Gx - f'x over x >= 0 by trying every passive set."""
    k = G.shape[0]
    best_val, best_x = None, None
    for mask in range(1 << k):
        idx = [i for i in range(k) if (mask >> i) & 1]
        x = np.zeros(k)
        if idx:
            sub = G[np.ix_(idx, idx)]
            if np.linalg.matrix_rank(sub) < len(idx):
                continue
            x[idx] = np.linalg.solve(sub, f[idx])
            if np.any(x < 0):
                continue
        val = 0.5 * x @ G @ x - f @ x
        if best_val is None or val < best_val - 1e-13 * (1 + abs(val)):
            best_val, best_x = val, x
    return best_x


def random_problem(rng, k, rows=None):
    rows = k + 3 if rows is None else rows
    C = rng.standard_normal((rows, k))
    b = rng.standard_normal(rows)
    return C.T @ C, C.T @ b, C, b


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_bpp_equals_brute_force(oracle_lib, k):
    rng = np.random.default_rng(100 + k)
    for _ in range(60):
        G, f, _, _ = random_problem(rng, k)
        x, F, rounds, st, _ = oracle.bpp(G, f)
        xb = brute_force(G, f)
        assert st & oracle.ST_CAPPED == 0
        np.testing.assert_allclose(x, xb, rtol=1e-9, atol=1e-10)
        for i in range(k):
            assert x[i] >= 0.0 and ((F >> i) & 1 or x[i] == 0.0)


@pytest.mark.parametrize("k", [4, 10, 30, 50, 64])
def test_bpp_kkt_and_scipy(oracle_lib, k):
    rng = np.random.default_rng(7 * k)
    for _ in range(20):
        G, f, C, b = random_problem(rng, k, rows=2 * k)
        x, F, rounds, st, y = oracle.bpp(G, f)
        assert st & (oracle.ST_CAPPED | oracle.ST_SINGULAR) == 0
        scale = np.abs(G).max() * max(1.0, np.abs(x).max()) + np.abs(f).max()
        yy = G @ x - f
        assert x.min() >= 0.0
        assert yy.min() >= -1e-10 * scale
        assert abs(x @ yy) <= 1e-9 * scale * max(1.0, np.abs(x).sum())
        # passive set and support agree; the reported y is zero on F
        for i in range(k):
            if (F >> i) & 1:
                assert y[i] == 0.0
        xs, _ = nnls(C, b)
        np.testing.assert_allclose(x, xs, rtol=1e-7, atol=1e-9)


def test_closed_form_k1(oracle_lib):
    for g, f in [(2.0, 3.0), (2.0, -3.0), (5.0, 0.0)]:
        x, F, rounds, st, _ = oracle.bpp(np.array([[g]]), np.array([f]))
        assert abs(x[0] - max(0.0, f / g)) <= 4e-16 * abs(f / g)


def test_closed_form_diagonal(oracle_lib):
    rng = np.random.default_rng(3)
    d = rng.uniform(0.5, 3.0, 12)
    f = rng.standard_normal(12)
    x, F, _, _, _ = oracle.bpp(np.diag(d), f)
    np.testing.assert_allclose(x, np.maximum(0.0, f / d), rtol=4e-16)
    assert F == sum(1 << i for i in range(12) if f[i] > 0)


def test_closed_form_unconstrained_feasible(oracle_lib):
    rng = np.random.default_rng(4)
    C = rng.uniform(0.1, 1.0, (20, 6))
    xt = rng.uniform(0.5, 2.0, 6)
    G, f = C.T @ C, C.T @ (C @ xt)
    x, F, rounds, st, _ = oracle.bpp(G, f)
    np.testing.assert_allclose(x, np.linalg.solve(G, f), rtol=1e-10)
    np.testing.assert_allclose(x, xt, rtol=1e-9)
    assert F == (1 << 6) - 1


def test_closed_form_nonpositive_rhs(oracle_lib):
    rng = np.random.default_rng(5)
    G, _, _, _ = random_problem(rng, 7)
    f = -np.abs(rng.standard_normal(7))
    x, F, rounds, st, _ = oracle.bpp(G, f)
    assert np.all(x == 0.0) and F == 0 and rounds == 1


def test_warm_start_invariance(oracle_lib):
    rng = np.random.default_rng(6)
    for _ in range(30):
        G, f, _, _ = random_problem(rng, 9)
        x0, F0, r0, _, _ = oracle.bpp(G, f)
        for start in (F0, (~F0) & 0x1FF, 0x155, 0x1FF):
            x, F, r, st, _ = oracle.bpp(G, f, F0=start, warm_cap=50)
            np.testing.assert_allclose(x, x0, rtol=1e-9, atol=1e-12)
        # starting from the answer takes a single round
        _, _, r1, _, _ = oracle.bpp(G, f, F0=F0)
        assert F0 == 0 or r1 == 1


def test_pinned_zero_column(oracle_lib):
    rng = np.random.default_rng(8)
    C = rng.standard_normal((12, 5))
    C[:, 2] = 0.0
    b = rng.standard_normal(12)
    G, f = C.T @ C, C.T @ b
    x, F, rounds, st, _ = oracle.bpp(G, f)
    assert st & oracle.ST_PINNED
    assert x[2] == 0.0 and not (F >> 2) & 1
    keep = [0, 1, 3, 4]
    xs, _ = nnls(C[:, keep], b)
    np.testing.assert_allclose(x[keep], xs, rtol=1e-8, atol=1e-10)


def test_singular_duplicate_column(oracle_lib):
    rng = np.random.default_rng(9)
    C = rng.uniform(0.1, 1.0, (15, 4))
    C[:, 3] = C[:, 1]
    b = C @ np.array([1.0, 2.0, 0.5, 0.0])
    G, f = C.T @ C, C.T @ b
    x, F, rounds, st, _ = oracle.bpp(G, f)
    # the residual is that of the best nonnegative fit, whichever copy is used
    assert st & oracle.ST_CAPPED == 0
    np.testing.assert_allclose(C @ x, b, atol=1e-9)


def test_cap_and_clamp(oracle_lib):
    rng = np.random.default_rng(10)
    # a problem that needs several rounds from the cold start
    for _ in range(50):
        G, f, _, _ = random_problem(rng, 12)
        _, _, r, _, _ = oracle.bpp(G, f)
        if r >= 3:
            break
    x, F, rounds, st, _ = oracle.bpp(G, f, max_rounds=2)
    assert st & oracle.ST_CAPPED and rounds == 2 and x.min() >= 0.0


def test_warm_fallback(oracle_lib):
    rng = np.random.default_rng(11)
    G, f, _, _ = random_problem(rng, 10)
    x0, F0, _, _, _ = oracle.bpp(G, f)
    bad = (~F0) & 0x3FF
    x, F, rounds, st, _ = oracle.bpp(G, f, F0=bad, warm_cap=1)
    if bad:
        assert st & oracle.ST_WARM_FALLBACK
    np.testing.assert_allclose(x, x0, rtol=1e-10, atol=1e-12)
    assert F == F0


def test_batched_matches_single(oracle_lib):
    rng = np.random.default_rng(12)
    G, _, C, _ = random_problem(rng, 6, rows=30)
    R = rng.standard_normal((40, 6)) @ G * 0.3 + rng.standard_normal((40, 6))
    X, masks, rounds, status = oracle.bpp_batched(G, R)
    for b in range(40):
        x, F, r, st, _ = oracle.bpp(G, R[b])
        assert np.array_equal(x, X[b]) and F == masks[b] and r == rounds[b]
