"""Pins of the MU and HALS oracle (Eq. muupdate, Eq. halsupdate) against what
the mathematics fixes, not against a retyped formula:
  * the NNLS optimum (from the BPP oracle, itself pinned by brute force and
    KKT) is a fixed point of both updates;
  * each HALS step is the exact minimiser of the objective along its
    coordinate over x_i >= 0, found here by a numerical 1-D search;
  * neither update increases 1/2 x'Gx - r'x (MU needs G, r >= 0);
  * closed forms for diagonal G, MU's zero locking, pinned indices;
  * Algorithm 1 with either update never increases ||A - WH||.
"""
import numpy as np
import pytest
from scipy.optimize import minimize_scalar

import oracle
from oracle import local

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def nmf_problem(rng, k, rows=None, m=80):
    """G = C'C (nonnegative C) and right-hand sides R = C'c for nonnegative c."""
    C = rng.uniform(0.0, 1.0, (m, k))
    G = C.T @ C
    n = 1 if rows is None else rows
    R = rng.uniform(0.0, 1.0, (n, m)) @ C
    return G, R


def objective(G, r, x):
    return 0.5 * x @ G @ x - r @ x


@pytest.mark.parametrize("k", [1, 3, 7, 12, 30])
def test_nnls_optimum_is_a_fixed_point(k):
    rng = np.random.default_rng(100 + k)
    G, R = nmf_problem(rng, k, rows=6)
    # push some right-hand sides negative so optima have active indices
    R[:3] -= 0.6 * R[:3].mean(axis=1, keepdims=True)
    X = np.stack([oracle.bpp(G, r)[0] for r in R])
    assert np.allclose(local.hals_update(G, R, X), X, rtol=1e-9, atol=1e-12)
    Xm = local.mu_update(G, R, X)
    assert np.allclose(Xm, X, rtol=1e-9, atol=1e-12)
    assert np.all(Xm[X == 0.0] == 0.0)


@pytest.mark.parametrize("k", [2, 5, 9])
def test_hals_steps_are_coordinate_minimisers(k):
    rng = np.random.default_rng(200 + k)
    G, R = nmf_problem(rng, k)
    R = R[0] - 0.3 * R[0].mean()
    x0 = rng.uniform(0.0, 1.0, k)
    x = x0.copy()
    for i in range(k):   # the sweep done by 1-D searches, in order
        def phi(t, i=i):
            y = x.copy()
            y[i] = t
            return objective(G, R, y)
        hi = 10.0 * (abs(R).sum() / G[i, i] + 1.0)
        res = minimize_scalar(phi, bounds=(0.0, hi), method="bounded", options={"xatol": 1e-12})
        x[i] = res.x if phi(res.x) < phi(0.0) else 0.0
    got = local.hals_update(G, R[None, :], x0[None, :])[0]
    assert np.allclose(got, x, rtol=1e-7, atol=1e-8)


@pytest.mark.parametrize("solver", ["mu", "hals"])
def test_updates_never_increase_the_objective(solver):
    rng = np.random.default_rng(300)
    k = 8
    G, R = nmf_problem(rng, k, rows=20)
    X = rng.uniform(0.0, 1.0, (20, k))
    upd = local.UPDATES[solver]
    prev = np.array([objective(G, r, x) for r, x in zip(R, X)])
    for _ in range(15):
        X = upd(G, R, X)
        cur = np.array([objective(G, r, x) for r, x in zip(R, X)])
        assert np.all(cur <= prev + 1e-12 * np.abs(prev))
        prev = cur
    # and both approach the NNLS optimum
    opt = np.array([objective(G, r, oracle.bpp(G, r)[0]) for r in R])
    assert np.all(prev >= opt - 1e-9 * np.abs(opt))


def test_diagonal_closed_forms():
    d = np.array([2.0, 0.5, 4.0, 1.0])
    G = np.diag(d)
    R = np.array([[1.0, -2.0, 3.0, 0.0], [-1.0, 1.0, 8.0, 2.0]])
    X = np.array([[0.3, 0.7, 0.0, 1.5], [2.0, 0.1, 1.0, 0.4]])
    assert np.array_equal(local.hals_update(G, R, X), np.maximum(R, 0.0) / d)
    Xm = local.mu_update(G, R, X)
    # x_j r_j / (x_j d_j) = r_j / d_j where x_j > 0; zeros stay zero
    expect = np.where(X > 0.0, R / d, 0.0)
    assert np.allclose(Xm, expect, rtol=1e-15, atol=0.0)


def test_pinned_index_is_zero():
    rng = np.random.default_rng(400)
    G, R = nmf_problem(rng, 5, rows=3)
    G[2, :] = 0.0
    G[:, 2] = 0.0
    X = rng.uniform(0.1, 1.0, (3, 5))
    for upd in (local.hals_update, local.mu_update):
        assert np.all(upd(G, R, X)[:, 2] == 0.0)


@pytest.mark.parametrize("solver", ["mu", "hals"])
def test_alg1_objective_is_monotone(solver):
    rng = np.random.default_rng(500)
    m, n, k = 60, 40, 5
    A = rng.uniform(0.0, 1.0, (m, 3)) @ rng.uniform(0.0, 1.0, (3, n)) + 0.05 * rng.uniform(0.0, 1.0, (m, n))
    W0, H0 = rng.uniform(0.0, 1.0, (m, k)), rng.uniform(0.0, 1.0, (n, k))
    out = local.anls(solver, k, W0, H0, 12, dense=A.astype(np.float32))
    seq = np.ravel(np.column_stack([out["r_half"], out["r_full"]]))
    assert np.all(np.diff(seq) <= 1e-12)
    assert seq[-1] < seq[0]


@pytest.mark.parametrize("solver", ["mu", "hals"])
def test_trace_form_loop_equals_direct(solver):
    """The row-chunked, trace-form Algorithm 1 gives the direct loop's
    factors and objectives (the expansion of ||A - WH||^2 is exact up to
    rounding)."""
    rng = np.random.default_rng(600)
    m, n, k = 130, 70, 6
    A = (rng.uniform(0.0, 1.0, (m, 4)) @ rng.uniform(0.0, 1.0, (4, n))).astype(np.float32)
    W0, H0 = rng.uniform(0.0, 1.0, (m, k)), rng.uniform(0.0, 1.0, (n, k))
    a = local.anls(solver, k, W0, H0, 6, dense=A)
    b = local.anls_trace(solver, k, W0, H0, 6, A, chunk=37)
    assert np.allclose(a["W"], b["W"], rtol=1e-12, atol=1e-14)
    assert np.allclose(a["Ht"], b["Ht"], rtol=1e-12, atol=1e-14)
    assert np.allclose(a["r_half"], b["r_half"], rtol=1e-9, atol=1e-12)
    assert np.allclose(a["r_full"], b["r_full"], rtol=1e-9, atol=1e-12)
