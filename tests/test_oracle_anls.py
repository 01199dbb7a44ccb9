"""Pins of the oracle's ANLS driver (Algorithm 1): non-increasing objective
(each half-step is an exact block minimisation, Eq. two-block), the expansion
of the objective against the direct residual, every subproblem of config 1
against exhaustive search, a planted exact factorisation as a fixed point,
and warm/cold equivalence.  CPU only."""
import json
import os

import numpy as np
import pytest

import oracle
from nmf_inputs import configs as C

from test_oracle_bpp import brute_force

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def config1_inputs():
    w = C.WORKLOADS["c1"]
    A = C.config1_matrix(w.m, w.n, w.rank)
    return w, A, C.init_w(w.seed, w.m, w.k), C.init_ht(w.seed, w.n, w.k)


def assert_monotone(r_half, r_full, r0=None):
    prev = np.inf if r0 is None else r0
    for rh, rf in zip(r_half, r_full):
        assert rh <= prev * (1 + 1e-12)
        assert rf <= rh * (1 + 1e-12)
        prev = rf


def test_config1_monotone_and_trace_equals_direct(oracle_lib):
    w, A, W0, H0 = config1_inputs()
    res = oracle.anls(w.k, W0, H0, w.iters, dense=A)
    fa, fr0 = oracle.objective_dense(A, W0, H0)
    assert_monotone(res["r_half"], res["r_full"], np.sqrt(fr0 / fa))
    fa, fr = oracle.objective_dense(A, res["W"], res["Ht"])
    assert abs(np.sqrt(fr / fa) - res["r_full"][-1]) < 1e-12
    assert res["capped"] == 0
    assert res["W"].min() >= 0 and res["Ht"].min() >= 0


def test_config1_every_subproblem_brute_force(oracle_lib):
    """Re-walk Algorithm 1 step by step and check each row / column NNLS
    against exhaustive search over all 2^5 passive sets, and the KKT signs."""
    w, A, W, Ht = config1_inputs()
    W = W.astype(np.float64)
    Ht = Ht.astype(np.float64)
    for t in range(w.iters):
        G = oracle.gram(Ht)
        R = oracle.rhs_dense_w(A, Ht)
        W, _, _, st = oracle.bpp_batched(G, R)
        assert np.all(st & oracle.ST_CAPPED == 0)
        for i in range(w.m):
            np.testing.assert_allclose(W[i], brute_force(G, R[i]), rtol=1e-9, atol=1e-11)
            y = G @ W[i] - R[i]
            assert y.min() >= -1e-10 * np.abs(R[i]).max()
        G = oracle.gram(W)
        R = oracle.rhs_dense_h(A, W)
        Ht, _, _, _ = oracle.bpp_batched(G, R)
        for j in range(w.n):
            np.testing.assert_allclose(Ht[j], brute_force(G, R[j]), rtol=1e-9, atol=1e-11)
    ref = oracle.anls(w.k, *config1_inputs()[2:], w.iters, dense=A)
    np.testing.assert_allclose(Ht, ref["Ht"], rtol=1e-12, atol=1e-14)


def test_config1_golden(oracle_lib):
    with open(os.path.join(GOLDEN, "config1_oracle.json")) as fh:
        g = json.load(fh)
    w, A, W0, H0 = config1_inputs()
    res = oracle.anls(w.k, W0, H0, w.iters, dense=A)
    np.testing.assert_allclose(res["r_half"], g["r_half"], rtol=1e-12)
    np.testing.assert_allclose(res["r_full"], g["r_full"], rtol=1e-12)
    assert list(res["rounds_w"]) == g["rounds_w"] and list(res["rounds_h"]) == g["rounds_h"]


def test_fixed_point_planted_exact(oracle_lib):
    """A = W* H* exactly with H* H*^T nonsingular: one W update from H*
    returns W* and the objective is zero (to rounding)."""
    rng = np.random.default_rng(21)
    m, n, k = 60, 45, 4
    Ws = rng.integers(0, 4, (m, k)).astype(np.float64)
    Hs = rng.integers(1, 4, (n, k)).astype(np.float64)
    A = (Ws @ Hs.T).astype(np.float32)          # small integers: exact
    G = oracle.gram(Hs)
    R = oracle.rhs_dense_w(A, Hs)
    W, _, _, _ = oracle.bpp_batched(G, R)
    np.testing.assert_allclose(W, Ws, atol=1e-9)
    res = oracle.anls(k, rng.uniform(size=(m, k)), Hs, 1, dense=A)
    # the trace expansion cancels to ~sqrt(eps); the direct residual is exact
    assert res["r_half"][0] < 1e-7
    fa, fr = oracle.objective_dense(A, W, Hs)
    assert fr < 1e-18 * fa


def test_rank1_closed_form(oracle_lib):
    """k = 1 and A = u v^T with u, v > 0: every NNLS is a scalar with a
    positive solution, so one iteration of Algorithm 1 from h > 0 gives
    w = A h / (h.h) = u (v.h)/(h.h), then h' = A^T w / (w.w) = v (h.h)/(v.h),
    and w h'^T = A exactly (closed form written out by hand)."""
    rng = np.random.default_rng(33)
    m, n = 40, 30
    u = rng.integers(1, 5, m).astype(np.float64)
    v = rng.integers(1, 5, n).astype(np.float64)
    A = np.outer(u, v).astype(np.float32)          # small integers: exact in FP32
    h = rng.uniform(0.5, 1.5, n)
    res = oracle.anls(1, rng.uniform(size=(m, 1)), h[:, None], 1, dense=A)
    w_ref = u * (v @ h) / (h @ h)
    h_ref = v * (h @ h) / (v @ h)
    np.testing.assert_allclose(res["W"][:, 0], w_ref, rtol=1e-13)
    np.testing.assert_allclose(res["Ht"][:, 0], h_ref, rtol=1e-13)
    fa, fr = oracle.objective_dense(A, res["W"], res["Ht"])
    assert fr < 1e-24 * fa
    # after the W half-step the residual is u (v - h (v.h)/(h.h))^T: relative
    # size sqrt(1 - (v.h)^2 / ((v.v)(h.h))); after the H half-step zero (the
    # trace form cancels to about sqrt(eps))
    r_half = np.sqrt(1.0 - (v @ h) ** 2 / ((v @ v) * (h @ h)))
    assert abs(res["r_half"][0] - r_half) < 1e-7
    assert res["r_full"][0] < 1e-6


def test_warm_equals_cold_trajectory(oracle_lib):
    w, A, W0, H0 = config1_inputs()
    cold = oracle.anls(w.k, W0, H0, w.iters, dense=A)
    warm = oracle.anls(w.k, W0, H0, w.iters, dense=A, warm=1, warm_cap=50)
    np.testing.assert_allclose(warm["r_full"], cold["r_full"], rtol=1e-10)
    np.testing.assert_allclose(warm["Ht"], cold["Ht"], rtol=1e-8, atol=1e-12)
    assert warm["rounds_w"][1:].sum() < cold["rounds_w"][1:].sum()


def test_sparse_small_monotone_and_golden(oracle_lib):
    w = C.WORKLOADS["c3s"]
    rp, ci, va = C.sparse_csr(w.seed, w.m, w.n, w.density, inst=w.inst)
    rpt, cit, vat = C.csr_transpose(w.m, w.n, rp, ci, va)
    W0 = C.init_w(w.seed, w.m, w.k, inst=w.inst)
    H0 = C.init_ht(w.seed, w.n, w.k, inst=w.inst)
    res = oracle.anls(w.k, W0, H0, w.iters, csr=(rp, ci, va), csr_t=(rpt, cit, vat), shape=(w.m, w.n))
    assert_monotone(res["r_half"], res["r_full"])
    fa, fr = oracle.objective_csr(w.m, w.n, rp, ci, va, res["W"], res["Ht"])
    assert abs(np.sqrt(max(fr, 0) / fa) - res["r_full"][-1]) < 1e-10
    dense = C.csr_to_dense(w.m, w.n, rp, ci, va)
    resd = oracle.anls(w.k, W0, H0, 3, dense=dense)
    np.testing.assert_allclose(resd["r_full"], res["r_full"][:3], rtol=1e-10)
    with open(os.path.join(GOLDEN, "config3_small_oracle.json")) as fh:
        g = json.load(fh)
    assert g["nnz"] == int(rp[-1])
    np.testing.assert_allclose(res["r_full"], g["r_full"], rtol=1e-12)


@pytest.mark.parametrize("name", ["c2s"])
def test_scaled_dense_monotone(oracle_lib, name):
    w = C.WORKLOADS[name]
    A = C.dense_rows(w, np.arange(w.m))
    res = oracle.anls(w.k, C.init_w(w.seed, w.m, w.k), C.init_ht(w.seed, w.n, w.k), 4, dense=A)
    assert_monotone(res["r_half"], res["r_full"])
    assert res["capped"] == 0
