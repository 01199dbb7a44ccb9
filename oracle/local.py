"""The other local NLS solvers of Algorithm 1: multiplicative updates (MU) and
hierarchical alternating least squares (HALS), plain FP64 CPU code.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module; the library never does.

Both update one factor given the Gram matrix G of the other factor and the
right-hand sides R (Section "Nonnegative Least Squares", Eq. muupdate and
Eq. halsupdate).  Every row x of X (a row of W, or a row of H^T, i.e. a
column of H) is updated independently:

  MU   x_j <- x_j r_j / (x^T G)_j          for all j at once, from the old x
  HALS x_i <- [r_i - sum_{l != i} G_li x_l]_+ / G_ii   for i = 1..k in order,
       each step using the values already updated in this sweep

Readings (the paper does not say): an index with G_ii <= 1e-14 max_l G_ll is
pinned at 0 (as in BPP); MU sets x_j = 0 where (x^T G)_j <= 0 (a zero row,
which MU can never leave).
"""
import numpy as np

import oracle

PIN_REL = 1e-14


def pinned(G):
    d = np.diag(np.asarray(G, dtype=np.float64))
    return d <= PIN_REL * (d.max() if d.size else 0.0)


def mu_update(G, R, X):
    """Eq. muupdate on every row of X (rows x k) with R (rows x k)."""
    G = np.asarray(G, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    D = X @ G                      # (x^T G)_j per row
    out = np.where(D > 0.0, X * R / np.where(D > 0.0, D, 1.0), 0.0)
    out[:, pinned(G)] = 0.0
    return out


def hals_update(G, R, X):
    """Eq. halsupdate on every row of X: one sweep over the indices in order."""
    G = np.asarray(G, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    X = np.array(X, dtype=np.float64, copy=True)
    k = G.shape[0]
    pin = pinned(G)
    for i in range(k):
        if pin[i]:
            X[:, i] = 0.0
            continue
        others = np.arange(k) != i
        s = R[:, i] - X[:, others] @ G[others, i]
        X[:, i] = np.maximum(s, 0.0) / G[i, i]
    return X


UPDATES = {"mu": mu_update, "hals": hals_update}


def anls(solver, k, W0, Ht0, T, *, dense):
    """Algorithm 1 with the MU or HALS local update for T iterations on a dense
    A (m x n), all in FP64.  Returns W, Ht and the relative objective after
    every W half-step (r_half) and full iteration (r_full)."""
    upd = UPDATES[solver]
    A = np.asarray(dense, dtype=np.float64)
    W = np.asarray(W0, dtype=np.float64).copy()
    Ht = np.asarray(Ht0, dtype=np.float64).copy()
    nA = np.linalg.norm(A)
    r_half, r_full = np.zeros(T), np.zeros(T)
    for t in range(T):
        GH = oracle.gram(Ht)
        W = upd(GH, A @ Ht, W)
        r_half[t] = np.linalg.norm(A - W @ Ht.T) / nA
        GW = oracle.gram(W)
        Ht = upd(GW, A.T @ W, Ht)
        r_full[t] = np.linalg.norm(A - W @ Ht.T) / nA
    return dict(W=W, Ht=Ht, r_half=r_half, r_full=r_full)


def _products(A, Ht, W, chunk):
    """A @ Ht and A^T @ W in FP64 over row blocks of a (possibly FP32) A."""
    m = A.shape[0]
    RW = None if Ht is None else np.empty((m, Ht.shape[1]))
    RH = None if W is None else np.zeros((A.shape[1], W.shape[1]))
    for r0 in range(0, m, chunk):
        blk = np.asarray(A[r0:r0 + chunk], dtype=np.float64)
        if RW is not None:
            RW[r0:r0 + chunk] = blk @ Ht
        if RH is not None:
            RH += blk.T @ W[r0:r0 + chunk]
    return RW, RH


def anls_trace(solver, k, W0, Ht0, T, A, chunk=20_000):
    """Algorithm 1 with the MU or HALS update on a large dense A (m x n, any
    float dtype, read in row blocks), FP64 throughout.  The relative objective
    comes from the expansion ||A - W H||^2 = ||A||^2 - 2 <R, X> + <G_W, G_H>
    with the right-hand sides R of the half-step (the trace form, no m x n
    temporary).  Returns W, Ht, r_half, r_full."""
    upd = UPDATES[solver]
    W = np.asarray(W0, dtype=np.float64).copy()
    Ht = np.asarray(Ht0, dtype=np.float64).copy()
    fro2 = 0.0
    for r0 in range(0, A.shape[0], chunk):
        fro2 += float(np.sum(np.asarray(A[r0:r0 + chunk], dtype=np.float64) ** 2))
    r_half, r_full = np.zeros(T), np.zeros(T)

    def rel(R, X, GW, GH):
        return np.sqrt(max(fro2 - 2.0 * float(np.sum(R * X)) + float(np.sum(GW * GH)), 0.0) / fro2)

    for t in range(T):
        GH = oracle.gram(Ht)
        RW, _ = _products(A, Ht, None, chunk)
        W = upd(GH, RW, W)
        GW = oracle.gram(W)
        r_half[t] = rel(RW, W, GW, GH)
        _, RH = _products(A, None, W, chunk)
        Ht = upd(GW, RH, Ht)
        GH = oracle.gram(Ht)
        r_full[t] = rel(RH, Ht, GW, GH)
    return dict(W=W, Ht=Ht, r_half=r_half, r_full=r_full, fro2=fro2)
