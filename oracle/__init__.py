"""FP64 CPU oracle for ANLS-BPP NMF -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package; the product path (paper_1509_09313_amd) never does, and the
two share no code.  The arithmetic lives in nmf_oracle.c (plain float64 loops)
and mlp.py (the warm-start network in float64 NumPy); this module only
marshals NumPy arrays into the C library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC = os.path.join(_HERE, "nmf_oracle.c")

ST_WARM_FALLBACK = 1
ST_CAPPED = 2
ST_PINNED = 4
ST_SINGULAR = 8

_lib = None


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-std=c11", SRC, "-o", LIB_PATH + ".tmp", "-lm"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("building the oracle failed:\n" + res.stderr)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    if verbose:
        print("built", LIB_PATH)
    return LIB_PATH


class _Matrix(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("colidx", ctypes.c_void_p), ("vals", ctypes.c_void_p),
                ("rowptr_t", ctypes.c_void_p), ("colidx_t", ctypes.c_void_p), ("vals_t", ctypes.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, ci, cd = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.orc_gram.argtypes = [i64, ci, vp, i64, vp]
        L.orc_rhs_dense_w.argtypes = [i64, i64, ci, vp, i64, vp, vp]
        L.orc_rhs_dense_h.argtypes = [i64, i64, ci, vp, i64, vp, vp]
        L.orc_rhs_csr.argtypes = [i64, ci, vp, vp, vp, vp, vp]
        L.orc_pinned_set.argtypes = [ci, vp]
        L.orc_pinned_set.restype = ctypes.c_uint64
        L.orc_bpp.argtypes = [ci, vp, vp, vp, vp, ci, ci, vp, vp]
        L.orc_bpp.restype = ci
        L.orc_bpp_batched.argtypes = [ci, i64, vp, vp, vp, vp, vp, vp, vp, ci, ci]
        L.orc_objective_dense.argtypes = [i64, i64, ci, vp, i64, vp, vp, vp, vp]
        L.orc_objective_csr.argtypes = [i64, i64, ci, vp, vp, vp, vp, vp, vp, vp]
        L.orc_anls.argtypes = [ctypes.POINTER(_Matrix), ci, vp, vp, ci, ci, ci, ci, cd, vp, vp, vp, vp,
                               vp, vp, vp]
        L.orc_anls.restype = ci
        L.orc_max_threads.restype = ci
        L.orc_set_threads.argtypes = [ci]
        L.orc_set_threads.restype = None
        L.orc_last_phase_seconds.argtypes = [vp]
        L.orc_last_phase_seconds.restype = None
        _lib = L
    return _lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def gram(X) -> np.ndarray:
    """G = X^T X (Algorithm 1's H H^T with X = H^T, and W^T W with X = W)."""
    X = _f64(X)
    rows, k = X.shape
    G = np.empty((k, k), dtype=np.float64)
    lib().orc_gram(rows, k, _p(X), k, _p(G))
    return G


def rhs_dense_w(A, Y) -> np.ndarray:
    """A @ Y with A float32 (m x n), Y (n x k): A H^T for Y = H^T."""
    A, Y = _f32(A), _f64(Y)
    m, n = A.shape
    k = Y.shape[1]
    R = np.empty((m, k), dtype=np.float64)
    lib().orc_rhs_dense_w(m, n, k, _p(A), n, _p(Y), _p(R))
    return R


def rhs_dense_h(A, Y) -> np.ndarray:
    """A^T @ Y with Y (m x k): (W^T A)^T for Y = W."""
    A, Y = _f32(A), _f64(Y)
    m, n = A.shape
    k = Y.shape[1]
    R = np.empty((n, k), dtype=np.float64)
    lib().orc_rhs_dense_h(m, n, k, _p(A), n, _p(Y), _p(R))
    return R


def rhs_csr(rowptr, colidx, vals, Y) -> np.ndarray:
    rowptr = np.ascontiguousarray(rowptr, np.int64)
    colidx = np.ascontiguousarray(colidx, np.int32)
    vals = _f32(vals)
    Y = _f64(Y)
    rows = rowptr.size - 1
    k = Y.shape[1]
    R = np.empty((rows, k), dtype=np.float64)
    lib().orc_rhs_csr(rows, k, _p(rowptr), _p(colidx), _p(vals), _p(Y), _p(R))
    return R


def pinned_set(G) -> int:
    G = _f64(G)
    return int(lib().orc_pinned_set(G.shape[0], _p(G)))


def bpp(G, f, F0: int = 0, max_rounds: int = 100, warm_cap: int = 8):
    """One NNLS problem min_{x>=0} 1/2 x'Gx - f'x.

    Returns (x, F, rounds, status, y)."""
    G, f = _f64(G), _f64(f)
    k = G.shape[0]
    x = np.zeros(k, dtype=np.float64)
    y = np.zeros(k, dtype=np.float64)
    F = ctypes.c_uint64(F0)
    r = ctypes.c_int(0)
    st = lib().orc_bpp(k, _p(G), _p(f), _p(x), ctypes.byref(F), max_rounds, warm_cap,
                       ctypes.byref(r), _p(y))
    return x, int(F.value), int(r.value), int(st), y


def bpp_batched(G, R, mask_in=None, max_rounds: int = 100, warm_cap: int = 8):
    """Rows of R as independent problems. Returns (X, masks, rounds, status)."""
    G, R = _f64(G), _f64(R)
    k = G.shape[0]
    batch = R.shape[0]
    X = np.zeros((batch, k), dtype=np.float64)
    masks = np.zeros(batch, dtype=np.uint64)
    rounds = np.zeros(batch, dtype=np.int32)
    status = np.zeros(batch, dtype=np.int32)
    mi = None if mask_in is None else np.ascontiguousarray(mask_in, dtype=np.uint64)
    lib().orc_bpp_batched(k, batch, _p(G), _p(R), _p(X), _p(mi), _p(masks), _p(rounds), _p(status),
                          max_rounds, warm_cap)
    return X, masks, rounds, status


def objective_dense(A, W, Ht):
    """(||A||_F^2, ||A - W H||_F^2) with H = Ht^T."""
    A, W, Ht = _f32(A), _f64(W), _f64(Ht)
    m, n = A.shape
    k = W.shape[1]
    fa, fr = ctypes.c_double(0), ctypes.c_double(0)
    lib().orc_objective_dense(m, n, k, _p(A), n, _p(W), _p(Ht), ctypes.byref(fa), ctypes.byref(fr))
    return fa.value, fr.value


def objective_csr(m, n, rowptr, colidx, vals, W, Ht):
    rowptr = np.ascontiguousarray(rowptr, np.int64)
    colidx = np.ascontiguousarray(colidx, np.int32)
    vals, W, Ht = _f32(vals), _f64(W), _f64(Ht)
    k = W.shape[1]
    fa, fr = ctypes.c_double(0), ctypes.c_double(0)
    lib().orc_objective_csr(m, n, k, _p(rowptr), _p(colidx), _p(vals), _p(W), _p(Ht),
                            ctypes.byref(fa), ctypes.byref(fr))
    return fa.value, fr.value


def anls(k, W0, Ht0, T, *, dense=None, csr=None, csr_t=None, shape=None, max_rounds=100, warm=0,
         warm_cap=8):
    """Algorithm 1 for T iterations from (W0, Ht0).

    dense: float32 (m x n) array, or csr=(rowptr, colidx, vals) with
    csr_t = CSR of A^T and shape=(m, n).  Returns a dict with W, Ht, r_half,
    r_full (relative objectives), rounds_w, rounds_h, capped, masks_w, masks_h.
    """
    keep = []
    M = _Matrix()
    if dense is not None:
        A = _f32(dense)
        keep.append(A)
        m, n = A.shape
        M.kind, M.m, M.n, M.A, M.lda = 0, m, n, A.ctypes.data, n
        fro2 = float(np.sum(A.astype(np.float64) ** 2))
    else:
        m, n = shape
        rp, ci, va = (np.ascontiguousarray(csr[0], np.int64), np.ascontiguousarray(csr[1], np.int32),
                      _f32(csr[2]))
        rpt, cit, vat = (np.ascontiguousarray(csr_t[0], np.int64),
                         np.ascontiguousarray(csr_t[1], np.int32), _f32(csr_t[2]))
        keep += [rp, ci, va, rpt, cit, vat]
        M.kind, M.m, M.n = 1, m, n
        M.rowptr, M.colidx, M.vals = rp.ctypes.data, ci.ctypes.data, va.ctypes.data
        M.rowptr_t, M.colidx_t, M.vals_t = rpt.ctypes.data, cit.ctypes.data, vat.ctypes.data
        fro2 = float(np.sum(va.astype(np.float64) ** 2))
    W = _f64(W0).copy()
    Ht = _f64(Ht0).copy()
    r_half = np.zeros(T)
    r_full = np.zeros(T)
    rw = np.zeros(T, dtype=np.int64)
    rh = np.zeros(T, dtype=np.int64)
    cap = ctypes.c_int64(0)
    mw = np.zeros(m, dtype=np.uint64)
    mh = np.zeros(n, dtype=np.uint64)
    rc = lib().orc_anls(ctypes.byref(M), k, _p(W), _p(Ht), T, max_rounds, warm, warm_cap, fro2,
                        _p(r_half), _p(r_full), _p(rw), _p(rh), ctypes.byref(cap), _p(mw), _p(mh))
    if rc != 0:
        raise MemoryError("oracle ANLS could not allocate its buffers")
    ph = np.zeros(6)
    lib().orc_last_phase_seconds(_p(ph))
    return dict(W=W, Ht=Ht, r_half=r_half, r_full=r_full, rounds_w=rw, rounds_h=rh,
                capped=int(cap.value), masks_w=mw, masks_h=mh, fro2=fro2,
                phase_seconds=dict(zip(("rhs_w", "bpp_w", "gram", "rhs_h", "bpp_h", "objective"), ph.tolist())))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def set_threads(n: int) -> None:
    """Thread count of the oracle's OpenMP loops from now on."""
    lib().orc_set_threads(int(n))


def kkt_residuals(G, f, x):
    """Violations of Eq. KKT for one solution: (min x, min y off-support, |x.y|)."""
    G, f, x = _f64(G), _f64(f), _f64(x)
    y = G @ x - f
    return float(np.min(x)), y, float(abs(np.dot(x, y)))
