"""Per-kernel parity of libnmf (through the C-ABI) against the FP64 CPU oracle
on identical seeded inputs, including ragged shapes and degenerate cases.

Tolerances come from the arithmetic of each kernel:
  Gram   FP64 sums of exact FP32 products: |dG| <= rows * 2^-52 * |X|^T|X|
  RHS    FP32 accumulation over L terms:   |dR| <= L * 2^-24 * |A||Y|
  SpMM   FP64 sums in the oracle's order, then one rounding: bit-identical
  BPP    FP64 solves, FP32 outputs: |dx| <= 4 ulp32(x) + 1e-9 max|x|
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from nmf_inputs import configs as C
from paper_1509_09313_amd import binding as L

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def padded(a, pad):
    """Device copy of a 2-D array with leading dimension cols + pad."""
    rows, cols = a.shape
    t = torch.zeros((rows, cols + pad), dtype=torch.float32, device="cuda")
    t[:, :cols] = cuda(a)
    return t[:, :cols]


# ------------------------------------------------------------------ Gram ----
@pytest.mark.parametrize("rows,k,pad", [(0, 5, 0), (1, 1, 0), (127, 5, 1), (128, 30, 0), (129, 30, 2),
                                        (1000, 50, 0), (5000, 64, 0), (20001, 33, 3), (300000, 30, 0)])
def test_gram(rows, k, pad):
    rng = np.random.default_rng(rows * 131 + k)
    X = rng.uniform(0.0, 1.0, (rows, k)).astype(np.float32)
    G = L.nmf_gram(padded(X, pad) if rows else cuda(X)).cpu().numpy()
    X64 = X.astype(np.float64)
    Go = oracle.gram(X64)
    bound = rows * 2.0 ** -52 * (np.abs(X64).T @ np.abs(X64))
    assert np.all(np.abs(G - Go) <= bound), np.max(np.abs(G - Go))
    assert np.array_equal(G, G.T)


# ------------------------------------------------------------ dense RHS ----
RHS_CASES = [(200, 150, 5, 0), (257, 131, 30, 0), (129, 1000, 50, 1), (33, 4097, 64, 0), (1000, 999, 33, 3),
             (4096, 256, 1, 0), (3, 5, 7, 0), (70000, 300, 30, 0), (20000, 2400, 30, 0)]


@pytest.mark.parametrize("m,n,k,pad", RHS_CASES)
def test_rhs_dense_f32(m, n, k, pad):
    rng = np.random.default_rng(m + 7 * n + k)
    A = rng.uniform(0.0, 1.0, (m, n)).astype(np.float32)
    Ht = rng.uniform(0.0, 1.0, (n, k)).astype(np.float32)
    W = rng.uniform(0.0, 1.0, (m, k)).astype(np.float32)
    Ad = padded(A, pad)
    A64 = A.astype(np.float64)
    Rw = L.nmf_rhs_dense(L.NMF_SIDE_W, Ad, cuda(Ht)).cpu().numpy().astype(np.float64)
    Rwo = oracle.rhs_dense_w(A, Ht.astype(np.float64))
    bw = 1.01 * n * U32 * (np.abs(A64) @ np.abs(Ht.astype(np.float64)))
    assert np.all(np.abs(Rw - Rwo) <= bw + 1e-30), np.max(np.abs(Rw - Rwo) / (bw + 1e-30))
    Rh = L.nmf_rhs_dense(L.NMF_SIDE_H, Ad, cuda(W)).cpu().numpy().astype(np.float64)
    Rho = oracle.rhs_dense_h(A, W.astype(np.float64))
    bh = 1.01 * (m + 1) * U32 * (np.abs(A64).T @ np.abs(W.astype(np.float64)))
    assert np.all(np.abs(Rh - Rho) <= bh + 1e-30), np.max(np.abs(Rh - Rho) / (bh + 1e-30))


@pytest.mark.parametrize("rows,cols,ld", [(777, 1030, 1030), (64, 64, 70), (1, 300, 301), (300, 1, 1), (0, 5, 5)])
def test_transpose_f32(rows, cols, ld):
    rng = np.random.default_rng(rows + 3 * cols)
    Xs = rng.standard_normal((rows, ld)).astype(np.float32)
    X = cuda(Xs)[:, :cols]
    Xt = L.nmf_transpose_f32(X).cpu().numpy()
    assert Xt.shape == (cols, rows) and np.array_equal(Xt, Xs[:, :cols].T)


@pytest.mark.parametrize("rows,n,k", [(200, 150_000, 30), (300, 70_001, 50), (2400, 40_000, 30)])
def test_rhs_dense_f32_split_contraction(rows, n, k):
    """Side W with few row tiles and a long contraction (A^T W over a
    resident A^T): the contraction is split into ranges whose FP32 partials
    are summed in FP64; each range is an FP32 chain of nmf_rhs_dense_chain
    terms, which bounds the error against the exact product."""
    rng = np.random.default_rng(rows + n + k)
    A = rng.uniform(0.0, 1.0, (rows, n)).astype(np.float32)
    Y = rng.uniform(0.0, 1.0, (n, k)).astype(np.float32)
    terms = ctypes.c_int64(0)
    assert L.lib().nmf_rhs_dense_chain(L.NMF_SIDE_W, rows, n, k, L.NMF_F32, ctypes.byref(terms)) == L.NMF_OK
    assert terms.value < n  # the split is taken
    R = L.nmf_rhs_dense(L.NMF_SIDE_W, cuda(A), cuda(Y)).cpu().numpy().astype(np.float64)
    Ro = oracle.rhs_dense_w(A, Y.astype(np.float64))
    b = 1.01 * (terms.value + 1) * U32 * (np.abs(A.astype(np.float64)) @ np.abs(Y.astype(np.float64)))
    assert np.all(np.abs(R - Ro) <= b + 1e-30), np.max(np.abs(R - Ro) / (b + 1e-30))


def test_rhs_dense_empty_contraction():
    A = torch.zeros((5, 0), dtype=torch.float32, device="cuda")
    R = L.nmf_rhs_dense(L.NMF_SIDE_W, A, torch.zeros((0, 4), dtype=torch.float32, device="cuda"))
    assert torch.count_nonzero(R).item() == 0


# ----------------------------------------------------------------- SpMM ----
@pytest.mark.parametrize("m,n,k,density", [(2000, 1500, 50, 1e-3), (3000, 2500, 30, 1e-2), (500, 400, 5, 0.05),
                                           (64, 64, 64, 0.3), (1, 10, 3, 0.5)])
def test_rhs_csr_bit_exact(m, n, k, density):
    rp, ci, va = C.sparse_csr(11 + m, m, n, density)
    rpt, cit, vat = C.csr_transpose(m, n, rp, ci, va)
    rng = np.random.default_rng(m)
    Ht = rng.uniform(0.0, 1.0, (n, k)).astype(np.float32)
    W = rng.uniform(0.0, 1.0, (m, k)).astype(np.float32)
    Rw = L.nmf_rhs_csr(cuda(rp), cuda(ci), cuda(va), cuda(Ht), m, n).cpu().numpy()
    Rh = L.nmf_rhs_csr(cuda(rpt), cuda(cit), cuda(vat), cuda(W), n, m).cpu().numpy()
    assert np.array_equal(Rw, oracle.rhs_csr(rp, ci, va, Ht.astype(np.float64)).astype(np.float32))
    assert np.array_equal(Rh, oracle.rhs_csr(rpt, cit, vat, W.astype(np.float64)).astype(np.float32))


@pytest.mark.parametrize("m,n,k,ld", [(2000, 1500, 50, 64), (3000, 2500, 30, 32), (700, 900, 5, 8),
                                      (300, 200, 64, 70), (130, 257, 33, 64)])
def test_rhs_csr_padded_and_strided(m, n, k, ld):
    """Y and R with leading dimensions above k (the line-aligned layout the
    ANLS driver uses, and an odd one) give the oracle's bits; R's padding
    columns are left alone.  Rows hold 0 to ~300 entries (several 128-entry
    blocks and 32-entry chunks, ragged ends)."""
    rp, ci, va = C.sparse_csr(23 + m, m, n, 0.3 if m <= 300 else 0.02)
    rng = np.random.default_rng(k)
    Ht = rng.uniform(0.0, 1.0, (n, k)).astype(np.float32)
    Yb = torch.full((n, ld), float("nan"), dtype=torch.float32, device="cuda")
    Yb[:, :k] = cuda(Ht)
    Rb = torch.full((m, k + 3), -1.0, dtype=torch.float32, device="cuda")
    L.nmf_rhs_csr(cuda(rp), cuda(ci), cuda(va), Yb[:, :k], m, n, R=Rb[:, :k])
    assert np.array_equal(Rb[:, :k].cpu().numpy(), oracle.rhs_csr(rp, ci, va, Ht.astype(np.float64)).astype(np.float32))
    assert torch.all(Rb[:, k:] == -1.0)


# ------------------------------------------------------------------ BPP ----
def nmf_like_problems(rng, k, batch, rows=None):
    """G = C^T C with nonnegative C (an NMF Gram) and right-hand sides
    C^T b for b mixing a nonnegative combination and noise, so that the
    solutions have varied active sets."""
    rows = rows or (3 * k + 10)
    Cm = rng.uniform(0.0, 1.0, (rows, k))
    G = Cm.T @ Cm
    xs = rng.uniform(0.0, 1.0, (batch, k)) * (rng.uniform(size=(batch, k)) < 0.7)
    B = xs @ Cm.T + 0.3 * rng.standard_normal((batch, rows))
    R = (B @ Cm).astype(np.float32)
    return G, R


def degenerate(G, f, x, tau_rel=1e-9):
    y = G @ x - f
    tau = tau_rel * (np.abs(G).max() * np.abs(x).max() + np.abs(f).max())
    return (np.abs(x) <= tau) & (np.abs(y) <= tau)


def compare_bpp(G, R, out, ref, check_rounds=True):
    X, masks, rounds, status = (t.cpu().numpy() for t in out)
    Xo, mo, ro, so = ref
    k = G.shape[0]
    masks = masks.view(np.uint64)
    tol = 4 * U32 * np.abs(Xo) + 1e-9 * max(1.0, np.abs(Xo).max())
    assert np.all(np.abs(X.astype(np.float64) - Xo) <= tol), np.max(np.abs(X - Xo))
    bad = 0
    for b in range(R.shape[0]):
        diff = int(masks[b]) ^ int(mo[b])
        if diff:
            deg = degenerate(G, R[b].astype(np.float64), Xo[b])
            dmask = sum(1 << i for i in range(k) if deg[i])
            assert diff & ~dmask == 0, (b, bin(diff))
            bad += 1
    assert np.array_equal(status.astype(np.int32), so)
    if check_rounds:
        assert np.mean(rounds.astype(np.int32) == ro) >= 0.999
    return bad


@pytest.mark.parametrize("k,batch", [(1, 5), (5, 1000), (8, 999), (9, 777), (16, 1024), (17, 513), (30, 4099),
                                     (32, 1000), (33, 600), (50, 2000), (56, 301), (57, 300), (64, 257)])
def test_bpp_cold(k, batch):
    rng = np.random.default_rng(1000 + k)
    G, R = nmf_like_problems(rng, k, batch)
    out = L.nnls_bpp_batched(cuda(G), cuda(R))
    ref = oracle.bpp_batched(G, R.astype(np.float64))
    compare_bpp(G, R, out, ref)


def test_bpp_empty_batch():
    G = torch.eye(4, dtype=torch.float64, device="cuda")
    R = torch.zeros((0, 4), dtype=torch.float32, device="cuda")
    X, m, r, s = L.nnls_bpp_batched(G, R)
    assert X.shape == (0, 4)


def test_bpp_pinned_and_singular():
    rng = np.random.default_rng(5)
    k, batch = 12, 500
    Cm = rng.uniform(0.0, 1.0, (40, k))
    Cm[:, 3] = 0.0             # zero column: pinned from the start
    Cm[:, 7] = Cm[:, 2]        # duplicate column: singular passive subset
    G = Cm.T @ Cm
    R = (rng.standard_normal((batch, 40)) @ Cm + 0.5 * Cm.sum(0)).astype(np.float32)
    out = L.nnls_bpp_batched(cuda(G), cuda(R))
    ref = oracle.bpp_batched(G, R.astype(np.float64))
    X = out[0].cpu().numpy()
    assert np.all(X[:, 3] == 0.0)
    st = out[3].cpu().numpy()
    assert np.all(st & L.NMF_BPP_PINNED)
    assert np.array_equal(st.astype(np.int32), ref[3])
    # x itself may differ where the duplicate columns trade weight; the fit does not
    res_gpu = Cm @ X.T.astype(np.float64)
    res_orc = Cm @ ref[0].T
    assert np.max(np.abs(res_gpu - res_orc)) <= 1e-5 * np.abs(res_orc).max()


def test_bpp_deferred_problems():
    """k > 32 with a singular G: G_U^{-1} is unavailable (the duplicate column
    fails its sweep pivot), so every round eliminates over F, and problems
    whose F outgrows the two-problem kernel's 28 pivot positions are finished
    by the one-problem kernel from their start.  The oracle's final sets show
    that such problems exist; statuses, fits and counters must not show where
    a problem was solved."""
    rng = np.random.default_rng(11)
    k, batch = 48, 700
    Cm = rng.uniform(0.0, 1.0, (150, k))
    Cm[:, 5] = 0.0             # pinned from the start
    Cm[:, 40] = Cm[:, 9]       # singular passive subsets
    G = Cm.T @ Cm
    xs = rng.uniform(0.2, 1.0, (batch, k)) * (rng.uniform(size=(batch, k)) < 0.5)
    R = ((xs @ Cm.T + 0.05 * rng.standard_normal((batch, 150))) @ Cm).astype(np.float32)
    ref = oracle.bpp_batched(G, R.astype(np.float64))
    sizes = np.array([bin(int(m)).count("1") for m in ref[1]])
    assert np.sum(sizes > 28) >= 50 and np.sum(sizes <= 28) >= 50, np.bincount(sizes)
    cnt = torch.zeros(L.NMF_BPP_COUNTERS, dtype=torch.int64, device="cuda")
    X, masks, rounds, st = (t.cpu().numpy() for t in L.nnls_bpp_batched(cuda(G), cuda(R), counters=cnt))
    assert np.all(np.isfinite(X)) and np.all(X >= 0.0)
    assert np.all(X[:, 5] == 0.0)
    assert np.array_equal(st.astype(np.int32), ref[3])
    res_gpu = Cm @ X.T.astype(np.float64)
    res_orc = Cm @ ref[0].T
    assert np.max(np.abs(res_gpu - res_orc)) <= 1e-5 * np.abs(res_orc).max()
    assert cnt.cpu().numpy()[0] == rounds.astype(np.int64).sum()
    assert np.mean(rounds.astype(np.int32) == ref[2]) >= 0.99


def test_bpp_solutions_in_place_of_rhs():
    """X may alias R (ldx == ldr): then no deferral mark may be written into
    x_0, and the one-row-per-lane form solves every problem.  Checked where
    the pivot-row kernel would defer (k = 48, singular G) and where it would
    not (k = 30), against the oracle."""
    rng = np.random.default_rng(13)
    k, batch = 48, 700
    Cm = rng.uniform(0.0, 1.0, (150, k))
    Cm[:, 40] = Cm[:, 9]
    G = Cm.T @ Cm
    xs = rng.uniform(0.2, 1.0, (batch, k)) * (rng.uniform(size=(batch, k)) < 0.5)
    R = ((xs @ Cm.T + 0.05 * rng.standard_normal((batch, 150))) @ Cm).astype(np.float32)
    ref = oracle.bpp_batched(G, R.astype(np.float64))
    Rd = cuda(R)
    X, masks, rounds, st = (t.cpu().numpy() for t in L.nnls_bpp_batched(cuda(G), Rd, X=Rd))
    assert np.all(np.isfinite(X)) and np.array_equal(X, Rd.cpu().numpy())
    assert np.array_equal(st.astype(np.int32), ref[3])
    res_gpu = Cm @ X.T.astype(np.float64)
    res_orc = Cm @ ref[0].T
    assert np.max(np.abs(res_gpu - res_orc)) <= 1e-5 * np.abs(res_orc).max()
    rng = np.random.default_rng(14)
    G, R = nmf_like_problems(rng, 30, 2000)
    ref = oracle.bpp_batched(G, R.astype(np.float64))
    Rd = cuda(R)
    out = L.nnls_bpp_batched(cuda(G), Rd, X=Rd)
    compare_bpp(G, R, out, ref)


@pytest.mark.parametrize("k", [40, 50, 64])
def test_bpp_counters_two_problem_kernel(k):
    """Round and pivot-step counters of the k > 32 kernels equal the sums of
    the per-problem records; the stored sets reproduce the solutions."""
    rng = np.random.default_rng(12 + k)
    batch = 3001
    G, R = nmf_like_problems(rng, k, batch)
    cnt = torch.zeros(L.NMF_BPP_COUNTERS, dtype=torch.int64, device="cuda")
    out = L.nnls_bpp_batched(cuda(G), cuda(R), counters=cnt)
    ref = oracle.bpp_batched(G, R.astype(np.float64))
    compare_bpp(G, R, out, ref)
    c = cnt.cpu().numpy()
    rounds = out[2].cpu().numpy().astype(np.int64)
    assert c[0] == rounds.sum()
    # warm start from the stored sets: one round each, same solutions
    cnt.zero_()
    out2 = L.nnls_bpp_batched(cuda(G), cuda(R), mask_in=out[1], counters=cnt)
    r2 = out2[2].cpu().numpy()
    m = out[1].cpu().numpy()
    assert np.all(r2[m != 0] == 1)
    assert cnt.cpu().numpy()[0] == r2.astype(np.int64).sum()
    np.testing.assert_allclose(out2[0].cpu().numpy(), out[0].cpu().numpy(), rtol=1e-6, atol=1e-9)


def test_bpp_cap_and_warm():
    rng = np.random.default_rng(6)
    k, batch = 30, 3000
    G, R = nmf_like_problems(rng, k, batch)
    # the cap: statuses and clamped iterates agree with the oracle
    out = L.nnls_bpp_batched(cuda(G), cuda(R), max_rounds=2)
    ref = oracle.bpp_batched(G, R.astype(np.float64), max_rounds=2)
    compare_bpp(G, R, out, ref)
    assert np.any(out[3].cpu().numpy() & L.NMF_BPP_CAPPED)
    # warm start from the answer: one round each
    cold = oracle.bpp_batched(G, R.astype(np.float64))
    mi = cuda(cold[1].view(np.int64))
    out = L.nnls_bpp_batched(cuda(G), cuda(R), mask_in=mi)
    ref = oracle.bpp_batched(G, R.astype(np.float64), mask_in=cold[1])
    compare_bpp(G, R, out, ref)
    r = out[2].cpu().numpy()
    assert np.all(r[cold[1] != 0] == 1)
    # adversarial warm start with a one-round budget: falls back to cold
    bad = (~cold[1]) & np.uint64((1 << k) - 1)
    out = L.nnls_bpp_batched(cuda(G), cuda(R), mask_in=cuda(bad.view(np.int64)), warm_cap=1)
    ref = oracle.bpp_batched(G, R.astype(np.float64), mask_in=bad, warm_cap=1)
    compare_bpp(G, R, out, ref)
    assert np.any(out[3].cpu().numpy() & L.NMF_BPP_WARM_FALLBACK)
    np.testing.assert_allclose(out[0].cpu().numpy(), cold[0], rtol=1e-5, atol=1e-7)


def test_bpp_in_place_masks_and_counters():
    rng = np.random.default_rng(7)
    k, batch = 20, 5000
    G, R = nmf_like_problems(rng, k, batch)
    masks = torch.zeros(batch, dtype=torch.int64, device="cuda")
    cnt = torch.zeros(L.NMF_BPP_COUNTERS, dtype=torch.int64, device="cuda")
    X1, _, r1, _ = L.nnls_bpp_batched(cuda(G), cuda(R), mask_in=masks, mask_out=masks, counters=cnt)
    c1 = cnt.cpu().numpy().copy()
    ref = oracle.bpp_batched(G, R.astype(np.float64))
    assert c1[0] == ref[2].sum()
    assert np.array_equal(masks.cpu().numpy().view(np.uint64), ref[1])
    # second call warm-starts from the stored masks in place: one round each
    X2, _, r2, _ = L.nnls_bpp_batched(cuda(G), cuda(R), mask_in=masks, mask_out=masks, counters=cnt)
    r2 = r2.cpu().numpy()
    assert np.all(r2[ref[1] != 0] == 1)
    np.testing.assert_allclose(X2.cpu().numpy(), X1.cpu().numpy(), rtol=1e-6, atol=1e-9)


# ------------------------------------------------------------ objective ----
def test_objective_dense_direct_and_trace():
    rng = np.random.default_rng(8)
    m, n, k = 1000, 777, 30
    A = rng.uniform(0.0, 1.0, (m, n)).astype(np.float32)
    W = rng.uniform(0.0, 0.2, (m, k)).astype(np.float32)
    Ht = rng.uniform(0.0, 0.2, (n, k)).astype(np.float32)
    M = L.Matrix(dense=cuda(A))
    out = L.nmf_objective(M, cuda(W), cuda(Ht)).cpu().numpy()
    fa, fr = oracle.objective_dense(A, W, Ht)
    assert abs(out[2] - fa) <= 1e-12 * fa
    assert abs(out[1] - fr) <= 1e-6 * fr
    assert abs(out[0] - np.sqrt(fr / fa)) <= 1e-6
    GW = L.nmf_gram(cuda(W))
    GH = L.nmf_gram(cuda(Ht))
    RH = L.nmf_rhs_dense(L.NMF_SIDE_H, cuda(A), cuda(W))
    out2 = L.nmf_objective(M, cuda(W), cuda(Ht), L.NMF_OBJ_TRACE, GW, GH, RH).cpu().numpy()
    assert abs(out2[0] - np.sqrt(fr / fa)) <= 1e-5


def test_objective_csr():
    m, n, k = 2000, 1500, 20
    rp, ci, va = C.sparse_csr(21, m, n, 5e-3)
    rpt, cit, vat = C.csr_transpose(m, n, rp, ci, va)
    rng = np.random.default_rng(9)
    W = rng.uniform(0.0, 0.3, (m, k)).astype(np.float32)
    Ht = rng.uniform(0.0, 0.3, (n, k)).astype(np.float32)
    M = L.Matrix(csr=(cuda(rp), cuda(ci), cuda(va)), csr_t=(cuda(rpt), cuda(cit), cuda(vat)), shape=(m, n))
    out = L.nmf_objective(M, cuda(W), cuda(Ht)).cpu().numpy()
    fa, fr = oracle.objective_csr(m, n, rp, ci, va, W, Ht)
    assert abs(out[2] - fa) <= 1e-12 * fa
    assert abs(out[1] - fr) <= 1e-9 * (fa + abs(fr))
    assert abs(M.fro2.item() - fa) <= 1e-12 * fa


# ----------------------------------------------------------- BF16x3 RHS ----
from oracle import split as osplit  # noqa: E402


@pytest.mark.parametrize("m,n,k,pad", [(200, 150, 5, 0), (257, 131, 30, 0), (129, 1000, 50, 1), (33, 4097, 64, 0),
                                       (1000, 999, 33, 3), (70000, 300, 30, 0), (20000, 2400, 30, 8),
                                       (40000, 700, 50, 0), (70000, 700, 30, 0)])
def test_rhs_dense_bf16x3(m, n, k, pad):
    """Bound: each of the 3L BF16 products is exact in FP32 and the chain is
    accumulated in FP32, so |R - oracle| <= 3 L 2^-24 (|A||Y|) (1 + small).
    The sizes give blocks with 1 to 13 chunks of the contraction: the single-
    staging loop, and the two-staging main loop with its two- and three-chunk
    tails, for one and two 32-column tiles of k."""
    rng = np.random.default_rng(3 * m + n + k)
    A = rng.uniform(0.0, 1.0, (m, n)).astype(np.float32)
    Ht = rng.uniform(0.0, 1.0, (n, k)).astype(np.float32)
    W = rng.uniform(0.0, 1.0, (m, k)).astype(np.float32)
    Ad = padded(A, pad)
    bt = L.nmf_split_bf16(Ad)
    btt = L.nmf_split_bf16(Ad, transpose=True)
    hb, lb = osplit.split_bits(A)
    hi, lo = L.unpack_bf16(bt, m, n)
    assert np.array_equal(hi, hb) and np.array_equal(lo, lb)
    hit, lot = L.unpack_bf16(btt, n, m)
    assert np.array_equal(hit, hb.T) and np.array_equal(lot, lb.T)
    A64 = np.abs(A.astype(np.float64))
    Rw = L.nmf_rhs_dense(L.NMF_SIDE_W, None, cuda(Ht), prec=L.NMF_BF16X3, B_bf16=bt, m=m, n=n)
    Rwo = osplit.rhs_w(A, Ht)
    bw = 1.01 * 3 * n * U32 * (A64 @ np.abs(Ht.astype(np.float64)))
    err = np.abs(Rw.cpu().numpy().astype(np.float64) - Rwo)
    assert np.all(err <= bw), np.max(err / bw)
    Rh = L.nmf_rhs_dense(L.NMF_SIDE_H, None, cuda(W), prec=L.NMF_BF16X3, B_bf16=btt, m=m, n=n)
    Rho = osplit.rhs_h(A, W)
    bh = 1.01 * 3 * (m + 1) * U32 * (A64.T @ np.abs(W.astype(np.float64)))
    err = np.abs(Rh.cpu().numpy().astype(np.float64) - Rho)
    assert np.all(err <= bh), np.max(err / bh)
    # and against the exact product: the dropped lo*lo term and the split error
    exact = A.astype(np.float64) @ Ht.astype(np.float64)
    bex = (3 * 2.0 ** -16 + 3.03 * n * U32) * (A64 @ np.abs(Ht.astype(np.float64)))
    assert np.all(np.abs(Rw.cpu().numpy() - exact) <= bex)
