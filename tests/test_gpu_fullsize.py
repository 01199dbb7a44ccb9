"""Parity at the full workload sizes, in the launch configurations bench.py
times, on outputs the FP64 oracle can compute one by one (sampled rows and
columns regenerated on the host from the seeded recipes), and whole-run
trajectories against stored oracle runs.

Bounds (from the arithmetic):
  Gram   FP64 sums of exact FP32 products:  |dG| <= rows 2^-52 (|X|^T |X|)
  RHS    |R - R_exact(operands)| <= terms 2^-24 (|A| |Y|), terms = the
         longest FP32 accumulation of the launch (nmf_rhs_dense_chain); the
         operands are FP32 A, Y or, for BF16x3, the three BF16 products
  CSR    bit-identical (FP64 accumulation in storage order, one rounding)
  BPP    same (G, R) on both sides: |dx| <= 4 ulp32(x) + 1e-9 max|x|, masks
         equal except at degenerate indices
  ANLS   |r_gpu - r_oracle| <= 1e-5 after every iteration from the same start
"""
import json
import os
import sys

import numpy as np
import pytest
import torch

import oracle
from nmf_inputs import configs as C
from nmf_inputs import device as gen
from nmf_inputs.philox import uniform_at
from oracle import split as osplit
from paper_1509_09313_amd import binding as L

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)
import bench  # noqa: E402

U32 = 2.0 ** -24
TOL_R = 1e-5


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check_bound(got, ref, bound, label):
    err = np.abs(np.asarray(got, np.float64) - ref)
    worst = float(np.max(err / np.maximum(bound, 1e-300)))
    print(f"{label}: max err / bound = {worst:.3e}")
    assert np.all(err <= bound), label


# ----------------------------------------------------------- video 1e6 x 2400
@pytest.fixture(scope="module")
def video():
    seed, m, n, k = C.seed_for(5), 1_000_000, 2_400, 30
    A = gen.video(seed, m, n)
    W0, Ht0 = gen.init_factors(seed, m, n, k)
    M = L.Matrix(dense=A, split=True)
    torch.cuda.synchronize()
    yield {"seed": seed, "m": m, "n": n, "k": k, "A": A, "W0": W0, "Ht0": Ht0, "M": M}
    del M, A
    torch.cuda.empty_cache()


def test_video_full_products_sampled(video):
    seed, m, n, k = video["seed"], video["m"], video["n"], video["k"]
    A, M = video["A"], video["M"]
    W0h, H0h = C.init_w(seed, m, k), C.init_ht(seed, n, k)
    assert np.array_equal(video["Ht0"].cpu().numpy(), H0h)
    # Gram matrices of both factors, whole
    for X, Xh, label in ((video["Ht0"], H0h, "G_H"), (video["W0"], W0h, "G_W")):
        G = L.nmf_gram(X).cpu().numpy()
        Xa = np.abs(Xh.astype(np.float64))
        check_bound(G, oracle.gram(Xh), 1.01 * Xh.shape[0] * 2.0 ** -52 * (Xa.T @ Xa), label)
    bt, btt = M.tiled
    rng = np.random.default_rng(11)
    rows = np.concatenate([[0, 1, m - 1], rng.choice(m, 45, replace=False)])
    Ar = C.video_rows(seed, n, rows)
    assert np.array_equal(Ar, A[cuda(rows)].cpu().numpy())
    absY = np.abs(H0h.astype(np.float64))
    # A H^T rows, FP32 and BF16x3, in the launch configuration of the full matrix
    Rf = L.nmf_rhs_dense(L.NMF_SIDE_W, A, video["Ht0"])[cuda(rows)].cpu().numpy()
    tf = L.rhs_dense_chain(L.NMF_SIDE_W, m, n, k, L.NMF_F32)
    check_bound(Rf, oracle.rhs_dense_w(Ar, H0h), 1.01 * tf * U32 * (np.abs(Ar.astype(np.float64)) @ absY), "R_W fp32")
    Rb = L.nmf_rhs_dense(L.NMF_SIDE_W, None, video["Ht0"], prec=L.NMF_BF16X3, B_bf16=bt, m=m, n=n)
    Rb = Rb[cuda(rows)].cpu().numpy()
    tb = L.rhs_dense_chain(L.NMF_SIDE_W, m, n, k, L.NMF_BF16X3)
    check_bound(Rb, osplit.rhs_w(Ar, H0h), 1.02 * tb * U32 * (np.abs(Ar.astype(np.float64)) @ absY), "R_W bf16x3")
    # A^T W columns: whole columns of A regenerated on the host
    cols = np.array([0, 1, 1234, n - 1])
    Ac = C.video_rows(seed, n, np.arange(m), cols)
    absW = np.abs(W0h.astype(np.float64))
    RHf = L.nmf_rhs_dense(L.NMF_SIDE_H, A, video["W0"])[cuda(cols)].cpu().numpy()
    tf = L.rhs_dense_chain(L.NMF_SIDE_H, m, n, k, L.NMF_F32)
    bound = 1.01 * tf * U32 * (np.abs(Ac.astype(np.float64)).T @ absW)
    check_bound(RHf, oracle.rhs_dense_h(Ac, W0h), bound, "R_H fp32")
    RHb = L.nmf_rhs_dense(L.NMF_SIDE_H, None, video["W0"], prec=L.NMF_BF16X3, B_bf16=btt, m=m, n=n)
    RHb = RHb[cuda(cols)].cpu().numpy()
    tb = L.rhs_dense_chain(L.NMF_SIDE_H, m, n, k, L.NMF_BF16X3)
    bound = 1.02 * tb * U32 * (np.abs(Ac.astype(np.float64)).T @ absW)
    check_bound(RHb, osplit.rhs_h(Ac, W0h), bound, "R_H bf16x3")
    print(f"accumulation chains: fp32 side H {tf}, bf16x3 side W {L.rhs_dense_chain(0, m, n, k, 1)} side H {tb}")


@pytest.mark.parametrize("k", [50, 64])
def test_video_full_products_wide_k(video, k):
    """The two-tile (k > 32) product kernels at full size: sampled rows of
    A H^T and whole columns of A^T W, FP32 and BF16x3, within the chain
    bounds, for k = 50 (ragged second tile) and k = 64."""
    seed, m, n = video["seed"], video["m"], video["n"]
    A, M = video["A"], video["M"]
    bt, btt = M.tiled
    W0, Ht0 = gen.init_factors(seed, m, n, k)
    # the seeded device generator's factors (bit-identical to the host
    # recipe, checked here on sampled rows) are the oracle's inputs too
    W0h, H0h = W0.cpu().numpy(), C.init_ht(seed, n, k)
    assert np.array_equal(Ht0.cpu().numpy(), H0h)
    probe = np.array([0, 1, 4097, m - 1])
    assert np.array_equal(W0h[probe], C.init_w(seed, m, k, rows=probe))
    rng = np.random.default_rng(12)
    rows = np.concatenate([[0, m - 1], rng.choice(m, 30, replace=False)])
    Ar = C.video_rows(seed, n, rows)
    absY = np.abs(H0h.astype(np.float64))
    for prec, tag in ((L.NMF_F32, "fp32"), (L.NMF_BF16X3, "bf16x3")):
        if prec == L.NMF_F32:
            R = L.nmf_rhs_dense(L.NMF_SIDE_W, A, Ht0)
            ref, slack = oracle.rhs_dense_w(Ar, H0h), 1.01
        else:
            R = L.nmf_rhs_dense(L.NMF_SIDE_W, None, Ht0, prec=prec, B_bf16=bt, m=m, n=n)
            ref, slack = osplit.rhs_w(Ar, H0h), 1.02
        t = L.rhs_dense_chain(L.NMF_SIDE_W, m, n, k, prec)
        check_bound(R[cuda(rows)].cpu().numpy(), ref, slack * t * U32 * (np.abs(Ar.astype(np.float64)) @ absY),
                    f"R_W {tag} k={k}")
    cols = np.array([0, 777, n - 1])
    Ac = C.video_rows(seed, n, np.arange(m), cols)
    absW = np.abs(W0h.astype(np.float64))
    for prec, tag in ((L.NMF_F32, "fp32"), (L.NMF_BF16X3, "bf16x3")):
        if prec == L.NMF_F32:
            R = L.nmf_rhs_dense(L.NMF_SIDE_H, A, W0)
            ref, slack = oracle.rhs_dense_h(Ac, W0h), 1.01
        else:
            R = L.nmf_rhs_dense(L.NMF_SIDE_H, None, W0, prec=prec, B_bf16=btt, m=m, n=n)
            ref, slack = osplit.rhs_h(Ac, W0h), 1.02
        t = L.rhs_dense_chain(L.NMF_SIDE_H, m, n, k, prec)
        check_bound(R[cuda(cols)].cpu().numpy(), ref, slack * t * U32 * (np.abs(Ac.astype(np.float64)).T @ absW),
                    f"R_H {tag} k={k}")


def test_video_full_bpp_launch():
    """The W-side NNLS launch at its full size (10^6 problems, k = 30) on
    host-made problems shaped like the workload's (G from the initial Ht,
    right-hand sides G w* - e with w* mostly positive), checked on sampled
    problems against the oracle and everywhere by the KKT conditions."""
    seed, m, n, k = C.seed_for(5), 1_000_000, 2_400, 30
    H0h = C.init_ht(seed, n, k)
    G = oracle.gram(H0h)
    b = np.arange(m)
    wstar = uniform_at(seed, C.mid(C.MID_VAL, 7), b[:, None], np.arange(k)[None, :]).astype(np.float64)
    wstar[wstar < 0.05] = 0.0                              # about 5% of indices active
    noise = uniform_at(seed, C.mid(C.MID_VAL, 8), b[:, None], np.arange(k)[None, :]).astype(np.float64)
    R = (wstar @ G - 0.5 * np.diag(G)[None, :] * noise * (wstar == 0.0)).astype(np.float32)
    X, masks, rounds, status = L.nnls_bpp_batched(cuda(G), cuda(R))
    X = X.cpu().numpy()
    masks = masks.cpu().numpy().view(np.uint64)
    st = status.cpu().numpy()
    assert np.all(st & L.NMF_BPP_CAPPED == 0)
    rng = np.random.default_rng(5)
    sample = np.concatenate([[0, m - 1], rng.choice(m, 3000, replace=False)])
    Xo, Mo, _, _ = oracle.bpp_batched(G, R[sample].astype(np.float64))
    tol = 4 * np.spacing(np.abs(Xo).astype(np.float32)).astype(np.float64) + 1e-9 * np.max(np.abs(Xo))
    assert np.all(np.abs(X[sample] - Xo) <= tol)
    agree = float(np.mean(masks[sample] == Mo))
    print(f"sampled masks equal: {agree:.5f}; mean rounds {rounds.float().mean().item():.3f}")
    assert agree >= 0.999
    # KKT everywhere (computed here from the returned X): x >= 0, y >= -tol off
    # the support, complementarity
    Gd, Xd, Rd = cuda(G), cuda(X.astype(np.float64)), cuda(R.astype(np.float64))
    Y = Xd @ Gd - Rd
    scale = (Xd.abs() @ Gd.abs() + Rd.abs()).max(dim=1, keepdim=True).values
    assert float(Xd.min()) >= 0.0
    assert float((Y / scale).min()) >= -1e-6
    assert float(((Xd * Y).abs() / scale).max()) <= 1e-6


def _golden_video():
    with open(os.path.join(HERE, "golden", "video_1e6x2400_k30_oracle.json")) as fh:
        return json.load(fh)


def _run(M, k, W0, Ht0, iters, **kw):
    W, Ht = W0.clone(), Ht0.clone()
    stats = L.new_stats(iters)
    L.nmf_anls_iter(M, k, W, Ht, iters, L.make_opts(**kw), stats)
    return W, Ht, L.decode_stats(stats)


def test_video_full_trajectories(video):
    """50 iterations at full size, plain FP32 and BF16x3 cold, every
    iteration against the FP64 oracle's run of the same 50 iterations."""
    ref = _golden_video()
    M, k = video["M"], video["k"]
    for prec, label in ((L.NMF_F32, "fp32"), (L.NMF_BF16X3, "bf16x3")):
        W, Ht, st = _run(M, k, video["W0"], video["Ht0"], 50, prec=prec)
        rf = np.array([s["r_full"] for s in st])
        rh = np.array([s["r_half"] for s in st])
        dr = max(np.max(np.abs(rf - ref["r_full"])), np.max(np.abs(rh - ref["r_half"])))
        r_direct = float(L.nmf_objective(M, W, Ht)[0])
        agree = bench.passive_set_agreement(W, Ht, ref, k)
        print(f"{label}: max |dr| over 50 iterations {dr:.2e}; final direct r {r_direct:.10f} "
              f"oracle {ref['r_full'][-1]:.10f}; support agreement W {agree['w']['agreement']:.6f} "
              f"H {agree['h']['agreement']:.6f}")
        assert dr <= TOL_R
        assert abs(r_direct - ref["r_full"][-1]) <= TOL_R
        assert all(s["capped"] == 0 for s in st)
        # final supports against the oracle's on every 1000th row of W and every row of H^T
        assert agree["w"]["agreement"] >= 0.999 and agree["h"]["agreement"] >= 0.999


def test_video_full_learned_form():
    """The bench's learned + BF16x3 configuration (5 cold iterations that
    collect samples, network training on the GPU, 45 warm-started iterations):
    the same trajectory as the oracle, and what the trained networks' start
    sets save against the trivial starts over the same 45 iterations.

    Measured on this workload the W-side network predicts the full set (every
    index passive) for every row: it needs as many passive-set solves as the
    full-set start and saves the empty start's free first round, but the
    previous iteration's sets need fewer solves still.  The asserts hold
    exactly that: no more solves than the full-set start, fewer KKT rounds
    than the empty start, and no more solves than the empty start."""
    a = bench.parse([])
    B = bench.Bench(a)
    B.learned_step()
    torch.cuda.synchronize()
    ref = _golden_video()
    st = L.decode_stats(B.st1) + L.decode_stats(B.st2)
    rf = np.array([s["r_full"] for s in st])
    dr = np.max(np.abs(rf - ref["r_full"]))
    r_final = B.final_r()
    assert dr <= TOL_R and abs(r_final - ref["r_full"][-1]) <= TOL_R
    assert sum(s["capped"] for s in st) == 0
    T0 = a.cold_iters

    def tot(stats, side, c):
        return sum(s[side][c] for s in stats[T0:])

    runs = {}
    for name, warm in (("cold", L.NMF_WARM_COLD), ("full_set", L.NMF_WARM_ALL), ("prev", L.NMF_WARM_PREV)):
        _, _, runs[name] = _run(B.M, a.k, B.W0, B.Ht0, a.iters, prec=L.NMF_BF16X3, warm=warm)
        assert max(abs(s["r_full"] - r) for s, r in zip(runs[name], ref["r_full"])) <= TOL_R
    fb = sum(s["fallback"] for s in st)
    line = [f"learned W solves {tot(st, 'bpp_w', 1)} rounds {tot(st, 'bpp_w', 0)}"]
    for name, r in runs.items():
        line.append(f"{name} W solves {tot(r, 'bpp_w', 1)} rounds {tot(r, 'bpp_w', 0)}")
    print(f"learned: max |dr| {dr:.2e}, final r {r_final:.10f}, fallbacks {fb}; iterations {T0 + 1}-{a.iters}: "
          + "; ".join(line))
    assert fb == 0
    assert tot(st, "bpp_w", 1) <= 1.001 * tot(runs["full_set"], "bpp_w", 1)
    assert tot(st, "bpp_w", 1) <= tot(runs["cold"], "bpp_w", 1)
    assert tot(st, "bpp_w", 0) < tot(runs["cold"], "bpp_w", 0)


# --------------------------------------------------- planted 172800 x 115200
def test_planted_full_sampled():
    """The dense planted workload at full size (A is 79.6 GB in FP32): FP32
    products on sampled rows and columns, then one ANLS iteration with the
    W-side solutions of sampled rows against the oracle's (its own G and R)."""
    seed, m, n, k = C.seed_for(2), 172_800, 115_200, 50
    A = gen.planted(seed, m, n, k)
    W0, Ht0 = gen.init_factors(seed, m, n, k)
    H0h = C.init_ht(seed, n, k)
    try:
        GH = L.nmf_gram(Ht0).cpu().numpy()
        Ha = np.abs(H0h.astype(np.float64))
        GHo = oracle.gram(H0h)
        check_bound(GH, GHo, 1.01 * n * 2.0 ** -52 * (Ha.T @ Ha), "G_H")
        rng = np.random.default_rng(2)
        rows = np.concatenate([[0, m - 1], rng.choice(m, 14, replace=False)])
        Ar = C.planted_rows(seed, n, k, rows)
        assert np.array_equal(Ar, A[cuda(rows)].cpu().numpy())
        RW = L.nmf_rhs_dense(L.NMF_SIDE_W, A, Ht0)
        tf = L.rhs_dense_chain(L.NMF_SIDE_W, m, n, k, L.NMF_F32)
        RWo = oracle.rhs_dense_w(Ar, H0h)
        check_bound(RW[cuda(rows)].cpu().numpy(), RWo, 1.01 * tf * U32 * (np.abs(Ar.astype(np.float64)) @ Ha),
                    "R_W fp32")
        cols = np.array([0, 77, n - 1])
        Ac = C.planted_rows(seed, n, k, np.arange(m), cols=cols)
        W0h = C.init_w(seed, m, k)
        RH = L.nmf_rhs_dense(L.NMF_SIDE_H, A, W0)[cuda(cols)].cpu().numpy()
        th = L.rhs_dense_chain(L.NMF_SIDE_H, m, n, k, L.NMF_F32)
        check_bound(RH, oracle.rhs_dense_h(Ac, W0h),
                    1.01 * th * U32 * (np.abs(Ac.astype(np.float64)).T @ np.abs(W0h.astype(np.float64))), "R_H fp32")
        # one full iteration; the W rows of the sample must satisfy Eq. KKT for
        # the oracle's own G_H and right-hand sides, up to the difference
        # between those and the GPU's (the FP32 product bound above)
        M = L.Matrix(dense=A)
        W, Ht, st = _run(M, k, W0, Ht0, 1, prec=L.NMF_F32)
        X = W[cuda(rows)].cpu().numpy().astype(np.float64)
        Y = X @ GHo - RWo
        bnd = 1.01 * tf * U32 * (np.abs(Ar.astype(np.float64)) @ Ha) + 1e-9 * (np.abs(X) @ np.abs(GHo) + np.abs(RWo))
        on = X > 0
        print(f"planted full: KKT on sampled W rows, max |y| on support / bound "
              f"{float(np.max(np.abs(Y[on]) / bnd[on])):.3e}, min y off support / bound "
              f"{float(np.min(Y[~on] / bnd[~on])) if (~on).any() else 0.0:.3e}; "
              f"r after 1 iteration {st[0]['r_full']:.6f} (half {st[0]['r_half']:.6f})")
        assert np.all(X >= 0.0)
        assert np.all(np.abs(Y[on]) <= bnd[on])
        assert np.all(Y[~on] >= -bnd[~on])
        assert st[0]["r_full"] <= st[0]["r_half"] + 1e-6 and st[0]["capped"] == 0
        # BF16x3 products on the same rows and columns (the planes of A and
        # A^T: 159 GB more), in the launch configuration of the benchmark's
        # --dense form (split contraction, whole rounds of workgroups)
        del M, W, Ht
        M = L.Matrix(dense=A, split=True)
        bt, btt = M.tiled
        RWb = L.nmf_rhs_dense(L.NMF_SIDE_W, None, Ht0, prec=L.NMF_BF16X3, B_bf16=bt, m=m, n=n)
        tb = L.rhs_dense_chain(L.NMF_SIDE_W, m, n, k, L.NMF_BF16X3)
        check_bound(RWb[cuda(rows)].cpu().numpy(), osplit.rhs_w(Ar, H0h),
                    1.02 * tb * U32 * (np.abs(Ar.astype(np.float64)) @ Ha), "R_W bf16x3")
        RHb = L.nmf_rhs_dense(L.NMF_SIDE_H, None, W0, prec=L.NMF_BF16X3, B_bf16=btt, m=m, n=n)[cuda(cols)]
        tbh = L.rhs_dense_chain(L.NMF_SIDE_H, m, n, k, L.NMF_BF16X3)
        check_bound(RHb.cpu().numpy(), osplit.rhs_h(Ac, W0h),
                    1.02 * tbh * U32 * (np.abs(Ac.astype(np.float64)).T @ np.abs(W0h.astype(np.float64))),
                    "R_H bf16x3")
        del M, RWb, RHb
    finally:
        del A
        torch.cuda.empty_cache()


# ------------------------------------------------------- sparse 207360 x 138240
def test_sparse_full_sampled():
    """The CSR workload at full size (density 1e-3, 28.7 M nonzeros): both
    SpMM products bit-identical to the oracle on sampled rows, and the
    W-side NNLS of sampled rows after one iteration against the oracle."""
    seed, m, n, k = C.seed_for(3), 207_360, 138_240, 50
    rp, ci, va = C.sparse_csr(seed, m, n, 1e-3)
    rpt, cit, vat = C.csr_transpose(m, n, rp, ci, va)
    d = [cuda(x) for x in (rp, ci, va, rpt, cit, vat)]
    W0, Ht0 = gen.init_factors(seed, m, n, k)
    H0h, W0h = C.init_ht(seed, n, k), C.init_w(seed, m, k)
    rng = np.random.default_rng(3)
    rows = np.concatenate([[0, m - 1], rng.choice(m, 200, replace=False)])
    cols = np.concatenate([[0, n - 1], rng.choice(n, 200, replace=False)])

    def sub(rowptr, colidx, vals, pick):
        lo, hi = rowptr[pick], rowptr[pick + 1]
        idx = np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)])
        return np.concatenate([[0], np.cumsum(hi - lo)]).astype(np.int64), colidx[idx], vals[idx]

    RW = L.nmf_rhs_csr(d[0], d[1], d[2], Ht0, m, n).cpu().numpy()
    RWo = oracle.rhs_csr(*sub(rp, ci, va, rows), H0h)
    assert np.array_equal(RW[rows], RWo.astype(np.float32))
    RH = L.nmf_rhs_csr(d[3], d[4], d[5], W0, n, m).cpu().numpy()
    assert np.array_equal(RH[cols], oracle.rhs_csr(*sub(rpt, cit, vat, cols), W0h).astype(np.float32))
    M = L.Matrix(csr=(d[0], d[1], d[2]), csr_t=(d[3], d[4], d[5]), shape=(m, n))
    W, Ht, st = _run(M, k, W0, Ht0, 1, prec=L.NMF_F32)
    GHo = oracle.gram(H0h)
    Xo, Mo, _, _ = oracle.bpp_batched(GHo, RWo.astype(np.float32).astype(np.float64))
    Xg = W[cuda(rows)].cpu().numpy().astype(np.float64)
    tol = 4 * np.spacing(np.abs(Xo).astype(np.float32)).astype(np.float64) + 1e-9 * np.max(np.abs(Xo))
    bad = np.abs(Xg - Xo) > tol
    print(f"sparse full: W rows outside 4 ulp: {int(bad.sum())} of {bad.size}; "
          f"r after 1 iteration {st[0]['r_full']:.6f}")
    # the only difference between the two sides is the FP64 summation order of
    # G_H, which moves solutions by far less than 4 ulp32
    assert not bad.any()
    assert st[0]["capped"] == 0


def test_csr_gather_beyond_4gib():
    """A factor Y above 4 GiB (16.8 M rows x 64 floats) takes the global-load
    gather path (buffer offsets are 32-bit): bit-identical to the oracle on
    rows whose entries reach the top of Y."""
    rows, cols, k, per_row = 2000, 16_800_000, 64, 40
    rng = np.random.default_rng(4)
    lists = [np.unique(rng.integers(0, cols, per_row)) for _ in range(rows)]
    lists[0] = np.array([0, cols - 1])
    lists[1] = np.arange(cols - 300, cols)
    lists[2] = np.array([], dtype=np.int64)
    rp = np.concatenate([[0], np.cumsum([len(x) for x in lists])]).astype(np.int64)
    ci = np.concatenate(lists).astype(np.int32)
    va = rng.uniform(0.0, 1.0, len(ci)).astype(np.float32)
    g = torch.Generator(device="cuda")
    g.manual_seed(4)
    Y = torch.rand((cols, k), generator=g, device="cuda")
    assert Y.numel() * 4 > 2 ** 32
    R = L.nmf_rhs_csr(cuda(rp), cuda(ci), cuda(va), Y, rows, cols).cpu().numpy()
    used, inv = np.unique(ci, return_inverse=True)
    Ysub = Y[cuda(used.astype(np.int64))].cpu().numpy().astype(np.float64)
    del Y
    torch.cuda.empty_cache()
    ref = oracle.rhs_csr(rp, inv.astype(np.int32), va, Ysub).astype(np.float32)
    assert np.array_equal(R, ref)


@pytest.mark.parametrize("solver", ["hals", "mu"])
def test_video_full_local_trajectory(video, solver):
    """Algorithm 1 with the HALS or MU update at full size, 50 iterations with
    BF16x3 right-hand sides (the benchmark's form), against the stored FP64
    oracle run (tests/golden/video_1e6x2400_k30_local_oracle.json): the trace
    objective after every half-step and the direct one at the end."""
    path = os.path.join(HERE, "golden", "video_1e6x2400_k30_local_oracle.json")
    with open(path) as fh:
        ref = json.load(fh)[solver]
    k, M = video["k"], video["M"]
    code = {"hals": L.NMF_SOLVER_HALS, "mu": L.NMF_SOLVER_MU}[solver]
    W, Ht = video["W0"].clone(), video["Ht0"].clone()
    T = len(ref["r_full"])
    st = L.new_stats(T)
    L.Anls(M, k, L.make_opts(prec=L.NMF_BF16X3, trace=True, solver=code)).run(W, Ht, T, st)
    torch.cuda.synchronize()
    dec = L.decode_stats(st)
    dh = np.abs(np.array([s["r_half"] for s in dec]) - ref["r_half"])
    df = np.abs(np.array([s["r_full"] for s in dec]) - ref["r_full"])
    direct = float(L.nmf_objective(M, W, Ht)[0])
    print(f"{solver}: r_50 {ref['r_full'][-1]:.10f}, max |dr| trace {max(dh.max(), df.max()):.2e}, "
          f"direct {abs(direct - ref['r_full'][-1]):.2e}")
    assert max(dh.max(), df.max()) <= TOL_R
    assert abs(direct - ref["r_full"][-1]) <= TOL_R


@pytest.mark.parametrize("k", [10, 20, 40, 50])
def test_video_full_ksweep(video, k):
    """The ranks of the paper's algorithmic comparison (k = 10..50; k = 30 is
    covered above) at full size: 10 cold-BPP iterations with FP32 and BF16x3
    right-hand sides against the stored FP64 oracle runs
    (tests/golden/video_1e6x2400_ksweep_oracle.json), every half-step."""
    with open(os.path.join(HERE, "golden", "video_1e6x2400_ksweep_oracle.json")) as fh:
        gold = json.load(fh)
    ref, T = gold["k"][str(k)], gold["iterations"]
    M = video["M"]
    W0, Ht0 = gen.init_factors(video["seed"], video["m"], video["n"], k)
    for prec, label in ((L.NMF_F32, "fp32"), (L.NMF_BF16X3, "bf16x3")):
        W, Ht, st = _run(M, k, W0, Ht0, T, prec=prec)
        rf = np.array([s["r_full"] for s in st])
        rh = np.array([s["r_half"] for s in st])
        dr = max(np.max(np.abs(rf - ref["r_full"])), np.max(np.abs(rh - ref["r_half"])))
        r_direct = float(L.nmf_objective(M, W, Ht)[0])
        print(f"k={k} {label}: max |dr| over {T} iterations {dr:.2e}; final direct r {r_direct:.10f} "
              f"oracle {ref['r_full'][-1]:.10f}")
        assert dr <= TOL_R
        assert abs(r_direct - ref["r_full"][-1]) <= TOL_R
        assert all(s["capped"] == 0 for s in st)
        del W, Ht
