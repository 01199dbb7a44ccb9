"""Many uneven instances at once (nmf_batch_*): the grouped persistent phase
kernels, graph capture and the autotuner, through the C-ABI, against the FP64
oracle per instance.

Parity bar: after the same iterations from the same initial factors, every
instance's relative objective ||A - WH||_F / ||A||_F (direct form) is within
1e-5 of the oracle's (BF16x3 right-hand sides, FP64 Gram and BPP)."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from nmf_inputs import configs as C
from nmf_inputs import device as gen
from paper_1509_09313_amd import binding as L

pytestmark = pytest.mark.gpu

TOL_R = 1e-5
HERE = os.path.dirname(os.path.abspath(__file__))

# ragged shapes: tiles of 128 / 64 rows with tails, every BPP class
# (k -> K: 1, 8 -> 8; 10, 16 -> 16; 20, 30 -> 32; 33, 50 -> 56; 64 -> 64)
# and both BF16 widths (k <= 32, k > 32)
SMALL = [(300, 200, 10), (130, 70, 20), (777, 513, 50), (200, 129, 8), (1000, 300, 33),
         (257, 600, 64), (513, 140, 16), (90, 300, 1), (2048, 256, 30), (640, 1280, 20)]


def build(shapes, seed, inst0=0):
    probs, host = [], []
    for i, (m, n, k) in enumerate(shapes):
        A = gen.planted(seed, m, n, k, 0.01, inst=inst0 + i)
        W, Ht = gen.init_factors(seed, m, n, k, inst=inst0 + i)
        probs.append({"A": A, "W": W, "Ht": Ht})
        host.append((m, n, k))
    return probs, host


def direct_r(pr):
    M = L.Matrix(dense=pr["A"])
    return float(L.nmf_objective(M, pr["W"], pr["Ht"])[0])


def test_batched_small_trajectory_vs_oracle():
    seed = C.seed_for(4) + 1000
    probs, shapes = build(SMALL, seed)
    T = 5
    refs = []
    for i, (m, n, k) in enumerate(shapes):
        A = C.planted_dense(seed, m, n, k, 0.01, inst=i)
        assert np.array_equal(A, probs[i]["A"].cpu().numpy())
        refs.append(oracle.anls(k, C.init_w(seed, m, k, inst=i), C.init_ht(seed, n, k, inst=i), T, dense=A))
    b = L.Batch(probs)
    counters = torch.zeros(2 * L.NMF_BPP_COUNTERS, dtype=torch.int64, device="cuda")
    worst = 0.0
    for t in range(T):
        b.iterate(1, counters)
        torch.cuda.synchronize()
        for i, pr in enumerate(probs):
            d = abs(direct_r(pr) - refs[i]["r_full"][t])
            worst = max(worst, d)
            assert d <= TOL_R, (i, shapes[i], t, d)
    c = counters.cpu().numpy()
    print(f"max |dr| {worst:.3e}; BPP rounds W {c[0]} H {c[L.NMF_BPP_COUNTERS]}")
    assert c[0] >= sum(m for m, _, _ in shapes) * T
    b.close()


def test_batched_graph_replays_match_eager():
    seed = C.seed_for(4) + 2000
    probs, shapes = build(SMALL[:6], seed)
    H0 = [pr["Ht"].clone() for pr in probs]
    T = 4
    b = L.Batch(probs)
    b.iterate(T, reset=True)
    torch.cuda.synchronize()
    eager = [(pr["W"].clone(), pr["Ht"].clone()) for pr in probs]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = b.graph(T)
    s.synchronize()
    for rep in range(3):
        for pr, h0 in zip(probs, H0):      # eager work between replays
            pr["Ht"].copy_(h0)
            pr["W"].zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            b.launch(g)
        s.synchronize()
        for i, pr in enumerate(probs):
            assert torch.equal(pr["W"], eager[i][0]), (rep, i)
            assert torch.equal(pr["Ht"], eager[i][1]), (rep, i)
    b.close()


def test_batched_autotune_restores_and_agrees():
    seed = C.seed_for(4) + 3000
    probs, shapes = build(SMALL, seed)
    before = [(pr["W"].clone(), pr["Ht"].clone()) for pr in probs]
    b = L.Batch(probs)
    best, ms = b.autotune()
    torch.cuda.synchronize()
    print("tuned", best.as_dict(), f"{ms:.3f} ms/iteration")
    assert ms > 0.0
    for i, pr in enumerate(probs):
        assert torch.equal(pr["W"], before[i][0]) and torch.equal(pr["Ht"], before[i][1]), i
    T = 3
    b.iterate(T)
    torch.cuda.synchronize()
    for i, (m, n, k) in enumerate(shapes):
        A = C.planted_dense(seed, m, n, k, 0.01, inst=i)
        ref = oracle.anls(k, C.init_w(seed, m, k, inst=i), C.init_ht(seed, n, k, inst=i), T, dense=A)
        d = abs(direct_r(probs[i]) - ref["r_full"][-1])
        assert d <= TOL_R, (i, d)
    b.close()


def test_batched_config4_full_vs_golden():
    """256 instances of the batched workload, 30 iterations in one captured
    graph with the autotuned work items, each instance against the oracle's
    r_30 (tests/golden/batched_256_oracle.json)."""
    with open(os.path.join(HERE, "golden", "batched_256_oracle.json")) as fh:
        ref = json.load(fh)
    seed = C.seed_for(4)
    shapes = C.batched_shapes(256, seed)
    assert [(r["m"], r["n"], r["k"]) for r in ref["instances"]] == [tuple(s) for s in shapes]
    probs, _ = build(shapes, seed)
    b = L.Batch(probs)
    best, ms = b.autotune()
    T = ref["iters"]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = b.graph(T)
        b.launch(g)
    s.synchronize()
    errs = np.array([abs(direct_r(pr) - r["r_full"][-1]) for pr, r in zip(probs, ref["instances"])])
    print(f"tuned {best.as_dict()} ({ms:.3f} ms/iteration); per-instance |dr|: max {errs.max():.3e} "
          f"mean {errs.mean():.3e} median {np.median(errs):.3e}")
    assert np.all(errs <= TOL_R), (int(errs.argmax()), float(errs.max()))
    b.close()


def test_batched_warm_prev_same_solutions_fewer_rounds():
    """Starting each NNLS from its previous passive set cannot change the
    unique solutions (up to rounding), and saves BPP rounds."""
    seed = C.seed_for(4) + 4000
    T = 6
    res = {}
    for warm in (0, 1):
        probs, shapes = build(SMALL, seed)
        t = L.batch_tune_default()
        t.warm_prev = warm
        b = L.Batch(probs, tune=t)
        counters = torch.zeros(2 * L.NMF_BPP_COUNTERS, dtype=torch.int64, device="cuda")
        b.iterate(T, counters, reset=True)
        torch.cuda.synchronize()
        res[warm] = ([direct_r(pr) for pr in probs], counters.cpu().numpy())
        b.close()
    (r0, c0), (r1, c1) = res[0], res[1]
    dr = np.max(np.abs(np.array(r0) - np.array(r1)))
    rounds0 = c0[0] + c0[L.NMF_BPP_COUNTERS]
    rounds1 = c1[0] + c1[L.NMF_BPP_COUNTERS]
    print(f"cold vs previous-set starts: max |dr| {dr:.2e}; BPP rounds {rounds0} -> {rounds1}")
    assert dr <= 1e-7
    assert rounds1 < rounds0


@pytest.mark.parametrize("tile_rows,wide", [(64, 0), (128, 1), (64, 1)])
def test_batched_tile_shapes_and_lane_classes_vs_oracle(tile_rows, wide):
    """The tile shapes and lane classes the autotuner chooses between: 64-row
    product tiles give right-hand sides bit-identical to the 128-row tiles
    (the same MFMA chain per output entry), and the wider NNLS lane classes
    the same unique solutions; every instance stays within 1e-5 of the oracle
    after 3 iterations."""
    seed = C.seed_for(4) + 5000
    T = 3
    probs, shapes = build(SMALL, seed)
    refs = []
    for i, (m, n, k) in enumerate(shapes):
        A = C.planted_dense(seed, m, n, k, 0.01, inst=i)
        refs.append(oracle.anls(k, C.init_w(seed, m, k, inst=i), C.init_ht(seed, n, k, inst=i), T, dense=A))
    out = {}
    for label, (tr, wd) in (("default", (128, 0)), ("chosen", (tile_rows, wide))):
        for pr, (m, n, k), i in zip(probs, shapes, range(len(shapes))):
            W, Ht = gen.init_factors(seed, m, n, k, inst=i)
            pr["W"].copy_(W)
            pr["Ht"].copy_(Ht)
        t = L.batch_tune_default()
        t.rhs_tile_rows, t.bpp_wide = tr, wd
        b = L.Batch(probs, tune=t)
        b.iterate(T, reset=True)
        torch.cuda.synchronize()
        out[label] = [(pr["W"].clone(), pr["Ht"].clone(), direct_r(pr)) for pr in probs]
        b.close()
    for i, ((Wd, Hd, rd), (Wc, Hc, rc)) in enumerate(zip(out["default"], out["chosen"])):
        assert abs(rc - refs[i]["r_full"][-1]) <= TOL_R, (i, shapes[i], rc, refs[i]["r_full"][-1])
        if wide == 0:
            assert torch.equal(Wd, Wc) and torch.equal(Hd, Hc), (i, shapes[i])
        else:
            assert abs(rc - rd) <= 1e-7, (i, shapes[i], rc, rd)
