"""Checks on the stored full-size oracle runs (tests/golden/video_1e6x2400_*):
what the mathematics fixes for them, without rerunning them (each takes
minutes of CPU time).

  * Algorithm 1 with an exact NNLS solve, or with one HALS sweep or one MU
    step per half-step, never increases ||A - WH|| (each half-step does not
    increase the objective of its block), so every stored trajectory is
    non-increasing across half-steps;
  * two independent oracle runs from the same start agree: the k-sweep file's
    k = 30 run is the first 10 iterations of the 50-iteration k = 30 run;
  * all files were computed on the same A (same ||A||^2).

Two orderings are checked as sanity checks on this workload, not as
theorems: a larger rank ends lower after the same iterations (the seeded
starts are nested, k = 10 ... 50), and BPP, which solves each NNLS exactly,
ends below HALS and MU, which only descend.
"""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def half_steps(run):
    return np.ravel(np.column_stack([run["r_half"], run["r_full"]]))


def test_trajectories_are_non_increasing():
    runs = [load("video_1e6x2400_k30_oracle.json")]
    loc = load("video_1e6x2400_k30_local_oracle.json")
    runs += [loc["hals"], loc["mu"]]
    runs += list(load("video_1e6x2400_ksweep_oracle.json")["k"].values())
    for run in runs:
        seq = half_steps(run)
        assert np.all(np.diff(seq) <= 1e-12 * seq[:-1])
        assert 0.0 < seq[-1] < seq[0] < 1.0


def test_ksweep_k30_equals_the_long_run_prefix():
    long = load("video_1e6x2400_k30_oracle.json")
    sweep = load("video_1e6x2400_ksweep_oracle.json")
    T = sweep["iterations"]
    run = sweep["k"]["30"]
    np.testing.assert_allclose(run["r_half"], long["r_half"][:T], rtol=1e-12)
    np.testing.assert_allclose(run["r_full"], long["r_full"][:T], rtol=1e-12)
    assert run["rounds_w"] == long["rounds_w"][:T] and run["rounds_h"] == long["rounds_h"][:T]


def test_same_matrix_in_every_file():
    f = [load(n)["fro2"] for n in ("video_1e6x2400_k30_oracle.json", "video_1e6x2400_k30_local_oracle.json",
                                   "video_1e6x2400_ksweep_oracle.json")]
    assert max(f) - min(f) <= 1e-9 * f[0]


def test_rank_and_solver_ordering():
    sweep = load("video_1e6x2400_ksweep_oracle.json")
    last = [sweep["k"][str(k)]["r_full"][-1] for k in (10, 20, 30, 40, 50)]
    assert all(b < a for a, b in zip(last, last[1:]))
    bpp = load("video_1e6x2400_k30_oracle.json")["r_full"]
    loc = load("video_1e6x2400_k30_local_oracle.json")
    for s in ("hals", "mu"):
        assert bpp[-1] <= loc[s]["r_full"][-1]


def test_stored_supports_are_consistent():
    """The stored final supports of the 50-iteration run: one mask per sampled
    row of W (every `sample_stride_w`-th of 10^6) and per row of H^T, within
    k bits; a support is a subset of the passive set it came from (BPP sets
    x = 0 off the passive set), and a W row with an empty support would be a
    zero row of the fitted W (none in a rank-10 + foreground matrix)."""
    run = load("video_1e6x2400_k30_oracle.json")
    k, m, n = 30, 1_000_000, 2_400
    assert len(run["support_w"]) == m // run["sample_stride_w"] and len(run["support_h"]) == n
    for sup, pas in (("support_w", "passive_w"), ("support_h", "passive_h")):
        for s_hex, p_hex in zip(run[sup], run[pas]):
            s_, p_ = int(s_hex, 16), int(p_hex, 16)
            assert s_ >> k == 0 and p_ >> k == 0
            assert s_ & ~p_ == 0
    assert all(int(x, 16) != 0 for x in run["support_w"])
