#!/usr/bin/env python3
"""ANLS-BPP NMF benchmark on one MI355X.

Workload: the video-like dense matrix, 1,000,000 x 2,400 (FP32, 9.6 GB, built
in HBM by the seeded generator), rank k = 30, 50 ANLS-BPP iterations from the
seeded U[0,1) initial factors.  One step is one such 50-iteration run:

  learned + BF16x3 form (the reported value): iterations 1-5 with cold BPP
    and BF16x3 right-hand sides while collecting (features, final passive
    set) samples, training of the W-side and H-side warm-start networks on
    the GPU, iterations 6-50 with the networks' start sets;
  plain FP32 form (timed beside it): 50 iterations, cold BPP, FP32 MFMA
    right-hand sides.

value = iterations / second of the learned + BF16x3 form (training included),
with the inputs (A, its BF16 planes, the initial factors) resident in HBM.
Both forms' final relative objective is checked against the FP64 oracle's
trajectory (tests/golden/video_1e6x2400_k30_oracle.json) when available.

Per-phase HIP events inside the timed region give the dominant kernel's
average duration for the roofline; the FP64 CPU oracle is timed on a bounded
row sample for the CPU baseline.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ANLS-BPP iters/sec at matched rel. objective (learned+BF16 vs plain FP32)"
GOLDEN = os.path.join(ROOT, "tests", "golden", "video_1e6x2400_k30_oracle.json")
LOCAL_GOLDEN = os.path.join(ROOT, "tests", "golden", "video_1e6x2400_k30_local_oracle.json")
KSWEEP_GOLDEN = os.path.join(ROOT, "tests", "golden", "video_1e6x2400_ksweep_oracle.json")
TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m", type=int, default=1_000_000)
    ap.add_argument("--n", type=int, default=2_400)
    ap.add_argument("--k", type=int, default=30)
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--cold-iters", type=int, default=5)
    ap.add_argument("--train-steps", type=int, default=20)
    ap.add_argument("--train-batch", type=int, default=1024)
    ap.add_argument("--collect-stride", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 256-instance batched measurement")
    ap.add_argument("--no-local", action="store_true", help="skip the HALS / MU local-solver measurement")
    ap.add_argument("--batched-reps", type=int, default=3)
    ap.add_argument("--pmc", action="store_true", help="copy calibration + product kernels only (for rocprofv3 --pmc)")
    ap.add_argument("--pmc-bpp", action="store_true",
                    help="batched BPP from cold and exact start sets at a mid-run state (for rocprofv3 --pmc)")
    ap.add_argument("--dense", action="store_true",
                    help="the dense planted workload at full size (172800 x 115200, k = 50, 30 iterations)")
    ap.add_argument("--ksweep", action="store_true",
                    help="time per iteration and its MM / NLS / Gram split for k = 10..50 on the video workload")
    ap.add_argument("--ksweep-iters", type=int, default=10)
    ap.add_argument("--sparse", action="store_true",
                    help="the CSR workload (207360 x 138240): alone, or with --pmc its SpMM kernels too")
    return ap.parse_args(argv)


class Bench:
    def __init__(self, a):
        import torch

        from nmf_inputs import configs as C
        from nmf_inputs import device as gen
        from paper_1509_09313_amd import binding as L
        self.torch, self.C, self.L, self.a, self.gen = torch, C, L, a, gen
        self.seed = C.seed_for(5)
        m, n, k = a.m, a.n, a.k
        t0 = time.perf_counter()
        self.A = gen.video(self.seed, m, n)
        self.W0, self.Ht0 = gen.init_factors(self.seed, m, n, k)
        self.M = L.Matrix(dense=self.A)
        torch.cuda.synchronize()
        self.t_gen = time.perf_counter() - t0
        t0 = time.perf_counter()
        self.M.add_split()
        torch.cuda.synchronize()
        self.t_split = time.perf_counter() - t0
        self.W = torch.empty_like(self.W0)
        self.Ht = torch.empty_like(self.Ht0)
        # learned form: collection buffers, networks, runners
        self.T1 = a.cold_iters
        self.T2 = a.iters - a.cold_iters
        sw, sh = a.collect_stride, 1
        self.cap_w = self.T1 * ((m + sw - 1) // sw)
        self.cap_h = self.T1 * ((n + sh - 1) // sh)
        f32, i64 = torch.float32, torch.int64
        self.phi_w = torch.zeros((self.cap_w, 2 * k), dtype=f32, device="cuda")
        self.phi_h = torch.zeros((self.cap_h, 2 * k), dtype=f32, device="cuda")
        self.mk_w = torch.zeros(self.cap_w, dtype=i64, device="cuda")
        self.mk_h = torch.zeros(self.cap_h, dtype=i64, device="cuda")
        o1 = L.make_opts(prec=L.NMF_BF16X3, trace=True, reset_masks=True)
        o1.collect, o1.collect_stride_w, o1.collect_stride_h = 1, sw, sh
        o1.coll_phi_w, o1.coll_mask_w, o1.coll_cap_w = self.phi_w.data_ptr(), self.mk_w.data_ptr(), self.cap_w
        o1.coll_phi_h, o1.coll_mask_h, o1.coll_cap_h = self.phi_h.data_ptr(), self.mk_h.data_ptr(), self.cap_h
        self.pw0 = torch.from_numpy(C.mlp_init(k, self.seed, side=0)).cuda()
        self.ph0 = torch.from_numpy(C.mlp_init(k, self.seed, side=1)).cuda()
        self.tw = L.MlpTrainer(k, self.pw0.clone(), batch=a.train_batch)
        self.th = L.MlpTrainer(k, self.ph0.clone(), batch=a.train_batch)
        o2 = L.make_opts(prec=L.NMF_BF16X3, warm=L.NMF_WARM_LEARNED, net_w=self.tw.params, net_h=self.th.params,
                         trace=True, reset_masks=True)
        self.run1 = L.Anls(self.M, k, o1)
        self.run2 = L.Anls(self.M, k, o2)
        self.st1 = L.new_stats(self.T1)
        self.st2 = L.new_stats(self.T2)
        oP = L.make_opts(prec=L.NMF_F32, trace=True, reset_masks=True)
        self.runP = L.Anls(self.M, k, oP)
        self.stP = L.new_stats(a.iters)

    # ---------------------------------------------------------------- forms --
    def learned_step(self, timers=None):
        t = self.torch
        self.W.copy_(self.W0)
        self.Ht.copy_(self.Ht0)
        if timers:
            timers[0].attach(self.run1.opts)
            timers[1].attach(self.run2.opts)
        self.run1.run(self.W, self.Ht, self.T1, self.st1)
        for tr, p0, phi, mk, cap in ((self.tw, self.pw0, self.phi_w, self.mk_w, self.cap_w),
                                     (self.th, self.ph0, self.phi_h, self.mk_h, self.cap_h)):
            tr.params.copy_(p0)
            tr.m.zero_()
            tr.v.zero_()
            tr.step = 0
            tr.train(phi, mk, cap, self.a.train_steps)
        self.run2.run(self.W, self.Ht, self.T2, self.st2)
        if timers:
            timers[0].detach(self.run1.opts)
            timers[1].detach(self.run2.opts)
        del t

    def plain_step(self, timer=None):
        self.W.copy_(self.W0)
        self.Ht.copy_(self.Ht0)
        if timer:
            timer.attach(self.runP.opts)
        self.runP.run(self.W, self.Ht, self.a.iters, self.stP)
        if timer:
            timer.detach(self.runP.opts)

    def final_r(self):
        return float(self.L.nmf_objective(self.M, self.W, self.Ht)[0].item())


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def bpp_flops(stats, k, key):
    """Algorithmic FP64 flops of the passive-set solves (Cholesky count):
    sum over solves of |F|^3/3 + 2|F|^2 + 2k|F| (solve, two triangular
    sweeps, dual)."""
    tot = 0.0
    for s in stats:
        c = s[key]
        tot += c[4] / 3.0 + 2.0 * c[3] + 2.0 * k * c[2]
    return tot


def roofline(bench, timers_l, stats_l):
    """Dominant kernel of the learned form over the timed region."""
    a = bench.a
    L = bench.L
    per = {p: [] for p in L.PHASES}
    for tm in timers_l:
        ph = tm.phase_ms()
        for p in L.PHASES:
            per[p] += ph[p]
    totals = {p: sum(v) for p, v in per.items()}
    launches = {p: len(v) for p, v in per.items()}
    dom = max(("rhs_w", "rhs_h", "bpp_w", "bpp_h", "gram_w", "gram_h", "infer_w", "infer_h"), key=lambda p: totals[p])
    avg_ms = totals[dom] / max(1, launches[dom])
    m, n, k = a.m, a.n, a.k
    out = {"kernel_phase": dom, "avg_ms": avg_ms,
           "phase_ms_per_iter": {p: totals[p] / max(1, launches[p]) for p in L.PHASES}}
    if dom in ("rhs_w", "rhs_h"):
        rows = m if dom == "rhs_w" else n
        contracted = n if dom == "rhs_w" else m
        alg_bytes = 4.0 * m * n + 4.0 * contracted * k + 4.0 * rows * k
        ach = alg_bytes / (avg_ms * 1e-3) / 1e9
        out.update(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                   algorithmic_bytes_per_launch=alg_bytes)
    elif dom in ("bpp_w", "bpp_h"):
        key = "bpp_w" if dom == "bpp_w" else "bpp_h"
        # counters of the last timed step (every step repeats the same run)
        n_it = sum(len(s) for s in stats_l)
        fl = sum(bpp_flops(s, k, key) for s in stats_l) / max(1, n_it)
        ach = fl / (avg_ms * 1e-3) / 1e12
        out.update(bound="alu", achieved=ach, peak=FP64_PEAK_TFLOPS, unit="TFLOP/s", frac=ach / FP64_PEAK_TFLOPS,
                   algorithmic_flops_per_launch=fl)
    else:
        rows = m if dom in ("gram_w", "infer_w") else n
        alg_bytes = 4.0 * rows * k
        ach = alg_bytes / (avg_ms * 1e-3) / 1e9
        out.update(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                   algorithmic_bytes_per_launch=alg_bytes)
    out["traffic"] = None
    try:
        with open(TRAFFIC) as fh:
            tr = json.load(fh)
        ent = tr.get(dom)
        if ent and ent.get("source_sha256") == source_digest(dom):
            out["traffic"] = ent["bytes_per_launch"]
    except (OSError, ValueError):
        pass
    return out


# sources that define each phase's kernels; counter results are tied to them
PHASE_SOURCES = {
    "rhs_w": ("rhs_bf16.hip", "nmf_common.h"), "rhs_h": ("rhs_bf16.hip", "nmf_common.h"),
    "bpp_w": ("bpp.hip", "nmf_common.h"), "bpp_h": ("bpp.hip", "nmf_common.h"),
    "gram_w": ("gram.hip", "nmf_common.h"), "gram_h": ("gram.hip", "nmf_common.h"),
    "infer_w": ("mlp.hip", "nmf_common.h"), "infer_h": ("mlp.hip", "nmf_common.h"),
}


def source_digest(phase):
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1509_09313_amd", "csrc")
    for f in PHASE_SOURCES[phase]:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def cpu_baseline(bench, seconds):
    """The FP64 oracle (as it stands) on a bounded sample of the workload: the
    first S rows for I ANLS-BPP iterations, about `seconds` of host work;
    the time per iteration is scaled by m / S to the full matrix."""
    import numpy as np

    import oracle
    a = bench.a
    W0 = bench.W0.cpu().numpy()
    H0 = bench.Ht0.cpu().numpy()

    def run(S, iters):
        A = bench.A[:S].cpu().numpy()
        t0 = time.perf_counter()
        oracle.anls(a.k, W0[:S], H0, iters, dense=A)
        return time.perf_counter() - t0

    S, I = min(a.m, 20_000), 1
    t = run(S, I)
    S2 = int(min(a.m, max(S, S * seconds / max(t, 1e-3))))
    if S2 > S:
        S, t = S2, run(S2, I)
    if t < 0.5 * seconds:
        I = int(min(a.iters, max(1, seconds // max(t, 1e-3))))
        if I > 1:
            t = run(S, I)
    per_iter = t / I * a.m / S
    return {"value": 1.0 / per_iter, "unit": "iters/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"{I} ANLS-BPP iteration(s) of the FP64 oracle on rows 0..{S - 1} ({S} x {a.n}, k={a.k}) "
                      f"from the benchmark's initial factors, {t:.2f} s, per iteration scaled by {a.m}/{S} to the "
                      f"full matrix",
            "seconds_per_iter_full": per_iter}


def local_forms(bench):
    """Algorithm 1 with the HALS and MU local updates (Eq. halsupdate,
    Eq. muupdate) on the same workload: BF16x3 right-hand sides, FP64 Gram,
    the update in FP64; `iters` iterations from the same seeded W, H per step.
    The final relative objective is compared with the FP64 oracle's."""
    import numpy as np

    a, L = bench.a, bench.L
    ref = None
    if os.path.exists(LOCAL_GOLDEN) and (a.m, a.n, a.k, a.iters) == (1_000_000, 2_400, 30, 50):
        with open(LOCAL_GOLDEN) as fh:
            ref = json.load(fh)
    out = {}
    for name, solver in (("hals", L.NMF_SOLVER_HALS), ("mu", L.NMF_SOLVER_MU)):
        run = L.Anls(bench.M, a.k, L.make_opts(prec=L.NMF_BF16X3, trace=True, solver=solver))
        stats = L.new_stats(a.iters)

        def step(timer=None):
            bench.W.copy_(bench.W0)
            bench.Ht.copy_(bench.Ht0)
            if timer:
                timer.attach(run.opts)
            run.run(bench.W, bench.Ht, a.iters, stats)
            if timer:
                timer.detach(run.opts)

        t = timed(step, a.steps, a.warmup)
        r = bench.final_r()
        tm = L.PhaseTimer(a.iters)
        step(tm)
        bench.torch.cuda.synchronize()
        ph = {p: float(np.mean(v)) for p, v in tm.phase_ms().items()}
        tm.close()
        o = None if ref is None else ref[name]["r_full"][-1]
        # the FP64 oracle's own time for the same 50 iterations, recorded when the stored run was
        # written (8 host threads of the machine that wrote it, not this one)
        o_s = None if ref is None else ref[name]["oracle_seconds"] / a.iters
        # the W-side update streams R (read) and W (read and written): 12 k bytes per row
        alg = 12.0 * a.k * a.m
        gbs = alg / (ph["bpp_w"] * 1e-3) / 1e9
        out[name] = {"iters_per_s": a.iters * a.steps / t, "ms_per_step": t / a.steps * 1e3, "final_r": r,
                     "oracle_r": o, "abs_dr_vs_oracle": None if o is None else abs(r - o),
                     "update_ms_per_iter": {"w": ph["bpp_w"], "h": ph["bpp_h"]},
                     "update_w_roofline": {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s",
                                           "frac": gbs / 8000.0, "algorithmic_bytes_per_launch": alg,
                                           "fp64_tflops": 2.0 * a.k * a.k * a.m / (ph["bpp_w"] * 1e-3) / 1e12},
                     "oracle_s_per_iter_recorded": o_s,
                     "phase_ms_per_iter": ph}
        print(f"# {name}: {out[name]['ms_per_step']:.1f} ms/step, final r {r:.8f}", file=sys.stderr, flush=True)
    out["note"] = ("the update phase is reported in the bpp_* slots of phase_ms_per_iter; "
                   "r after the same number of iterations differs between solvers (BPP solves each NNLS exactly)")
    return out


KS = (10, 20, 30, 40, 50)

BATCH_GOLDEN = os.path.join(ROOT, "tests", "golden", "batched_256_oracle.json")


def batched(a):
    """The 256-instance batched workload: autotuned work items, 30 iterations
    captured as one graph, each launch from the same initial factors (cold
    BPP, then previous passive sets); per-instance error against the FP64
    oracle's r_30 and the HBM rate of the whole iteration."""
    import numpy as np
    import torch

    from nmf_inputs import configs as C
    from nmf_inputs import device as gen
    from paper_1509_09313_amd import binding as L
    seed = C.seed_for(4)
    shapes = C.batched_shapes(256, seed)
    T = 30
    probs = []
    for i, (m, n, k) in enumerate(shapes):
        A = gen.planted(seed, m, n, k, 0.01, inst=i)
        W, Ht = gen.init_factors(seed, m, n, k, inst=i)
        probs.append({"A": A, "W": W, "Ht": Ht})
    H0 = [p["Ht"].clone() for p in probs]
    torch.cuda.synchronize()
    b = L.Batch(probs)
    best, tuned_ms = b.autotune()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = b.graph(T)
    times = []
    for rep in range(1 + a.batched_reps):
        for p, h in zip(probs, H0):
            p["Ht"].copy_(h)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(s):
            e0.record(s)
            b.launch(g)
            e1.record(s)
        s.synchronize()
        if rep > 0:
            times.append(e0.elapsed_time(e1))
    ms_run = float(np.mean(times))
    errs = None
    if os.path.exists(BATCH_GOLDEN):
        with open(BATCH_GOLDEN) as fh:
            ref = json.load(fh)
        errs = []
        for p, r in zip(probs, ref["instances"]):
            M = L.Matrix(dense=p["A"])
            errs.append(abs(float(L.nmf_objective(M, p["W"], p["Ht"])[0]) - r["r_full"][-1]))
    alg = float(sum(8.0 * m * n + 16.0 * k * (m + n) for m, n, k in shapes))
    ach = alg / (ms_run / T * 1e-3) / 1e9
    b.close()
    return {"workload": "256 planted dense instances, m log-uniform [500,8000], n log-uniform [500,4000], "
                        "k in {10,20,50}, BF16x3 products, FP64 Gram/BPP, 30 iterations per graph launch",
            "iters_per_s": T / (ms_run * 1e-3), "ms_per_30_iterations": ms_run, "tune": best.as_dict(),
            "tuner_ms_per_iteration_from_cold": tuned_ms,
            "max_abs_dr_vs_oracle": None if errs is None else float(max(errs)),
            "mean_abs_dr_vs_oracle": None if errs is None else float(np.mean(errs)),
            "algorithmic_bytes_per_iteration": alg, "achieved_GBps": ach, "hbm_frac": ach / HBM_PEAK_GBS}


def sparse_inputs(torch):
    """The CSR workload (207,360 x 138,240, density 1e-3) built on the host
    from its seeded recipe and uploaded: CSR(A) and CSR(A^T)."""
    from nmf_inputs import configs as C
    seed, m, n = C.seed_for(3), 207_360, 138_240
    rp, ci, va = C.sparse_csr(seed, m, n, 1e-3)
    rpt, cit, vat = C.csr_transpose(m, n, rp, ci, va)
    d = [torch.from_numpy(x).cuda() for x in (rp, ci, va, rpt, cit, vat)]
    return seed, m, n, d


def pmc_mode(a):
    """Launches a plain copy of known size, then each product kernel a few
    times (BF16x3 and FP32 on the video-like matrix, both Gram passes, and
    with --sparse the CSR products of the sparse workload), for rocprofv3
    counter collection (FETCH_SIZE / WRITE_SIZE, MFMA busy cycles)."""
    import torch
    b = Bench(a)
    L = b.L
    src = torch.empty(1 << 29, dtype=torch.float32, device="cuda")   # 2 GiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    bt, btt = b.M.tiled
    for _ in range(3):
        L.nmf_rhs_dense(L.NMF_SIDE_W, None, b.Ht0, prec=L.NMF_BF16X3, B_bf16=bt, m=a.m, n=a.n)
        L.nmf_rhs_dense(L.NMF_SIDE_H, None, b.W0, prec=L.NMF_BF16X3, B_bf16=btt, m=a.m, n=a.n)
    for _ in range(3):
        L.nmf_rhs_dense(L.NMF_SIDE_W, b.A, b.Ht0)
        L.nmf_rhs_dense(L.NMF_SIDE_H, b.A, b.W0)
    for _ in range(3):
        L.nmf_gram(b.W0)
        L.nmf_gram(b.Ht0)
    if a.sparse:
        seed, m, n, d = sparse_inputs(torch)
        W0, Ht0 = b.gen.init_factors(seed, m, n, 50)
        for _ in range(3):
            L.nmf_rhs_csr(d[0], d[1], d[2], Ht0, m, n)
            L.nmf_rhs_csr(d[3], d[4], d[5], W0, n, m)
    torch.cuda.synchronize()
    print(json.dumps({"pmc": "done", "copy_bytes": 2 * src.numel() * 4}))


def pmc_bpp_mode(a):
    """For rocprofv3 counter collection on the NNLS kernel: the state after 6
    BF16x3 iterations of Algorithm 1 from the seeded start (W side: G = H H^T,
    R = A H^T), then batched BPP three times from a cold start and three times
    from the exact final passive sets, alternating."""
    import torch

    from nmf_inputs import configs as C
    from nmf_inputs import device as gen
    from paper_1509_09313_amd import binding as L
    m, n, k = a.m, a.n, a.k
    seed = C.seed_for(5)
    A = gen.video(seed, m, n)
    W0, Ht0 = gen.init_factors(seed, m, n, k)
    M = L.Matrix(dense=A, split=True)
    W, Ht = W0.clone(), Ht0.clone()
    L.Anls(M, k, L.make_opts(prec=L.NMF_BF16X3)).run(W, Ht, 6)
    G = L.nmf_gram(Ht)
    R = L.nmf_rhs_dense(L.NMF_SIDE_W, None, Ht, prec=L.NMF_BF16X3, B_bf16=M.tiled[0], m=m, n=n)
    X = torch.empty_like(W)
    _, mask, _, _ = L.nnls_bpp_batched(G, R, X)
    for _ in range(3):
        L.nnls_bpp_batched(G, R, X)
        L.nnls_bpp_batched(G, R, X, mask_in=mask)
    torch.cuda.synchronize()
    print(json.dumps({"pmc_bpp": "done", "problems": m, "k": k}))


def dense_mode(a):
    """The dense planted workload at full size (172,800 x 115,200, rank-50
    U[0,1) factors plus 0.01 U[0,1) noise; A is 79.6 GB in FP32), k = 50, 30
    cold-BPP iterations per step: plain FP32 products, then BF16x3 products
    from the padded planes of A and A^T (159 GB more, made after the FP32
    form).  Reports iterations/s, the phase split, the products' rate (HBM
    bytes and FP32 MFMA flops) and the final relative objective of each form
    (the two must agree within 1e-5; the FP64 oracle cannot run this size, the
    sampled full-size tests check it instead)."""
    import numpy as np
    import torch

    from nmf_inputs import configs as C
    from nmf_inputs import device as gen
    from paper_1509_09313_amd import binding as L
    seed, m, n, k, T = C.seed_for(2), 172_800, 115_200, 50, 30
    t0 = time.perf_counter()
    A = gen.planted(seed, m, n, k)
    W0, Ht0 = gen.init_factors(seed, m, n, k)
    M = L.Matrix(dense=A)
    torch.cuda.synchronize()
    print(f"# dense inputs: {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    W, Ht = torch.empty_like(W0), torch.empty_like(Ht0)
    prod_bytes = 2.0 * (4.0 * m * n + 4.0 * n * k + 4.0 * m * k)
    prod_flops = 2.0 * 2.0 * m * n * k

    def form(prec):
        run = L.Anls(M, k, L.make_opts(prec=prec, trace=True, reset_masks=True))
        stats = L.new_stats(T)

        def step(timer=None):
            W.copy_(W0)
            Ht.copy_(Ht0)
            if timer:
                timer.attach(run.opts)
            run.run(W, Ht, T, stats)
            if timer:
                timer.detach(run.opts)

        t = timed(step, a.steps, a.warmup)
        tm = L.PhaseTimer(T)
        step(tm)
        torch.cuda.synchronize()
        ph = {p: float(np.mean(v)) for p, v in tm.phase_ms().items()}
        tm.close()
        r = float(L.nmf_objective(M, W, Ht)[0])
        mm = (ph["rhs_w"] + ph["rhs_h"]) * 1e-3
        st = L.decode_stats(stats)
        out = {"iters_per_s": T * a.steps / t, "ms_per_iter": t / (a.steps * T) * 1e3, "final_r": r,
               "phase_ms_per_iter": ph, "products_GBps": prod_bytes / mm / 1e9,
               "products_hbm_frac": prod_bytes / mm / 8e12,
               "products_fp32_mfma_TFLOPs": prod_flops / mm / 1e12, "capped": int(sum(s["capped"] for s in st))}
        print(f"# dense {'fp32' if prec == L.NMF_F32 else 'bf16x3'}: {out['ms_per_iter']:.2f} ms/iter, "
              f"products {out['products_GBps']:.0f} GB/s, r {r:.8f}", file=sys.stderr, flush=True)
        return out

    res = {"workload": f"planted dense {m}x{n} (rank 50 U[0,1) factors + 0.01 U[0,1) noise), k={k}, {T} cold-BPP "
                       f"iterations per step from the seeded start"}
    res["fp32"] = form(L.NMF_F32)
    M.add_split()
    torch.cuda.synchronize()
    res["bf16x3"] = form(L.NMF_BF16X3)
    res["abs_dr_bf16x3_vs_fp32"] = abs(res["bf16x3"]["final_r"] - res["fp32"]["final_r"])
    print(json.dumps({"dense": res}))


def sparse_mode(a):
    """The CSR workload at full size: plain FP32 SpMM right-hand sides, FP64
    Gram and BPP, `iters` iterations per step from the seeded start (cold
    BPP), with the SpMM rate on algorithmic bytes."""
    import numpy as np
    import torch

    from nmf_inputs import device as gen
    from paper_1509_09313_amd import binding as L
    t0 = time.perf_counter()
    seed, m, n, d = sparse_inputs(torch)
    k, T = 50, 30
    W0, Ht0 = gen.init_factors(seed, m, n, k)
    M = L.Matrix(csr=(d[0], d[1], d[2]), csr_t=(d[3], d[4], d[5]), shape=(m, n))
    torch.cuda.synchronize()
    print(f"# sparse inputs: {time.perf_counter() - t0:.1f}s (host generation)", file=sys.stderr, flush=True)
    W, Ht = torch.empty_like(W0), torch.empty_like(Ht0)
    nnz = int(d[2].numel())
    # algorithmic bytes of one SpMM: int32 column + FP32 value per nonzero, the
    # row pointers, Y read once, R written once
    alg_w = 8.0 * nnz + 8.0 * (m + 1) + 4.0 * n * k + 4.0 * m * k
    alg_h = 8.0 * nnz + 8.0 * (n + 1) + 4.0 * m * k + 4.0 * n * k

    def form(warm):
        run = L.Anls(M, k, L.make_opts(prec=L.NMF_F32, warm=warm, trace=True, reset_masks=True))
        stats = L.new_stats(T)

        def step(timer=None):
            W.copy_(W0)
            Ht.copy_(Ht0)
            if timer:
                timer.attach(run.opts)
            run.run(W, Ht, T, stats)
            if timer:
                timer.detach(run.opts)

        t = timed(step, a.steps, a.warmup)
        tm = L.PhaseTimer(T)
        step(tm)
        torch.cuda.synchronize()
        ph = {p: float(np.mean(v)) for p, v in tm.phase_ms().items()}
        tm.close()
        r = float(L.nmf_objective(M, W, Ht)[0])
        st = L.decode_stats(stats)
        return {"iters_per_s": T * a.steps / t, "ms_per_step": t / a.steps * 1e3, "final_r": r,
                "phase_ms_per_iter": ph,
                "spmm_w_GBps": alg_w / (ph["rhs_w"] * 1e-3) / 1e9, "spmm_h_GBps": alg_h / (ph["rhs_h"] * 1e-3) / 1e9,
                "bpp_rounds_per_problem": float(np.mean([(s["bpp_w"][0] + s["bpp_h"][0]) / (m + n) for s in st])),
                "capped": int(sum(s["capped"] for s in st))}

    res = {"workload": f"CSR {m}x{n}, density 1e-3 ({nnz} nonzeros), k={k}, {T} iterations per step, "
                       f"FP32 SpMM, FP64 Gram/BPP, cold BPP"}
    res.update(form(L.NMF_WARM_COLD))
    res["warm_prev"] = form(L.NMF_WARM_PREV)
    res["warm_prev"]["abs_dr_vs_cold"] = abs(res["warm_prev"]["final_r"] - res["final_r"])
    print(json.dumps({"sparse": res}))


def ksweep_mode(a):
    """The rank axis of the paper's algorithmic comparison on one GPU: for
    k = 10, 20, 30, 40, 50 on the video-like workload, iterations per second
    and the per-iteration time split into the paper's local tasks (MM: the
    two right-hand-side products, NLS: the two local solves, Gram: the two
    Gram matrices; Section "Time Breakdown"), for Algorithm 1 with BPP
    (FP32 and BF16x3 products), HALS and MU.  `ksweep_iters` iterations per
    step from the seeded start; the BPP forms' relative objective is compared
    with the FP64 oracle's after the same number of iterations."""
    import numpy as np
    import torch

    from nmf_inputs import configs as C
    from nmf_inputs import device as gen
    from paper_1509_09313_amd import binding as L
    m, n, T = a.m, a.n, a.ksweep_iters
    seed = C.seed_for(5)
    A = gen.video(seed, m, n)
    M = L.Matrix(dense=A)
    M.add_split()
    ref = None
    if os.path.exists(KSWEEP_GOLDEN) and (m, n) == (1_000_000, 2_400):
        with open(KSWEEP_GOLDEN) as fh:
            ref = json.load(fh)
        if ref["iterations"] != T:
            ref = None
    forms = (("bpp_fp32", dict(prec=L.NMF_F32)), ("bpp_bf16x3", dict(prec=L.NMF_BF16X3)),
             ("hals_bf16x3", dict(prec=L.NMF_BF16X3, solver=L.NMF_SOLVER_HALS)),
             ("mu_bf16x3", dict(prec=L.NMF_BF16X3, solver=L.NMF_SOLVER_MU)))
    out = {"workload": f"video-like dense {m}x{n}, {T} iterations per step from the seeded start, cold BPP",
           "ks": list(KS), "forms": {}}
    for name, kw in forms:
        rows = []
        for k in KS:
            W0, Ht0 = gen.init_factors(seed, m, n, k)
            W, Ht = torch.empty_like(W0), torch.empty_like(Ht0)
            run = L.Anls(M, k, L.make_opts(trace=True, reset_masks=True, **kw))
            stats = L.new_stats(T)

            def step(timer=None):
                W.copy_(W0)
                Ht.copy_(Ht0)
                if timer:
                    timer.attach(run.opts)
                run.run(W, Ht, T, stats)
                if timer:
                    timer.detach(run.opts)

            t = timed(step, a.steps, a.warmup)
            r = float(L.nmf_objective(M, W, Ht)[0])
            tm = L.PhaseTimer(T)
            step(tm)
            torch.cuda.synchronize()
            ph = {p: float(np.mean(v)) for p, v in tm.phase_ms().items()}
            tm.close()
            o = o_s = None
            if ref is not None and name.startswith("bpp"):
                o = ref["k"][str(k)]["r_full"][-1]
                # the FP64 oracle's own time for these iterations, recorded when the stored run was
                # written (on the machine that wrote it)
                o_s = ref["k"][str(k)]["oracle_seconds"] / ref["iterations"]
            ms = t / (a.steps * T) * 1e3
            split = {"MM": ph["rhs_w"] + ph["rhs_h"], "NLS": ph["bpp_w"] + ph["bpp_h"],
                     "Gram": ph["gram_w"] + ph["gram_h"]}
            split["rest"] = ms - sum(split.values())
            # algorithmic bytes of the two products: A once each, the other factor read, R written
            mm_bytes = 2.0 * (4.0 * m * n + 4.0 * n * k + 4.0 * m * k)
            mm_gbs = mm_bytes / (split["MM"] * 1e-3) / 1e9
            rows.append({"k": k, "iters_per_s": 1e3 / ms, "ms_per_iter": ms, "split_ms": split, "final_r": r,
                         "oracle_r": o, "abs_dr_vs_oracle": None if o is None else abs(r - o),
                         "mm_GBps": mm_gbs, "mm_hbm_frac": mm_gbs / 8000.0, "oracle_s_per_iter_recorded": o_s})
            print(f"# {name} k={k}: {ms:.2f} ms/iter (MM {split['MM']:.2f} at {mm_gbs:.0f} GB/s, "
                  f"NLS {split['NLS']:.2f}, Gram {split['Gram']:.2f}), r {r:.8f}", file=sys.stderr, flush=True)
            del run, W, Ht, W0, Ht0
        out["forms"][name] = rows
    print(json.dumps({"ksweep": out}))


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported: the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    if a.pmc:
        pmc_mode(a)
        return
    if a.pmc_bpp:
        pmc_bpp_mode(a)
        return
    if a.sparse:
        sparse_mode(a)
        return
    if a.ksweep:
        ksweep_mode(a)
        return
    if a.dense:
        dense_mode(a)
        return
    import numpy as np
    b = Bench(a)
    L = b.L
    print(f"# inputs: generate {b.t_gen:.2f}s, one-time BF16 split {b.t_split:.3f}s", file=sys.stderr, flush=True)

    # learned + BF16x3 form, with per-phase events over the timed steps
    timers = [(L.PhaseTimer(b.T1), L.PhaseTimer(b.T2)) for _ in range(a.steps)]
    it = iter(timers)
    for _ in range(a.warmup):
        b.learned_step()
    b.torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(a.steps):
        b.learned_step(next(it))
    b.torch.cuda.synchronize()
    t_learned = time.perf_counter() - t0
    r_learned = b.final_r()
    st_l = L.decode_stats(b.st1) + L.decode_stats(b.st2)
    print(f"# learned+bf16x3: {t_learned / a.steps * 1e3:.1f} ms/step, final r {r_learned:.8f}", file=sys.stderr,
          flush=True)
    roof = roofline(b, [t for pair in timers for t in pair], [L.decode_stats(b.st1), L.decode_stats(b.st2)])

    plain = None
    if not a.no_plain:
        tp = L.PhaseTimer(a.iters)
        t_plain = timed(b.plain_step, a.steps, a.warmup)
        r_plain = b.final_r()
        b.plain_step(tp)
        b.torch.cuda.synchronize()
        ph = tp.phase_ms()
        st_p = L.decode_stats(b.stP)
        plain = {"iters_per_s": a.iters * a.steps / t_plain, "ms_per_step": t_plain / a.steps * 1e3,
                 "final_r": r_plain, "phase_ms_per_iter": {p: float(np.mean(v)) for p, v in ph.items()},
                 "bpp_rounds_w_per_row": float(np.mean([s["bpp_w"][0] for s in st_p]) / a.m),
                 "bpp_solves_w_per_row": float(np.mean([s["bpp_w"][1] for s in st_p]) / a.m)}
        print(f"# plain fp32: {plain['ms_per_step']:.1f} ms/step, final r {r_plain:.8f}", file=sys.stderr, flush=True)

    oracle_r = None
    if os.path.exists(GOLDEN) and (a.m, a.n, a.k, a.iters) == (1_000_000, 2_400, 30, 50):
        with open(GOLDEN) as fh:
            oracle_r = json.load(fh)["r_full"][-1]

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(b, a.cpu_seconds)

    loc = None
    if not a.no_local:
        loc = local_forms(b)

    bat = None
    if not a.no_batched:
        bat = batched(a)
        print(f"# batched 256 instances: {bat['ms_per_30_iterations']:.1f} ms per 30 iterations", file=sys.stderr,
              flush=True)

    value = a.iters * a.steps / t_learned
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": t_learned / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3 products (fp32 accumulate) + f64 Gram/BPP",
        "data": "synthetic",
        "config": {"workload": f"video-like dense {a.m}x{a.n} (rank-10 background + 2% foreground), k={a.k}, "
                               f"{a.iters} ANLS-BPP iterations per step; learned warm start after {a.cold_iters} "
                               f"cold iterations + BF16x3 right-hand sides",
                   "m": a.m, "n": a.n, "k": a.k, "iters_per_step": a.iters, "train_steps": a.train_steps,
                   "train_batch": a.train_batch, "collect_stride_w": a.collect_stride},
        "final_r": r_learned,
        "oracle_r": oracle_r,
        "abs_dr_vs_oracle": None if oracle_r is None else abs(r_learned - oracle_r),
        "plain_fp32": plain,
        "speedup_vs_plain_fp32": None if plain is None else value / plain["iters_per_s"],
        "matched_objective": None if plain is None else (
            abs(r_learned - plain["final_r"]) <= 1e-5 if oracle_r is None
            else (abs(r_learned - oracle_r) <= 1e-5 and abs(plain["final_r"] - oracle_r) <= 1e-5)),
        "bpp_solves_w_per_row_learned": float(np.mean([s["bpp_w"][1] for s in st_l[b.T1:]]) / a.m),
        "bpp_fallbacks_learned": int(sum(s["fallback"] for s in st_l)),
        "one_time_split_s": b.t_split,
        "roofline": roof,
        "cpu_baseline": cpu,
        "local_solvers": loc,
        "batched": bat,
    }
    for pair in timers:
        for t in pair:
            t.close()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
