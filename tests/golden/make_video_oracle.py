"""FP64 oracle trajectory for the full video-like workload (1,000,000 x 2,400,
k = 30, 50 ANLS-BPP iterations, cold BPP), stored in
tests/golden/video_1e6x2400_k30_oracle.json.

Calls only oracle/ and the host recipes of nmf_inputs; A is generated on the
host (row chunks in parallel processes), so no value comes from a GPU.
Needs about 12 GB of host memory; run from the repository root:
    python tests/golden/make_video_oracle.py
"""
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from nmf_inputs import configs as C  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "video_1e6x2400_k30_oracle.json")
M, N, K, T = 1_000_000, 2_400, 30, 50
CHUNK = 10_000
SAMPLE_STRIDE = 1000


def hex_mask(x):
    return format(sum(1 << i for i in range(len(x)) if x[i] > 0.0), "x")


def rows_chunk(r0):
    return r0, C.video_rows(C.seed_for(5), N, np.arange(r0, min(M, r0 + CHUNK)))


def main(workers=6):
    t0 = time.time()
    A = np.empty((M, N), dtype=np.float32)
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        for r0, blk in ex.map(rows_chunk, range(0, M, CHUNK)):
            A[r0:r0 + blk.shape[0]] = blk
    t_gen = time.time() - t0
    print(f"generated A in {t_gen:.0f}s", flush=True)
    W0 = C.init_w(C.seed_for(5), M, K)
    H0 = C.init_ht(C.seed_for(5), N, K)
    t1 = time.time()
    res = oracle.anls(K, W0, H0, T, dense=A)
    t_orc = time.time() - t1
    print(f"oracle {T} iterations in {t_orc:.0f}s", flush=True)
    out = {
        "workload": "video-like 1,000,000 x 2,400 (rank-10 background x 0.1 + 2% U[0,1) foreground), k=30, "
                    "50 iterations, cold BPP, W and H initialised U[0,1) from seed 150909318",
        "source": "oracle.anls (FP64 CPU oracle), inputs from the host recipes of nmf_inputs",
        "r_half": [float(x) for x in res["r_half"]],
        "r_full": [float(x) for x in res["r_full"]],
        "rounds_w": [int(x) for x in res["rounds_w"]],
        "rounds_h": [int(x) for x in res["rounds_h"]],
        "capped": res["capped"],
        # final supports {i : x_i > 0} and passive sets of a row sample of W (every
        # SAMPLE_STRIDE-th row) and of every row of H^T, as hexadecimal bit masks
        "sample_stride_w": SAMPLE_STRIDE,
        "support_w": [hex_mask(x) for x in res["W"][::SAMPLE_STRIDE]],
        "support_h": [hex_mask(x) for x in res["Ht"]],
        "passive_w": [format(int(v), "x") for v in res["masks_w"][::SAMPLE_STRIDE]],
        "passive_h": [format(int(v), "x") for v in res["masks_h"]],
        "fro2": res["fro2"],
        "oracle_seconds": t_orc,
        "host_threads": os.cpu_count(),
    }
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
