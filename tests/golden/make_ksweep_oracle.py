"""FP64 oracle trajectories of Algorithm 1 (cold BPP) on the video-like
workload (1,000,000 x 2,400) for k = 10, 20, 30, 40, 50, the first 10
iterations each, stored in tests/golden/video_1e6x2400_ksweep_oracle.json.
These are the ranks of the paper's algorithmic comparison (time per iteration
as k varies).

Calls only oracle/ and the host recipes of nmf_inputs; A is generated on the
host (row chunks in parallel processes), so no value comes from a GPU.
Needs about 30 GB of host memory; run from the repository root:
    python tests/golden/make_ksweep_oracle.py
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
OUT = os.path.join(HERE, "video_1e6x2400_ksweep_oracle.json")
M, N, T = 1_000_000, 2_400, 10
KS = (10, 20, 30, 40, 50)
CHUNK = 10_000


def rows_chunk(r0):
    return r0, C.video_rows(C.seed_for(5), N, np.arange(r0, min(M, r0 + CHUNK)))


def main(workers=6):
    t0 = time.time()
    A = np.empty((M, N), dtype=np.float32)
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        for r0, blk in ex.map(rows_chunk, range(0, M, CHUNK)):
            A[r0:r0 + blk.shape[0]] = blk
    print(f"generated A in {time.time() - t0:.0f}s", flush=True)
    out = {"workload": "video-like 1,000,000 x 2,400 (rank-10 background x 0.1 + 2% U[0,1) foreground), "
                       f"{T} iterations, cold BPP, W and H initialised U[0,1) from seed 150909318 at each k",
           "source": "oracle.anls (FP64 CPU oracle), inputs from the host recipes of nmf_inputs",
           "iterations": T, "host_threads": os.cpu_count(), "k": {}}
    for k in KS:
        t1 = time.time()
        res = oracle.anls(k, C.init_w(C.seed_for(5), M, k), C.init_ht(C.seed_for(5), N, k), T, dense=A)
        out["k"][str(k)] = {"r_half": [float(x) for x in res["r_half"]],
                            "r_full": [float(x) for x in res["r_full"]],
                            "rounds_w": [int(x) for x in res["rounds_w"]],
                            "rounds_h": [int(x) for x in res["rounds_h"]],
                            "capped": res["capped"], "oracle_seconds": time.time() - t1}
        out["fro2"] = res["fro2"]
        print(f"k={k}: r_{T} = {res['r_full'][-1]:.10f} in {time.time() - t1:.0f}s", flush=True)
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
