"""FP64 oracle trajectories of Algorithm 1 with the HALS and MU local updates
on the video-like workload (1,000,000 x 2,400, k = 30, 50 iterations, from the
benchmark's seeded initial factors), stored in
tests/golden/video_1e6x2400_k30_local_oracle.json.

Calls only oracle/ (oracle.local.anls_trace) and the host recipes of
nmf_inputs; A is generated on the host in row chunks, so no value comes from
a GPU.  Needs about 12 GB of host memory; run from the repository root:
    python tests/golden/make_local_oracle.py
"""
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from nmf_inputs import configs as C  # noqa: E402
from oracle import local  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "video_1e6x2400_k30_local_oracle.json")
M, N, K, T = 1_000_000, 2_400, 30, 50
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
    W0 = C.init_w(C.seed_for(5), M, K)
    H0 = C.init_ht(C.seed_for(5), N, K)
    out = {"workload": "video-like 1,000,000 x 2,400 (rank-10 background x 0.1 + 2% U[0,1) foreground), k=30, "
                       "50 iterations, W and H initialised U[0,1) from seed 150909318",
           "source": "oracle.local.anls_trace (FP64 CPU oracle, trace-form objective), inputs from the host "
                     "recipes of nmf_inputs"}
    for solver in ("hals", "mu"):
        t1 = time.time()
        res = local.anls_trace(solver, K, W0, H0, T, A)
        out[solver] = {"r_half": [float(x) for x in res["r_half"]], "r_full": [float(x) for x in res["r_full"]],
                       "oracle_seconds": time.time() - t1}
        print(f"{solver}: r_50 = {res['r_full'][-1]:.10f} in {time.time() - t1:.0f}s", flush=True)
    out["fro2"] = res["fro2"]
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
