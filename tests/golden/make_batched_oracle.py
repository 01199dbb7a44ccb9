"""FP64 oracle trajectories for the batched workload: 256 independent dense
NMF problems (m log-uniform in [500, 8000], n log-uniform in [500, 4000],
k in {10, 20, 50}), each a planted rank-k matrix with U[0,1) factors plus
0.01 U[0,1) noise, 30 ANLS-BPP iterations from U[0,1) initial factors;
stored in tests/golden/batched_256_oracle.json.

Calls only oracle/ and the host recipes of nmf_inputs (no GPU).  Run from the
repository root:  python tests/golden/make_batched_oracle.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from nmf_inputs import configs as C  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "batched_256_oracle.json")
COUNT, T = 256, 30


def main():
    seed = C.seed_for(4)
    shapes = C.batched_shapes(COUNT, seed)
    out = {"workload": f"{COUNT} planted dense problems, shapes from nmf_inputs.configs.batched_shapes, "
                       f"rank k planted, noise 0.01 U[0,1), {T} iterations, cold BPP, seed {seed}",
           "source": "oracle.anls (FP64 CPU oracle), inputs from the host recipes of nmf_inputs",
           "iters": T, "instances": []}
    t0 = time.time()
    for i, (m, n, k) in enumerate(shapes):
        A = C.planted_dense(seed, m, n, k, 0.01, inst=i)
        W0 = C.init_w(seed, m, k, inst=i)
        H0 = C.init_ht(seed, n, k, inst=i)
        res = oracle.anls(k, W0, H0, T, dense=A)
        out["instances"].append({"m": m, "n": n, "k": k,
                                 "r_half": [float(x) for x in res["r_half"]],
                                 "r_full": [float(x) for x in res["r_full"]],
                                 "capped": res["capped"]})
        print(f"{i}: {m}x{n} k={k} r_T={res['r_full'][-1]:.9f} ({time.time() - t0:.0f}s)", flush=True)
    out["oracle_seconds"] = time.time() - t0
    out["host_threads"] = oracle.max_threads()
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
