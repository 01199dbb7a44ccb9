"""Writes the stored expected values under tests/golden/ from the CPU oracle.

Calls only oracle/ and nmf_inputs (the shared seeded input generators); no
value here ever comes from the GPU path.  Run from the repository root:
    python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from nmf_inputs import configs as C  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def masks_digest(m):
    return hashlib.sha256(np.ascontiguousarray(m, dtype=np.uint64).tobytes()).hexdigest()


def config1():
    w = C.WORKLOADS["c1"]
    A = C.config1_matrix(w.m, w.n, w.rank)
    W0 = C.init_w(w.seed, w.m, w.k)
    H0 = C.init_ht(w.seed, w.n, w.k)
    res = oracle.anls(w.k, W0, H0, w.iters, dense=A)
    return {
        "workload": "200x150 planted rank-5 + |N(0,0.01)|, k=5, 10 iterations, cold BPP",
        "source": "oracle.anls (FP64 CPU oracle); Algorithm 1 with BPP subproblems",
        "r_half": [float(x) for x in res["r_half"]],
        "r_full": [float(x) for x in res["r_full"]],
        "rounds_w": [int(x) for x in res["rounds_w"]],
        "rounds_h": [int(x) for x in res["rounds_h"]],
        "masks_w_sha256": masks_digest(res["masks_w"]),
        "masks_h_sha256": masks_digest(res["masks_h"]),
        "A_sha256": hashlib.sha256(A.tobytes()).hexdigest(),
    }


def config3_small():
    w = C.WORKLOADS["c3s"]
    rp, ci, va = C.sparse_csr(w.seed, w.m, w.n, w.density, inst=w.inst)
    rpt, cit, vat = C.csr_transpose(w.m, w.n, rp, ci, va)
    W0 = C.init_w(w.seed, w.m, w.k, inst=w.inst)
    H0 = C.init_ht(w.seed, w.n, w.k, inst=w.inst)
    res = oracle.anls(w.k, W0, H0, w.iters, csr=(rp, ci, va), csr_t=(rpt, cit, vat), shape=(w.m, w.n))
    return {
        "workload": "2000x1500 CSR, density 1e-3, k=50, 30 iterations, cold BPP",
        "source": "oracle.anls (FP64 CPU oracle)",
        "nnz": int(rp[-1]),
        "r_half": [float(x) for x in res["r_half"]],
        "r_full": [float(x) for x in res["r_full"]],
        "rounds_w": [int(x) for x in res["rounds_w"]],
        "rounds_h": [int(x) for x in res["rounds_h"]],
    }


if __name__ == "__main__":
    oracle.build()
    for name, fn in (("config1_oracle.json", config1), ("config3_small_oracle.json", config3_small)):
        with open(os.path.join(HERE, name), "w") as fh:
            json.dump(fn(), fh, indent=1)
        print("wrote", name)
