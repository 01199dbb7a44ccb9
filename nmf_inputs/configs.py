"""Seeded synthetic workloads shaped like the paper's dense, sparse and video data.

The paper's own datasets (Section "Datasets": DSYN, SSYN, the Video recording and
Webbase) are not available; these recipes stand in for them.  Everything is
addressable element by element through Philox counters, so a row, a column or a
single entry of a 79.6 GB matrix can be rebuilt on the host without the rest.

Recipes (all values are float32 once stored; intermediate sums are float64 and
added in index order, so host and device reproduce them bit for bit):

* planted dense  A = fl32( sum_{l<r} W0[i,l] H0[l,j]  +  s * u[i,j] ),
  W0, H0, u ~ U[0,1); each product of two 24-bit uniforms is exact in float64.
* video-like     B = fl64(sum_{l<10} Wb[i,l] Hb[l,j]) * 0.1  (values in [0,1));
  entry replaced by an independent U[0,1) value where a U[0,1) draw is < 0.02.
* sparse         per row, Bernoulli(density) column positions drawn by geometric
  gaps; values 1 - U[0,1) in (0, 1].
* initial factors W (m x k) and H (k x n) ~ U[0,1).

This module holds input generation only; none of the factorisation's
arithmetic lives here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .philox import uniform, uniform_at

SEED_BASE = 150909313

# matrix identifiers (second key word)
MID_W0 = 1
MID_H0 = 2
MID_NOISE = 3
MID_WINIT = 4
MID_HINIT = 5
MID_FGMASK = 6
MID_FGVAL = 7
MID_WB = 8
MID_HB = 9
MID_GAUSS = 10
MID_GAP = 11
MID_VAL = 12
MID_SHAPES = 13
MID_MLP = 14

VIDEO_RANK = 10
VIDEO_FG_DENSITY = 0.02
VIDEO_SCALE = 0.1


def seed_for(config: int) -> int:
    return SEED_BASE + int(config)


def mid(base: int, inst: int | None = None) -> int:
    """Key word 1: the matrix id, tagged with an instance number for batches."""
    return int(base) if inst is None else int(base) + 256 * (int(inst) + 1)


# ----------------------------------------------------------------------------
# dense planted matrices (configs 2 and 4, and their scaled test instances)
# ----------------------------------------------------------------------------

def planted_rows(seed: int, n: int, r: int, rows, noise: float = 0.01,
                 inst: int | None = None, cols=None) -> np.ndarray:
    """Rows `rows` (and optionally only columns `cols`) of a planted matrix."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.arange(n, dtype=np.int64) if cols is None else np.asarray(cols, np.int64)
    w0 = uniform_at(seed, mid(MID_W0, inst), rows[:, None], np.arange(r)[None, :]).astype(np.float64)
    h0 = uniform_at(seed, mid(MID_H0, inst), np.arange(r)[:, None], cols[None, :]).astype(np.float64)
    s = np.zeros((rows.size, cols.size), dtype=np.float64)
    for l in range(r):
        s += w0[:, l:l + 1] * h0[l:l + 1, :]
    u = uniform_at(seed, mid(MID_NOISE, inst), rows[:, None], cols[None, :]).astype(np.float64)
    s += np.float64(noise) * u
    return s.astype(np.float32)


def planted_dense(seed: int, m: int, n: int, r: int, noise: float = 0.01,
                  inst: int | None = None) -> np.ndarray:
    return planted_rows(seed, n, r, np.arange(m), noise, inst)


# ----------------------------------------------------------------------------
# video-like matrix (config 5): low-rank background plus sparse foreground
# ----------------------------------------------------------------------------

def video_rows(seed: int, n: int, rows, cols=None) -> np.ndarray:
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.arange(n, dtype=np.int64) if cols is None else np.asarray(cols, np.int64)
    wb = uniform_at(seed, MID_WB, rows[:, None], np.arange(VIDEO_RANK)[None, :]).astype(np.float64)
    hb = uniform_at(seed, MID_HB, np.arange(VIDEO_RANK)[:, None], cols[None, :]).astype(np.float64)
    s = np.zeros((rows.size, cols.size), dtype=np.float64)
    for l in range(VIDEO_RANK):
        s += wb[:, l:l + 1] * hb[l:l + 1, :]
    s *= np.float64(VIDEO_SCALE)
    fg = uniform_at(seed, MID_FGMASK, rows[:, None], cols[None, :]) < np.float32(VIDEO_FG_DENSITY)
    val = uniform_at(seed, MID_FGVAL, rows[:, None], cols[None, :]).astype(np.float64)
    s = np.where(fg, val, s)
    return s.astype(np.float32)


def video_dense(seed: int, m: int, n: int) -> np.ndarray:
    return video_rows(seed, n, np.arange(m))


# ----------------------------------------------------------------------------
# config 1: tiny planted matrix with half-normal noise (host only)
# ----------------------------------------------------------------------------

def config1_matrix(m: int = 200, n: int = 150, r: int = 5, sigma: float = 0.01) -> np.ndarray:
    """A = W0 H0 + |N(0, sigma^2)| via Box-Muller on two U[0,1) streams."""
    seed = seed_for(1)
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    w0 = uniform(seed, MID_W0, 0, m, 0, r).astype(np.float64)
    h0 = uniform(seed, MID_H0, 0, r, 0, n).astype(np.float64)
    s = np.zeros((m, n), dtype=np.float64)
    for l in range(r):
        s += w0[:, l:l + 1] * h0[l:l + 1, :]
    u1 = 1.0 - uniform_at(seed, MID_NOISE, i, j).astype(np.float64)   # (0, 1]
    u2 = uniform_at(seed, MID_GAUSS, i, j).astype(np.float64)
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    s += sigma * np.abs(z)
    return s.astype(np.float32)


# ----------------------------------------------------------------------------
# initial factors
# ----------------------------------------------------------------------------

def init_w(seed: int, m: int, k: int, inst: int | None = None, rows=None) -> np.ndarray:
    rows = np.arange(m) if rows is None else np.asarray(rows)
    return uniform_at(seed, mid(MID_WINIT, inst), rows[:, None], np.arange(k)[None, :])


def init_ht(seed: int, n: int, k: int, inst: int | None = None, cols=None) -> np.ndarray:
    """H (k x n) drawn with counter (l, j), returned transposed as Ht (n x k)."""
    cols = np.arange(n) if cols is None else np.asarray(cols)
    return uniform_at(seed, mid(MID_HINIT, inst), np.arange(k)[None, :], cols[:, None])


# ----------------------------------------------------------------------------
# sparse matrices (config 3)
# ----------------------------------------------------------------------------

def sparse_csr(seed: int, m: int, n: int, density: float, inst: int | None = None, workers: int = 1):
    """Erdos-Renyi CSR: every entry is nonzero independently with prob. `density`.

    Row i's positions come from geometric gaps g_t = floor(log(u_t)/log(1-p)),
    u_t in (0,1] from the row's own Philox stream (counter (i, t)).  Returns
    (rowptr int64[m+1], colidx int32[nnz], vals float32[nnz]); columns sorted.
    workers > 1 builds the row chunks on that many host threads (the result
    does not depend on it).
    """
    lp = math.log1p(-density)
    mean = n * density
    t_cap = int(mean + 8.0 * math.sqrt(mean + 1.0) + 16)
    counts = np.zeros(m, dtype=np.int64)
    chunk = max(1, min(m, 2_000_000 // max(t_cap, 1)))

    def rows_chunk(r0):
        r1 = min(m, r0 + chunk)
        nr = r1 - r0
        t = t_cap
        while True:
            u = 1.0 - uniform(seed, mid(MID_GAP, inst), r0, nr, 0, t).astype(np.float64)
            gaps = np.floor(np.log(u) / lp).astype(np.int64)
            pos = np.cumsum(gaps + 1, axis=1) - 1
            if np.all(pos[:, -1] >= n):
                break
            t *= 2
        keep = pos < n
        counts[r0:r1] = keep.sum(axis=1)
        vals = 1.0 - uniform(seed, mid(MID_VAL, inst), r0, nr, 0, t)
        return pos[keep].astype(np.int32), vals[keep].astype(np.float32)

    starts = range(0, m, chunk)
    if workers > 1:
        import concurrent.futures as cf
        with cf.ThreadPoolExecutor(max_workers=workers) as ex:
            parts = list(ex.map(rows_chunk, starts))
    else:
        parts = [rows_chunk(r0) for r0 in starts]
    rows_cols = [p[0] for p in parts]
    rows_vals = [p[1] for p in parts]
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    colidx = np.concatenate(rows_cols) if rows_cols else np.zeros(0, np.int32)
    vals = np.concatenate(rows_vals) if rows_vals else np.zeros(0, np.float32)
    return rowptr, colidx, vals


def csr_transpose(m: int, n: int, rowptr, colidx, vals):
    """CSR of A^T (n x m) from CSR of A; a pure re-indexing of the same entries."""
    rowptr = np.asarray(rowptr, np.int64)
    nnz = int(rowptr[-1])
    rows = np.repeat(np.arange(m, dtype=np.int64), np.diff(rowptr))
    order = np.argsort(colidx[:nnz], kind="stable")
    colT = rows[order].astype(np.int32)
    valT = np.asarray(vals)[order]
    counts = np.bincount(colidx[:nnz], minlength=n)
    rpT = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rpT[1:])
    return rpT, colT, valT


def csr_to_dense(m: int, n: int, rowptr, colidx, vals) -> np.ndarray:
    a = np.zeros((m, n), dtype=np.float32)
    rows = np.repeat(np.arange(m), np.diff(rowptr))
    a[rows, colidx] = vals
    return a


# ----------------------------------------------------------------------------
# config 4: shapes of the batched instances
# ----------------------------------------------------------------------------

def batched_shapes(count: int = 256, seed: int | None = None):
    """(m, n, k) per instance: m, n log-uniform in [500,8000] / [500,4000]."""
    seed = seed_for(4) if seed is None else seed
    idx = np.arange(count)
    u = [uniform_at(seed, MID_SHAPES, idx, np.full(count, c)).astype(np.float64) for c in range(3)]
    lm = math.log(500.0) + u[0] * (math.log(8000.0) - math.log(500.0))
    ln = math.log(500.0) + u[1] * (math.log(4000.0) - math.log(500.0))
    ms = np.floor(np.exp(lm)).astype(np.int64)
    ns = np.floor(np.exp(ln)).astype(np.int64)
    ks = np.array([10, 20, 50])[np.minimum(2, np.floor(u[2] * 3).astype(np.int64))]
    return [(int(a), int(b), int(c)) for a, b, c in zip(ms, ns, ks)]


# ----------------------------------------------------------------------------
# learned warm start: initial network weights (He-normal, biases zero)
# ----------------------------------------------------------------------------

MLP_HIDDEN = 128


def mlp_layout(k: int, hidden: int = MLP_HIDDEN):
    """Offsets of the flat float32 parameter vector: W1[2k][h], b1[h], W2[h][h],
    b2[h], W3[h][k], b3[k] (weights stored input-major)."""
    sizes = [("W1", 2 * k * hidden), ("b1", hidden), ("W2", hidden * hidden),
             ("b2", hidden), ("W3", hidden * k), ("b3", k)]
    off, out = 0, {}
    for name, sz in sizes:
        out[name] = (off, sz)
        off += sz
    out["total"] = (0, off)
    return out


def mlp_init(k: int, seed: int, side: int = 0, hidden: int = MLP_HIDDEN) -> np.ndarray:
    lay = mlp_layout(k, hidden)
    total = lay["total"][1]
    p = np.zeros(total, dtype=np.float32)
    fan = {"W1": 2 * k, "W2": hidden, "W3": hidden}
    for li, name in enumerate(("W1", "W2", "W3")):
        off, sz = lay[name]
        idx = np.arange(sz)
        m_id = mid(MID_MLP, side)
        u1 = 1.0 - uniform_at(seed, m_id, np.full(sz, 2 * li), idx).astype(np.float64)
        u2 = uniform_at(seed, m_id, np.full(sz, 2 * li + 1), idx).astype(np.float64)
        z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
        p[off:off + sz] = (z * math.sqrt(2.0 / fan[name])).astype(np.float32)
    return p


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    kind: str          # "planted" | "video" | "sparse" | "config1"
    m: int
    n: int
    k: int
    iters: int
    seed: int
    rank: int = 0      # planted rank
    density: float = 0.0
    inst: int | None = None


WORKLOADS = {
    "c1": Workload("c1", "config1", 200, 150, 5, 10, seed_for(1), rank=5),
    "c2": Workload("c2", "planted", 172_800, 115_200, 50, 30, seed_for(2), rank=50),
    "c2s": Workload("c2s", "planted", 1_728, 1_152, 50, 30, seed_for(2), rank=50),
    "c3": Workload("c3", "sparse", 207_360, 138_240, 50, 30, seed_for(3), density=1e-3),
    "c3s": Workload("c3s", "sparse", 2_000, 1_500, 50, 30, seed_for(3), density=1e-3, inst=1),
    "c5": Workload("c5", "video", 1_000_000, 2_400, 30, 50, seed_for(5)),
    "c5s": Workload("c5s", "video", 20_000, 2_400, 30, 50, seed_for(5)),
}


def dense_rows(w: Workload, rows, cols=None) -> np.ndarray:
    if w.kind == "planted":
        return planted_rows(w.seed, w.n, w.rank, rows, inst=w.inst, cols=cols)
    if w.kind == "video":
        return video_rows(w.seed, w.n, rows, cols)
    if w.kind == "config1":
        a = config1_matrix(w.m, w.n, w.rank)
        a = a[np.asarray(rows)]
        return a if cols is None else a[:, np.asarray(cols)]
    raise ValueError(f"{w.name} is not dense")
