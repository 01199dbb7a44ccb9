"""Philox-4x32-10 counter-based generator (host side, NumPy).

Written from the published definition of Philox (Salmon, Moraes, Dror and
Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3", SC'11): ten rounds of a
multiply-hi/lo bijection on a 4x32-bit counter, keyed by a 2x32-bit key that is
advanced by the Weyl constants between rounds.

Every generated value is addressed by (key, counter), so any element of any
synthetic matrix can be regenerated on its own, on the host or the device,
without generating its neighbours.
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Return the four 32-bit output words (as uint32 arrays) for the counters.

    All arguments broadcast against each other; they are interpreted modulo 2^32.
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & _MASK for c in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & _MASK
    k1 = np.asarray(k1, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    c0, c1, c2, c3 = c0.copy(), c1.copy(), c2.copy(), c3.copy()
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def word0(seed: int, mid: int, rows, cols):
    """First output word for counter (row, col, 0, 0) under key (seed, mid)."""
    out = philox4x32_10(rows, cols, 0, 0, seed, mid)
    return out[0]


def u01_from_word(w):
    """U[0,1) as float32: the top 24 bits times 2^-24 (exact in float32)."""
    return ((np.asarray(w, dtype=np.uint32) >> np.uint32(8)).astype(np.float32)
            * np.float32(2.0 ** -24))


def uniform(seed: int, mid: int, row0: int, nrows: int, col0: int, ncols: int) -> np.ndarray:
    """Block [row0, row0+nrows) x [col0, col0+ncols) of the U[0,1) matrix (float32)."""
    r = np.arange(row0, row0 + nrows, dtype=np.uint64)[:, None]
    c = np.arange(col0, col0 + ncols, dtype=np.uint64)[None, :]
    return u01_from_word(word0(seed, mid, r, c))


def uniform_at(seed: int, mid: int, rows, cols) -> np.ndarray:
    """U[0,1) float32 values at explicit (row, col) index arrays."""
    return u01_from_word(word0(seed, mid, np.asarray(rows, np.uint64), np.asarray(cols, np.uint64)))
