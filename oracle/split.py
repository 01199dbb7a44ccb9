"""FP64 oracle of the split-precision right-hand sides -- TEST INFRASTRUCTURE ONLY.

Each FP32 value x is written as hi + lo with hi = bf16(x) (round to nearest
even) and lo = bf16(x - hi), where x - hi is exact in FP32.  The products use
three of the four cross terms, hi*hi + hi*lo + lo*hi, dropping lo*lo; here
they are formed and summed in float64, so the only difference left to the
GPU's FP32-accumulated MFMA chains is its accumulation rounding.
"""
from __future__ import annotations

import numpy as np


def bf16_rne_bits(x) -> np.ndarray:
    """uint16 bit patterns of bf16(x), round to nearest even (finite x)."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    bias = np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))
    return ((u + bias) >> np.uint64(16)).astype(np.uint16)


def bf16_to_f32(bits) -> np.ndarray:
    return (np.asarray(bits, dtype=np.uint32) << np.uint32(16)).view(np.float32)


def split(x):
    """(hi, lo) as float32 arrays holding bf16 values."""
    x = np.asarray(x, dtype=np.float32)
    hi = bf16_to_f32(bf16_rne_bits(x))
    lo = bf16_to_f32(bf16_rne_bits(x - hi))
    return hi, lo


def split_bits(x):
    x = np.asarray(x, dtype=np.float32)
    hb = bf16_rne_bits(x)
    lb = bf16_rne_bits(x - bf16_to_f32(hb))
    return hb, lb


def product3(A, Y):
    """A @ Y as hi(A) hi(Y) + hi(A) lo(Y) + lo(A) hi(Y), in float64."""
    ah, al = (t.astype(np.float64) for t in split(A))
    yh, yl = (t.astype(np.float64) for t in split(Y))
    return ah @ yh + ah @ yl + al @ yh


def rhs_w(A, Ht):
    """Split-precision A H^T."""
    return product3(A, Ht)


def rhs_h(A, W):
    """Split-precision (W^T A)^T = A^T W."""
    return product3(np.ascontiguousarray(np.asarray(A, np.float32).T), W)
