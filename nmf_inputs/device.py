"""Device-side builders for the synthetic workloads (thin ctypes layer over
libnmf_inputs.so, which implements the same Philox recipes as configs.py).

Large matrices (e.g. the 172,800 x 115,200 planted matrix, 79.6 GB) are built
directly in device memory; the host recipes regenerate any sampled row for the
CPU oracle.  torch supplies device memory and the stream only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import configs as C

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnmf_inputs.so")
SRC = os.path.join(_HERE, "csrc", "gen.hip")

_lib = None


def build(verbose: bool = False) -> str:
    cmd = ["hipcc", "--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-std=c++17",
           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           SRC, "-o", LIB_PATH + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("building libnmf_inputs.so failed:\n" + res.stderr)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    if verbose:
        print("built", LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        i64, u32, vp = ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p
        L.nmfin_uniform.argtypes = [u32, u32, i64, i64, i64, i64, vp, i64, i64, vp]
        L.nmfin_planted.argtypes = [u32, u32, i64, i64, ctypes.c_int, ctypes.c_double, vp, vp, vp, i64, vp]
        L.nmfin_video.argtypes = [u32, u32, u32, i64, i64, vp, vp, vp, i64, vp]
        for f in (L.nmfin_uniform, L.nmfin_planted, L.nmfin_video):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what} failed with status {rc}")


def uniform(seed, mid, rows, cols, *, transpose=False, row0=0, col0=0, out=None):
    """U[0,1) block as a float32 device tensor; transpose stores it (cols x rows)."""
    import torch
    if out is None:
        shape = (cols, rows) if transpose else (rows, cols)
        out = torch.empty(shape, dtype=torch.float32, device="cuda")
    ld_r, ld_c = (1, rows) if transpose else (cols, 1)
    if transpose:
        ld_r, ld_c = 1, out.stride(0)
    else:
        ld_r, ld_c = out.stride(0), 1
    _check(lib().nmfin_uniform(seed, mid, row0, rows, col0, cols, ctypes.c_void_p(out.data_ptr()),
                               ld_r, ld_c, _stream()), "nmfin_uniform")
    return out


def planted(seed, m, n, r, noise=0.01, inst=None, lda=None):
    import torch
    lda = n if lda is None else lda
    w0 = uniform(seed, C.mid(C.MID_W0, inst), m, r)
    h0t = uniform(seed, C.mid(C.MID_H0, inst), r, n, transpose=True)
    a = torch.empty((m, lda), dtype=torch.float32, device="cuda")
    _check(lib().nmfin_planted(seed, C.mid(C.MID_NOISE, inst), m, n, r, float(noise),
                               ctypes.c_void_p(w0.data_ptr()), ctypes.c_void_p(h0t.data_ptr()),
                               ctypes.c_void_p(a.data_ptr()), lda, _stream()), "nmfin_planted")
    del w0, h0t
    return a


def video(seed, m, n, lda=None):
    import torch
    lda = n if lda is None else lda
    wb = uniform(seed, C.MID_WB, m, C.VIDEO_RANK)
    hbt = uniform(seed, C.MID_HB, C.VIDEO_RANK, n, transpose=True)
    a = torch.empty((m, lda), dtype=torch.float32, device="cuda")
    _check(lib().nmfin_video(seed, C.MID_FGMASK, C.MID_FGVAL, m, n, ctypes.c_void_p(wb.data_ptr()),
                             ctypes.c_void_p(hbt.data_ptr()), ctypes.c_void_p(a.data_ptr()), lda,
                             _stream()), "nmfin_video")
    del wb, hbt
    return a


def init_factors(seed, m, n, k, inst=None):
    """W (m x k) and Ht (n x k) U[0,1) device tensors, same values as configs.init_*."""
    w = uniform(seed, C.mid(C.MID_WINIT, inst), m, k)
    ht = uniform(seed, C.mid(C.MID_HINIT, inst), k, n, transpose=True)
    return w, ht


def dense(w: C.Workload, lda=None):
    """Device copy of a dense workload's A."""
    import torch
    if w.kind == "planted":
        return planted(w.seed, w.m, w.n, w.rank, inst=w.inst, lda=lda)
    if w.kind == "video":
        return video(w.seed, w.m, w.n, lda=lda)
    if w.kind == "config1":
        a = C.config1_matrix(w.m, w.n, w.rank)
        return torch.from_numpy(np.ascontiguousarray(a)).cuda()
    raise ValueError(w.name)
