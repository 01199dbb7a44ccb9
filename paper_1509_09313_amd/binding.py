"""Python binding of libnmf (ctypes).  Argument marshalling only: every step
of the computation runs in the HIP kernels of libnmf.so.  torch supplies device
memory and the current stream.  There is no fallback: if libnmf.so is missing
or was not built for this GPU, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnmf.so")

NMF_OK, NMF_EINVAL, NMF_EUNSUPPORTED, NMF_EHIP, NMF_EWORKSPACE = 0, 1, 2, 3, 4
NMF_F32, NMF_BF16X3 = 0, 1
NMF_SIDE_W, NMF_SIDE_H = 0, 1
NMF_DENSE, NMF_CSR = 0, 1
NMF_OBJ_DIRECT, NMF_OBJ_TRACE = 0, 1
NMF_WARM_COLD, NMF_WARM_PREV, NMF_WARM_LEARNED, NMF_WARM_ALL = 0, 1, 2, 3
NMF_SOLVER_BPP, NMF_SOLVER_HALS, NMF_SOLVER_MU = 0, 1, 2
NMF_BPP_WARM_FALLBACK, NMF_BPP_CAPPED, NMF_BPP_PINNED, NMF_BPP_SINGULAR = 1, 2, 4, 8
NMF_BPP_COUNTERS = 6
NMF_BATCH_RESET = 1
PHASES = ("rhs_w", "infer_w", "bpp_w", "gram_w", "rhs_h", "infer_h", "bpp_h", "gram_h", "other")
NMF_PHASES = len(PHASES)


class NmfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libnmf error {code}: {msg}")
        self.code = code


vp = ctypes.c_void_p
i64 = ctypes.c_int64
ci = ctypes.c_int


class nmf_matrix(ctypes.Structure):
    _fields_ = [("kind", ci), ("m", i64), ("n", i64),
                ("A", vp), ("lda", i64),
                ("A_bf16", vp), ("At_bf16", vp),
                ("At", vp), ("ldat", i64),
                ("nnz", i64),
                ("rowptr", vp), ("colidx", vp), ("vals", vp),
                ("rowptr_t", vp), ("colidx_t", vp), ("vals_t", vp),
                ("fro2", vp)]


class nmf_opts(ctypes.Structure):
    _fields_ = [("prec", ci), ("warm", ci), ("max_rounds", ci), ("warm_cap", ci),
                ("trace_objective", ci), ("reset_masks", ci),
                ("net_w", vp), ("net_h", vp),
                ("collect", ci), ("collect_stride_w", ci), ("collect_stride_h", ci),
                ("coll_phi_w", vp), ("coll_mask_w", vp), ("coll_cap_w", i64), ("coll_off_w", i64),
                ("coll_phi_h", vp), ("coll_mask_h", vp), ("coll_cap_h", i64), ("coll_off_h", i64),
                ("phase_events", ctypes.POINTER(vp)), ("phase_events_cap", ci), ("solver", ci)]


class nmf_iter_stats(ctypes.Structure):
    _fields_ = [("r_half", ctypes.c_double), ("r_full", ctypes.c_double),
                ("bpp_w", ctypes.c_uint64 * NMF_BPP_COUNTERS),
                ("bpp_h", ctypes.c_uint64 * NMF_BPP_COUNTERS),
                ("capped", ctypes.c_uint64), ("fallback", ctypes.c_uint64)]


STATS_WORDS = ctypes.sizeof(nmf_iter_stats) // 8


class nmf_batch_problem(ctypes.Structure):
    _fields_ = [("m", i64), ("n", i64), ("k", ci), ("pad", ci), ("A_bf16", vp), ("At_bf16", vp),
                ("W", vp), ("ldw", i64), ("Ht", vp), ("ldh", i64)]


class nmf_batch_tune(ctypes.Structure):
    _fields_ = [("gram_tiles", ci), ("rhs_w_chunks", ci), ("rhs_h_chunks", ci), ("bpp_problems", ci),
                ("grid_scale", ci), ("warm_prev", ci), ("rhs_tile_rows", ci), ("bpp_wide", ci)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1509_09313_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        sz = ctypes.POINTER(ctypes.c_size_t)
        M = ctypes.POINTER(nmf_matrix)
        O = ctypes.POINTER(nmf_opts)
        BP = ctypes.POINTER(nmf_batch_problem)
        BT = ctypes.POINTER(nmf_batch_tune)
        sig = {
            "nmf_last_error": ([], ctypes.c_char_p),
            "nmf_version": ([], ctypes.c_char_p),
            "nmf_gram_workspace_bytes": ([i64, ci, sz], ci),
            "nmf_gram": ([i64, ci, vp, i64, vp, vp, ctypes.c_size_t, vp], ci),
            "nmf_gram_noalloc": ([i64, ci, vp, i64, vp, vp], ci),
            "nmf_rhs_dense_workspace_bytes": ([ci, i64, i64, ci, ci, sz], ci),
            "nmf_rhs_dense_chain": ([ci, i64, i64, ci, ci, ctypes.POINTER(i64)], ci),
            "nmf_rhs_dense": ([ci, i64, i64, ci, vp, i64, vp, vp, i64, vp, i64, ci, vp, ctypes.c_size_t, vp], ci),
            "nmf_split_bf16_bytes": ([i64, i64, ci], ctypes.c_size_t),
            "nmf_split_bf16": ([i64, i64, vp, i64, ci, vp, vp], ci),
            "nmf_transpose_f32": ([i64, i64, vp, i64, vp, i64, vp], ci),
            "nmf_rhs_csr": ([i64, i64, ci, vp, vp, vp, vp, i64, vp, i64, vp], ci),
            "nnls_bpp_batched": ([ci, i64, vp, vp, i64, vp, i64, vp, vp, vp, vp, ci, ci, vp, vp], ci),
            "nmf_local_update": ([ci, ci, i64, vp, vp, i64, vp, i64, vp], ci),
            "nmf_fro2_workspace_bytes": ([M, sz], ci),
            "nmf_fro2": ([M, vp, vp, ctypes.c_size_t, vp], ci),
            "nmf_objective_workspace_bytes": ([M, ci, ci, sz], ci),
            "nmf_objective": ([M, ci, vp, vp, ci, vp, vp, vp, vp, vp, ctypes.c_size_t, vp], ci),
            "nmf_anls_workspace_bytes": ([M, ci, O, sz], ci),
            "nmf_anls_iter": ([M, ci, vp, vp, ci, O, vp, vp, ctypes.c_size_t, vp], ci),
            "nmf_mlp_param_count": ([ci], ci),
            "nmf_events_create": ([ci, ctypes.POINTER(vp)], ci),
            "nmf_events_destroy": ([ci, ctypes.POINTER(vp)], ci),
            "nmf_events_elapsed_ms": ([vp, vp, ctypes.POINTER(ctypes.c_float)], ci),
            "nmf_features": ([ci, i64, vp, vp, i64, vp, vp], ci),
            "nmf_mlp_predict": ([ci, i64, vp, vp, i64, vp, vp, vp], ci),
            "nmf_mlp_train_workspace_bytes": ([ci, ci, sz], ci),
            "nmf_mlp_grad": ([ci, ci, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp], ci),
            "nmf_mlp_train": ([ci, vp, vp, vp, vp, vp, i64, vp, ci, ci, ctypes.c_float, i64, vp, vp,
                               ctypes.c_size_t, vp], ci),
            "nmf_batch_workspace_bytes": ([ci, BP, BT, sz], ci),
            "nmf_batch_plan_create": ([ci, BP, BT, vp, ctypes.c_size_t, ctypes.POINTER(vp)], ci),
            "nmf_batch_plan_destroy": ([vp], ci),
            "nmf_batch_iterate": ([vp, ci, vp, ci, vp], ci),
            "nmf_batch_graph_create": ([vp, ci, vp, ci, vp, ctypes.POINTER(vp)], ci),
            "nmf_batch_graph_launch": ([vp, vp], ci),
            "nmf_batch_graph_destroy": ([vp], ci),
            "nmf_batch_autotune": ([ci, BP, vp, ctypes.c_size_t, BT, ctypes.POINTER(ctypes.c_double), vp], ci),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        L.nmf_batch_tune_default.argtypes = [BT]
        L.nmf_batch_tune_default.restype = None
        _lib = L
    return _lib


def _check(rc):
    if rc != NMF_OK:
        raise NmfError(rc, lib().nmf_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ws(nbytes):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() == 2 and t.numel() > 0 and t.stride(1) != 1:
        raise ValueError(f"{name} must be row-major with unit column stride")
    return t


def _ld(t):
    return t.stride(0) if t.dim() == 2 else t.shape[-1]


def version() -> str:
    return lib().nmf_version().decode()


def nmf_gram(X, G=None):
    """G = X^T X (k x k, float64) for X (rows x k, float32)."""
    _dev(X, torch.float32, "X")
    rows, k = X.shape
    if G is None:
        G = torch.empty((k, k), dtype=torch.float64, device="cuda")
    nb = ctypes.c_size_t(0)
    _check(lib().nmf_gram_workspace_bytes(rows, k, ctypes.byref(nb)))
    ws = _ws(nb.value)
    _check(lib().nmf_gram(rows, k, _ptr(X), _ld(X), _ptr(G), _ptr(ws), nb.value, _stream()))
    return G


def nmf_gram_noalloc(X, G):
    """G = X^T X into the caller's G (k x k, float64), with no workspace and no
    allocation (the library's static device scratch)."""
    _dev(X, torch.float32, "X")
    _dev(G, torch.float64, "G")
    rows, k = X.shape
    if tuple(G.shape) != (k, k) or not G.is_contiguous():
        raise ValueError("G must be a contiguous k x k tensor")
    _check(lib().nmf_gram_noalloc(rows, k, _ptr(X), _ld(X), _ptr(G), _stream()))
    return G


def rhs_dense_chain(side, m, n, k, prec=NMF_F32) -> int:
    """Longest FP32 accumulation chain of nmf_rhs_dense on the current device."""
    t = i64(0)
    _check(lib().nmf_rhs_dense_chain(side, m, n, k, prec, ctypes.byref(t)))
    return int(t.value)


def nmf_split_bf16(X, transpose=False):
    """Padded BF16 (hi, lo) form of X (or of X^T) as a uint8 device buffer."""
    _dev(X, torch.float32, "X")
    rows, cols = X.shape
    nb = lib().nmf_split_bf16_bytes(rows, cols, int(transpose))
    out = torch.empty(max(int(nb), 16), dtype=torch.uint8, device="cuda")
    _check(lib().nmf_split_bf16(rows, cols, _ptr(X), _ld(X), int(transpose), _ptr(out), _stream()))
    return out


def nmf_transpose_f32(X):
    """X^T as a new contiguous FP32 device tensor (the library's transpose)."""
    _dev(X, torch.float32, "X")
    rows, cols = X.shape
    out = torch.empty((cols, rows), dtype=torch.float32, device="cuda")
    _check(lib().nmf_transpose_f32(rows, cols, _ptr(X), _ld(X), _ptr(out), rows, _stream()))
    return out


def unpack_bf16(buf, rows, cols):
    """Host helper for tests: (hi, lo) uint16 arrays (rows x cols) of the
    padded BF16 form of an operand with `rows` rows and `cols` columns."""
    import numpy as np
    Rp, Cp = -(-rows // 128) * 128, -(-cols // 64) * 64
    t = buf.cpu().numpy().view(np.uint16).reshape(2, Rp, Cp)
    return t[0, :rows, :cols], t[1, :rows, :cols]


def nmf_rhs_dense(side, A, Y, R=None, prec=NMF_F32, B_bf16=None, m=None, n=None):
    """side W: R = A @ Y (Y = Ht); side H: R = A^T @ Y (Y = W).  For BF16X3
    pass the padded BF16 form of A (side W) or of A^T (side H) as B_bf16."""
    _dev(Y, torch.float32, "Y")
    k = Y.shape[1]
    if A is not None:
        _dev(A, torch.float32, "A")
        m, n = A.shape
    rows_out = m if side == NMF_SIDE_W else n
    if R is None:
        R = torch.empty((rows_out, k), dtype=torch.float32, device="cuda")
    nb = ctypes.c_size_t(0)
    _check(lib().nmf_rhs_dense_workspace_bytes(side, m, n, k, prec, ctypes.byref(nb)))
    ws = _ws(nb.value)
    _check(lib().nmf_rhs_dense(side, m, n, k, _ptr(A), _ld(A) if A is not None else n, _ptr(B_bf16), _ptr(Y), _ld(Y),
                               _ptr(R), _ld(R), prec, _ptr(ws), nb.value, _stream()))
    return R


def nmf_rhs_csr(rowptr, colidx, vals, Y, rows, cols, R=None):
    _dev(Y, torch.float32, "Y")
    k = Y.shape[1]
    if R is None:
        R = torch.empty((rows, k), dtype=torch.float32, device="cuda")
    _check(lib().nmf_rhs_csr(rows, cols, k, _ptr(rowptr), _ptr(colidx), _ptr(vals), _ptr(Y), _ld(Y), _ptr(R), _ld(R),
                             _stream()))
    return R


def nmf_local_update(solver, G, R, X):
    """One HALS or MU update of the rows of X (rows x k float32, in place)
    from G (k x k float64) and R (rows x k float32).  Returns X."""
    _dev(G, torch.float64, "G")
    _dev(R, torch.float32, "R")
    _dev(X, torch.float32, "X")
    rows, k = X.shape
    _check(lib().nmf_local_update(solver, k, rows, _ptr(G), _ptr(R), _ld(R), _ptr(X), _ld(X), _stream()))
    return X


def nnls_bpp_batched(G, R, X=None, mask_in=None, mask_out=None, rounds=None, status=None, max_rounds=100,
                     warm_cap=8, counters=None):
    """Rows of R (batch x k, float32) against G (k x k, float64).  Returns
    (X, mask_out, rounds, status); masks are int64 tensors holding the uint64
    bit patterns."""
    _dev(G, torch.float64, "G")
    _dev(R, torch.float32, "R")
    batch, k = R.shape
    if X is None:
        X = torch.empty((batch, k), dtype=torch.float32, device="cuda")
    if mask_out is None:
        mask_out = torch.empty(batch, dtype=torch.int64, device="cuda")
    if rounds is None:
        rounds = torch.empty(batch, dtype=torch.uint8, device="cuda")
    if status is None:
        status = torch.empty(batch, dtype=torch.uint8, device="cuda")
    _check(lib().nnls_bpp_batched(k, batch, _ptr(G), _ptr(R), _ld(R), _ptr(X), _ld(X), _ptr(mask_in), _ptr(mask_out),
                                  _ptr(rounds), _ptr(status), max_rounds, warm_cap, _ptr(counters), _stream()))
    return X, mask_out, rounds, status


class Matrix:
    """Owner of the device tensors behind one nmf_matrix."""

    def __init__(self, *, dense=None, csr=None, csr_t=None, shape=None, split=False):
        self.keep = []
        s = nmf_matrix()
        if dense is not None:
            _dev(dense, torch.float32, "A")
            self.m, self.n = dense.shape
            s.kind, s.m, s.n, s.A, s.lda = NMF_DENSE, self.m, self.n, dense.data_ptr(), _ld(dense)
            self.keep.append(dense)
            self.A = dense
        else:
            self.m, self.n = shape
            rp, ci_, va = csr
            rpt, cit, vat = csr_t
            s.kind, s.m, s.n = NMF_CSR, self.m, self.n
            s.nnz = int(va.numel())
            s.rowptr, s.colidx, s.vals = rp.data_ptr(), ci_.data_ptr(), va.data_ptr()
            s.rowptr_t, s.colidx_t, s.vals_t = rpt.data_ptr(), cit.data_ptr(), vat.data_ptr()
            self.keep += [rp, ci_, va, rpt, cit, vat]
            self.A = None
        self.s = s
        self.fro2 = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.s.fro2 = self.fro2.data_ptr()
        nb = ctypes.c_size_t(0)
        _check(lib().nmf_fro2_workspace_bytes(ctypes.byref(self.s), ctypes.byref(nb)))
        ws = _ws(nb.value)
        _check(lib().nmf_fro2(ctypes.byref(self.s), _ptr(self.fro2), _ptr(ws), nb.value, _stream()))
        if split:
            self.add_split()

    def add_split(self):
        bt = nmf_split_bf16(self.A)
        btt = nmf_split_bf16(self.A, transpose=True)
        self.keep += [bt, btt]
        self.tiled = (bt, btt)
        self.s.A_bf16, self.s.At_bf16 = bt.data_ptr(), btt.data_ptr()

    def add_transposed(self):
        """The FP32 form's second orientation: a resident copy of A^T, which
        nmf_anls_iter's side-H product then streams by rows."""
        at = nmf_transpose_f32(self.A)
        self.keep.append(at)
        self.At = at
        self.s.At, self.s.ldat = at.data_ptr(), _ld(at)

    def drop_transposed(self):
        """Releases the resident A^T (the FP32 side-H product then streams A)."""
        at = getattr(self, "At", None)
        if at is not None:
            self.keep = [t for t in self.keep if t is not at]
            self.At = None
            self.s.At, self.s.ldat = None, 0

    def ref(self):
        return ctypes.byref(self.s)


def nmf_objective(M: Matrix, W, Ht, mode=NMF_OBJ_DIRECT, G_W=None, G_H=None, R_H=None):
    """Tensor [r, ||A-WH||^2, ||A||^2] (float64, device)."""
    k = W.shape[1]
    out = torch.empty(3, dtype=torch.float64, device="cuda")
    nb = ctypes.c_size_t(0)
    _check(lib().nmf_objective_workspace_bytes(M.ref(), k, mode, ctypes.byref(nb)))
    ws = _ws(nb.value)
    _check(lib().nmf_objective(M.ref(), k, _ptr(W), _ptr(Ht), mode, _ptr(G_W), _ptr(G_H), _ptr(R_H), _ptr(out),
                               _ptr(ws), nb.value, _stream()))
    return out


def make_opts(prec=NMF_F32, warm=NMF_WARM_COLD, max_rounds=100, warm_cap=8, trace=True, reset_masks=True,
              net_w=None, net_h=None, solver=NMF_SOLVER_BPP):
    o = nmf_opts()
    o.prec, o.warm, o.max_rounds, o.warm_cap = prec, warm, max_rounds, warm_cap
    o.solver = solver
    o.trace_objective, o.reset_masks = int(trace), int(reset_masks)
    o.net_w = None if net_w is None else net_w.data_ptr()
    o.net_h = None if net_h is None else net_h.data_ptr()
    return o


class Anls:
    """Keeps the workspace of nmf_anls_iter alive between calls (the stored
    passive sets carry over for the previous-iterate warm start)."""

    def __init__(self, M: Matrix, k: int, opts: nmf_opts):
        self.M, self.k, self.opts = M, k, opts
        nb = ctypes.c_size_t(0)
        _check(lib().nmf_anls_workspace_bytes(M.ref(), k, ctypes.byref(opts), ctypes.byref(nb)))
        self.ws_bytes = nb.value
        self.ws = _ws(nb.value)

    def run(self, W, Ht, iters, stats=None):
        _dev(W, torch.float32, "W")
        _dev(Ht, torch.float32, "Ht")
        _check(lib().nmf_anls_iter(self.M.ref(), self.k, _ptr(W), _ptr(Ht), iters, ctypes.byref(self.opts),
                                   _ptr(stats), _ptr(self.ws), self.ws_bytes, _stream()))
        return stats


def new_stats(iters):
    return torch.zeros((iters, STATS_WORDS), dtype=torch.int64, device="cuda")


def decode_stats(stats):
    """Host dicts from a stats tensor."""
    raw = stats.cpu().contiguous()
    arr = (nmf_iter_stats * raw.shape[0]).from_buffer_copy(raw.numpy().tobytes())
    out = []
    for s in arr:
        out.append(dict(r_half=s.r_half, r_full=s.r_full, bpp_w=list(s.bpp_w), bpp_h=list(s.bpp_h),
                        capped=s.capped, fallback=s.fallback))
    return out


def nmf_anls_iter(M: Matrix, k, W, Ht, iters, opts=None, stats=None):
    opts = opts or make_opts()
    runner = Anls(M, k, opts)
    runner.run(W, Ht, iters, stats)
    return runner


# ---------------------------------------------------------------- network --
def nmf_mlp_param_count(k):
    return lib().nmf_mlp_param_count(k)


def nmf_features(G, R):
    _dev(G, torch.float64, "G")
    _dev(R, torch.float32, "R")
    batch, k = R.shape
    phi = torch.empty((batch, 2 * k), dtype=torch.float32, device="cuda")
    _check(lib().nmf_features(k, batch, _ptr(G), _ptr(R), _ld(R), _ptr(phi), _stream()))
    return phi


def nmf_mlp_predict(G, R, params, mask_out=None):
    _dev(G, torch.float64, "G")
    _dev(R, torch.float32, "R")
    batch, k = R.shape
    if mask_out is None:
        mask_out = torch.empty(batch, dtype=torch.int64, device="cuda")
    _check(lib().nmf_mlp_predict(k, batch, _ptr(G), _ptr(R), _ld(R), _ptr(params), _ptr(mask_out), _stream()))
    return mask_out


def nmf_mlp_grad(k, params, phi, masks, batch=None):
    batch = phi.shape[0] if batch is None else batch
    nb = ctypes.c_size_t(0)
    _check(lib().nmf_mlp_train_workspace_bytes(k, batch, ctypes.byref(nb)))
    ws = _ws(nb.value)
    grad = torch.empty(nmf_mlp_param_count(k), dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    _check(lib().nmf_mlp_grad(k, batch, _ptr(params), _ptr(phi), _ptr(masks), _ptr(grad), _ptr(loss), _ptr(ws),
                              nb.value, _stream()))
    return grad, loss


class MlpTrainer:
    """Parameters and Adam moments of one network, trained by nmf_mlp_train."""

    def __init__(self, k, params, batch=1024, lr=1e-3):
        self.k, self.batch, self.lr = k, batch, lr
        self.params = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.step = 0
        nb = ctypes.c_size_t(0)
        _check(lib().nmf_mlp_train_workspace_bytes(k, batch, ctypes.byref(nb)))
        self.ws_bytes = nb.value
        self.ws = _ws(nb.value)
        self.loss = torch.zeros(1, dtype=torch.float64, device="cuda")

    def train(self, phi, masks, nsamples, steps, order=None):
        _check(lib().nmf_mlp_train(self.k, _ptr(self.params), _ptr(self.m), _ptr(self.v), _ptr(phi), _ptr(masks),
                                   int(nsamples), _ptr(order), int(steps), self.batch, ctypes.c_float(self.lr),
                                   self.step, _ptr(self.loss), _ptr(self.ws), self.ws_bytes, _stream()))
        self.step += steps
        return self.loss


class PhaseTimer:
    """hipEvent pairs around every phase of `iters` ANLS iterations (see
    nmf_opts.phase_events); read back after the stream has completed."""

    def __init__(self, iters):
        self.iters = iters
        self.n = 2 * NMF_PHASES * iters
        self.events = (vp * self.n)()
        _check(lib().nmf_events_create(self.n, self.events))

    def attach(self, opts):
        opts.phase_events = self.events
        opts.phase_events_cap = self.n
        return opts

    def detach(self, opts):
        opts.phase_events = None
        opts.phase_events_cap = 0
        return opts

    def phase_ms(self):
        """{phase: [ms per iteration]} (the events must have completed)."""
        out = {p: [] for p in PHASES}
        ms = ctypes.c_float(0)
        for t in range(self.iters):
            for ph, name in enumerate(PHASES):
                a = self.events[2 * (t * NMF_PHASES + ph)]
                b = self.events[2 * (t * NMF_PHASES + ph) + 1]
                _check(lib().nmf_events_elapsed_ms(a, b, ctypes.byref(ms)))
                out[name].append(ms.value)
        return out

    def close(self):
        if self.events is not None:
            lib().nmf_events_destroy(self.n, self.events)
            self.events = None


# ---------------------------------------------------------------- batches ----
def batch_tune_default() -> nmf_batch_tune:
    t = nmf_batch_tune()
    lib().nmf_batch_tune_default(ctypes.byref(t))
    return t


class Batch:
    """Many independent dense NMF problems run together by the grouped,
    persistent phase kernels of libnmf (nmf_batch_*).

    problems: list of dicts with keys A (m x n float32, CUDA), W (m x k),
    Ht (n x k).  The padded BF16 planes of A in both orientations are made
    here (nmf_split_bf16) and kept alive with the tensors."""

    def __init__(self, problems, tune=None):
        self.items = []
        P = (nmf_batch_problem * len(problems))()
        for i, pr in enumerate(problems):
            A, W, Ht = pr["A"], pr["W"], pr["Ht"]
            _dev(A, torch.float32, "A")
            _dev(W, torch.float32, "W")
            _dev(Ht, torch.float32, "Ht")
            m, n = A.shape
            k = W.shape[1]
            bt = nmf_split_bf16(A)
            btt = nmf_split_bf16(A, transpose=True)
            self.items.append((A, W, Ht, bt, btt))
            P[i] = nmf_batch_problem(m, n, k, 0, bt.data_ptr(), btt.data_ptr(), W.data_ptr(), _ld(W),
                                     Ht.data_ptr(), _ld(Ht))
        self.P = P
        self.count = len(problems)
        nb = ctypes.c_size_t(0)
        _check(lib().nmf_batch_workspace_bytes(self.count, P, None, ctypes.byref(nb)))
        self.ws = _ws(nb.value)
        self.plan = None
        self.graphs = []
        self.tune = None
        self.make_plan(tune)

    def make_plan(self, tune=None):
        if self.plan is not None:
            _check(lib().nmf_batch_plan_destroy(self.plan))
            self.plan = None
        torch.cuda.synchronize()
        h = vp()
        t = ctypes.byref(tune) if tune is not None else None
        _check(lib().nmf_batch_plan_create(self.count, self.P, t, _ptr(self.ws), self.ws.numel(), ctypes.byref(h)))
        self.plan = h
        self.tune = tune if tune is not None else batch_tune_default()
        self.fresh = True   # the kept passive sets are uninitialised until a reset

    def autotune(self):
        best = nmf_batch_tune()
        ms = ctypes.c_double(0.0)
        _check(lib().nmf_batch_autotune(self.count, self.P, _ptr(self.ws), self.ws.numel(), ctypes.byref(best),
                                        ctypes.byref(ms), _stream()))
        self.make_plan(best)
        return best, ms.value

    def iterate(self, iters, counters=None, reset=False):
        """Enqueues `iters` iterations; reset (or a new plan) starts every NNLS cold."""
        flags = NMF_BATCH_RESET if (reset or self.fresh) else 0
        _check(lib().nmf_batch_iterate(self.plan, int(iters), _ptr(counters), flags, _stream()))
        self.fresh = False

    def graph(self, iters, counters=None, reset=True):
        """Captures `iters` iterations on the current (non-default) stream;
        with reset every launch starts cold."""
        g = vp()
        flags = NMF_BATCH_RESET if reset else 0
        _check(lib().nmf_batch_graph_create(self.plan, int(iters), _ptr(counters), flags, _stream(),
                                            ctypes.byref(g)))
        self.graphs.append(g)
        return g

    def launch(self, g):
        _check(lib().nmf_batch_graph_launch(g, _stream()))

    def close(self):
        for g in self.graphs:
            lib().nmf_batch_graph_destroy(g)
        self.graphs = []
        if self.plan is not None:
            lib().nmf_batch_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
