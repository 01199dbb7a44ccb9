"""The C-ABI boundary on the host: libnmf.so loads, exports every function
include/libnmf.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "libnmf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(nmf_\w+|nnls_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_1509_09313_amd import binding as libnmf
    if not os.path.exists(libnmf.LIB_PATH):
        from paper_1509_09313_amd import build
        build.build()
    return libnmf


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("nmf_gram", "nmf_rhs_dense", "nmf_rhs_csr", "nnls_bpp_batched", "nmf_anls_iter",
                     "nmf_objective"):
        assert required in names


def test_every_declared_symbol_is_exported(L):
    lib = L.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_validation_without_gpu(L):
    lib = L.lib()
    G = ctypes.c_void_p(16)
    # k outside [1, 64]
    assert lib.nmf_gram(10, 0, G, 1, G, G, 1 << 20, None) == L.NMF_EINVAL
    assert b"k=0" in lib.nmf_last_error()
    assert lib.nmf_gram(10, 65, G, 65, G, G, 1 << 20, None) == L.NMF_EINVAL
    # ldx < k
    assert lib.nmf_gram(10, 8, G, 4, G, G, 1 << 20, None) == L.NMF_EINVAL
    # workspace too small
    nb = ctypes.c_size_t(0)
    assert lib.nmf_gram_workspace_bytes(1000, 8, ctypes.byref(nb)) == L.NMF_OK and nb.value > 0
    assert lib.nmf_gram(1000, 8, G, 8, G, G, nb.value - 1, None) == L.NMF_EWORKSPACE
    # the variant without a workspace checks the same arguments first
    assert lib.nmf_gram_noalloc(10, 0, G, 1, G, None) == L.NMF_EINVAL
    assert lib.nmf_gram_noalloc(10, 8, G, 4, G, None) == L.NMF_EINVAL
    assert lib.nmf_gram_noalloc(10, 8, G, 8, None, None) == L.NMF_EINVAL
    # BPP: bad caps and sizes
    assert lib.nnls_bpp_batched(8, 10, G, G, 8, G, 8, None, None, None, None, 0, 8, None, None) == L.NMF_EINVAL
    assert lib.nnls_bpp_batched(8, 10, G, G, 4, G, 8, None, None, None, None, 10, 8, None, None) == L.NMF_EINVAL
    assert lib.nnls_bpp_batched(8, 10, None, G, 8, G, 8, None, None, None, None, 10, 8, None, None) == L.NMF_EINVAL
    # RHS: bad side, bad prec, lda < n, missing tiled BF16 operand
    z = ctypes.c_void_p(0)
    assert lib.nmf_rhs_dense(7, 4, 4, 2, G, 4, z, G, 2, G, 2, 0, G, 1 << 20, None) == L.NMF_EINVAL
    assert lib.nmf_rhs_dense(0, 4, 4, 2, G, 4, z, G, 2, G, 2, 9, G, 1 << 20, None) == L.NMF_EINVAL
    assert lib.nmf_rhs_dense(0, 4, 4, 2, G, 3, z, G, 2, G, 2, 0, G, 1 << 20, None) == L.NMF_EINVAL
    assert lib.nmf_rhs_dense(0, 4, 4, 2, z, 4, z, G, 2, G, 2, 1, G, 1 << 20, None) == L.NMF_EINVAL
    assert lib.nmf_split_bf16_bytes(300, 70, 0) == 2 * 384 * 128 * 2
    assert lib.nmf_split_bf16_bytes(300, 70, 1) == 2 * 128 * 320 * 2
    # FP32 transpose: short leading dimensions, null pointers, empty matrices
    assert lib.nmf_transpose_f32(4, 6, G, 5, G, 4, None) == L.NMF_EINVAL
    assert lib.nmf_transpose_f32(4, 6, G, 6, G, 3, None) == L.NMF_EINVAL
    assert lib.nmf_transpose_f32(4, 6, None, 6, G, 4, None) == L.NMF_EINVAL
    assert lib.nmf_transpose_f32(-1, 6, G, 6, G, 4, None) == L.NMF_EINVAL
    assert lib.nmf_transpose_f32(0, 6, None, 6, None, 0, None) == L.NMF_OK
    # CSR: ld < k
    assert lib.nmf_rhs_csr(4, 4, 8, G, G, G, G, 4, G, 8, None) == L.NMF_EINVAL
    # HALS / MU: bad solver, k, ld; ANLS with HALS takes no warm start
    assert lib.nmf_local_update(0, 8, 10, G, G, 8, G, 8, None) == L.NMF_EINVAL
    assert lib.nmf_local_update(L.NMF_SOLVER_HALS, 0, 10, G, G, 8, G, 8, None) == L.NMF_EINVAL
    assert lib.nmf_local_update(L.NMF_SOLVER_MU, 8, 10, G, G, 4, G, 8, None) == L.NMF_EINVAL
    assert lib.nmf_local_update(L.NMF_SOLVER_MU, 8, 10, None, G, 8, G, 8, None) == L.NMF_EINVAL
    # objective and ANLS: null matrix / bad opts
    assert lib.nmf_objective(None, 4, G, G, 0, None, None, None, G, G, 1 << 20, None) == L.NMF_EINVAL
    M = L.nmf_matrix()
    M.kind, M.m, M.n, M.A, M.lda = L.NMF_DENSE, 10, 8, 16, 8
    o = L.make_opts(max_rounds=0)
    assert lib.nmf_anls_workspace_bytes(ctypes.byref(M), 4, ctypes.byref(o), ctypes.byref(nb)) == L.NMF_EINVAL
    o = L.make_opts(prec=L.NMF_BF16X3)
    assert lib.nmf_anls_workspace_bytes(ctypes.byref(M), 4, ctypes.byref(o), ctypes.byref(nb)) == L.NMF_EINVAL
    o = L.make_opts(warm=L.NMF_WARM_LEARNED)
    assert lib.nmf_anls_workspace_bytes(ctypes.byref(M), 4, ctypes.byref(o), ctypes.byref(nb)) == L.NMF_EINVAL
    o = L.make_opts(solver=L.NMF_SOLVER_HALS, warm=L.NMF_WARM_PREV)
    assert lib.nmf_anls_workspace_bytes(ctypes.byref(M), 4, ctypes.byref(o), ctypes.byref(nb)) == L.NMF_EINVAL
    o = L.make_opts(solver=7)
    assert lib.nmf_anls_workspace_bytes(ctypes.byref(M), 4, ctypes.byref(o), ctypes.byref(nb)) == L.NMF_EINVAL
    o = L.make_opts(solver=L.NMF_SOLVER_MU)
    assert lib.nmf_anls_workspace_bytes(ctypes.byref(M), 4, ctypes.byref(o), ctypes.byref(nb)) == L.NMF_OK
    o = L.make_opts()
    assert lib.nmf_anls_workspace_bytes(ctypes.byref(M), 4, ctypes.byref(o), ctypes.byref(nb)) == L.NMF_OK
    assert nb.value > 0
    # a resident A^T needs ldat >= m; it changes the FP32 form's workspace (A^T W as side W of A^T)
    M.At, M.ldat = 16, 9
    assert lib.nmf_anls_workspace_bytes(ctypes.byref(M), 4, ctypes.byref(o), ctypes.byref(nb)) == L.NMF_EINVAL
    M.ldat = 10
    nb2 = ctypes.c_size_t(0)
    assert lib.nmf_anls_workspace_bytes(ctypes.byref(M), 4, ctypes.byref(o), ctypes.byref(nb2)) == L.NMF_OK
    assert nb2.value > 0


def test_struct_layouts_match_header(L):
    # sizes of the C structs as the library sees them are fixed by the header;
    # the Python mirror must agree field for field.
    assert ctypes.sizeof(L.nmf_iter_stats) == 8 * (2 + 2 * L.NMF_BPP_COUNTERS + 2)
    assert L.nmf_matrix.fro2.offset == ctypes.sizeof(L.nmf_matrix) - 8
    assert ctypes.sizeof(L.nmf_batch_problem) == 8 * 2 + 4 * 2 + 8 * 6
    assert ctypes.sizeof(L.nmf_batch_tune) == 4 * 8


def test_batch_host_validation_without_gpu(L):
    lib = L.lib()
    G = 16  # a non-null stand-in; nothing here dereferences device pointers
    P = (L.nmf_batch_problem * 2)()
    P[0] = L.nmf_batch_problem(300, 200, 10, 0, G, G, G, 10, G, 10)
    P[1] = L.nmf_batch_problem(1000, 513, 50, 0, G, G, G, 50, G, 50)
    nb = ctypes.c_size_t(0)
    assert lib.nmf_batch_workspace_bytes(2, P, None, ctypes.byref(nb)) == L.NMF_OK
    t = L.batch_tune_default()
    nd = ctypes.c_size_t(0)
    assert lib.nmf_batch_workspace_bytes(2, P, ctypes.byref(t), ctypes.byref(nd)) == L.NMF_OK
    # the size for any tuning the autotuner tries covers the default one
    assert 0 < nd.value <= nb.value
    # the factors alone: W, Ht, their backups, Gram matrices, right-hand sides
    assert nd.value > 4 * (2 * (300 + 200) * 10 + 2 * (1000 + 513) * 50)
    assert lib.nmf_batch_workspace_bytes(0, P, None, ctypes.byref(nb)) == L.NMF_EINVAL
    bad = (L.nmf_batch_problem * 1)()
    bad[0] = L.nmf_batch_problem(300, 200, 0, 0, G, G, G, 10, G, 10)
    assert lib.nmf_batch_workspace_bytes(1, bad, None, ctypes.byref(nb)) == L.NMF_EINVAL
    bad[0] = L.nmf_batch_problem(300, 200, 10, 0, G, G, G, 4, G, 10)
    assert lib.nmf_batch_workspace_bytes(1, bad, None, ctypes.byref(nb)) == L.NMF_EINVAL
    bad[0] = L.nmf_batch_problem(300, 200, 10, 0, None, G, G, 10, G, 10)
    assert lib.nmf_batch_workspace_bytes(1, bad, None, ctypes.byref(nb)) == L.NMF_EINVAL
    t.warm_prev = 2
    assert lib.nmf_batch_workspace_bytes(2, P, ctypes.byref(t), ctypes.byref(nb)) == L.NMF_EINVAL
    t.warm_prev = 1
    t.bpp_problems = 10
    assert lib.nmf_batch_workspace_bytes(2, P, ctypes.byref(t), ctypes.byref(nb)) == L.NMF_EINVAL
    # a workspace one byte short is refused before anything reaches the device
    h = ctypes.c_void_p()
    assert lib.nmf_batch_plan_create(2, P, None, ctypes.c_void_p(G), nd.value - 1, ctypes.byref(h)) == L.NMF_EWORKSPACE
    assert h.value is None
    assert lib.nmf_batch_iterate(None, 1, None, 0, None) == L.NMF_EINVAL
    assert lib.nmf_batch_graph_create(None, 1, None, 0, None, ctypes.byref(h)) == L.NMF_EINVAL
