"""HALS and MU local updates (Eq. halsupdate, Eq. muupdate) through the C-ABI
against the FP64 oracle (oracle/local.py).

Kernel parity: the same FP32 inputs on both sides; the oracle computes in
FP64 and the kernel in FP64 with one rounding to FP32, so the bar is
|x_gpu - x_oracle| <= 4 ulp32(x_oracle) + 1e-9 max|x_oracle| (the last term
covers values that the summation order moves across the clamp at 0).

Algorithm 1 with either update: |r_gpu - r_oracle| <= 1e-5 after every
half-step (FP32 factors and FP32 products on the GPU, FP64 in the oracle).
"""
import numpy as np
import pytest
import torch

from oracle import local
from nmf_inputs import configs as C
from paper_1509_09313_amd import binding as L

pytestmark = pytest.mark.gpu

SOLVERS = {"hals": L.NMF_SOLVER_HALS, "mu": L.NMF_SOLVER_MU}


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def problem(rng, k, rows, pin=None):
    C_ = rng.uniform(0.0, 1.0, (3 * k + 5, k))
    if pin is not None:
        C_[:, pin] = 0.0
    G = C_.T @ C_
    G = 0.5 * (G + G.T)                                           # exactly symmetric, like nmf_gram's
    R = (rng.uniform(0.0, 1.0, (rows, C_.shape[0])) @ C_).astype(np.float32)
    R[: rows // 3] -= np.float32(0.5) * R[: rows // 3].mean()     # some negative entries
    X = rng.uniform(0.0, 1.0, (rows, k)).astype(np.float32)
    X[rng.uniform(size=X.shape) < 0.1] = 0.0                      # zeros (MU keeps them)
    if rows > 4:
        X[3] = 0.0                                                # a zero row
    return G, R, X


def check(got, ref, label):
    ref32 = ref.astype(np.float32).astype(np.float64)
    tol = 4 * np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64) + 1e-9 * np.max(np.abs(ref))
    err = np.abs(got.astype(np.float64) - ref)
    assert np.all(err <= tol), (label, float(np.max(err / np.maximum(tol, 1e-300))))
    return float(np.mean(got.astype(np.float64) == ref32))


@pytest.mark.parametrize("solver", ["hals", "mu"])
@pytest.mark.parametrize("k,rows", [(1, 7), (5, 64), (8, 65), (13, 1000), (30, 5000), (33, 129), (64, 300)])
def test_local_update_vs_oracle(solver, k, rows):
    rng = np.random.default_rng(1000 * k + rows)
    pin = k // 2 if k > 2 else None
    G, R, X = problem(rng, k, rows, pin)
    ref = local.UPDATES[solver](G, R.astype(np.float64), X.astype(np.float64))
    Xg = cuda(X)
    L.nmf_local_update(SOLVERS[solver], cuda(G), cuda(R), Xg)
    got = Xg.cpu().numpy()
    same = check(got, ref, f"{solver} k={k} rows={rows}")
    if pin is not None:
        assert np.all(got[:, pin] == 0.0)
    if solver == "mu":
        assert np.all(got[X == 0.0] == 0.0)
    print(f"{solver} k={k} rows={rows}: {100 * same:.2f}% bitwise equal to the rounded oracle")


@pytest.mark.parametrize("solver", ["hals", "mu"])
def test_local_update_strided_and_empty(solver):
    rng = np.random.default_rng(7)
    k, rows = 20, 300
    G, R, X = problem(rng, k, rows)
    Rb = torch.full((rows, k + 3), float("nan"), dtype=torch.float32, device="cuda")
    Rb[:, :k] = cuda(R)
    Xb = torch.full((rows, k + 5), -7.0, dtype=torch.float32, device="cuda")
    Xb[:, :k] = cuda(X)
    L.nmf_local_update(SOLVERS[solver], cuda(G), Rb[:, :k], Xb[:, :k])
    ref = local.UPDATES[solver](G, R.astype(np.float64), X.astype(np.float64))
    check(Xb[:, :k].cpu().numpy(), ref, solver)
    assert torch.all(Xb[:, k:] == -7.0)
    E = torch.zeros((0, k), dtype=torch.float32, device="cuda")
    L.nmf_local_update(SOLVERS[solver], cuda(G), E, E)


@pytest.mark.parametrize("solver", ["hals", "mu"])
def test_anls_local_trajectory(solver):
    """Algorithm 1 with HALS or MU on the planted 2000 x 300 case (k = 30) and
    on config 1 (200 x 150, k = 5), 10 iterations, against the oracle."""
    for (m, n, k, seed) in ((2000, 300, 30, C.seed_for(4) + 77), (200, 150, 5, C.seed_for(1))):
        A = C.planted_dense(seed, m, n, min(k, 10), 0.01)
        W0, H0 = C.init_w(seed, m, k), C.init_ht(seed, n, k)
        T = 10
        ref = local.anls(solver, k, W0, H0, T, dense=A)
        M = L.Matrix(dense=cuda(A))
        W, Ht = cuda(W0), cuda(H0)
        run = L.Anls(M, k, L.make_opts(prec=L.NMF_F32, trace=True, solver=SOLVERS[solver]))
        st = L.new_stats(T)
        run.run(W, Ht, T, st)
        torch.cuda.synchronize()
        dec = L.decode_stats(st)
        rh = np.array([s["r_half"] for s in dec])
        rf = np.array([s["r_full"] for s in dec])
        worst = max(np.max(np.abs(rh - ref["r_half"])), np.max(np.abs(rf - ref["r_full"])))
        direct = float(L.nmf_objective(M, W, Ht)[0])
        print(f"{solver} {m}x{n} k={k}: r_10 {ref['r_full'][-1]:.8f}, max |dr| {worst:.2e}")
        assert worst <= 1e-5
        assert abs(direct - ref["r_full"][-1]) <= 1e-5
        assert all(s["bpp_w"][0] == 0 for s in dec)


@pytest.mark.parametrize("solver", ["hals", "mu"])
def test_local_update_every_k(solver):
    """Each k in 1..64 is its own compiled kernel: all of them, 131 rows (two
    full 64-row tiles and a ragged one), against the oracle."""
    for k in range(1, 65):
        rng = np.random.default_rng(5000 + k)
        G, R, X = problem(rng, k, 131, k - 1 if k > 3 else None)
        ref = local.UPDATES[solver](G, R.astype(np.float64), X.astype(np.float64))
        Xg = cuda(X)
        L.nmf_local_update(SOLVERS[solver], cuda(G), cuda(R), Xg)
        check(Xg.cpu().numpy(), ref, f"{solver} k={k}")


@pytest.mark.parametrize("solver", ["hals", "mu"])
def test_anls_local_sparse(solver):
    """Algorithm 1 with HALS or MU behind the CSR right-hand sides (2000 x
    1500 at density 0.05, k = 20, 10 iterations) against the oracle run on
    the same matrix made dense."""
    m, n, k, T, seed = 2000, 1500, 20, 10, C.seed_for(3) + 91
    rp, ci, va = C.sparse_csr(seed, m, n, 0.05)
    rpt, cit, vat = C.csr_transpose(m, n, rp, ci, va)
    W0, H0 = C.init_w(seed, m, k), C.init_ht(seed, n, k)
    ref = local.anls(solver, k, W0, H0, T, dense=C.csr_to_dense(m, n, rp, ci, va))
    M = L.Matrix(csr=(cuda(rp), cuda(ci), cuda(va)), csr_t=(cuda(rpt), cuda(cit), cuda(vat)), shape=(m, n))
    W, Ht = cuda(W0), cuda(H0)
    st = L.new_stats(T)
    L.Anls(M, k, L.make_opts(prec=L.NMF_F32, trace=True, solver=SOLVERS[solver])).run(W, Ht, T, st)
    torch.cuda.synchronize()
    dec = L.decode_stats(st)
    worst = max(np.max(np.abs(np.array([s["r_half"] for s in dec]) - ref["r_half"])),
                np.max(np.abs(np.array([s["r_full"] for s in dec]) - ref["r_full"])))
    direct = float(L.nmf_objective(M, W, Ht)[0])
    print(f"{solver} sparse {m}x{n} nnz={int(rp[-1])} k={k}: r_10 {ref['r_full'][-1]:.8f}, max |dr| {worst:.2e}")
    assert worst <= 1e-5
    assert abs(direct - ref["r_full"][-1]) <= 1e-5
