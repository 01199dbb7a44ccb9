"""Pins of the warm-start network oracle: the backward pass against central
finite differences of the loss, closed forms of the forward pass and of the
first Adam step, and the feature map's invariants.  CPU only."""
import numpy as np

from oracle import mlp
from nmf_inputs import configs as C


def small_problem(k=6, batch=9, seed=0):
    rng = np.random.default_rng(seed)
    p = C.mlp_init(k, 1234).astype(np.float64)
    p += 0.05 * rng.standard_normal(p.size)        # nonzero biases too
    phi = rng.standard_normal((batch, 2 * k))
    t = (rng.uniform(size=(batch, k)) < 0.6).astype(np.float64)
    return p, phi, t


def test_backward_matches_finite_differences():
    k = 6
    p, phi, t = small_problem(k)
    z, cache = mlp.forward(p, phi, k)
    g = mlp.backward(p, cache, z, t, k)
    rng = np.random.default_rng(1)
    idx = rng.choice(p.size, 200, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        lp = mlp.loss(mlp.forward(p + e, phi, k)[0], t)
        lm = mlp.loss(mlp.forward(p - e, phi, k)[0], t)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (i, fd, g[i])


def test_forward_closed_forms():
    k = 5
    P = {n: np.zeros(s) for n, s in (("W1", (2 * k, 128)), ("b1", (128,)), ("W2", (128, 128)),
                                     ("b2", (128,)), ("W3", (128, k)), ("b3", (k,)))}
    P["b3"] = np.arange(k, dtype=np.float64) - 2.0
    z, _ = mlp.forward(mlp.pack(P), np.ones((3, 2 * k)), k)
    assert np.array_equal(z, np.tile(P["b3"], (3, 1)))
    assert abs(mlp.loss(np.zeros((4, k)), np.ones((4, k))) - np.log(2.0)) < 1e-15
    # one hidden unit passes x_0 through both ReLUs
    P["b3"][:] = 0.0
    P["W1"][0, 0] = 1.0
    P["W2"][0, 0] = 1.0
    P["W3"][0, :] = 2.0
    phi = np.zeros((2, 2 * k))
    phi[:, 0] = [3.0, -3.0]
    z, _ = mlp.forward(mlp.pack(P), phi, k)
    assert np.array_equal(z[0], np.full(k, 6.0)) and np.array_equal(z[1], np.zeros(k))


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(2)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m, v = mlp.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    np.testing.assert_allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_features_invariants():
    rng = np.random.default_rng(3)
    k = 7
    X = rng.uniform(size=(30, k))
    X[:, 4] = 0.0
    G = X.T @ X
    R = rng.standard_normal((11, k))
    phi = mlp.features(G, R)
    assert phi.shape == (11, 2 * k)
    np.testing.assert_allclose(np.linalg.norm(phi[:, :k], axis=1), 1.0, rtol=1e-14)
    assert np.all(phi[:, 4] == 0.0)
    d = np.diag(G)
    np.testing.assert_allclose(phi[0, k:], d / d.mean(), rtol=1e-15)
    # invariant to scaling the problem (C -> cC, b -> cb)
    np.testing.assert_allclose(mlp.features(4.0 * G, 2.0 * R), phi, rtol=1e-12, atol=1e-15)


def test_features_closed_form():
    """Hand-worked feature vectors (Section "Block Principal Pivoting": the
    network's input is the problem's right-hand side scaled by the square
    roots of the Gram diagonal, then normalised, beside the diagonal over its
    mean).  The Gram matrices are not diagonal and their diagonals are
    distinct perfect squares, so s_i = f_i / sqrt(G_ii) is a small integer and
    the unscaled f_i, f_i / G_ii and f_i * sqrt(G_ii) all give other
    directions after the normalisation."""
    G = np.array([[4.0, 2.0, 0.0], [2.0, 9.0, 3.0], [0.0, 3.0, 16.0]])
    R = np.array([[2.0, -6.0, 8.0],     # s = (1, -2, 2), ||s|| = 3
                  [0.0, 0.0, 0.0],      # zero right-hand side: s = 0
                  [-4.0, 3.0, 0.0]])    # s = (-2, 1, 0), ||s|| = sqrt(5)
    phi = mlp.features(G, R)
    g = np.array([12.0, 27.0, 48.0]) / 29.0            # (4, 9, 16) / (29 / 3)
    r5 = np.sqrt(5.0)
    want = np.array([[1 / 3, -2 / 3, 2 / 3, *g],
                     [0.0, 0.0, 0.0, *g],
                     [-2 / r5, 1 / r5, 0.0, *g]])
    np.testing.assert_allclose(phi, want, rtol=1e-15, atol=1e-16)
    # the closed form tells the candidate scalings apart
    for d_pow in (0.0, 1.0, -0.5):
        alt = R[0] / np.diag(G) ** d_pow
        alt = alt / np.linalg.norm(alt)
        assert np.max(np.abs(alt - want[0, :3])) > 0.05, d_pow

    # a pinned index (G_ii <= 1e-14 max G_ll) has s_i = 0; the diagonal part
    # keeps its zero and the mean counts it
    G2 = np.array([[25.0, 0.0, 5.0], [0.0, 0.0, 0.0], [5.0, 0.0, 1.0]])
    R2 = np.array([[10.0, 7.0, -1.0]])                   # s = (2, 0, -1)
    phi2 = mlp.features(G2, R2)
    want2 = np.array([[2 / r5, 0.0, -1 / r5, 75 / 26, 0.0, 3 / 26]])
    np.testing.assert_allclose(phi2, want2, rtol=1e-15, atol=1e-16)


def test_targets_and_predict_roundtrip():
    k = 6
    masks = np.array([0, 1, 0b101101, 63], dtype=np.uint64)
    t = mlp.targets(masks, k)
    assert t.shape == (4, k) and t[2].tolist() == [1, 0, 1, 1, 0, 1]
    P = {n: np.zeros(s) for n, s in (("W1", (2 * k, 128)), ("b1", (128,)), ("W2", (128, 128)),
                                     ("b2", (128,)), ("W3", (128, k)), ("b3", (k,)))}
    P["b3"] = np.array([1.0, -1.0, 1.0, -1.0, 1.0, -1.0])
    m, z = mlp.predict_masks(mlp.pack(P), np.zeros((2, 2 * k)), k, pinned=0b10000)
    assert int(m[0]) == 0b000101
