"""FP64 oracle of the learned warm start -- TEST INFRASTRUCTURE ONLY.

The paper's BPP (Section "Block Principal Pivoting") searches for the passive
set of each NNLS problem; this network predicts a starting passive set from
the problem's data.  Definition (float64, NumPy; matrix products are the only
library primitive used):

  features  phi = [ s / ||s||_2 ,  diag(G) / mean(diag(G)) ]   (length 2k)
            s_i = f_i / sqrt(G_ii), and s_i = 0 for pinned indices
            (G_ii <= 1e-14 max_l G_ll), the same pinning as the BPP oracle
  network   h1 = relu(phi W1 + b1), h2 = relu(h1 W2 + b2), z = h2 W3 + b3
  target    t_i = 1 if index i is passive in the converged BPP solution
  loss      mean over batch and outputs of BCE(sigmoid(z), t)
            = mean( log(1 + exp(z)) - t z )
  update    Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected)
  predict   F0 = { i : z_i > 0 }  (sigmoid > 1/2), minus pinned indices

Parameter vector layout (float32 on the device, float64 here):
W1[2k][h], b1[h], W2[h][h], b2[h], W3[h][k], b3[k], input-major.
"""
from __future__ import annotations

import numpy as np

HIDDEN = 128


def unpack(p, k, hidden=HIDDEN):
    p = np.asarray(p, dtype=np.float64)
    out, off = {}, 0
    for name, shape in (("W1", (2 * k, hidden)), ("b1", (hidden,)), ("W2", (hidden, hidden)),
                        ("b2", (hidden,)), ("W3", (hidden, k)), ("b3", (k,))):
        sz = int(np.prod(shape))
        out[name] = p[off:off + sz].reshape(shape)
        off += sz
    assert off == p.size, (off, p.size)
    return out


def pack(d):
    return np.concatenate([d[n].ravel() for n in ("W1", "b1", "W2", "b2", "W3", "b3")])


def features(G, R):
    """phi (batch x 2k) from the Gram matrix G (k x k) and right-hand sides R."""
    G = np.asarray(G, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    d = np.diag(G).copy()
    dmax = d.max() if d.size else 0.0
    pinned = d <= 1e-14 * dmax
    root = np.sqrt(np.where(pinned, 1.0, d))
    s = np.where(pinned[None, :], 0.0, R / root[None, :])
    nrm = np.sqrt(np.sum(s * s, axis=1, keepdims=True))
    s = np.where(nrm > 0.0, s / np.where(nrm > 0.0, nrm, 1.0), 0.0)
    mean = d.mean()
    g = d / mean if mean > 0.0 else np.zeros_like(d)
    return np.concatenate([s, np.broadcast_to(g, s.shape)], axis=1)


def forward(p, phi, k):
    P = unpack(p, k)
    a1 = phi @ P["W1"] + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"] + P["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ P["W3"] + P["b3"]
    return z, (phi, a1, h1, a2, h2)


def loss(z, t):
    z = np.asarray(z, np.float64)
    return float(np.mean(np.logaddexp(0.0, z) - t * z))


def backward(p, cache, z, t, k):
    """Gradient of `loss` with respect to the flat parameter vector."""
    P = unpack(p, k)
    phi, a1, h1, a2, h2 = cache
    B = z.shape[0]
    dz = (1.0 / (1.0 + np.exp(-z)) - t) / (B * k)
    g = {}
    g["W3"] = h2.T @ dz
    g["b3"] = dz.sum(axis=0)
    dh2 = (dz @ P["W3"].T) * (a2 > 0.0)
    g["W2"] = h1.T @ dh2
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ P["W2"].T) * (a1 > 0.0)
    g["W1"] = phi.T @ dh1
    g["b1"] = dh1.sum(axis=0)
    return pack(g)


def adam_step(p, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam update (t counts from 1). Returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def targets(masks, k):
    masks = np.asarray(masks, dtype=np.uint64)
    bits = (masks[:, None] >> np.arange(k, dtype=np.uint64)[None, :]) & np.uint64(1)
    return bits.astype(np.float64)


def predict_masks(p, phi, k, pinned: int = 0):
    z, _ = forward(p, phi, k)
    bits = (z > 0.0).astype(np.uint64)
    m = np.sum(bits << np.arange(k, dtype=np.uint64)[None, :], axis=1, dtype=np.uint64)
    return m & ~np.uint64(pinned), z
