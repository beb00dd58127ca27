"""The selector network: a multilayer perceptron 16 -> 64 -> 64 -> K with
ReLU, trained with soft targets built from measured kernel times.  Plain
float64 NumPy definitions (forward, loss, analytic backward, Adam).

Inputs are standardised features x = (f - mu) / sigma.  With
h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), z = W3 h2 + b3, classes that do
not apply to a sample (mask false) get probability 0:
    p_c = exp(z_c) / sum_{valid k} exp(z_k).
Soft targets from times t_c (valid classes): q_c proportional to
exp(-(t_c / t_min - 1) / tau), so near-optimal configurations share the
target mass.  Loss: mean over samples of -sum_c q_c log p_c.
Adam (Kingma and Ba): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""

from __future__ import annotations

import numpy as np

NFEAT, H1, H2 = 16, 64, 64

SHAPES = (("W1", (H1, NFEAT)), ("b1", (H1,)), ("W2", (H2, H1)), ("b2", (H2,)))


def shapes(nclass):
    return SHAPES + (("W3", (nclass, H2)), ("b3", (nclass,)))


def unpack(flat, nclass):
    """Split a flat parameter vector (W1, b1, W2, b2, W3, b3, mu, sigma)."""
    out, k = {}, 0
    for name, shp in shapes(nclass):
        size = int(np.prod(shp))
        out[name] = np.asarray(flat[k:k + size], dtype=np.float64).reshape(shp)
        k += size
    out["mu"] = np.asarray(flat[k:k + NFEAT], dtype=np.float64)
    out["sigma"] = np.asarray(flat[k + NFEAT:k + 2 * NFEAT], dtype=np.float64)
    return out


def nparams(nclass):
    return sum(int(np.prod(s)) for _, s in shapes(nclass)) + 2 * NFEAT


def forward(P, F, mask):
    X = (np.asarray(F, dtype=np.float64) - P["mu"]) / P["sigma"]
    A1 = X @ P["W1"].T + P["b1"]
    Hh1 = np.maximum(A1, 0.0)
    A2 = Hh1 @ P["W2"].T + P["b2"]
    Hh2 = np.maximum(A2, 0.0)
    Z = Hh2 @ P["W3"].T + P["b3"]
    Zm = np.where(mask, Z, -np.inf)
    Zm = Zm - Zm.max(axis=1, keepdims=True)
    E = np.where(mask, np.exp(Zm), 0.0)
    Pr = E / E.sum(axis=1, keepdims=True)
    return {"X": X, "H1": Hh1, "H2": Hh2, "Z": Z, "P": Pr}


def soft_targets(times, tau):
    """times: (B, K) with +inf for classes that do not apply."""
    t = np.asarray(times, dtype=np.float64)
    valid = np.isfinite(t)
    tmin = np.where(valid, t, np.inf).min(axis=1, keepdims=True)
    w = np.where(valid, np.exp(-(t / tmin - 1.0) / tau), 0.0)
    return w / w.sum(axis=1, keepdims=True), valid


def loss(P, F, mask, Q):
    cache = forward(P, F, mask)
    logp = np.log(np.where(mask, cache["P"], 1.0))
    return float(-(Q * logp).sum() / F.shape[0]), cache


def backward(P, F, mask, Q):
    """Gradients of loss with respect to W1, b1, W2, b2, W3, b3."""
    B = F.shape[0]
    L, c = loss(P, F, mask, Q)
    dZ = np.where(mask, c["P"] - Q, 0.0) / B
    g = {"W3": dZ.T @ c["H2"], "b3": dZ.sum(axis=0)}
    dH2 = (dZ @ P["W3"]) * (c["H2"] > 0)
    g["W2"] = dH2.T @ c["H1"]
    g["b2"] = dH2.sum(axis=0)
    dH1 = (dH2 @ P["W2"]) * (c["H1"] > 0)
    g["W1"] = dH1.T @ c["X"]
    g["b1"] = dH1.sum(axis=0)
    return L, g


def adam(P, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on the trained tensors (in place); t counts from 1."""
    for k in g:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)


def select(P, F, mask):
    """Index of the most probable valid class (lowest index on ties)."""
    c = forward(P, F, mask)
    Z = np.where(mask, c["Z"], -np.inf)
    return np.argmax(Z, axis=1)
