"""FP64 reference of the learned Newton seed network (test infrastructure
only; see oracle/__init__.py).

Network: 10 -> 128 -> 128 -> 128 -> 4, SiLU after the three hidden layers.
Loss (per batch of m pairs): the mean over pairs of the squared distance
between the surface points given by the predicted (p, q) of each particle
(Eq. lub:spheroid, in the canonical pair frames, lengths in units of
R_perp,i) and the target closest points:
    L = 1/m sum_k |y_i(p_i,q_i) - t_i|^2 + |y_j(p_j,q_j) - t_j|^2.
Plain numpy, written out layer by layer; the backward pass is the chain
rule by hand and is checked against central finite differences in the
tests.

Parameter layout (flat float vector, the order the GPU library uses):
W1 (10 x 128, row-major, input-major), b1 (128), W2 (128 x 128), b2,
W3 (128 x 128), b3, W4 (128 x 4), b4 (4): 34,948 values.
"""
from __future__ import annotations

import numpy as np

SIZES = [(10, 128), (128, 128), (128, 128), (128, 4)]
N_PARAMS = sum(a * b + b for a, b in SIZES)


def unpack(theta):
    out = []
    o = 0
    for a, b in SIZES:
        W = theta[o:o + a * b].reshape(a, b)
        o += a * b
        bb = theta[o:o + b]
        o += b
        out.append((W, bb))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, X):
    """Outputs (m,4) and the cache of pre-activations for backward."""
    layers = unpack(np.asarray(theta, dtype=np.float64))
    a = np.asarray(X, dtype=np.float64)
    cache = [a]
    for k, (W, b) in enumerate(layers):
        z = a @ W + b
        if k < 3:
            cache.append(z)
            a = silu(z)
            cache.append(a)
        else:
            a = z
    return a, cache


def surface(p, q, rpar, rperp):
    return np.stack([rperp * np.cos(p) * np.cos(q), rperp * np.cos(p) * np.sin(q),
                     rpar * np.sin(p)], axis=1)


def loss_and_dy(Y, X, T):
    """Loss and dL/dY.  Semi-axes in units of R_perp,i come from the
    features: particle i (X[:,7], 1), particle j (X[:,8], X[:,9])."""
    m = Y.shape[0]
    L = 0.0
    dY = np.zeros_like(Y)
    for part, (rpa, rpe) in enumerate(((X[:, 7], np.ones(m)), (X[:, 8], X[:, 9]))):
        p, q = Y[:, 2 * part], Y[:, 2 * part + 1]
        y = surface(p, q, rpa, rpe)
        r = y - T[:, 3 * part:3 * part + 3]
        L += np.sum(r * r)
        dp = np.stack([-rpe * np.sin(p) * np.cos(q), -rpe * np.sin(p) * np.sin(q),
                       rpa * np.cos(p)], axis=1)
        dq = np.stack([-rpe * np.cos(p) * np.sin(q), rpe * np.cos(p) * np.cos(q),
                       np.zeros(m)], axis=1)
        dY[:, 2 * part] = 2.0 * np.sum(r * dp, axis=1) / m
        dY[:, 2 * part + 1] = 2.0 * np.sum(r * dq, axis=1) / m
    return L / m, dY


def loss(theta, X, T):
    Y, _ = forward(theta, X)
    return loss_and_dy(Y, X, T)[0]


def grad(theta, X, T):
    """Loss and its gradient with respect to the flat parameters."""
    layers = unpack(np.asarray(theta, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    Y, cache = forward(theta, X)
    L, dY = loss_and_dy(Y, X, T)
    grads = [None] * 4
    delta = dY
    # cache: [x, z1, a1, z2, a2, z3, a3]
    acts = [cache[0], cache[2], cache[4], cache[6]]
    zs = [cache[1], cache[3], cache[5]]
    for k in range(3, -1, -1):
        W, _ = layers[k]
        grads[k] = (acts[k].T @ delta, delta.sum(axis=0))
        if k > 0:
            delta = (delta @ W.T) * dsilu(zs[k - 1])
    return L, pack(grads)


def init(seed: int = 0):
    """He-style uniform initialisation (the GPU library draws its own with
    the same law; tests compare on explicitly passed weights)."""
    rng = np.random.default_rng(seed)
    layers = []
    for a, b in SIZES:
        lim = np.sqrt(6.0 / a)
        layers.append((rng.uniform(-lim, lim, size=(a, b)), np.zeros(b)))
    return pack(layers)
