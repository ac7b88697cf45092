"""CPU pins of the learned-seed ingredients.

* Constructed training pairs: their closest points and gaps are the
  oracle's (the labels are what the oracle computes).
* Canonical features: invariant under a global rotation, under flipping
  either symmetry axis and under rotating either particle about its axis.
* FP64 reference network: backward pass against central finite
  differences; the loss vanishes at the targets' own parameters.
"""
import numpy as np
import pytest

from paper_1308_6482_amd import seed_data as S


def test_constructed_labels_match_oracle(ref):
    P = S.sample_pairs(seed=5, m=300)
    for k in range(300):
        o = ref.closest_points(P["d"][k], P["q_i"][k], P["semi_i"][k], P["q_j"][k],
                               P["semi_j"][k])
        assert o["status"] == 0
        scale = P["semi_i"][k].max() + P["semi_j"][k].max()
        assert abs(o["h"] - P["h"][k]) < 1e-10 * scale
        assert np.allclose(o["n"], P["n"][k], atol=1e-7)
        assert np.allclose(o["yi"], P["yi"][k], atol=1e-6 * scale)
        assert np.allclose(o["yj"], P["yj"][k], atol=1e-6 * scale)


def rot(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    from paper_1308_6482_amd.workloads import quat_matrix
    return quat_matrix(q[None])[0]


def test_features_invariant():
    rng = np.random.default_rng(1)
    P = S.sample_pairs(seed=6, m=200)
    X0, Fi, Fj = S.features(P["d"], P["axis_i"], P["semi_i"], P["axis_j"], P["semi_j"])
    R = rot(rng)
    X1, _, _ = S.features(P["d"] @ R.T, P["axis_i"] @ R.T, P["semi_i"],
                          P["axis_j"] @ R.T, P["semi_j"])
    assert np.allclose(X0, X1, atol=1e-9)
    X2, _, _ = S.features(P["d"], -P["axis_i"], P["semi_i"], -P["axis_j"], P["semi_j"])
    assert np.allclose(X0, X2, atol=1e-12)
    assert np.allclose(X0[:, 1], 0, atol=1e-12) and np.all(X0[:, 2] >= 0)
    assert np.allclose(np.linalg.norm(X0[:, 3:7], axis=1), 1, atol=1e-12)
    # the targets are surface points of each particle
    T = P["T"].astype(np.float64)
    rp = P["semi_i"][:, 1]
    for part, semi in ((0, P["semi_i"]), (1, P["semi_j"])):
        y = T[:, 3 * part:3 * part + 3] * rp[:, None]
        f = (y[:, 0] ** 2 + y[:, 1] ** 2) / semi[:, 1] ** 2 + y[:, 2] ** 2 / semi[:, 0] ** 2
        assert np.allclose(f, 1, atol=1e-5)


def test_seed_normal_from_exact_parameters():
    P = S.sample_pairs(seed=7, m=100)
    X, Fi, Fj = S.features(P["d"], P["axis_i"], P["semi_i"], P["axis_j"], P["semi_j"])
    rp = P["semi_i"][:, 1][:, None]
    Y = np.zeros((100, 4))
    for part, semi in ((0, P["semi_i"]), (1, P["semi_j"])):
        y = P["T"][:, 3 * part:3 * part + 3].astype(np.float64) * rp
        Y[:, 2 * part] = np.arcsin(np.clip(y[:, 2] / semi[:, 0], -1, 1))
        Y[:, 2 * part + 1] = np.arctan2(y[:, 1], y[:, 0])
    n = S.seed_normal(Y, P["semi_i"], P["semi_j"], Fi, Fj)
    assert np.allclose(n, P["n"], atol=1e-4)


def test_reference_gradient_finite_differences():
    from oracle import mlp_ref as M
    rng = np.random.default_rng(3)
    P = S.sample_pairs(seed=8, m=16)
    theta = M.init(seed=2) * 0.5 + rng.normal(size=M.N_PARAMS) * 0.01
    X, T = P["X"].astype(np.float64), P["T"].astype(np.float64)
    L, g = M.grad(theta, X, T)
    idx = rng.choice(M.N_PARAMS, size=60, replace=False)
    # include biases and the last layer explicitly
    idx = np.concatenate([idx, [1280, 1280 + 127, M.N_PARAMS - 1, M.N_PARAMS - 5]])
    for k in idx:
        e = np.zeros(M.N_PARAMS)
        eps = 1e-6 * max(1.0, abs(theta[k]))
        e[k] = eps
        fd = (M.loss(theta + e, X, T) - M.loss(theta - e, X, T)) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (k, fd, g[k])


def test_reference_loss_zero_at_targets():
    from oracle import mlp_ref as M
    P = S.sample_pairs(seed=9, m=50)
    X, T = P["X"].astype(np.float64), P["T"].astype(np.float64)
    rp = np.ones(50)
    Y = np.zeros((50, 4))
    for part, (rpa, rpe) in enumerate(((X[:, 7], rp), (X[:, 8], X[:, 9]))):
        y = T[:, 3 * part:3 * part + 3]
        Y[:, 2 * part] = np.arcsin(np.clip(y[:, 2] / rpa, -1, 1))
        Y[:, 2 * part + 1] = np.arctan2(y[:, 1], y[:, 0])
    L, dY = M.loss_and_dy(Y, X, T)
    assert L < 1e-10
