"""The oracle's placement of pairs at a prescribed gap (the learned seed's
training and held-out pairs): spheres in closed form, and the independent
construction from support points -- the support points of i along n and of
j along -n, a gap h apart along n, are the unique closest points of the two
convex bodies -- reproduced from the direction of that construction's centre
offset alone."""
import numpy as np

from paper_1308_6482_amd import seed_data as S
from paper_1308_6482_amd import workloads as W


def test_spheres_closed_form(ref):
    rng = np.random.default_rng(3)
    m = 200
    a = rng.uniform(2, 8, size=m)
    b = rng.uniform(2, 8, size=m)
    u = rng.normal(size=(m, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    g = np.exp(rng.uniform(np.log(1e-4), 0.0, size=m))
    q = W.random_quaternions(rng, m)
    out = ref.place_pairs(u, g, q, np.stack([a, a], 1), q[::-1].copy(), np.stack([b, b], 1))
    assert np.all(out["status"] == 0)
    assert np.allclose(out["s"], a + b + g, rtol=0, atol=1e-11 * 16)
    assert np.allclose(out["n"], u, atol=1e-10)
    assert np.allclose(out["yi"], a[:, None] * u, atol=1e-9)
    assert np.allclose(out["yj"], -b[:, None] * u, atol=1e-9)


def test_matches_support_point_construction(ref):
    P = S.sample_pairs(seed=17, m=2000)
    d = P["d"]
    dn = np.linalg.norm(d, axis=1)
    out = ref.place_pairs(d / dn[:, None], P["h"], P["q_i"], P["semi_i"], P["q_j"],
                          P["semi_j"])
    assert np.all(out["status"] == 0)
    R = np.maximum(P["semi_i"].max(axis=1), P["semi_j"].max(axis=1))
    assert np.max(np.abs(out["s"] - dn) / R) < 1e-9
    assert np.max(np.abs(out["h"] - P["h"]) / (1 + P["h"])) < 1e-11
    assert np.max(np.linalg.norm(out["n"] - P["n"], axis=1)) < 1e-7
    assert np.max(np.linalg.norm(out["yi"] - P["yi"], axis=1) / R) < 1e-7
    assert np.max(np.linalg.norm(out["yj"] - P["yj"], axis=1) / R) < 1e-7


def test_config4_draws(ref):
    from oracle import seed_pairs as SP
    P = SP.labelled_pairs(2, 4000)
    assert np.all(P["status"] == 0)
    assert np.max(np.abs(P["h"] - P["target"]) / P["target"]) < 1e-7
    # the label's gap direction points from i to j and the offset is s u
    assert np.all(np.sum(P["n"] * P["u"], axis=1) > 0)
    a = np.minimum(P["semi_i"].min(axis=1), P["semi_j"].min(axis=1))
    g = P["target"] / a
    assert g.min() >= 1e-4 * (1 - 1e-12) and g.max() <= 1.0
