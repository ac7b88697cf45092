"""Pins of the oracle's link-wise lubrication laws (Sec. II.D, Eq.
methods:dlub; Clausen's averaged-normal variant).

* One link through a fluid site: two spheres of radius 0.5 whose only sites
  are (0,0,0) and (2,0,0); the single pair of links has h* = 0.8, lambda* =
  1/R, and the force of Eq. methods:dlub in closed form.
* One direct link, gap below the clipping gap: the clipped lubrication term
  plus the link-wise repulsion in closed form.
* An independent enumeration for spheroid pairs: links counted from the
  sites of j outward (the reverse of the oracle's direction), gaps by
  bisection along the link; same link count and smallest gap.
* Pair swap: evaluating (j, i) finds the same undirected links and gives
  the opposite force.
* Galilean invariance (common velocity: no force) and a rigid rotation of
  the pair as one body (no force in the link-direction law, whose force
  follows the link).
* Lattice translation: shifting both particles by a lattice vector changes
  nothing.
"""
import itertools

import numpy as np
import pytest

import oracle as O


def P(model=O.MODEL_LINK, h_c=0.0, eps_c=0.0, mu=1.0 / 6.0, q_bar=0.6):
    return O.make_params(mu=mu, h_c=h_c, eps_c=eps_c, model=model, q_bar=q_bar)


QI = np.array([1.0, 0.0, 0.0, 0.0])


def test_single_link_through_fluid_site(ref):
    ri = np.array([0.1, 0.0, 0.0])
    rj = np.array([1.9, 0.0, 0.0])
    vi, vj = np.array([0.3, 0.1, -0.2]), np.array([-0.4, 0.05, 0.1])
    wi, wj = np.array([0.0, 0.2, 0.3]), np.array([0.1, -0.1, 0.0])
    mu, qb = 1.0 / 6.0, 0.6
    o = ref.link_eval(ri, rj - ri, QI, [0.5, 0.5], vi, wi, QI, [0.5, 0.5], vj, wj, P())
    assert o["links"] == 1 and o["status"] == ref.REFP_ACTIVE
    assert abs(o["h"] - 0.8) < 1e-14
    u = np.array([-1.0, 0.0, 0.0])            # from j's side to i
    pi, pj = np.array([0.6, 0, 0]), np.array([1.4, 0, 0])
    Vi = vi + np.cross(wi, pi - ri)
    Vj = vj + np.cross(wj, pj - rj)
    lam = 2.0                                  # mean of the two curvatures 1/R
    f = -3 * qb * mu / (2 * 1.0 * lam) * (u @ (Vi - Vj)) * (1 / 0.8 ** 2 - 1.0)
    assert np.allclose(o["F"], f * u, rtol=1e-13, atol=1e-15)
    assert np.allclose(o["Ti"], np.cross(pi - ri, f * u), atol=1e-15)
    assert np.allclose(o["Tj"], np.cross(pj - rj, -f * u), atol=1e-15)


def test_single_direct_link_clipped(ref):
    ri = np.array([0.1, 0.0, 0.0])
    rj = np.array([1.15, 0.0, 0.0])
    vi, vj = np.array([0.2, 0.0, 0.0]), np.array([-0.1, 0.0, 0.0])
    z = np.zeros(3)
    hc, ec = 0.1, 10.0
    o = ref.link_eval(ri, rj - ri, QI, [0.5, 0.5], vi, z, QI, [0.5, 0.5], vj, z,
                      P(h_c=hc, eps_c=ec))
    assert o["links"] == 1
    hs = 0.65 - 0.6
    assert abs(o["h"] - hs) < 1e-14
    u = np.array([-1.0, 0.0, 0.0])
    lub = -3 * 0.6 / 6.0 / (2 * 2.0) * (u @ (vi - vj)) * (1 / hc ** 2 - 1.0)
    rep = ec * (hc - hs)
    assert np.allclose(o["F"], (lub + rep) * u, rtol=1e-12)
    # the Clausen variant along the averaged normal: here the same direction
    o2 = ref.link_eval(ri, rj - ri, QI, [0.5, 0.5], vi, z, QI, [0.5, 0.5], vj, z,
                       P(O.MODEL_LINK_NAVG, h_c=hc, eps_c=ec))
    assert np.allclose(o2["F"], o["F"], rtol=1e-12)


def unit(x):
    return x / np.linalg.norm(x)


def quat_matrix(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def inside(c, Q, semi, x):
    xb = Q.T @ (x - c)
    return (xb[0] / semi[1]) ** 2 + (xb[1] / semi[1]) ** 2 + (xb[2] / semi[0]) ** 2 <= 1.0


def dirs():
    return [np.array(c, dtype=float) for c in itertools.product((-1, 0, 1), repeat=3)
            if 0 < sum(abs(k) for k in c) <= 2]


def enumerate_from_j(ri, qi, si, rj, qj, sj):
    """(count, smallest gap) of the links with h* < |c|, found from the
    sites of j, gaps by bisection on the implicit functions."""
    Qi, Qj = quat_matrix(qi), quat_matrix(qj)
    e = np.sqrt(np.diag(Qj @ np.diag([sj[1] ** 2, sj[1] ** 2, sj[0] ** 2]) @ Qj.T))
    lo, hi = np.floor(rj - e).astype(int), np.ceil(rj + e).astype(int)
    ins_i = lambda x: inside(ri, Qi, si, x)  # noqa: E731
    ins_j = lambda x: inside(rj, Qj, sj, x)  # noqa: E731

    def cross(f_in, a, b):
        # a inside, b outside (or the reverse): bisection on the segment
        lo_, hi_ = 0.0, 1.0
        ina = f_in(a)
        for _ in range(80):
            m = 0.5 * (lo_ + hi_)
            if f_in(a + m * (b - a)) == ina:
                lo_ = m
            else:
                hi_ = m
        return a + 0.5 * (lo_ + hi_) * (b - a)

    count, hmin, border = 0, np.inf, 0
    for xs in itertools.product(*(range(a, b + 1) for a, b in zip(lo, hi))):
        xs = np.array(xs, dtype=float)
        if not ins_j(xs) or ins_i(xs):
            continue
        for c in dirs():
            x1 = xs + c
            if ins_j(x1):
                continue
            if ins_i(x1):
                xb = x1
            else:
                xb = xs + 2 * c
                if not ins_i(xb) or ins_j(xb):
                    continue
            pj = cross(ins_j, xs, xb)
            pi = cross(ins_i, xb, xs)
            hs = np.dot(pi - pj, c) / np.linalg.norm(c)
            cl = np.linalg.norm(c)
            if abs(hs - cl) < 1e-9:
                border += 1
            if hs < cl:
                count += 1
                hmin = min(hmin, hs)
    return count, hmin, border


@pytest.fixture(scope="module")
def spheroid_pairs():
    """Spheroid pairs near contact at random lattice offsets."""
    rng = np.random.default_rng(31)
    pairs = []
    while len(pairs) < 12:
        si = np.array([rng.uniform(2, 6), rng.uniform(1.5, 4)])
        sj = np.array([rng.uniform(2, 6), rng.uniform(1.5, 4)])
        qi, qj = unit(rng.normal(size=4)), unit(rng.normal(size=4))
        u = unit(rng.normal(size=3))
        h = rng.uniform(0.05, 1.2)
        lo_, hi_ = 0.0, 30.0
        for _ in range(60):
            m = 0.5 * (lo_ + hi_)
            o = O.closest_points(m * u, qi, si, qj, sj)
            lo_, hi_ = (m, hi_) if o["h"] < h else (lo_, m)
        ri = rng.uniform(20, 21, size=3)
        pairs.append((ri, hi_ * u, qi, si, qj, sj))
    return pairs


def test_links_by_enumeration_from_j(ref, spheroid_pairs):
    z = np.zeros(3)
    total = 0
    for ri, d, qi, si, qj, sj in spheroid_pairs:
        o = ref.link_eval(ri, d, qi, si, z, z, qj, sj, z, z, P())
        cnt, hmin, border = enumerate_from_j(ri, qi, si, ri + d, qj, sj)
        assert border == 0
        assert o["links"] == cnt
        if cnt:
            assert abs(o["h"] - hmin) < 1e-9
        total += cnt
    assert total > 30


@pytest.mark.parametrize("model", [O.MODEL_LINK, O.MODEL_LINK_NAVG])
def test_swap_antisymmetry(ref, spheroid_pairs, model):
    rng = np.random.default_rng(32)
    for ri, d, qi, si, qj, sj in spheroid_pairs:
        vi, wi, vj, wj = (rng.normal(size=3) for _ in range(4))
        prm = P(model, h_c=0.02, eps_c=5.0)
        a = ref.link_eval(ri, d, qi, si, vi, wi, qj, sj, vj, wj, prm)
        b = ref.link_eval(ri + d, -d, qj, sj, vj, wj, qi, si, vi, wi, prm)
        assert a["links"] == b["links"]
        sc = np.linalg.norm(a["F"]) + 1e-300
        assert np.allclose(b["F"], -np.array(a["F"]), rtol=0, atol=1e-11 * sc)
        assert np.allclose(b["Ti"], a["Tj"], rtol=0, atol=1e-10 * sc * 8)


def test_galilean_and_rigid_rotation(ref, spheroid_pairs):
    rng = np.random.default_rng(33)
    checked = 0
    for ri, d, qi, si, qj, sj in spheroid_pairs:
        V = rng.normal(size=3)
        Om = rng.normal(size=3)
        rj = ri + d
        # common translation
        a = ref.link_eval(ri, d, qi, si, V, np.zeros(3), qj, sj, V, np.zeros(3), P())
        assert np.allclose(a["F"], 0, atol=1e-12)
        # rigid rotation of the pair about the origin: v = Om x r, w = Om
        a = ref.link_eval(ri, d, qi, si, np.cross(Om, ri), Om, qj, sj, np.cross(Om, rj), Om,
                          P())
        lin = ref.link_eval(ri, d, qi, si, np.cross(Om, ri), np.zeros(3), qj, sj,
                            np.zeros(3), np.zeros(3), P())
        if a["links"]:
            sc = np.linalg.norm(lin["F"]) + 1e-12
            assert np.linalg.norm(a["F"]) < 1e-10 * sc
            checked += 1
    assert checked > 5


def test_lattice_translation(ref, spheroid_pairs):
    rng = np.random.default_rng(34)
    for ri, d, qi, si, qj, sj in spheroid_pairs[:6]:
        vi, wi, vj, wj = (rng.normal(size=3) for _ in range(4))
        a = ref.link_eval(ri, d, qi, si, vi, wi, qj, sj, vj, wj, P())
        b = ref.link_eval(ri + np.array([7.0, -3.0, 12.0]), d, qi, si, vi, wi, qj, sj, vj,
                          wj, P())
        assert a["links"] == b["links"]
        sc = np.linalg.norm(a["F"]) + 1e-300
        assert np.allclose(a["F"], b["F"], rtol=0, atol=1e-10 * sc)
