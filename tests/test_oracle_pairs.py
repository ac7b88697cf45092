"""Pair set and per-particle sums of the oracle.

* Pair set (Sec. III.A, pruning): all pairs with centre distance below
  R_max,i + R_max,j + max cut-off under the minimum image.  Checked against
  an independent enumeration of the 27 periodic images (ties within 1e-9
  of the bound excluded: the two computations round differently).
* Walls: centre-to-wall distance minus bounding radius below the cut-off.
* Sums: Newton's third law makes the total force vanish without walls;
  the subset evaluation reproduces the full evaluation bit for bit (same
  pairs, same orientation, same order).
"""
import itertools

import numpy as np
import pytest

from paper_1308_6482_amd import workloads as W


def images_bruteforce(r, semi, L, periodic, dmax):
    n = r.shape[0]
    rmax = semi.max(axis=1)
    shifts = [np.array(s) * np.asarray(L) for s in itertools.product(
        *[(-1, 0, 1) if periodic[k] else (0,) for k in range(3)])]
    pairs, ties = set(), set()
    for i in range(n):
        for j in range(i + 1, n):
            d = min(np.linalg.norm(r[j] - r[i] + s) for s in shifts)
            bound = rmax[i] + rmax[j] + dmax
            if abs(d - bound) < 1e-9:
                ties.add((i, j))
            elif d < bound:
                pairs.add((i, j))
    return pairs, ties


def test_pair_set_periodic(ref):
    rng = np.random.default_rng(0)
    L = (30.0, 25.0, 40.0)
    n = 150
    r = rng.uniform(0, 1, size=(n, 3)) * L
    semi = np.stack([rng.uniform(1, 6, n), rng.uniform(1, 6, n)], axis=1)
    P = ref.make_params()
    for per in [(1, 1, 1), (1, 1, 0), (0, 0, 0)]:
        dom = ref.make_domain(L=L, periodic=per)
        ij, wall = ref.candidates(r, semi, dom, P)
        assert wall.shape[0] == 0
        got = set(map(tuple, ij.tolist()))
        exp, ties = images_bruteforce(r, semi, L, per, 2 / 3)
        assert exp - got == set()
        assert got - exp <= ties
        # sorted by (i, j), i < j
        assert np.all(ij[:, 0] < ij[:, 1])
        key = ij[:, 0].astype(np.int64) * n + ij[:, 1]
        assert np.all(np.diff(key) > 0)


def test_wall_candidates(ref):
    L = (50.0, 50.0, 30.0)
    r = np.array([[1, 1, 4.5], [2, 2, 4.7], [3, 3, 25.6], [4, 4, 15.0]], float)
    semi = np.array([[4.0, 2.0]] * 4)
    P = ref.make_params(delta_n=0.67, delta_t=0.5, delta_r=0.25)
    dom = ref.make_domain(L=L, periodic=(1, 1, 0), n_walls=2)
    ij, wall = ref.candidates(r, semi, dom, P)
    assert wall.tolist() == [[0, 0], [2, 1]]


def test_centre_test_symmetric(ref):
    rng = np.random.default_rng(1)
    dom = ref.make_domain(L=(10.0, 10.0, 10.0), periodic=(1, 1, 1))
    for _ in range(2000):
        a, b = rng.uniform(-20, 20, size=(2, 3))
        ra, rb = rng.uniform(0.5, 3, size=2)
        assert ref.centre_test(a, b, ra, rb, 0.67, dom) == ref.centre_test(b, a, rb, ra, 0.67, dom)


@pytest.fixture(scope="module")
def cfg1():
    return W.config1()


def test_total_force_vanishes(ref, cfg1):
    w = cfg1
    dom = ref.make_domain(**w.domain())
    P = ref.make_params(**w.params)
    f, t, st = ref.compute(w.r, w.q, w.semi, w.v, w.w, dom, P)
    assert st["active"] > 5
    assert np.allclose(f.sum(axis=0), 0, atol=1e-12 * np.abs(f).max())


def test_subset_matches_full(ref, cfg1):
    w = cfg1
    dom = ref.make_domain(**w.domain())
    for hc, ec in ((0.0, 0.0), (0.01, 100.0)):
        P = ref.make_params(**dict(w.params, h_c=hc, eps_c=ec))
        f, t, st = ref.compute(w.r, w.q, w.semi, w.v, w.w, dom, P)
        idx = np.arange(0, w.n, 3)
        fs, ts, _ = ref.compute_subset(w.r, w.q, w.semi, w.v, w.w, dom, P, idx)
        assert np.array_equal(fs, f[idx])
        assert np.array_equal(ts, t[idx])


def test_compute_rejects_bad_inputs(ref, cfg1):
    w = cfg1
    dom = ref.make_domain(**w.domain())
    P = ref.make_params(**w.params)
    q = w.q.copy()
    q[3] *= 1.01
    with pytest.raises(ValueError):
        ref.compute(w.r, q, w.semi, w.v, w.w, dom, P)
    r = w.r.copy()
    r[0, 0] = np.nan
    with pytest.raises(ValueError):
        ref.compute(r, w.q, w.semi, w.v, w.w, dom, P)


def test_config2_statistics(ref):
    """The 4096-prolate suspension: no overlaps from the placement, and a
    plausible number of lubrication-active pairs."""
    w = W.config2()
    dom = ref.make_domain(**w.domain())
    P = ref.make_params(**w.params)
    ij, _ = ref.candidates(w.r, w.semi, dom, P)
    F, Ti, Tj, h, status = ref.eval_pairs(w.r, w.q, w.semi, w.v, w.w, dom, P, ij)
    assert np.all(status != ref.REFP_FAILED)
    assert h.min() > 0          # placement never overlaps
    active = np.sum(status == ref.REFP_ACTIVE)
    assert 0.5 * w.n < active < 4 * w.n


def test_partners_subset_equals_pair_set(ref):
    """The per-particle partner lists (used on samples of systems too large
    for the full pair set) give back the full candidate set."""
    from paper_1308_6482_amd import workloads as W
    for wl in (W.config1(), W.config3(n=600)):
        dom = ref.make_domain(**wl.domain())
        P = ref.make_params(**wl.params)
        ij, _ = ref.candidates(wl.r, wl.semi, dom, P)
        parts = ref.partners_subset(wl.r, wl.semi, dom, P, np.arange(wl.n))
        pairs = sorted({(min(k, int(j)), max(k, int(j))) for k in range(wl.n)
                        for j in parts[k]})
        assert np.array_equal(np.array(pairs, dtype=np.int32).reshape(-1, 2), ij)
