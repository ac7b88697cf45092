"""Pins of the oracle against closed forms that do not come from the
paper's appendix formulas.

* Sphere gap (Sec. III.A): h = |d| - a - b along d.
* Ladd's normal law for equal spheres (Eq. methods:llub), exact.
* Two unequal spheres: the classical leading resistance terms of Stokes flow
  (Jeffrey & Onishi 1984; O'Neill & Majumdar), whose h^-1 and ln h
  coefficients the spheroid formulas must reduce to for spheres (the paper
  states the equivalence with Nguyen-Ladd's sphere corrections, Sec. IV.A).
* Sphere-wall (b -> infinity): Goldman, Cox & Brenner's leading terms
  6 pi a^2/h, (16/5) pi a, (4/5) pi a^2, (16/5) pi a^3 (6 pi 8/15, 8 pi 1/10,
  6 pi 2/15, 8 pi 2/5 in their normalisation).
* Contact model, Eqs. lub:frep and lub:model.
"""
import numpy as np
import pytest

def unit(v):
    return v / np.linalg.norm(v)


def rand_unit(rng):
    return unit(rng.normal(size=3))


def rand_quat(rng):
    return unit(rng.normal(size=4))


def frame(e3, rng):
    t = rng.normal(size=3)
    e1 = unit(t - t.dot(e3) * e3)
    e2 = np.cross(e3, e1)
    return e1, e2


@pytest.mark.parametrize("a,b", [(4.0, 4.0), (2.0, 5.0), (8.0, 3.0)])
def test_sphere_gap_closed_form(ref, a, b):
    rng = np.random.default_rng(7)
    for h in (1e-4, 0.03, 0.4, -0.05):
        e3 = rand_unit(rng)
        d = (a + b + h) * e3
        o = ref.closest_points(d, rand_quat(rng), [a, a], rand_quat(rng), [b, b])
        assert o["status"] == 0
        assert abs(o["h"] - h) < 1e-12 * (a + b)
        assert np.allclose(o["n"], e3, atol=1e-13)
        assert np.allclose(o["yi"], a * e3, atol=1e-12 * a)
        assert np.allclose(o["yj"], -b * e3, atol=1e-12 * b)


def test_ladd_equal_spheres(ref):
    """Eq. methods:llub: f = -(3 pi mu R^2/2) rr.(v_i - v_j)(1/h - 1/Dc)."""
    rng = np.random.default_rng(3)
    R, mu, Dn = 4.0, 1.0 / 6.0, 2.0 / 3.0
    for h in (1e-3, 0.1, 0.5):
        e3 = rand_unit(rng)
        d = (2 * R + h) * e3
        vi, vj = rng.normal(size=3), rng.normal(size=3)
        P = ref.make_params(mu=mu, delta_n=Dn, delta_t=0.5, delta_r=0.25)
        # only the normal element contributes when h >= delta_t
        P.delta_t = 1e-9
        P.delta_r = 1e-9
        o = ref.pair_eval(d, rand_quat(rng), [R, R], vi, [0, 0, 0],
                          rand_quat(rng), [R, R], vj, [0, 0, 0], P)
        rhat = -e3  # r_ij = r_i - r_j
        f = -(3 * np.pi * mu * R * R / 2) * rhat * rhat.dot(vi - vj) * (1 / h - 1 / Dn)
        assert np.allclose(o["F"], f, rtol=1e-12, atol=1e-14)


def classical(a, b):
    """Leading coefficients for sphere i (radius a) near sphere j (b):
    normal 1/h, and the ln-terms for tangential translation, the couplings
    and rotation (Jeffrey & Onishi 1984)."""
    s = a + b
    return dict(
        normal=6 * np.pi * a * a * b * b / s ** 2,
        trans=8 / 5 * np.pi * a * b * (2 * a * a + a * b + 2 * b * b) / s ** 3,
        couple=4 / 5 * np.pi * a * a * b * (4 * a + b) / s ** 2,
        rot=16 / 5 * np.pi * a ** 3 * b / s,
    )


@pytest.mark.parametrize("a,b", [(4.0, 4.0), (2.0, 5.0), (8.0, 3.0), (3.0, 300.0)])
def test_two_sphere_leading_terms(ref, a, b):
    rng = np.random.default_rng(11)
    c = classical(a, b)
    mu, delta = 0.7, 0.5
    z = np.zeros(3)
    for h in (1e-4, 1e-2, 0.2):
        Lg = np.log(h / delta)
        e3 = rand_unit(rng)
        e1, e2 = frame(e3, rng)
        d = (a + b + h) * e3
        P = ref.make_params(mu=mu, delta_n=delta, delta_t=delta, delta_r=delta)
        qi, qj = rand_quat(rng), rand_quat(rng)
        # 1) normal translation of i towards j
        o = ref.pair_eval(d, qi, [a, a], 1.3 * e3, z, qj, [b, b], z, z, P)
        assert np.allclose(o["F"], -mu * c["normal"] * (1 / h - 1 / delta) * 1.3 * e3,
                           rtol=1e-9, atol=1e-12)
        assert np.allclose(o["Ti"], 0, atol=1e-9 * abs(o["F"]).max() * a)
        # 2) tangential translation of i: drag and rolling torque
        U = 0.9
        o = ref.pair_eval(d, qi, [a, a], U * e1, z, qj, [b, b], z, z, P)
        assert np.allclose(o["F"], mu * c["trans"] * Lg * U * e1, rtol=1e-9, atol=1e-12)
        assert np.allclose(o["Ti"], mu * c["couple"] * Lg * U * np.cross(e3, e1),
                           rtol=1e-9, atol=1e-12 * a)
        # drag acts at the contact point: the torque about the centre has the
        # sense of (a e3) x F, i.e. rolling on the neighbour
        assert np.dot(o["Ti"], np.cross(e3, o["F"])) > 0
        # 3) rotation of i about e2
        W = 1.1
        o = ref.pair_eval(d, qi, [a, a], z, W * e2, qj, [b, b], z, z, P)
        assert np.allclose(o["F"], -mu * c["couple"] * Lg * W * np.cross(e3, e2),
                           rtol=1e-9, atol=1e-12)
        assert np.allclose(o["Ti"], mu * c["rot"] * Lg * W * e2, rtol=1e-9,
                           atol=1e-12 * a ** 3)
        # 4) spin about the line of centres: no singular term
        o = ref.pair_eval(d, qi, [a, a], z, W * e3, qj, [b, b], z, z, P)
        scale = mu * c["rot"] * abs(Lg) * W
        assert np.allclose(o["F"], 0, atol=1e-12 * scale)
        assert np.allclose(o["Ti"], 0, atol=1e-12 * scale)


def gcb_coefficients(a):
    """The Goldman-Cox-Brenner leading coefficients for radius a, from the
    cited fixture (literature normalisation: prefactor, fraction, power)."""
    import os
    from fractions import Fraction
    path = os.path.join(os.path.dirname(__file__), "golden", "sphere_wall_gcb.txt")
    out = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        name, pref, frac, power = line.split()
        out[name] = {"6pi": 6.0, "8pi": 8.0}[pref] * np.pi * float(Fraction(frac)) \
            * a ** int(power)
    return out


def test_sphere_wall_goldman_cox_brenner(ref):
    """The particle-wall pair of the oracle (wall as a surface with infinite
    radii) against the Goldman-Cox-Brenner leading terms."""
    rng = np.random.default_rng(5)
    a = 3.0
    g = gcb_coefficients(a)
    mu, delta = 0.4, 0.5
    z = np.zeros(3)
    P = ref.make_params(mu=mu, delta_n=delta, delta_t=delta, delta_r=delta)
    Ltop = 50.0
    dom = ref.make_domain(L=(100, 100, Ltop), periodic=(1, 1, 0), n_walls=2)
    for side in (0, 1):
        for h in (1e-4, 1e-2, 0.3):
            zc = a + h if side == 0 else Ltop - a - h
            r = np.array([10.0, 20.0, zc])
            e3 = np.array([0, 0, -1.0]) if side == 0 else np.array([0, 0, 1.0])
            Lg = np.log(h / delta)
            o = ref.wall_eval(r, rand_quat(rng), [a, a], 0.8 * e3, z, side, dom, P)
            assert abs(o["h"] - h) < 1e-12 * Ltop
            assert np.allclose(o["F"], -mu * g["K33_times_h"] * (1 / h - 1 / delta)
                               * 0.8 * e3, rtol=1e-9)
            e1 = np.array([1.0, 0, 0])
            o = ref.wall_eval(r, rand_quat(rng), [a, a], 0.8 * e1, z, side, dom, P)
            assert np.allclose(o["F"], mu * g["tangential_ln"] * Lg * 0.8 * e1, rtol=1e-9)
            assert np.allclose(o["Ti"], mu * g["coupling_ln"] * Lg * 0.8
                               * np.cross(e3, e1), rtol=1e-9, atol=1e-13)
            e2 = np.cross(e3, e1)
            o = ref.wall_eval(r, rand_quat(rng), [a, a], z, 0.5 * e2, side, dom, P)
            assert np.allclose(o["F"], -mu * g["coupling_ln"] * Lg * 0.5
                               * np.cross(e3, e2), rtol=1e-9)
            assert np.allclose(o["Ti"], mu * g["rotation_ln"] * Lg * 0.5 * e2,
                               rtol=1e-9)


def test_moving_wall_is_relative_motion(ref):
    """Only relative velocities enter Eq. lub:resistance: a wall moving with
    U under a resting sphere equals the sphere moving with -U."""
    a = 2.0
    P = ref.make_params(mu=1.0, h_c=0.0, eps_c=0.0)
    U = np.array([0.3, -0.2, 0.0])
    dom_m = ref.make_domain(L=(100, 100, 40), periodic=(1, 1, 0), n_walls=2,
                            wall_vel=((0, 0, 0), tuple(U)))
    dom_s = ref.make_domain(L=(100, 100, 40), periodic=(1, 1, 0), n_walls=2)
    r = np.array([1.0, 2.0, 40 - a - 0.05])
    q = [1, 0, 0, 0]
    o1 = ref.wall_eval(r, q, [a, a], np.zeros(3), np.zeros(3), 1, dom_m, P)
    o2 = ref.wall_eval(r, q, [a, a], -U, np.zeros(3), 1, dom_s, P)
    assert np.allclose(o1["F"], o2["F"], rtol=1e-13, atol=1e-15)
    assert np.allclose(o1["Ti"], o2["Ti"], rtol=1e-13, atol=1e-15)


def test_unequal_cutoffs_rotation_torque(ref):
    """With separate cut-offs the torque on a rotating sphere near a wall is
    -mu w [K~55 + 2a K~15 + a^2 K~11] (the combination the paper notes
    involves both Delta_t and Delta_r, Sec. IV.A)."""
    a, mu, h = 2.0, 1.0, 0.01
    P = ref.make_params(mu=mu, delta_n=2 / 3, delta_t=0.5, delta_r=0.25)
    dom = ref.make_domain(L=(100, 100, 40), periodic=(1, 1, 0), n_walls=2)
    r = np.array([0.0, 0.0, a + h])
    W = 0.7
    o = ref.wall_eval(r, [1, 0, 0, 0], [a, a], np.zeros(3), [0, W, 0], 0, dom, P)
    e3 = np.array([0, 0, -1.0])
    e1 = np.array([1.0, 0, 0])
    e2 = np.cross(e3, e1)     # = -y
    Lt, Lr = np.log(h / 0.5), np.log(h / 0.25)
    c11 = -16 / 5 * np.pi * a
    c15 = 12 / 5 * np.pi * a * a
    c55 = -24 / 5 * np.pi * a ** 3
    w2 = W * np.dot([0, 1, 0], e2)
    expect = -mu * w2 * (c55 * Lr + 2 * a * c15 * Lt + a * a * c11 * Lt)
    assert np.isclose(np.dot(o["Ti"], e2), expect, rtol=1e-10)


def test_contact_model(ref):
    """Eqs. lub:frep and lub:model: gap clipped at h_c inside K~, Hookean
    repulsion eps_c (h_c - h) for 0<h<h_c, capped at eps_c h_c for h<=0,
    along -x3 on particle i."""
    a, b = 3.0, 2.0
    hc, ec = 0.01, 100.0
    P = ref.make_params(mu=1.0, h_c=hc, eps_c=ec)
    P0 = ref.make_params(mu=1.0, h_c=hc, eps_c=0.0)
    z = np.zeros(3)
    e3 = unit(np.array([0.3, -0.4, 0.8]))
    q = [1, 0, 0, 0]
    for h in (0.5 * hc, 1e-6, -0.02, -0.2):
        d = (a + b + h) * e3
        o = ref.pair_eval(d, q, [a, a], z, z, q, [b, b], z, z, P)
        Fr = ec * (hc - h) if h > 0 else ec * hc
        assert np.allclose(o["F"], -Fr * e3, rtol=1e-10)
        # viscous part evaluated at h_c
        vi = np.array([0.2, 0.1, -0.3])
        o1 = ref.pair_eval(d, q, [a, a], vi, z, q, [b, b], z, z, P0)
        dh = (a + b + hc) * e3
        o2 = ref.pair_eval(dh, q, [a, a], vi, z, q, [b, b], z, z, P0)
        assert np.allclose(o1["F"], o2["F"], rtol=1e-9)
    # continuity of the repulsion at h = h_c and above
    d = (a + b + hc * (1 + 1e-9)) * e3
    o = ref.pair_eval(d, q, [a, a], z, z, q, [b, b], z, z, P)
    assert np.allclose(o["F"], 0, atol=1e-6)
    # h_c = 0 and overlap: unresolved, no contribution
    P00 = ref.make_params(mu=1.0, h_c=0.0, eps_c=0.0)
    o = ref.pair_eval((a + b - 0.01) * e3, q, [a, a], z, z, q, [b, b], z, z, P00)
    assert o["status"] == ref.REFP_UNRESOLVED
    assert np.allclose(o["F"], 0)


def test_beyond_cutoffs_inactive(ref):
    P = ref.make_params()
    q = [1, 0, 0, 0]
    z = np.zeros(3)
    o = ref.pair_eval([8.0 + 2 / 3 + 1e-9, 0, 0], q, [4, 4], [1, 0, 0], z, q, [4, 4],
                      z, z, P)
    assert o["status"] == ref.REFP_INACTIVE
    assert np.allclose(o["F"], 0)
