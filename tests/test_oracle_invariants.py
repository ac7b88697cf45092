"""Invariances the resistance law must satisfy (Sec. III.B; Appendix),
checked on the oracle.  A dropped term, a wrong sign of a Gamma/kappa
contribution or a transposed frame breaks at least one of them.

* i<->j swap: computing the pair from j's side gives equal and opposite
  forces (the paper's own Newton's-third-law check, Sec. IV.B), up to the
  O(h ln h) difference of the torque reference points.
* 90-degree relabel and pi rotation of the tangential frame act on the
  printed K as the corresponding rotation of force and velocity axes.
* Global rotation, translation, Galilean invariance, linearity.
* Dimensional scaling of the h^-1 and ln h terms.
* Symmetry of the 12x12 pair resistance matrix (reciprocity of the
  rigid-body transfer) and positive semi-definiteness where it holds.
"""
import numpy as np
import pytest


def unit(v):
    return v / np.linalg.norm(v)


def rquat(rng):
    return unit(rng.normal(size=4))


def quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def place(ref, qi, si, qj, sj, u, gap):
    lo, hi = 0.0, 2 * (si.max() + sj.max()) + 2
    for _ in range(90):
        mid = 0.5 * (lo + hi)
        o = ref.closest_points(mid * u, qi, si, qj, sj)
        hi, lo = (mid, lo) if (o["status"] == 0 and o["h"] > gap) else (hi, mid)
    return hi * u


SHAPES = [np.array(s) for s in ([8.0, 4.0], [1.0, 3.0], [3.0, 1.0], [2.0, 6.0],
                                [5.0, 5.0], [7.0, 2.5])]


def random_pair(ref, rng, gap):
    si = SHAPES[rng.integers(len(SHAPES))]
    sj = SHAPES[rng.integers(len(SHAPES))]
    qi, qj = rquat(rng), rquat(rng)
    u = unit(rng.normal(size=3))
    d = place(ref, qi, si, qj, sj, u, gap)
    vel = [rng.normal(size=3) for _ in range(4)]
    return d, qi, si, qj, sj, vel


@pytest.mark.parametrize("seed", range(10))
def test_swap_newton_third_law(ref, seed):
    """Both surfaces computed independently (Sec. IV.B): the pair seen from
    j gives the opposite force, and each particle's torque agrees."""
    rng = np.random.default_rng(300 + seed)
    P = ref.make_params(mu=1.0, delta_n=0.67, delta_t=0.5, delta_r=0.25)
    for gap in (1e-4, 1e-2, 0.1):
        d, qi, si, qj, sj, (vi, wi, vj, wj) = random_pair(ref, rng, gap)
        a = ref.pair_eval(d, qi, si, vi, wi, qj, sj, vj, wj, P)
        b = ref.pair_eval(-d, qj, sj, vj, wj, qi, si, vi, wi, P)
        assert a["status"] == b["status"] == 0
        assert abs(a["h"] - b["h"]) < 1e-12
        assert np.allclose(a["n"], -b["n"], atol=1e-12)
        sF = np.linalg.norm(a["F"])
        sT = max(np.linalg.norm(a["Ti"]), np.linalg.norm(a["Tj"]),
                 sF * max(si.max(), sj.max()))
        # the reference points of the torques differ by h n: O(h ln h)
        tol = 1e-9 + 10 * gap * np.log(1 / gap)
        assert np.linalg.norm(a["F"] + b["F"]) <= 1e-9 * sF + 1e-12
        assert np.linalg.norm(a["Ti"] - b["Tj"]) <= tol * sT
        assert np.linalg.norm(a["Tj"] - b["Ti"]) <= tol * sT


def test_swap_isolates_each_element(ref):
    """The swap check per resistance element: with only one relative
    velocity component non-zero at a time (in i's frame), the forces on
    both sides agree.  A sign error in one Gamma or kappa term shows up in
    exactly the columns that use it."""
    rng = np.random.default_rng(77)
    P = ref.make_params(mu=1.0, delta_n=1.0, delta_t=1.0, delta_r=1.0)
    z = np.zeros(3)
    for _ in range(20):
        d, qi, si, qj, sj, _ = random_pair(ref, rng, 1e-3)
        base = ref.pair_eval(d, qi, si, z, z, qj, sj, z, z, P)
        E = np.array(base["e"])
        for col in range(6):
            vj = E[col] if col < 3 else z
            wj = E[col - 3] if col >= 3 else z
            # rotation of j about its contact point: subtract the lever arm
            if col >= 3:
                vj = -np.cross(wj, base["yj"])
            a = ref.pair_eval(d, qi, si, z, z, qj, sj, vj, wj, P)
            b = ref.pair_eval(-d, qj, sj, vj, wj, qi, si, z, z, P)
            scale = (np.abs(a["Fbar"]).max() + np.abs(b["Fbar"]).max()
                     + 1e-6 * np.abs(a["Kt"]).max())
            assert np.linalg.norm(a["F"] + b["F"]) < 1e-8 * scale, (col, a["F"], b["F"])


def rot(axis, ang):
    axis = unit(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K


def mat_to_quat(R):
    w = np.sqrt(max(0.0, 1 + R[0, 0] + R[1, 1] + R[2, 2])) / 2
    x = np.copysign(np.sqrt(max(0.0, 1 + R[0, 0] - R[1, 1] - R[2, 2])) / 2, R[2, 1] - R[1, 2])
    y = np.copysign(np.sqrt(max(0.0, 1 - R[0, 0] + R[1, 1] - R[2, 2])) / 2, R[0, 2] - R[2, 0])
    z = np.copysign(np.sqrt(max(0.0, 1 - R[0, 0] - R[1, 1] + R[2, 2])) / 2, R[1, 0] - R[0, 1])
    return np.array([w, x, y, z])


def test_global_rotation(ref):
    rng = np.random.default_rng(4)
    P = ref.make_params(mu=1.0 / 6, h_c=0.01, eps_c=100.0)
    for _ in range(20):
        d, qi, si, qj, sj, (vi, wi, vj, wj) = random_pair(ref, rng, 10 ** rng.uniform(-3, -0.5))
        R = rot(rng.normal(size=3), rng.uniform(0, 2 * np.pi))
        qR = mat_to_quat(R)
        assert np.allclose(ref.quat_to_matrix(qR), R, atol=1e-12)
        a = ref.pair_eval(d, qi, si, vi, wi, qj, sj, vj, wj, P)
        b = ref.pair_eval(R @ d, quat_mul(qR, qi), si, R @ vi, R @ wi,
                          quat_mul(qR, qj), sj, R @ vj, R @ wj, P)
        sF = np.linalg.norm(a["F"]) + 1e-30
        sT = np.linalg.norm(a["Ti"]) + np.linalg.norm(a["Tj"]) + sF
        assert np.linalg.norm(R @ a["F"] - b["F"]) < 1e-8 * sF
        assert np.linalg.norm(R @ a["Ti"] - b["Ti"]) < 1e-8 * sT
        assert np.linalg.norm(R @ a["Tj"] - b["Tj"]) < 1e-8 * sT


def test_galilean_and_linearity(ref):
    rng = np.random.default_rng(6)
    P = ref.make_params(mu=0.3, h_c=0.0, eps_c=0.0)
    for _ in range(20):
        d, qi, si, qj, sj, (vi, wi, vj, wj) = random_pair(ref, rng, 10 ** rng.uniform(-3, -0.5))
        U = rng.normal(size=3) * 5
        a = ref.pair_eval(d, qi, si, vi, wi, qj, sj, vj, wj, P)
        b = ref.pair_eval(d, qi, si, vi + U, wi, qj, sj, vj + U, wj, P)
        s = np.linalg.norm(a["F"]) + 1e-30
        assert np.linalg.norm(a["F"] - b["F"]) < 1e-9 * s * 10
        c = ref.pair_eval(d, qi, si, 2.5 * vi, 2.5 * wi, qj, sj, 2.5 * vj, 2.5 * wj, P)
        assert np.allclose(c["F"], 2.5 * a["F"], rtol=1e-10, atol=1e-14)
        assert np.allclose(c["Ti"], 2.5 * a["Ti"], rtol=1e-10, atol=1e-14)
        z = np.zeros(3)
        e = ref.pair_eval(d, qi, si, vi, vi * 0, qj, sj, vi, z, P)
        assert np.allclose(e["F"], 0, atol=1e-12)


def test_dimensional_scaling(ref):
    """Lengths (semi-axes, separation, cut-offs) scaled by s with velocities
    fixed: translation-induced force scales as s (h^-1 and ln h terms),
    torque as s^2; rotation-induced force s^2, torque s^3."""
    rng = np.random.default_rng(8)
    z = np.zeros(3)
    for _ in range(10):
        d, qi, si, qj, sj, (vi, wi, vj, wj) = random_pair(ref, rng, 10 ** rng.uniform(-3, -0.5))
        s = rng.uniform(0.3, 3.0)
        P1 = ref.make_params(mu=1.0, delta_n=0.67, delta_t=0.5, delta_r=0.25)
        Ps = ref.make_params(mu=1.0, delta_n=0.67 * s, delta_t=0.5 * s, delta_r=0.25 * s)
        a = ref.pair_eval(d, qi, si, vi, z, qj, sj, vj, z, P1)
        b = ref.pair_eval(s * d, qi, s * si, vi, z, qj, s * sj, vj, z, Ps)
        assert np.allclose(b["F"], s * a["F"], rtol=1e-8, atol=1e-12)
        assert np.allclose(b["Ti"], s * s * a["Ti"], rtol=1e-8, atol=1e-12)
        a = ref.pair_eval(d, qi, si, z, wi, qj, sj, z, wj, P1)
        b = ref.pair_eval(s * d, qi, s * si, z, wi, qj, s * sj, z, wj, Ps)
        assert np.allclose(b["F"], s * s * a["F"], rtol=1e-8, atol=1e-12)
        assert np.allclose(b["Ti"], s ** 3 * a["Ti"], rtol=1e-8, atol=1e-12)


def block(R3):
    P = np.zeros((6, 6))
    P[:3, :3] = R3
    P[3:, 3:] = R3
    return P


@pytest.mark.parametrize("seed", range(20))
def test_frame_relabel_invariance(ref, seed):
    """Appendix K with general cubic coefficients: rotating the tangential
    frame by 90 degrees (x1 -> x2, x2 -> -x1: S1<->S2, Gamma_k ->
    (-1)^m Gamma_{3-m}) or by 180 degrees (all Gamma change sign) must act
    on K as the same rotation of force and velocity axes."""
    rng = np.random.default_rng(seed)
    S1, S2 = rng.uniform(0.5, 10, size=2)
    iS1p, iS2p = rng.uniform(0.0, 2.0, size=2)
    G = rng.normal(size=4) * 0.1
    Gp = rng.normal(size=4) * 0.1
    ph = rng.uniform(0, 2 * np.pi)
    C, aux = ref.K_coeffs(S1, S2, iS1p, iS2p, G, Gp, np.cos(ph), np.sin(ph))
    # 90 degrees: new x1 = old x2, new x2 = -old x1
    Gn = np.array([G[3], -G[2], G[1], -G[0]])
    Gpn = np.array([Gp[3], -Gp[2], Gp[1], -Gp[0]])
    Cn, _ = ref.K_coeffs(S2, S1, iS2p, iS1p, Gn, Gpn, np.cos(ph), np.sin(ph))
    R = np.array([[0, 1.0, 0], [-1.0, 0, 0], [0, 0, 1.0]])
    Pm = block(R)
    scale = np.abs(C).max()
    assert np.allclose(Cn, Pm @ C @ Pm.T, atol=1e-10 * scale)
    # 180 degrees
    Cp, _ = ref.K_coeffs(S1, S2, iS1p, iS2p, -G, -Gp, np.cos(ph), np.sin(ph))
    Pm = block(np.diag([-1.0, -1.0, 1.0]))
    assert np.allclose(Cp, Pm @ C @ Pm.T, atol=1e-10 * scale)
    # symmetric, and the sixth row/column holds only K36
    assert np.allclose(C, C.T)
    assert np.allclose(C[5, [0, 1, 3, 4, 5]], 0)


def pair_matrix(ref, d, qi, si, qj, sj, P):
    """12x12 map (v_i, w_i, v_j, w_j) -> (f_i, t_i, f_j, t_j)."""
    A = np.zeros((12, 12))
    z = np.zeros(3)
    for c in range(12):
        e = np.zeros(12)
        e[c] = 1.0
        o = ref.pair_eval(d, qi, si, e[0:3], e[3:6], qj, sj, e[6:9], e[9:12], P)
        A[:, c] = np.concatenate([o["F"], o["Ti"], -o["F"], o["Tj"]])
    return A


def test_pair_matrix_symmetric(ref):
    rng = np.random.default_rng(10)
    P = ref.make_params(mu=1.0, h_c=0.0, eps_c=0.0)
    for _ in range(10):
        d, qi, si, qj, sj, _ = random_pair(ref, rng, 10 ** rng.uniform(-3, -0.5))
        A = pair_matrix(ref, d, qi, si, qj, sj, P)
        assert np.allclose(A, A.T, atol=1e-9 * np.abs(A).max())


def test_psd_where_it_holds(ref):
    """Dissipation: -A is positive semi-definite for sphere pairs,
    sphere-wall and spheroid-wall pairs with equal cut-offs (no K36)."""
    rng = np.random.default_rng(12)
    P = ref.make_params(mu=1.0, delta_n=0.5, delta_t=0.5, delta_r=0.5)
    for _ in range(10):
        a, b = rng.uniform(1, 8, size=2)
        u = unit(rng.normal(size=3))
        h = 10 ** rng.uniform(-4, -0.5)
        d = (a + b + h) * u
        A = pair_matrix(ref, d, rquat(rng), np.array([a, a]), rquat(rng),
                        np.array([b, b]), P)
        ev = np.linalg.eigvalsh(-(A + A.T) / 2)
        assert ev.min() > -1e-9 * ev.max()
    dom = ref.make_domain(L=(100, 100, 50), periodic=(1, 1, 0), n_walls=2)
    for _ in range(10):
        s = SHAPES[rng.integers(len(SHAPES))]
        q = rquat(rng)
        z0 = np.sqrt(ref.quat_to_matrix(q)[2] @ np.diag([s[1] ** 2, s[1] ** 2, s[0] ** 2])
                     @ ref.quat_to_matrix(q)[2])
        r = np.array([3.0, 4.0, z0 + 10 ** rng.uniform(-4, -0.5)])
        M = np.zeros((6, 6))
        for c in range(6):
            e = np.zeros(6)
            e[c] = 1
            o = ref.wall_eval(r, q, s, e[:3], e[3:], 0, dom, P)
            M[:, c] = np.concatenate([o["F"], o["Ti"]])
        ev = np.linalg.eigvalsh(-(M + M.T) / 2)
        assert np.allclose(M, M.T, atol=1e-9 * np.abs(M).max())
        assert ev.min() > -1e-9 * ev.max()
