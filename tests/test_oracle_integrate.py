"""Pins of the reference integrator (sub-stepped update of Sec. II) and of
the contact-only law used by the growth stage (Sec. IV.C).

* Constant force on a free particle: the semi-implicit Euler step has the
  closed form v_N = v_0 + N dt F/m, r_N = r_0 + N dt v_0 + dt^2 F/m N(N+1)/2,
  with m = density 4/3 pi R_par R_perp^2.
* Damping alone: v_N = v_0 (1 - damping dt)^N.
* Constant torque on a sphere: w_N = w_0 + N dt T / (2/5 m a^2).
* Torque-free symmetric top: L stays fixed, the spin L.a / I_par is
  constant and the axis precesses about L at |L| / I_perp (Euler's
  solution), within the step's O(dt) error.
* Pair forces only (periodic box): total momentum sum m v is conserved.
* Lees-Edwards re-entry: through the top a particle moves by -offset in x
  and loses the image velocity; the offset advances by U dt per sub-step.
* Contact-only law: sphere pair F = -eps_c (h_c - h) n on i for 0 < h <= h_c,
  -eps_c h_c for overlaps, nothing beyond h_c, no torque.
* Kinematic advance with a constant angular velocity w: 1 + dt/2 (0, w) is
  sqrt(1 + a^2) times the unit quaternion of a rotation by 2 atan(a) about
  w (a = dt |w| / 2), so after N steps q_N = (cos N phi, sin N phi w/|w|) q_0
  with phi = atan(a) (left product: the rotation acts in the world frame),
  and r_N = r_0 + N dt v.
"""
import numpy as np
import pytest

import oracle as O
from oracle import integrate as I


def free_domain():
    return O.make_domain(L=(1e4, 1e4, 1e4), periodic=(0, 0, 0))


def params():
    return O.make_params(mu=1.0 / 6.0, delta_n=0.67, delta_t=0.5, delta_r=0.25,
                         h_c=0.01, eps_c=100.0)


def unit(x):
    return x / np.linalg.norm(x)


def test_constant_force_closed_form():
    rng = np.random.default_rng(1)
    semi = np.array([[6.0, 3.0]])
    r0 = np.array([[500.0, 400.0, 300.0]])
    q0 = unit(rng.normal(size=(1, 4)))
    v0 = rng.normal(size=(1, 3))
    w0 = np.zeros((1, 3))
    F = rng.normal(size=(1, 3))
    dt, N, rho = 0.05, 40, 1.3
    r, q, v, w, f, t, _ = I.integrate(r0, q0, semi, v0, w0, free_domain(), params(), dt, N,
                                      density=rho, f_ext=F)
    m = rho * 4.0 / 3.0 * np.pi * 6.0 * 3.0 * 3.0
    assert np.allclose(v, v0 + N * dt * F / m, rtol=1e-13, atol=1e-15)
    assert np.allclose(r, r0 + N * dt * v0 + dt * dt * F / m * N * (N + 1) / 2,
                       rtol=1e-13, atol=1e-11)
    assert np.array_equal(f, np.zeros((1, 3)))


def test_damping_closed_form():
    semi = np.array([[4.0, 4.0]])
    v0 = np.array([[0.3, -0.2, 0.1]])
    w0 = np.array([[0.01, 0.02, -0.03]])
    dt, N, g = 0.1, 25, 0.7
    r, q, v, w, *_ = I.integrate(np.array([[50.0, 50.0, 50.0]]), np.array([[1.0, 0, 0, 0]]),
                                 semi, v0, w0, free_domain(), params(), dt, N, damping=g)
    assert np.allclose(v, v0 * (1 - g * dt) ** N, rtol=1e-12)
    # a sphere: L = I w, so the spin decays the same way
    assert np.allclose(w, w0 * (1 - g * dt) ** N, rtol=1e-12)


def test_constant_torque_sphere():
    a = 3.5
    semi = np.array([[a, a]])
    T = np.array([[0.2, -0.1, 0.05]])
    dt, N, rho = 0.02, 30, 0.8
    r, q, v, w, *_ = I.integrate(np.array([[50.0, 50.0, 50.0]]), np.array([[1.0, 0, 0, 0]]),
                                 semi, np.zeros((1, 3)), np.zeros((1, 3)), free_domain(),
                                 params(), dt, N, density=rho, t_ext=T)
    m = rho * 4.0 / 3.0 * np.pi * a ** 3
    assert np.allclose(w, N * dt * T / (0.4 * m * a * a), rtol=1e-12)
    # the orientation stays a unit quaternion
    assert abs(np.linalg.norm(q) - 1.0) < 1e-14


def test_torque_free_symmetric_top():
    semi = np.array([[8.0, 3.0]])  # prolate: I_par < I_perp
    rho = 1.0
    m, Ipa, Ipe = (x[0] for x in I.mass_inertia(semi, rho))
    q0 = np.array([[np.cos(0.3), np.sin(0.3), 0.0, 0.0]])  # axis tilted about x
    a0 = I.body_axes(q0)[0]
    w0 = np.array([[0.02, 0.05, 0.01]])
    aw = a0 @ w0[0]
    L0 = Ipe * w0[0] + (Ipa - Ipe) * aw * a0
    T_end, dt = 60.0, 0.002
    N = int(round(T_end / dt))
    r, q, v, w, *_ = I.integrate(np.array([[50.0, 50.0, 50.0]]), q0, semi, np.zeros((1, 3)),
                                 w0, free_domain(), params(), dt, N, density=rho)
    a1 = I.body_axes(q)[0]
    L1 = Ipe * w[0] + (Ipa - Ipe) * (a1 @ w[0]) * a1
    # conserved up to the rounding of 30,000 steps
    assert np.allclose(L1, L0, rtol=1e-10, atol=0)
    # the spin a.L is conserved by the motion, here within the step's error
    assert abs(a1 @ L0 - a0 @ L0) < 2e-4 * np.linalg.norm(L0)
    # Euler: the axis precesses about L at |L| / I_perp
    lh = L0 / np.linalg.norm(L0)
    ang = np.linalg.norm(L0) / Ipe * T_end
    par = (a0 @ lh) * lh
    perp = a0 - par
    expect = par + np.cos(ang) * perp + np.sin(ang) * np.cross(lh, perp)
    assert np.linalg.norm(a1 - expect) < 2e-3, np.linalg.norm(a1 - expect)
    # and the step error shrinks with dt (first order)
    r2, q2, *_ = I.integrate(np.array([[50.0, 50.0, 50.0]]), q0, semi, np.zeros((1, 3)), w0,
                             free_domain(), params(), 2 * dt, N // 2, density=rho)
    e2 = np.linalg.norm(I.body_axes(q2)[0] - expect)
    assert e2 > 1.5 * np.linalg.norm(a1 - expect)


def test_momentum_conserved_by_pair_forces():
    from paper_1308_6482_amd import workloads as W
    wl = W.config2(n=300)
    rng = np.random.default_rng(3)
    v0 = rng.normal(scale=0.05, size=(wl.n, 3))
    w0 = rng.normal(scale=0.01, size=(wl.n, 3))
    dom = O.make_domain(L=wl.L, periodic=(1, 1, 1))
    P = O.make_params(**wl.params)
    rho = 1.0
    m = I.mass_inertia(wl.semi, rho)[0]
    r, q, v, w, f, t, _ = I.integrate(wl.r, wl.q, wl.semi, v0, w0, dom, P, 0.1, 8,
                                      density=rho)
    p0 = (m[:, None] * v0).sum(axis=0)
    p1 = (m[:, None] * v).sum(axis=0)
    scale = (m[:, None] * np.abs(v - v0)).sum()
    assert scale > 0
    assert np.allclose(p1, p0, rtol=0, atol=1e-10 * scale)


def test_lees_edwards_reentry():
    L = (40.0, 40.0, 40.0)
    U, off0, dt = 0.4, 5.0, 0.5
    dom = O.make_domain(L=L, periodic=(1, 1, 1), lees_edwards=(off0, U))
    r0 = np.array([[10.0, 20.0, 39.9], [30.0, 20.0, 0.05]])
    v0 = np.array([[0.0, 0.0, 1.0], [0.1, 0.0, -1.0]])
    z = np.zeros((2, 3))
    q0 = np.array([[1.0, 0, 0, 0], [1.0, 0, 0, 0]])
    semi = np.array([[1.0, 1.0], [1.0, 1.0]])
    r, q, v, w, f, t, dom1 = I.integrate(r0, q0, semi, v0, z, dom, params(), dt, 1)
    off1 = off0 + U * dt
    assert dom1.le_offset == off1
    # particle 0 leaves through the top: x - offset, z - L, v_x - U
    assert np.allclose(r[0], [10.0 - off1, 20.0, 39.9 + 0.5 - 40.0])
    assert np.allclose(v[0], [-U, 0.0, 1.0])
    # particle 1 leaves through the bottom: x + offset (wrapped), v_x + U
    assert np.allclose(r[1], [(30.0 + 0.05 + off1) % 40.0, 20.0, 0.05 - 0.5 + 40.0])
    assert np.allclose(v[1], [0.1 + U, 0.0, -1.0])


@pytest.mark.parametrize("h", [0.05, 0.2, -0.1, 0.31])
def test_contact_only_law(ref, h):
    a, b, hc, ec = 4.0, 2.5, 0.3, 50.0
    u = unit(np.array([0.3, -0.4, 0.8]))
    P = O.make_params(h_c=hc, eps_c=ec, model=O.MODEL_CONTACT)
    rng = np.random.default_rng(5)
    vi, wi, vj, wj = (rng.normal(size=3) for _ in range(4))
    q = np.array([1.0, 0, 0, 0])
    o = ref.pair_eval((a + b + h) * u, q, [a, a], vi, wi, q, [b, b], vj, wj, P)
    if h > hc:
        assert o["status"] == ref.REFP_INACTIVE
        return
    assert o["status"] == ref.REFP_ACTIVE
    Fr = ec * (hc - h) if h > 0 else ec * hc
    assert np.allclose(o["F"], -Fr * u, rtol=1e-12, atol=1e-12)
    assert np.allclose(o["Ti"], 0, atol=1e-10 * Fr) and np.allclose(o["Tj"], 0, atol=1e-10 * Fr)


def test_advance_closed_form():
    rng = np.random.default_rng(7)
    n, N, dt = 6, 25, 0.3
    r0 = rng.normal(size=(n, 3)) * 50.0
    q0 = rng.normal(size=(n, 4))
    q0 /= np.linalg.norm(q0, axis=1)[:, None]
    v = rng.normal(size=(n, 3))
    w = rng.normal(size=(n, 3)) * 0.2
    r, q = r0, q0
    for _ in range(N):
        r, q = I.advance(r, q, v, w, dt)
    wn = np.linalg.norm(w, axis=1)
    phi = N * np.arctan(0.5 * dt * wn)
    rot = np.concatenate([np.cos(phi)[:, None], np.sin(phi)[:, None] * w / wn[:, None]], axis=1)
    assert np.allclose(q, I.quat_mul(rot, q0), rtol=0, atol=1e-13)
    # the right product (body-frame rotation) differs for these orientations
    assert not np.allclose(q, I.quat_mul(q0, rot), rtol=0, atol=1e-3)
    assert np.allclose(r, r0 + N * dt * v, rtol=1e-14, atol=1e-12)
    # the symmetry axis turns about w by 2 N phi (Rodrigues)
    a0, a = I.body_axes(q0), I.body_axes(q)
    k = w / wn[:, None]
    th = 2.0 * phi
    rod = (a0 * np.cos(th)[:, None] + np.cross(k, a0) * np.sin(th)[:, None]
           + k * (np.sum(k * a0, axis=1) * (1.0 - np.cos(th)))[:, None])
    assert np.allclose(a, rod, rtol=0, atol=1e-12)


def test_advance_zero_spin_keeps_orientation():
    rng = np.random.default_rng(8)
    q0 = rng.normal(size=(4, 4))
    q0 /= np.linalg.norm(q0, axis=1)[:, None]
    r, q = I.advance(np.zeros((4, 3)), q0, np.ones((4, 3)), np.zeros((4, 3)), 2.0)
    assert np.array_equal(q, q0 / np.linalg.norm(q0, axis=1)[:, None])
    assert np.array_equal(r, np.full((4, 3), 2.0))
