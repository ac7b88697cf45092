"""FP64 reference of the sub-stepped particle update and of the growth stage
of the packing generator.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle``): only ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg use it.

Sec. II: the particle time step is decoupled from the fluid's and made a
fraction of it, with the hydrodynamic force from the fluid held fixed over a
fluid step and the lubrication (and contact) forces evaluated again at every
sub-step.  The paper fixes no scheme beyond that; this reference takes the
semi-implicit Euler step with the angular momentum in the world frame:

    F = f_ext + f(state),  T = t_ext + t(state)
    v <- v + dt (F / m - damping v)
    L = I(q) w;  L <- L + dt (T - damping L)
    q <- p(dt I(q)^-1 L) q      p(u): rotation by the angle |u| about u
    r <- r + dt v;  w <- I(q)^-1 L

m = density 4/3 pi R_par R_perp^2; inertia I_par = 2/5 m R_perp^2 about the
symmetry axis, I_perp = 1/5 m (R_par^2 + R_perp^2) across it (the solid
ellipsoid).  Periodic axes are wrapped into [0, L); with Lees-Edwards images
the offset advances by the image velocity times dt first, and a particle
leaving through z = L_z (z = 0) re-enters at -offset (+offset) in x with its
x velocity lowered (raised) by the image velocity.

Sec. IV.C, growth stage: particles placed at a reduced linear size grow to
slightly beyond their final size, free to move and turn, with the Hookean
repulsion of Eq. lub:frep as the only interaction and damped velocities.
Here the scale rises linearly, s_k = s0 + (s1 - s0) (k + 1) / n_steps for
steps k = 0 .. n_steps - 1, one update per step.
"""
from __future__ import annotations

import numpy as np

from . import MODEL_CONTACT, compute, make_domain, make_params


def body_axes(q):
    """Symmetry axis Q(q) e_z of unit quaternions (w, x, y, z), shape (n,3)."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    return np.stack([2.0 * (x * z + w * y), 2.0 * (y * z - w * x),
                     1.0 - 2.0 * (x * x + y * y)], axis=1)


def mass_inertia(semi, density):
    a, b = semi[:, 0], semi[:, 1]
    m = density * (4.0 / 3.0 * np.pi) * a * b * b
    return m, 0.4 * m * b * b, 0.2 * m * (a * a + b * b)


def quat_mul(p, q):
    """Hamilton product p q of (n,4) arrays (w, x, y, z)."""
    p0, p1, p2, p3 = p.T
    q0, q1, q2, q3 = q.T
    return np.stack([p0 * q0 - p1 * q1 - p2 * q2 - p3 * q3,
                     p0 * q1 + p1 * q0 + p2 * q3 - p3 * q2,
                     p0 * q2 - p1 * q3 + p2 * q0 + p3 * q1,
                     p0 * q3 + p1 * q2 - p2 * q1 + p3 * q0], axis=1)


def omega_from_L(L, a, Ipa, Ipe):
    """I^-1 L with I = I_perp 1 + (I_par - I_perp) a a^T."""
    aL = np.sum(a * L, axis=1)
    return L / Ipe[:, None] + ((1.0 / Ipa - 1.0 / Ipe) * aL)[:, None] * a


def update(r, q, semi, v, w, F, T, dt, density, damping, domain):
    """One particle update (no force evaluation); returns new (r, q, v, w).
    domain: an oracle Domain whose Lees-Edwards offset is that of the new
    time."""
    m, Ipa, Ipe = mass_inertia(semi, density)
    v = v + dt * (F / m[:, None] - damping * v)
    a = body_axes(q)
    aw = np.sum(a * w, axis=1)
    L = Ipe[:, None] * w + ((Ipa - Ipe) * aw)[:, None] * a
    L = L + dt * (T - damping * L)
    om = omega_from_L(L, a, Ipa, Ipe)
    on = np.linalg.norm(om, axis=1)
    half = 0.5 * on * dt
    safe = np.where(on > 0.0, on, 1.0)
    p = np.concatenate([np.cos(half)[:, None], (np.sin(half) / safe)[:, None] * om], axis=1)
    qn = quat_mul(p, q)
    qn = qn / np.linalg.norm(qn, axis=1)[:, None]
    q = np.where((on > 0.0)[:, None], qn, q)
    w = omega_from_L(L, body_axes(q), Ipa, Ipe)
    r = r + dt * v
    Lb = np.array(domain.L[:])
    per = [bool(domain.periodic[k]) for k in range(3)]
    if domain.lees_edwards:
        c = np.floor(r[:, 2] / Lb[2])
        r[:, 2] -= c * Lb[2]
        r[:, 0] -= c * domain.le_offset
        v[:, 0] -= c * domain.le_velocity
        per[2] = False
    for k in range(3):
        if per[k]:
            r[:, k] -= Lb[k] * np.floor(r[:, k] / Lb[k])
    return r, q, v, w


def advance(r, q, v, w, dt):
    """Kinematic advance by the particles' own velocities, no forces (the
    motion between evaluations of a prescribed flow): r + dt v, and the
    orientation q + dt/2 (0, w) q normalised (first-order step of
    dq/dt = 1/2 (0, w) q, world-frame angular velocity).  Returns (r, q)."""
    r = np.asarray(r, dtype=np.float64) + dt * np.asarray(v, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    wq = np.concatenate([np.zeros((len(w), 1)), w], axis=1)
    qn = q + 0.5 * dt * quat_mul(wq, q)
    return r, qn / np.linalg.norm(qn, axis=1)[:, None]


def _domain_args(domain):
    return dict(L=tuple(domain.L[:]), periodic=tuple(domain.periodic[:]),
                n_walls=domain.n_walls,
                wall_vel=tuple(tuple(domain.wall_vel[s][:]) for s in range(2)),
                lees_edwards=(domain.le_offset, domain.le_velocity)
                if domain.lees_edwards else None)


def advance_offset(domain, dt):
    """The domain with its Lees-Edwards offset advanced by U dt, kept in
    [0, L_x) (fmod, then + L_x if negative)."""
    if not domain.lees_edwards:
        return domain
    Lx = domain.L[0]
    off = np.fmod(domain.le_offset + domain.le_velocity * dt, Lx)
    if off < 0.0:
        off = off + Lx
    args = _domain_args(domain)
    args["lees_edwards"] = (float(off), domain.le_velocity)
    return make_domain(**args)


def integrate(r, q, semi, v, w, domain, params, dt, n_sub, density=1.0, damping=0.0,
              f_ext=None, t_ext=None):
    """n_sub sub-steps; returns (r, q, v, w, f, t, domain) with f, t the last
    sub-step's correction and domain carrying the advanced offset."""
    r, q, v, w = (np.array(x, dtype=np.float64) for x in (r, q, v, w))
    semi = np.asarray(semi, dtype=np.float64)
    f = t = None
    for _ in range(n_sub):
        f, t, _st = compute(r, q, semi, v, w, domain, params)
        F = f if f_ext is None else f + f_ext
        T = t if t_ext is None else t + t_ext
        domain = advance_offset(domain, dt)
        r, q, v, w = update(r, q, semi, v, w, F, T, dt, density, damping, domain)
    return r, q, v, w, f, t, domain


def grow(r, q, semi, v, w, domain, n_steps, scale0, scale1, dt, density=1.0,
         damping=0.0, h_c=0.1, eps_c=100.0, mu=1.0 / 6.0):
    """Growth stage; returns (r, q, v, w, domain)."""
    r, q, v, w = (np.array(x, dtype=np.float64) for x in (r, q, v, w))
    semi = np.asarray(semi, dtype=np.float64)
    P = make_params(mu=mu, delta_n=0.67, delta_t=0.5, delta_r=0.25, h_c=h_c, eps_c=eps_c,
                    model=MODEL_CONTACT)
    for k in range(n_steps):
        s = scale0 + (scale1 - scale0) * float(k + 1) / float(n_steps)
        sk = semi * s
        f, t, _st = compute(r, q, sk, v, w, domain, P)
        domain = advance_offset(domain, dt)
        r, q, v, w = update(r, q, sk, v, w, f, t, dt, density, damping, domain)
    return r, q, v, w, domain
