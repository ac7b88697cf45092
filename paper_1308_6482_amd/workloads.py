"""Seeded synthetic suspensions shaped like the paper's workloads.

The paper (Sec. IV) simulates spheres and spheroids (aspect ratios 1/3 and
3, radii of a few lattice units) at volume fractions 0.1-0.5 in periodic
boxes, sheared; it uses no public dataset.  These generators produce inputs
of that shape.  They hold none of the lubrication method's arithmetic: the
only geometry here is an overlap test for placement, the Perram-Wertheim
contact function of two ellipsoids (a 1-D concave maximisation), which the
method itself never uses.

Every array is float64, C-contiguous:
  r    (n,3) centres          q (n,4) unit quaternions (w,x,y,z), body z =
  semi (n,2) (R_par, R_perp)  symmetry axis
  v    (n,3) velocities       w (n,3) angular velocities
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

# cut-offs of the paper's sphere validation (Eq. results:cutoffs) with the
# normal cut-off written as 0.67 lattice units
DELTA_N, DELTA_T, DELTA_R = 0.67, 0.5, 0.25
MU = 1.0 / 6.0          # tau = 1, rho = 1
H_C, EPS_C = 0.01, 100.0  # production contact parameters (Sec. IV.C)


@dataclass
class Workload:
    name: str
    r: np.ndarray
    q: np.ndarray
    semi: np.ndarray
    v: np.ndarray
    w: np.ndarray
    L: tuple
    periodic: tuple
    n_walls: int = 0
    wall_vel: tuple = ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    params: dict = field(default_factory=lambda: dict(
        mu=MU, delta_n=DELTA_N, delta_t=DELTA_T, delta_r=DELTA_R, h_c=H_C,
        eps_c=EPS_C))
    meta: dict = field(default_factory=dict)
    # Lees-Edwards images: (offset, velocity) of the image one box up in z
    lees_edwards: tuple = None

    @property
    def n(self) -> int:
        return self.r.shape[0]

    def domain(self) -> dict:
        return dict(L=self.L, periodic=self.periodic, n_walls=self.n_walls,
                    wall_vel=self.wall_vel, lees_edwards=self.lees_edwards)

    def with_params(self, **kw) -> "Workload":
        p = dict(self.params)
        p.update(kw)
        return Workload(self.name, self.r, self.q, self.semi, self.v, self.w,
                        self.L, self.periodic, self.n_walls, self.wall_vel, p,
                        dict(self.meta), self.lees_edwards)


# ---------------------------------------------------------------------------
# elementary random draws
# ---------------------------------------------------------------------------

def random_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform on SO(3): normalised 4-D Gaussian, sign fixed to w >= 0."""
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[q[:, 0] < 0] *= -1.0
    return q


def quat_matrix(q: np.ndarray) -> np.ndarray:
    """Rotation matrices (n,3,3) of unit quaternions (w,x,y,z)."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    return np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                     2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                     2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
                    axis=1).reshape(-1, 3, 3)


def symmetry_axes(q: np.ndarray) -> np.ndarray:
    """Body z axes (n,3) in the world frame of unit quaternions."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    return np.stack([2 * (x * z + w * y), 2 * (y * z - w * x), 1 - 2 * (x * x + y * y)],
                    axis=1)


def shape_matrices(q: np.ndarray, semi: np.ndarray) -> np.ndarray:
    """Q diag(R_perp^2, R_perp^2, R_par^2) Q^T = R_perp^2 I + (R_par^2 -
    R_perp^2) a a^T for each particle (a: symmetry axis)."""
    a = symmetry_axes(q)
    p2 = semi[:, 1] ** 2
    dd = semi[:, 0] ** 2 - p2
    M = dd[:, None, None] * a[:, :, None] * a[:, None, :]
    M[:, [0, 1, 2], [0, 1, 2]] += p2[:, None]
    return M


def shear_velocities(rng: np.random.Generator, r: np.ndarray,
                     gamma_dot: float = 1e-3, sigma: float = 1e-4):
    """Simple shear v = gamma_dot z x + noise, omega = gamma_dot/2 y + noise
    (the vorticity of the shear field)."""
    n = r.shape[0]
    v = rng.normal(scale=sigma, size=(n, 3))
    v[:, 0] += gamma_dot * r[:, 2]
    w = rng.normal(scale=sigma, size=(n, 3))
    w[:, 1] += gamma_dot / 2.0
    return v, w


# ---------------------------------------------------------------------------
# Perram-Wertheim overlap test
# ---------------------------------------------------------------------------

def pw_contact(d: np.ndarray, MA: np.ndarray, MB: np.ndarray,
               iters: int = 48) -> np.ndarray:
    """max over l in [0,1] of l(1-l) d^T [(1-l) MA + l MB]^{-1} d for each
    row (Perram & Wertheim 1985).  The ellipsoids x^T MA^{-1} x <= 1 and
    (x-d)^T MB^{-1} (x-d) <= 1 overlap iff the value is < 1.  Golden-section
    search: the value returned never exceeds the true maximum."""
    def F(lam):
        Cm = (1 - lam)[:, None, None] * MA + lam[:, None, None] * MB
        x = np.linalg.solve(Cm, d[..., None])[..., 0]
        return lam * (1 - lam) * np.einsum("ni,ni->n", d, x)

    g = (np.sqrt(5.0) - 1.0) / 2.0
    a = np.zeros(d.shape[0])
    b = np.ones(d.shape[0])
    for _ in range(iters):
        c1 = b - g * (b - a)
        c2 = a + g * (b - a)
        left = F(c1) > F(c2)   # concave: the maximum lies in [a, c2]
        b = np.where(left, c2, b)
        a = np.where(left, a, c1)
    return F(0.5 * (a + b))


# ---------------------------------------------------------------------------
# random sequential addition in a box
# ---------------------------------------------------------------------------

_GEN_SO = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib",
                       "librsagen.so")
_gen = None


def build_generator(force: bool = True) -> str:
    """Compile the placement routine (csrc/rsa_gen.c) with gcc."""
    if force or not os.path.exists(_GEN_SO):
        os.makedirs(os.path.dirname(_GEN_SO), exist_ok=True)
        src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc",
                           "rsa_gen.c")
        tmp = _GEN_SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               src, "-o", tmp, "-lm"])
        os.replace(tmp, _GEN_SO)
    return _GEN_SO


def _genlib():
    global _gen
    if _gen is None:
        if not os.path.exists(_GEN_SO):
            build_generator(force=True)
        g = ctypes.CDLL(_GEN_SO)
        D = ctypes.POINTER(ctypes.c_double)
        g.rsa_create.restype = ctypes.c_void_p
        g.rsa_create.argtypes = [ctypes.c_int64, D, D,
                                 ctypes.POINTER(ctypes.c_int32)]
        g.rsa_run.restype = ctypes.c_int64
        g.rsa_run.argtypes = [ctypes.c_void_p, ctypes.c_int64, D, D,
                              ctypes.c_double]
        g.rsa_placed.restype = ctypes.c_int64
        g.rsa_placed.argtypes = [ctypes.c_void_p]
        g.rsa_set_lees_edwards.restype = None
        g.rsa_set_lees_edwards.argtypes = [ctypes.c_void_p, ctypes.c_double]
        g.rsa_fetch.argtypes = [ctypes.c_void_p, D, D]
        g.rsa_destroy.argtypes = [ctypes.c_void_p]
        _gen = g
    return _gen


def rsa(rng: np.random.Generator, semi: np.ndarray, L, periodic,
        max_trials: int = 10_000_000, wall_margin: float = 0.0,
        chunk: int = 65536, le_offset: float | None = None):
    """Random sequential addition: place the particles with the given
    semi-axes one after the other at uniform random positions and
    orientations, rejecting every trial that overlaps an accepted particle
    (Perram-Wertheim test) or crosses a wall on a non-periodic axis.
    Returns (r, q, trials); fewer particles than requested if max_trials
    runs out.  le_offset: overlap test with Lees-Edwards images (the image
    one box up in z shifted by le_offset in x)."""
    g = _genlib()
    semi = np.ascontiguousarray(semi, dtype=np.float64)
    n = semi.shape[0]
    Lv = np.ascontiguousarray(L, dtype=np.float64)
    per = np.ascontiguousarray(periodic, dtype=np.int32)
    D = ctypes.POINTER(ctypes.c_double)
    st = g.rsa_create(n, semi.ctypes.data_as(D), Lv.ctypes.data_as(D),
                      per.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if le_offset is not None:
        g.rsa_set_lees_edwards(st, float(le_offset))
    trials = 0
    try:
        while g.rsa_placed(st) < n and trials < max_trials:
            m = min(chunk, max_trials - trials)
            pos = np.ascontiguousarray(rng.uniform(0.0, 1.0, size=(m, 3)))
            quat = np.ascontiguousarray(random_quaternions(rng, m))
            trials += g.rsa_run(st, m, pos.ctypes.data_as(D),
                                quat.ctypes.data_as(D), float(wall_margin))
        k = g.rsa_placed(st)
        r = np.zeros((k, 3))
        q = np.zeros((k, 4))
        g.rsa_fetch(st, r.ctypes.data_as(D), q.ctypes.data_as(D))
    finally:
        g.rsa_destroy(st)
    return r, q, trials


# ---------------------------------------------------------------------------
# the configurations
# ---------------------------------------------------------------------------

def _streams(seed: int, k: int = 4):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(k)]


def config1(seed: int = 0, n: int = 36) -> Workload:
    """Equal spheres of radius 4 in a periodic 32^3 box.  64 spheres would
    be volume fraction 0.52, beyond random sequential addition; capped at
    0.3 the box holds 36 (0.2945).  v, omega i.i.d. N(0,1)."""
    g_pos, g_ori, g_vel, _ = _streams(seed)
    L = (32.0, 32.0, 32.0)
    semi = np.full((n, 2), 4.0)
    r, q, _ = rsa(g_pos, semi, L, (1, 1, 1))
    if r.shape[0] != n:
        raise RuntimeError("config1: random sequential addition ran out of trials")
    q = random_quaternions(g_ori, n)
    v = g_vel.normal(size=(n, 3))
    w = g_vel.normal(size=(n, 3))
    return Workload("spheres36_R4_L32_phi0.29", r, q, semi, v, w, L, (1, 1, 1),
                    meta=dict(phi=n * 4.0 / 3.0 * np.pi * 64.0 / 32.0 ** 3))


def config2(seed: int = 0, n: int = 4096, phi: float = 0.3) -> Workload:
    """Prolate spheroids, semi-axes (8,4,4), uniform orientations, random
    sequential addition to the volume fraction in a periodic cube;
    simple-shear velocities."""
    g_pos, _, g_vel, _ = _streams(seed)
    semi = np.tile(np.array([8.0, 4.0]), (n, 1))
    vol = n * 4.0 / 3.0 * np.pi * 8.0 * 4.0 * 4.0
    Lx = (vol / phi) ** (1.0 / 3.0)
    L = (Lx, Lx, Lx)
    r, q, trials = rsa(g_pos, semi, L, (1, 1, 1))
    if r.shape[0] != n:
        raise RuntimeError("config2: random sequential addition ran out of trials")
    v, w = shear_velocities(g_vel, r)
    return Workload(f"prolates{n}_8x4x4_phi{phi}", r, q, semi, v, w, L,
                    (1, 1, 1), meta=dict(phi=phi, rsa_trials=trials))


def sheared(seed: int = 0, n: int = 4096, phi: float = 0.3, offset_frac: float = 0.37,
            polydisperse: bool = False) -> Workload:
    """A periodic cube under simple shear with Lees-Edwards images (the
    paper's sheared periodic systems, Sec. IV.C): the image one box up in z
    is offset by offset_frac L in x (accumulated strain) and moves with
    gamma_dot L in x.  Prolates (8,4,4), or with polydisperse=True aspect
    ratios log-uniform in [1/3, 3] and R_perp in [3, 8]; placed by random
    sequential addition with the same images; velocities follow the shear
    field plus noise."""
    g_pos, g_shape, g_vel, _ = _streams(seed + 7)
    if polydisperse:
        semi = polydisperse_semi(g_shape, n, 1.0 / 3.0, 3.0, 3.0, 8.0)
        semi = semi[np.argsort(-semi.max(axis=1), kind="stable")]
    else:
        semi = np.tile(np.array([8.0, 4.0]), (n, 1))
    vol = float(np.sum(4.0 / 3.0 * np.pi * semi[:, 0] * semi[:, 1] ** 2))
    Lx = (vol / phi) ** (1.0 / 3.0)
    L = (Lx, Lx, Lx)
    off = offset_frac * Lx
    r, q, trials = rsa(g_pos, semi, L, (1, 1, 1), le_offset=off)
    if r.shape[0] != n:
        raise RuntimeError("sheared: random sequential addition ran out of trials")
    v, w = shear_velocities(g_vel, r)
    gd = 1e-3
    kind = "polydisperse" if polydisperse else "prolates"
    return Workload(f"sheared_{kind}{n}_phi{phi}_le{offset_frac}", r, q, semi, v, w, L,
                    (1, 1, 1), meta=dict(phi=phi, rsa_trials=trials),
                    lees_edwards=(off, gd * Lx))


def lattice_box(seed: int = 0, n: int = 2347, L: int = 128, semi=(4.0, 4.0)) -> Workload:
    """Particles on the lattice of a periodic cube of integer edge L (the
    link-wise laws need lattice images): the paper's many-particle
    benchmarks use spheres of radius 4 in 128^3 (n = 2347 is volume fraction
    0.3).  semi = (R_par, R_perp) of every particle; random sequential
    addition; simple-shear velocities."""
    g_pos, _, g_vel, _ = _streams(seed + 11)
    sm = np.tile(np.array(semi, dtype=np.float64), (n, 1))
    Lb = (float(L), float(L), float(L))
    r, q, trials = rsa(g_pos, sm, Lb, (1, 1, 1))
    if r.shape[0] != n:
        raise RuntimeError("lattice_box: random sequential addition ran out of trials")
    v, w = shear_velocities(g_vel, r)
    phi = n * 4.0 / 3.0 * np.pi * semi[0] * semi[1] ** 2 / float(L) ** 3
    return Workload(f"lattice{n}_L{L}_{semi[0]:g}x{semi[1]:g}_phi{phi:.2f}", r, q, sm, v, w, Lb,
                    (1, 1, 1), meta=dict(phi=phi, rsa_trials=trials))


def polydisperse_semi(rng: np.random.Generator, n: int, lam_lo: float,
                      lam_hi: float, rperp_lo: float, rperp_hi: float):
    lam = np.exp(rng.uniform(np.log(lam_lo), np.log(lam_hi), size=n))
    rperp = rng.uniform(rperp_lo, rperp_hi, size=n)
    return np.stack([lam * rperp, rperp], axis=1)


def config3(seed: int = 0, n: int = 65536, phi: float = 0.4,
            max_trials: int | None = None) -> Workload:
    """Polydisperse spheroids (aspect ratio log-uniform in [1/3,3],
    equatorial semi-axis uniform in [3,8]) between two walls z=0, z=L,
    periodic in x and y, shear velocities (walls co-moving with the shear
    field).  Placed by random sequential addition, largest first, which
    lets the small particles fill the voids of the large ones."""
    g_pos, g_shape, g_vel, _ = _streams(seed)
    semi = polydisperse_semi(g_shape, n, 1.0 / 3.0, 3.0, 3.0, 8.0)
    vol = float(np.sum(4.0 / 3.0 * np.pi * semi[:, 0] * semi[:, 1] ** 2))
    Lx = (vol / phi) ** (1.0 / 3.0)
    L = (Lx, Lx, Lx)
    order = np.argsort(-semi.max(axis=1), kind="stable")
    semi = semi[order]
    r, q, trials = rsa(g_pos, semi, L, (1, 1, 0),
                       max_trials=max_trials or 200 * n)
    m = r.shape[0]
    semi = semi[:m]
    v, w = shear_velocities(g_vel, r)
    gd = 1e-3
    return Workload(f"polydisperse{n}_walls_phi{phi}", r, q, semi, v, w, L,
                    (1, 1, 0), n_walls=2,
                    wall_vel=((0.0, 0.0, 0.0), (gd * Lx, 0.0, 0.0)),
                    meta=dict(phi_target=phi,
                              phi=float(np.sum(4.0 / 3.0 * np.pi * semi[:, 0]
                                               * semi[:, 1] ** 2)) / Lx ** 3,
                              rsa_trials=trials, placed=m))


# Growth schedule of config5 (Sec. IV.C's packing generator, run on the GPU by
# the library's growth stage, lub_grow): (scale0, scale1, steps, h_c, eps_ref)
# per call; the contact stiffness is eps_ref scale0^3, so that accelerations
# (force over a mass that scales with the volume) do not depend on the size.
# Five ramps from 30 % to the final size with a contact range of 0.3, a ramp
# to 103 % with a range of 0.05, a relaxation there, then the size is reset:
# the overshoot leaves a minimum separation (min gap ~0.15 lattice units).
CONFIG5_GROWTH = [(0.3, 0.45, 2000, 0.3, 1000.0), (0.45, 0.6, 2000, 0.3, 1000.0),
                  (0.6, 0.75, 2000, 0.3, 1000.0), (0.75, 0.9, 2000, 0.3, 1000.0),
                  (0.9, 1.0, 2000, 0.3, 1000.0), (1.0, 1.03, 2000, 0.05, 1000.0),
                  (1.03, 1.03, 1000, 0.05, 1000.0)]


def grow_suspension(r, q, semi, L, periodic, n_walls, stages, device="cuda:0",
                    dt=0.2, damping=1.0):
    """Growth stage of the packing generator on the GPU (the library's
    lub_grow, contact repulsion only, damped velocities): particles placed at
    scale stages[0][0] grow through the stages; returns the final (r, q)."""
    import torch
    from . import lub as L_
    smax = max(max(s0, s1) for s0, s1, *_ in stages)
    params = dict(mu=MU, delta_n=DELTA_N, delta_t=DELTA_T, delta_r=DELTA_R, h_c=H_C,
                  eps_c=EPS_C)
    lb = L_.Lub(L, periodic, params, smax * float(semi.max()), n_walls=n_walls,
                device=int(str(device).split(":")[-1]) if ":" in str(device) else 0)
    z = np.zeros_like(r)
    dev = [torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).to(device)
           for x in (r, q, semi, z, z)]
    for s0, s1, steps, hc, eps in stages:
        lb.grow(*dev, n_steps=steps, scale0=s0, scale1=s1, dt=dt, density=1.0,
                damping=damping, h_c=hc, eps_c=eps * s0 ** 3)
    torch.cuda.synchronize()
    lb.close()
    return dev[0].cpu().numpy(), dev[1].cpu().numpy()


def _cache_dir():
    return os.environ.get("LUB_WORKLOAD_CACHE",
                          os.path.join(os.environ.get("TMPDIR", "/tmp"), "lub_workloads"))


def config5(seed: int = 0, n: int = 1 << 20, side: float = 2048.0, phi: float = 0.5,
            device: str = "cuda:0", stages=None, cache: bool = True) -> Workload:
    """Full-scale suspension: n spheroids (default 1,048,576) with aspect
    ratio log-uniform in [1/4, 4] and equatorial semi-axis uniform in [4, 8]
    at volume fraction phi in a side x side x L box (L = 680 at the defaults),
    periodic in x and y, walls at z = 0 and z = L, shear velocities (walls
    co-moving with the shear field).

    Placed with the paper's growth method (Sec. IV.C): random sequential
    addition at 30 % of the linear size (volume fraction 0.0135), then the
    growth stage on the GPU (lub_grow: contact repulsion only, damped
    motion) to 103 % of the size and a reset to the true size.  Needs the
    GPU; the result is cached in $LUB_WORKLOAD_CACHE (default
    $TMPDIR/lub_workloads) keyed by the arguments and the library build."""
    import hashlib
    stages = stages or CONFIG5_GROWTH
    g_pos, g_shape, g_vel, _ = _streams(seed)
    semi = polydisperse_semi(g_shape, n, 0.25, 4.0, 4.0, 8.0)
    vol = float(np.sum(4.0 / 3.0 * np.pi * semi[:, 0] * semi[:, 1] ** 2))
    Lz = vol / (phi * side * side)
    L = (side, side, Lz)
    key = hashlib.sha256(repr((seed, n, side, phi, stages)).encode())
    from . import lub as L_
    with open(L_.LIB_PATH, "rb") as fh:
        key.update(fh.read())
    path = os.path.join(_cache_dir(), f"config5_{key.hexdigest()[:24]}.npz")
    meta = dict(phi=phi, growth_stages=[list(s) for s in stages])
    if cache and os.path.exists(path):
        z = np.load(path)
        r, q = z["r"], z["q"]
        meta.update(rsa_trials=int(z["trials"]), generate_s=0.0, cached=True)
    else:
        import time
        t0 = time.perf_counter()
        r0, q0, trials = rsa(g_pos, semi * stages[0][0], L, (1, 1, 0), max_trials=50 * n)
        if r0.shape[0] != n:
            raise RuntimeError("config5: random sequential addition ran out of trials")
        t1 = time.perf_counter()
        r, q = grow_suspension(r0, q0, semi, L, (1, 1, 0), 2, stages, device)
        t2 = time.perf_counter()
        meta.update(rsa_trials=trials, rsa_s=t1 - t0, grow_s=t2 - t1, generate_s=t2 - t0,
                    cached=False)
        if cache:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = path + f".tmp{os.getpid()}.npz"
            np.savez(tmp, r=r, q=q, trials=trials)
            os.replace(tmp, path)
    v, w = shear_velocities(g_vel, r)
    gd = 1e-3
    return Workload(f"fullscale{n}_walls_phi{phi}_grown", r, q, semi, v, w, L,
                    (1, 1, 0), n_walls=2,
                    wall_vel=((0.0, 0.0, 0.0), (gd * Lz, 0.0, 0.0)), meta=meta)


def config4_pair_inputs(seed: int, m: int, lam=(1.0 / 3.0, 3.0), rperp=(3.0, 8.0),
                        gap=(1e-4, 1.0)) -> dict:
    """Isolated pairs for the learned Newton seed: both shapes from the
    polydisperse law of config3 (aspect ratio log-uniform in [1/3, 3],
    R_perp uniform in [3, 8]), independent uniform orientations, the
    direction u of the centre offset uniform on the sphere, and a target gap
    g a with g log-uniform in [1e-4, 1] and a the smallest semi-axis of the
    pair.  The centre separation along u that gives that gap is found on the
    oracle's gap (test infrastructure); only the draws are made here."""
    g_shape, g_ori, g_dir, g_gap = _streams(seed)
    semi_i = polydisperse_semi(g_shape, m, lam[0], lam[1], rperp[0], rperp[1])
    semi_j = polydisperse_semi(g_shape, m, lam[0], lam[1], rperp[0], rperp[1])
    q_i = random_quaternions(g_ori, m)
    q_j = random_quaternions(g_ori, m)
    u = g_dir.normal(size=(m, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    a = np.minimum(semi_i.min(axis=1), semi_j.min(axis=1))
    target = a * np.exp(g_gap.uniform(np.log(gap[0]), np.log(gap[1]), size=m))
    return dict(q_i=q_i, q_j=q_j, semi_i=semi_i, semi_j=semi_j, u=u, target=target)


def pair_lattice(q_i, semi_i, q_j, semi_j, d, spacing: float | None = None,
                 name: str = "pairs") -> Workload:
    """Isolated pairs as one system, so that the library evaluates them
    with its ordinary call: pair k's particle i sits on site k of a cubic
    lattice and its particle j at that site + d[k]; the spacing keeps every
    particle of one pair beyond the pruning bound of every particle of
    another.  Particle 2k is i, 2k + 1 is j of pair k; no walls, no periodic
    axes; zero velocities; h_c = eps_c = 0."""
    m = d.shape[0]
    rmax = max(float(semi_i.max()), float(semi_j.max()))
    reach = float(np.linalg.norm(d, axis=1).max()) + 2.0 * rmax
    spacing = spacing or 2.0 * reach + 2.0
    side = int(np.ceil(m ** (1.0 / 3.0)))
    k = np.arange(m)
    sites = spacing * (np.stack([k % side, (k // side) % side, k // (side * side)], 1) + 0.5)
    r = np.empty((2 * m, 3))
    r[0::2] = sites
    r[1::2] = sites + d
    q = np.empty((2 * m, 4))
    q[0::2] = q_i
    q[1::2] = q_j
    semi = np.empty((2 * m, 2))
    semi[0::2] = semi_i
    semi[1::2] = semi_j
    L = side * spacing + spacing
    z = np.zeros((2 * m, 3))
    return Workload(name, r, q, semi, z, z.copy(), (L, L, L), (0, 0, 0),
                    params=dict(mu=MU, delta_n=DELTA_N, delta_t=DELTA_T, delta_r=DELTA_R,
                                h_c=0.0, eps_c=0.0),
                    meta=dict(pairs=m, spacing=spacing))
