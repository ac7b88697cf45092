"""Training pairs and input features of the learned Newton seed.

The seed network maps 10 features of a pair of spheroids to 4 surface
parameters (p, q on each particle, Eq. lub:spheroid) of the points of
closest approach.  Everything is expressed in *canonical pair frames*,
which remove the symmetries of the problem so the outputs never wrap:

  frame of i: z = symmetry axis of i, signed so that j's centre lies on the
              z >= 0 side; x = the component of d = r_j - r_i normal to z
              (any normal if d is along the axis); y = z x x.
  frame of j: the same with the roles swapped (d -> -d).

Features (10): d in frame i divided by R_perp,i (3; the y component is 0
by construction), the rotation from frame i to frame j as a unit
quaternion with w >= 0 (4), R_par,i/R_perp,i, R_par,j/R_perp,i,
R_perp,j/R_perp,i (3).
Targets: the closest points as body-frame surface points of each particle
(3 + 3, divided by R_perp,i); the loss is the squared distance between the
surface points the predicted (p, q) give and the targets, which is periodic
in q and insensitive at the poles.

Training pairs are constructed with known closest points: for two convex
bodies, the support points of i along a unit n and of j along -n, placed a
distance h > 0 apart along n, are the unique closest points and h the gap.
Shapes follow the polydisperse suspension (aspect ratio log-uniform in
[1/3, 3], R_perp uniform in [3, 8]), orientations and n uniform, gap
g * a with g log-uniform in [1e-4, 1] and a the smallest semi-axis.
"""
from __future__ import annotations

import numpy as np

from . import workloads as W

N_IN, N_HID, N_OUT = 10, 128, 4


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _perp(z):
    """A unit vector normal to each row of z."""
    a = np.abs(z)
    e = np.zeros_like(z)
    idx = np.argmin(a, axis=1)
    e[np.arange(z.shape[0]), idx] = 1.0
    return _unit(np.cross(z, e))


def canonical_frame(axis, d):
    """Rows x, y, z of the canonical frame (m,3,3) for symmetry axes
    `axis` (m,3, unit) and centre offsets `d` (m,3) towards the partner."""
    z = axis * np.where(np.sum(axis * d, axis=1) < 0, -1.0, 1.0)[:, None]
    x = d - np.sum(d * z, axis=1)[:, None] * z
    nx = np.linalg.norm(x, axis=1)
    small = nx <= 1e-12 * np.maximum(np.linalg.norm(d, axis=1), 1e-300)
    x /= np.where(small, 1.0, nx)[:, None]
    if small.any():
        x[small] = _perp(z[small])
    y = np.cross(z, x)
    return np.stack([x, y, z], axis=1)


def matrix_to_quat(R):
    """Unit quaternions (w,x,y,z), w >= 0, of rotation matrices (m,3,3)."""
    m = R.shape[0]
    q = np.zeros((m, 4))
    tr = R[:, 0, 0] + R[:, 1, 1] + R[:, 2, 2]
    q[:, 0] = np.sqrt(np.maximum(0.0, 1 + tr)) / 2
    q[:, 1] = np.sqrt(np.maximum(0.0, 1 + R[:, 0, 0] - R[:, 1, 1] - R[:, 2, 2])) / 2
    q[:, 2] = np.sqrt(np.maximum(0.0, 1 - R[:, 0, 0] + R[:, 1, 1] - R[:, 2, 2])) / 2
    q[:, 3] = np.sqrt(np.maximum(0.0, 1 - R[:, 0, 0] - R[:, 1, 1] + R[:, 2, 2])) / 2
    q[:, 1] = np.copysign(q[:, 1], R[:, 2, 1] - R[:, 1, 2])
    q[:, 2] = np.copysign(q[:, 2], R[:, 0, 2] - R[:, 2, 0])
    q[:, 3] = np.copysign(q[:, 3], R[:, 1, 0] - R[:, 0, 1])
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def features(d, axis_i, semi_i, axis_j, semi_j):
    """The 10 features (m,10) and the two canonical frames."""
    Fi = canonical_frame(axis_i, d)
    Fj = canonical_frame(axis_j, -d)
    rp = semi_i[:, 1]
    dl = np.sum(Fi * d[:, None, :], axis=2) / rp[:, None]
    Rrel = np.matmul(Fi, np.transpose(Fj, (0, 2, 1)))  # columns: frame-j axes in frame i
    q = matrix_to_quat(Rrel)
    X = np.concatenate([dl, q, np.stack([semi_i[:, 0] / rp, semi_j[:, 0] / rp,
                                         semi_j[:, 1] / rp], axis=1)], axis=1)
    return X, Fi, Fj


def surface_point(p, q, semi):
    """Eq. lub:spheroid in the (canonical) body frame."""
    return np.stack([semi[:, 1] * np.cos(p) * np.cos(q),
                     semi[:, 1] * np.cos(p) * np.sin(q),
                     semi[:, 0] * np.sin(p)], axis=1)


def support_offsets(M, n):
    """M n / sqrt(n.M n) for each row: the point of the body (centre at 0)
    whose outward normal is n."""
    Mn = np.sum(M * n[:, None, :], axis=2)
    return Mn / np.sqrt(np.sum(n * Mn, axis=1))[:, None]


def _support_offsets_axis(axis, semi, n):
    """The point of a spheroid (centre at 0, symmetry axis `axis`) whose
    outward normal is the unit n: M n / sqrt(n.M n) with M = R_perp^2 I +
    (R_par^2 - R_perp^2) a a^T."""
    p2 = semi[:, 1] ** 2
    dd = semi[:, 0] ** 2 - p2
    an = np.sum(axis * n, axis=1)
    Mn = p2[:, None] * n + (dd * an)[:, None] * axis
    return Mn / np.sqrt(p2 + dd * an * an)[:, None]


def _sample_chunk(ss, m, lam, rperp, gap):
    g_shape, g_ori, g_dir, g_gap = [np.random.default_rng(s) for s in ss.spawn(4)]
    semi_i = W.polydisperse_semi(g_shape, m, lam[0], lam[1], rperp[0], rperp[1])
    semi_j = W.polydisperse_semi(g_shape, m, lam[0], lam[1], rperp[0], rperp[1])
    q_i = W.random_quaternions(g_ori, m)
    q_j = W.random_quaternions(g_ori, m)
    n = _unit(g_dir.normal(size=(m, 3)))
    a = np.minimum(semi_i.min(axis=1), semi_j.min(axis=1))
    h = a * np.exp(g_gap.uniform(np.log(gap[0]), np.log(gap[1]), size=m))
    axis_i = W.symmetry_axes(q_i)
    axis_j = W.symmetry_axes(q_j)
    yi = _support_offsets_axis(axis_i, semi_i, n)     # y_i - r_i
    yj = _support_offsets_axis(axis_j, semi_j, -n)    # y_j - r_j
    d = yi + h[:, None] * n - yj
    X, Fi, Fj = features(d, axis_i, semi_i, axis_j, semi_j)
    rp = semi_i[:, 1][:, None]
    T = np.concatenate([np.sum(Fi * yi[:, None, :], axis=2) / rp,
                        np.sum(Fj * yj[:, None, :], axis=2) / rp], axis=1)
    return dict(q_i=q_i, q_j=q_j, semi_i=semi_i, semi_j=semi_j, d=d, n=n, h=h,
                yi=yi, yj=yj, X=X.astype(np.float32), T=T.astype(np.float32),
                axis_i=axis_i, axis_j=axis_j)


def sample_pairs(seed: int, m: int, lam=(1.0 / 3.0, 3.0), rperp=(3.0, 8.0),
                 gap=(1e-4, 1.0), chunk: int = 1 << 17, threads: int = 8):
    """m constructed pairs: dict with orientations q_i, q_j, semi-axes,
    centre offset d, gap h, closest points (relative to each centre), the
    features X (m,10) and targets T (m,6).  Generated in chunks with their
    own child seeds (the result does not depend on the thread count)."""
    nch = max(1, (m + chunk - 1) // chunk)
    seqs = np.random.SeedSequence(seed).spawn(nch)
    sizes = [min(chunk, m - k * chunk) for k in range(nch)]
    if nch == 1:
        return _sample_chunk(seqs[0], m, lam, rperp, gap)
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(lambda k: _sample_chunk(seqs[k], sizes[k], lam, rperp, gap),
                            range(nch)))
    return {key: np.concatenate([p[key] for p in parts]) for key in parts[0]}


def seed_normal(Y, semi_i, semi_j, Fi, Fj):
    """Seed of the common normal (world frame, from i to j) implied by
    predicted surface parameters Y = (p_i, q_i, p_j, q_j): the outward
    normal of i at its predicted point and minus that of j, averaged."""
    def normal(p, q, semi, F):
        nb = np.stack([np.cos(p) * np.cos(q) / semi[:, 1],
                       np.cos(p) * np.sin(q) / semi[:, 1],
                       np.sin(p) / semi[:, 0]], axis=1)
        return _unit(np.einsum("mji,mj->mi", F, nb))
    ni = normal(Y[:, 0], Y[:, 1], semi_i, Fi)
    nj = normal(Y[:, 2], Y[:, 3], semi_j, Fj)
    return _unit(ni - nj)


def labelled_features(P) -> dict:
    """Features X (m,10) and targets T (m,6) of pairs labelled elsewhere (the
    oracle's closest points): P holds q_i, q_j, semi_i, semi_j, the centre
    offset d (or u and the separation s) and the closest points yi, yj
    relative to each centre."""
    d = P["d"] if "d" in P else P["s"][:, None] * P["u"]
    axis_i = W.symmetry_axes(P["q_i"])
    axis_j = W.symmetry_axes(P["q_j"])
    X, Fi, Fj = features(d, axis_i, P["semi_i"], axis_j, P["semi_j"])
    rp = P["semi_i"][:, 1][:, None]
    T = np.concatenate([np.sum(Fi * P["yi"][:, None, :], axis=2) / rp,
                        np.sum(Fj * P["yj"][:, None, :], axis=2) / rp], axis=1)
    return dict(X=X.astype(np.float32), T=T.astype(np.float32), d=d)
