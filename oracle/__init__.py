"""FP64 CPU oracle of the lubrication correction for spheroids.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU
library never imports, links or calls it; the two share no code.

The arithmetic lives in ``lubref.c`` (plain C, IEEE double, no FP
contraction); this module only marshals numpy arrays through ctypes and
builds the shared object with gcc when it is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liblubref.so")

REFP_ACTIVE, REFP_INACTIVE, REFP_UNRESOLVED, REFP_FAILED = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile ``lubref.c`` into ``liblubref.so`` with gcc (OpenMP)."""
    if force or not os.path.exists(_SO):
        src = os.path.join(_HERE, "lubref.c")
        tmp = _SO + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-fPIC", "-shared", src, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _SO)
    return _SO


MODEL_FULL, MODEL_NORMAL, MODEL_LADD, MODEL_CONTACT = 0, 1, 2, 3
MODEL_LINK, MODEL_LINK_NAVG = 4, 5


class Params(C.Structure):
    _fields_ = [("mu", C.c_double), ("delta_n", C.c_double),
                ("delta_t", C.c_double), ("delta_r", C.c_double),
                ("h_c", C.c_double), ("eps_c", C.c_double),
                ("model", C.c_int32), ("reserved", C.c_int32),
                ("q_bar", C.c_double)]


class Domain(C.Structure):
    _fields_ = [("L", C.c_double * 3), ("periodic", C.c_int32 * 3),
                ("n_walls", C.c_int32), ("wall_vel", (C.c_double * 3) * 2),
                ("lees_edwards", C.c_int32), ("reserved", C.c_int32),
                ("le_offset", C.c_double), ("le_velocity", C.c_double)]


class PairResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("fallback", C.c_int32),
                ("iters_lh", C.c_int32), ("iters_polish", C.c_int32),
                ("h", C.c_double), ("n", C.c_double * 3),
                ("yi", C.c_double * 3), ("yj", C.c_double * 3),
                ("certificate", C.c_double), ("e", (C.c_double * 3) * 3),
                ("S1", C.c_double), ("S2", C.c_double),
                ("invS1p", C.c_double), ("invS2p", C.c_double),
                ("G", C.c_double * 4), ("Gp", C.c_double * 4),
                ("cphi", C.c_double), ("sphi", C.c_double),
                ("lam1", C.c_double), ("lam2", C.c_double),
                ("cchi", C.c_double), ("schi", C.c_double),
                ("kappa", C.c_double * 4), ("C", (C.c_double * 6) * 6),
                ("Kt", (C.c_double * 6) * 6), ("Fbar", C.c_double * 6),
                ("F", C.c_double * 3), ("Ti", C.c_double * 3),
                ("Tj", C.c_double * 3), ("links", C.c_int32), ("pad_", C.c_int32)]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            val = getattr(self, name)
            if isinstance(val, C.Array):
                val = np.ctypeslib.as_array(val).copy()
            out[name] = val
        return out


class Stats(C.Structure):
    _fields_ = [("candidates", C.c_int64), ("wall_candidates", C.c_int64),
                ("active", C.c_int64), ("overlaps", C.c_int64),
                ("unresolved", C.c_int64), ("failed", C.c_int64),
                ("fallbacks", C.c_int64), ("iters_lh_total", C.c_int64),
                ("iters_lh_max", C.c_int64), ("iters_polish_total", C.c_int64),
                ("threads", C.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None
_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_I64 = C.POINTER(C.c_int64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        L = C.CDLL(_SO)
        L.ref_quat_to_matrix.argtypes = [_D, _D]
        L.ref_centre_test.argtypes = [_D, _D, C.c_double, C.c_double,
                                      C.c_double, C.POINTER(Domain)]
        L.ref_candidates.argtypes = [C.c_int64, _D, _D, C.POINTER(Domain),
                                     C.POINTER(Params), C.c_int64, _I32, _I64,
                                     C.c_int64, _I32, _I64]
        L.ref_pair_eval.argtypes = [_D, _D, _D, _D, _D, _D, _D, _D, _D,
                                    C.POINTER(Params), C.POINTER(PairResult)]
        L.ref_wall_eval.argtypes = [_D, _D, _D, _D, _D, C.c_int,
                                    C.POINTER(Domain), C.POINTER(Params),
                                    C.POINTER(PairResult)]
        L.ref_closest_points.argtypes = [_D, _D, _D, _D, _D,
                                         C.POINTER(PairResult)]
        L.ref_K_coeffs.argtypes = [C.c_double, C.c_double, C.c_double,
                                   C.c_double, _D, _D, C.c_double, C.c_double,
                                   _D, _D]
        L.ref_K_coeffs.restype = None
        L.ref_compute.argtypes = [C.c_int64, _D, _D, _D, _D, _D,
                                  C.POINTER(Domain), C.POINTER(Params), C.c_int,
                                  _D, _D, C.POINTER(Stats)]
        L.ref_compute_subset.argtypes = [C.c_int64, _D, _D, _D, _D, _D,
                                         C.POINTER(Domain), C.POINTER(Params),
                                         C.c_int64, _I64, C.c_int, _D, _D,
                                         C.POINTER(Stats)]
        L.ref_partners_subset.argtypes = [C.c_int64, _D, _D, C.POINTER(Domain),
                                          C.POINTER(Params), C.c_int64, _I64,
                                          C.c_int64, _I32, _I64]
        L.ref_eval_pairs.argtypes = [C.c_int64, _D, _D, _D, _D, _D,
                                     C.POINTER(Domain), C.POINTER(Params),
                                     C.c_int64, _I32, C.c_int, _D, _D, _D, _D,
                                     _I32, _I32]
        L.ref_link_eval.argtypes = [_D] * 10 + [C.POINTER(Params), C.POINTER(PairResult)]
        L.ref_eval_pairs_detail.argtypes = [C.c_int64, _D, _D, _D, _D, _D,
                                            C.POINTER(Domain), C.POINTER(Params),
                                            C.c_int64, _I32, C.c_int, _D, _D, _D, _D,
                                            _I32, _D, _D, _D, _D, _D, _I32, _I32]
        L.ref_place_pairs.argtypes = [C.c_int64, _D, _D, _D, _D, _D, _D, C.c_int, _D, _D,
                                      _D, _D, _D, _I32, _I32]
        _lib = L
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t=_D):
    return a.ctypes.data_as(t)


def make_params(mu=1.0 / 6.0, delta_n=2.0 / 3.0, delta_t=0.5, delta_r=0.25,
                h_c=0.0, eps_c=0.0, model=MODEL_FULL, q_bar=0.6) -> Params:
    return Params(mu, delta_n, delta_t, delta_r, h_c, eps_c, int(model), 0, float(q_bar))


def make_domain(L=(1e9, 1e9, 1e9), periodic=(0, 0, 0), n_walls=0,
                wall_vel=((0.0, 0.0, 0.0), (0.0, 0.0, 0.0)), lees_edwards=None) -> Domain:
    """lees_edwards: None, or (offset, velocity) of the image one box up in z
    (Lees-Edwards images of a sheared periodic box)."""
    d = Domain()
    for k in range(3):
        d.L[k] = float(L[k])
        d.periodic[k] = int(periodic[k])
    d.n_walls = int(n_walls)
    for s in range(2):
        for k in range(3):
            d.wall_vel[s][k] = float(wall_vel[s][k])
    if lees_edwards is not None:
        d.lees_edwards = 1
        d.le_offset = float(lees_edwards[0])
        d.le_velocity = float(lees_edwards[1])
    return d


def quat_to_matrix(q) -> np.ndarray:
    q = _d(q)
    Q = np.zeros(9)
    lib().ref_quat_to_matrix(_p(q), _p(Q))
    return Q.reshape(3, 3)


def pair_eval(d, qi, semii, vi, wi, qj, semij, vj, wj, params: Params) -> dict:
    o = PairResult()
    a = [_d(x) for x in (d, qi, semii, vi, wi, qj, semij, vj, wj)]
    lib().ref_pair_eval(*[_p(x) for x in a], C.byref(params), C.byref(o))
    return o.as_dict()


def link_eval(ri, d, qi, semii, vi, wi, qj, semij, vj, wj, params: Params) -> dict:
    """Link-wise laws for one pair: ri absolute centre of i, d offset of j."""
    o = PairResult()
    a = [_d(x) for x in (ri, d, qi, semii, vi, wi, qj, semij, vj, wj)]
    lib().ref_link_eval(*[_p(x) for x in a], C.byref(params), C.byref(o))
    return o.as_dict()


def wall_eval(ri, qi, semii, vi, wi, side, domain: Domain, params: Params) -> dict:
    o = PairResult()
    a = [_d(x) for x in (ri, qi, semii, vi, wi)]
    lib().ref_wall_eval(*[_p(x) for x in a], int(side), C.byref(domain),
                        C.byref(params), C.byref(o))
    return o.as_dict()


def closest_points(d, qi, semii, qj, semij) -> dict:
    o = PairResult()
    a = [_d(x) for x in (d, qi, semii, qj, semij)]
    lib().ref_closest_points(*[_p(x) for x in a], C.byref(o))
    return o.as_dict()


def K_coeffs(S1, S2, invS1p, invS2p, G, Gp, cphi, sphi):
    Cm = np.zeros(36)
    aux = np.zeros(8)
    G = _d(G)
    Gp = _d(Gp)
    lib().ref_K_coeffs(float(S1), float(S2), float(invS1p), float(invS2p),
                       _p(G), _p(Gp), float(cphi), float(sphi), _p(Cm), _p(aux))
    return Cm.reshape(6, 6), aux


def centre_test(ri, rj, rmax_i, rmax_j, dmax, domain: Domain) -> bool:
    return bool(lib().ref_centre_test(_p(_d(ri)), _p(_d(rj)), float(rmax_i),
                                      float(rmax_j), float(dmax),
                                      C.byref(domain)))


def candidates(r, semi, domain: Domain, params: Params):
    """Brute-force candidate lists: (pairs (P,2) int32 sorted by (i,j),
    wall pairs (W,2) int32 (particle, side))."""
    r = _d(r)
    semi = _d(semi)
    n = r.shape[0]
    npairs = C.c_int64(0)
    nwall = C.c_int64(0)
    L = lib()
    L.ref_candidates(n, _p(r), _p(semi), C.byref(domain), C.byref(params), 0,
                     None, C.byref(npairs), 0, None, C.byref(nwall))
    ij = np.zeros((max(npairs.value, 1), 2), dtype=np.int32)
    wall = np.zeros((max(nwall.value, 1), 2), dtype=np.int32)
    rc = L.ref_candidates(n, _p(r), _p(semi), C.byref(domain), C.byref(params),
                          npairs.value, _p(ij, _I32), C.byref(npairs),
                          nwall.value, _p(wall, _I32), C.byref(nwall))
    assert rc == 0
    return ij[:npairs.value], wall[:nwall.value]


def compute(r, q, semi, v, w, domain: Domain, params: Params, nthreads=0):
    """Per-particle force and torque (n,3) each, plus stats dict."""
    r, q, semi, v, w = (_d(x) for x in (r, q, semi, v, w))
    n = r.shape[0]
    f = np.zeros((n, 3))
    t = np.zeros((n, 3))
    st = Stats()
    rc = lib().ref_compute(n, _p(r), _p(q), _p(semi), _p(v), _p(w),
                           C.byref(domain), C.byref(params), int(nthreads),
                           _p(f), _p(t), C.byref(st))
    if rc != 0:
        raise ValueError(f"ref_compute rejected its inputs (rc={rc})")
    return f, t, st.as_dict()


def compute_subset(r, q, semi, v, w, domain: Domain, params: Params, idx,
                   nthreads=0):
    r, q, semi, v, w = (_d(x) for x in (r, q, semi, v, w))
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    m = idx.shape[0]
    f = np.zeros((m, 3))
    t = np.zeros((m, 3))
    st = Stats()
    rc = lib().ref_compute_subset(r.shape[0], _p(r), _p(q), _p(semi), _p(v),
                                  _p(w), C.byref(domain), C.byref(params), m,
                                  _p(idx, _I64), int(nthreads), _p(f), _p(t),
                                  C.byref(st))
    if rc != 0:
        raise ValueError(f"ref_compute_subset rejected its inputs (rc={rc})")
    return f, t, st.as_dict()


def partners_subset(r, semi, domain: Domain, params: Params, idx, cap=512):
    """Candidate partners of the particles idx (brute force): list of
    sorted int arrays."""
    r, semi = _d(r), _d(semi)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    m = idx.shape[0]
    out = np.full((m, cap), -1, dtype=np.int32)
    cnt = np.zeros(m, dtype=np.int64)
    rc = lib().ref_partners_subset(r.shape[0], _p(r), _p(semi), C.byref(domain),
                                   C.byref(params), m, _p(idx, _I64), cap,
                                   _p(out, _I32), _p(cnt, _I64))
    if rc != 0:
        raise ValueError(f"ref_partners_subset failed (rc={rc})")
    return [out[s, :cnt[s]].copy() for s in range(m)]


def eval_pairs(r, q, semi, v, w, domain: Domain, params: Params, ij,
               nthreads=0, with_links=False):
    """Per-pair (F, Ti, Tj, h, status) for an explicit pair list; j<0 means
    a wall (-1: z=0, -2: z=L).  with_links: also the number of contributing
    links of each pair (link-wise laws)."""
    r, q, semi, v, w = (_d(x) for x in (r, q, semi, v, w))
    ij = np.ascontiguousarray(ij, dtype=np.int32)
    m = ij.shape[0]
    F = np.zeros((m, 3))
    Ti = np.zeros((m, 3))
    Tj = np.zeros((m, 3))
    h = np.zeros(m)
    status = np.zeros(m, dtype=np.int32)
    links = np.zeros(m, dtype=np.int32)
    lib().ref_eval_pairs(r.shape[0], _p(r), _p(q), _p(semi), _p(v), _p(w),
                         C.byref(domain), C.byref(params), m, _p(ij, _I32),
                         int(nthreads), _p(F), _p(Ti), _p(Tj), _p(h),
                         _p(status, _I32), _p(links, _I32))
    if with_links:
        return F, Ti, Tj, h, status, links
    return F, Ti, Tj, h, status


def place_pairs(u, target, qi, semii, qj, semij, nthreads=0) -> dict:
    """Pairs at a prescribed gap: for each row, the centre separation s along
    the unit u at which the oracle gap equals target, and the oracle's
    closest points there (dict of s, h, n, yi, yj, iters_lh, status)."""
    u, target, qi, semii, qj, semij = (_d(x) for x in (u, target, qi, semii, qj, semij))
    m = u.shape[0]
    out = dict(s=np.zeros(m), h=np.zeros(m), n=np.zeros((m, 3)), yi=np.zeros((m, 3)),
               yj=np.zeros((m, 3)), iters_lh=np.zeros(m, dtype=np.int32),
               status=np.zeros(m, dtype=np.int32))
    rc = lib().ref_place_pairs(m, _p(u), _p(target), _p(qi), _p(semii), _p(qj), _p(semij),
                               int(nthreads), _p(out["s"]), _p(out["h"]), _p(out["n"]),
                               _p(out["yi"]), _p(out["yj"]), _p(out["iters_lh"], _I32),
                               _p(out["status"], _I32))
    if rc != 0:
        raise ValueError(f"ref_place_pairs failed (rc={rc})")
    return out


def eval_pairs_detail(r, q, semi, v, w, domain: Domain, params: Params, ij, nthreads=0):
    """eval_pairs with the intermediate results of every pair: dict of F, Ti,
    Tj, h, status, n, yi, yj, e1 (m,3), Kt (m,6,6, without the viscosity),
    iters_lh, iters_polish."""
    r, q, semi, v, w = (_d(x) for x in (r, q, semi, v, w))
    ij = np.ascontiguousarray(ij, dtype=np.int32)
    m = ij.shape[0]
    o = {k: np.zeros((m, 3)) for k in ("F", "Ti", "Tj", "n", "yi", "yj", "e1")}
    o["h"] = np.zeros(m)
    o["Kt"] = np.zeros((m, 6, 6))
    for k in ("status", "iters_lh", "iters_polish"):
        o[k] = np.zeros(m, dtype=np.int32)
    lib().ref_eval_pairs_detail(r.shape[0], _p(r), _p(q), _p(semi), _p(v), _p(w),
                                C.byref(domain), C.byref(params), m, _p(ij, _I32),
                                int(nthreads), _p(o["F"]), _p(o["Ti"]), _p(o["Tj"]),
                                _p(o["h"]), _p(o["status"], _I32), _p(o["n"]), _p(o["yi"]),
                                _p(o["yj"]), _p(o["e1"]), _p(o["Kt"]),
                                _p(o["iters_lh"], _I32), _p(o["iters_polish"], _I32))
    return o
