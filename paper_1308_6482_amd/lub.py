"""Thin ctypes binding of the gfx950 lubrication library (include/lub.h).

Argument marshalling only: every step of the correction runs in the HIP
kernels of ``_lib/liblub.so``.  PyTorch provides device memory and streams.
There is no CPU fallback: if the library is missing or no GPU is present,
the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "liblub.so")

LUB_OK, LUB_EINVAL, LUB_EDOMAIN, LUB_ECAPACITY, LUB_ENOMEM, LUB_EDEVICE = 0, -1, -2, -3, -4, -5
LUB_FP64, LUB_MIXED = 0, 1
LUB_SEED_PLAIN, LUB_SEED_MLP = 0, 1

EXPORTS = ["lub_create", "lub_set_params", "lub_set_domain", "lub_compute",
           "lub_get_stats", "lub_reset_timers", "lub_get_pairs",
           "lub_get_pair_results", "lub_mlp_set_weights", "lub_mlp_get_weights",
           "lub_mlp_init", "lub_mlp_forward", "lub_mlp_grad", "lub_mlp_train",
           "lub_get_domain", "lub_integrate", "lub_advance", "lub_grow",
           "lub_compute_static",
           "lub_mlp_save", "lub_mlp_load", "lub_get_pair_detail",
           "lub_destroy", "lub_strerror"]
LUB_MLP_PARAMS = 34948
LUB_MLP_STATE = 3 * LUB_MLP_PARAMS + 1


class lub_step_t(C.Structure):
    _fields_ = [("dt", C.c_double), ("n_sub", C.c_int32), ("reserved", C.c_int32),
                ("density", C.c_double), ("damping", C.c_double)]


class lub_grow_t(C.Structure):
    _fields_ = [("n_steps", C.c_int32), ("reserved", C.c_int32),
                ("scale0", C.c_double), ("scale1", C.c_double), ("dt", C.c_double),
                ("density", C.c_double), ("damping", C.c_double), ("h_c", C.c_double),
                ("eps_c", C.c_double)]


class lub_params_t(C.Structure):
    _fields_ = [("mu", C.c_double), ("delta_n", C.c_double),
                ("delta_t", C.c_double), ("delta_r", C.c_double),
                ("h_c", C.c_double), ("eps_c", C.c_double),
                ("model", C.c_int32), ("reserved", C.c_int32), ("q_bar", C.c_double)]


class lub_domain_t(C.Structure):
    _fields_ = [("L", C.c_double * 3), ("periodic", C.c_int32 * 3),
                ("n_walls", C.c_int32), ("wall_vel", (C.c_double * 3) * 2),
                ("lees_edwards", C.c_int32), ("reserved", C.c_int32),
                ("le_offset", C.c_double), ("le_velocity", C.c_double)]


class lub_opts_t(C.Structure):
    _fields_ = [("device", C.c_int32), ("precision", C.c_int32),
                ("seed_mode", C.c_int32), ("newton_max_iter", C.c_int32),
                ("rmax_bound", C.c_double), ("sync", C.c_int32),
                ("timing", C.c_int32), ("max_neighbors", C.c_int64),
                ("graph", C.c_int32), ("warm_start", C.c_int32),
                ("reserved", C.c_int32), ("skin", C.c_double),
                ("newton_tol", C.c_double), ("host_pointers", C.c_int32),
                ("record_detail", C.c_int32)]


class lub_stats_t(C.Structure):
    _fields_ = [("n", C.c_int64), ("candidates", C.c_int64),
                ("wall_candidates", C.c_int64), ("evaluated", C.c_int64),
                ("active", C.c_int64), ("overlaps", C.c_int64),
                ("unresolved", C.c_int64), ("unconverged", C.c_int64),
                ("fallbacks", C.c_int64), ("newton_iters", C.c_int64),
                ("newton_max", C.c_int32), ("error", C.c_int32),
                ("iter_hist", C.c_int64 * 32), ("timed_calls", C.c_int64),
                ("stage_ms", C.c_double * 4), ("warm_seeded", C.c_int64),
                ("max_degree", C.c_int64), ("pair_kernel_ms", C.c_double),
                ("list_builds", C.c_int64), ("search_kernel_ms", C.c_double)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_
             if k not in ("iter_hist", "stage_ms")}
        d["iter_hist"] = list(self.iter_hist)
        d["stage_ms"] = list(self.stage_ms)
        return d


class lub_train_cfg_t(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("lr_decay", C.c_float), ("reserved", C.c_int32)]


_lib = None
_P = C.c_void_p
_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_I64 = C.POINTER(C.c_int64)


class LubError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {lib().lub_strerror(code).decode()} ({code})")


def lib():
    """Load liblub.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        L.lub_create.argtypes = [C.POINTER(_P), C.POINTER(lub_domain_t),
                                 C.POINTER(lub_params_t), C.POINTER(lub_opts_t)]
        L.lub_set_params.argtypes = [_P, C.POINTER(lub_params_t)]
        L.lub_set_domain.argtypes = [_P, C.POINTER(lub_domain_t)]
        L.lub_compute.argtypes = [_P, C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P]
        L.lub_get_stats.argtypes = [_P, C.POINTER(lub_stats_t)]
        L.lub_reset_timers.argtypes = [_P]
        L.lub_get_pairs.argtypes = [_P, C.c_int64, _I32, _I64, C.c_int64, _I32, _I64]
        L.lub_get_pair_results.argtypes = [_P, C.c_int64, _I32, _D, _D, _D, _D,
                                           _I32, _I32, _I64]
        _F = C.POINTER(C.c_float)
        L.lub_get_pair_detail.argtypes = [_P, C.c_int64, _D, _D, _D, _D, _D, _I64]
        L.lub_mlp_set_weights.argtypes = [_P, _F, C.c_int64]
        L.lub_mlp_get_weights.argtypes = [_P, _F, C.c_int64]
        L.lub_mlp_init.argtypes = [_P, C.c_uint64]
        L.lub_mlp_save.argtypes = [_P, _F, C.c_int64]
        L.lub_mlp_load.argtypes = [_P, _F, C.c_int64]
        L.lub_mlp_forward.argtypes = [_P, C.c_int64, _P, _P, _P]
        L.lub_mlp_grad.argtypes = [_P, C.c_int64, _P, _P, _F, _F, _P]
        L.lub_mlp_train.argtypes = [_P, C.c_int64, _P, _P, C.POINTER(lub_train_cfg_t),
                                    _F, _P]
        L.lub_get_domain.argtypes = [_P, C.POINTER(lub_domain_t)]
        L.lub_integrate.argtypes = [_P, C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                    C.POINTER(lub_step_t), _P]
        L.lub_advance.argtypes = [_P, C.c_int64, _P, _P, _P, _P, C.c_double, _P]
        L.lub_grow.argtypes = [_P, C.c_int64, _P, _P, _P, _P, _P, C.POINTER(lub_grow_t), _P]
        L.lub_compute_static.argtypes = [C.POINTER(lub_domain_t), C.POINTER(lub_params_t),
                                         C.POINTER(lub_opts_t), C.c_int64, _P, _P, _P, _P,
                                         _P, _P, _P, _P, C.POINTER(lub_stats_t)]
        L.lub_destroy.argtypes = [_P]
        L.lub_destroy.restype = None
        L.lub_strerror.argtypes = [C.c_int]
        L.lub_strerror.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != LUB_OK:
        raise LubError(rc, where)


LUB_MODEL_FULL, LUB_MODEL_NORMAL, LUB_MODEL_LADD, LUB_MODEL_CONTACT = 0, 1, 2, 3
LUB_MODEL_LINK, LUB_MODEL_LINK_NAVG = 4, 5


def make_params(mu, delta_n, delta_t, delta_r, h_c=0.0, eps_c=0.0,
                model=LUB_MODEL_FULL, q_bar=0.6) -> lub_params_t:
    return lub_params_t(mu, delta_n, delta_t, delta_r, h_c, eps_c, int(model), 0,
                        float(q_bar))


def make_domain(L, periodic=(1, 1, 1), n_walls=0,
                wall_vel=((0.0, 0.0, 0.0), (0.0, 0.0, 0.0)),
                lees_edwards=None) -> lub_domain_t:
    """lees_edwards: None, or (offset, velocity) of the image one box up in z."""
    d = lub_domain_t()
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


def make_opts(rmax_bound, precision=LUB_FP64, device=0, seed_mode=LUB_SEED_PLAIN,
              newton_max_iter=0, sync=1, max_neighbors=0, timing=0,
              graph=0, warm_start=0, skin=0.0, newton_tol=0.0,
              host_pointers=0, record_detail=0) -> lub_opts_t:
    return lub_opts_t(device, precision, seed_mode, newton_max_iter,
                      float(rmax_bound), sync, timing, max_neighbors, graph, warm_start, 0,
                      float(skin), float(newton_tol), int(host_pointers), int(record_detail))


# --- the C entry points, same names ------------------------------------------

def lub_create(domain: lub_domain_t, params: lub_params_t, opts: lub_opts_t):
    h = _P()
    _check(lib().lub_create(C.byref(h), C.byref(domain), C.byref(params),
                            C.byref(opts)), "lub_create")
    return h


def lub_set_params(h, params: lub_params_t):
    _check(lib().lub_set_params(h, C.byref(params)), "lub_set_params")


def lub_set_domain(h, domain: lub_domain_t):
    _check(lib().lub_set_domain(h, C.byref(domain)), "lub_set_domain")


def _ptr(t):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("lub_compute takes torch.cuda tensors")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("lub_compute takes contiguous float64 tensors")
    return t.data_ptr()


def lub_compute(h, r, q, semi, v, w, f, t, stream=None, check=True) -> int:
    """r, q, semi, v, w, f, t: contiguous float64 torch.cuda tensors of shape
    (n,3), (n,4), (n,2), (n,3), (n,3), (n,3), (n,3).  f and t are written."""
    import torch
    n = r.shape[0]
    for a, cols in ((r, 3), (q, 4), (semi, 2), (v, 3), (w, 3), (f, 3), (t, 3)):
        if a.shape != (n, cols):
            raise ValueError(f"bad shape {tuple(a.shape)}, expected ({n},{cols})")
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    elif hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    ptrs = [_ptr(x) if n > 0 else 0 for x in (r, q, semi, v, w, f, t)]
    rc = lib().lub_compute(h, n, *ptrs, stream)
    if check:
        _check(rc, "lub_compute")
    return rc


def lub_compute_static(domain: lub_domain_t, params: lub_params_t, opts: lub_opts_t,
                       r, q, semi, v, w, f, t, stream=None, stats=True):
    """The allocation-free evaluation (no handle): same arrays as
    lub_compute.  With stats=True the call waits and returns the statistics
    dict (raising on a device-side error); with stats=False it returns None
    without waiting."""
    n = r.shape[0]
    for a, cols in ((r, 3), (q, 4), (semi, 2), (v, 3), (w, 3), (f, 3), (t, 3)):
        if a.shape != (n, cols):
            raise ValueError(f"bad shape {tuple(a.shape)}, expected ({n},{cols})")
    ptrs = [_ptr(x) if n > 0 else 0 for x in (r, q, semi, v, w, f, t)]
    st = lub_stats_t() if stats else None
    rc = lib().lub_compute_static(C.byref(domain), C.byref(params), C.byref(opts), n, *ptrs,
                                  _stream_handle(stream), C.byref(st) if stats else None)
    _check(rc, "lub_compute_static")
    return st.as_dict() if stats else None


def lub_compute_host(h, r, q, semi, v, w, stream=None):
    """lub_compute on a handle created with host_pointers=1: numpy float64
    arrays in, numpy (f, t) out (the call waits for the results)."""
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (r, q, semi, v, w)]
    n = arrs[0].shape[0]
    for a, cols in zip(arrs, (3, 4, 2, 3, 3)):
        if a.shape != (n, cols):
            raise ValueError(f"bad shape {a.shape}, expected ({n},{cols})")
    f = np.zeros((n, 3))
    t = np.zeros((n, 3))
    ptrs = [a.ctypes.data for a in arrs] + [f.ctypes.data, t.ctypes.data]
    _check(lib().lub_compute(h, n, *ptrs, _stream_handle(stream)), "lub_compute")
    return f, t


def _stream_handle(stream):
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return stream


def _state_ptrs(n, r, q, semi, v, w):
    for a, cols in ((r, 3), (q, 4), (semi, 2), (v, 3), (w, 3)):
        if a.shape != (n, cols):
            raise ValueError(f"bad shape {tuple(a.shape)}, expected ({n},{cols})")
    return [_ptr(x) if n > 0 else 0 for x in (r, q, semi, v, w)]


def lub_get_domain(h) -> lub_domain_t:
    d = lub_domain_t()
    _check(lib().lub_get_domain(h, C.byref(d)), "lub_get_domain")
    return d


def lub_integrate(h, r, q, semi, v, w, f, t, dt, n_sub, density=1.0, damping=0.0,
                  f_ext=None, t_ext=None, stream=None):
    """Sub-stepped update: r, q, v, w (float64 torch.cuda tensors) are
    updated in place; f, t receive the last sub-step's correction."""
    n = r.shape[0]
    ptrs = _state_ptrs(n, r, q, semi, v, w)
    for a in (f, t) + tuple(x for x in (f_ext, t_ext) if x is not None):
        if a.shape != (n, 3):
            raise ValueError(f"bad shape {tuple(a.shape)}, expected ({n},3)")
    ext = [_ptr(x) if (x is not None and n > 0) else 0 for x in (f_ext, t_ext)]
    out = [_ptr(x) if n > 0 else 0 for x in (f, t)]
    st = lub_step_t(float(dt), int(n_sub), 0, float(density), float(damping))
    _check(lib().lub_integrate(h, n, *ptrs, *ext, *out, C.byref(st), _stream_handle(stream)),
           "lub_integrate")


def lub_advance(h, r, q, v, w, dt, stream=None):
    """Kinematic advance: r += dt v, q <- normalise(q + dt/2 (0, w) q), in
    place (float64 torch.cuda tensors)."""
    n = r.shape[0]
    for a, cols in ((r, 3), (q, 4), (v, 3), (w, 3)):
        if a.shape != (n, cols):
            raise ValueError(f"bad shape {tuple(a.shape)}, expected ({n},{cols})")
    ptrs = [_ptr(x) if n > 0 else 0 for x in (r, q, v, w)]
    _check(lib().lub_advance(h, n, *ptrs, float(dt), _stream_handle(stream)), "lub_advance")


def lub_grow(h, r, q, semi, v, w, n_steps, scale0, scale1, dt, density=1.0, damping=0.0,
             h_c=0.1, eps_c=100.0, stream=None):
    """Growth stage of the packing generator: r, q, v, w updated in place."""
    n = r.shape[0]
    ptrs = _state_ptrs(n, r, q, semi, v, w)
    cfg = lub_grow_t(int(n_steps), 0, float(scale0), float(scale1), float(dt),
                     float(density), float(damping), float(h_c), float(eps_c))
    _check(lib().lub_grow(h, n, *ptrs, C.byref(cfg), _stream_handle(stream)), "lub_grow")


def lub_get_stats(h) -> dict:
    st = lub_stats_t()
    _check(lib().lub_get_stats(h, C.byref(st)), "lub_get_stats")
    return st.as_dict()


def lub_reset_timers(h):
    _check(lib().lub_reset_timers(h), "lub_reset_timers")


def lub_get_pairs(h):
    """(pairs (P,2) int32 sorted, wall pairs (W,2) int32 (particle, side))."""
    L = lib()
    npairs, nwall = C.c_int64(), C.c_int64()
    rc = L.lub_get_pairs(h, 0, None, C.byref(npairs), 0, None, C.byref(nwall))
    if rc not in (LUB_OK, LUB_ECAPACITY):
        _check(rc, "lub_get_pairs")
    ij = np.zeros((max(npairs.value, 1), 2), dtype=np.int32)
    wall = np.zeros((max(nwall.value, 1), 2), dtype=np.int32)
    _check(L.lub_get_pairs(h, npairs.value, ij.ctypes.data_as(_I32), C.byref(npairs),
                           nwall.value, wall.ctypes.data_as(_I32), C.byref(nwall)),
           "lub_get_pairs")
    return ij[:npairs.value], wall[:nwall.value]


def lub_get_pair_results(h) -> dict:
    L = lib()
    m = C.c_int64()
    rc = L.lub_get_pair_results(h, 0, None, None, None, None, None, None, None,
                                C.byref(m))
    if rc not in (LUB_OK, LUB_ECAPACITY):
        _check(rc, "lub_get_pair_results")
    k = m.value
    ij = np.zeros((max(k, 1), 2), dtype=np.int32)
    hg = np.zeros(max(k, 1))
    F = np.zeros((max(k, 1), 3))
    Ti = np.zeros((max(k, 1), 3))
    Tj = np.zeros((max(k, 1), 3))
    st = np.zeros(max(k, 1), dtype=np.int32)
    it = np.zeros(max(k, 1), dtype=np.int32)
    _check(L.lub_get_pair_results(h, k, ij.ctypes.data_as(_I32), hg.ctypes.data_as(_D),
                                  F.ctypes.data_as(_D), Ti.ctypes.data_as(_D),
                                  Tj.ctypes.data_as(_D), st.ctypes.data_as(_I32),
                                  it.ctypes.data_as(_I32), C.byref(m)),
           "lub_get_pair_results")
    return dict(ij=ij[:k], h=hg[:k], F=F[:k], Ti=Ti[:k], Tj=Tj[:k], status=st[:k],
                iters=it[:k])


def lub_get_pair_detail(h) -> dict:
    """Per evaluated pair (order of lub_get_pair_results): n, yi, yj, e1
    (m,3) and Kt (m,16); needs a handle created with record_detail=1."""
    L = lib()
    m = C.c_int64()
    rc = L.lub_get_pair_detail(h, 0, None, None, None, None, None, C.byref(m))
    if rc not in (LUB_OK, LUB_ECAPACITY):
        _check(rc, "lub_get_pair_detail")
    k = max(m.value, 1)
    out = dict(n=np.zeros((k, 3)), yi=np.zeros((k, 3)), yj=np.zeros((k, 3)),
               e1=np.zeros((k, 3)), Kt=np.zeros((k, 16)))
    _check(L.lub_get_pair_detail(h, k, *[out[x].ctypes.data_as(_D)
                                         for x in ("n", "yi", "yj", "e1", "Kt")], C.byref(m)),
           "lub_get_pair_detail")
    return {x: v[:m.value] for x, v in out.items()}


def _fptr(t, cols):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 \
            or not t.is_contiguous() or t.dim() != 2 or t.shape[1] != cols:
        raise TypeError(f"expected a contiguous float32 cuda tensor (m,{cols})")
    return t.data_ptr()


def _stream(stream):
    import torch
    return torch.cuda.current_stream().cuda_stream if stream is None else stream


def lub_mlp_set_weights(h, theta):
    th = np.ascontiguousarray(theta, dtype=np.float32)
    _check(lib().lub_mlp_set_weights(h, th.ctypes.data_as(C.POINTER(C.c_float)),
                                     th.size), "lub_mlp_set_weights")


def lub_mlp_get_weights(h):
    th = np.zeros(LUB_MLP_PARAMS, dtype=np.float32)
    _check(lib().lub_mlp_get_weights(h, th.ctypes.data_as(C.POINTER(C.c_float)),
                                     th.size), "lub_mlp_get_weights")
    return th


def lub_mlp_save(h):
    """The training state (weights, Adam moments, step count) as a float32
    array of LUB_MLP_STATE values."""
    st = np.zeros(LUB_MLP_STATE, dtype=np.float32)
    _check(lib().lub_mlp_save(h, st.ctypes.data_as(C.POINTER(C.c_float)), st.size),
           "lub_mlp_save")
    return st


def lub_mlp_load(h, state):
    st = np.ascontiguousarray(state, dtype=np.float32)
    _check(lib().lub_mlp_load(h, st.ctypes.data_as(C.POINTER(C.c_float)), st.size),
           "lub_mlp_load")


def lub_mlp_init(h, seed=0):
    _check(lib().lub_mlp_init(h, int(seed)), "lub_mlp_init")


def lub_mlp_forward(h, X, Y, stream=None):
    """Y (m,4) = network(X (m,10)); float32 cuda tensors."""
    m = X.shape[0]
    _check(lib().lub_mlp_forward(h, m, _fptr(X, 10), _fptr(Y, 4), _stream(stream)),
           "lub_mlp_forward")


def lub_mlp_grad(h, X, T, stream=None):
    m = X.shape[0]
    loss = np.zeros(1, dtype=np.float32)
    g = np.zeros(LUB_MLP_PARAMS, dtype=np.float32)
    Fp = C.POINTER(C.c_float)
    _check(lib().lub_mlp_grad(h, m, _fptr(X, 10), _fptr(T, 6), loss.ctypes.data_as(Fp),
                              g.ctypes.data_as(Fp), _stream(stream)), "lub_mlp_grad")
    return float(loss[0]), g


def lub_mlp_train(h, X, T, epochs=4, batch=2048, lr=1e-3, beta1=0.9, beta2=0.999,
                  eps=1e-8, lr_decay=1.0, stream=None):
    m = X.shape[0]
    cfg = lub_train_cfg_t(epochs, batch, lr, beta1, beta2, eps, lr_decay, 0)
    out = np.zeros(max(epochs, 1), dtype=np.float32)
    _check(lib().lub_mlp_train(h, m, _fptr(X, 10), _fptr(T, 6), C.byref(cfg),
                               out.ctypes.data_as(C.POINTER(C.c_float)), _stream(stream)),
           "lub_mlp_train")
    return out[:epochs]


def lub_destroy(h):
    lib().lub_destroy(h)


def lub_strerror(code: int) -> str:
    return lib().lub_strerror(code).decode()


# --- convenience ---------------------------------------------------------------

class Lub:
    """Owns one handle; ``compute`` takes and returns torch.cuda tensors.
    ``skin`` > 0 reuses the neighbour lists across calls (lub_opts_t.skin)."""

    def __init__(self, L, periodic, params: dict, rmax_bound, n_walls=0,
                 wall_vel=((0, 0, 0), (0, 0, 0)), precision=LUB_FP64, device=0,
                 sync=1, newton_max_iter=0, max_neighbors=0, timing=0,
                 seed_mode=LUB_SEED_PLAIN, graph=0, warm_start=0, lees_edwards=None,
                 skin=0.0, newton_tol=0.0, host_pointers=0, record_detail=0):
        self.domain_args = dict(L=L, periodic=periodic, n_walls=n_walls, wall_vel=wall_vel,
                                lees_edwards=lees_edwards)
        self.h = lub_create(make_domain(L, periodic, n_walls, wall_vel, lees_edwards),
                            make_params(**params),
                            make_opts(rmax_bound, precision, device, seed_mode=seed_mode,
                                      newton_max_iter=newton_max_iter, sync=sync,
                                      max_neighbors=max_neighbors, timing=timing,
                                      graph=graph, warm_start=warm_start, skin=skin,
                                      newton_tol=newton_tol, host_pointers=host_pointers,
                                      record_detail=record_detail))

    def compute(self, r, q, semi, v, w, f=None, t=None, stream=None, check=True):
        import torch
        n = r.shape[0]
        if f is None:
            f = torch.empty((n, 3), dtype=torch.float64, device=r.device)
        if t is None:
            t = torch.empty((n, 3), dtype=torch.float64, device=r.device)
        lub_compute(self.h, r, q, semi, v, w, f, t, stream, check)
        return f, t

    def stats(self):
        return lub_get_stats(self.h)

    def integrate(self, r, q, semi, v, w, dt, n_sub, density=1.0, damping=0.0,
                  f_ext=None, t_ext=None, f=None, t=None, stream=None):
        import torch
        n = r.shape[0]
        if f is None:
            f = torch.empty((n, 3), dtype=torch.float64, device=r.device)
        if t is None:
            t = torch.empty((n, 3), dtype=torch.float64, device=r.device)
        lub_integrate(self.h, r, q, semi, v, w, f, t, dt, n_sub, density, damping,
                      f_ext, t_ext, stream)
        d = lub_get_domain(self.h)
        if d.lees_edwards:
            self.domain_args["lees_edwards"] = (d.le_offset, d.le_velocity)
        return f, t

    def advance(self, r, q, v, w, dt, stream=None):
        lub_advance(self.h, r, q, v, w, dt, stream)

    def grow(self, r, q, semi, v, w, **kw):
        lub_grow(self.h, r, q, semi, v, w, **kw)
        d = lub_get_domain(self.h)
        if d.lees_edwards:
            self.domain_args["lees_edwards"] = (d.le_offset, d.le_velocity)

    def set_domain(self, **kw):
        """Replace domain fields (e.g. lees_edwards=(offset, velocity))."""
        self.domain_args.update(kw)
        lub_set_domain(self.h, make_domain(**self.domain_args))

    def reset_timers(self):
        lub_reset_timers(self.h)

    def pairs(self):
        return lub_get_pairs(self.h)

    def pair_results(self):
        return lub_get_pair_results(self.h)

    def pair_detail(self):
        return lub_get_pair_detail(self.h)

    def close(self):
        if self.h:
            lub_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @classmethod
    def for_workload(cls, wl, precision=LUB_FP64, **kw):
        kw.setdefault("lees_edwards", wl.lees_edwards)
        return cls(wl.L, wl.periodic, wl.params, float(wl.semi.max()),
                   n_walls=wl.n_walls, wall_vel=wl.wall_vel, precision=precision,
                   **kw)


def to_device(wl, device="cuda:0"):
    """The workload's arrays as contiguous float64 tensors on the GPU."""
    import torch
    return [torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to(device)
            for a in (wl.r, wl.q, wl.semi, wl.v, wl.w)]
