"""GPU tests of the sub-stepped particle update (lub_integrate, Sec. II) and
the growth stage of the packing generator (lub_grow, Sec. IV.C), through
the C ABI, against the reference integrator over the FP64 oracle.

Bars: the state after the sub-steps is compared with the reference; the
change of each velocity (and angular velocity) over the call must agree to
tol times the rms change over all particles, positions to tol times the rms
displacement.  tol = 1e-9 in FP64 mode; 1e-4 in mixed mode, where each pair
force carries up to 1e-5 relative error and a particle sums several pairs
over several sub-steps; 1e-7 for the growth trajectory (stiff contacts).
The Lees-Edwards offset after the call is equal bit for bit (both sides
advance it with the same host arithmetic).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from oracle import integrate as I  # noqa: E402
from paper_1308_6482_amd import lub as L  # noqa: E402
from paper_1308_6482_amd import workloads as W  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def wrapped_diff(a, b, Lbox):
    d = a - b
    return d - np.array(Lbox) * np.round(d / np.array(Lbox))


def rms(x):
    return float(np.sqrt(np.mean(np.sum(x ** 2, axis=1))))


def check_state(g, o, s0, Lbox, tol):
    r0, v0, w0 = s0
    (rg, qg, vg, wg), (ro, qo, vo, wo) = g, o
    dr = rms(wrapped_diff(ro, r0, Lbox))
    er = np.abs(wrapped_diff(rg, ro, Lbox)).max() / dr
    ev = np.abs(vg - vo).max() / rms(vo - v0)
    ew = np.abs(wg - wo).max() / rms(wo - w0)
    eq = np.abs(qg - qo).max()
    print(f"errors: r {er:.2e} v {ev:.2e} w {ew:.2e} q {eq:.2e}")
    assert er < tol and ev < tol and ew < tol and eq < tol


@pytest.mark.parametrize("precision,tol", [(L.LUB_FP64, 1e-9), (L.LUB_MIXED, 1e-4)])
def test_integrate_lees_edwards(ref, precision, tol):
    wl = W.sheared(n=2000)
    print(f"[gpu] lub_integrate, sheared 2000 prolates, precision={precision}", flush=True)
    rng = np.random.default_rng(11)
    v0 = wl.v + rng.normal(scale=0.01, size=(wl.n, 3))
    w0 = wl.w + rng.normal(scale=1e-3, size=(wl.n, 3))
    fext = rng.normal(scale=0.5, size=(wl.n, 3))
    text = rng.normal(scale=0.5, size=(wl.n, 3))
    dt, nsub = 0.1, 5
    lb = L.Lub.for_workload(wl, precision=precision)
    r, q, semi, v, w = (dev(x) for x in (wl.r, wl.q, wl.semi, v0, w0))
    f, t = lb.integrate(r, q, semi, v, w, dt, nsub, f_ext=dev(fext), t_ext=dev(text))
    torch.cuda.synchronize()
    st = lb.stats()
    assert st["error"] == 0 and st["unconverged"] == 0 and st["active"] > 0
    dg = L.lub_get_domain(lb.h)
    lb.close()
    dom = O.make_domain(**wl.domain())
    P = O.make_params(**wl.params)
    ro, qo, vo, wo, fo, to, domo = I.integrate(wl.r, wl.q, wl.semi, v0, w0, dom, P, dt, nsub,
                                               f_ext=fext, t_ext=text)
    assert dg.le_offset == domo.le_offset
    g = tuple(x.cpu().numpy() for x in (r, q, v, w))
    check_state(g, (ro, qo, vo, wo), (wl.r, v0, w0), wl.L, tol)


def test_integrate_walls(ref):
    wl = W.config3(n=3000)
    print("[gpu] lub_integrate, 3000 polydisperse between walls, FP64", flush=True)
    rng = np.random.default_rng(12)
    v0 = wl.v + rng.normal(scale=0.01, size=(wl.n, 3))
    w0 = wl.w.copy()
    dt, nsub = 0.1, 4
    lb = L.Lub.for_workload(wl, precision=L.LUB_FP64)
    r, q, semi, v, w = (dev(x) for x in (wl.r, wl.q, wl.semi, v0, w0))
    lb.integrate(r, q, semi, v, w, dt, nsub, density=1.2, damping=0.05)
    torch.cuda.synchronize()
    lb.close()
    dom = O.make_domain(**wl.domain())
    P = O.make_params(**wl.params)
    ro, qo, vo, wo, *_ = I.integrate(wl.r, wl.q, wl.semi, v0, w0, dom, P, dt, nsub,
                                     density=1.2, damping=0.05)
    g = tuple(x.cpu().numpy() for x in (r, q, v, w))
    check_state(g, (ro, qo, vo, wo), (wl.r, v0, w0), (wl.L[0], wl.L[1], 1e300), 1e-9)


def test_integrate_graph_equals_eager():
    wl = W.sheared(n=2000)
    print("[gpu] lub_integrate in graph mode vs eager", flush=True)
    stream = torch.cuda.Stream()
    states = []
    for graph in (0, 1):
        lb = L.Lub.for_workload(wl, precision=L.LUB_MIXED, graph=graph, sync=1 - graph)
        r, q, semi, v, w = (dev(x) for x in (wl.r, wl.q, wl.semi, wl.v, wl.w))
        with torch.cuda.stream(stream):
            lb.integrate(r, q, semi, v, w, 0.1, 3, stream=stream)
        stream.synchronize()
        states.append([x.cpu().numpy() for x in (r, q, v, w)])
        lb.close()
    for a, b in zip(*states):
        assert np.array_equal(a, b)


def test_integrate_errors():
    wl = W.config1()
    lb = L.Lub.for_workload(wl)
    r, q, semi, v, w = (dev(x) for x in (wl.r, wl.q, wl.semi, wl.v, wl.w))
    for kw in (dict(dt=0.0, n_sub=1), dict(dt=0.1, n_sub=0), dict(dt=0.1, n_sub=1, density=0.0),
               dict(dt=0.1, n_sub=1, damping=-1.0)):
        with pytest.raises(L.LubError):
            lb.integrate(r, q, semi, v, w, **kw)
    lb.close()


def test_advance_matches_oracle():
    """The kinematic advance against the reference, several steps in a row
    on a ragged particle count (FP64 both sides: within a few ulps)."""
    rng = np.random.default_rng(11)
    n, dt = 1000 * 3 + 37, 0.7
    r0 = rng.uniform(0.0, 300.0, size=(n, 3))
    q0 = rng.normal(size=(n, 4))
    q0 /= np.linalg.norm(q0, axis=1)[:, None]
    v = rng.normal(size=(n, 3))
    w = rng.normal(size=(n, 3)) * 0.05
    lb = L.Lub.for_workload(W.config1())
    r, q, vd, wd = dev(r0), dev(q0), dev(v), dev(w)
    ro, qo = r0, q0
    for _ in range(5):
        lb.advance(r, q, vd, wd, dt)
        ro, qo = I.advance(ro, qo, v, w, dt)
    torch.cuda.synchronize()
    rg, qg = r.cpu().numpy(), q.cpu().numpy()
    assert np.abs(rg - ro).max() <= 1e-13 * np.abs(ro).max()
    assert np.abs(qg - qo).max() <= 1e-14
    assert np.array_equal(vd.cpu().numpy(), v) and np.array_equal(wd.cpu().numpy(), w)
    # no particles: nothing to do; bad arguments: an error
    e = torch.empty((0, 3), dtype=torch.float64, device="cuda")
    lb.advance(e, torch.empty((0, 4), dtype=torch.float64, device="cuda"), e, e, dt)
    with pytest.raises(L.LubError):
        lb.advance(r, q, vd, wd, float("nan"))
    lb.close()


def seeded_small(n, phi, seed):
    """Spheroids at 30 % of their linear size placed without overlap in a
    periodic cube sized for volume fraction phi at full size."""
    rng = np.random.default_rng(seed)
    semi = W.polydisperse_semi(rng, n, 0.5, 2.0, 3.0, 5.0)
    vol = float(np.sum(4.0 / 3.0 * np.pi * semi[:, 0] * semi[:, 1] ** 2))
    Lx = (vol / phi) ** (1.0 / 3.0)
    r, q, _ = W.rsa(rng, semi * 0.3, (Lx, Lx, Lx), (1, 1, 1))
    assert r.shape[0] == n
    return r, q, semi, (Lx, Lx, Lx)


GROW = dict(scale0=0.3, scale1=1.05, dt=0.2, density=1.0, damping=1.0, h_c=0.3, eps_c=1000.0)


def test_grow_matches_oracle(ref):
    r0, q0, semi, Lb = seeded_small(300, 0.45, 5)
    print("[gpu] lub_grow, 300 spheroids, first 20 steps vs the reference", flush=True)
    n_steps = 20
    cfg = dict(GROW, scale1=0.3 + 0.75 * n_steps / 1200.0)
    rng = np.random.default_rng(6)
    v0 = rng.normal(scale=0.05, size=r0.shape)
    w0 = np.zeros_like(r0)
    params = dict(mu=1.0 / 6.0, delta_n=0.67, delta_t=0.5, delta_r=0.25, h_c=0.01, eps_c=100.0)
    lb = L.Lub(Lb, (1, 1, 1), params, 1.05 * float(semi.max()), precision=L.LUB_FP64)
    r, q, s, v, w = (dev(x) for x in (r0, q0, semi, v0, w0))
    lb.grow(r, q, s, v, w, n_steps=n_steps, **cfg)
    torch.cuda.synchronize()
    # the handle's own law is back afterwards
    f, t = lb.compute(r, q, s, v, w)
    lb.close()
    dom = O.make_domain(L=Lb, periodic=(1, 1, 1))
    ro, qo, vo, wo, _ = I.grow(r0, q0, semi, v0, w0, dom, n_steps, **cfg)
    g = tuple(x.cpu().numpy() for x in (r, q, v, w))
    # stiff contacts (eps_c = 1000, a period of a few steps) carry the
    # rounding-level difference of the two closest-point solvers from step
    # to step: a looser bar than for one evaluation
    check_state(g, (ro, qo, vo, wo), (r0, v0, w0), Lb, 1e-7)


def test_grow_packs_without_overlap(ref):
    """Grow to 1.05 and reset: at the final size no pair overlaps and the
    volume fraction is the target, above what random sequential addition
    of these shapes reaches directly."""
    phi = 0.45
    r0, q0, semi, Lb = seeded_small(500, phi, 7)
    print("[gpu] lub_grow, 500 spheroids to volume fraction 0.45", flush=True)
    params = dict(mu=1.0 / 6.0, delta_n=0.67, delta_t=0.5, delta_r=0.25, h_c=0.01, eps_c=100.0)
    lb = L.Lub(Lb, (1, 1, 1), params, 1.05 * float(semi.max()), precision=L.LUB_FP64)
    r, q, s, v, w = (dev(x) for x in (r0, q0, semi, np.zeros_like(r0), np.zeros_like(r0)))
    lb.grow(r, q, s, v, w, n_steps=1200, **GROW)
    torch.cuda.synchronize()
    lb.close()
    rr, qq = r.cpu().numpy(), q.cpu().numpy()
    assert np.all(np.abs(np.linalg.norm(qq, axis=1) - 1) < 1e-12)
    dom = O.make_domain(L=Lb, periodic=(1, 1, 1))
    P = O.make_params(h_c=0.0, eps_c=0.0)
    ij, _ = ref.candidates(rr, semi, dom, P)
    z = np.zeros_like(rr)
    F, Ti, Tj, h, st = ref.eval_pairs(rr, qq, semi, z, z, dom, P, ij)
    ok = st != ref.REFP_FAILED
    print(f"pairs within the cut-off {len(ij)}, min gap {h[ok].min():.4f}")
    assert ok.all()
    assert h.min() > 0.0
    vol = float(np.sum(4.0 / 3.0 * np.pi * semi[:, 0] * semi[:, 1] ** 2))
    assert abs(vol / Lb[0] ** 3 - phi) < 1e-12
