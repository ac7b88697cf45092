"""Boundary options through the C ABI: host arrays (lub_opts_t.host_pointers)
give the results of device arrays, and the Newton tolerance newton_tol."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_1308_6482_amd import lub as L  # noqa: E402
from paper_1308_6482_amd import workloads as W  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()


@pytest.mark.parametrize("prec", [L.LUB_FP64, L.LUB_MIXED])
def test_host_pointers_equal_device(prec):
    wl = W.config2()
    print(f"[gpu] host pointers precision={prec}", flush=True)
    lb = L.Lub.for_workload(wl, precision=prec)
    f, t = lb.compute(*L.to_device(wl))
    torch.cuda.synchronize()
    st_dev = lb.stats()
    lb.close()
    hb = L.Lub.for_workload(wl, precision=prec, host_pointers=1)
    fh, th = L.lub_compute_host(hb.h, wl.r, wl.q, wl.semi, wl.v, wl.w)
    st_host = hb.stats()
    # a second call on the same handle (staging buffers reused): the first
    # 2048 particles of the same box
    m = 2048
    wl2 = W.Workload(wl.name, wl.r[:m].copy(), wl.q[:m].copy(), wl.semi[:m].copy(),
                     wl.v[:m].copy(), wl.w[:m].copy(), wl.L, wl.periodic,
                     params=dict(wl.params))
    fh2, th2 = L.lub_compute_host(hb.h, wl2.r, wl2.q, wl2.semi, wl2.v, wl2.w)
    hb.close()
    assert st_host["active"] == st_dev["active"] and st_host["error"] == 0
    assert np.array_equal(fh, f.cpu().numpy()) and np.array_equal(th, t.cpu().numpy())
    lb2 = L.Lub.for_workload(wl2, precision=prec)
    f2, t2 = lb2.compute(*L.to_device(wl2))
    torch.cuda.synchronize()
    lb2.close()
    assert np.array_equal(fh2, f2.cpu().numpy()) and np.array_equal(th2, t2.cpu().numpy())


def test_host_pointers_reject_integrate_and_graph():
    wl = W.config1()
    with pytest.raises(L.LubError):
        L.Lub.for_workload(wl, host_pointers=1, graph=1)
    hb = L.Lub.for_workload(wl, host_pointers=1)
    r, q, semi, v, w = L.to_device(wl)
    with pytest.raises(L.LubError):
        hb.integrate(r, q, semi, v, w, 0.1, 1)
    hb.close()


def test_newton_tol(ref):
    """The tolerance of the closest-point solve: a looser one needs no more
    iterations and costs accuracy in proportion (1e-10 stays within the
    mixed-precision bar; the default 1e-14 meets the FP64 bar); a tolerance
    >= 1e-2 is rejected."""
    wl = W.config2()
    dom = ref.make_domain(**wl.domain())
    P = ref.make_params(**wl.params)
    res = {}
    for tol in (0.0, 1e-10):
        print(f"[gpu] newton_tol={tol}", flush=True)
        lb = L.Lub.for_workload(wl, precision=L.LUB_FP64, newton_tol=tol)
        lb.compute(*L.to_device(wl))
        torch.cuda.synchronize()
        st, pr = lb.stats(), lb.pair_results()
        lb.close()
        F, Ti, Tj, h, status = ref.eval_pairs(wl.r, wl.q, wl.semi, wl.v, wl.w, dom, P,
                                              pr["ij"])
        act = status == 0
        nF = np.linalg.norm(F[act], axis=1)
        res[tol] = (st, (np.linalg.norm(pr["F"][act] - F[act], axis=1) / nF).max())
        print(f"  iterations {st['newton_iters']} max rel err F {res[tol][1]:.2e}")
    assert res[1e-10][0]["newton_iters"] <= res[0.0][0]["newton_iters"]
    assert res[0.0][1] <= 1e-9
    assert res[1e-10][1] <= 1e-5
    with pytest.raises(L.LubError):
        L.Lub.for_workload(wl, newton_tol=1e-2)
