"""The allocation-free entry point lub_compute_static (workspace in a fixed
device array of the library) against lub_compute through a handle: two
calls in a row, the second with a smaller input, each compared element by
element with the handle's result for the same options."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _handle_result(L, wl, prec, torch):
    lb = L.Lub.for_workload(wl, precision=prec, sync=1, max_neighbors=128)
    r, q, semi, v, w = L.to_device(wl)
    f, t = lb.compute(r, q, semi, v, w)
    torch.cuda.synchronize()
    st = lb.stats()
    lb.close()
    return f.cpu().numpy(), t.cpu().numpy(), st


def _static_result(L, wl, prec, torch):
    dom = L.make_domain(**wl.domain())
    par = L.make_params(**wl.params)
    opts = L.make_opts(float(wl.semi.max()), precision=prec, max_neighbors=128)
    r, q, semi, v, w = L.to_device(wl)
    f = torch.full((wl.n, 3), np.nan, dtype=torch.float64, device="cuda")
    t = torch.full((wl.n, 3), np.nan, dtype=torch.float64, device="cuda")
    st = L.lub_compute_static(dom, par, opts, r, q, semi, v, w, f, t)
    torch.cuda.synchronize()
    return f.cpu().numpy(), t.cpu().numpy(), st


def test_static_matches_handle_two_calls():
    import torch
    from paper_1308_6482_amd import lub as L
    from paper_1308_6482_amd import workloads as W
    assert torch.cuda.is_available()
    cases = [(W.config2(), L.LUB_MIXED), (W.config1(), L.LUB_FP64)]
    assert cases[1][0].n < cases[0][0].n
    for wl, prec in cases:
        print(f"no-alloc: {wl.name} n={wl.n} precision={prec}", flush=True)
        fs, ts, ss = _static_result(L, wl, prec, torch)
        fh, th, sh = _handle_result(L, wl, prec, torch)
        for k in ("candidates", "evaluated", "active", "overlaps", "unconverged"):
            assert ss[k] == sh[k], (k, ss[k], sh[k])
        assert ss["error"] == 0
        scale_f = np.abs(fh).max()
        scale_t = np.abs(th).max()
        tol = 1e-12 if prec == L.LUB_FP64 else 1e-6
        assert np.all(np.isfinite(fs)) and np.all(np.isfinite(ts))
        assert np.abs(fs - fh).max() <= tol * scale_f
        assert np.abs(ts - th).max() <= tol * scale_t


def test_static_large_path_matches_handle():
    """Systems beyond the one-workgroup cell build (binning, staged records,
    scatter, record build): 12,000 then 6,000 prolates, as above."""
    import torch
    from paper_1308_6482_amd import lub as L
    from paper_1308_6482_amd import workloads as W
    assert torch.cuda.is_available()
    for n, prec in ((12000, L.LUB_MIXED), (6000, L.LUB_FP64)):
        wl = W.config2(n=n)
        print(f"no-alloc: {wl.name} n={wl.n} precision={prec}", flush=True)
        fs, ts, ss = _static_result(L, wl, prec, torch)
        fh, th, sh = _handle_result(L, wl, prec, torch)
        for k in ("candidates", "evaluated", "active", "overlaps", "unconverged"):
            assert ss[k] == sh[k], (k, ss[k], sh[k])
        assert ss["error"] == 0 and ss["active"] > 0
        tol = 1e-12 if prec == L.LUB_FP64 else 1e-6
        assert np.all(np.isfinite(fs)) and np.all(np.isfinite(ts))
        assert np.abs(fs - fh).max() <= tol * np.abs(fh).max()
        assert np.abs(ts - th).max() <= tol * np.abs(th).max()


def test_static_rejects_sizes_beyond_the_maximum():
    import torch
    from paper_1308_6482_amd import lub as L
    n = L.lib  # noqa: F841
    wl_n = 16385
    dom = L.make_domain((1000.0, 1000.0, 1000.0), (1, 1, 1))
    par = L.make_params(1 / 6, 0.67, 0.5, 0.25)
    opts = L.make_opts(4.0)
    z3 = torch.zeros((wl_n, 3), dtype=torch.float64, device="cuda")
    q = torch.zeros((wl_n, 4), dtype=torch.float64, device="cuda")
    q[:, 0] = 1.0
    semi = torch.full((wl_n, 2), 4.0, dtype=torch.float64, device="cuda")
    with pytest.raises(L.LubError) as e:
        L.lub_compute_static(dom, par, opts, z3, q, semi, z3, z3, z3.clone(), z3.clone())
    assert e.value.code == L.LUB_EINVAL
    opts = L.make_opts(4.0, max_neighbors=256)
    with pytest.raises(L.LubError) as e:
        L.lub_compute_static(dom, par, opts, z3[:10], q[:10], semi[:10], z3[:10], z3[:10],
                             z3[:10].clone(), z3[:10].clone())
    assert e.value.code == L.LUB_EINVAL
