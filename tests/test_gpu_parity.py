"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.

Bars:
  * candidate pair lists: bit-exact (same FP64 centre test);
  * LUB_FP64: per-pair force and torque within 1e-9 relative, per-particle
    sums within 1e-9 of max(|ref|, 1e-3 rms) -- the two sides use different
    closest-point algorithms and formula routes, both converged to round-off;
  * LUB_MIXED: per-pair force within 1e-5 relative and torque within 1e-5 of
    max(|T_ref|, a |F_ref|) for pairs with h/a >= 1e-3 (a = smallest
    semi-axis of the pair); per-particle sums within 1e-5 of
    max(|ref|, sum over its pairs of the per-pair scale) -- the bound a sum
    of terms with 1e-5 relative error obeys however much they cancel.
"""
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
    return True


def run_gpu(wl, precision=L.LUB_FP64, **kw):
    print(f"[gpu] {wl.name} n={wl.n} precision={precision}", flush=True)
    lb = L.Lub.for_workload(wl, precision=precision, **kw)
    r, q, semi, v, w = L.to_device(wl)
    f, t = lb.compute(r, q, semi, v, w)
    torch.cuda.synchronize()
    out = dict(f=f.cpu().numpy(), t=t.cpu().numpy(), stats=lb.stats(),
               pairs=lb.pairs(), res=lb.pair_results())
    lb.close()
    return out


def run_oracle(ref, wl):
    dom = ref.make_domain(**wl.domain())
    P = ref.make_params(**wl.params)
    f, t, st = ref.compute(wl.r, wl.q, wl.semi, wl.v, wl.w, dom, P)
    ij, wall = ref.candidates(wl.r, wl.semi, dom, P)
    return dict(f=f, t=t, stats=st, pairs=ij, walls=wall, dom=dom, P=P)


def per_pair_errors(ref, wl, g, o):
    """Errors of every GPU-evaluated pair against the oracle's evaluation of
    the same pair; returns (errF, errT, h/a, status arrays)."""
    res = g["res"]
    ij = res["ij"]
    F, Ti, Tj, h, st = ref.eval_pairs(wl.r, wl.q, wl.semi, wl.v, wl.w, o["dom"],
                                      o["P"], ij)
    i = ij[:, 0]
    j = ij[:, 1]
    a = wl.semi[i].min(axis=1)
    a = np.where(j >= 0, np.minimum(a, wl.semi[np.maximum(j, 0)].min(axis=1)), a)
    nF = np.linalg.norm(F, axis=1)
    Rl = wl.semi[i].max(axis=1)
    eF = np.linalg.norm(res["F"] - F, axis=1) / np.maximum(nF, 1e-300)
    sTi = np.maximum(np.linalg.norm(Ti, axis=1), a * nF)
    sTj = np.maximum(np.linalg.norm(Tj, axis=1), a * nF)
    eT = np.maximum(np.linalg.norm(res["Ti"] - Ti, axis=1) / np.maximum(sTi, 1e-300),
                    np.where(j >= 0, np.linalg.norm(res["Tj"] - Tj, axis=1)
                             / np.maximum(sTj, 1e-300), 0.0))
    active = st == ref.REFP_ACTIVE
    assert np.array_equal(res["status"] == 0, active), "active sets differ"
    eF = np.where(active, eF, 0.0)
    eT = np.where(active, eT, 0.0)
    assert np.allclose(res["h"], h, rtol=0, atol=1e-9 * Rl.max())
    return eF, eT, h / a, active


def contribution_scale(ref, wl, o):
    """Per particle, the sum of the magnitudes of the pair contributions to
    its force and torque (oracle values).  A sum whose terms each carry a
    relative error e has an error of at most e times this scale, however
    much the terms cancel."""
    ij = np.concatenate([o["pairs"], np.stack([o["walls"][:, 0], -1 - o["walls"][:, 1]],
                                              axis=1)]) if len(o["walls"]) else o["pairs"]
    sf = np.zeros(wl.n)
    st = np.zeros(wl.n)
    if len(ij):
        F, Ti, Tj, h, stt = ref.eval_pairs(wl.r, wl.q, wl.semi, wl.v, wl.w, o["dom"],
                                           o["P"], ij)
        i, j = ij[:, 0], ij[:, 1]
        a = wl.semi[i].min(axis=1)
        a = np.where(j >= 0, np.minimum(a, wl.semi[np.maximum(j, 0)].min(axis=1)), a)
        nF = np.linalg.norm(F, axis=1)
        # the same torque scale as the per-pair gate: max(|T|, a |F|)
        np.add.at(sf, i, nF)
        np.add.at(st, i, np.maximum(np.linalg.norm(Ti, axis=1), a * nF))
        m = j >= 0
        np.add.at(sf, j[m], nF[m])
        np.add.at(st, j[m], np.maximum(np.linalg.norm(Tj[m], axis=1), a[m] * nF[m]))
    return sf, st


def particle_errors(g, o, ref=None, wl=None):
    """Per-particle error of f and t: |delta| / max(|ref|, 1e-3 rms), and,
    when ref and wl are given, / max(|ref|, sum of |pair contributions|)."""
    scales = contribution_scale(ref, wl, o) if ref is not None else (None, None)
    out = []
    for key, sc in zip(("f", "t"), scales):
        ref_ = o[key]
        nrm = np.linalg.norm(ref_, axis=1)
        if sc is None:
            rms = np.sqrt(np.mean(np.sum(ref_ ** 2, axis=1)))
            den = np.maximum(nrm, max(1e-3 * rms, 1e-300))
        else:
            den = np.maximum(np.maximum(nrm, sc), 1e-300)
        out.append(np.linalg.norm(g[key] - ref_, axis=1) / den)
    return out


def check_pairs(g, o):
    gp, gw = g["pairs"]
    assert np.array_equal(gp, o["pairs"]), "candidate pair lists differ"
    assert np.array_equal(gw, o["walls"]), "wall candidate lists differ"


@pytest.mark.parametrize("hc,ec", [(0.0, 0.0), (0.01, 100.0)])
def test_config1_fp64(ref, hc, ec):
    wl = W.config1().with_params(h_c=hc, eps_c=ec)
    g = run_gpu(wl)
    o = run_oracle(ref, wl)
    check_pairs(g, o)
    assert g["stats"]["error"] == 0
    assert g["stats"]["candidates"] == o["stats"]["candidates"]
    assert g["stats"]["active"] == o["stats"]["active"]
    eF, eT, ha, act = per_pair_errors(ref, wl, g, o)
    assert eF.max() < 1e-9 and eT.max() < 1e-9, (eF.max(), eT.max())
    ef, et = particle_errors(g, o)
    assert ef.max() < 1e-9 and et.max() < 1e-9, (ef.max(), et.max())


@pytest.fixture(scope="module")
def cfg2():
    return W.config2()


@pytest.mark.parametrize("precision,tol", [(L.LUB_FP64, 1e-9), (L.LUB_MIXED, 1e-5)])
def test_config2(ref, cfg2, precision, tol):
    wl = cfg2
    g = run_gpu(wl, precision)
    o = run_oracle(ref, wl)
    check_pairs(g, o)
    st = g["stats"]
    assert st["error"] == 0 and st["unconverged"] == 0
    assert st["active"] == o["stats"]["active"]
    eF, eT, ha, act = per_pair_errors(ref, wl, g, o)
    gate = act & (ha >= 1e-3)
    print(f"pairs active={act.sum()} gated={gate.sum()} maxF={eF[gate].max():.3e} "
          f"maxT={eT[gate].max():.3e} p99F={np.quantile(eF[gate], 0.99):.3e}")
    assert eF[gate].max() < tol and eT[gate].max() < tol
    ef, et = particle_errors(g, o, ref, wl)
    e1f, e1t = particle_errors(g, o)
    print(f"particles max f={ef.max():.3e} t={et.max():.3e} "
          f"(rms-floor definition: f={e1f.max():.3e} t={e1t.max():.3e})")
    assert ef.max() < tol and et.max() < tol


def test_walls_polydisperse(ref):
    wl = W.config3(n=6000)
    g = run_gpu(wl, L.LUB_MIXED)
    o = run_oracle(ref, wl)
    check_pairs(g, o)
    assert g["stats"]["wall_candidates"] > 0
    eF, eT, ha, act = per_pair_errors(ref, wl, g, o)
    gate = act & (ha >= 1e-3)
    assert eF[gate].max() < 1e-5 and eT[gate].max() < 1e-5, (eF[gate].max(), eT[gate].max())
    ef, et = particle_errors(g, o, ref, wl)
    print(f"particles (contribution scale) max f={ef.max():.3e} t={et.max():.3e}")
    assert ef.max() < 1e-5 and et.max() < 1e-5
    g64 = run_gpu(wl, L.LUB_FP64)
    ef, et = particle_errors(g64, o)
    assert ef.max() < 1e-9 and et.max() < 1e-9


@pytest.mark.timeout(600)
def test_config3_full(ref):
    """65,536 polydisperse spheroids between walls at the full size: more
    particles than the single-workgroup cell build takes, so the multi-kernel
    build runs; every pair and particle against the oracle."""
    wl = W.config3()
    assert wl.n > 1 << 15
    g = run_gpu(wl, L.LUB_MIXED)
    o = run_oracle(ref, wl)
    check_pairs(g, o)
    eF, eT, ha, act = per_pair_errors(ref, wl, g, o)
    gate = act & (ha >= 1e-3)
    print(f"pairs evaluated={len(act)} active={act.sum()} max eF={eF[gate].max():.3e} "
          f"eT={eT[gate].max():.3e}")
    assert eF[gate].max() < 1e-5 and eT[gate].max() < 1e-5
    ef, et = particle_errors(g, o, ref, wl)
    assert ef.max() < 1e-5 and et.max() < 1e-5, (ef.max(), et.max())


@pytest.mark.timeout(600)
def test_long_backward_lists(ref):
    """33,000 unit spheres at volume fraction 0.25 with a cut-off of 5 (about
    86 partners each, so that most particles find more than 32 of their
    pairs in their partners' searches): the forward search's backward lists
    are ranked over several chunks.  Every pair and particle against the
    oracle."""
    rng = np.random.default_rng(21)
    n = 33000
    semi = np.ones((n, 2))
    Lx = (n * 4.0 / 3.0 * np.pi / 0.25) ** (1.0 / 3.0)
    r, q, _ = W.rsa(rng, semi, (Lx, Lx, Lx), (1, 1, 1))
    assert r.shape[0] == n
    wl = small("spheres33000_cut5", r, q, semi, rng.normal(size=(n, 3)),
               rng.normal(size=(n, 3)), L_=(Lx, Lx, Lx), delta_n=5.0, delta_t=5.0,
               delta_r=2.0, h_c=0.01, eps_c=100.0)
    g = run_gpu(wl, L.LUB_MIXED)
    assert g["stats"]["error"] == 0
    assert g["stats"]["max_degree"] > 80, g["stats"]["max_degree"]
    o = run_oracle(ref, wl)
    check_pairs(g, o)
    eF, eT, ha, act = per_pair_errors(ref, wl, g, o)
    gate = act & (ha >= 1e-3)
    print(f"pairs evaluated={len(act)} active={act.sum()} max degree="
          f"{g['stats']['max_degree']} max eF={eF[gate].max():.3e} eT={eT[gate].max():.3e}")
    assert eF[gate].max() < 1e-5 and eT[gate].max() < 1e-5
    ef, et = particle_errors(g, o, ref, wl)
    assert ef.max() < 1e-5 and et.max() < 1e-5, (ef.max(), et.max())


def small(name, r, q, semi, v, w, L_=(60.0, 60.0, 60.0), periodic=(1, 1, 1),
          n_walls=0, **params):
    p = dict(mu=1.0 / 6.0, delta_n=0.67, delta_t=0.5, delta_r=0.25, h_c=0.0, eps_c=0.0)
    p.update(params)
    arr = [np.ascontiguousarray(np.asarray(x, dtype=np.float64)) for x in (r, q, semi, v, w)]
    return W.Workload(name, *arr, L=L_, periodic=periodic, n_walls=n_walls, params=p)


def test_edge_cases(ref):
    rng = np.random.default_rng(3)
    q1 = [[1, 0, 0, 0]]
    # one particle: nothing to do, zero output
    wl = small("one", [[1, 2, 3]], q1, [[4, 2]], [[1, 0, 0]], [[0, 0, 0]])
    g = run_gpu(wl)
    assert np.all(g["f"] == 0) and g["stats"]["candidates"] == 0
    # coaxial prolates tip to tip (pole contact), side by side, small overlap
    cases = []
    for h in (1e-3, 0.05, -0.02):
        cases.append(("tips", [[10, 10, 10], [10, 10, 10 + 16 + h]], [[1, 0, 0, 0]] * 2))
        cases.append(("sides", [[10, 10, 10], [10, 10 + 8 + h, 10]], [[1, 0, 0, 0]] * 2))
    for name, r, q in cases:
        wl = small(name, r, q, [[8, 4], [8, 4]], rng.normal(size=(2, 3)),
                   rng.normal(size=(2, 3)), h_c=0.01, eps_c=100.0)
        for prec, tol in ((L.LUB_FP64, 1e-9), (L.LUB_MIXED, 1e-5)):
            g = run_gpu(wl, prec)
            o = run_oracle(ref, wl)
            ef, et = particle_errors(g, o)
            assert ef.max() < tol and et.max() < tol, (name, prec, ef.max(), et.max())
    # ragged: a few particles spread over several cells, with walls
    wl = W.config3(n=1000)
    g = run_gpu(wl)
    o = run_oracle(ref, wl)
    check_pairs(g, o)
    ef, et = particle_errors(g, o)
    assert ef.max() < 1e-9 and et.max() < 1e-9


def test_sparse_large_grid(ref):
    """96 prolates in close pairs scattered over a periodic 3000^3 box: a
    grid of millions of cells for few particles, so the multi-kernel cell
    build runs on one partial block and the cell scan on hundreds of tiles;
    some pairs straddle the periodic faces."""
    rng = np.random.default_rng(11)
    L_ = 3000.0
    r, q = [], []
    for k in range(48):
        c = rng.uniform(0.0, L_, size=3)
        if k % 8 == 0:
            c[k % 3] = L_ - 2.0  # the partner lies across the face
        h = rng.uniform(0.005, 0.6)
        off = np.zeros(3)
        ax = (k + 1) % 3
        off[ax] = (16.0 if ax == 2 else 8.0) + h  # tip to tip along the axis z
        for x in (c, np.mod(c + off, L_)):
            r.append(x)
            q.append([1.0, 0.0, 0.0, 0.0])
    n = len(r)
    wl = small("sparse", r, q, [[8.0, 4.0]] * n, rng.normal(size=(n, 3)),
               rng.normal(size=(n, 3)), L_=(L_, L_, L_), h_c=0.01, eps_c=100.0)
    for prec, tol in ((L.LUB_FP64, 1e-9), (L.LUB_MIXED, 1e-5)):
        g = run_gpu(wl, prec)
        o = run_oracle(ref, wl)
        check_pairs(g, o)
        assert g["stats"]["error"] == 0
        assert g["stats"]["active"] == o["stats"]["active"] > 0
        ef, et = particle_errors(g, o)
        assert ef.max() < tol and et.max() < tol, (prec, ef.max(), et.max())


def test_empty_input():
    lb = L.Lub((50, 50, 50), (1, 1, 1), dict(mu=1, delta_n=0.67, delta_t=0.5,
                                             delta_r=0.25), 4.0)
    z = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    zq = torch.zeros((0, 4), dtype=torch.float64, device="cuda")
    zs = torch.zeros((0, 2), dtype=torch.float64, device="cuda")
    lb.compute(z, zq, zs, z, z)
    assert lb.stats()["candidates"] == 0
    lb.close()


def test_errors():
    wl = W.config1()
    r, q, semi, v, w = L.to_device(wl)
    lb = L.Lub.for_workload(wl)
    bad = r.clone()
    bad[3, 1] = float("nan")
    with pytest.raises(L.LubError) as e:
        lb.compute(bad, q, semi, v, w)
    assert e.value.code == L.LUB_EINVAL
    badq = q.clone()
    badq[0] *= 1.01
    with pytest.raises(L.LubError) as e:
        lb.compute(r, badq, semi, v, w)
    assert e.value.code == L.LUB_EINVAL
    with pytest.raises(L.LubError) as e:
        lb.compute(r, q, semi * 2.0, v, w)      # larger than rmax_bound
    assert e.value.code == L.LUB_EINVAL
    lb.compute(r, q, semi, v, w)                 # recovers
    lb.close()
    with pytest.raises(L.LubError) as e:
        tiny = L.Lub((12.0, 40, 40), (1, 1, 1), wl.params, 4.0)
        tiny.compute(r, q, semi, v, w)
    assert e.value.code == L.LUB_EDOMAIN
    lb = L.Lub.for_workload(wl, max_neighbors=1, sync=1)
    lb.compute(r, q, semi, v, w)     # a fixed limit of 64 is enough here
    lb.close()
    dense = small("stack", np.tile([[20.0, 20.0, 20.0]], (80, 1)) + np.random.default_rng(0)
                  .normal(scale=0.5, size=(80, 3)), np.tile([[1.0, 0, 0, 0]], (80, 1)),
                  np.full((80, 2), 2.0), np.zeros((80, 3)), np.zeros((80, 3)))
    r, q, semi, v, w = L.to_device(dense)
    lb = L.Lub.for_workload(dense, max_neighbors=64)
    with pytest.raises(L.LubError) as e:
        lb.compute(r, q, semi, v, w)
    assert e.value.code == L.LUB_ECAPACITY
    lb.close()


def test_deterministic(cfg2):
    wl = cfg2
    a = run_gpu(wl, L.LUB_MIXED)
    b = run_gpu(wl, L.LUB_MIXED)
    assert np.array_equal(a["f"], b["f"]) and np.array_equal(a["t"], b["t"])


@pytest.mark.parametrize("model", [L.LUB_MODEL_NORMAL, L.LUB_MODEL_LADD])
def test_reduced_models_spheres(ref, model):
    """The paper's comparison models on 36 spheres (h_c = 0 and the
    production clipping), both precisions, against the oracle's own
    implementations of the same laws."""
    for hc, ec in ((0.0, 0.0), (0.01, 100.0)):
        wl = W.config1().with_params(h_c=hc, eps_c=ec, model=model)
        o = run_oracle(ref, wl)
        assert o["stats"]["active"] > 0
        for prec, tol in ((L.LUB_FP64, 1e-9), (L.LUB_MIXED, 1e-5)):
            g = run_gpu(wl, prec)
            check_pairs(g, o)
            assert g["stats"]["active"] == o["stats"]["active"]
            # the exact torques vanish (forces through the centres): their
            # error is judged on the contribution scale, sum of a |F|
            ef, et = particle_errors(g, o, ref, wl)
            print(f"model={model} hc={hc} prec={prec} f={ef.max():.3e} t={et.max():.3e}")
            assert ef.max() < tol and et.max() < tol
            if model == L.LUB_MODEL_LADD:
                assert np.abs(g["t"]).max() == 0.0


def test_normal_only_spheroids(ref, cfg2):
    for wl, tol in ((cfg2.with_params(model=L.LUB_MODEL_NORMAL), 1e-5),
                    (W.config3(n=3000).with_params(model=L.LUB_MODEL_NORMAL), 1e-5)):
        g = run_gpu(wl, L.LUB_MIXED)
        o = run_oracle(ref, wl)
        check_pairs(g, o)
        eF, eT, ha, act = per_pair_errors(ref, wl, g, o)
        gate = act & (ha >= 1e-3)
        print(f"{wl.name} normal-only active={act.sum()} eF={eF[gate].max():.3e} "
              f"eT={eT[gate].max():.3e}")
        assert eF[gate].max() < tol and eT[gate].max() < tol
        ef, et = particle_errors(g, o, ref, wl)
        assert ef.max() < tol and et.max() < tol


def test_ladd_rejects_spheroids(cfg2):
    wl = cfg2.with_params(model=L.LUB_MODEL_LADD)
    lb = L.Lub.for_workload(wl)
    r, q, semi, v, w = L.to_device(wl)
    with pytest.raises(L.LubError) as e:
        lb.compute(r, q, semi, v, w)
    assert e.value.code == L.LUB_EINVAL
    lb.close()


@pytest.mark.parametrize("precision,tol", [(L.LUB_FP64, 1e-9), (L.LUB_MIXED, 1e-5)])
def test_tangent_sphere_fallback(ref, cfg2, precision, tol):
    """Newton capped at 3 iterations fails from the line of centres for most
    pairs; they go through the tangent-sphere iteration (Sec. III.A, both
    phases) and a Newton polish from its normal in the second pass of the
    pair stage, and must still meet the bars against the oracle."""
    wl = cfg2
    g = run_gpu(wl, precision, newton_max_iter=3)
    o = run_oracle(ref, wl)
    check_pairs(g, o)
    st = g["stats"]
    pp = st["evaluated"] - st["wall_candidates"]
    print(f"fallbacks {st['fallbacks']} of {pp} particle pairs, unconverged "
          f"{st['unconverged']}, iterations/pair {st['newton_iters'] / max(pp, 1):.2f}")
    assert st["error"] == 0 and st["unconverged"] == 0
    assert st["fallbacks"] > 0.3 * pp
    # each slot is counted once, by the pass that finished it
    assert sum(st["iter_hist"]) == st["evaluated"]
    # the failed attempts plus the polish: more than the cap
    assert st["newton_max"] > 3
    assert st["active"] == o["stats"]["active"]
    eF, eT, ha, act = per_pair_errors(ref, wl, g, o)
    gate = act & (ha >= 1e-3)
    assert eF[gate].max() < tol and eT[gate].max() < tol, (eF[gate].max(), eT[gate].max())
    ef, et = particle_errors(g, o, ref, wl)
    assert ef.max() < tol and et.max() < tol


@pytest.mark.parametrize("kind,n,precision,tol", [
    ("prolates", 4096, L.LUB_MIXED, 1e-5), ("prolates", 4096, L.LUB_FP64, 1e-9),
    ("polydisperse", 6000, L.LUB_MIXED, 1e-5), ("prolates", 60, L.LUB_FP64, 1e-9)])
def test_lees_edwards(ref, kind, n, precision, tol):
    """Sheared periodic cube with Lees-Edwards images (offset 0.37 L): pair
    lists bit-exact, pairs and particle sums at the bars.  n = 60 makes the
    grid three cells or fewer per axis (z and x searched whole)."""
    wl = W.sheared(n=n, polydisperse=kind == "polydisperse")
    g = run_gpu(wl, precision)
    o = run_oracle(ref, wl)
    check_pairs(g, o)
    st = g["stats"]
    assert st["error"] == 0 and st["unconverged"] == 0
    assert st["active"] == o["stats"]["active"] > 0
    # pairs across the sheared boundary are present
    ij = o["pairs"]
    dz = wl.r[ij[:, 1], 2] - wl.r[ij[:, 0], 2]
    assert np.sum(np.abs(dz) > wl.L[2] / 2) > (0 if n < 100 else 20)
    eF, eT, ha, act = per_pair_errors(ref, wl, g, o)
    gate = act & (ha >= 1e-3)
    print(f"pairs active={act.sum()} max eF={eF[gate].max():.3e} eT={eT[gate].max():.3e}")
    assert eF[gate].max() < tol and eT[gate].max() < tol
    ef, et = particle_errors(g, o, ref, wl)
    assert ef.max() < tol and et.max() < tol


def test_lees_edwards_zero_offset_is_periodic(cfg2):
    """Offset and image velocity 0: the plain periodic result, bit for bit."""
    wl = cfg2
    a = run_gpu(wl, L.LUB_MIXED)
    wl0 = W.Workload(wl.name, wl.r, wl.q, wl.semi, wl.v, wl.w, wl.L, wl.periodic,
                     params=wl.params, lees_edwards=(0.0, 0.0))
    b = run_gpu(wl0, L.LUB_MIXED)
    assert np.array_equal(a["f"], b["f"]) and np.array_equal(a["t"], b["t"])


def test_lees_edwards_offset_update_graph():
    """A new offset between calls (set_domain): graph replay recaptures and
    equals eager evaluation bit for bit."""
    wl = W.sheared(n=4096)
    print("[gpu] Lees-Edwards offset updates, graph vs eager", flush=True)
    r, q, semi, v, w = L.to_device(wl)
    stream = torch.cuda.Stream()
    eager = L.Lub.for_workload(wl, precision=L.LUB_MIXED)
    graph = L.Lub.for_workload(wl, precision=L.LUB_MIXED, graph=1, sync=0)
    f = torch.empty((wl.n, 3), dtype=torch.float64, device="cuda")
    t = torch.empty_like(f)
    off, U = wl.lees_edwards
    for k, o in enumerate((off, off + 1.5, off + 1.5, off - 40.0)):
        for lb in (eager, graph):
            lb.set_domain(lees_edwards=(o, U))
        fe, te = eager.compute(r, q, semi, v, w)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            graph.compute(r, q, semi, v, w, f, t, stream=stream)
        stream.synchronize()
        assert torch.equal(f, fe) and torch.equal(t, te), f"step {k}"
    eager.close()
    graph.close()
