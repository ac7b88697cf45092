"""GPU regression tests of workspace growth on a reused handle.

Every device buffer group of a handle is sized by the largest call so far
and reallocated when a call needs more.  These tests make each group grow
after a smaller call and check the results against the oracle (or, for the
network, against the FP64 reference gradient):

* lub_mlp_grad on a batch larger than an earlier one (batch scratch);
* a large sphere ringed by about a hundred small ones: more than the
  default 64 partners, so the automatic limit widens the neighbour segments
  and the evaluation slots (and, in the learned-seed mode, the seed buffers)
  between two evaluations of one call;
* one handle evaluating 700, then 6000, then 700 particles (particle, cell,
  segment and slot buffers).
"""
import dataclasses

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_1308_6482_amd import lub as L  # noqa: E402
from paper_1308_6482_amd import seed_data as S  # noqa: E402
from paper_1308_6482_amd import workloads as W  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()


def cuda32(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def oracle_forces(ref, wl):
    dom = ref.make_domain(**wl.domain())
    P = ref.make_params(**wl.params)
    f, t, _ = ref.compute(wl.r, wl.q, wl.semi, wl.v, wl.w, dom, P)
    return f, t


def rel_particle_error(g, o):
    rms = np.sqrt(np.mean(np.sum(o ** 2, axis=1)))
    den = np.maximum(np.linalg.norm(o, axis=1), max(1e-3 * rms, 1e-300))
    return (np.linalg.norm(g - o, axis=1) / den).max()


def test_grad_batch_grows():
    from oracle import mlp_ref as M
    print("[gpu] lub_mlp_grad 128 then 8192 samples", flush=True)
    lb = L.Lub((100.0, 100.0, 100.0), (1, 1, 1),
               dict(mu=1 / 6, delta_n=0.67, delta_t=0.5, delta_r=0.25), 10.0)
    theta = torch.as_tensor(M.init(seed=5).astype(np.float32) * 0.8).to(
        torch.bfloat16).float().numpy()
    L.lub_mlp_set_weights(lb.h, theta)
    P = S.sample_pairs(seed=13, m=8192)
    X = torch.as_tensor(P["X"]).to(torch.bfloat16).float().numpy()
    L.lub_mlp_grad(lb.h, cuda32(X[:128]), cuda32(P["T"][:128]))
    loss, g = L.lub_mlp_grad(lb.h, cuda32(X), cuda32(P["T"]))
    Lr, gr = M.grad(theta.astype(np.float64), X.astype(np.float64),
                    P["T"].astype(np.float64))
    print(f"loss gpu {loss:.6f} ref {Lr:.6f}")
    assert abs(loss - Lr) < 2e-2 * Lr
    e = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    print(f"gradient normwise rel diff {e:.3e}")
    assert e < 5e-2
    # a training step with a smaller batch reuses the larger scratch
    losses = L.lub_mlp_train(lb.h, cuda32(X), cuda32(P["T"]), epochs=1, batch=256,
                             lr=1e-3)
    assert np.all(np.isfinite(losses))
    lb.close()


def ring_workload():
    """Sphere of radius 8 at the box centre and 100 spheres of radius 1 on
    Fibonacci directions around it, gaps 0.05 to 0.5 (all candidates of the
    large one, none of each other: small centres are more than 2.67 apart)."""
    m = 100
    k = np.arange(m) + 0.5
    z = 1.0 - 2.0 * k / m
    phi = np.pi * (1.0 + 5.0 ** 0.5) * k
    u = np.stack([np.sqrt(1 - z * z) * np.cos(phi), np.sqrt(1 - z * z) * np.sin(phi), z], 1)
    rng = np.random.default_rng(21)
    gap = rng.uniform(0.05, 0.5, size=m)
    c = np.array([30.0, 30.0, 30.0])
    r = np.concatenate([c[None], c + u * (9.0 + gap)[:, None]])
    n = m + 1
    q = W.random_quaternions(rng, n)
    semi = np.concatenate([[[8.0, 8.0]], np.ones((m, 2))])
    params = dict(mu=1.0 / 6.0, delta_n=0.67, delta_t=0.5, delta_r=0.25, h_c=0.0, eps_c=0.0)
    return W.Workload("ring101", r, q, semi, rng.normal(size=(n, 3)),
                      rng.normal(size=(n, 3)), (60.0, 60.0, 60.0), (1, 1, 1),
                      params=params)


@pytest.mark.parametrize("seed_mode", [L.LUB_SEED_PLAIN, L.LUB_SEED_MLP])
def test_segments_widen(ref, seed_mode):
    wl = ring_workload()
    print(f"[gpu] ring101 automatic segment widening seed_mode={seed_mode}", flush=True)
    fo, to = oracle_forces(ref, wl)
    lb = L.Lub.for_workload(wl, precision=L.LUB_FP64, sync=1, max_neighbors=0,
                            seed_mode=seed_mode)
    if seed_mode == L.LUB_SEED_MLP:
        L.lub_mlp_init(lb.h, 3)
    r, q, semi, v, w = L.to_device(wl)
    f, t = lb.compute(r, q, semi, v, w)
    torch.cuda.synchronize()
    st = lb.stats()
    print(f"candidates {st['candidates']} active {st['active']}")
    assert st["candidates"] == 100 and st["unconverged"] == 0
    ef = rel_particle_error(f.cpu().numpy(), fo)
    et = rel_particle_error(t.cpu().numpy(), to)
    print(f"max rel err f={ef:.3e} t={et:.3e}")
    assert ef < 1e-9 and et < 1e-9
    lb.close()


@pytest.mark.parametrize("seed_mode", [L.LUB_SEED_PLAIN, L.LUB_SEED_MLP])
def test_handle_reuse_growing_n(ref, seed_mode):
    full = W.config3(n=6000)
    sub = dataclasses.replace(full, name="first700", r=full.r[:700], q=full.q[:700],
                              semi=full.semi[:700], v=full.v[:700], w=full.w[:700])
    lb = L.Lub.for_workload(full, precision=L.LUB_FP64, seed_mode=seed_mode)
    if seed_mode == L.LUB_SEED_MLP:
        L.lub_mlp_init(lb.h, 3)
    for wl in (sub, full, sub):
        print(f"[gpu] reused handle n={wl.n} seed_mode={seed_mode}", flush=True)
        fo, to = oracle_forces(ref, wl)
        f, t = lb.compute(*L.to_device(wl))
        torch.cuda.synchronize()
        ef = rel_particle_error(f.cpu().numpy(), fo)
        et = rel_particle_error(t.cpu().numpy(), to)
        print(f"n={wl.n} max rel err f={ef:.3e} t={et:.3e}")
        assert ef < 1e-9 and et < 1e-9
    lb.close()


@pytest.mark.parametrize("max_neighbors", [128, 192, 320])
def test_neighbour_group_sizes(ref, max_neighbors):
    """The neighbour kernel's lanes per particle follow the segment size
    (16 up to 128 entries, 32 up to 256, a whole wavefront above): the same
    system with each, against the oracle's pair set and forces."""
    wl = W.config3(n=3000)
    print(f"[gpu] polydisperse3000 max_neighbors={max_neighbors}", flush=True)
    dom = ref.make_domain(**wl.domain())
    P = ref.make_params(**wl.params)
    fo, to, _ = ref.compute(wl.r, wl.q, wl.semi, wl.v, wl.w, dom, P)
    ij, walls = ref.candidates(wl.r, wl.semi, dom, P)
    lb = L.Lub.for_workload(wl, precision=L.LUB_FP64, max_neighbors=max_neighbors)
    f, t = lb.compute(*L.to_device(wl))
    torch.cuda.synchronize()
    gp, gw = lb.pairs()
    lb.close()
    assert np.array_equal(gp, ij) and np.array_equal(gw, walls)
    assert rel_particle_error(f.cpu().numpy(), fo) < 1e-9
    assert rel_particle_error(t.cpu().numpy(), to) < 1e-9
