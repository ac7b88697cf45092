"""GPU tests of the graph mode of lub_compute (the launch sequence captured
once per counter set and replayed).

Every replay is checked against an eager evaluation of the same inputs,
bit for bit (both are deterministic), with the program's own eager work and
synchronisations between replays, and with the inputs changed in place
between replays (a replay must read the current values).  Statistics after
a replay equal the eager ones.
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


@pytest.mark.parametrize("name,precision,seed_mode", [
    ("prolates4096", L.LUB_MIXED, L.LUB_SEED_PLAIN),
    ("walls3000", L.LUB_FP64, L.LUB_SEED_PLAIN),
    ("spheres36", L.LUB_FP64, L.LUB_SEED_MLP),
])
def test_graph_replays_match_eager(name, precision, seed_mode):
    wl = {"prolates4096": W.config2, "spheres36": W.config1,
          "walls3000": lambda: W.config3(n=3000)}[name]()
    print(f"[gpu] graph replays {name} precision={precision} seed_mode={seed_mode}",
          flush=True)
    stream = torch.cuda.Stream()
    eager = L.Lub.for_workload(wl, precision=precision, seed_mode=seed_mode)
    graph = L.Lub.for_workload(wl, precision=precision, seed_mode=seed_mode, sync=0,
                               graph=1)
    if seed_mode == L.LUB_SEED_MLP:
        for lb in (eager, graph):
            L.lub_mlp_init(lb.h, 7)
    r, q, semi, v, w = L.to_device(wl)
    f = torch.empty((wl.n, 3), dtype=torch.float64, device="cuda")
    t = torch.empty_like(f)
    rng = np.random.default_rng(5)
    for k in range(6):
        if k == 3:
            # move every particle a little, in place: later replays must see it
            with torch.cuda.stream(stream):
                r.add_(torch.as_tensor(rng.normal(scale=1e-3, size=(wl.n, 3)),
                                       device="cuda"))
        stream.synchronize()
        fe, te = eager.compute(r, q, semi, v, w)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            graph.compute(r, q, semi, v, w, f, t, stream=stream)
        stream.synchronize()
        # unrelated eager work between replays
        x = torch.randn((256, 256), device="cuda")
        (x @ x).sum().item()
        assert torch.equal(f, fe) and torch.equal(t, te), f"replay {k} differs"
        se, sg = eager.stats(), graph.stats()
        for key in ("candidates", "evaluated", "active", "newton_iters", "newton_max"):
            assert se[key] == sg[key], (k, key, se[key], sg[key])
        assert sg["error"] == 0
    eager.close()
    graph.close()


def test_graph_mode_arguments():
    wl = W.config1()
    r, q, semi, v, w = L.to_device(wl)
    with pytest.raises(L.LubError) as e:
        L.Lub.for_workload(wl, graph=1, timing=1)
    assert e.value.code == L.LUB_EINVAL
    lb = L.Lub.for_workload(wl, graph=1)
    with pytest.raises(L.LubError) as e:
        lb.compute(r, q, semi, v, w, stream=0)
    assert e.value.code == L.LUB_EINVAL
    lb.close()
