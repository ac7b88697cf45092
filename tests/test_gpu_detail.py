"""Per-output parity: the intermediate results of every evaluated pair
(lub_get_pair_detail) against the oracle's (ref_eval_pairs_detail) -- the
closest points y_i*, y_j*, the gap direction n, the frame axis x1 and each of
the 16 corrective elements K~ (Appendix with Eq. lub:resistance-correction).

Bars: the closest points and n come from the FP64 Newton solve in both
precisions: 1e-9 of the largest semi-axis.  K~: FP64 1e-9, mixed (FP32
coefficients) 1e-5, each relative to the largest |K~| element of the pair
(the scale the transfer multiplies).  At the poles of a spheroid x1 is any
tangent (the elements then depend on that choice, the forces do not): such
pairs are left out of the element comparison and must be rare."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_1308_6482_amd import lub as L  # noqa: E402
from paper_1308_6482_amd import workloads as W  # noqa: E402

KIDX = [(0, 0), (0, 1), (0, 2), (0, 3), (0, 4), (1, 1), (1, 2), (1, 3), (1, 4), (2, 2),
        (2, 3), (2, 4), (2, 5), (3, 3), (3, 4), (4, 4)]
KNAMES = [f"K{r_ + 1}{c_ + 1}" for r_, c_ in KIDX]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()


@pytest.mark.parametrize("name", ["config2", "config3"])
@pytest.mark.parametrize("prec,kbar", [(L.LUB_FP64, 1e-9), (L.LUB_MIXED, 1e-5)])
def test_pair_detail_against_oracle(ref, name, prec, kbar):
    wl = W.config2() if name == "config2" else W.config3(n=6000)
    print(f"[gpu] pair detail {wl.name} precision={prec}", flush=True)
    lb = L.Lub.for_workload(wl, precision=prec, record_detail=1)
    lb.compute(*L.to_device(wl))
    torch.cuda.synchronize()
    pr = lb.pair_results()
    dt = lb.pair_detail()
    lb.close()
    dom = ref.make_domain(**wl.domain())
    P = ref.make_params(**wl.params)
    o = ref.eval_pairs_detail(wl.r, wl.q, wl.semi, wl.v, wl.w, dom, P, pr["ij"])
    act = o["status"] == 0
    assert np.array_equal(pr["status"] == 0, act)
    i, j = pr["ij"][:, 0], pr["ij"][:, 1]
    R = wl.semi.max()
    pp = j >= 0
    assert np.abs(dt["n"][act] - o["n"][act]).max() <= 1e-9
    assert np.abs(dt["yi"][act] - o["yi"][act]).max() <= 1e-9 * R
    assert np.abs(dt["yj"][act & pp] - o["yj"][act & pp]).max() <= 1e-9 * R
    same_frame = np.abs(np.sum(dt["e1"] * o["e1"], axis=1) - 1.0) < 1e-9
    assert np.mean(~same_frame[act]) < 0.01
    m = act & same_frame
    Ko = np.stack([o["Kt"][:, r_, c_] for r_, c_ in KIDX], axis=1)
    scale = np.maximum(np.abs(Ko).max(axis=1), 1e-300)
    err = np.abs(dt["Kt"] - Ko) / scale[:, None]
    worst = err[m].max(axis=0)
    print("K~ element errors:", " ".join(f"{k}:{e:.1e}" for k, e in zip(KNAMES, worst)))
    assert worst.max() <= kbar, worst
    # inactive pairs carry no elements
    assert np.all(dt["Kt"][~act] == 0.0)


def test_detail_needs_the_option():
    wl = W.config1()
    lb = L.Lub.for_workload(wl)
    lb.compute(*L.to_device(wl))
    with pytest.raises(L.LubError):
        lb.pair_detail()
    lb.close()
