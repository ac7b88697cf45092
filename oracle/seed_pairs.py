"""Oracle-labelled pairs of the learned Newton seed (test infrastructure).

The draws (shapes, orientations, centre direction u, target gap) come from
the input generator; the centre separation along u that gives the target
gap and the closest points there (the labels) come from the oracle
(ref_place_pairs).  Run as a script it writes the pairs to an .npz file:

    python -m oracle.seed_pairs --seed 1 --m 2097152 --out PATH

(seed 1: the 2,097,152 training pairs; seed 2: the 262,144 held-out pairs.)
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1308_6482_amd import workloads as W  # noqa: E402


def labelled_pairs(seed: int, m: int, nthreads: int = 0) -> dict:
    """Draws of the input generator plus the oracle's placement and labels:
    q_i, q_j, semi_i, semi_j, u, target, and s (separation), d = s u (offset
    of j's centre), h, n, yi, yj (closest points relative to each centre),
    iters_lh, status (0: placed)."""
    inp = W.config4_pair_inputs(seed, m)
    out = oracle.place_pairs(inp["u"], inp["target"], inp["q_i"], inp["semi_i"],
                             inp["q_j"], inp["semi_j"], nthreads=nthreads)
    res = dict(inp)
    res.update(out)
    res["d"] = out["s"][:, None] * inp["u"]
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seed", type=int, required=True)
    ap.add_argument("--m", type=int, required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    t0 = time.perf_counter()
    P = labelled_pairs(a.seed, a.m, a.threads)
    el = time.perf_counter() - t0
    bad = int(np.sum(P["status"] != 0))
    print(f"seed {a.seed}: {a.m} pairs in {el:.1f} s, {bad} not placed, mean Lin-Han "
          f"iterations {P['iters_lh'].mean():.1f}", flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    keep = ("q_i", "q_j", "semi_i", "semi_j", "u", "target", "s", "h", "n", "yi", "yj",
            "iters_lh", "status")
    np.savez(a.out, **{k: P[k] for k in keep})


if __name__ == "__main__":
    main()
