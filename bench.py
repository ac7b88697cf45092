#!/usr/bin/env python
"""Benchmark of the lubrication correction on one MI355X.

Metric: lubrication-corrected pairs per second (pairs with a non-zero
correction, particle-particle and particle-wall) for one full evaluation
(staging, cell list, neighbour lists, closest points, geometry,
resistance, transfer, per-particle sums) with inputs resident in HBM.

Default workload: 4096 prolate spheroids (semi-axes 8,4,4) at volume
fraction 0.3 in a periodic cube, simple-shear velocities, seed 0, mixed
precision.  One step = one lub_compute call on that suspension.

Prints one JSON line.  --gpus N with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of the pair kernel per unit, counted from the kernel's
# source by an operation-counting host build (adds and multiplies, FMA = 2;
# divisions, square roots and logarithms listed apart and not counted):
#   per evaluated pair (set-up and final evaluation): 100 FP64 flops
#   per Newton iteration (incl. line-search trials):  306 FP64 flops
#   per active pair, LUB_MIXED: 225 FP64 + 450 FP32 flops; LUB_FP64: 675 FP64
FLOPS_EVAL = 100
FLOPS_ITER = 306
FLOPS_POST = {"mixed": 225 + 450, "fp64": 675}
# MI355X vector ALU peak, non-packed FMA: 256 CUs x 64 lanes x 2 flops x 2.4 GHz
# (the same for FP64 and unpacked FP32; packed FP32 is not used)
PEAK_ALU_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--workload", choices=["prolates4096", "spheres36", "polydisperse65536"],
                    default="prolates4096")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="budget of the CPU oracle baseline (0: skip)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 512 MiB device copy after the timed region "
                         "(reference for the HBM traffic counters)")
    return ap.parse_args()


def workload(name):
    from paper_1308_6482_amd import workloads as W
    if name == "prolates4096":
        return W.config2()
    if name == "spheres36":
        return W.config1()
    return W.config3()


def pair_kernel_traffic(precision):
    """HBM bytes per launch of the pair kernel from the committed counter
    summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "pair_kernel_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, "paper_1308_6482_amd", "csrc", "lub_pair.hip"), "rb").read()
    if rec.get("source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return rec.get(precision, {}).get("bytes_per_launch")


def cpu_baseline(wl, seconds, gpu_pairs):
    """The FP64 oracle on the host cores over the same suspension (whole
    evaluations repeated for about `seconds`), plus the error of the GPU
    pair results against it."""
    import numpy as np
    import oracle
    dom = oracle.make_domain(**wl.domain())
    P = oracle.make_params(**wl.params)
    f, t, st = oracle.compute(wl.r, wl.q, wl.semi, wl.v, wl.w, dom, P)
    reps = 0
    t0 = time.perf_counter()
    while True:
        f, t, st = oracle.compute(wl.r, wl.q, wl.semi, wl.v, wl.w, dom, P)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    value = st["active"] * reps / el
    # GPU accuracy on every evaluated pair (force and torque, h/a >= 1e-3)
    ij = gpu_pairs["ij"]
    F, Ti, Tj, h, status = oracle.eval_pairs(wl.r, wl.q, wl.semi, wl.v, wl.w, dom, P, ij)
    i, j = ij[:, 0], ij[:, 1]
    a = wl.semi[i].min(axis=1)
    a = np.where(j >= 0, np.minimum(a, wl.semi[np.maximum(j, 0)].min(axis=1)), a)
    act = (status == 0) & (h / a >= 1e-3)
    nF = np.linalg.norm(F, axis=1)
    eF = np.linalg.norm(gpu_pairs["F"] - F, axis=1)[act] / nF[act]
    sT = np.maximum(np.linalg.norm(Ti, axis=1), a * nF)[act]
    eT = np.linalg.norm(gpu_pairs["Ti"] - Ti, axis=1)[act] / sT
    return dict(value=value, unit="pairs/s", cores=int(st["threads"]), kind="oracle",
                sample=f"whole evaluations of the same {wl.n}-particle suspension, "
                       f"{reps} repeats in {el:.1f} s"), \
        dict(pairs_checked=int(act.sum()), max_rel_err_force=float(eF.max()),
             max_rel_err_torque=float(eT.max()))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np  # noqa: F401
    import torch
    from paper_1308_6482_amd import lub as L

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    wl = workload(args.workload)
    prec = L.LUB_MIXED if args.precision == "mixed" else L.LUB_FP64
    lb = L.Lub.for_workload(wl, precision=prec, sync=0, timing=1)
    r, q, semi, v, w = L.to_device(wl)
    f = torch.empty((wl.n, 3), dtype=torch.float64, device="cuda")
    t = torch.empty((wl.n, 3), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    # first call synchronous: sizes the workspace and validates the inputs
    lb.compute(r, q, semi, v, w, f, t)
    st = lb.stats()
    if st["error"]:
        raise RuntimeError(f"lub_compute failed: {L.lub_strerror(st['error'])}")
    for _ in range(args.warmup):
        lb.compute(r, q, semi, v, w, f, t, stream=stream.cuda_stream)
    torch.cuda.synchronize()
    lb.reset_timers()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lb.compute(r, q, semi, v, w, f, t, stream=stream.cuda_stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = lb.stats()
    if st["error"] or st["unconverged"]:
        raise RuntimeError(f"invalid run: error={st['error']} unconverged={st['unconverged']}")
    if args.calibrate_copy:
        x = torch.empty(512 * 2 ** 20, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
    ms = (t1 - t0) * 1e3 / args.steps
    active = st["active"]
    value = active / (ms * 1e-3)
    pair_ms = st["stage_ms"][2] / max(st["timed_calls"], 1)
    flops = (FLOPS_EVAL * st["evaluated"] + FLOPS_ITER * st["newton_iters"]
             + FLOPS_POST[args.precision] * active)
    achieved = flops / (pair_ms * 1e-3) / 1e12
    res = dict(
        metric="lubrication-corrected pairs/sec on 1 GPU at rel err <=1e-5 vs FP64 oracle",
        value=value, unit="pairs/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=ms, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64+f32" if args.precision == "mixed" else "f64",
        data="synthetic (seeded random sequential addition, simple-shear velocities)",
        config=dict(workload=wl.name, n_particles=wl.n, box=list(wl.L),
                    periodic=list(wl.periodic), walls=wl.n_walls, seed=0,
                    precision=args.precision, cutoffs=[wl.params["delta_n"], wl.params["delta_t"],
                                                       wl.params["delta_r"]],
                    h_c=wl.params["h_c"], eps_c=wl.params["eps_c"], mu=wl.params["mu"],
                    parallelism="single GPU"),
        pairs=dict(candidates=st["candidates"], wall_candidates=st["wall_candidates"],
                   evaluated=st["evaluated"], active=active, overlaps=st["overlaps"],
                   newton_iters_mean=st["newton_iters"] / max(st["evaluated"], 1),
                   newton_max=st["newton_max"]),
        stage_ms={k: v_ / max(st["timed_calls"], 1) for k, v_ in zip(
            ["cells", "neighbours", "pairs", "reduction"], st["stage_ms"])},
        roofline=dict(bound="alu", kernel="k_pairs", achieved=achieved,
                      peak=PEAK_ALU_TFLOPS, unit="TFLOP/s", frac=achieved / PEAK_ALU_TFLOPS,
                      flops_per_launch=flops, launch_ms=pair_ms,
                      traffic=pair_kernel_traffic(args.precision)),
    )
    if args.cpu_seconds > 0:
        lb2 = L.Lub.for_workload(wl, precision=prec)
        lb2.compute(r, q, semi, v, w)
        pr = lb2.pair_results()
        lb2.close()
        cb, acc = cpu_baseline(wl, args.cpu_seconds, pr)
        res["cpu_baseline"] = cb
        res["accuracy"] = acc
    lb.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
