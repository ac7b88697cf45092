#!/usr/bin/env python
"""Benchmark of the lubrication correction on one MI355X.

Metric: lubrication-corrected pairs per second (pairs with a non-zero
correction, particle-particle and particle-wall) for one full evaluation
(staging, cell list, neighbour lists, closest points, geometry,
resistance, transfer, per-particle sums) with inputs resident in HBM.

Default workload: 4096 prolate spheroids (semi-axes 8,4,4) at volume
fraction 0.3 in a periodic cube, simple-shear velocities, seed 0, mixed
precision.  One step = one lub_compute call on that suspension.

Prints one JSON line.  --gpus N with N > 1 exits: the benchmark runs on one GPU.
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
    ap.add_argument("--workload", choices=["prolates4096", "spheres36", "polydisperse65536",
                                           "fullscale1M"],
                    default="prolates4096")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="budget of the CPU oracle baseline (0: skip)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 512 MiB device copy after the timed region "
                         "(reference for the HBM traffic counters)")
    ap.add_argument("--model", choices=["full", "normal", "ladd"], default="full",
                    help="resistance law: the full contact-based model, normal only, or "
                         "Ladd's sphere law (spheres only)")
    ap.add_argument("--compare-models", type=int, default=1,
                    help="also time the normal-only model on the same workload (1) or not (0)")
    ap.add_argument("--trajectory-dt", type=float, default=None,
                    help="warm-start leg: positions advanced by v dt between the K timed "
                         "evaluations (0: skip the leg; default 1 for the full-scale "
                         "system, 0.1 otherwise)")
    ap.add_argument("--skin", type=float, nargs="*", default=None,
                    help="trajectory leg: also time reused neighbour lists with these skins "
                         "(default 4 for the full-scale system, 1 otherwise; none given: "
                         "skip)")
    ap.add_argument("--seed", choices=["plain", "mlp", "both"], default="both",
                    help="Newton start: line of centres, learned network, or time both "
                         "(the JSON value is the plain form unless --seed mlp)")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no GPU work: read two rocprofv3 --pmc runs of this script with "
                         "--calibrate-copy (FETCH_SIZE, then WRITE_SIZE), scale each by the "
                         "copy kernel's reading and write profiles/pair_kernel_traffic.json")
    ap.add_argument("--dynamics", type=int, default=1,
                    help="also time the sheared box with Lees-Edwards images, the "
                         "sub-stepped integrator and the growth stage (1) or not (0)")
    ap.add_argument("--train-pairs", type=int, default=1 << 21)
    ap.add_argument("--train-epochs", type=int, default=6)
    return ap.parse_args()


def workload(name):
    from paper_1308_6482_amd import workloads as W
    if name == "prolates4096":
        return W.config2()
    if name == "spheres36":
        return W.config1()
    if name == "fullscale1M":
        return W.config5()
    return W.config3()


TRAFFIC_JSON = os.path.join(ROOT, "profiles", "pair_kernel_traffic.json")
COPY_BYTES = 512 * 2 ** 20


def pair_kernel_source_hash():
    h = hashlib.sha256()
    for f in ("lub_pair.hip", "lub_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1308_6482_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def pair_kernel_traffic(precision):
    """HBM bytes per launch of the pair kernel from the committed counter
    summary, if it was taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_JSON):
        return None
    rec = json.load(open(TRAFFIC_JSON))
    if rec.get("source_sha256") != pair_kernel_source_hash():
        return None
    return rec.get(precision, {}).get("bytes_per_launch")


def _counter_means(directory, counter):
    """Mean value of `counter` per dispatch, number of dispatches and largest
    value, by kernel name, over every counter_collection.csv under
    `directory`."""
    import csv
    import glob
    tot, num, big = {}, {}, {}
    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {directory}")
    for fn in files:
        for row in csv.DictReader(open(fn)):
            if row["Counter_Name"] != counter:
                continue
            k = row["Kernel_Name"]
            v = float(row["Counter_Value"])
            tot[k] = tot.get(k, 0.0) + v
            num[k] = num.get(k, 0) + 1
            big[k] = max(big.get(k, 0.0), v)
    return {k: (tot[k] / num[k], num[k], big[k]) for k in tot}


def traffic_summary(fetch_dir, write_dir, precision):
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the pair kernel, each
    scaled by bytes / reading of the calibration copy (512 MiB read and
    written by one kernel); writes the JSON the bench line reads."""
    fe = _counter_means(fetch_dir, "FETCH_SIZE")
    wr = _counter_means(write_dir, "WRITE_SIZE")

    def copy_kernel(tab):
        # the calibration dispatch is the largest one of the copy kernel
        for k in tab:
            if "copyBuffer" in k:
                return k
        big = [k for k in tab if "elementwise" in k]
        return max(big, key=lambda k: tab[k][2]) if big else None

    kf, kw = copy_kernel(fe), copy_kernel(wr)
    if kf is None or kw is None:
        raise SystemExit("no calibration copy kernel in the counter runs")
    f_fetch = COPY_BYTES / (fe[kf][2] * 1024.0)
    f_write = COPY_BYTES / (wr[kw][2] * 1024.0)
    # the main pass of the pair stage (the tangent-sphere pass is k_pairs<R, true>)
    kern = [k for k in fe if "k_pairs" in k and "true>" not in k]
    if len(kern) != 1:
        raise SystemExit(f"expected one main pair kernel, found {kern}")
    kp = kern[0]
    fetch_b = fe[kp][0] * 1024.0 * f_fetch
    write_b = wr[kp][0] * 1024.0 * f_write
    rec = json.load(open(TRAFFIC_JSON)) if os.path.exists(TRAFFIC_JSON) else {}
    if rec.get("source_sha256") != pair_kernel_source_hash():
        rec = {}
    rec["source_sha256"] = pair_kernel_source_hash()
    rec[precision] = dict(kernel=kp, dispatches=fe[kp][1], fetch_kib=fe[kp][0],
                          write_kib=wr[kp][0], copy_kernel=kf, copy_fetch_kib=fe[kf][2],
                          copy_write_kib=wr[kw][2], scale_fetch=f_fetch, scale_write=f_write,
                          bytes_per_launch=fetch_b + write_b)
    os.makedirs(os.path.dirname(TRAFFIC_JSON), exist_ok=True)
    json.dump(rec, open(TRAFFIC_JSON, "w"), indent=1, sort_keys=True)
    others = {k: (fe[k][0] * 1024.0 * f_fetch, wr.get(k, (0.0, 0))[0] * 1024.0 * f_write)
              for k in fe if k.startswith("lub::") or "k_" in k}
    print(json.dumps(dict(pair_kernel=rec[precision],
                          per_kernel_bytes={k: dict(fetch=a, write=b)
                                            for k, (a, b) in others.items()}), indent=1))


def cpu_baseline(wl, seconds, gpu_pairs):
    """The FP64 oracle on the host cores over the same suspension, plus the
    error of the GPU pair results against it.  Up to 200,000 particles:
    whole evaluations repeated for about `seconds`.  Larger systems (whose
    whole evaluation by the oracle's brute-force pair search would take far
    longer): all pairs of a random sample of particles, sized to about
    `seconds`, and the accuracy on the pairs touching a 1% sample."""
    import numpy as np
    import oracle
    dom = oracle.make_domain(**wl.domain())
    P = oracle.make_params(**wl.params)
    if wl.n <= 200_000:
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
        sample = (f"whole evaluations of the same {wl.n}-particle suspension, "
                  f"{reps} repeats in {el:.1f} s")
        ij = gpu_pairs["ij"]
        res = gpu_pairs
    else:
        rng = np.random.default_rng(3)
        m = 64
        while True:
            idx = np.sort(rng.choice(wl.n, size=m, replace=False))
            t0 = time.perf_counter()
            _, _, st = oracle.compute_subset(wl.r, wl.q, wl.semi, wl.v, wl.w, dom, P, idx)
            el = time.perf_counter() - t0
            if el >= 0.3 * seconds or m >= 1 << 16:
                break
            m *= 4
        # each active pair is counted once per sampled end, as the oracle
        # evaluates it once per sampled end
        value = st["active"] / el
        sample = (f"all pairs of {m} random particles of the {wl.n}-particle suspension "
                  f"(brute-force partner search included), {el:.1f} s")
        # accuracy: the GPU pairs touching a 1% sample
        keep = np.zeros(wl.n, dtype=bool)
        keep[rng.choice(wl.n, size=wl.n // 100, replace=False)] = True
        ij_all = gpu_pairs["ij"]
        sel = keep[ij_all[:, 0]] | ((ij_all[:, 1] >= 0) & keep[np.maximum(ij_all[:, 1], 0)])
        ij = ij_all[sel]
        res = {k: gpu_pairs[k][sel] for k in ("F", "Ti", "Tj")}
    # GPU accuracy on the checked pairs (force and torque, h/a >= 1e-3)
    F, Ti, Tj, h, status = oracle.eval_pairs(wl.r, wl.q, wl.semi, wl.v, wl.w, dom, P, ij)
    i, j = ij[:, 0], ij[:, 1]
    a = wl.semi[i].min(axis=1)
    a = np.where(j >= 0, np.minimum(a, wl.semi[np.maximum(j, 0)].min(axis=1)), a)
    act = (status == 0) & (h / a >= 1e-3)
    nF = np.linalg.norm(F, axis=1)
    eF = np.linalg.norm(res["F"] - F, axis=1)[act] / nF[act]
    sT = np.maximum(np.linalg.norm(Ti, axis=1), a * nF)[act]
    eT = np.linalg.norm(res["Ti"] - Ti, axis=1)[act] / sT
    return dict(value=value, unit="pairs/s", cores=int(st["threads"]), kind="oracle",
                sample=sample), \
        dict(pairs_checked=int(act.sum()), max_rel_err_force=float(eF.max()),
             max_rel_err_torque=float(eT.max()),
             p99_rel_err_force=float(np.quantile(eF, 0.99)))


def train_seed(L, torch, n_train, epochs):
    """Train the seed network on the GPU with the library's own kernels on
    constructed pairs shaped like the polydisperse suspension; returns the
    weights and a report (losses, held-out loss, wall time)."""
    import numpy as np
    from paper_1308_6482_amd import seed_data as S
    t0 = time.perf_counter()
    P = S.sample_pairs(seed=1, m=n_train)
    H = S.sample_pairs(seed=2, m=1 << 18)
    t_gen = time.perf_counter() - t0
    lb = L.Lub((100.0, 100.0, 100.0), (1, 1, 1),
               dict(mu=1 / 6, delta_n=0.67, delta_t=0.5, delta_r=0.25), 10.0)
    L.lub_mlp_init(lb.h, 1)
    X = torch.as_tensor(P["X"]).cuda()
    T = torch.as_tensor(P["T"]).cuda()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    losses = L.lub_mlp_train(lb.h, X, T, epochs=epochs, batch=4096, lr=2e-3, lr_decay=0.7)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    Xh = torch.as_tensor(H["X"]).cuda()
    Th = torch.as_tensor(H["T"]).cuda()
    held, _ = L.lub_mlp_grad(lb.h, Xh, Th)
    theta = L.lub_mlp_get_weights(lb.h)
    lb.close()
    return theta, dict(train_pairs=n_train, heldout_pairs=1 << 18, epochs=epochs,
                       epoch_loss=[float(x) for x in losses], heldout_loss=float(held),
                       generate_s=t_gen, train_s=t_train)


def neighbour_capacity(L, torch, wl, prec, skin=0.0):
    """One synchronous evaluation (the library widens its neighbour segments
    on demand) gives the largest candidate count (of the superset, with a
    skin); the timed handles, which run asynchronously, get that with
    headroom for moving particles."""
    lb = L.Lub.for_workload(wl, precision=prec, sync=1, skin=skin)
    lb.compute(*L.to_device(wl))
    deg = lb.stats()["max_degree"]
    lb.close()
    return min(512, 64 * -(-int(1.5 * deg + 1) // 64))


def _timed_loop(lb, torch, args, arrays, stream):
    """W untimed steps, then exactly K timed steps bracketed by device
    synchronisations; returns ms per step (wall clock)."""
    r, q, semi, v, w, f, t = arrays
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            lb.compute(r, q, semi, v, w, f, t, stream=stream)
        torch.cuda.synchronize()
        lb.reset_timers()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            lb.compute(r, q, semi, v, w, f, t, stream=stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    return (t1 - t0) * 1e3 / args.steps


def measure(L, torch, wl, prec, args, theta=None):
    """Two timed loops of `args.steps` evaluations each on one stream: the
    launch sequence replayed as a HIP graph (the headline), and eager
    launches with HIP events around each stage (stage times, pair-kernel
    duration).  Returns (stats of the event loop, ms per step with graphs,
    ms per step eager, outputs)."""
    mode = L.LUB_SEED_MLP if theta is not None else L.LUB_SEED_PLAIN
    r, q, semi, v, w = L.to_device(wl)
    f = torch.empty((wl.n, 3), dtype=torch.float64, device="cuda")
    t = torch.empty((wl.n, 3), dtype=torch.float64, device="cuda")
    arrays = (r, q, semi, v, w, f, t)
    stream = torch.cuda.Stream()
    results = {}
    for kind in ("graph", "eager"):
        kw = dict(graph=1) if kind == "graph" else dict(timing=1)
        lb = L.Lub.for_workload(wl, precision=prec, sync=0, seed_mode=mode,
                                max_neighbors=args.max_neighbors, **kw)
        if theta is not None:
            L.lub_mlp_set_weights(lb.h, theta)
        # first call: sizes the workspace; its statistics validate the inputs
        with torch.cuda.stream(stream):
            lb.compute(r, q, semi, v, w, f, t, stream=stream)
        torch.cuda.synchronize()
        st = lb.stats()
        if st["error"]:
            raise RuntimeError(f"lub_compute failed: {L.lub_strerror(st['error'])}")
        ms = _timed_loop(lb, torch, args, arrays, stream)
        st = lb.stats()
        lb.close()
        if st["error"] or st["unconverged"]:
            raise RuntimeError(f"invalid run: error={st['error']} "
                               f"unconverged={st['unconverged']}")
        results[kind] = (st, ms)
    return results["eager"][0], results["graph"][1], results["eager"][1], (f, t)


def trajectory(L, torch, wl, prec, args, warm, skin=0.0):
    """K evaluations along a moving suspension (positions advanced in place
    by v dt after each evaluation, graph replay), with or without the warm
    start, or (skin > 0) with reused neighbour lists;
    returns a report of the last evaluation and the timing."""
    import numpy as np
    r0, q, semi, v, w = L.to_device(wl)
    r = r0.clone()
    f = torch.empty((wl.n, 3), dtype=torch.float64, device="cuda")
    t = torch.empty((wl.n, 3), dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()
    cap = args.max_neighbors
    if skin > 0.0:
        # the superset needs wider segments
        cap = neighbour_capacity(L, torch, wl, prec, skin)
    lb = L.Lub.for_workload(wl, precision=prec, sync=0, graph=1, warm_start=int(warm),
                            max_neighbors=cap, skin=skin)
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            lb.compute(r, q, semi, v, w, f, t, stream=stream)
            r.add_(v, alpha=args.trajectory_dt)
        torch.cuda.synchronize()
        st0 = lb.stats()
        if st0["error"]:
            raise RuntimeError(f"lub_compute failed: {L.lub_strerror(st0['error'])}")
        t0 = time.perf_counter()
        for _ in range(args.steps):
            lb.compute(r, q, semi, v, w, f, t, stream=stream)
            r.add_(v, alpha=args.trajectory_dt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    st = lb.stats()
    lb.close()
    if st["error"]:
        raise RuntimeError(f"invalid run: error={L.lub_strerror(st['error'])}")
    ms = (t1 - t0) * 1e3 / args.steps
    hist = np.array(st["iter_hist"], dtype=np.int64)
    cdf = np.cumsum(hist) / max(hist.sum(), 1)
    extra = {}
    if skin > 0.0:
        extra = dict(skin=skin, list_searches=st["list_builds"] - st0["list_builds"],
                     calls=args.steps)
    return dict(value=st["active"] / (ms * 1e-3), ms_per_step=ms, active=st["active"],
                overlaps=st["overlaps"], evaluated=st["evaluated"],
                unconverged=st["unconverged"], unresolved=st["unresolved"],
                warm_seeded=st["warm_seeded"], fallbacks=st["fallbacks"],
                newton_iters_mean=st["newton_iters"] / max(st["evaluated"], 1),
                newton_iters_p50=int(np.searchsorted(cdf, 0.5)),
                newton_iters_p99=int(np.searchsorted(cdf, 0.99)),
                newton_max=st["newton_max"], **extra)


def dynamics(L, torch, args):
    """Lees-Edwards evaluation (graph replay), sub-stepped integration and
    the growth stage on a sheared periodic cube of 4096 prolates."""
    import numpy as np
    from paper_1308_6482_amd import workloads as W
    prec = L.LUB_MIXED if args.precision == "mixed" else L.LUB_FP64
    wl = W.sheared(n=4096)
    args = argparse.Namespace(**vars(args))
    args.max_neighbors = neighbour_capacity(L, torch, wl, prec)
    st, ms, ms_e, _ = measure(L, torch, wl, prec, args)
    out = dict(workload=wl.name, lees_edwards=dict(
        value=st["active"] / (ms * 1e-3), unit="pairs/s", ms_per_step=ms,
        ms_per_step_eager=ms_e, active=st["active"]))
    # integrator: sub-steps of 0.1 with the correction evaluated each time,
    # searching every sub-step or reusing the neighbour lists (skin 1)
    nsub = max(args.steps // 4, 1)
    for key, skin in (("integrator", 0.0), ("integrator_reused_lists", 1.0)):
        r, q, semi, v, w = L.to_device(wl)
        cap = args.max_neighbors if skin == 0.0 else neighbour_capacity(L, torch, wl, prec, skin)
        lb = L.Lub.for_workload(wl, precision=prec, sync=0, max_neighbors=cap, skin=skin)
        f = torch.empty((wl.n, 3), dtype=torch.float64, device="cuda")
        t = torch.empty_like(f)
        lb.integrate(r, q, semi, v, w, 0.1, 5, f=f, t=t)
        torch.cuda.synchronize()
        b0 = lb.stats()["list_builds"]
        t0 = time.perf_counter()
        lb.integrate(r, q, semi, v, w, 0.1, nsub, f=f, t=t)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sti = lb.stats()
        lb.close()
        if sti["error"]:
            raise RuntimeError(f"lub_integrate failed: {L.lub_strerror(sti['error'])}")
        out[key] = dict(substeps=nsub, dt=0.1, ms_per_substep=(t1 - t0) * 1e3 / nsub,
                        active_last=sti["active"])
        if skin > 0.0:
            out[key].update(skin=skin, list_searches=sti["list_builds"] - b0)
    # growth stage: 4096 polydisperse spheroids from 30 % size to volume
    # fraction 0.45, 1200 steps
    rng = np.random.default_rng(7)
    n = 4096
    sm = W.polydisperse_semi(rng, n, 0.5, 2.0, 3.0, 5.0)
    vol = float(np.sum(4.0 / 3.0 * np.pi * sm[:, 0] * sm[:, 1] ** 2))
    Lx = (vol / 0.45) ** (1.0 / 3.0)
    r0, q0, _ = W.rsa(rng, sm * 0.3, (Lx, Lx, Lx), (1, 1, 1))
    params = dict(mu=1.0 / 6.0, delta_n=0.67, delta_t=0.5, delta_r=0.25, h_c=0.01,
                  eps_c=100.0)
    lb = L.Lub((Lx, Lx, Lx), (1, 1, 1), params, 1.05 * float(sm.max()), precision=prec)
    dev = [torch.as_tensor(x, dtype=torch.float64, device="cuda")
           for x in (r0, q0, sm, np.zeros_like(r0), np.zeros_like(r0))]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lb.grow(*dev, n_steps=1200, scale0=0.3, scale1=1.05, dt=0.2, density=1.0, damping=1.0,
            h_c=0.3, eps_c=1000.0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lb.close()
    out["growth"] = dict(n=n, phi=0.45, steps=1200, seconds=t1 - t0,
                         ms_per_step=(t1 - t0) * 1e3 / 1200)
    return out


def link_laws(L, torch, args):
    """The link-wise laws (Ding and Aidun; Clausen's averaged normal) on
    2347 spheres of radius 4 in a periodic 128^3 lattice (volume fraction
    0.3), graph replay; FP64."""
    from paper_1308_6482_amd import workloads as W
    wl0 = W.lattice_box()
    out = dict(workload=wl0.name)
    for name, model in (("link", L.LUB_MODEL_LINK), ("link_navg", L.LUB_MODEL_LINK_NAVG)):
        wl = wl0.with_params(model=model, h_c=0.0, eps_c=0.0)
        a2 = argparse.Namespace(**vars(args))
        a2.max_neighbors = neighbour_capacity(L, torch, wl, L.LUB_FP64)
        st, ms, ms_e, _ = measure(L, torch, wl, L.LUB_FP64, a2)
        out[name] = dict(value=st["active"] / (ms * 1e-3), unit="pairs/s", ms_per_step=ms,
                         ms_per_step_eager=ms_e, active=st["active"],
                         evaluated=st["evaluated"], links=st["newton_iters"],
                         links_per_s=st["newton_iters"] / (ms * 1e-3),
                         pair_stage_ms=st["stage_ms"][2] / max(st["timed_calls"], 1))
    return out


def summary(st, ms, args, ms_eager=None):
    active = st["active"]
    # the pair kernel's own duration, from events stamped by its dispatch
    pair_ms = st["pair_kernel_ms"] / max(st["timed_calls"], 1)
    flops = (FLOPS_EVAL * st["evaluated"] + FLOPS_ITER * st["newton_iters"]
             + FLOPS_POST[args.precision] * active)
    return dict(value=active / (ms * 1e-3), ms_per_step=ms, ms_per_step_eager=ms_eager,
                newton_iters_mean=st["newton_iters"] / max(st["evaluated"], 1),
                newton_max=st["newton_max"], fallbacks=st["fallbacks"],
                pair_kernel_ms=pair_ms, flops_per_launch=flops,
                achieved_tflops=flops / (pair_ms * 1e-3) / 1e12,
                stage_ms={k: v_ / max(st["timed_calls"], 1) for k, v_ in zip(
                    ["cells", "neighbours", "pairs", "reduction"], st["stage_ms"])})


def main():
    args = parse()
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary, args.precision)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np  # noqa: F401
    import torch
    from paper_1308_6482_amd import lub as L

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    models = {"full": L.LUB_MODEL_FULL, "normal": L.LUB_MODEL_NORMAL, "ladd": L.LUB_MODEL_LADD}
    wl = workload(args.workload).with_params(model=models[args.model])
    prec = L.LUB_MIXED if args.precision == "mixed" else L.LUB_FP64
    args.max_neighbors = neighbour_capacity(L, torch, wl, prec)
    if args.trajectory_dt is None:
        args.trajectory_dt = 1.0 if args.workload == "fullscale1M" else 0.1
    forms = {}
    mlp_report = None
    theta = None
    if args.seed in ("mlp", "both"):
        theta, mlp_report = train_seed(L, torch, args.train_pairs, args.train_epochs)
    if args.seed in ("plain", "both"):
        st, ms, ms_e, out_plain = measure(L, torch, wl, prec, args)
        forms["plain"] = (st, ms, ms_e)
    if args.seed in ("mlp", "both"):
        st, ms, ms_e, out_mlp = measure(L, torch, wl, prec, args, theta)
        forms["mlp"] = (st, ms, ms_e)
        if "plain" in forms:
            # equal accuracy: the same converged closest points
            fp, tp = out_plain
            fm, tm = out_mlp
            mlp_report["max_rel_diff_vs_plain"] = float(max(
                (fm - fp).abs().max() / fp.abs().max(), (tm - tp).abs().max() / tp.abs().max()))
    head = "mlp" if args.seed == "mlp" else "plain"
    st, ms, ms_e = forms[head]
    if args.calibrate_copy:
        # a plain copy of known size (512 MiB read, 512 MiB written) as the
        # reference reading of the traffic counters; a device-to-device copy
        # and, in case the copy runs on a DMA engine, an elementwise kernel
        x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
    sm = summary(st, ms, args, ms_e)
    active = st["active"]
    res = dict(
        metric="lubrication-corrected pairs/sec on 1 GPU at rel err <=1e-5 vs FP64 oracle",
        value=sm["value"], unit="pairs/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=ms, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64+f32" if args.precision == "mixed" else "f64",
        data="synthetic (seeded random sequential addition, simple-shear velocities)",
        config=dict(workload=wl.name, n_particles=wl.n, box=list(wl.L),
                    periodic=list(wl.periodic), walls=wl.n_walls, seed=0,
                    precision=args.precision, newton_seed=head,
                    cutoffs=[wl.params["delta_n"], wl.params["delta_t"], wl.params["delta_r"]],
                    h_c=wl.params["h_c"], eps_c=wl.params["eps_c"], mu=wl.params["mu"],
                    model=args.model,
                    launch="HIP graph replay", parallelism="single GPU"),
        pairs=dict(candidates=st["candidates"], wall_candidates=st["wall_candidates"],
                   evaluated=st["evaluated"], active=active, overlaps=st["overlaps"],
                   newton_iters_mean=sm["newton_iters_mean"], newton_max=st["newton_max"]),
        ms_per_step_eager=ms_e,
        stage_ms=sm["stage_ms"],
        roofline=dict(bound="alu", kernel="k_pairs (main pass)", achieved=sm["achieved_tflops"],
                      peak=PEAK_ALU_TFLOPS, unit="TFLOP/s",
                      frac=sm["achieved_tflops"] / PEAK_ALU_TFLOPS,
                      flops_per_launch=sm["flops_per_launch"], launch_ms=sm["pair_kernel_ms"],
                      traffic=pair_kernel_traffic(args.precision)),
        seed_forms={k: summary(v_[0], v_[1], args, v_[2]) for k, v_ in forms.items()},
    )
    if mlp_report:
        res["mlp_seed"] = mlp_report
    if args.trajectory_dt > 0:
        # the paper's continuation between time steps: the same moving
        # suspension with and without the warm start (last evaluation's counts)
        res["warm_start"] = dict(
            dt=args.trajectory_dt,
            warm=trajectory(L, torch, wl, prec, args, True),
            plain=trajectory(L, torch, wl, prec, args, False))
        skins = args.skin
        if skins is None:
            skins = [4.0] if args.workload == "fullscale1M" else [1.0]
        for sk in skins:
            res["warm_start"][f"reused_lists_skin{sk:g}"] = trajectory(L, torch, wl, prec,
                                                                      args, False, sk)
            # with the warm start kept per superset entry
            res["warm_start"][f"reused_lists_warm_skin{sk:g}"] = trajectory(
                L, torch, wl, prec, args, True, sk)
    if args.compare_models and args.model == "full":
        # the paper's "normal only" comparison model on the same suspension
        wn = wl.with_params(model=L.LUB_MODEL_NORMAL)
        stn, msn, msn_e, _ = measure(L, torch, wn, prec, args)
        res["models"] = {"normal": dict(value=stn["active"] / (msn * 1e-3), ms_per_step=msn,
                                        ms_per_step_eager=msn_e, active=stn["active"],
                                        newton_iters_mean=stn["newton_iters"]
                                        / max(stn["evaluated"], 1))}
    if args.dynamics:
        res["dynamics"] = dynamics(L, torch, args)
        res["link_laws"] = link_laws(L, torch, args)
    if args.cpu_seconds > 0:
        lb2 = L.Lub.for_workload(wl, precision=prec)
        r, q, semi, v, w = L.to_device(wl)
        lb2.compute(r, q, semi, v, w)
        pr = lb2.pair_results()
        lb2.close()
        cb, acc = cpu_baseline(wl, args.cpu_seconds, pr)
        res["cpu_baseline"] = cb
        res["accuracy"] = acc
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
