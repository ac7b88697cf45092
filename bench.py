#!/usr/bin/env python
"""Benchmark of the lubrication correction on one MI355X.

Metric: lubrication-corrected pairs per second (pairs with a non-zero
correction, particle-particle and particle-wall) with the inputs resident
in HBM.  A step is one full evaluation (staging, cell list, neighbour
lists, closest points, geometry, resistance, transfer, per-particle sums)
followed by the advance of the suspension by one time step.

Default workload (the full-scale configuration): 1,048,576 spheroids with
aspect ratios log-uniform in [1/4, 4] and R_perp in [4, 8] at volume
fraction 0.5 in a 2048 x 2048 x 680 box, periodic in x and y, walls at
z = 0 and z = L, placed by the paper's growth method (Sec. IV.C) and moving
in a simple shear field; mixed precision.  Between evaluations the
positions advance by v dt and the orientations by the angular velocity
(dt = 1).  The timed steps are steps W .. W+K-1 of that trajectory; the
100-evaluation protocol (per-step counts, Newton iteration percentiles,
accuracy against the FP64 oracle on a 1 % particle sample every 10th step)
runs the same trajectory untimed.

Prints one JSON line.  --gpus N with N > 1 exits: the benchmark runs on one
GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of the pair kernel per unit, counted from the kernel's
# source by an operation-counting host build (adds and multiplies, FMA = 2;
# divisions, square roots and logarithms listed apart and not counted):
#   per evaluated pair (set-up and final evaluation): 144 FP64 flops (the
#     count of 100 with the line of centres as the start, plus 44 for the
#     plain start (M_i + M_j)^-1 d: sums 6, cofactors 18, product 15, norm 5
#     and sign check 5, against 5 for normalising d)
#   per Newton iteration (incl. line-search trials):  306 FP64 flops
#   per active pair, LUB_MIXED: 225 FP64 + 450 FP32 flops; LUB_FP64: 675 FP64
FLOPS_EVAL = 144
FLOPS_ITER = 306
FLOPS_POST = {"mixed": (225, 450), "fp64": (675, 0)}
# Neighbour search per candidate pair (both directions of the centre test and
# the support-function reject of the owned entry): 55 FP64 flops
FLOPS_CAND = 55
# MI355X vector ALU peak, non-packed FMA: 256 CUs x 64 lanes x 2 flops x 2.4 GHz
# (the same for FP64 and unpacked FP32; packed FP32 is not used)
PEAK_ALU_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
METRIC = "lubrication-corrected pairs/sec on 1 GPU at rel err <=1e-5 vs FP64 oracle"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--workload", choices=["fullscale1M", "prolates4096", "spheres36",
                                           "polydisperse65536"], default="fullscale1M")
    ap.add_argument("--dt", type=float, default=None,
                    help="time step of the trajectory (default 1 for the full-scale "
                         "system, 0.1 otherwise)")
    ap.add_argument("--protocol-steps", type=int, default=100,
                    help="evaluations of the untimed protocol pass (counts, iteration "
                         "percentiles, accuracy every --snap-every steps)")
    ap.add_argument("--snap-every", type=int, default=10)
    ap.add_argument("--sample-frac", type=float, default=0.01,
                    help="particle sample of the accuracy checks (full-scale system)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="budget of the CPU oracle baseline (0: skip the oracle leg)")
    ap.add_argument("--seed", choices=["plain", "mlp", "warm", "both"], default="both",
                    help="Newton start: line of centres, learned network, previous "
                         "evaluation's normal (warm), or all three (both); the JSON value "
                         "is the plain form unless one form is chosen")
    ap.add_argument("--extras", type=int, default=1,
                    help="also run the variants (warm start, reused lists, normal-only "
                         "law), the 4096-prolate single-evaluation leg, the dynamics "
                         "and the link-wise laws (1) or not (0)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 512 MiB device copy after the timed region "
                         "(reference for the HBM traffic counters)")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no GPU work: read two rocprofv3 --pmc runs of this script with "
                         "--calibrate-copy (FETCH_SIZE, then WRITE_SIZE), scale each by the "
                         "copy kernel's reading and write profiles/kernel_traffic.json")
    ap.add_argument("--heldout-pairs", type=int, default=1 << 18,
                    help="the learned seed's held-out pairs (oracle-labelled) evaluated "
                         "with both starts (part of the oracle leg; 0: skip)")
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


# ---------------------------------------------------------------------------
# HBM traffic of the dominant kernels from two rocprofv3 --pmc runs
# ---------------------------------------------------------------------------

TRAFFIC_JSON = os.path.join(ROOT, "profiles", "kernel_traffic.json")
COPY_BYTES = 512 * 2 ** 20
TRAFFIC_SOURCES = {"k_pairs": ("lub_pair.hip", "lub_newton.h", "lub_internal.h"),
                   "k_neighbors": ("lub_neighbors.hip", "lub_internal.h")}


def kernel_source_hash(kind):
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES[kind]:
        h.update(open(os.path.join(ROOT, "paper_1308_6482_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def kernel_traffic(kind, workload_name, precision):
    """HBM bytes per launch of a kernel from the committed counter summary,
    if it was taken on the current kernel source and workload."""
    if not os.path.exists(TRAFFIC_JSON):
        return None
    rec = json.load(open(TRAFFIC_JSON)).get(kind, {})
    if rec.get("source_sha256") != kernel_source_hash(kind):
        return None
    ent = rec.get(f"{workload_name}/{precision}")
    return ent.get("bytes_per_launch") if ent else None


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


def traffic_summary(fetch_dir, write_dir, workload_name, precision):
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the main pair pass and
    the neighbour search, each scaled by bytes / reading of the calibration
    copy (512 MiB read and written by one kernel); writes the JSON the bench
    line reads."""
    fe = _counter_means(fetch_dir, "FETCH_SIZE")
    wr = _counter_means(write_dir, "WRITE_SIZE")

    def copy_kernel(tab):
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
    rec = json.load(open(TRAFFIC_JSON)) if os.path.exists(TRAFFIC_JSON) else {}
    out = {}
    for kind, pick in (("k_pairs", lambda k: "k_pairs" in k and "true>" not in k),
                       ("k_neighbors", lambda k: "k_neighbors" in k)):
        names = [k for k in fe if pick(k)]
        if not names:
            continue
        # the most frequent instantiation (the probe before the timed region
        # may use another lane-group size)
        kp = max(names, key=lambda k: fe[k][1])
        ent = dict(kernel=kp, dispatches=fe[kp][1], fetch_kib=fe[kp][0],
                   write_kib=wr.get(kp, (0.0,))[0], copy_kernel=kf,
                   copy_fetch_kib=fe[kf][2], copy_write_kib=wr[kw][2], scale_fetch=f_fetch,
                   scale_write=f_write,
                   bytes_per_launch=fe[kp][0] * 1024.0 * f_fetch
                   + wr.get(kp, (0.0,))[0] * 1024.0 * f_write)
        r = rec.get(kind, {})
        if r.get("source_sha256") != kernel_source_hash(kind):
            r = {}
        r["source_sha256"] = kernel_source_hash(kind)
        r[f"{workload_name}/{precision}"] = ent
        rec[kind] = r
        out[kind] = ent
    os.makedirs(os.path.dirname(TRAFFIC_JSON), exist_ok=True)
    json.dump(rec, open(TRAFFIC_JSON, "w"), indent=1, sort_keys=True)
    print(json.dumps(out, indent=1))


# ---------------------------------------------------------------------------
# learned seed
# ---------------------------------------------------------------------------

def train_seed(L, torch, n_train, epochs):
    """Train the seed network on the GPU with the library's own kernels on
    constructed pairs shaped like the polydisperse suspension; returns the
    weights and a report (losses, held-out loss, wall time)."""
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


# ---------------------------------------------------------------------------
# the trajectory
# ---------------------------------------------------------------------------

def advance(lb, r, q, v, w, dt):
    """One time step of the suspension in place, by the library's kinematic
    advance (one kernel on the current stream): r += v dt, and the
    orientation q <- normalise(q + dt/2 (0, w) q) (quaternion product)."""
    lb.advance(r, q, v, w, dt)


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


def make_handle(L, wl, prec, cap, theta=None, **kw):
    mode = L.LUB_SEED_MLP if theta is not None else L.LUB_SEED_PLAIN
    lb = L.Lub.for_workload(wl, precision=prec, seed_mode=mode, max_neighbors=cap, **kw)
    if theta is not None:
        L.lub_mlp_set_weights(lb.h, theta)
    return lb


def percentile_iters(hist, p):
    import numpy as np
    hist = np.asarray(hist, dtype=np.int64)
    cdf = np.cumsum(hist) / max(hist.sum(), 1)
    return int(np.searchsorted(cdf, p))


def protocol_pass(L, torch, wl, prec, args, cap, theta=None, sample=None, **kw):
    """The trajectory untimed, with the statistics of every step and, every
    args.snap_every steps, a snapshot of the state and of the pairs touching
    the particle sample (for the oracle checks)."""
    import numpy as np
    r, q, semi, v, w = L.to_device(wl)
    lb = make_handle(L, wl, prec, cap, theta, sync=0, **kw)
    steps = []
    snaps = []
    hist = np.zeros(32, dtype=np.int64)
    for k in range(args.protocol_steps):
        lb.compute(r, q, semi, v, w)
        st = lb.stats()
        if st["error"]:
            raise RuntimeError(f"lub_compute failed at step {k}: {L.lub_strerror(st['error'])}")
        steps.append({key: st[key] for key in ("active", "evaluated", "candidates",
                                                "wall_candidates", "overlaps", "unresolved",
                                                "unconverged", "fallbacks", "newton_iters",
                                                "newton_max", "warm_seeded", "list_builds")})
        hist += np.asarray(st["iter_hist"], dtype=np.int64)
        if sample is not None and args.snap_every > 0 and k % args.snap_every == 0:
            pr = lb.pair_results()
            ij = pr["ij"]
            sel = sample[ij[:, 0]] | ((ij[:, 1] >= 0) & sample[np.maximum(ij[:, 1], 0)])
            snaps.append(dict(step=k, r=r.cpu().numpy(), q=q.cpu().numpy(),
                              pairs={key: pr[key][sel] for key in pr}))
        advance(lb, r, q, v, w, args.dt)
    torch.cuda.synchronize()
    lb.close()
    act = np.array([s["active"] for s in steps], dtype=np.int64)
    ev = np.array([s["evaluated"] for s in steps], dtype=np.int64)
    it = np.array([s["newton_iters"] for s in steps], dtype=np.int64)
    summary = dict(steps=args.protocol_steps, dt=args.dt,
                   active_first=int(act[0]), active_last=int(act[-1]),
                   active_mean=float(act.mean()), evaluated_mean=float(ev.mean()),
                   candidates_mean=float(np.mean([s["candidates"] for s in steps])),
                   overlaps_max=int(max(s["overlaps"] for s in steps)),
                   unresolved_max=int(max(s["unresolved"] for s in steps)),
                   unconverged_total=int(sum(s["unconverged"] for s in steps)),
                   fallbacks_total=int(sum(s["fallbacks"] for s in steps)),
                   warm_seeded_total=int(sum(s["warm_seeded"] for s in steps)),
                   newton_iters_mean=float(it.sum() / max(ev.sum(), 1)),
                   newton_iters_p50=percentile_iters(hist, 0.5),
                   newton_iters_p99=percentile_iters(hist, 0.99),
                   newton_max=int(max(s["newton_max"] for s in steps)),
                   list_searches=int(steps[-1]["list_builds"] - steps[0]["list_builds"] + 1)
                   if kw.get("skin", 0.0) > 0.0 else args.protocol_steps)
    return summary, steps, snaps


def timed_pass(L, torch, wl, prec, args, cap, theta=None, **kw):
    """W untimed steps, then exactly K timed steps of the trajectory (graph
    replay), bracketed by device synchronisations; returns ms per step."""
    r, q, semi, v, w = L.to_device(wl)
    f = torch.empty((wl.n, 3), dtype=torch.float64, device="cuda")
    t = torch.empty_like(f)
    stream = torch.cuda.Stream()
    lb = make_handle(L, wl, prec, cap, theta, sync=0, graph=1, **kw)
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            lb.compute(r, q, semi, v, w, f, t, stream=stream)
            advance(lb, r, q, v, w, args.dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            lb.compute(r, q, semi, v, w, f, t, stream=stream)
            advance(lb, r, q, v, w, args.dt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    st = lb.stats()
    lb.close()
    if st["error"]:
        raise RuntimeError(f"invalid timed run: {L.lub_strerror(st['error'])}")
    return (t1 - t0) * 1e3 / args.steps


def eager_pass(L, torch, wl, prec, args, cap, theta=None, **kw):
    """The same K steps launched eagerly with HIP events around each stage
    and the pair kernel's own dispatch stamps; returns per-step stage times
    (ms) and the pair-kernel duration, averaged over the K steps."""
    r, q, semi, v, w = L.to_device(wl)
    f = torch.empty((wl.n, 3), dtype=torch.float64, device="cuda")
    t = torch.empty_like(f)
    stream = torch.cuda.Stream()
    lb = make_handle(L, wl, prec, cap, theta, sync=0, timing=1, **kw)
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            lb.compute(r, q, semi, v, w, f, t, stream=stream)
            advance(lb, r, q, v, w, args.dt)
        torch.cuda.synchronize()
        lb.reset_timers()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            lb.compute(r, q, semi, v, w, f, t, stream=stream)
            advance(lb, r, q, v, w, args.dt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    st = lb.stats()
    lb.close()
    n = max(st["timed_calls"], 1)
    return dict(ms_per_step_eager=(t1 - t0) * 1e3 / args.steps,
                stage_ms={k: v_ / n for k, v_ in zip(
                    ["cells", "neighbours", "pairs", "reduction"], st["stage_ms"])},
                pair_kernel_ms=st["pair_kernel_ms"] / n,
                search_kernel_ms=st["search_kernel_ms"] / n)


def measure_form(L, torch, wl, prec, args, cap, theta=None, sample=None, **kw):
    """Protocol pass, timed pass and eager pass of one form on the trajectory."""
    summary, steps, snaps = protocol_pass(L, torch, wl, prec, args, cap, theta, sample, **kw)
    ms = timed_pass(L, torch, wl, prec, args, cap, theta, **kw)
    # the protocol pass ran the same trajectory: its counts of the timed
    # steps W .. W+K-1 (the evaluation is deterministic)
    window = steps[args.warmup:args.warmup + args.steps]
    timed_active = sum(s_["active"] for s_ in window)
    ev = eager_pass(L, torch, wl, prec, args, cap, theta, **kw)
    out = dict(value=timed_active / (args.steps * ms * 1e-3), unit="pairs/s", ms_per_step=ms,
               active_per_step_timed=timed_active / args.steps, protocol=summary, **ev)
    return out, snaps, window


def detail_snapshot(L, torch, wl, prec, cap, sample):
    """One evaluation of the initial state with the per-pair intermediate
    results recorded (closest points, gap direction, frame axis, the 16
    corrective elements), restricted to the pairs touching the sample."""
    import numpy as np
    lb = make_handle(L, wl, prec, cap, None, sync=1, record_detail=1)
    lb.compute(*L.to_device(wl))
    pr = lb.pair_results()
    dt = lb.pair_detail()
    lb.close()
    ij = pr["ij"]
    sel = sample[ij[:, 0]] | ((ij[:, 1] >= 0) & sample[np.maximum(ij[:, 1], 0)])
    out = {k: v[sel] for k, v in pr.items()}
    out.update({k: v[sel] for k, v in dt.items()})
    return out


KIDX = [(0, 0), (0, 1), (0, 2), (0, 3), (0, 4), (1, 1), (1, 2), (1, 3), (1, 4), (2, 2),
        (2, 3), (2, 4), (2, 5), (3, 3), (3, 4), (4, 4)]


def per_output_errors(wl, det, oracle, dom, P):
    """Every output of the pair path against the oracle on the same pairs:
    the gap, the closest points, the gap direction, each corrective element
    (relative to the pair's largest element; pairs whose frame axis differs,
    at a spheroid's pole, are left out of the elements), force and torque."""
    import numpy as np
    ij = det["ij"]
    o = oracle.eval_pairs_detail(wl.r, wl.q, wl.semi, wl.v, wl.w, dom, P, ij)
    i, j = ij[:, 0], ij[:, 1]
    a = wl.semi[i].min(axis=1)
    a = np.where(j >= 0, np.minimum(a, wl.semi[np.maximum(j, 0)].min(axis=1)), a)
    act = o["status"] == 0
    gate = act & (o["h"] / a >= 1e-3)
    pp = act & (j >= 0)
    Ko = np.stack([o["Kt"][:, r_, c_] for r_, c_ in KIDX], axis=1)
    same = np.abs(np.sum(det["e1"] * o["e1"], axis=1) - 1.0) < 1e-9
    km = gate & same
    scale = np.maximum(np.abs(Ko).max(axis=1), 1e-300)
    ek = (np.abs(det["Kt"] - Ko) / scale[:, None])[km]
    nF = np.linalg.norm(o["F"], axis=1)
    eF = np.linalg.norm(det["F"] - o["F"], axis=1)[gate] / nF[gate]
    sT = np.maximum(np.linalg.norm(o["Ti"], axis=1), a * nF)[gate]
    eT = np.linalg.norm(det["Ti"] - o["Ti"], axis=1)[gate] / sT
    names = [f"K{r_ + 1}{c_ + 1}" for r_, c_ in KIDX]
    return dict(
        pairs=int(len(ij)), active=int(act.sum()), gated=int(gate.sum()),
        frame_differs=int((act & ~same).sum()),
        h_abs_over_a=float((np.abs(det["h"] - o["h"]) / a)[act].max()),
        h_rel=float((np.abs(det["h"] - o["h"]) / np.abs(o["h"]))[gate].max()),
        yi_over_a=float((np.linalg.norm(det["yi"] - o["yi"], axis=1) / a)[act].max()),
        yj_over_a=float((np.linalg.norm(det["yj"] - o["yj"], axis=1) / a)[pp].max()),
        n=float(np.linalg.norm(det["n"] - o["n"], axis=1)[act].max()),
        K={nm: float(ek[:, k].max()) if ek.size else 0.0 for k, nm in enumerate(names)},
        force=float(eF.max()), torque=float(eT.max()),
        lin_han_iters_mean=float(o["iters_lh"][act & (j >= 0)].mean()))


def roofline_entries(form, stats_k, args, wl_name):
    """Achieved / peak of the pair kernel and the neighbour search on the
    timed steps (counted work of the protocol's steps W..W+K-1 over the
    launch durations measured with events in the eager pass)."""
    post64, post32 = FLOPS_POST[args.precision]
    ev = sum(s["evaluated"] for s in stats_k)
    it = sum(s["newton_iters"] for s in stats_k)
    act = sum(s["active"] for s in stats_k)
    cand = sum(s["candidates"] for s in stats_k)
    k = max(len(stats_k), 1)
    flops_pair = (FLOPS_EVAL * ev + FLOPS_ITER * it + (post64 + post32) * act) / k
    flops_nbr = FLOPS_CAND * cand / k
    pair_ms = form["pair_kernel_ms"]
    nbr_ms = form["search_kernel_ms"]
    pair = dict(bound="alu", kernel="k_pairs (main pass)", unit="TFLOP/s",
                achieved=flops_pair / (pair_ms * 1e-3) / 1e12, peak=PEAK_ALU_TFLOPS,
                flops_per_launch=flops_pair, launch_ms=pair_ms,
                fp64_flops_per_launch=(FLOPS_EVAL * ev + FLOPS_ITER * it + post64 * act) / k,
                fp32_flops_per_launch=post32 * act / k,
                traffic=kernel_traffic("k_pairs", wl_name, args.precision))
    pair["frac"] = pair["achieved"] / PEAK_ALU_TFLOPS
    pair["frac_fp64"] = pair["fp64_flops_per_launch"] / (pair_ms * 1e-3) / 1e12 / PEAK_ALU_TFLOPS
    pair["frac_fp32"] = pair["fp32_flops_per_launch"] / (pair_ms * 1e-3) / 1e12 / PEAK_ALU_TFLOPS
    nbr = dict(bound="alu", kernel="k_neighbors_flat (neighbour search walk)", unit="TFLOP/s",
               achieved=flops_nbr / (nbr_ms * 1e-3) / 1e12, peak=PEAK_ALU_TFLOPS,
               flops_per_launch=flops_nbr, launch_ms=nbr_ms,
               stage_ms=form["stage_ms"]["neighbours"],
               traffic=kernel_traffic("k_neighbors", wl_name, args.precision))
    nbr["frac"] = nbr["achieved"] / PEAK_ALU_TFLOPS
    return pair, nbr


# ---------------------------------------------------------------------------
# the oracle leg: CPU baseline and accuracy (the only part that runs it)
# ---------------------------------------------------------------------------

def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def pair_errors(wl, r, q, pairs, ref, dom, P):
    """Errors of GPU pair results against the oracle's evaluation of the same
    pairs at the given state: force and torque (h/a >= 1e-3, per-pair
    scales) and the gap."""
    import numpy as np
    ij = pairs["ij"]
    F, Ti, Tj, h, status = ref.eval_pairs(r, q, wl.semi, wl.v, wl.w, dom, P, ij)
    i, j = ij[:, 0], ij[:, 1]
    a = wl.semi[i].min(axis=1)
    a = np.where(j >= 0, np.minimum(a, wl.semi[np.maximum(j, 0)].min(axis=1)), a)
    act = (status == 0) & (h / a >= 1e-3)
    nF = np.linalg.norm(F, axis=1)
    eF = np.linalg.norm(pairs["F"] - F, axis=1)[act] / nF[act]
    sT = np.maximum(np.linalg.norm(Ti, axis=1), a * nF)[act]
    eT = np.linalg.norm(pairs["Ti"] - Ti, axis=1)[act] / sT
    jj = j >= 0
    sTj = np.maximum(np.linalg.norm(Tj, axis=1), a * nF)[act & jj]
    eTj = np.linalg.norm(pairs["Tj"] - Tj, axis=1)[act & jj] / sTj
    eh = np.abs(pairs["h"] - h) / np.maximum(a, 1e-300)
    same_status = bool(np.array_equal(pairs["status"] == 0, status == 0))
    return dict(pairs=int(len(ij)), checked=int(act.sum()), status_equal=same_status,
                max_rel_err_force=float(eF.max()) if eF.size else 0.0,
                p99_rel_err_force=float(np.quantile(eF, 0.99)) if eF.size else 0.0,
                max_rel_err_torque=float(max(eT.max() if eT.size else 0.0,
                                             eTj.max() if eTj.size else 0.0)),
                max_abs_err_gap_over_a=float(eh.max()) if eh.size else 0.0)


def heldout_leg(L, torch, theta, prec, m):
    """The learned seed's held-out evaluation: m pairs placed by the oracle at
    gaps log-uniform in [1e-4, 1] of the smallest semi-axis (labels: the
    oracle's closest points), evaluated by the library as isolated pairs with
    the plain and the learned start (cut-offs widened so that every pair is
    solved): Newton iteration p50/p99, fallbacks, and |dh|/h, |dy*|/a
    against the labels."""
    import numpy as np
    from oracle import seed_pairs as SP
    from paper_1308_6482_amd import workloads as W
    t0 = time.perf_counter()
    P = SP.labelled_pairs(2, m)
    t_label = time.perf_counter() - t0
    ok = np.flatnonzero(P["status"] == 0)
    wl = W.pair_lattice(P["q_i"][ok], P["semi_i"][ok], P["q_j"][ok], P["semi_j"][ok],
                        P["d"][ok], name=f"heldout{m}")
    wl = wl.with_params(delta_n=10.0, delta_t=10.0, delta_r=10.0)
    a = np.minimum(P["semi_i"][ok].min(axis=1), P["semi_j"][ok].min(axis=1))
    out = dict(pairs=int(m), placed=int(ok.size), label_s=t_label)
    for form, th in (("plain", None), ("mlp", theta)):
        if form == "mlp" and th is None:
            continue
        lb = make_handle(L, wl, prec, 64, th, sync=1, record_detail=1)
        lb.compute(*L.to_device(wl))
        st = lb.stats()
        pr = lb.pair_results()
        dt = lb.pair_detail()
        lb.close()
        k = pr["ij"][:, 0] // 2
        it = pr["iters"]
        hist = np.bincount(np.minimum(it, 31), minlength=32)
        cdf = np.cumsum(hist) / max(hist.sum(), 1)
        solved = pr["status"] != 3
        dh = np.abs(pr["h"] - P["h"][ok][k]) / P["h"][ok][k]
        dyi = np.linalg.norm(dt["yi"] - P["yi"][ok][k], axis=1) / a[k]
        dyj = np.linalg.norm(dt["yj"] - P["yj"][ok][k], axis=1) / a[k]
        out[form] = dict(evaluated=int(len(k)), unconverged=int(st["unconverged"]),
                         fallbacks=int(st["fallbacks"]),
                         fallback_rate=float(st["fallbacks"] / max(len(k), 1)),
                         newton_iters_mean=float(it.mean()),
                         newton_iters_p50=int(np.searchsorted(cdf, 0.5)),
                         newton_iters_p99=int(np.searchsorted(cdf, 0.99)),
                         newton_max=int(it.max()), iter_hist=[int(x) for x in hist],
                         max_rel_err_h=float(dh[solved].max()),
                         max_err_y_over_a=float(max(dyi[solved].max(), dyj[solved].max())))
    return out


def cpu_leg(wl, snaps_by_form, seconds, det=None):
    """The FP64 oracle on the host cores: its pairs/s on the pairs the GPU
    evaluated around the particle sample at the first step (1 thread and all
    threads, median of 5 after a warm-up), and the accuracy of every
    snapshot of every form against it."""
    import numpy as np
    import oracle
    dom = oracle.make_domain(**wl.domain())
    P = oracle.make_params(**wl.params)
    first = snaps_by_form["plain"][0] if "plain" in snaps_by_form else \
        next(iter(snaps_by_form.values()))[0]
    ij = first["pairs"]["ij"]
    # bounded sample: as many of those pairs as one thread evaluates in
    # about seconds / 12 (6 runs of each thread count)
    t0 = time.perf_counter()
    oracle.eval_pairs(first["r"], first["q"], wl.semi, wl.v, wl.w, dom, P, ij[:2000],
                      nthreads=1)
    per_pair = (time.perf_counter() - t0) / min(len(ij), 2000)
    m = int(min(len(ij), max(2000, seconds / 12.0 / max(per_pair, 1e-9))))
    sub = ij[:m]

    def timed(nthreads):
        runs = []
        for k in range(6):
            t0 = time.perf_counter()
            F, Ti, Tj, h, st = oracle.eval_pairs(first["r"], first["q"], wl.semi, wl.v, wl.w,
                                                 dom, P, sub, nthreads=nthreads)
            runs.append(time.perf_counter() - t0)
        active = int(np.sum(st == 0))
        med = float(np.median(runs[1:]))
        return active / med, med, active

    v1, med1, act = timed(1)
    nthr = os.cpu_count() or 1
    vn, medn, _ = timed(nthr)
    _, _, st_all = oracle.compute_subset(first["r"], first["q"], wl.semi, wl.v, wl.w, dom, P,
                                         np.arange(min(64, wl.n)), nthreads=nthr)
    base = dict(value=vn, unit="pairs/s", cores=int(st_all["threads"]), kind="oracle",
                sample=(f"{m} pairs touching a {len(first['pairs']['ij'])}-pair neighbourhood "
                        f"of a particle sample at step 0 ({act} active), evaluated by the "
                        f"oracle's per-pair path; median of 5 after 1 warm-up"),
                value_1thread=v1, median_s_1thread=med1, median_s_all=medn,
                cpu_model=cpu_model(), host_cpus=nthr)
    acc = {}
    for form, snaps in snaps_by_form.items():
        per = [dict(step=s["step"], **pair_errors(wl, s["r"], s["q"], s["pairs"], oracle, dom, P))
               for s in snaps]
        acc[form] = dict(
            snapshots=len(per), pairs_checked=int(sum(p["checked"] for p in per)),
            max_rel_err_force=max(p["max_rel_err_force"] for p in per),
            max_rel_err_torque=max(p["max_rel_err_torque"] for p in per),
            p99_rel_err_force=max(p["p99_rel_err_force"] for p in per),
            max_abs_err_gap_over_a=max(p["max_abs_err_gap_over_a"] for p in per),
            status_equal=all(p["status_equal"] for p in per), per_snapshot=per)
    if det is not None:
        acc["per_output_step0"] = per_output_errors(wl, det, oracle, dom, P)
        base["lin_han_iters_mean"] = acc["per_output_step0"]["lin_han_iters_mean"]
    return base, acc


# ---------------------------------------------------------------------------
# secondary legs
# ---------------------------------------------------------------------------

def single_eval(L, torch, wl, prec, args, theta=None, **kw):
    """K graph-replayed evaluations of the same input, and an eager loop with
    stage events: ms per step, stage times, pair-kernel duration, counts."""
    r, q, semi, v, w = L.to_device(wl)
    f = torch.empty((wl.n, 3), dtype=torch.float64, device="cuda")
    t = torch.empty_like(f)
    stream = torch.cuda.Stream()
    cap = neighbour_capacity(L, torch, wl, prec)
    out = {}
    for kind in ("graph", "eager"):
        extra = dict(graph=1) if kind == "graph" else dict(timing=1)
        lb = make_handle(L, wl, prec, cap, theta, sync=0, **extra, **kw)
        with torch.cuda.stream(stream):
            for _ in range(args.warmup):
                lb.compute(r, q, semi, v, w, f, t, stream=stream)
            torch.cuda.synchronize()
            lb.reset_timers()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                lb.compute(r, q, semi, v, w, f, t, stream=stream)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
        st = lb.stats()
        lb.close()
        if st["error"] or st["unconverged"]:
            raise RuntimeError(f"invalid run: error={st['error']} unconverged={st['unconverged']}")
        out[kind] = (st, (t1 - t0) * 1e3 / args.steps)
    st, ms = out["graph"]
    ste, mse = out["eager"]
    n = max(ste["timed_calls"], 1)
    return dict(value=st["active"] / (ms * 1e-3), unit="pairs/s", ms_per_step=ms,
                ms_per_step_eager=mse, active=st["active"], evaluated=st["evaluated"],
                candidates=st["candidates"],
                newton_iters_mean=st["newton_iters"] / max(st["evaluated"], 1),
                newton_max=st["newton_max"], fallbacks=st["fallbacks"],
                pair_kernel_ms=ste["pair_kernel_ms"] / n,
                search_kernel_ms=ste["search_kernel_ms"] / n,
                stage_ms={k: v_ / n for k, v_ in zip(
                    ["cells", "neighbours", "pairs", "reduction"], ste["stage_ms"])}), \
        (f, t)


def dynamics(L, torch, args):
    """Lees-Edwards evaluation (graph replay), sub-stepped integration and
    the growth stage on a sheared periodic cube of 4096 prolates."""
    import numpy as np
    from paper_1308_6482_amd import workloads as W
    prec = L.LUB_MIXED if args.precision == "mixed" else L.LUB_FP64
    wl = W.sheared(n=4096)
    a2 = argparse.Namespace(**vars(args))
    a2.steps, a2.warmup = 50, 5
    le, _ = single_eval(L, torch, wl, prec, a2)
    out = dict(workload=wl.name, lees_edwards=dict(value=le["value"], unit="pairs/s",
                                                   ms_per_step=le["ms_per_step"],
                                                   active=le["active"]))
    nsub = 50
    for key, skin in (("integrator", 0.0), ("integrator_reused_lists", 1.0)):
        r, q, semi, v, w = L.to_device(wl)
        cap = neighbour_capacity(L, torch, wl, prec, skin)
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
    a2 = argparse.Namespace(**vars(args))
    a2.steps, a2.warmup = 20, 3
    for name, model in (("link", L.LUB_MODEL_LINK), ("link_navg", L.LUB_MODEL_LINK_NAVG)):
        wl = wl0.with_params(model=model, h_c=0.0, eps_c=0.0)
        s, _ = single_eval(L, torch, wl, L.LUB_FP64, a2)
        out[name] = dict(value=s["value"], unit="pairs/s", ms_per_step=s["ms_per_step"],
                         active=s["active"], evaluated=s["evaluated"],
                         pair_stage_ms=s["stage_ms"]["pairs"])
    return out


# ---------------------------------------------------------------------------

def main():
    args = parse()
    if args.traffic_summary:
        wl_name = "fullscale1M" if args.workload == "fullscale1M" else args.workload
        traffic_summary(*args.traffic_summary, wl_name, args.precision)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only (the build has no "
                                   "multi-GPU path); run it with --gpus 1"}), flush=True)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1308_6482_amd import lub as L

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    L.lib()
    if args.dt is None:
        args.dt = 1.0 if args.workload == "fullscale1M" else 0.1
    args.protocol_steps = max(args.protocol_steps, args.warmup + args.steps)
    prec = L.LUB_MIXED if args.precision == "mixed" else L.LUB_FP64
    t0 = time.perf_counter()
    wl = workload(args.workload)
    gen_s = time.perf_counter() - t0
    cap = neighbour_capacity(L, torch, wl, prec)
    sample = None
    if args.cpu_seconds > 0:
        rng = np.random.default_rng(3)
        sample = np.zeros(wl.n, dtype=bool)
        k = max(1, int(round(args.sample_frac * wl.n))) if wl.n > 20000 else wl.n
        sample[rng.choice(wl.n, size=k, replace=False)] = True

    theta, mlp_report = None, None
    if args.seed in ("mlp", "both"):
        from paper_1308_6482_amd import train_seed as TS
        theta, rec = TS.load_weights()
        if theta is not None:
            # trained on oracle-labelled pairs by train_seed.py (GPU); the
            # bench times a short training run of the same kernels beside
            _, speed = train_seed(L, torch, 1 << 18, 2)
            mlp_report = dict(weights="paper_1308_6482_amd/data/seed_weights.npz", training=rec,
                              training_speed_check=speed)
        else:
            theta, mlp_report = train_seed(L, torch, args.train_pairs, args.train_epochs)
            mlp_report["weights"] = "trained here on constructed pairs (no committed weights)"
    forms, snaps, windows = {}, {}, {}
    if args.seed in ("plain", "both"):
        forms["plain"], snaps["plain"], windows["plain"] = measure_form(
            L, torch, wl, prec, args, cap, sample=sample)
    if args.seed in ("mlp", "both"):
        forms["mlp"], snaps["mlp"], windows["mlp"] = measure_form(
            L, torch, wl, prec, args, cap, theta, sample=sample)
    if args.seed in ("warm", "both"):
        # the paper's continuation between time steps (Sec. III.A): each
        # pair's solve starts from its normal of the previous evaluation
        forms["warm"], snaps["warm"], windows["warm"] = measure_form(
            L, torch, wl, prec, args, cap, sample=sample, warm_start=1)
    head = {"mlp": "mlp", "warm": "warm"}.get(args.seed, "plain")
    hf = forms[head]
    pair_rl, nbr_rl = roofline_entries(hf, windows[head], args, args.workload)
    dominant = nbr_rl if nbr_rl["launch_ms"] >= pair_rl["launch_ms"] else pair_rl
    if args.calibrate_copy:
        # a plain copy of known size (512 MiB read, 512 MiB written) as the
        # reference reading of the traffic counters
        x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()

    res = dict(
        metric=METRIC, value=hf["value"], unit="pairs/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=hf["ms_per_step"], higher_is_better=True,
        scaling="weak", vs_baseline=None,
        dtype="f64+f32" if args.precision == "mixed" else "f64",
        data="synthetic (seeded; growth-method packing, simple-shear velocities)",
        config=dict(workload=wl.name, n_particles=wl.n, box=list(wl.L),
                    periodic=list(wl.periodic), walls=wl.n_walls, seed=0,
                    volume_fraction=wl.meta.get("phi"), precision=args.precision,
                    newton_seed=head, dt=args.dt,
                    cutoffs=[wl.params["delta_n"], wl.params["delta_t"],
                             wl.params["delta_r"]],
                    h_c=wl.params["h_c"], eps_c=wl.params["eps_c"], mu=wl.params["mu"],
                    launch="HIP graph replay", step="one evaluation + advance by dt",
                    parallelism="single GPU"),
        roofline=dict(dominant),
        roofline_pair_kernel=pair_rl, roofline_neighbour_search=nbr_rl,
        seed_forms=forms,
        generation=dict(seconds=gen_s, **{k: v_ for k, v_ in wl.meta.items()
                                          if k != "growth_stages"}),
    )
    res["roofline"]["frac"] = dominant["frac"]
    if mlp_report:
        res["mlp_seed"] = mlp_report
    print(f"main forms measured: {res['value']:.4g} pairs/s", file=sys.stderr, flush=True)

    if args.extras:
        var = {}
        for name, kw in (("reused_lists_skin4", dict(skin=4.0)),
                         ("reused_lists_warm_skin4", dict(skin=4.0, warm_start=1))):
            a2 = argparse.Namespace(**vars(args))
            a2.snap_every = 0
            capk = cap if "skin" not in kw else neighbour_capacity(L, torch, wl, prec,
                                                                  kw["skin"])
            var[name], _, _ = measure_form(L, torch, wl, prec, a2, capk, **kw)
        if theta is not None:
            a2 = argparse.Namespace(**vars(args))
            a2.snap_every = 0
            var["warm_start_mlp_new_pairs"], _, _ = measure_form(L, torch, wl, prec, a2,
                                                                 cap, theta, warm_start=1)
        wn = wl.with_params(model=L.LUB_MODEL_NORMAL)
        a2 = argparse.Namespace(**vars(args))
        a2.snap_every = 0
        var["normal_only_law"], _, _ = measure_form(L, torch, wn, prec, a2, cap)
        res["variants"] = var
        from paper_1308_6482_amd import workloads as W
        w2 = W.config2()
        a2 = argparse.Namespace(**vars(args))
        a2.steps, a2.warmup = 200, 20
        sec = {}
        sec["plain"], _ = single_eval(L, torch, w2, prec, a2)
        if theta is not None:
            sec["mlp"], _ = single_eval(L, torch, w2, prec, a2, theta)
        res["prolates4096"] = dict(workload=w2.name, step="one evaluation of the same input",
                                   forms=sec)
        w3 = W.config3()
        a2.steps, a2.warmup = 100, 10
        sec3 = {}
        sec3["plain"], _ = single_eval(L, torch, w3, prec, a2)
        if theta is not None:
            sec3["mlp"], _ = single_eval(L, torch, w3, prec, a2, theta)
        res["polydisperse65536"] = dict(workload=w3.name,
                                        step="one evaluation of the same input", forms=sec3)
        res["dynamics"] = dynamics(L, torch, args)
        res["link_laws"] = link_laws(L, torch, args)
    if args.cpu_seconds > 0:
        det = detail_snapshot(L, torch, wl, prec, cap, sample)
        base, acc = cpu_leg(wl, snaps, args.cpu_seconds, det)
        if args.heldout_pairs > 0:
            res["heldout"] = heldout_leg(L, torch, theta, prec, args.heldout_pairs)
        res["cpu_baseline"] = base
        res["accuracy"] = acc
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
