#!/usr/bin/env python3
"""Throughput of the hull path on one MI355X.

One step = the whole hot path over one scan resident in HBM: the one-pass
SC + MSC + SM call (classify, geometry, exact voxel walk, low/high counts, all
three masks) and then the FDK hull. The workload of the
headline figures is the full-scale scan: a 256x256x64 grid of 0.78125 x
0.78125 x 2.5 mm voxels, 2e8 histories at 360 gantry angles (WEPL noise 3 mm
plus 2% uniform outliers, 6.4 GB of SoA FP32 fields), MSC count threshold 5,
SM keeps M > 0.6 max M, FDK on 1 mm x 5 mm detector bins with Shepp-Logan.

Prints one JSON line: throughput (histories/s), per-rule rates, step latency
percentiles, the roofline of the dominant kernel (the walk) and of the whole
counting pass, the FDK hull's kernels, a CPU baseline (the oracle timed on a
bounded sample on this host), and extra keys for the small SC case
(64x64x16, 1e5 histories), the 200x200x32 case (1e7 histories: per-rule
rates, FDK, binned SC, online accumulation), the 16-scan batch and serving.
"""
import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs at 2.4 GHz; HBM3E 8 TB/s; FP32 vector 157.3 TFLOP/s, i.e.
# 128 FMA lanes per CU per clock. 32-bit integer VALU operations issue at the
# same lane rate: a chain of independent v_add_u32 runs at 5.3e13 lane-ops/s on
# the chip, above the 64-lanes-per-clock figure (3.93e13) that the walk's
# roofline was first priced against, so that figure is no bound and is only
# reported beside the real one.
PEAK_INT_TOPS = 256 * 128 * 2.4e9 / 1e12
PEAK_INT_TOPS_64 = 256 * 64 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
OPS_PER_VISIT = 6   # choose axis (2 compares), index, decision variable, address, count
# FDK backprojection per voxel and angle: the voxel centre turned into the
# gantry frame (4 multiplies, 2 adds), the magnification U = (D + x_L) / D
# and its reciprocal (3), u* and v* (2), the weight 1/U^2 (1), the bilinear
# sample (2 subtracts for the fractions, 3 lerps of 3 operations) and the
# weighted accumulation (2): 25 FP32 operations
FLOPS_PER_VOXEL_ANGLE = 25


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "counting_pass_traffic_256x256x64_2e8.md")


def measured_traffic():
    """HBM bytes of the walk kernel (per launch) and of the counting pass (per
    call) on the full-scale scan, from the committed FETCH_SIZE / WRITE_SIZE
    summary; None when the counting kernels have changed since it was taken
    (their sources no longer hash to the recorded value)."""
    import hashlib
    try:
        fields = {}
        for line in open(TRAFFIC_PROFILE):
            k, sep, v = line.partition(":")
            if sep:
                fields[k.strip()] = v.strip()
        h = hashlib.sha256()
        for f in fields["kernel_sources"].split():
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != fields["kernel_sources_sha256"]:
            return None
        return {"walk": float(fields["walk_traffic_bytes_per_launch"]),
                "pass": float(fields["pass_traffic_bytes_per_call"])}
    except (OSError, KeyError, ValueError):
        return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def timed_on(torch, stream, fn, reps, groups=3):
    """Mean ms of `reps` calls of fn between two events on `stream` (one
    untimed call first), the median over `groups` such groups, so that one
    group disturbed by the host does not set the figure."""
    fn()
    torch.cuda.synchronize()
    means = []
    for _ in range(groups):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        means.append(a.elapsed_time(b) / reps)
    return float(np.median(means))


def to_device(torch, gen, spec, dev, step=20_000_000):
    """The scan's histories generated in chunks straight into device arrays."""
    n = spec.n_hist
    arr = {k: torch.empty(n, dtype=torch.float32, device=dev) for k in gen.FIELDS}
    for h0 in range(0, n, step):
        h = gen.generate(spec, h0, min(n, h0 + step))
        for k in gen.FIELDS:
            arr[k][h0:h0 + h[k].size].copy_(torch.from_numpy(h[k]))
    return arr


def profile_avg(fn, reps):
    """Per-kernel (ms per call, launches per call) averaged over reps calls."""
    acc = {}
    for _ in range(reps):
        for k, (ms, n) in fn().items():
            a = acc.setdefault(k, [0.0, 0])
            a[0] += ms
            a[1] = n
    return {k: (v[0] / reps, v[1]) for k, v in acc.items()}


# ---------------------------------------------------------------------------
# headline: the full-scale scan

def headline(torch, gen, H, dev, args):
    spec = gen.config_spec(3)
    n = spec.n_hist
    grid = spec.grid
    V = grid.voxels
    geo = spec.fbp_geometry(du=1.0, dv=5.0)
    t0 = time.time()
    hist = H.Histories(to_device(torch, gen, spec, dev))
    log(f"full-scale scan: {n} histories generated on the host and copied in "
        f"{time.time() - t0:.1f} s")
    params = H.make_params(wepl_low=1.0, wepl_high=5.0, msc_n_t=5, msc_mode=H.HULL_MSC_COUNT,
                           sm_frac_num=3, sm_frac_den=5, sm_mode=H.HULL_SM_FRACTION)
    fbp = H.make_fbp_params(geo)
    N = torch.zeros(V, dtype=torch.int32, device=dev)
    M = torch.zeros(V, dtype=torch.int32, device=dev)
    sc, msc, sm, fmask = (torch.zeros(V, dtype=torch.uint8, device=dev) for _ in range(4))
    image = torch.zeros(V, dtype=torch.float32, device=dev)
    ws_all = H.workspace(H.HULL_OP_ALL, grid, n, dev)
    ws_fbp = H.workspace(H.HULL_OP_FBP, grid, n, dev, fbp)
    stats = torch.zeros(6, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        # the FDK hull and the counting pass are independent, but the pass
        # already runs its batches on two streams: the FDK hull on a third
        # stream beside it made the step 0.4-0.6 ms longer than after it
        # (20.50-20.65 against 20.10 ms), and in the pass's last batch, where
        # one stream is idle, only 0.1 ms shorter
        H.hull_all(hist, grid, params, N, M, sc, msc, sm, stats=stats, ws=ws_all, stream=stream)
        H.hull_fbp(hist, grid, fbp, image, fmask, ws=ws_fbp, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K whole steps, events on the stream the library launches on
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    evs[0].record(stream)
    for _ in range(args.steps):
        step()
    evs[1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = float(evs[0].elapsed_time(evs[1]) / args.steps)
    if args.copy_probe:
        src = torch.ones(1 << 26, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.headline_only:
        return {"ms_per_step": ms_step}, None

    # latency: at least 100 more steps, one event pair each
    L = max(100, args.steps)
    lev = [torch.cuda.Event(enable_timing=True) for _ in range(L + 1)]
    lev[0].record(stream)
    for k in range(L):
        step()
        lev[k + 1].record(stream)
    torch.cuda.synchronize()
    per_step = np.array([lev[k].elapsed_time(lev[k + 1]) for k in range(L)])

    st = H.stats_dict(stats)
    visits = st["n_visits_low"] + st["n_visits_high"]
    n_class = st["n_low"] + st["n_high"]
    reps = max(3, min(args.steps, 10))
    # the counting pass alone (hull_all with ACCUMULATE and no masks launches
    # only the slice-binned counting kernels), per kernel with an event pair
    # around each launch, and as one call
    prof = profile_avg(lambda: H.hull_count_profile(hist, grid, params, N, M,
                                                    flags=H.HULL_ACCUMULATE, ws=ws_all,
                                                    stream=stream), reps)
    t_pass = timed_on(torch, stream, lambda: H.hull_all(hist, grid, params, N, M,
                                                        flags=H.HULL_ACCUMULATE, ws=ws_all,
                                                        stream=stream), reps)
    t_all = timed_on(torch, stream, lambda: H.hull_all(hist, grid, params, N, M, sc, msc, sm,
                                                       ws=ws_all, stream=stream), reps)
    t_sc = timed_on(torch, stream, lambda: H.hull_sc(hist, grid, 1.0, N, sc, ws=ws_all,
                                                     stream=stream), reps)
    t_msc = timed_on(torch, stream, lambda: H.hull_msc(hist, grid, 1.0, 5, H.HULL_MSC_COUNT,
                                                       H.HULL_NBR_INPLANE4, N, msc, ws=ws_all,
                                                       stream=stream), reps)
    t_sm = timed_on(torch, stream, lambda: H.hull_sm(hist, grid, 5.0, 3, 5, H.HULL_SM_FRACTION,
                                                     H.HULL_SCOPE_VOLUME, H.HULL_NBR_INPLANE4, M,
                                                     sm, ws=ws_all, stream=stream), reps)
    t_fbp = timed_on(torch, stream, lambda: H.hull_fbp(hist, grid, fbp, image, fmask, ws=ws_fbp,
                                                       stream=stream), reps)
    fprof = profile_avg(lambda: H.hull_fbp_profile(hist, grid, fbp, image, fmask, ws=ws_fbp,
                                                   stream=stream), reps)

    walk_ms, walk_launches = prof["walk"]
    pass_kernel_ms = sum(v[0] for v in prof.values())
    traffic = measured_traffic()
    walk_tops = visits * OPS_PER_VISIT / (walk_ms * 1e-3) / 1e12
    pass_tops = visits * OPS_PER_VISIT / (t_pass * 1e-3) / 1e12
    # algorithmic HBM bytes of one counting pass: every WEPL, the other seven
    # fields of the classified histories, N and M read and written once
    pass_bytes = 4 * n + 28 * n_class + 2 * 2 * 4 * V
    pass_gbs = pass_bytes / (t_pass * 1e-3) / 1e9
    nbins = int(fbp.nu) * int(fbp.nv) * int(fbp.n_angles)
    bin_ms = fprof["fbp_bin"][0]
    bp_ms = fprof["fbp_backproject"][0]
    bin_bytes = 32 * n + 12 * nbins   # every field of every history read; sums and counts
    bp_flops = FLOPS_PER_VOXEL_ANGLE * V * int(fbp.n_angles)

    result = {
        "metric": "proton histories/sec per hull algorithm (SC/MSC/SM) + %HBM roofline; p99 latency",
        "value": n / (ms_step * 1e-3),
        "unit": "histories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "wall_ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32 walk / fp32 geometry+FDK",
        "data": "synthetic",
        "config": {"workload": "full-scale head phantom 256x256x64 (0.78125x0.78125x2.5 mm) + 3 "
                               "inserts, 2e8 histories, 360 angles, sigma 3 mm + 2% outliers; "
                               "SC+MSC(count 5)+SM(0.6 max) one pass (batches on two streams), "
                               "then the FDK hull (1x5 mm bins)",
                   "histories": n, "grid": list(grid.n), "angles": spec.n_angles},
        "per_rule_histories_per_s": {
            "sc": n / (t_sc * 1e-3), "msc": n / (t_msc * 1e-3), "sm": n / (t_sm * 1e-3),
            "all_one_pass": n / (t_all * 1e-3), "fbp": n / (t_fbp * 1e-3),
            "counting_pass": n / (t_pass * 1e-3)},
        "latency_ms": {"p50": float(np.percentile(per_step, 50)),
                       "p99": float(np.percentile(per_step, 99)), "steps": L},
        "walk": {"pass_ms": t_pass, "voxel_visits": visits, "visits_per_s": visits / (t_pass * 1e-3),
                 "n_low": st["n_low"], "n_high": st["n_high"],
                 "hbm_algorithmic_bytes": pass_bytes, "hbm_algorithmic_GBs": pass_gbs,
                 "hbm_frac": pass_gbs / PEAK_HBM_GBS,
                 "kernels_ms_per_call": {k: v[0] for k, v in prof.items()},
                 "launches_per_call": {k: v[1] for k, v in prof.items()},
                 "kernels_sum_ms": pass_kernel_ms},
        "roofline": {"bound": "alu", "kernel": "k_walk_tiles",
                     "per_unit": "6 int32 lane-ops per voxel visit",
                     "units": visits / walk_launches, "launches_per_call": walk_launches,
                     "avg_launch_ms": walk_ms / walk_launches,
                     "achieved": walk_tops, "peak": PEAK_INT_TOPS, "unit": "TOP/s",
                     "frac": walk_tops / PEAK_INT_TOPS,
                     "frac_at_64_lanes_per_clock": walk_tops / PEAK_INT_TOPS_64,
                     "traffic": traffic["walk"] if traffic else None},
        "roofline_pass": {"bound": "alu",
                          "kernel": "counting pass: k_bin_classify + k_bin_scan_groups + k_bin_scan_sums + "
                                    "k_bin_plan + k_bin_scatter + k_item_setup + k_walk_tiles + "
                                    "k_reduce_tiles + k_walk_overflow, one hull_all call",
                          "per_unit": "6 int32 lane-ops per voxel visit", "units": visits,
                          "achieved": pass_tops, "peak": PEAK_INT_TOPS, "unit": "TOP/s",
                          "frac": pass_tops / PEAK_INT_TOPS,
                          "frac_at_64_lanes_per_clock": pass_tops / PEAK_INT_TOPS_64,
                          "traffic": traffic["pass"] if traffic else None},
        "fdk": {"ms": t_fbp, "kernels_ms_per_call": {k: v[0] for k, v in fprof.items()},
                "bins": nbins,
                "roofline_bin": {"bound": "hbm", "kernel": "k_fbp_bin_lds",
                                 "per_unit": "32 B per history + 12 B per bin",
                                 "achieved": bin_bytes / (bin_ms * 1e-3) / 1e9,
                                 "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                 "frac": bin_bytes / (bin_ms * 1e-3) / 1e9 / PEAK_HBM_GBS},
                "roofline_backproject": {
                    "bound": "alu", "kernel": "k_fbp_backproject_tiles",
                    "per_unit": f"{FLOPS_PER_VOXEL_ANGLE} FP32 operations per voxel and angle",
                    "achieved": bp_flops / (bp_ms * 1e-3) / 1e12, "peak": PEAK_FP32_TFLOPS,
                    "unit": "TFLOP/s", "frac": bp_flops / (bp_ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS}},
        "cpu_baseline": None,
    }
    del hist, N, M, sc, msc, sm, fmask, image, ws_all, ws_fbp
    torch.cuda.empty_cache()
    return result, (spec, geo)


# ---------------------------------------------------------------------------
# the small SC case: 64x64x16, 1e5 noise-free histories at 90 angles

def config1(torch, gen, H, dev):
    spec = gen.config_spec(1)
    h = gen.generate(spec)
    hist = H.Histories.from_numpy(h, dev)
    V = spec.grid.voxels
    N = torch.zeros(V, dtype=torch.int32, device=dev)
    sc = torch.zeros(V, dtype=torch.uint8, device=dev)
    ws = H.workspace(H.HULL_OP_SC, spec.grid, spec.n_hist, dev)
    st = torch.zeros(6, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    H.hull_sc(hist, spec.grid, 1.0, N, sc, stats=st, ws=ws, stream=stream)
    torch.cuda.synchronize()
    s = H.stats_dict(st)
    ms = timed_on(torch, stream, lambda: H.hull_sc(hist, spec.grid, 1.0, N, sc, ws=ws,
                                                   stream=stream), 50)
    # the same call as a one-job batch plan captured in a HIP graph: one graph
    # launch instead of a dozen kernel launches
    job = H.make_job(H.HULL_OP_SC, hist, spec.grid, N=N, sc_mask=sc)
    plan = H.BatchPlan([job], keep=(hist, N, sc), tuning=H.hullmi_tuning(1, 1, 0))
    g_ms = timed_on(torch, stream, lambda: plan.launch(stream), 50)
    plan.close()
    return {"workload": "SC only, noise-free head phantom 64x64x16 (1x1x2.5 mm), 1e5 histories, "
                        "90 angles; carve if WEPL < 1 mm",
            "ms": ms, "histories_per_s": spec.n_hist / (ms * 1e-3),
            "graph_ms": g_ms, "graph_histories_per_s": spec.n_hist / (g_ms * 1e-3),
            "voxel_visits": s["n_visits_low"], "n_low": s["n_low"],
            "note": "launch-latency bound: 3 MB of inputs and 2.5e6 voxel visits per call; "
                    "graph_ms replays the call captured as a one-job batch plan"}


# ---------------------------------------------------------------------------
# the 200x200x32 case: per-rule rates, FDK, binned SC, online accumulation

def config2(torch, gen, H, dev, args):
    spec = gen.config_spec(2)
    geo = spec.fbp_geometry(du=1.0, dv=5.0)
    h = gen.generate(spec)
    hist = H.Histories.from_numpy(h, dev)
    grid = spec.grid
    V = grid.voxels
    n = spec.n_hist
    params = H.make_params()
    fbp = H.make_fbp_params(geo)
    N = torch.zeros(V, dtype=torch.int32, device=dev)
    M = torch.zeros(V, dtype=torch.int32, device=dev)
    sc, msc, sm, fmask = (torch.zeros(V, dtype=torch.uint8, device=dev) for _ in range(4))
    image = torch.zeros(V, dtype=torch.float32, device=dev)
    ws_all = H.workspace(H.HULL_OP_ALL, grid, n, dev)
    ws_fbp = H.workspace(H.HULL_OP_FBP, grid, n, dev, fbp)
    stats = torch.zeros(6, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    side = torch.cuda.Stream(device=dev)
    fork, join = torch.cuda.Event(), torch.cuda.Event()

    def step():
        fork.record(stream)
        side.wait_event(fork)
        H.hull_fbp(hist, grid, fbp, image, fmask, ws=ws_fbp, stream=side)
        H.hull_all(hist, grid, params, N, M, sc, msc, sm, stats=stats, ws=ws_all, stream=stream)
        join.record(side)
        stream.wait_event(join)

    reps = max(5, args.steps)
    t_step = timed_on(torch, stream, step, reps)
    st = H.stats_dict(stats)
    visits = st["n_visits_low"] + st["n_visits_high"]
    prof = profile_avg(lambda: H.hull_count_profile(hist, grid, params, N, M,
                                                    flags=H.HULL_ACCUMULATE, ws=ws_all,
                                                    stream=stream), 5)
    t_pass = timed_on(torch, stream, lambda: H.hull_all(hist, grid, params, N, M,
                                                        flags=H.HULL_ACCUMULATE, ws=ws_all,
                                                        stream=stream), reps)
    t_all = timed_on(torch, stream, lambda: H.hull_all(hist, grid, params, N, M, sc, msc, sm,
                                                       ws=ws_all, stream=stream), reps)
    t_sc = timed_on(torch, stream, lambda: H.hull_sc(hist, grid, 1.0, N, sc, ws=ws_all,
                                                     stream=stream), reps)
    t_msc = timed_on(torch, stream, lambda: H.hull_msc(hist, grid, 1.0, 5, H.HULL_MSC_COUNT,
                                                       H.HULL_NBR_INPLANE4, N, msc, ws=ws_all,
                                                       stream=stream), reps)
    t_sm = timed_on(torch, stream, lambda: H.hull_sm(hist, grid, 5.0, 3, 5, H.HULL_SM_FRACTION,
                                                     H.HULL_SCOPE_VOLUME, H.HULL_NBR_INPLANE4, M,
                                                     sm, ws=ws_all, stream=stream), reps)
    t_fbp = timed_on(torch, stream, lambda: H.hull_fbp(hist, grid, fbp, image, fmask, ws=ws_fbp,
                                                       stream=stream), reps)
    fprof = profile_avg(lambda: H.hull_fbp_profile(hist, grid, fbp, image, fmask, ws=ws_fbp,
                                                   stream=stream), 5)
    t_sm_edge = timed_on(torch, stream, lambda: H.hull_sm(hist, grid, 5.0, 1, 2, H.HULL_SM_EDGE,
                                                          H.HULL_SCOPE_SLICE, H.HULL_NBR_INPLANE4,
                                                          M, sm, ws=ws_all, stream=stream), reps)
    # binned SC (the paper's own SC: per-bin 3-sigma WEPL cuts on the FDK
    # bins, one carve line per bin whose kept mean is below 1 mm, 5 x 5 mean
    # above 0.4) and the FDK hull after the same cuts
    bsc = H.make_bsc_params(wepl_low=1.0, cut_sigmas=3, window=5, thr_num=2, thr_den=5)
    nbins = int(fbp.nu) * int(fbp.nv) * int(fbp.n_angles)
    ws_bsc = H.workspace(H.HULL_OP_SC_BINNED, grid, n, dev, fbp)
    bmask = torch.zeros(V, dtype=torch.uint8, device=dev)
    bstats = torch.zeros(6, dtype=torch.int64, device=dev)
    t_bsc = timed_on(torch, stream, lambda: H.hull_sc_binned(hist, grid, fbp, bsc, bmask,
                                                             stats=bstats, ws=ws_bsc,
                                                             stream=stream), reps)
    bst = H.bsc_stats_dict(bstats)
    ws_fcut = H.workspace(H.HULL_OP_FBP_CUT, grid, n, dev, fbp)
    t_fcut = timed_on(torch, stream, lambda: H.hull_fbp_cut(hist, grid, fbp, 3, image, fmask,
                                                            ws=ws_fcut, stream=stream), reps)
    # algorithmic HBM bytes of one binned SC call: per history the eight
    # fields read once and its 8-byte (bin, w_q) record written and read
    # back; per bin the sums written and read (28 B), the kept range written
    # (8 B), the kept count and sum written and read (24 B), the range read
    # by the cut (28 B with the sums it replaces); per voxel the carved flag
    # written and read and the mask written
    bsc_bytes = 48 * n + 88 * nbins + 3 * V
    bsc_gbs = bsc_bytes / (t_bsc * 1e-3) / 1e9
    walk_ms, walk_launches = prof["walk"]
    walk_tops = visits * OPS_PER_VISIT / (walk_ms * 1e-3) / 1e12
    pass_tops = visits * OPS_PER_VISIT / (t_pass * 1e-3) / 1e12
    bp_ms = fprof["fbp_backproject"][0]
    bp_flops = FLOPS_PER_VOXEL_ANGLE * V * int(fbp.n_angles)
    out = {
        "workload": "head phantom 200x200x32 (1x1x3 mm) + 3 inserts, 1e7 histories, 180 angles, "
                    "sigma 3 mm; SC+MSC(count 5)+SM(0.6 max) one pass + FDK hull",
        "ms_per_step": t_step, "histories_per_s": n / (t_step * 1e-3),
        "per_rule_histories_per_s": {
            "sc": n / (t_sc * 1e-3), "msc": n / (t_msc * 1e-3), "sm": n / (t_sm * 1e-3),
            "all_one_pass": n / (t_all * 1e-3), "counting_pass": n / (t_pass * 1e-3),
            "fbp": n / (t_fbp * 1e-3), "sc_binned": n / (t_bsc * 1e-3),
            "fbp_after_cuts": n / (t_fcut * 1e-3), "sm_edge_threshold": n / (t_sm_edge * 1e-3)},
        "walk": {"pass_ms": t_pass, "voxel_visits": visits,
                 "kernels_ms_per_call": {k: v[0] for k, v in prof.items()},
                 "roofline_walk_frac": walk_tops / PEAK_INT_TOPS,
                 "roofline_pass_frac": pass_tops / PEAK_INT_TOPS},
        "fdk": {"ms": t_fbp, "kernels_ms_per_call": {k: v[0] for k, v in fprof.items()},
                "roofline_backproject": {
                    "bound": "alu", "per_unit": f"{FLOPS_PER_VOXEL_ANGLE} FP32 operations per "
                                                "voxel and angle",
                    "achieved": bp_flops / (bp_ms * 1e-3) / 1e12, "peak": PEAK_FP32_TFLOPS,
                    "unit": "TFLOP/s", "frac": bp_flops / (bp_ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS}},
        "binned_sc": {
            "workload": "same scan; FDK bins 1 mm x 5 mm x 180 angles, 3-sigma WEPL cuts, carve "
                        "bins with kept mean < 1 mm, 5x5 mean > 0.4",
            "ms": t_bsc, "histories_per_s": n / (t_bsc * 1e-3), "bins": nbins,
            "bins_used": bst["n_bins_used"], "bins_carved": bst["n_bins_carved"],
            "histories_cut": bst["n_cut"], "voxel_visits": bst["n_visits"],
            "roofline": {"bound": "hbm", "per_unit": "48 B per history + 88 B per bin + 3 B per voxel",
                         "achieved": bsc_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": bsc_gbs / PEAK_HBM_GBS, "bytes": bsc_bytes}},
    }
    if args.config2_only:
        return out
    log("streaming: one push per gantry angle")
    out["streaming"] = bench_stream(torch, gen, H, h, spec, params, hist)
    return out


def bench_stream(torch, gen, H, h, spec, params, hist, reps=3):
    """Online accumulation of the scan as it is acquired: one push per gantry
    angle (180 chunks of ~55,600 histories) into a session, then the three
    masks read back to the host. From pinned host memory (the copies overlap
    the counting of the previous chunk) and from device chunks."""
    n = spec.n_hist
    edges = [(k * n) // spec.n_angles for k in range(spec.n_angles + 1)]
    mc = max(b - a for a, b in zip(edges[:-1], edges[1:]))
    pinned = {f: torch.from_numpy(h[f]).pin_memory() for f in gen.FIELDS}
    sess = H.Session(spec.grid, params, max_chunk=mc)
    out = {}
    try:
        for mode in ("host", "device"):
            best = None
            for _ in range(reps + 1):
                sess.reset()
                sess.read(counts=False, masks=False)
                t0 = time.perf_counter()
                for a, b in zip(edges[:-1], edges[1:]):
                    if mode == "host":
                        sess.push({f: pinned[f][a:b] for f in gen.FIELDS})
                    else:
                        sess.push(hist.slice(a, b))
                t1 = time.perf_counter()
                sess.read(counts=False, masks=True)
                t2 = time.perf_counter()
                if best is None or t2 - t0 < best[0]:
                    best = (t2 - t0, t1 - t0, t2 - t1)
            out[mode] = {"ms": best[0] * 1e3, "histories_per_s": n / best[0],
                         "push_ms": best[1] * 1e3, "final_read_ms": best[2] * 1e3}
        out["chunks"] = spec.n_angles
        out["workload"] = ("the 200x200x32 scan pushed one gantry angle at a time into a session; "
                           "SC/MSC/SM masks read to the host at the end (host: pinned memory, "
                           "copy included)")
    finally:
        sess.close()
    return out


# ---------------------------------------------------------------------------
# batch and serving

def bench_batch(torch, gen, H, dev, reps=5):
    """16 scans of uneven size on four grids (log-uniform 1e5..5e7 histories,
    ellipsoids jittered +-15%, sigma U[1, 5] mm), each the one-pass SC + MSC +
    SM call: one autotuned, graph-captured plan against the same 16 calls made
    one after another on one stream."""
    specs = gen.batch_specs()
    params = H.make_params()
    jobs, keep, total, stats = [], [], 0, []
    for sp in specs:
        h = gen.generate(sp)
        hist = H.Histories.from_numpy(h, dev)
        del h
        V = sp.grid.voxels
        outs = dict(N=torch.zeros(V, dtype=torch.int32, device=dev),
                    M=torch.zeros(V, dtype=torch.int32, device=dev),
                    sc_mask=torch.zeros(V, dtype=torch.uint8, device=dev),
                    msc_mask=torch.zeros(V, dtype=torch.uint8, device=dev),
                    sm_mask=torch.zeros(V, dtype=torch.uint8, device=dev))
        st = torch.zeros(6, dtype=torch.int64, device=dev)
        jobs.append(H.make_job(H.HULL_OP_ALL, hist, sp.grid, params, stats=st, **outs))
        keep.append((hist, outs, sp))
        stats.append(st)
        total += sp.n_hist
    stream = torch.cuda.current_stream()
    ws_bytes = max(H.hull_workspace_bytes(H.HULL_OP_ALL, sp.grid, sp.n_hist) for sp in specs)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)

    def sequential():
        for hist, o, sp in keep:
            H.hull_all(hist, sp.grid, params, o["N"], o["M"], o["sc_mask"], o["msc_mask"],
                       o["sm_mask"], ws=ws, stream=stream)

    t_seq = timed_on(torch, stream, sequential, reps)
    t0 = time.perf_counter()
    plan = H.BatchPlan(jobs, keep=keep)
    t_plan_s = time.perf_counter() - t0
    t_batch = timed_on(torch, stream, lambda: plan.launch(stream), reps)
    tune = plan.tuning
    plan.close()
    visits = sum(H.stats_dict(st)["n_visits_low"] + H.stats_dict(st)["n_visits_high"]
                 for st in stats)
    # the default launch choices in the same plan shape, for comparison
    plan = H.BatchPlan(jobs, keep=keep, tuning=H.hullmi_tuning(4, 1, 0))
    t_default = timed_on(torch, stream, lambda: plan.launch(stream), reps)
    plan.close()
    return {"workload": "16 scans, log-uniform 1e5..5e7 histories on 64x64x16 / 128x128x32 / "
                        "200x200x32 / 256x256x64 grids, SC+MSC+SM one pass each",
            "histories": total, "scans": len(specs),
            "batched_ms": t_batch, "sequential_ms": t_seq, "untuned_plan_ms": t_default,
            "batched_histories_per_s": total / (t_batch * 1e-3),
            "sequential_histories_per_s": total / (t_seq * 1e-3),
            "speedup": t_seq / t_batch,
            "voxel_visits": visits, "batched_visits_per_s": visits / (t_batch * 1e-3),
            "tuning": tune.as_dict(),
            "plan_s_incl_autotune": t_plan_s}


def bench_serve(torch, gen, H, full=True):
    """Requests arriving one by one with their histories in (pinned) host
    memory, leaving as masks in host memory. Rules SC : MSC : SM = 1 : 1 : 1,
    grids 128x128x32 / 200x200x32 / 256x256x64, log-uniform history counts.
    A calibration pass (the warm-up requests, one at a time) measures the
    sequential capacity; the recorded trace then arrives as a Poisson process
    at 0.7 of it, once at a server with 4 slots (continuous batching) and once
    at a server with 1 slot (sequential per-scan launches, the same offered
    load). Latency = arrival to masks on the host (copies included);
    device_ms = copy-in to copy-out on the worker's stream. The same trace
    queued all at once gives the saturated throughput of both."""
    import threading
    h_hi = 1e8 if full else 1e7
    n_req, warm = (2000, 100) if full else (300, 30)
    rng = np.random.default_rng(0x5EED0005)
    grids = gen.BATCH_GRIDS[1:]
    pools = []
    for gi, g in enumerate(grids):
        sp = gen.ScanSpec(g, int(h_hi), 180, gen.head_phantom(g, inserts=g.n[0] >= 200),
                          0x5EED0005 + 100 * (gi + 1), sigma=3.0)
        h = gen.generate(sp)
        perm = rng.permutation(sp.n_hist)     # any prefix is then a uniform subsample
        pool = {}
        for k in H.FIELDS:
            t = torch.empty(sp.n_hist, dtype=torch.float32, pin_memory=True)
            a = t.numpy()
            np.take(h[k], perm, out=a)
            pool[k] = (t, a)
        del h, perm
        pools.append(pool)
    ops = (H.HULL_OP_SC, H.HULL_OP_MSC, H.HULL_OP_SM)
    mask_of = {H.HULL_OP_SC: "sc_mask", H.HULL_OP_MSC: "msc_mask", H.HULL_OP_SM: "sm_mask"}
    trace = []
    for _ in range(warm + n_req):
        gi = int(rng.integers(len(grids)))
        nh = int(round(np.exp(rng.uniform(np.log(1e5), np.log(h_hi)))))
        trace.append((int(rng.choice(ops)), gi, nh))
    params = H.make_params()

    def submit(srv, req):
        op, gi, nh = req
        hist = {k: pools[gi][k][1][:nh] for k in H.FIELDS}
        out = {mask_of[op]: np.empty(grids[gi].voxels, dtype=np.uint8)}
        return srv.submit(op, hist, grids[gi], params, **out)

    budget = 64 << 30
    srv4 = H.Server(hbm_budget=budget, max_slots=4)
    srv1 = H.Server(hbm_budget=budget, max_slots=1)
    # calibration: the warm-up part of the trace, one request at a time
    svc = []
    for req in trace[:warm]:
        r = srv1.wait(submit(srv1, req))
        svc.append((r["t_done_ns"] - r["t_arrive_ns"]) * 1e-9)
    for req in trace[: warm // 4]:
        srv4.wait(submit(srv4, req))
    cap = 1.0 / float(np.mean(svc[len(svc) // 3:]))
    lam = 0.7 * cap
    rec = trace[warm:]
    gaps = rng.exponential(1.0 / lam, size=len(rec))
    hist_total = sum(nh for _, _, nh in rec)

    def poisson(srv):
        tickets = [None] * len(rec)

        def producer():
            t = time.perf_counter()
            for i, req in enumerate(rec):
                t += gaps[i]
                d = t - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                tickets[i] = submit(srv, req)

        th = threading.Thread(target=producer)
        th.start()
        res = []
        for i in range(len(rec)):
            while tickets[i] is None:
                time.sleep(0.0002)
            res.append(srv.wait(tickets[i]))
        th.join()
        lat = np.array([(r["t_done_ns"] - r["t_arrive_ns"]) * 1e-6 for r in res])
        dev_ms = np.array([r["device_ms"] for r in res])
        span = (max(r["t_done_ns"] for r in res) - min(r["t_arrive_ns"] for r in res)) * 1e-9
        return {"latency_ms": {"p50": float(np.percentile(lat, 50)),
                               "p99": float(np.percentile(lat, 99))},
                "device_ms": {"p50": float(np.percentile(dev_ms, 50)),
                              "p99": float(np.percentile(dev_ms, 99))},
                "histories_per_s": hist_total / span,
                "all_ok": all(r["status"] == H.HULL_OK for r in res)}

    def saturated(srv):
        t_sub = [submit(srv, req) for req in rec]
        res = [srv.wait(t) for t in t_sub]
        span = (max(r["t_done_ns"] for r in res) - min(r["t_arrive_ns"] for r in res)) * 1e-9
        return hist_total / span, all(r["status"] == H.HULL_OK for r in res)

    log(f"serving: {n_req} requests at {lam:.1f}/s, 4 slots")
    served = poisson(srv4)
    log("serving: the same trace, 1 slot")
    seq = poisson(srv1)
    log("serving: saturated")
    sat4, ok4 = saturated(srv4)
    sat1, ok1 = saturated(srv1)
    st = srv4.stats()
    srv4.close()
    srv1.close()
    return {"workload": f"{n_req} requests after {warm} warm-up, log-uniform 1e5..{h_hi:.0e} "
                        "histories, SC:MSC:SM 1:1:1, grids 128x128x32 / 200x200x32 / 256x256x64, "
                        "pinned host inputs, masks back on the host; Poisson arrivals at 0.7 of "
                        "the sequential capacity",
            "all_ok": served["all_ok"] and seq["all_ok"] and ok4 and ok1,
            "lambda_req_per_s": lam, "sequential_capacity_req_per_s": cap,
            "served": {k: v for k, v in served.items() if k != "all_ok"},
            "sequential": {k: v for k, v in seq.items() if k != "all_ok"},
            "saturated_histories_per_s": {"served_4_slots": sat4, "sequential_1_slot": sat1},
            "arena_peak_bytes": st["bytes_peak"], "slots": 4}


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on a bounded sample of the headline workload

def cpu_baseline(gen, spec, geo, sample, single):
    import oracle
    n = spec.n_hist
    chunk = 10_000
    starts = np.linspace(0, n - chunk, max(1, sample // chunk)).astype(np.int64)
    parts = [gen.generate(spec, int(s), int(s) + chunk) for s in starts]
    sub = {k: np.concatenate([p[k] for p in parts]) for k in gen.FIELDS}
    S = len(sub["wepl"])
    G = oracle.grid_of(spec.grid)
    gomp = ctypes.CDLL("libgomp.so.1")
    threads = int(gomp.omp_get_max_threads())
    c0 = time.perf_counter()
    rN, rM, _ = oracle.counts(sub, G)
    c1 = time.perf_counter()
    oracle.sc(rN)
    oracle.msc(rN, G, 5)
    oracle.sm(rM, G, 3, 5)
    c2 = time.perf_counter()
    oracle.fbp(sub, G, oracle.fbp_params(geo))
    c3 = time.perf_counter()
    per_hist = (c1 - c0) / S
    fixed = (c2 - c1) + (c3 - c2)
    # one thread on a smaller part of the same sample
    S1 = min(single, S)
    sub1 = {k: v[:: max(1, S // S1)][:S1] for k, v in sub.items()}
    gomp.omp_set_num_threads(1)
    try:
        d0 = time.perf_counter()
        oracle.counts(sub1, G)
        d1 = time.perf_counter()
    finally:
        gomp.omp_set_num_threads(threads)
    per_hist1 = (d1 - d0) / len(sub1["wepl"])
    return {"value": n / (per_hist * n + fixed), "unit": "histories/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"{S} histories of the full-scale scan (10,000-history runs at {len(starts)} "
                      f"evenly spaced offsets, every gantry angle): counts {c1 - c0:.2f} s, the "
                      f"three masks {c2 - c1:.2f} s, FDK hull {c3 - c2:.2f} s, {threads} threads; "
                      f"value = full-scan estimate (per-history counting time x 2e8 + the masks "
                      f"+ the FDK hull, whose backprojection is a fixed cost per scan)",
            "counting_histories_per_s": 1.0 / per_hist,
            "single_thread": {"histories": len(sub1["wepl"]), "s": d1 - d0,
                              "counting_histories_per_s": 1.0 / per_hist1}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2_000_000,
                    help="histories of the full-scale scan the oracle counts on all threads")
    ap.add_argument("--cpu-single", type=int, default=250_000,
                    help="histories of that sample the oracle counts on one thread")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the full-scale headline (no small, 200x200x32, batch or serving "
                         "figures)")
    ap.add_argument("--headline-only", action="store_true",
                    help="the timed steps of the headline and nothing else (for profiles)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 16-scan batch figures")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving figures")
    ap.add_argument("--serve-small", action="store_true",
                    help="serve 300 requests of up to 1e7 histories instead of 2000 of up to 1e8")
    ap.add_argument("--config2-only", action="store_true",
                    help="time the 200x200x32 case alone (its per-rule calls, FDK and binned SC; "
                         "for a profile of their kernels)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed region, run one 256 MiB device-to-device copy: the "
                         "known-size kernel that scales hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the hull path is measured "
              "on a single MI355X", file=sys.stderr)
        sys.exit(2)

    import torch

    import gen
    from paper_1402_1720_amd import hullmi as H

    dev = torch.device("cuda:0")
    if args.config2_only:
        print(json.dumps(config2(torch, gen, H, dev, args)), flush=True)
        return
    result, ctx = headline(torch, gen, H, dev, args)
    if args.headline_only:
        print(json.dumps(result), flush=True)
        return
    if not args.no_extras:
        log("small SC case")
        result["config1"] = config1(torch, gen, H, dev)
        torch.cuda.empty_cache()
        log("200x200x32 case")
        result["config2"] = config2(torch, gen, H, dev, args)
        torch.cuda.empty_cache()
        if not args.no_batch:
            log("batch: 16 scans")
            b = bench_batch(torch, gen, H, dev)
            # how close the batch comes to the voxel-visit rate of one large
            # scan's counting pass: the most a single fused launch could gain
            b["visit_rate_vs_full_scale_pass"] = (b["batched_visits_per_s"] /
                                                  result["walk"]["visits_per_s"])
            result["batch"] = b
            torch.cuda.empty_cache()
        if not args.no_serve:
            log("serving")
            result["serving"] = bench_serve(torch, gen, H, full=not args.serve_small)
            torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("CPU baseline: the oracle on a sample of the full-scale scan")
        spec, geo = ctx
        result["cpu_baseline"] = cpu_baseline(gen, spec, geo, args.cpu_sample, args.cpu_single)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
