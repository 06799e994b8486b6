#!/usr/bin/env python3
"""Throughput of the hull path on one MI355X.

One step = the whole hot path over one scan resident in HBM: the one-pass
SC + MSC + SM call (classify, geometry, exact voxel walk, low/high counts, all
three masks) and the FDK hull. The workload is the 200x200x32 scan with 1e7
histories at 180 gantry angles (WEPL noise 3 mm, MSC count threshold 5, SM
keeps M > 0.6 max M, FDK on 1 mm x 5 mm detector bins with Shepp-Logan).

Prints one JSON line with throughput (histories/s), per-rule rates, step
latency percentiles, the roofline of the dominant kernel (the walk) and a CPU
baseline (the oracle timed on a bounded sample on this host).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs at 2.4 GHz, 64 int32 lanes per CU per clock; HBM3E 8 TB/s.
PEAK_INT_TOPS = 256 * 64 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0
OPS_PER_VISIT = 6   # choose axis (2 compares), index, decision variable, address, count


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "counting_pass_traffic_200x200x32_1e7.md")


def measured_traffic():
    """HBM bytes of one counting pass from the committed FETCH_SIZE / WRITE_SIZE
    summary, or None when the counting kernels have changed since it was
    taken (their sources no longer hash to the recorded value)."""
    import hashlib
    try:
        fields = {}
        for line in open(TRAFFIC_PROFILE):
            k, sep, v = line.partition(":")
            if sep and k.strip() in ("traffic_bytes_per_pass", "kernel_sources",
                                     "kernel_sources_sha256"):
                fields[k.strip()] = v.strip()
        h = hashlib.sha256()
        for f in fields["kernel_sources"].split():
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != fields["kernel_sources_sha256"]:
            return None
        return float(fields["traffic_bytes_per_pass"])
    except (OSError, KeyError, ValueError):
        return None


def _timed_on(torch, stream, fn, reps):
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def bench_batch(torch, gen, H, dev, reps=5):
    """16 scans of uneven size on four grids (log-uniform 1e5..5e7 histories,
    ellipsoids jittered +-15%, sigma U[1, 5] mm), each the one-pass SC + MSC +
    SM call: one autotuned, graph-captured plan against the same 16 calls made
    one after another on one stream."""
    specs = gen.batch_specs()
    params = H.make_params()
    jobs, keep, total = [], [], 0
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
        jobs.append(H.make_job(H.HULL_OP_ALL, hist, sp.grid, params, **outs))
        keep.append((hist, outs, sp))
        total += sp.n_hist
    stream = torch.cuda.current_stream()
    ws_bytes = max(H.hull_workspace_bytes(H.HULL_OP_ALL, sp.grid, sp.n_hist) for sp in specs)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)

    def sequential():
        for hist, o, sp in keep:
            H.hull_all(hist, sp.grid, params, o["N"], o["M"], o["sc_mask"], o["msc_mask"],
                       o["sm_mask"], ws=ws, stream=stream)

    t_seq = _timed_on(torch, stream, sequential, reps)
    t0 = time.perf_counter()
    plan = H.BatchPlan(jobs, keep=keep)
    t_plan_s = time.perf_counter() - t0
    t_batch = _timed_on(torch, stream, lambda: plan.launch(stream), reps)
    tune = plan.tuning
    plan.close()
    return {"workload": "16 scans, log-uniform 1e5..5e7 histories on 64x64x16 / 128x128x32 / "
                        "200x200x32 / 256x256x64 grids, SC+MSC+SM one pass each",
            "histories": total, "scans": len(specs),
            "batched_ms": t_batch, "sequential_ms": t_seq,
            "batched_histories_per_s": total / (t_batch * 1e-3),
            "sequential_histories_per_s": total / (t_seq * 1e-3),
            "speedup": t_seq / t_batch,
            "tuning": {"streams": tune.streams, "use_graph": tune.use_graph,
                       "walk_blocks": tune.walk_blocks},
            "plan_s_incl_autotune": t_plan_s}


def bench_serve(torch, gen, H, full=False):
    """Requests arriving one by one with their histories in (pinned) host
    memory, leaving as masks in host memory. Rules SC : MSC : SM = 1 : 1 : 1,
    grids 128x128x32 / 200x200x32 / 256x256x64, log-uniform history counts.
    A calibration pass measures the sequential capacity; the recorded trace
    then arrives as a Poisson process at 0.7 of it. Latency = arrival to masks
    on the host (copies included); device_ms = copy-in to copy-out on the
    worker's stream. The same trace queued all at once gives the saturated
    throughput, and served one request at a time the sequential baseline."""
    import threading
    import numpy as np
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
        del h
        pools.append(pool)
    ops = (H.HULL_OP_SC, H.HULL_OP_MSC, H.HULL_OP_SM)
    mask_of = {H.HULL_OP_SC: "sc_mask", H.HULL_OP_MSC: "msc_mask", H.HULL_OP_SM: "sm_mask"}
    trace = []
    for _ in range(warm + n_req):
        gi = int(rng.integers(len(grids)))
        n = int(round(np.exp(rng.uniform(np.log(1e5), np.log(h_hi)))))
        trace.append((int(rng.choice(ops)), gi, n))
    params = H.make_params()

    def submit(srv, req):
        op, gi, n = req
        hist = {k: pools[gi][k][1][:n] for k in H.FIELDS}
        out = {mask_of[op]: np.empty(grids[gi].voxels, dtype=np.uint8)}
        return srv.submit(op, hist, grids[gi], params, **out)

    srv = H.Server(hbm_budget=48 << 30, max_slots=4)
    # calibration: the warm-up part of the trace, one request at a time
    svc = []
    for req in trace[:warm]:
        r = srv.wait(submit(srv, req))
        svc.append((r["t_done_ns"] - r["t_arrive_ns"]) * 1e-9)
    cap = 1.0 / float(np.mean(svc[len(svc) // 3:]))
    lam = 0.7 * cap
    rec = trace[warm:]
    gaps = rng.exponential(1.0 / lam, size=len(rec))
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
    hist_total = sum(n for _, _, n in rec)
    ok = all(r["status"] == H.HULL_OK for r in res)
    # saturated: the whole recorded trace queued at once, so the server's
    # slots overlap copies and compute as far as they can
    t_sub = [submit(srv, req) for req in rec]
    sat = [srv.wait(t) for t in t_sub]
    sat_span = (max(r["t_done_ns"] for r in sat) - min(r["t_arrive_ns"] for r in sat)) * 1e-9
    ok = ok and all(r["status"] == H.HULL_OK for r in sat)
    # sequential baseline on the same trace
    seq = []
    for req in rec:
        r = srv.wait(submit(srv, req))
        seq.append((r["t_done_ns"] - r["t_arrive_ns"]) * 1e-9)
    st = srv.stats()
    srv.close()
    return {"workload": f"{n_req} requests after {warm} warm-up, log-uniform 1e5..{h_hi:.0e} "
                        "histories, SC:MSC:SM 1:1:1, grids 128x128x32 / 200x200x32 / 256x256x64, "
                        "pinned host inputs, masks back on the host",
            "all_ok": ok, "lambda_req_per_s": lam, "sequential_capacity_req_per_s": cap,
            "latency_ms": {"p50": float(np.percentile(lat, 50)),
                           "p99": float(np.percentile(lat, 99))},
            "device_ms": {"p50": float(np.percentile(dev_ms, 50)),
                          "p99": float(np.percentile(dev_ms, 99))},
            "served_histories_per_s": hist_total / span,
            "saturated_histories_per_s": hist_total / sat_span,
            "sequential_histories_per_s": hist_total / float(np.sum(seq)),
            "sequential_latency_ms_p50": float(np.percentile(np.array(seq) * 1e3, 50)),
            "arena_peak_bytes": st["bytes_peak"], "slots": 4}


def bench_stream(torch, gen, H, h, spec, params, hist, reps=3):
    """Online accumulation of the bench scan as it is acquired: one push per
    gantry angle (180 chunks of ~55,600 histories) into a session, then the
    three masks read back to the host. From pinned host memory (the copies
    overlap the counting of the previous chunk) and from device chunks."""
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
                r = sess.read(counts=False, masks=True)
                t2 = time.perf_counter()
                if best is None or t2 - t0 < best[0]:
                    best = (t2 - t0, t1 - t0, t2 - t1)
            out[mode] = {"ms": best[0] * 1e3, "histories_per_s": n / best[0],
                         "push_ms": best[1] * 1e3, "final_read_ms": best[2] * 1e3}
        out["chunks"] = spec.n_angles
        out["workload"] = ("bench scan pushed one gantry angle at a time into a session; SC/MSC/SM "
                           "masks read to the host at the end (host: pinned memory, copy included)")
    finally:
        sess.close()
    return out


def bench_full_scale(torch, gen, H, dev, reps):
    """The full-scale scan (256x256x64 grid, 2e8 histories at 360 angles, 2%
    outliers): histories generated in chunks straight into device arrays
    (6.4 GB resident), then the counting pass and hull_all with all three
    masks, each timed with HIP events over `reps` calls."""
    spec = gen.config_spec(3)
    n = spec.n_hist
    arr = {k: torch.empty(n, dtype=torch.float32, device=dev) for k in gen.FIELDS}
    t0 = time.time()
    step = 20_000_000
    for h0 in range(0, n, step):
        h = gen.generate(spec, h0, min(n, h0 + step))
        for k in gen.FIELDS:
            arr[k][h0:h0 + h[k].size].copy_(torch.from_numpy(h[k]))
    log(f"generated {n} histories in {time.time() - t0:.1f} s")
    hist = H.Histories(arr)
    grid = spec.grid
    V = grid.voxels
    params = H.make_params(wepl_low=1.0, wepl_high=5.0, msc_n_t=5, msc_mode=H.HULL_MSC_COUNT,
                           sm_frac_num=3, sm_frac_den=5, sm_mode=H.HULL_SM_FRACTION)
    N = torch.zeros(V, dtype=torch.int32, device=dev)
    M = torch.zeros(V, dtype=torch.int32, device=dev)
    masks = [torch.zeros(V, dtype=torch.uint8, device=dev) for _ in range(3)]
    ws = H.workspace(H.HULL_OP_ALL, grid, n, dev)
    st = torch.zeros(6, dtype=torch.int64, device=dev)
    s = torch.cuda.current_stream()
    H.hull_all(hist, grid, params, N, M, *masks, stats=st, ws=ws, stream=s)
    torch.cuda.synchronize()
    stats = H.stats_dict(st)
    visits = stats["n_visits_low"] + stats["n_visits_high"]
    out = {"workload": "full-scale head phantom 256x256x64 (0.78125x0.78125x2.5 mm), 2e8 "
                       "histories, 360 angles, sigma 3 mm + 2% outliers; SC+MSC+SM one pass",
           "histories": n, "voxel_visits": visits, "stats": stats}
    for name, fn in (("counting_pass", lambda: H.hull_all(hist, grid, params, N, M,
                                                          flags=H.HULL_ACCUMULATE, ws=ws,
                                                          stream=s)),
                     ("hull_all", lambda: H.hull_all(hist, grid, params, N, M, *masks, ws=ws,
                                                     stream=s))):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        for _ in range(reps):
            fn()
        b.record(s)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        out[name] = {"ms": ms, "histories_per_s": n / (ms * 1e-3), "visits_per_s": visits / (ms * 1e-3)}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2_000_000)
    ap.add_argument("--no-batch", action="store_true", help="skip the 16-scan batch figures")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving figures")
    ap.add_argument("--serve-full", action="store_true",
                    help="serve 2000 requests of up to 1e8 histories (minutes) instead of 300 of "
                         "up to 1e7")
    ap.add_argument("--bsc-only", action="store_true",
                    help="time the binned SC alone (for a profile of its kernels)")
    ap.add_argument("--full-scale", action="store_true",
                    help="time the full-scale scan instead (256x256x64, 2e8 histories, 360 "
                         "angles, generated on the device in chunks): counting pass and hull_all")
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
    if args.full_scale:
        bench_full_scale(torch, gen, H, dev, max(1, args.steps))
        return
    spec = gen.config_spec(2)
    geo = spec.fbp_geometry(du=1.0, dv=5.0)
    t0 = time.time()
    h = gen.generate(spec)
    log(f"generated {spec.n_hist} histories in {time.time() - t0:.1f} s")
    hist = H.Histories.from_numpy(h, dev)
    grid = spec.grid
    V = grid.voxels
    n = spec.n_hist
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
    side = torch.cuda.Stream(device=dev)   # default priority, like every stream here
    fork, join = torch.cuda.Event(), torch.cuda.Event()

    if args.bsc_only:
        bsc = H.make_bsc_params()
        ws_bsc = H.workspace(H.HULL_OP_SC_BINNED, grid, n, dev, fbp)
        bmask = torch.zeros(V, dtype=torch.uint8, device=dev)
        ms = _timed_on(torch, stream, lambda: H.hull_sc_binned(hist, grid, fbp, bsc, bmask,
                                                               ws=ws_bsc, stream=stream),
                       args.steps)
        print(json.dumps({"binned_sc_ms": ms, "histories_per_s": n / (ms * 1e-3)}), flush=True)
        return

    def step():
        # the FDK hull and the counting pass are independent: FDK runs on a
        # second stream and the step ends when both are done
        fork.record(stream)
        side.wait_event(fork)
        H.hull_fbp(hist, grid, fbp, image, fmask, ws=ws_fbp, stream=side)
        H.hull_all(hist, grid, params, N, M, sc, msc, sm, stats=stats, ws=ws_all, stream=stream)
        join.record(side)
        stream.wait_event(join)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K whole steps, events on the stream the library launches on
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    evs[0].record(stream)
    for k in range(args.steps):
        step()
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    per_step = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)])
    ms_step = float(evs[0].elapsed_time(evs[-1]) / args.steps)
    if args.copy_probe:
        src = torch.ones(1 << 26, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    st = H.stats_dict(stats)
    visits = st["n_visits_low"] + st["n_visits_high"]

    def timed(fn, reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        torch.cuda.synchronize()
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    reps = max(3, args.steps)
    # the counting pass alone: with ACCUMULATE and no masks hull_all launches
    # only the slice-binned counting kernels (classify, scan, plan, scatter,
    # item set-up, tile walk, reduce, overflow walk) on `stream`
    t_walk = timed(lambda: H.hull_all(hist, grid, params, N, M, flags=H.HULL_ACCUMULATE,
                                      ws=ws_all, stream=stream), reps)
    t_all = timed(lambda: H.hull_all(hist, grid, params, N, M, sc, msc, sm, ws=ws_all,
                                     stream=stream), reps)
    t_sc = timed(lambda: H.hull_sc(hist, grid, 1.0, N, sc, stream=stream), reps)
    t_msc = timed(lambda: H.hull_msc(hist, grid, 1.0, 5, H.HULL_MSC_COUNT, H.HULL_NBR_INPLANE4, N,
                                     msc, stream=stream), reps)
    t_sm = timed(lambda: H.hull_sm(hist, grid, 5.0, 3, 5, H.HULL_SM_FRACTION, H.HULL_SCOPE_VOLUME,
                                   H.HULL_NBR_INPLANE4, M, sm, ws=ws_all, stream=stream), reps)
    t_fbp = timed(lambda: H.hull_fbp(hist, grid, fbp, image, fmask, ws=ws_fbp, stream=stream), reps)
    # SM with the per-slice threshold from each slice's strongest edge
    t_sm_edge = timed(lambda: H.hull_sm(hist, grid, 5.0, 1, 2, H.HULL_SM_EDGE, H.HULL_SCOPE_SLICE,
                                        H.HULL_NBR_INPLANE4, M, sm, ws=ws_all, stream=stream), reps)

    # binned SC (the paper's own SC: per-bin 3-sigma WEPL cuts on the FDK
    # bins, one carve line per bin whose kept mean is below 1 mm, 5 x 5 mean
    # above 0.4) on the same resident scan
    bsc = H.make_bsc_params(wepl_low=1.0, cut_sigmas=3, window=5, thr_num=2, thr_den=5)
    nbins = int(fbp.nu) * int(fbp.nv) * int(fbp.n_angles)
    ws_bsc = H.workspace(H.HULL_OP_SC_BINNED, grid, n, dev, fbp)
    bmask = torch.zeros(V, dtype=torch.uint8, device=dev)
    bstats = torch.zeros(6, dtype=torch.int64, device=dev)
    t_bsc = timed(lambda: H.hull_sc_binned(hist, grid, fbp, bsc, bmask, stats=bstats, ws=ws_bsc,
                                           stream=stream), reps)
    bst = H.bsc_stats_dict(bstats)
    # FDK hull after the same 3-sigma cuts
    ws_fcut = H.workspace(H.HULL_OP_FBP_CUT, grid, n, dev, fbp)
    t_fcut = timed(lambda: H.hull_fbp_cut(hist, grid, fbp, 3, image, fmask, ws=ws_fcut,
                                          stream=stream), reps)
    # algorithmic HBM bytes of one call: per history the eight fields read once
    # and its 8-byte (bin, w_q) record written and read back; per bin the sums
    # written and read (28 B), the kept range written (8 B), the kept count
    # and sum written and read (24 B), the range read by the cut (28 B with
    # the sums it replaces); per voxel the carved flag written and read and
    # the mask written
    bsc_bytes = 48 * n + 88 * nbins + 3 * V
    bsc_gbs = bsc_bytes / (t_bsc * 1e-3) / 1e9

    # algorithmic work of one walk launch: 6 int lane-ops per voxel visit
    achieved_tops = visits * OPS_PER_VISIT / (t_walk * 1e-3) / 1e12
    # algorithmic HBM bytes of one walk launch: every WEPL, the other seven
    # fields of the classified histories, N and M written back once
    n_class = st["n_low"] + st["n_high"]
    alg_bytes = 4 * n + 28 * n_class + 2 * 4 * V
    hbm_gbs = alg_bytes / (t_walk * 1e-3) / 1e9

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
        "config": {"workload": "head phantom 200x200x32 (1x1x3 mm), 1e7 histories, 180 angles, "
                               "sigma 3 mm; SC+MSC(count 5)+SM(0.6 max) one pass + FDK hull",
                   "histories": n, "grid": list(grid.n), "angles": spec.n_angles},
        "per_rule_histories_per_s": {
            "sc": n / (t_sc * 1e-3), "msc": n / (t_msc * 1e-3), "sm": n / (t_sm * 1e-3),
            "all_one_pass": n / (t_all * 1e-3), "fbp": n / (t_fbp * 1e-3),
            "sc_binned": n / (t_bsc * 1e-3), "fbp_after_cuts": n / (t_fcut * 1e-3),
            "sm_edge_threshold": n / (t_sm_edge * 1e-3)},
        "latency_ms": {"p50": float(np.percentile(per_step, 50)),
                       "p99": float(np.percentile(per_step, 99))},
        "walk": {"ms": t_walk, "voxel_visits": visits, "visits_per_s": visits / (t_walk * 1e-3),
                 "n_low": st["n_low"], "n_high": st["n_high"],
                 "hbm_algorithmic_GBs": hbm_gbs, "hbm_frac": hbm_gbs / PEAK_HBM_GBS},
        "roofline": {"bound": "alu",
                     "kernel": "counting pass: k_bin_classify + k_bin_scan_blocks + k_bin_plan + "
                               "k_bin_scatter + k_item_setup + k_walk_tiles + k_reduce_tiles + "
                               "k_walk_overflow",
                     "per_unit": "6 int32 lane-ops per voxel visit", "units": visits,
                     "achieved": achieved_tops,
                     "peak": PEAK_INT_TOPS, "unit": "TOP/s", "frac": achieved_tops / PEAK_INT_TOPS,
                     "traffic": measured_traffic()},
        "cpu_baseline": None,
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

    log("streaming: one push per gantry angle")
    result["streaming"] = bench_stream(torch, gen, H, h, spec, params, hist)

    # free the single-scan buffers before the batch and serving figures
    del hist, N, M, sc, msc, sm, fmask, image, ws_all, ws_fbp, ws_bsc, bmask, ws_fcut
    torch.cuda.empty_cache()
    if not args.no_batch:
        log("batch: 16 scans")
        result["batch"] = bench_batch(torch, gen, H, dev)
        torch.cuda.empty_cache()
    if not args.no_serve:
        log("serving")
        result["serving"] = bench_serve(torch, gen, H, full=args.serve_full)
        torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        import oracle
        S = min(args.cpu_sample, n)
        sub = {k: v[:S] for k, v in h.items()}
        G = oracle.grid_of(grid)
        c0 = time.perf_counter()
        rN, rM, _ = oracle.counts(sub, G)
        oracle.sc(rN)
        oracle.msc(rN, G, 5)
        oracle.sm(rM, G, 3, 5)
        c1 = time.perf_counter()
        oracle.fbp(sub, G, oracle.fbp_params(geo))
        c2 = time.perf_counter()
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        # per-history work scales with the sample; the FDK backprojection is a
        # fixed cost per scan, so the full-scan estimate adds it once
        per_hist = (c1 - c0) / S
        result["cpu_baseline"] = {
            "value": n / (per_hist * n + (c2 - c1)), "unit": "histories/s", "cores": cores,
            "kind": "oracle",
            "sample": f"first {S} histories of the same scan: counts + SC/MSC/SM masks "
                      f"({c1 - c0:.2f} s) and FDK ({c2 - c1:.2f} s); value = full-scan estimate "
                      f"(per-history time x 1e7 + one FDK)"}

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
