"""Batches and serving on the GPU: a scan run inside a batch plan (several
streams, graph-captured, replayed) or through the server (host in, host out,
admitted into a shared arena next to other requests) gives exactly the
result of the same scan run alone through its per-scan call, and the alone
results of a small scan match the oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import gen
import oracle
from paper_1402_1720_amd import hullmi as H

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _scans(n_scans=8, h_lo=2e3, h_hi=3e5, seed=0x5EED0104):
    specs = gen.batch_specs(n_scans=n_scans, h_lo=h_lo, h_hi=h_hi, seed=seed)
    return specs, [gen.generate(s) for s in specs]


# one op per scan, cycling through every kind of call and mode
_OPS = [
    (H.HULL_OP_ALL, H.make_params()),
    (H.HULL_OP_SC, H.make_params()),
    (H.HULL_OP_MSC, H.make_params(msc_n_t=50, msc_mode=H.HULL_MSC_NEIGHBOR_DIFF)),
    (H.HULL_OP_SM, H.make_params(sm_mode=H.HULL_SM_MAX_SLOPE, sm_scope=H.HULL_SCOPE_SLICE,
                                 nbr=H.HULL_NBR_SPATIAL6)),
    (H.HULL_OP_FBP, None),
    (H.HULL_OP_ALL, H.make_params(sm_scope=H.HULL_SCOPE_SLICE)),
    (H.HULL_OP_SC_BINNED, None),
    (H.HULL_OP_FBP_CUT, None),
]
_BINS = (H.HULL_OP_FBP, H.HULL_OP_FBP_CUT, H.HULL_OP_SC_BINNED)    # ops that take detector bins
_COUNTING = (H.HULL_OP_SC, H.HULL_OP_MSC, H.HULL_OP_SM, H.HULL_OP_ALL)
_BSC = H.make_bsc_params(wepl_low=1.0, cut_sigmas=3, window=5, thr_num=2, thr_den=5)


def _outputs(op, V):
    z32 = lambda: torch.zeros(V, dtype=torch.int32, device=DEV)
    z8 = lambda: torch.zeros(V, dtype=torch.uint8, device=DEV)
    return {H.HULL_OP_SC: lambda: dict(N=z32(), sc_mask=z8()),
            H.HULL_OP_MSC: lambda: dict(N=z32(), msc_mask=z8()),
            H.HULL_OP_SM: lambda: dict(M=z32(), sm_mask=z8()),
            H.HULL_OP_ALL: lambda: dict(N=z32(), M=z32(), sc_mask=z8(), msc_mask=z8(), sm_mask=z8()),
            H.HULL_OP_FBP: lambda: dict(image=torch.zeros(V, dtype=torch.float32, device=DEV),
                                        fbp_mask=z8()),
            H.HULL_OP_FBP_CUT: lambda: dict(image=torch.zeros(V, dtype=torch.float32, device=DEV),
                                            fbp_mask=z8()),
            H.HULL_OP_SC_BINNED: lambda: dict(bsc_mask=z8())}[op]()


def _alone(op, params, fbp, hist, grid, outs, stats):
    """The per-scan call of one job."""
    p = params
    if op == H.HULL_OP_SC:
        H.hull_sc(hist, grid, p.wepl_low, outs["N"], outs["sc_mask"], stats=stats)
    elif op == H.HULL_OP_MSC:
        H.hull_msc(hist, grid, p.wepl_low, p.msc_n_t, p.msc_mode, p.nbr, outs["N"],
                   outs["msc_mask"], stats=stats)
    elif op == H.HULL_OP_SM:
        H.hull_sm(hist, grid, p.wepl_high, p.sm_frac_num, p.sm_frac_den, p.sm_mode, p.sm_scope,
                  p.nbr, outs["M"], outs["sm_mask"], stats=stats)
    elif op == H.HULL_OP_ALL:
        H.hull_all(hist, grid, p, outs["N"], outs["M"], outs["sc_mask"], outs["msc_mask"],
                   outs["sm_mask"], stats=stats)
    elif op == H.HULL_OP_FBP:
        H.hull_fbp(hist, grid, fbp, outs["image"], outs["fbp_mask"])
    elif op == H.HULL_OP_FBP_CUT:
        H.hull_fbp_cut(hist, grid, fbp, _BSC.cut_sigmas, outs["image"], outs["fbp_mask"])
    else:
        H.hull_sc_binned(hist, grid, fbp, _BSC, outs["bsc_mask"], stats=stats)


@pytest.fixture(scope="module")
def batch_case():
    specs, data = _scans()
    data[2] = {k: v[:0] for k, v in data[2].items()}     # an empty scan in the mix
    case = []
    for i, (spec, h) in enumerate(zip(specs, data)):
        op, params = _OPS[i % len(_OPS)]
        grid = H.make_grid(spec.grid)
        V = spec.grid.voxels
        fbp = H.make_fbp_params(spec.fbp_geometry()) if op in _BINS else None
        hist = H.Histories.from_numpy(h, DEV)
        ref = _outputs(op, V)
        ref_stats = torch.zeros(6, dtype=torch.int64, device=DEV)
        _alone(op, params or H.make_params(), fbp, hist, grid, ref, ref_stats)
        case.append(dict(op=op, params=params or H.make_params(), fbp=fbp, hist=hist, grid=grid,
                         V=V, ref=ref, ref_stats=ref_stats, spec=spec, h=h))
    torch.cuda.synchronize()
    return case


def _plan(case, tuning, flags=0):
    jobs, keep = [], []
    for c in case:
        outs = _outputs(c["op"], c["V"])
        stats = torch.zeros(6, dtype=torch.int64, device=DEV)
        jobs.append(H.make_job(c["op"], c["hist"], c["grid"], c["params"], c["fbp"], flags=flags,
                               stats=stats if c["op"] in _COUNTING else None, bsc=_BSC,
                               bsc_stats=stats if c["op"] == H.HULL_OP_SC_BINNED else None,
                               **outs))
        keep.append((outs, stats))
    return H.BatchPlan(jobs, keep=keep + [c["hist"] for c in case], tuning=tuning), keep


def _same(case, keep, factor=1):
    for c, (outs, stats) in zip(case, keep):
        for k, ref in c["ref"].items():
            got = outs[k]
            want = ref * factor if k in ("N", "M") else ref
            assert torch.equal(got, want), (c["op"], k, c["spec"].grid.n, c["spec"].n_hist)
        if c["op"] in _COUNTING + (H.HULL_OP_SC_BINNED,) and factor == 1:
            assert torch.equal(stats, c["ref_stats"]), c["op"]


def test_alone_results_match_the_oracle(batch_case):
    # the per-scan results the batch is held to: the smallest one-pass scan
    # against the oracle's mirror of the same call, bit for bit
    c = min((c for c in batch_case if c["op"] == H.HULL_OP_ALL), key=lambda c: c["spec"].n_hist)
    G = oracle.grid_of(c["spec"].grid)
    p = c["params"]
    op = oracle.OrParams(p.wepl_low, p.wepl_high, p.msc_n_t, p.msc_mode, p.sm_frac_num,
                         p.sm_frac_den, p.sm_mode, p.sm_scope, p.nbr)
    N, M, sc, msc, sm, st = oracle.hull_all(c["h"], G, op)
    for k, want in (("N", N), ("M", M), ("sc_mask", sc), ("msc_mask", msc), ("sm_mask", sm)):
        assert np.array_equal(c["ref"][k].cpu().numpy(), want), k
    assert c["ref_stats"].cpu().tolist() == [st[k] for k in H.STATS_FIELDS]


def test_alone_binned_sc_matches_the_oracle(batch_case):
    c = next(c for c in batch_case if c["op"] == H.HULL_OP_SC_BINNED)
    r = oracle.sc_binned(c["h"], oracle.grid_of(c["spec"].grid),
                         oracle.fbp_params(c["spec"].fbp_geometry()),
                         oracle.bsc_params(wepl_low=1.0, cut_sigmas=3, window=5, thr_num=2,
                                           thr_den=5))
    assert np.array_equal(c["ref"]["bsc_mask"].cpu().numpy(), r["mask"])
    assert H.bsc_stats_dict(c["ref_stats"]) == r["stats"]
    assert r["stats"]["n_bins_carved"] > 0


@pytest.mark.parametrize("streams,graph", [(1, 0), (3, 0), (3, 1), (8, 1)])
def test_batch_equals_alone_over_replays(batch_case, streams, graph):
    plan, keep = _plan(batch_case, H.hullmi_tuning(streams, graph, 0))
    t = plan.tuning
    assert (t.streams, t.use_graph) == (min(streams, len(batch_case)), graph)
    for rep in range(3):
        # eager work between replays: poison every output first
        for outs, stats in keep:
            for v in outs.values():
                v.fill_(7)
            stats.fill_(-1)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        _same(batch_case, keep)
    plan.close()


def test_batch_accumulates_across_graph_replays(batch_case):
    # the counting ops add up; the binned SC ignores the flag and rewrites
    case = [c for c in batch_case if c["op"] in _COUNTING + (H.HULL_OP_SC_BINNED,)]
    plan, keep = _plan(case, H.hullmi_tuning(2, 1, 0), flags=H.HULL_ACCUMULATE)
    for outs, stats in keep:
        for v in outs.values():
            v.zero_()
    torch.cuda.synchronize()
    for rep in range(1, 4):
        plan.launch()
        torch.cuda.synchronize()
        for c, (outs, stats) in zip(case, keep):
            for k in ("N", "M"):
                if k in outs:
                    assert torch.equal(outs[k], c["ref"][k] * rep), (c["op"], k, rep)
            if c["op"] == H.HULL_OP_SC_BINNED:
                assert torch.equal(outs["bsc_mask"], c["ref"]["bsc_mask"]), rep
                assert torch.equal(stats, c["ref_stats"]), rep
    plan.close()


def test_autotuned_plan_is_cached_and_correct(batch_case):
    plan, keep = _plan(batch_case, None)
    t = plan.tuning
    assert 1 <= t.streams <= 16 and t.use_graph in (0, 1) and t.walk_blocks >= 0
    assert 0 <= t.ranges_per_group <= 64 and 0 <= t.length_classes <= 16
    assert 0 <= t.run_stride <= 256
    plan.launch()
    torch.cuda.synchronize()
    _same(batch_case, keep)
    plan2, keep2 = _plan(batch_case, None)         # same shapes: the cached choice
    assert plan2.tuning.as_dict() == t.as_dict()
    plan.close()
    plan2.close()


# every value the autotuner tries for a knob of the counting pass, and the
# extremes the ABI allows: the counts and masks never change
@pytest.mark.parametrize("knobs", [dict(walk_blocks=37), dict(walk_blocks=128),
                                   dict(walk_blocks=256), dict(ranges_per_group=1),
                                   dict(ranges_per_group=2), dict(ranges_per_group=4),
                                   dict(ranges_per_group=8), dict(ranges_per_group=64),
                                   dict(length_classes=1), dict(length_classes=8),
                                   dict(run_stride=1), dict(run_stride=4), dict(run_stride=16),
                                   dict(run_stride=64), dict(run_stride=256),
                                   dict(walk_blocks=64, ranges_per_group=3, length_classes=5,
                                        run_stride=3)])
def test_launch_choices_change_nothing(batch_case, knobs):
    t = H.hullmi_tuning(2, 1)
    for k, v in knobs.items():
        setattr(t, k, v)
    plan, keep = _plan(batch_case, t)
    assert plan.tuning.as_dict() == t.as_dict()
    plan.launch()
    torch.cuda.synchronize()
    _same(batch_case, keep)
    plan.close()


def test_jobs_may_share_their_histories(batch_case):
    """Two jobs reading one scan's histories with outputs of their own are a
    valid plan (only writes may not overlap); both equal the scan alone."""
    c = next(c for c in batch_case if c["op"] == H.HULL_OP_ALL and c["spec"].n_hist > 0)
    keep, jobs = [], []
    for _ in range(2):
        outs = _outputs(c["op"], c["V"])
        st = torch.zeros(6, dtype=torch.int64, device=DEV)
        jobs.append(H.make_job(c["op"], c["hist"], c["grid"], c["params"], stats=st, **outs))
        keep.append((outs, st))
    plan = H.BatchPlan(jobs, keep=keep + [c["hist"]], tuning=H.hullmi_tuning(2, 0))
    plan.launch()
    torch.cuda.synchronize()
    _same([c, c], keep)
    plan.close()
    # two chunks accumulating into one volume would race on it: refused
    N = keep[0][0]["N"]
    bad = [H.make_job(H.HULL_OP_SC, c["hist"].slice(a, b), c["grid"], c["params"],
                      flags=H.HULL_ACCUMULATE, N=N) for a, b in ((0, 100), (100, 200))]
    with pytest.raises(H.HullError):
        H.BatchPlan(bad, tuning=H.hullmi_tuning(2, 0))


def test_range_counters_at_their_cap():
    """5 x 65,535 copies of one line in one slice, walked by a single
    workgroup: the plan makes five ranges of exactly 65,535 items, each
    filling the same 16-bit LDS counters to their largest value; the sums are
    exact."""
    g = gen.Grid((24, 20, 4), (1.0, 1.0, 2.5))
    n = 5 * 65_535
    one = dict(x_in=-30.0, y_in=-4.3, z_in=1.1, x_out=30.0, y_out=5.7, z_out=1.4, angle_deg=0.0)
    h = {k: np.full(n, v, np.float32) for k, v in one.items()}
    h["wepl"] = np.full(n, 0.5, np.float32)
    rN, rM, rst = oracle.counts(h, oracle.grid_of(g))
    assert rN.max() == n
    hist = H.Histories.from_numpy(h, DEV)
    V = g.voxels
    N = torch.zeros(V, dtype=torch.int32, device=DEV)
    M = torch.zeros(V, dtype=torch.int32, device=DEV)
    st = torch.zeros(6, dtype=torch.int64, device=DEV)
    job = H.make_job(H.HULL_OP_ALL, hist, g, H.make_params(), stats=st, N=N, M=M)
    plan = H.BatchPlan([job], keep=[hist, N, M, st], tuning=H.hullmi_tuning(1, 0, 1))
    plan.launch()
    torch.cuda.synchronize()
    assert np.array_equal(N.cpu().numpy(), rN) and np.array_equal(M.cpu().numpy(), rM)
    assert H.stats_dict(st) == rst
    plan.close()


def test_split_ranges_flush_at_every_piece():
    """Coarse ranges of equal estimated work over 3 x 65,535 short lines (3
    voxels each) and 65,535 long ones (28 voxels) in one slice: the first two
    hold about 85,000 short lines each, more than a 16-bit counter can take, so
    the plan splits them into pieces of at most 65,535 items; the workgroup
    that walks a coarse range must write out its tile at every piece boundary.
    Two walk workgroups, one coarse range each at a time; the sums are exact."""
    g = gen.Grid((24, 20, 4), (1.0, 1.0, 2.5))
    short = dict(x_in=-30.0, y_in=50.7, z_in=1.1, x_out=30.0, y_out=-9.3, z_out=1.15, angle_deg=0.0)
    long = dict(x_in=-30.0, y_in=-4.3, z_in=1.1, x_out=30.0, y_out=5.7, z_out=1.4, angle_deg=0.0)
    ns, nl = 3 * 65_535, 65_535
    h = {k: np.concatenate([np.full(ns, short[k], np.float32), np.full(nl, long[k], np.float32)])
         for k in short}
    h["wepl"] = np.full(ns + nl, 0.5, np.float32)
    rN, rM, rst = oracle.counts(h, oracle.grid_of(g))
    assert rN.max() == ns and rst["n_visits_low"] == 3 * ns + 28 * nl
    hist = H.Histories.from_numpy(h, DEV)
    V = g.voxels
    N = torch.zeros(V, dtype=torch.int32, device=DEV)
    M = torch.zeros(V, dtype=torch.int32, device=DEV)
    st = torch.zeros(6, dtype=torch.int64, device=DEV)
    job = H.make_job(H.HULL_OP_ALL, hist, g, H.make_params(), stats=st, N=N, M=M)
    plan = H.BatchPlan([job], keep=[hist, N, M, st], tuning=H.hullmi_tuning(1, 0, 2, 1))
    plan.launch()
    torch.cuda.synchronize()
    assert np.array_equal(N.cpu().numpy(), rN) and np.array_equal(M.cpu().numpy(), rM)
    assert H.stats_dict(st) == rst
    plan.close()


# ---------------------------------------------------------------------------
# serving

_HOST_OUT = {H.HULL_OP_SC: ("N", "sc_mask"), H.HULL_OP_MSC: ("N", "msc_mask"),
             H.HULL_OP_SM: ("M", "sm_mask"),
             H.HULL_OP_ALL: ("N", "M", "sc_mask", "msc_mask", "sm_mask"),
             H.HULL_OP_FBP: ("image", "fbp_mask"), H.HULL_OP_FBP_CUT: ("image", "fbp_mask"),
             H.HULL_OP_SC_BINNED: ("bsc_mask",)}
_NP = {"N": np.int32, "M": np.int32, "image": np.float32}


def _submit_all(srv, case):
    tickets = []
    for c in case:
        outs = {k: np.full(c["V"], 3, dtype=_NP.get(k, np.uint8)) for k in _HOST_OUT[c["op"]]}
        t = srv.submit(c["op"], c["h"], c["grid"], c["params"], c["fbp"], bsc=_BSC, **outs)
        tickets.append((t, outs))
    return tickets


def _check_served(case, tickets, srv):
    for c, (t, outs) in zip(case, tickets):
        r = srv.wait(t)
        assert r["status"] == H.HULL_OK
        assert r["t_arrive_ns"] <= r["t_admit_ns"] <= r["t_done_ns"]
        assert r["device_ms"] + 1e-3 >= r["compute_ms"] >= 0.0
        for k, a in outs.items():
            assert np.array_equal(a, c["ref"][k].cpu().numpy()), (c["op"], k)
        zero = dict.fromkeys(H.BSC_STATS_FIELDS, 0)
        if c["op"] in _COUNTING:
            assert [r["stats"][k] for k in H.STATS_FIELDS] == c["ref_stats"].cpu().tolist()
            assert r["bsc_stats"] == zero
        elif c["op"] == H.HULL_OP_SC_BINNED:
            assert r["bsc_stats"] == H.bsc_stats_dict(c["ref_stats"])
            assert all(v == 0 for v in r["stats"].values())
        else:
            assert r["bsc_stats"] == zero and all(v == 0 for v in r["stats"].values())


def test_served_mix_equals_alone(batch_case):
    srv = H.Server(hbm_budget=4 << 30, max_slots=4)
    tickets = _submit_all(srv, batch_case + batch_case)     # every scan twice, interleaved
    _check_served(batch_case + batch_case, tickets, srv)
    st = srv.stats()
    assert st["completed"] == 2 * len(batch_case) and st["failed"] == 0
    assert st["queued"] == 0 and st["running"] == 0 and st["bytes_in_use"] == 0
    assert 0 < st["bytes_peak"] <= st["bytes_budget"]
    srv.close()


def test_served_one_at_a_time_under_a_tight_budget(batch_case):
    fps = [H.hull_footprint_bytes(c["op"], c["grid"], c["spec"].n_hist if c["h"]["wepl"].size else 0,
                                  c["fbp"]) for c in batch_case]
    budget = max(fps) + 4096
    srv = H.Server(hbm_budget=budget, max_slots=3)
    tickets = _submit_all(srv, batch_case)
    _check_served(batch_case, tickets, srv)
    assert srv.stats()["bytes_peak"] <= budget
    srv.close()


def test_server_errors_and_timeouts(batch_case):
    c = max(batch_case, key=lambda c: c["h"]["wepl"].size)
    fp = H.hull_footprint_bytes(c["op"], c["grid"], c["h"]["wepl"].size, c["fbp"])
    srv = H.Server(hbm_budget=fp // 2, max_slots=2)
    with pytest.raises(H.HullError) as e:
        srv.submit(c["op"], c["h"], c["grid"], c["params"], c["fbp"])
    assert e.value.status == H.HULL_ENOMEM
    bad = dict(c["h"])
    bad["wepl"] = bad["wepl"][:-1].copy()                  # lengths disagree
    with pytest.raises(ValueError):
        srv.submit(c["op"], bad, c["grid"], c["params"], c["fbp"])
    with pytest.raises(H.HullError) as e:
        srv.wait(12345)
    assert e.value.status == H.HULL_EINVAL
    srv.close()
    srv = H.Server(hbm_budget=2 * fp, max_slots=1)
    t = srv.submit(c["op"], c["h"], c["grid"], c["params"], c["fbp"])
    r = srv.wait(t, timeout_us=0)       # a scan of this size is not done within microseconds
    if r is None:
        r = srv.wait(t)
    assert r["status"] == H.HULL_OK
    with pytest.raises(H.HullError):
        srv.wait(t)                     # retired
    srv.close()
