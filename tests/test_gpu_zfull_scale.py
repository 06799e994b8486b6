"""Full-scale parity: the 256x256x64 scan (0.78125 x 0.78125 x 2.5 mm voxels)
with 2e8 histories at 360 gantry angles, WEPL noise 3 mm and 2% uniform
outliers, resident on the device and counted by one hull_all call in the
launch configuration the benchmark times: six internal batches of
33,341,440 histories (the last 33,292,800), alternating between the caller's
stream and the library's second stream and accumulating into one N and one M,
one walk workgroup per CU with eight coarse ranges each, 259-counter tile
rows.

The oracle counts the same histories chunk by chunk on the host (counts are
integers, so chunking cannot change them; the oracle's own chunking pin fixes
that). Compared bit for bit: the full N and M volumes (the crossing counts of
Sections 3.3 and 3.4), the counters, and every mask rule on those volumes —
SC (Algorithm 1), MSC by count and by the neighbour difference of Algorithm 2
(in-plane and 3-D neighbourhoods), SM by fraction of max M and by Algorithm
3's steepest-slope threshold, per volume and per slice. The FDK hull of the
same scan (the other half of the benchmark step, Section 3.1) is held to the
FP64 oracle's image within 1e-4 of its largest magnitude.

The oracle pass takes a few minutes on 16 host cores; progress lines go to
the terminal (capture disabled) so that a quiet stretch never exceeds about
ten seconds."""
import time

import numpy as np
import pytest
import torch

import gen
import oracle
from paper_1402_1720_amd import hullmi as H

pytestmark = [pytest.mark.gpu, pytest.mark.slow, pytest.mark.timeout(1500)]
DEV = torch.device("cuda:0")
CHUNK = 10_000_000


def test_config3_full_volume_bit_exact(capfd):
    def say(*a):
        with capfd.disabled():
            print("[full-scale]", *a, flush=True)

    spec = gen.config_spec(3)
    n = spec.n_hist
    grid = spec.grid
    V = grid.voxels
    G = oracle.grid_of(grid)
    say(f"{n} histories on {grid.n}: generating into device arrays and counting on the host")
    arr = {k: torch.empty(n, dtype=torch.float32, device=DEV) for k in gen.FIELDS}
    host = {k: np.empty(n, np.float32) for k in gen.FIELDS}   # for the FDK oracle
    rN = np.zeros(V, np.int64)
    rM = np.zeros(V, np.int64)
    rst = dict.fromkeys(H.STATS_FIELDS, 0)
    t0 = time.time()
    for h0 in range(0, n, CHUNK):
        h1 = min(n, h0 + CHUNK)
        h = gen.generate(spec, h0, h1)
        for k in gen.FIELDS:
            arr[k][h0:h1].copy_(torch.from_numpy(h[k]))
            host[k][h0:h1] = h[k]
        cN, cM, cst = oracle.counts(h, G)
        rN += cN
        rM += cM
        for k in rst:
            rst[k] += cst[k]
        say(f"oracle: {h1} of {n} histories, {time.time() - t0:.0f} s")
    assert rN.max() < 2**31 and rM.max() < 2**31
    rN = rN.astype(np.int32)
    rM = rM.astype(np.int32)

    hist = H.Histories(arr)
    ws = H.workspace(H.HULL_OP_ALL, grid, n, DEV)
    N = torch.zeros(V, dtype=torch.int32, device=DEV)
    M = torch.zeros(V, dtype=torch.int32, device=DEV)
    sc, msc, sm = (torch.zeros(V, dtype=torch.uint8, device=DEV) for _ in range(3))
    st = torch.zeros(6, dtype=torch.int64, device=DEV)
    say("hull_all on the device (SC, MSC count 5, SM 3/5 of max M)")
    H.hull_all(hist, grid, H.make_params(), N, M, sc, msc, sm, stats=st, ws=ws)
    torch.cuda.synchronize()
    gN, gM = N.cpu().numpy(), M.cpu().numpy()
    bad_n = np.flatnonzero(gN != rN)
    bad_m = np.flatnonzero(gM != rM)
    assert bad_n.size == 0, f"N differs at {bad_n.size} voxels, first {bad_n[:8]}"
    assert bad_m.size == 0, f"M differs at {bad_m.size} voxels, first {bad_m[:8]}"
    gst = H.stats_dict(st)
    assert gst == rst, (gst, rst)
    assert rst["n_visits_low"] + rst["n_visits_high"] > 3e10   # a real full-scale pass
    assert np.array_equal(sc.cpu().numpy(), oracle.sc(rN))
    assert np.array_equal(msc.cpu().numpy(), oracle.msc(rN, G, 5))
    assert np.array_equal(sm.cpu().numpy(), oracle.sm(rM, G, 3, 5)[0])
    say("N, M, counters and the default masks bit-exact; other rules next")

    # the other rules, each through its own per-scan call (a second count of
    # the whole scan every time, which must give the same volume again)
    cases = [("msc", H.HULL_MSC_NEIGHBOR_DIFF, 50, H.HULL_NBR_INPLANE4),
             ("msc", H.HULL_MSC_NEIGHBOR_DIFF, 50, H.HULL_NBR_SPATIAL6),
             ("sm", H.HULL_SM_MAX_SLOPE, H.HULL_SCOPE_VOLUME, H.HULL_NBR_INPLANE4),
             ("sm", H.HULL_SM_MAX_SLOPE, H.HULL_SCOPE_SLICE, H.HULL_NBR_INPLANE4),
             ("sm", H.HULL_SM_MAX_SLOPE, H.HULL_SCOPE_VOLUME, H.HULL_NBR_SPATIAL6),
             ("sm", H.HULL_SM_FRACTION, H.HULL_SCOPE_SLICE, H.HULL_NBR_INPLANE4)]
    mask = torch.zeros(V, dtype=torch.uint8, device=DEV)
    for rule, mode, a, nbr in cases:
        if rule == "msc":
            H.hull_msc(hist, grid, 1.0, a, mode, nbr, N, mask, ws=ws)
            torch.cuda.synchronize()
            assert np.array_equal(N.cpu().numpy(), rN), (rule, mode, a, nbr)
            ref = oracle.msc(rN, G, a, mode, nbr)
        else:
            H.hull_sm(hist, grid, 5.0, 3, 5, mode, a, nbr, M, mask, ws=ws)
            torch.cuda.synchronize()
            assert np.array_equal(M.cpu().numpy(), rM), (rule, mode, a, nbr)
            ref = oracle.sm(rM, G, 3, 5, mode, a, nbr)[0]
        got = mask.cpu().numpy()
        assert np.array_equal(got, ref), (rule, mode, a, nbr, int((got != ref).sum()))
        say(f"{rule} mode {mode} ({a}, nbr {nbr}) bit-exact, {int(ref.sum())} voxels kept")

    # the FDK hull of the full scan: FP32 image within 1e-4 of the FP64 oracle
    geo = spec.fbp_geometry(du=1.0, dv=5.0)
    fbp = H.make_fbp_params(geo)
    img = torch.zeros(V, dtype=torch.float32, device=DEV)
    fmask = torch.zeros(V, dtype=torch.uint8, device=DEV)
    H.hull_fbp(hist, grid, fbp, img, fmask)
    torch.cuda.synchronize()
    say("FDK hull on the device done; oracle FDK (FP64)")
    ref, rmask, _, _ = oracle.fbp(host, G, oracle.fbp_params(geo))
    got = img.cpu().numpy().astype(np.float64)
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max() / scale
    assert err <= 1e-4, err
    near = np.abs(ref - geo.threshold) <= 1e-4 * scale
    gm = fmask.cpu().numpy()
    assert np.array_equal(gm[~near], rmask[~near])
    say(f"FDK image within {err:.1e} of the oracle's largest value, masks equal")
