"""GPU parity of the binned SC (Section 3.2 as the paper ran it, with the data
cuts of Section 2.2): per-bin kept counts and sums, the carved volume, the
mask and the counters equal the oracle's exactly."""
import sys

import numpy as np
import pytest
import torch

import gen
import oracle
from paper_1402_1720_amd import hullmi as H

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_bsc(h, grid, geo, bp=None, ws=None):
    bp = bp or dict(wepl_low=1.0, cut_sigmas=3, window=5, thr_num=2, thr_den=5)
    P = H.make_fbp_params(geo)
    nb = int(geo.nu) * int(geo.nv) * int(geo.n_angles)
    V = grid.voxels
    kn = torch.empty(nb, dtype=torch.int32, device=DEV)
    ks = torch.empty(nb, dtype=torch.int64, device=DEV)
    carved = torch.empty(V, dtype=torch.uint8, device=DEV)
    mask = torch.empty(V, dtype=torch.uint8, device=DEV)
    st = torch.empty(6, dtype=torch.int64, device=DEV)
    H.hull_sc_binned(H.Histories.from_numpy(h, DEV), grid, P, H.make_bsc_params(**bp), mask,
                     kept_n=kn, kept_sum=ks, carved=carved, stats=st, ws=ws)
    torch.cuda.synchronize()
    return dict(kept_n=kn.cpu().numpy().view(np.uint32), kept_sum=ks.cpu().numpy(),
                carved=carved.cpu().numpy(), mask=mask.cpu().numpy(), stats=H.bsc_stats_dict(st))


def cpu_bsc(h, grid, geo, bp=None):
    bp = bp or dict(wepl_low=1.0, cut_sigmas=3, window=5, thr_num=2, thr_den=5)
    return oracle.sc_binned(h, oracle.grid_of(grid), oracle.fbp_params(geo), oracle.bsc_params(**bp))


def check_equal(g, r, what=""):
    for k in ("kept_n", "kept_sum", "carved", "mask"):
        if not np.array_equal(g[k], r[k]):
            bad = np.flatnonzero(g[k] != r[k])
            raise AssertionError(f"{what} {k}: {bad.size} differ, first {bad[:5]} "
                                 f"gpu {g[k][bad[:5]]} oracle {r[k][bad[:5]]}")
    assert g["stats"] == r["stats"], (what, g["stats"], r["stats"])


def run_both(h, grid, geo, bp=None, what=""):
    say(what, "n", len(h["wepl"]))
    g = gpu_bsc(h, grid, geo, bp)
    r = cpu_bsc(h, grid, geo, bp)
    check_equal(g, r, what)
    return g, r


def test_config1_both_bin_heights():
    spec = gen.config_spec(1)
    h = gen.generate(spec)
    for dv in (5.0, 2.5):
        g, r = run_both(h, spec.grid, spec.fbp_geometry(du=1.0, dv=dv), what=f"config1 dv {dv}")
        assert r["stats"]["n_bins_carved"] > 0


def test_config2_full_scan():
    """The 200x200x32 scan with 1e7 noisy histories and 180 angles, 1 mm x
    5 mm bins, paper parameters; the launch configuration the benchmark times."""
    spec = gen.config_spec(2)
    h = gen.generate(spec)
    g, r = run_both(h, spec.grid, spec.fbp_geometry(du=1.0, dv=5.0), what="config2")
    assert r["stats"]["n_cut"] > 0 and r["stats"]["n_bins_carved"] > 100_000


def test_outliers_the_cut_removes():
    """The full-scale scan's first 2e6 histories (its first 3.6 gantry angles,
    about 55 per bin): noise, 2% uniform outliers, bins matched to the slices."""
    spec = gen.config_spec(3)
    h = gen.generate(spec, 0, 2_000_000)
    g, r = run_both(h, spec.grid, spec.fbp_geometry(du=1.0, dv=2.5), what="outliers")
    assert r["stats"]["n_cut"] > 1000


@pytest.mark.parametrize("bp", [dict(wepl_low=1.0, cut_sigmas=0, window=5, thr_num=2, thr_den=5),
                                dict(wepl_low=2.5, cut_sigmas=1, window=3, thr_num=1, thr_den=2),
                                dict(wepl_low=1.0, cut_sigmas=64, window=1, thr_num=0, thr_den=1),
                                dict(wepl_low=-0.5, cut_sigmas=2, window=7, thr_num=3, thr_den=4)])
def test_parameters(bp):
    spec = gen.config_spec(1, n_hist=300_000)
    h = gen.generate(spec)
    h = {k: v.copy() for k, v in h.items()}
    h["wepl"] += np.random.default_rng(3).normal(0, 1.0, h["wepl"].size).astype(np.float32)
    run_both(h, spec.grid, spec.fbp_geometry(du=1.0, dv=2.5), bp, what=str(bp))


def test_unsorted_histories_and_wide_wepl_take_the_global_sums():
    """Shuffled angles defeat the per-chunk LDS planes, WEPL beyond 1024 mm
    skips the packed sums; odd values: NaN, beyond 2^16 mm, off the detector,
    parallel to it, an angle that cannot be binned."""
    spec = gen.config_spec(1, n_hist=400_000)
    h = gen.generate(spec)
    perm = np.random.default_rng(11).permutation(h["wepl"].size)
    h = {k: v[perm].copy() for k, v in h.items()}
    rng = np.random.default_rng(12)
    wide = rng.random(h["wepl"].size) < 0.01
    h["wepl"][wide] = rng.uniform(-60000, 60000, wide.sum()).astype(np.float32)
    h["wepl"][0] = np.float32("nan")
    h["wepl"][1] = 70000.0
    h["y_in"][2] = 1e9
    h["x_out"][3] = h["x_in"][3]
    h["angle_deg"][4] = 3e9
    run_both(h, spec.grid, spec.fbp_geometry(du=1.0, dv=2.5), what="unsorted")


def test_sums_of_squares_beyond_64_bits():
    """5000 histories of about 60 m WEPL in one bin: sum w_q^2 exceeds 2^64,
    and the few 0.1 mm ones are more than 3 sigma away and are cut."""
    g = gen.Grid((16, 16, 4), (1.0, 1.0, 2.5))
    geo = gen.FbpGeometry(src_dist=2000.0, du=1.0, dv=2.5, nu=32, nv=4, u0=-16.0, v0=-5.0,
                          n_angles=4, angle0=0.0, dangle=90.0)
    rng = np.random.default_rng(21)
    w = np.concatenate([rng.uniform(59000, 61000, 5000), [0.1] * 3]).astype(np.float32)
    n = w.size
    h = dict(x_in=np.full(n, -100.0), y_in=np.full(n, 3.5), z_in=np.full(n, 1.25),
             x_out=np.full(n, 100.0), y_out=np.full(n, 3.5), z_out=np.full(n, 1.25),
             angle_deg=np.zeros(n), wepl=w)
    h = {k: np.asarray(v, np.float32) for k, v in h.items()}
    wq = np.rint(w.astype(np.float64) * 1024).astype(np.int64)
    assert sum(int(x) * int(x) for x in wq) > 2 ** 64
    gres, r = run_both(h, g, geo, what="wide sums")
    assert r["stats"]["n_cut"] == 3


def test_distant_source_takes_the_integer_set_up():
    """A source 20 m away: the bin lines' coordinates exceed 2^23 (1/1024
    voxel), beyond the exact FP64 slice set-up, so the carve takes the
    64-bit integer one; same result as the oracle."""
    spec = gen.config_spec(1, n_hist=200_000)
    h = gen.generate(spec)
    geo = spec.fbp_geometry(du=1.0, dv=2.5)
    geo = gen.FbpGeometry(src_dist=20000.0, du=geo.du, dv=geo.dv, nu=geo.nu, nv=geo.nv,
                          u0=geo.u0, v0=geo.v0, n_angles=geo.n_angles, angle0=geo.angle0,
                          dangle=geo.dangle)
    assert 20000.0 / spec.grid.d[0] * 1024 > 2 ** 23
    g, r = run_both(h, spec.grid, geo, what="distant source")
    assert r["stats"]["n_bins_carved"] > 0


def test_detector_plane_beyond_the_lds():
    """Fine bins: a detector plane of 16-byte sums larger than the LDS turns
    the per-chunk planes of the first pass off; 8-byte kept sums still fit
    one plane (or none)."""
    g = gen.Grid((32, 32, 16), (1.0, 1.0, 2.5))
    spec = gen.ScanSpec(g, 300_000, 36, gen.head_phantom(g), 0x5EED0110, sigma=1.0)
    h = gen.generate(spec)
    for du, dv, cut_planes in ((0.2, 0.8, 1), (0.1, 0.5, 0)):
        geo = spec.fbp_geometry(du=du, dv=dv)
        assert geo.nu * geo.nv * 16 > 160 * 1024
        assert (geo.nu * geo.nv * 8 <= 160 * 1024) == (cut_planes == 1)
        run_both(h, g, geo, what=f"fine bins {du} x {dv}")


def test_empty_and_tiny_inputs_and_workspace_reuse():
    spec = gen.config_spec(1, n_hist=1000)
    geo = spec.fbp_geometry(du=1.0, dv=2.5)
    h = gen.generate(spec)
    empty = {k: v[:0] for k, v in h.items()}
    run_both(empty, spec.grid, geo, what="empty")
    for n in (1, 63, 1000):
        run_both({k: v[:n] for k, v in h.items()}, spec.grid, geo, what=f"n={n}")
    # one workspace for two calls in a row, the second smaller
    P = H.make_fbp_params(geo)
    ws = H.workspace(H.HULL_OP_SC_BINNED, spec.grid, 1000, DEV, P)
    for n in (1000, 400):
        part = {k: v[:n] for k, v in h.items()}
        check_equal(gpu_bsc(part, spec.grid, geo, ws=ws), cpu_bsc(part, spec.grid, geo), "reuse")


def test_outputs_left_to_the_workspace():
    """kept_n, kept_sum, carved and stats may be omitted: the mask is the same."""
    spec = gen.config_spec(1, n_hist=100_000)
    geo = spec.fbp_geometry(du=1.0, dv=2.5)
    h = gen.generate(spec)
    mask = torch.empty(spec.grid.voxels, dtype=torch.uint8, device=DEV)
    H.hull_sc_binned(H.Histories.from_numpy(h, DEV), spec.grid, H.make_fbp_params(geo),
                     H.make_bsc_params(), mask)
    torch.cuda.synchronize()
    assert np.array_equal(mask.cpu().numpy(), cpu_bsc(h, spec.grid, geo)["mask"])
