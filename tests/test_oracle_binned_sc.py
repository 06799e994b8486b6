"""Pins of the oracle's binned SC (Section 3.2 as the paper ran it, with the
data cuts of Section 2.2): exact-fraction statistics, hand-derived bin lines,
a library box filter, the FDK oracle's FP64 bin means, and a noise-free
invariant that a sign or rotation mistake breaks."""
import statistics
from fractions import Fraction

import numpy as np
import pytest
from scipy import ndimage

import gen
import oracle

# 16 x 16 x 4 grid of 1 x 1 x 2.5 mm voxels, centred; 32 x 4 detector bins of
# 1 x 2.5 mm (powers of two or exact reciprocals are not needed: bin centres
# sit half a bin away from every edge), four gantry angles 90 degrees apart.
GRID = oracle.make_grid((16, 16, 4), (1.0, 1.0, 2.5), (-8.0, -8.0, -5.0))
BINS = oracle.OrFbpParams(2000.0, 1.0, 2.5, -16.0, -5.0, 32, 4, 4, 0.0, 90.0, 0, 0.6)


def _through(k, iu, iv, wepl, p=BINS):
    """Histories parallel to the beam axis crossing x = 0 at the centre of bin
    (iu, iv) at gantry angle k: their crossing point is exactly the centre."""
    n = len(wepl)
    u = p.u0_mm + (iu + 0.5) * p.du_mm
    v = p.v0_mm + (iv + 0.5) * p.dv_mm
    return dict(x_in=np.full(n, -100.0, np.float32), y_in=np.full(n, u, np.float32),
                z_in=np.full(n, v, np.float32), x_out=np.full(n, 100.0, np.float32),
                y_out=np.full(n, u, np.float32), z_out=np.full(n, v, np.float32),
                angle_deg=np.full(n, p.angle0_deg + k * p.dangle_deg, np.float32),
                wepl=np.asarray(wepl, np.float32))


def _cat(parts):
    return {f: np.concatenate([p[f] for p in parts]) for f in gen.FIELDS}


def _bin(k, iu, iv, p=BINS):
    return (k * p.nv + iv) * p.nu + iu


def _exact_keep(ms, k):
    """WEPL values m/1024 (exact), kept iff not more than k population
    standard deviations from the mean, decided with fractions."""
    w = [Fraction(m, 1024) for m in ms]
    mu = statistics.mean(w)
    var = statistics.pvariance(w)
    return [m for m, x in zip(ms, w) if k == 0 or (x - mu) ** 2 <= k * k * var]


def test_cuts_match_exact_fractions():
    rng = np.random.default_rng(0xB5C1)
    parts, expect = [], {}
    for trial in range(40):
        k, iu, iv = int(rng.integers(4)), int(rng.integers(32)), int(rng.integers(4))
        if _bin(k, iu, iv) in expect:
            continue
        n = int(rng.integers(1, 40))
        ms = rng.integers(-2048, 200 * 1024, n).tolist()
        if trial % 3 == 0:   # a few far outliers
            ms += rng.integers(300 * 1024, 400 * 1024, 2).tolist()
        parts.append(_through(k, iu, iv, [m / 1024 for m in ms]))
        expect[_bin(k, iu, iv)] = _exact_keep(ms, 3)
    r = oracle.sc_binned(_cat(parts), GRID, BINS)
    for b, kept in expect.items():
        assert r["kept_n"][b] == len(kept), b
        assert r["kept_sum"][b] == sum(kept), b
    others = np.setdiff1d(np.arange(r["kept_n"].size), list(expect))
    assert not r["kept_n"][others].any()
    assert r["stats"]["n_binned"] == sum(len(p["wepl"]) for p in parts)
    assert r["stats"]["n_cut"] == r["stats"]["n_binned"] - sum(len(v) for v in expect.values())


def test_three_sigma_boundary_and_the_cut_decides_the_carve():
    # nine zeros and one x: |x - mean| = 0.9|x| = 3 sigma exactly -> kept
    r = oracle.sc_binned(_through(0, 5, 1, [0.0] * 9 + [40.0]), GRID, BINS)
    assert r["kept_n"][_bin(0, 5, 1)] == 10 and r["stats"]["n_cut"] == 0
    # ten zeros and one x: 10|x|/11 > 3 sqrt(10)|x|/11 -> cut
    r = oracle.sc_binned(_through(0, 5, 1, [0.0] * 10 + [40.0]), GRID, BINS)
    assert r["kept_n"][_bin(0, 5, 1)] == 10 and r["stats"]["n_cut"] == 1
    # 19 x 0.5 mm and one 50 mm outlier: mean 2.975 mm keeps the bin's line
    # without cuts; the cut drops the outlier and the line (mean 0.5) carves
    h = _through(0, 19, 2, [0.5] * 19 + [50.0])
    line = oracle.line_cells(*oracle.bsc_line(BINS, GRID, 0, 19, 2)[1:], GRID)
    with_cut = oracle.sc_binned(h, GRID, BINS)
    no_cut = oracle.sc_binned(h, GRID, BINS, oracle.bsc_params(cut_sigmas=0))
    assert with_cut["stats"]["n_bins_carved"] == 1 and no_cut["stats"]["n_bins_carved"] == 0
    assert np.flatnonzero(with_cut["carved"]).tolist() == line.tolist()
    assert not no_cut["carved"].any()


def test_mean_at_the_cutoff_is_not_carved():
    # kept mean exactly E_L: "below" is strict
    r = oracle.sc_binned(_through(2, 7, 0, [0.5, 1.5]), GRID, BINS)
    assert r["stats"]["n_bins_carved"] == 0
    r = oracle.sc_binned(_through(2, 7, 0, [0.5, 1.5 - 1 / 1024]), GRID, BINS)
    assert r["stats"]["n_bins_carved"] == 1


def test_bins_follow_the_crossing_point():
    """A history is binned where its line crosses x = 0, at the nearest
    gantry angle bin (modulo the full turn)."""
    rng = np.random.default_rng(0xB5C2)
    n = 3000
    k = rng.integers(0, 4, n)
    iu = rng.integers(0, 32, n)
    iv = rng.integers(0, 4, n)
    fu = rng.uniform(0.05, 0.95, n)   # away from bin edges
    fv = rng.uniform(0.05, 0.95, n)
    u = BINS.u0_mm + (iu + fu) * BINS.du_mm
    v = BINS.v0_mm + (iv + fv) * BINS.dv_mm
    slope_y = rng.uniform(-0.2, 0.2, n)
    slope_z = rng.uniform(-0.05, 0.05, n)
    # angles within 40 degrees of the bin's angle, some written one turn up
    ang = k * 90.0 + rng.uniform(-40, 40, n) + 360.0 * rng.integers(0, 2, n)
    h = dict(x_in=np.full(n, -100.0), y_in=u - 100.0 * slope_y, z_in=v - 100.0 * slope_z,
             x_out=np.full(n, 100.0), y_out=u + 100.0 * slope_y, z_out=v + 100.0 * slope_z,
             angle_deg=ang, wepl=np.full(n, 7.0))
    h = {f: np.asarray(a, np.float32) for f, a in h.items()}
    r = oracle.sc_binned(h, GRID, BINS, oracle.bsc_params(cut_sigmas=0))
    expect = np.bincount(_bin(k, iu, iv), minlength=r["kept_n"].size)
    assert np.array_equal(r["kept_n"], expect)
    assert np.array_equal(r["kept_sum"], expect * 7 * 1024)


def test_bin_lines_hand_derived():
    """Source (-2000, 0, 0) through the bin centre: at gantry angle 0 the bin
    (iu 19, iv 2) line runs along x at y in [3.486, 3.514] mm and z within
    0.005 mm of 1.25 mm, i.e. voxel row (j 11, k 2); at 90 degrees the object
    has turned, so the same bin's line runs along y through column (i 11, k 2).
    The bin at iu 0 (u = -15.5 mm) misses the 16 mm grid."""
    st, qin, qout = oracle.bsc_line(BINS, GRID, 0, 19, 2)
    assert st == oracle.OK
    assert qin.tolist() == [-1992 * 1024, 8 * 1024, 2 * 1024]
    assert qout.tolist() == [8 * 1024, 11 * 1024 + 512, 2 * 1024 + 512]
    cells = oracle.line_cells(qin, qout, GRID)
    assert cells.tolist() == [i + 16 * (11 + 16 * 2) for i in range(16)]
    st, qin, qout = oracle.bsc_line(BINS, GRID, 1, 19, 2)
    cells = oracle.line_cells(qin, qout, GRID)
    assert st == oracle.OK and cells.tolist() == [11 + 16 * (j + 16 * 2) for j in range(16)]
    st, qin, qout = oracle.bsc_line(BINS, GRID, 0, 0, 2)
    assert st == oracle.OK and oracle.line_cells(qin, qout, GRID).size == 0
    # the whole call carves exactly those lines
    h = _cat([_through(0, 19, 2, [0.25] * 3), _through(1, 19, 2, [0.0]), _through(0, 0, 2, [0.1])])
    r = oracle.sc_binned(h, GRID, BINS)
    row = {i + 16 * (11 + 16 * 2) for i in range(16)} | {11 + 16 * (j + 16 * 2) for j in range(16)}
    assert set(np.flatnonzero(r["carved"]).tolist()) == row
    assert r["stats"]["n_bins_carved"] == 3 and r["stats"]["n_visits"] == 32


@pytest.mark.parametrize("window,num,den", [(5, 2, 5), (3, 1, 2), (1, 0, 1), (7, 3, 4)])
def test_blur_matches_a_library_box_filter(window, num, den):
    rng = np.random.default_rng(window * 100 + num)
    g = oracle.make_grid((23, 17, 3), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    carved = (rng.random((3, 17, 23)) < 0.45).astype(np.uint8)
    kern = np.ones((1, window, window), np.int64)
    s = ndimage.correlate((1 - carved).astype(np.int64), kern, mode="constant", cval=0)
    expect = (den * s > num * window * window).astype(np.uint8)
    assert np.array_equal(oracle.bsc_blur(carved, g, window, num, den), expect.reshape(-1))


def test_without_cuts_bins_match_the_fdk_oracles_fp64_means():
    """Same bins as the FDK hull's: with the cuts off, kept count and fixed
    point sum give the FDK oracle's FP64 bin mean to within half a unit of
    1/1024 mm (each WEPL rounded once)."""
    spec = gen.config_spec(1, n_hist=60_000)
    h = gen.generate(spec)
    h = {k: v.copy() for k, v in h.items()}
    h["wepl"] += np.float32(0.3) * np.random.default_rng(5).standard_normal(h["wepl"].size).astype(np.float32)
    geo = spec.fbp_geometry(du=1.0, dv=2.5)
    P = oracle.fbp_params(geo)
    means, used = oracle.fbp_bin(h, P)
    r = oracle.sc_binned(h, oracle.grid_of(spec.grid), P, oracle.bsc_params(cut_sigmas=0))
    n = r["kept_n"].astype(np.float64)
    assert used == r["stats"]["n_binned"] == int(n.sum())
    filled = n > 0
    assert np.all(means[~filled] == 0.0)
    mine = r["kept_sum"][filled] / 1024.0 / n[filled]
    assert np.max(np.abs(mine - means[filled])) <= 2.0 ** -11 + 1e-12


def _cylinder_scan():
    g = gen.Grid((64, 64, 8), (1.0, 1.0, 2.5))
    ph = (gen.Ellipsoid((8.0, -5.0, 0.0), (14.0, 20.0, 1e4), 1.0),)
    spec = gen.ScanSpec(g, 200_000, 90, ph, 0x5EED0777, sigma=0.0)
    return g, spec, gen.generate(spec)


def _inset_voxels(g, d):
    """Voxels whose closed box lies inside the cylinder shrunk by d mm."""
    nx, ny, nz = g.n
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny))
    x0 = g.origin[0] + ii * g.d[0]
    y0 = g.origin[1] + jj * g.d[1]
    ok = np.ones_like(x0, bool)
    for cx in (x0, x0 + g.d[0]):
        for cy in (y0, y0 + g.d[1]):
            ok &= ((cx - 8.0) / (14.0 - d)) ** 2 + ((cy + 5.0) / (20.0 - d)) ** 2 < 1.0
    return np.broadcast_to(ok.reshape(-1), (nz, nx * ny)).reshape(-1)


def test_noise_free_cylinder_keeps_every_voxel_a_millimetre_inside():
    """Noise-free z-invariant object of RSP 1 with curvature radius >= 9.8 mm:
    if a bin's centre line reached a voxel box 1 mm inside the boundary, every
    history of that 1 mm wide bin would pass at least 0.5 mm inside it, along
    a chord of at least 2 sqrt(2 * 9.8 * 0.5 - 0.25) > 6 mm, so the bin's mean
    (cut or not) is above 1 mm and the line is not carved. Mirroring the
    rotation or the detector axis breaks this by thousands of voxels."""
    g, spec, h = _cylinder_scan()
    G = oracle.grid_of(g)
    P = oracle.fbp_params(spec.fbp_geometry(du=1.0, dv=2.5))
    inset = _inset_voxels(g, 1.0)
    r = oracle.sc_binned(h, G, P)
    assert not (inset & r["carved"].astype(bool)).any()
    assert r["mask"][inset].all()
    assert r["stats"]["n_bins_carved"] > 0.5 * r["stats"]["n_bins_used"]
    for f, fn in (("angle_deg", lambda a: (-a) % 360), ("y_in", np.negative)):
        m = dict(h)
        m[f] = fn(h[f]).astype(np.float32)
        if f == "y_in":
            m["y_out"] = -h["y_out"]
        bad = oracle.sc_binned(m, G, P)
        assert (inset & bad["carved"].astype(bool)).sum() > 1000


def test_mirror_call_and_argument_checks():
    g, spec, h = _cylinder_scan()
    h = {k: v[:20000] for k, v in h.items()}
    G = oracle.grid_of(g)
    P = oracle.fbp_params(spec.fbp_geometry(du=1.0, dv=2.5))
    r = oracle.sc_binned(h, G, P)
    kn, ks, carved, mask, st = oracle.hull_sc_binned(h, G, P, oracle.bsc_params())
    assert np.array_equal(kn, r["kept_n"]) and np.array_equal(ks, r["kept_sum"])
    assert np.array_equal(carved, r["carved"]) and np.array_equal(mask, r["mask"])
    assert st == r["stats"]
    for bad in (oracle.bsc_params(window=4), oracle.bsc_params(thr_den=0),
                oracle.bsc_params(cut_sigmas=-1), oracle.bsc_params(cut_sigmas=65),
                oracle.bsc_params(wepl_low=float("nan")), oracle.bsc_params(wepl_low=70000.0)):
        with pytest.raises(ValueError):
            oracle.sc_binned(h, G, P, bad)
