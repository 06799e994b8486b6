"""Pins for the oracle's counts N and M (Sections 3.3-3.4) and the SC hull on
synthetic scans: conservation, order independence, and the containment
invariant of a noise-free SC hull."""
import numpy as np

import gen
import oracle


def _spec1(n=30_000):
    return gen.config_spec(1, n_hist=n)


def test_conservation_and_stats():
    spec = _spec1()
    h = gen.generate(spec)
    G = oracle.grid_of(spec.grid)
    N, M, st = oracle.counts(h, G)
    assert N.sum() == st["n_visits_low"] and M.sum() == st["n_visits_high"]
    w = h["wepl"]
    assert st["n_low"] == int((w < 1.0).sum()) and st["n_high"] == int((w > 5.0).sum())
    assert st["n_skipped"] == 0


def test_counts_equal_per_line_enumeration():
    spec = _spec1(3000)
    h = gen.generate(spec)
    G = oracle.grid_of(spec.grid)
    N, M, _ = oracle.counts(h, G)
    status, qin, qout = oracle.quantize(h, G)
    low = (h["wepl"] < 1.0) & (status == 0)
    high = (h["wepl"] > 5.0) & (status == 0)
    refN = np.zeros_like(N)
    refM = np.zeros_like(M)
    for i in np.nonzero(low)[0]:
        refN[oracle.line_cells(qin[i], qout[i], G)] += 1
    for i in np.nonzero(high)[0]:
        refM[oracle.line_cells(qin[i], qout[i], G)] += 1
    assert np.array_equal(N, refN) and np.array_equal(M, refM)


def test_order_and_chunking_do_not_matter():
    spec = _spec1(20_000)
    h = gen.generate(spec)
    G = oracle.grid_of(spec.grid)
    N, M, _ = oracle.counts(h, G)
    perm = np.random.default_rng(1).permutation(len(h["wepl"]))
    Np, Mp, _ = oracle.counts({k: v[perm] for k, v in h.items()}, G)
    assert np.array_equal(N, Np) and np.array_equal(M, Mp)
    a, b = 7_777, 20_000
    N1, M1, _ = oracle.counts({k: v[:a] for k, v in h.items()}, G)
    N2, M2, _ = oracle.counts({k: v[a:b] for k, v in h.items()}, G)
    assert np.array_equal(N, N1 + N2) and np.array_equal(M, M1 + M2)


def test_noise_free_sc_hull_contains_the_shrunk_skull():
    """Every line through a point p with ball(p, r') inside the skull E has a chord
    of at least 2 r' in E, where the RSP is at least rho_min = 1.04, so its WEPL is
    at least 2 r' rho_min. With r' = E_L / (2 rho_min) + 0.01 mm (margin for FP32
    and 1/1024-voxel rounding, both near 1e-3 mm) no such line is low. Points of
    s * E with s = 1 - r'/a_min have that ball inside E (support functions:
    s h_E(u) + r' <= h_E(u) because h_E(u) >= a_min). So every voxel whose closed
    box lies in s * E must survive SC (Section 3.2)."""
    spec = _spec1(100_000)
    h = gen.generate(spec)
    G = oracle.grid_of(spec.grid)
    N, _, _ = oracle.counts(h, G, want_m=False)
    sc = oracle.sc(N)
    skull = spec.phantom[0]
    r = 1.0 / (2 * 1.04) + 0.01
    s = 1.0 - r / min(skull.semi)
    (nx, ny, nz), (dx, dy, dz), (x0, y0, z0) = spec.grid.n, spec.grid.d, spec.grid.origin
    inside = np.ones((nz, ny, nx), dtype=bool)
    for cx in (0, 1):
        for cy in (0, 1):
            for cz in (0, 1):
                x = x0 + (np.arange(nx) + cx) * dx
                y = y0 + (np.arange(ny) + cy) * dy
                z = z0 + (np.arange(nz) + cz) * dz
                zz, yy, xx = np.meshgrid(z, y, x, indexing="ij")
                q = (xx / (s * skull.semi[0])) ** 2 + (yy / (s * skull.semi[1])) ** 2 + \
                    (zz / (s * skull.semi[2])) ** 2
                inside &= q <= 1.0
    inside = inside.reshape(-1)
    assert inside.sum() > 5000
    assert sc[inside].all()
    # and SC carves most of the air: the hull is within a few voxels of the skull
    truth = gen.phantom_rsp(spec.phantom, gen.voxel_centres(spec.grid)).reshape(-1) > 0
    assert sc.sum() < 1.25 * truth.sum()


def test_msc_count_hull_contains_sc_hull():
    spec = gen.config_spec(2, n_hist=200_000)
    h = gen.generate(spec)
    G = oracle.grid_of(spec.grid)
    N, M, _ = oracle.counts(h, G)
    sc = oracle.sc(N)
    for nt in (1, 5, 50):
        msc = oracle.msc(N, G, nt, oracle.MSC_COUNT)
        assert np.all(msc >= sc)
    assert np.array_equal(oracle.msc(N, G, 1, oracle.MSC_COUNT), sc)


def test_cutoffs_are_strict():
    """I_L takes WEPL < E_L and I_H takes WEPL > E_H (Sections 3.2, 3.4): a WEPL
    equal to a cutoff is in neither set."""
    n = 6
    one_below = float(np.nextafter(np.float32(1.0), np.float32(0.0)))
    five_above = float(np.nextafter(np.float32(5.0), np.float32(9.0)))
    w = np.array([1.0, one_below, 5.0, five_above, -3.0, 3.0], dtype=np.float32)
    h = dict(x_in=np.full(n, -100, np.float32), y_in=np.zeros(n, np.float32),
             z_in=np.zeros(n, np.float32), x_out=np.full(n, 100, np.float32),
             y_out=np.zeros(n, np.float32), z_out=np.zeros(n, np.float32),
             angle_deg=np.zeros(n, np.float32), wepl=w)
    G = oracle.make_grid((8, 8, 2), (1.0, 1.0, 1.0), (-4.0, -4.0, -1.0))
    N, M, st = oracle.counts(h, G, 1.0, 5.0)
    assert st["n_low"] == 2 and st["n_high"] == 1
    assert N.sum() == 2 * 8 and M.sum() == 8
