"""Pins for the oracle's FDK hull (Section 3.1): the Shepp-Logan filter against
its Fourier series, the binning on hand-placed histories, and reconstructions
of a uniform sphere in parallel-beam and cone-beam geometry."""
import math
from dataclasses import replace

import numpy as np
import pytest

import gen
import oracle


def _params(**kw):
    base = dict(src_dist=1e12, du=1.0, dv=1.0, nu=1, nv=1, u0=0.0, v0=0.0, n_angles=1,
                angle0=0.0, dangle=360.0, threshold=0.6)
    base.update(kw)
    return oracle.fbp_params(gen.FbpGeometry(**base))


@pytest.mark.parametrize("omega", [0.0, 0.3, 1.0, 2.5])
def test_shepp_logan_frequency_response(omega):
    """sum_n cos(n x) / (4 n^2 - 1) = -(pi/2) |sin(x/2)| (from the Fourier series
    of |sin(x/2)|), so the kernel -2 / (pi^2 du^2 (4 n^2 - 1)) scaled by du maps
    cos(omega j) to |sin(omega/2)| / (pi du) * cos(omega j); 0 at DC."""
    du = 0.5
    nu = 4001
    p = _params(nu=nu, du=du, u0=-0.5 * nu * du)
    j = np.arange(nu)
    row = np.cos(omega * j)
    q = oracle.fbp_filter(p, row)
    mid = slice(nu // 2 - 100, nu // 2 + 100)
    want = abs(math.sin(omega / 2)) / (math.pi * du) * row[mid]
    # truncating the kernel at the row ends leaves a tail of order 1/(pi^2 du L)
    assert np.abs(q[mid] - want).max() < 2e-3


def test_binning_means_and_angle_bins():
    # detector 4 x 2 bins of 1 mm from (-2,-1), 2 angles 0 / 180 degrees
    p = _params(nu=4, nv=2, u0=-2.0, v0=-1.0, n_angles=2, dangle=180.0)
    # lines crossing x = 0 at (u, v): entry (-100, u, v) and exit (100, u, v)
    us = np.array([-1.5, -1.2, 0.5, 0.5, 1.9, 3.0, 0.5], dtype=np.float32)
    vs = np.array([-0.5, -0.9, 0.2, 0.2, 0.99, 0.0, 0.2], dtype=np.float32)
    ang = np.array([0.0, 0.0, 180.0, 180.0, 359.0, 0.0, 1e30], dtype=np.float32)
    w = np.array([1.0, 3.0, 10.0, 20.0, 7.0, 99.0, 5.0], dtype=np.float32)
    h = dict(x_in=np.full(7, -100, np.float32), y_in=us, z_in=vs, x_out=np.full(7, 100, np.float32),
             y_out=us, z_out=vs, angle_deg=ang, wepl=w)
    proj, used = oracle.fbp_bin(h, p)
    proj = proj.reshape(2, 2, 4)
    # u = 3.0 is off the detector; 1e30 degrees cannot be binned
    assert used == 5
    assert proj[0, 0, 0] == 2.0                 # mean of 1 and 3
    assert proj[1, 1, 2] == 15.0                # mean of 10 and 20 at 180 degrees
    assert proj[0, 1, 3] == 7.0                 # 359 degrees rounds to bin 2 == bin 0
    assert proj.sum() == 24.0


def _bin_centre_rays(src_dist, R, nu, nv, n_angles, du=1.0, dv=1.0, centre=(0.0, 0.0, 0.0)):
    """One history per detector bin: the ray from the source (-D, 0, 0) through the
    bin centre on the plane x = 0, with the WEPL of a centred sphere of RSP 1 in
    closed form, 2 sqrt(R^2 - d^2) (d: distance from the sphere centre to the ray).
    An off-centre sphere sits at R(theta) * centre in the lab frame at gantry
    angle theta: the object turns in front of the fixed beam (Section 2.2)."""
    geo = gen.FbpGeometry(src_dist=src_dist, du=du, dv=dv, nu=nu, nv=nv, u0=-0.5 * nu * du,
                          v0=-0.5 * nv * dv, n_angles=n_angles, angle0=0.0,
                          dangle=360.0 / n_angles)
    k, iv, iu = np.meshgrid(np.arange(n_angles), np.arange(nv), np.arange(nu), indexing="ij")
    u = geo.u0 + (iu.reshape(-1) + 0.5) * du
    v = geo.v0 + (iv.reshape(-1) + 0.5) * dv
    D, T = src_dist, 100.0
    pin = np.stack([np.full(u.shape, -T), u * (D - T) / D, v * (D - T) / D], 1)
    pout = np.stack([np.full(u.shape, T), u * (D + T) / D, v * (D + T) / D], 1)
    pin, pout = pin.astype(np.float32), pout.astype(np.float32)
    a, b = pin.astype(np.float64), pout.astype(np.float64)
    th = np.deg2rad(k.reshape(-1) * geo.dangle)
    cx, cy, cz = centre
    lab_c = np.stack([np.cos(th) * cx - np.sin(th) * cy, np.sin(th) * cx + np.cos(th) * cy,
                      np.full(th.shape, cz)], 1)
    a = a - lab_c
    dirn = (b - a - lab_c) / np.linalg.norm(b - a - lab_c, axis=1, keepdims=True)
    dist = np.linalg.norm(a - (a * dirn).sum(1, keepdims=True) * dirn, axis=1)
    w = 2.0 * np.sqrt(np.clip(R * R - dist * dist, 0.0, None))
    h = dict(x_in=pin[:, 0], y_in=pin[:, 1], z_in=pin[:, 2], x_out=pout[:, 0], y_out=pout[:, 1],
             z_out=pout[:, 2], angle_deg=(k.reshape(-1) * geo.dangle).astype(np.float32),
             wepl=w.astype(np.float32))
    return geo, h


def test_parallel_beam_sphere_reconstructs_its_density():
    """As the source recedes FDK becomes parallel-beam FBP, which reconstructs a
    uniform sphere slice by slice (each slice is a disk): interior ~ 1, air ~ 0."""
    R = 30.0
    geo, h = _bin_centre_rays(1e7, R, nu=90, nv=18, n_angles=180)
    grid = gen.Grid((64, 64, 8), (1.0, 1.0, 2.0))
    G = oracle.grid_of(grid)
    img, mask, _, used = oracle.fbp(h, G, oracle.fbp_params(geo))
    assert used == len(h["wepl"])
    c = gen.voxel_centres(grid).reshape(-1, 3)
    r = np.linalg.norm(c, axis=1)
    inner = r < 0.8 * R
    outer = (r > 1.2 * R) & (np.hypot(c[:, 0], c[:, 1]) < 44.0)
    assert abs(img[inner].mean() - 1.0) < 0.01
    assert np.abs(img[inner] - 1.0).max() < 0.05
    assert np.abs(img[outer]).max() < 0.05
    # the 0.6 threshold (Section 3.1) separates them
    assert mask[inner].all() and not mask[outer].any()


def test_cone_beam_sphere_central_slices():
    """A 150 mm source distance makes the cone-beam weights matter: the cosine
    pre-weight D / sqrt(D^2 + u^2 + v^2) and the 1/U^2 distance weight. In the
    mid-plane FDK is the exact fan-beam formula, so the reconstructed disk must
    be flat from the centre to the rim."""
    R = 30.0
    geo, h = _bin_centre_rays(150.0, R, nu=160, nv=12, n_angles=360)
    grid = gen.Grid((64, 64, 4), (1.0, 1.0, 1.0))
    G = oracle.grid_of(grid)
    img, _, _, _ = oracle.fbp(h, G, oracle.fbp_params(geo))
    c = gen.voxel_centres(grid).reshape(-1, 3)
    rxy = np.hypot(c[:, 0], c[:, 1])
    mid = np.abs(c[:, 2]) < 1.0
    for lo, hi in ((0.0, 0.3), (0.3, 0.6), (0.6, 0.8)):
        ring = mid & (rxy >= lo * R) & (rxy < hi * R)
        assert abs(img[ring].mean() - 1.0) < 0.006, (lo, hi, img[ring].mean())
    far = mid & (rxy > 1.2 * R) & (rxy < 40.0)
    assert np.abs(img[far]).max() < 0.05


def test_off_centre_sphere_lands_where_it_is():
    """The backprojection must undo the gantry rotation: an off-centre sphere is
    reconstructed at its own position."""
    R, centre = 12.0, (15.0, 6.0, 0.0)
    geo, h = _bin_centre_rays(400.0, R, nu=120, nv=8, n_angles=180, centre=centre)
    grid = gen.Grid((64, 64, 4), (1.0, 1.0, 1.0))
    img, mask, _, _ = oracle.fbp(h, oracle.grid_of(grid), oracle.fbp_params(geo))
    c = gen.voxel_centres(grid).reshape(-1, 3)
    d = np.linalg.norm(c - np.array(centre), axis=1)
    assert abs(img[d < 0.7 * R].mean() - 1.0) < 0.02
    assert np.abs(img[d > 1.3 * R]).max() < 0.1
    got = c[mask.astype(bool)].mean(axis=0)
    assert np.allclose(got[:2], centre[:2], atol=0.3)


def test_fdk_hull_of_the_head_phantom():
    """The FBP hull (Section 3.1: Shepp-Logan, threshold 0.6) of a noise-free
    head keeps the skull interior and drops the air, given the paper's density
    of histories per detector bin (1 mm x 5 mm bins, Section 3.1)."""
    g = gen.Grid((200, 200, 32), (1.0, 1.0, 3.0))
    spec = gen.ScanSpec(g, 3_600_000, 60, gen.head_phantom(g, inserts=True), seed=12)
    h = gen.generate(spec)
    G = oracle.grid_of(spec.grid)
    geo = spec.fbp_geometry(du=1.0, dv=5.0)
    img, mask, _, _ = oracle.fbp(h, G, oracle.fbp_params(geo))
    cen = gen.voxel_centres(spec.grid)
    truth = gen.phantom_rsp(spec.phantom, cen).reshape(-1)
    core = gen.phantom_rsp(tuple(replace(e, semi=tuple(0.9 * s for s in e.semi))
                                 for e in spec.phantom[:1]), cen).reshape(-1) > 0
    mid = np.zeros_like(core)
    mid.reshape(32, 200, 200)[8:24] = True
    assert mask[core & mid].mean() > 0.99
    assert mask[(truth == 0) & mid].mean() < 0.02


def test_cuts_off_is_the_plain_fdk_hull():
    spec = gen.config_spec(1, n_hist=40_000)
    h = gen.generate(spec)
    P = oracle.fbp_params(spec.fbp_geometry(du=1.0, dv=2.5))
    G = oracle.grid_of(spec.grid)
    img, mask, proj, used = oracle.fbp(h, G, P)
    img0, mask0, _, kept = oracle.fbp_cut(h, G, P, k=0)
    assert kept == used
    assert np.array_equal(img, img0) and np.array_equal(mask, mask0)


def test_cuts_remove_outliers_from_the_fdk_hull():
    """Twelve histories per bin along each bin-centre ray of a uniform sphere:
    eleven carry the sphere's chord, and in a third of the bins the twelfth
    carries a far outlier (+150 mm). With n = 12 one outlier x among equal
    values v lies 11|x - v|/12 from the mean while 3 sigma is
    3 sqrt(11)|x - v|/12, so the cut drops exactly the outliers and leaves
    the equal values (0.083|x - v| from the mean): the hull after the cuts is
    the clean scan's, and without cuts the outliers spoil it."""
    R = 30.0
    geo, h = _bin_centre_rays(1e7, R, nu=90, nv=18, n_angles=180)
    grid = gen.Grid((64, 64, 8), (1.0, 1.0, 2.0))
    G = oracle.grid_of(grid)
    P = oracle.fbp_params(geo)
    clean_img, clean_mask, _, _ = oracle.fbp(h, G, P)
    rng = np.random.default_rng(7)
    reps = {k: np.repeat(v, 12) for k, v in h.items()}
    bad = rng.random(len(h["wepl"])) < 1 / 3
    w = reps["wepl"].reshape(-1, 12).copy()
    w[bad, 11] += np.float32(150.0)
    reps["wepl"] = w.reshape(-1)
    img, mask, proj, kept = oracle.fbp_cut(reps, G, P, k=3)
    assert kept == len(reps["wepl"]) - int(bad.sum())
    assert np.abs(img - clean_img).max() < 1e-9
    assert np.array_equal(mask, clean_mask)
    raw, raw_mask, _, _ = oracle.fbp(reps, G, P)
    assert np.abs(raw - clean_img).max() > 0.5
    b, keep, binned, cut = oracle.bsc_cut(reps, P, 3)
    assert binned == len(reps["wepl"]) and cut == int(bad.sum())
    assert np.array_equal(~keep.reshape(-1, 12)[:, 11], bad)
