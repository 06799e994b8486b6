"""GPU parity of the FDK hull (Section 3.1): FP32 image within 1e-4 of the
FP64 oracle's maximum |f|, masks equal except where the oracle's value lies
within that tolerance of the threshold."""
import numpy as np
import pytest
import torch

import gen
import oracle
from paper_1402_1720_amd import hullmi as H
from tests.test_oracle_fbp import _bin_centre_rays

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL = 1e-4


def _run(h, grid, geo):
    V = grid.voxels
    img = torch.zeros(V, dtype=torch.float32, device=DEV)
    mask = torch.zeros(V, dtype=torch.uint8, device=DEV)
    H.hull_fbp(H.Histories.from_numpy(h, DEV), grid, H.make_fbp_params(geo), img, mask)
    torch.cuda.synchronize()
    ref, rmask, _, _ = oracle.fbp(h, oracle.grid_of(grid), oracle.fbp_params(geo))
    return img.cpu().numpy().astype(np.float64), mask.cpu().numpy(), ref, rmask


def _check(img, mask, ref, rmask, thr):
    scale = np.abs(ref).max()
    err = np.abs(img - ref).max() / scale
    assert err <= TOL, err
    near = np.abs(ref - thr) <= TOL * scale
    assert np.array_equal(mask[~near], rmask[~near])
    return err


def test_fbp_cone_beam_sphere():
    geo, h = _bin_centre_rays(150.0, 30.0, nu=160, nv=12, n_angles=360)
    grid = gen.Grid((64, 64, 4), (1.0, 1.0, 1.0))
    img, mask, ref, rmask = _run(h, grid, geo)
    _check(img, mask, ref, rmask, geo.threshold)


def test_fbp_config2_full():
    """The benchmark workload: 200x200x32, 1e7 noisy histories, 180 angles,
    1 mm x 5 mm detector bins, Shepp-Logan, threshold 0.6."""
    spec = gen.config_spec(2)
    h = gen.generate(spec)
    geo = spec.fbp_geometry(du=1.0, dv=5.0)
    img, mask, ref, rmask = _run(h, spec.grid, geo)
    err = _check(img, mask, ref, rmask, geo.threshold)
    print("config2 FBP max rel err", err, flush=True)
    # the hull keeps the head
    cen = gen.voxel_centres(spec.grid).reshape(-1, 3)
    inside = gen.phantom_rsp(spec.phantom[:1], cen * 1.1) > 0
    assert mask[inside].mean() > 0.99


def test_fbp_edge_histories():
    spec = gen.config_spec(1, n_hist=5000)
    h = gen.generate(spec)
    h = {k: v.copy() for k, v in h.items()}
    h["wepl"][0] = np.float32("nan")
    h["wepl"][1] = 70000.0          # beyond 2^16 mm: not binned
    h["x_out"][2] = h["x_in"][2]    # parallel to the detector plane
    h["y_in"][3] = 1e9              # off the detector
    h["angle_deg"][4] = 3e9         # cannot be binned
    geo = spec.fbp_geometry(du=1.0, dv=2.5)
    img, mask, ref, rmask = _run(h, spec.grid, geo)
    _check(img, mask, ref, rmask, geo.threshold)


@pytest.mark.parametrize("order", ["shuffled", "angle pairs"])
def test_fbp_histories_out_of_angle_order(order):
    """The LDS plane follows the gantry angle of the histories it bins and
    sends every other angle to the global sums: histories in random order
    (almost all global, the plane switching every round) and histories whose
    angle alternates between two values give the oracle's image too."""
    spec = gen.config_spec(2, n_hist=1_000_000)
    h = gen.generate(spec)
    rng = np.random.default_rng(5)
    if order == "shuffled":
        perm = rng.permutation(spec.n_hist)
    else:
        half = spec.n_hist // 2
        perm = np.empty(spec.n_hist, np.int64)
        perm[0::2] = np.arange(half)
        perm[1::2] = np.arange(half, spec.n_hist)
    h = {k: v[perm] for k, v in h.items()}
    geo = spec.fbp_geometry(du=1.0, dv=5.0)
    img, mask, ref, rmask = _run(h, spec.grid, geo)
    _check(img, mask, ref, rmask, geo.threshold)


@pytest.mark.parametrize("du,dv,path", [
    (0.05, 0.5, "detector plane beyond the LDS: global binning; footprints beyond the stage"),
    (0.25, 1.0, "one LDS plane per block"),
    (0.5, 2.5, "an LDS plane per block, two blocks per CU"),
])
def test_fbp_fine_detectors_take_the_fallback_paths(du, dv, path):
    """Fine detector sampling pushes the binning and the backprojection onto
    their fallbacks (global sums, unstaged samples); they must give the same
    image as the staged paths do, i.e. the oracle's within tolerance."""
    g = gen.Grid((32, 32, 16), (1.0, 1.0, 2.5))
    spec = gen.ScanSpec(g, 200_000, 36, gen.head_phantom(g), 0x5EED0110, sigma=1.0)
    h = gen.generate(spec)
    geo = spec.fbp_geometry(du=du, dv=dv)
    plane_bytes = geo.nu * geo.nv * 12
    if path.startswith("detector plane beyond"):
        assert plane_bytes > 160 * 1024
    elif path.startswith("one LDS plane"):
        assert 80 * 1024 < plane_bytes <= 160 * 1024
    else:
        assert plane_bytes <= 80 * 1024
    img, mask, ref, rmask = _run(h, g, geo)
    _check(img, mask, ref, rmask, geo.threshold)


# ---------------------------------------------------------------------------
# FDK hull after the data cuts

def _run_cut(h, grid, geo, k):
    V = grid.voxels
    img = torch.zeros(V, dtype=torch.float32, device=DEV)
    mask = torch.zeros(V, dtype=torch.uint8, device=DEV)
    H.hull_fbp_cut(H.Histories.from_numpy(h, DEV), grid, H.make_fbp_params(geo), k, img, mask)
    torch.cuda.synchronize()
    ref, rmask, _, _ = oracle.fbp_cut(h, oracle.grid_of(grid), oracle.fbp_params(geo), k)
    return img.cpu().numpy().astype(np.float64), mask.cpu().numpy(), ref, rmask


def _with_outliers(h, frac, seed):
    h = {k: v.copy() for k, v in h.items()}
    rng = np.random.default_rng(seed)
    bad = rng.random(h["wepl"].size) < frac
    h["wepl"][bad] = rng.uniform(0.0, 300.0, int(bad.sum())).astype(np.float32)
    return h


@pytest.mark.parametrize("k", [3, 0, 1])
def test_fbp_cut_config2_with_outliers(k):
    """The benchmark scan with 2% uniform outliers: FP32 image within 1e-4 of
    the FP64 oracle's after the same exact cuts."""
    spec = gen.config_spec(2)
    h = _with_outliers(gen.generate(spec), 0.02, 0x5EED00C7)
    geo = spec.fbp_geometry(du=1.0, dv=5.0)
    img, mask, ref, rmask = _run_cut(h, spec.grid, geo, k)
    err = _check(img, mask, ref, rmask, geo.threshold)
    print("config2 FDK after cuts, k", k, "max rel err", err, flush=True)


def test_fbp_cut_sphere_outliers_and_fallbacks():
    """One far outlier in a third of the bins of a sphere scan (the cut removes
    exactly those), and fine bins whose planes do not fit the LDS."""
    geo, h = _bin_centre_rays(150.0, 30.0, nu=160, nv=12, n_angles=360)
    reps = {k: np.repeat(v, 12) for k, v in h.items()}
    rng = np.random.default_rng(9)
    w = reps["wepl"].reshape(-1, 12).copy()
    w[rng.random(w.shape[0]) < 1 / 3, 11] += np.float32(150.0)
    reps["wepl"] = w.reshape(-1)
    grid = gen.Grid((64, 64, 4), (1.0, 1.0, 1.0))
    img, mask, ref, rmask = _run_cut(reps, grid, geo, 3)
    _check(img, mask, ref, rmask, geo.threshold)
    g = gen.Grid((32, 32, 16), (1.0, 1.0, 2.5))
    spec = gen.ScanSpec(g, 200_000, 36, gen.head_phantom(g), 0x5EED0111, sigma=1.0)
    hh = _with_outliers(gen.generate(spec), 0.05, 3)
    for du, dv in ((0.2, 0.8), (0.1, 0.5)):
        img, mask, ref, rmask = _run_cut(hh, g, spec.fbp_geometry(du=du, dv=dv), 3)
        _check(img, mask, ref, rmask, 0.6)
