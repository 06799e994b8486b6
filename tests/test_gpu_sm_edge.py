"""GPU parity of the SM threshold from the strongest edge of each slice (the
EDGE rule, Section 3.4's text): M, the per-slice thresholds' masks equal the
oracle's exactly, through hull_sm and hull_all, with edge lists in LDS and
(for slices with many edge pixels) in global memory."""
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


def run_sm(h, grid, num, den, wepl_high=5.0):
    V = grid.voxels
    M = torch.zeros(V, dtype=torch.int32, device=DEV)
    mask = torch.zeros(V, dtype=torch.uint8, device=DEV)
    H.hull_sm(H.Histories.from_numpy(h, DEV), grid, wepl_high, num, den, H.HULL_SM_EDGE,
              H.HULL_SCOPE_SLICE, H.HULL_NBR_INPLANE4, M, mask)
    torch.cuda.synchronize()
    return M.cpu().numpy(), mask.cpu().numpy()


def check(h, grid, num, den, what, wepl_high=5.0):
    say(what)
    gM, gmask = run_sm(h, grid, num, den, wepl_high)
    G = oracle.grid_of(grid)
    _, rM, _ = oracle.counts(h, G, 1.0, wepl_high, want_n=False)
    assert np.array_equal(gM, rM), what
    rmask, mt = oracle.sm(rM, G, num, den, oracle.SM_EDGE, oracle.SCOPE_SLICE)
    if not np.array_equal(gmask, rmask):
        bad = np.flatnonzero(gmask != rmask)
        plane = grid.n[0] * grid.n[1]
        raise AssertionError(f"{what}: {bad.size} voxels differ, slices {np.unique(bad // plane)[:8]}")
    return mt


@pytest.mark.parametrize("num,den", [(1, 2), (0, 1), (1, 1)])
def test_config2_scan(num, den):
    spec = gen.config_spec(2)
    h = gen.generate(spec)
    mt = check(h, spec.grid, num, den, f"config2 {num}/{den}")
    assert (mt > 0).sum() >= 20


def test_one_pass_call_and_small_scans():
    spec = gen.config_spec(1)
    h = gen.generate(spec)
    h = {k: v.copy() for k, v in h.items()}
    h["wepl"] += np.random.default_rng(8).normal(0, 3.0, h["wepl"].size).astype(np.float32)
    check(h, spec.grid, 1, 2, "config1 noisy")
    V = spec.grid.voxels
    N, M = (torch.zeros(V, dtype=torch.int32, device=DEV) for _ in range(2))
    sm = torch.zeros(V, dtype=torch.uint8, device=DEV)
    p = H.make_params(sm_mode=H.HULL_SM_EDGE, sm_scope=H.HULL_SCOPE_SLICE, sm_frac_num=1,
                      sm_frac_den=2)
    H.hull_all(H.Histories.from_numpy(h, DEV), spec.grid, p, N, M, sm_mask=sm)
    torch.cuda.synchronize()
    G = oracle.grid_of(spec.grid)
    _, rM, _ = oracle.counts(h, G, 1.0, 5.0, want_n=False)
    assert np.array_equal(sm.cpu().numpy(), oracle.sm(rM, G, 1, 2, oracle.SM_EDGE, oracle.SCOPE_SLICE)[0])


def test_many_edge_pixels_take_the_global_lists():
    """A wide, sparse scan (2048 x 48 slices, few histories per voxel) makes M
    noisy: with the hysteresis fraction at 0 every thinned pixel joins, more
    than an LDS list holds."""
    g = gen.Grid((2048, 48, 3), (0.1, 1.0, 2.0))
    spec = gen.ScanSpec(g, 400_000, 60, gen.head_phantom(g), 0x5EED0333, sigma=2.0,
                        fan=(1.05 * np.hypot(102.4, 24.0), 3.2))
    h = gen.generate(spec)
    check(h, g, 0, 1, "wide sparse 0/1")
    check(h, g, 1, 3, "wide sparse 1/3")


def test_bad_scope_is_rejected():
    spec = gen.config_spec(1, n_hist=1000)
    h = gen.generate(spec)
    V = spec.grid.voxels
    M = torch.zeros(V, dtype=torch.int32, device=DEV)
    mask = torch.zeros(V, dtype=torch.uint8, device=DEV)
    with pytest.raises(H.HullError):
        H.hull_sm(H.Histories.from_numpy(h, DEV), spec.grid, 5.0, 1, 2, H.HULL_SM_EDGE,
                  H.HULL_SCOPE_VOLUME, H.HULL_NBR_INPLANE4, M, mask)
