"""The measurement entry points: hull_count_profile runs the counting pass of
hull_all with an event pair around every launch, hull_fbp_profile does the
same for hull_fbp. Their results must be those of the plain calls (the counts
bit-exact against the oracle, the FDK image bit-identical to hull_fbp's) and
the reported launches must match the pass's structure."""
import numpy as np
import pytest
import torch

import gen
import oracle
from paper_1402_1720_amd import hullmi as H

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def test_count_profile_counts_and_launches():
    spec = gen.config_spec(2, n_hist=300_000)
    h = gen.generate(spec)
    hist = H.Histories.from_numpy(h, DEV)
    V = spec.grid.voxels
    N = torch.zeros(V, dtype=torch.int32, device=DEV)
    M = torch.zeros(V, dtype=torch.int32, device=DEV)
    st = torch.zeros(6, dtype=torch.int64, device=DEV)
    prof = H.hull_count_profile(hist, spec.grid, H.make_params(), N, M, stats=st)
    rN, rM, rst = oracle.counts(h, oracle.grid_of(spec.grid))
    assert np.array_equal(N.cpu().numpy(), rN) and np.array_equal(M.cpu().numpy(), rM)
    assert H.stats_dict(st) == rst
    assert set(prof) == set(H.PROF_KERNELS[:8])
    for k, (ms, n) in prof.items():
        assert n == 1, k                  # one internal batch: one launch of each
        assert ms > 0.0, k
    # adding a second pass doubles the counts
    prof2 = H.hull_count_profile(hist, spec.grid, H.make_params(), N, M, flags=H.HULL_ACCUMULATE)
    assert np.array_equal(N.cpu().numpy(), 2 * rN)
    assert prof2["walk"][1] == 1


def test_count_profile_over_internal_batches():
    """The smallest workspace (2^16 histories: too small to split in two)
    runs 300,000 histories in five internal batches on the caller's stream:
    five launches of every counting kernel, and hull_all's counts."""
    spec = gen.config_spec(1, n_hist=300_000)
    h = gen.generate(spec)
    hist = H.Histories.from_numpy(h, DEV)
    V = spec.grid.voxels
    N = torch.zeros(V, dtype=torch.int32, device=DEV)
    M = torch.zeros(V, dtype=torch.int32, device=DEV)
    ws = H.workspace(H.HULL_OP_ALL, spec.grid, 1 << 16, DEV)
    prof = H.hull_count_profile(hist, spec.grid, H.make_params(), N, M, ws=ws)
    assert all(n == 5 for _, n in prof.values())
    N2 = torch.zeros_like(N)
    M2 = torch.zeros_like(M)
    H.hull_all(hist, spec.grid, H.make_params(), N2, M2)
    torch.cuda.synchronize()
    assert torch.equal(N, N2) and torch.equal(M, M2)


def test_fbp_profile_equals_hull_fbp():
    spec = gen.config_spec(2, n_hist=500_000)
    h = gen.generate(spec)
    hist = H.Histories.from_numpy(h, DEV)
    V = spec.grid.voxels
    fbp = H.make_fbp_params(spec.fbp_geometry(du=1.0, dv=5.0))
    img = torch.zeros(V, dtype=torch.float32, device=DEV)
    mask = torch.zeros(V, dtype=torch.uint8, device=DEV)
    img2 = torch.zeros_like(img)
    mask2 = torch.zeros_like(mask)
    H.hull_fbp(hist, spec.grid, fbp, img, mask)
    prof = H.hull_fbp_profile(hist, spec.grid, fbp, img2, mask2)
    assert torch.equal(img, img2) and torch.equal(mask, mask2)
    assert set(prof) == set(H.PROF_KERNELS[8:])
    assert all(ms > 0.0 and n == 1 for ms, n in prof.values())


def test_profile_rejects_a_missing_output_array():
    spec = gen.config_spec(1, n_hist=1000)
    hist = H.Histories.from_numpy(gen.generate(spec), DEV)
    N = torch.zeros(spec.grid.voxels, dtype=torch.int32, device=DEV)
    with pytest.raises(H.HullError):
        H.hull_count_profile(hist, spec.grid, H.make_params(), N, None)
