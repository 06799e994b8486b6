"""Pins for the hull rules on hand-built count volumes (results derived by hand
from the set definitions and Algorithms 2-3, Sections 3.3-3.4)."""
import numpy as np
import pytest

import oracle


def G(nx, ny, nz):
    return oracle.make_grid((nx, ny, nz), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))


def test_sc_is_the_uncarved_set():
    N = np.array([0, 3, 0, 1, 0, 0], dtype=np.int32)
    assert list(oracle.sc(N)) == [1, 0, 1, 0, 1, 1]


def test_msc_neighbour_difference_spike():
    # a 3x3 slice with one voxel 60 above its neighbours, N_t = 50: only the
    # spike has N(v) - N(w) >= 50 for some neighbour w.
    N = np.zeros(9, dtype=np.int32)
    N[4] = 60
    m = oracle.msc(N, G(3, 3, 1), 50, oracle.MSC_NEIGHBOR_DIFF)
    assert list(m) == [1, 1, 1, 1, 0, 1, 1, 1, 1]


def test_msc_neighbour_difference_row():
    # 100 | 40 | 0: 100-40 = 60 >= 50 removes the first voxel; 40-0 = 40 keeps
    # the second; the third has no smaller neighbour.
    m = oracle.msc(np.array([100, 40, 0], dtype=np.int32), G(3, 1, 1), 50,
                   oracle.MSC_NEIGHBOR_DIFF)
    assert list(m) == [0, 1, 1]


def test_msc_neighbourhoods_in_plane_vs_spatial():
    g = G(1, 1, 2)                               # two voxels stacked in z
    for N, six in (([70, 0], [0, 1]), ([0, 70], [1, 0])):
        N = np.array(N, dtype=np.int32)
        assert list(oracle.msc(N, g, 50, oracle.MSC_NEIGHBOR_DIFF, oracle.NBR_INPLANE4)) == [1, 1]
        assert list(oracle.msc(N, g, 50, oracle.MSC_NEIGHBOR_DIFF, oracle.NBR_SPATIAL6)) == six


def test_msc_spatial_neighbours_on_a_cube():
    # 2x2x2: slice 1 all 70, slice 0 all 0. In-plane nothing differs; in 3-D every
    # voxel of slice 1 sits 70 above the voxel below it.
    N = np.array([0, 0, 0, 0, 70, 70, 70, 70], dtype=np.int32)
    g = G(2, 2, 2)
    assert oracle.msc(N, g, 50, oracle.MSC_NEIGHBOR_DIFF, oracle.NBR_INPLANE4).all()
    m = oracle.msc(N, g, 50, oracle.MSC_NEIGHBOR_DIFF, oracle.NBR_SPATIAL6)
    assert list(m) == [1, 1, 1, 1, 0, 0, 0, 0]
    m = oracle.msc(N[::-1].copy(), g, 50, oracle.MSC_NEIGHBOR_DIFF, oracle.NBR_SPATIAL6)
    assert list(m) == [0, 0, 0, 0, 1, 1, 1, 1]


def test_msc_neighbour_difference_threshold_is_inclusive():
    # Algorithm 2 removes v when N(v) - N(w) >= N_t: a difference of exactly 50 removes
    m = oracle.msc(np.array([50, 0, 49, 0], dtype=np.int32), G(2, 2, 1), 50,
                   oracle.MSC_NEIGHBOR_DIFF)
    assert list(m) == [0, 1, 1, 1]


def test_msc_neighbour_difference_constant_volume_keeps_all():
    N = np.full(4 * 3 * 2, 1234, dtype=np.int32)
    assert oracle.msc(N, G(4, 3, 2), 1, oracle.MSC_NEIGHBOR_DIFF).all()


def test_msc_count_threshold():
    N = np.array([0, 4, 5, 6, 100], dtype=np.int32)
    assert list(oracle.msc(N, G(5, 1, 1), 5, oracle.MSC_COUNT)) == [1, 1, 0, 0, 0]


@pytest.mark.parametrize("M,expect,mt", [
    # slopes 1,1,18,1,0: steepest drop after the third voxel, M_t = 28
    ([30, 29, 28, 10, 9], [1, 1, 0, 0, 0], 28),
    # slopes 10 at voxels 0 and 2: ties go to the later voxel, M_t = 10
    ([12, 2, 10, 0], [1, 0, 0, 0], 10),
    # the steepest voxel is the maximum itself: H3 is empty
    ([5, 9, 2, 2], [0, 0, 0, 0], 9),
    # constant: every slope is 0, the last voxel wins, M_t = 7
    ([7, 7, 7], [0, 0, 0], 7),
])
def test_sm_max_slope(M, expect, mt):
    mask, thr = oracle.sm(np.array(M, dtype=np.int32), G(len(M), 1, 1), mode=oracle.SM_MAX_SLOPE)
    assert list(mask) == expect and thr[0] == mt


def test_sm_fraction_is_strict_and_exact():
    # keep 5 M > 3 max M; max = 10 so keep M > 6
    mask, thr = oracle.sm(np.array([0, 5, 10, 6, 7], dtype=np.int32), G(5, 1, 1), 3, 5)
    assert list(mask) == [0, 0, 1, 0, 1] and thr[0] == 10


def test_sm_slice_scope():
    M = np.array([0, 10, 4, 2, 100, 60], dtype=np.int32)   # 3 voxels x 2 slices
    mask, thr = oracle.sm(M, G(3, 1, 2), 1, 2, scope=oracle.SCOPE_SLICE)
    # slice 0: max 10 -> keep 2M > 10; slice 1: max 100 -> keep 2M > 100
    assert list(mask) == [0, 1, 0, 0, 1, 1] and list(thr) == [10, 100]
    mask, thr = oracle.sm(M, G(3, 1, 2), 1, 2, scope=oracle.SCOPE_VOLUME)
    assert list(mask) == [0, 0, 0, 0, 1, 1] and list(thr) == [100]


def test_sm_max_slope_slice_scope_and_spatial_neighbours():
    # two 2-voxel slices; in 3-D the big drop is between slices
    M = np.array([5, 4, 50, 49], dtype=np.int32)
    g = G(2, 1, 2)
    mask, thr = oracle.sm(M, g, mode=oracle.SM_MAX_SLOPE, nbr=oracle.NBR_SPATIAL6)
    # slopes: v0: 1; v1: 0; v2: 50-5=45, 1 -> 45; v3: 49-4=45 -> tie, later voxel v3, M_t = 49
    assert list(mask) == [0, 0, 1, 0] and thr[0] == 49
    mask, thr = oracle.sm(M, g, mode=oracle.SM_MAX_SLOPE, scope=oracle.SCOPE_SLICE)
    # per slice, in-plane: slice 0 slopes (1, 0) -> M_t = 5; slice 1 slopes (1, 0) -> M_t = 50
    assert list(mask) == [0, 0, 0, 0] and list(thr) == [5, 50]
