"""The oracle's whole-call mirrors (same argument layouts as the GPU
library's per-scan calls, host pointers) are the compositions of the pinned
oracle steps: classify + walk + count, then the rule of each call."""
import numpy as np
import pytest

import gen
import oracle


@pytest.fixture(scope="module")
def scan():
    spec = gen.config_spec(1, n_hist=6000)
    return spec, gen.generate(spec), oracle.grid_of(spec.grid)


def test_sc_msc_sm_mirrors(scan):
    spec, h, G = scan
    N, M, st = oracle.counts(h, G, 1.0, 5.0)
    Nl, _, stl = oracle.counts(h, G, 1.0, 5.0, want_m=False)
    _, Mh, sth = oracle.counts(h, G, 1.0, 5.0, want_n=False)
    n1, m1, s1 = oracle.hull_sc(h, G, 1.0)
    assert np.array_equal(n1, Nl) and np.array_equal(m1, oracle.sc(Nl)) and s1 == stl
    n2, m2, s2 = oracle.hull_msc(h, G, 1.0, 50, oracle.MSC_NEIGHBOR_DIFF, oracle.NBR_SPATIAL6)
    assert np.array_equal(n2, Nl) and s2 == stl
    assert np.array_equal(m2, oracle.msc(Nl, G, 50, oracle.MSC_NEIGHBOR_DIFF, oracle.NBR_SPATIAL6))
    n3, m3, s3 = oracle.hull_sm(h, G, 5.0, 3, 5, oracle.SM_MAX_SLOPE, oracle.SCOPE_SLICE,
                                oracle.NBR_INPLANE4)
    assert np.array_equal(n3, Mh) and s3 == sth
    assert np.array_equal(m3, oracle.sm(Mh, G, 3, 5, oracle.SM_MAX_SLOPE, oracle.SCOPE_SLICE)[0])
    # the one-pass mirror: both counts at once, stats of both classes
    p = oracle.OrParams(1.0, 5.0, 5, oracle.MSC_COUNT, 3, 5, oracle.SM_FRACTION,
                        oracle.SCOPE_VOLUME, oracle.NBR_INPLANE4)
    a = oracle.hull_all(h, G, p)
    assert np.array_equal(a[0], N) and np.array_equal(a[1], M) and a[5] == st
    assert np.array_equal(a[2], oracle.sc(N))
    assert np.array_equal(a[3], oracle.msc(N, G, 5))
    assert np.array_equal(a[4], oracle.sm(M, G, 3, 5)[0])
    # invalid modes are refused
    with pytest.raises(ValueError):
        oracle.hull_msc(h, G, 1.0, 5, 7, 0)
    with pytest.raises(ValueError):
        oracle.hull_all(h, G, oracle.OrParams(1.0, 5.0, 5, 0, 3, 5, 0, 9, 0))


def test_fbp_mirror(scan):
    spec, h, G = scan
    p = oracle.fbp_params(spec.fbp_geometry())
    img, mask = oracle.hull_fbp(h, G, p)
    img2, mask2, _, _ = oracle.fbp(h, G, p)
    assert np.array_equal(img, img2) and np.array_equal(mask, mask2)
