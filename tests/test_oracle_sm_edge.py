"""Pins of the oracle's edge-based SM threshold (Section 3.4: per slice, the
largest M on the edge of largest gradient sets M_t; M >= M_t is kept). The
rule is this project's statement of a Canny-like detector (the paper's
modification is not given): Sobel gradient with L1 magnitude, four-direction
thinning, an 8-connected hysteresis component grown from the strongest pixel.
Pinned against a reference built from library routines (scipy's Sobel filter
and connected-component labelling, a vectorised thinning), invariances, and
shapes whose hull is known."""
import numpy as np
import pytest
from scipy import ndimage

import oracle


def _grid(nx, ny, nz):
    return oracle.make_grid((nx, ny, nz), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))


def edge_ref(m, num, den):
    """m: [ny, nx] int. The same definition through library routines."""
    m = m.astype(np.int64)
    ny, nx = m.shape
    gx = ndimage.sobel(m, axis=1, mode="constant")   # d/di, smoothed along j
    gy = ndimage.sobel(m, axis=0, mode="constant")
    G = np.abs(gx) + np.abs(gy)
    interior = np.zeros_like(G, bool)
    interior[1:-1, 1:-1] = True
    G = np.where(interior, G, 0)
    ax, ay = np.abs(gx), np.abs(gy)
    d = np.where(5 * ay <= 2 * ax, 0, np.where(5 * ax <= 2 * ay, 1, np.where((gx > 0) == (gy > 0), 2, 3)))
    pad = np.pad(G, 1)
    steps = {0: (0, 1), 1: (1, 0), 2: (1, 1), 3: (-1, 1)}   # (dj, di) for d = (di, dj)
    edge = np.zeros_like(G, bool)
    for k, (dj, di) in steps.items():
        before = pad[1 - dj:1 - dj + ny, 1 - di:1 - di + nx]
        after = pad[1 + dj:1 + dj + ny, 1 + di:1 + di + nx]
        edge |= (d == k) & (G > 0) & (G > before) & (G >= after)
    if not edge.any():
        return np.zeros_like(m, np.uint8), -1
    flat = np.where(edge.reshape(-1), G.reshape(-1), -1)
    seed = len(flat) - 1 - int(np.argmax(flat[::-1]))      # largest G, ties: largest index
    ok = edge & (den * G >= num * flat[seed])
    lab, _ = ndimage.label(ok, structure=np.ones((3, 3), int))
    comp = lab == lab.reshape(-1)[seed]
    mt = int(m[comp].max())
    return (m >= mt).astype(np.uint8), mt


def smooth_field(rng, ny, nx):
    base = rng.normal(size=(ny, nx))
    f = ndimage.gaussian_filter(base, 2.5)
    yy, xx = np.mgrid[0:ny, 0:nx]
    blob = 1.0 / (1.0 + np.exp((np.hypot(xx - nx * 0.45, yy - ny * 0.55) - 0.3 * min(nx, ny)) / 1.5))
    return np.rint(4000 * blob + 300 * f / f.std() + 500).clip(0).astype(np.int32)


@pytest.mark.parametrize("num,den", [(1, 2), (1, 4), (3, 4), (0, 1)])
def test_matches_the_library_reference(num, den):
    rng = np.random.default_rng(num * 10 + den)
    ny, nx, nz = 37, 53, 5
    M = np.stack([smooth_field(rng, ny, nx) for _ in range(nz)])
    M[2] = rng.integers(0, 3, (ny, nx))          # a noisy low slice
    M[3] = 17                                     # a flat slice: no edge
    mask, mt = oracle.sm(M.reshape(-1), _grid(nx, ny, nz), num, den, oracle.SM_EDGE,
                         oracle.SCOPE_SLICE)
    mask = mask.reshape(nz, ny, nx)
    for k in range(nz):
        rmask, rmt = edge_ref(M[k], num, den)
        assert mt[k] == rmt, k
        assert np.array_equal(mask[k], rmask), k
    assert mt[3] == -1 and not mask[3].any()


def test_invariances():
    rng = np.random.default_rng(5)
    ny, nx = 41, 41
    m = np.stack([smooth_field(rng, ny, nx) for _ in range(3)])
    g = _grid(nx, ny, 3)
    run = lambda a: oracle.sm(np.ascontiguousarray(a).reshape(-1), _grid(a.shape[2], a.shape[1], a.shape[0]),
                              1, 2, oracle.SM_EDGE, oracle.SCOPE_SLICE)
    mask, mt = run(m)
    mask = mask.reshape(m.shape)
    # gradients scale with M and ignore an added constant: the same hull
    m2, mt2 = run(3 * m + 1000)
    assert np.array_equal(m2.reshape(m.shape), mask) and np.array_equal(mt2, 3 * mt + 1000)
    # swapping x and y swaps the directions, thinning and neighbourhoods alike
    mt_t = run(np.transpose(m, (0, 2, 1)))
    assert np.array_equal(mt_t[0].reshape(m.shape[0], nx, ny), np.transpose(mask, (0, 2, 1)))
    assert np.array_equal(mt_t[1], mt)


def test_soft_disk_hull_lies_inside_the_steepest_ring():
    """M falls off a disk of radius R = 20 over a few voxels (a logistic of
    width 1.5): the strongest edge is the ring of steepest descent at r ~ R,
    so the hull is a centred disk a little smaller than R."""
    ny = nx = 64
    yy, xx = np.mgrid[0:ny, 0:nx]
    r = np.hypot(xx - 31.5, yy - 31.5)
    m = np.rint(5000.0 / (1.0 + np.exp((r - 20.0) / 1.5))).astype(np.int32)
    mask, mt = oracle.sm(m.reshape(-1), _grid(nx, ny, 1), 1, 2, oracle.SM_EDGE, oracle.SCOPE_SLICE)
    mask = mask.reshape(ny, nx).astype(bool)
    assert mask[r <= 15.0].all() and not mask[r >= 20.0].any()
    assert 1000 < mt[0] < 5000


def test_rejects_volume_scope():
    m = np.zeros(27, np.int32)
    with pytest.raises(ValueError):
        oracle.sm(m, _grid(3, 3, 3), 1, 2, oracle.SM_EDGE, oracle.SCOPE_VOLUME)


def test_sector_boundary_ties_go_to_the_axis():
    """A ramp M = 5i + 2j + 10 has gx = 40, gy = 16 everywhere inside, exactly on
    the 2/5 sector boundary: the thinning runs along x (edge = the column next
    to the border, whose top pixel holds the largest M), not diagonally."""
    ny, nx = 12, 15
    jj, ii = np.mgrid[0:ny, 0:nx]
    m = (5 * ii + 2 * jj + 10).astype(np.int32)
    mask, mt = oracle.sm(m.reshape(-1), _grid(nx, ny, 1), 1, 2, oracle.SM_EDGE, oracle.SCOPE_SLICE)
    assert mt[0] == 5 * 1 + 2 * (ny - 2) + 10
    rmask, rmt = edge_ref(m, 1, 2)
    assert rmt == mt[0] and np.array_equal(mask.reshape(ny, nx), rmask)
