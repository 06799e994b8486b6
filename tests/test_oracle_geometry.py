"""Pins for the oracle's geometry step: lab -> object frame (the object turns by
theta in front of a fixed horizontal beam, Section 2.2), voxel units and
rounding to 1/1024 voxel, plus its skip rules."""
import math

import numpy as np
import pytest

import oracle

Q = 1024


def _hist(xi, yi, zi, xo, yo, zo, ang, w=0.5):
    f = lambda v: np.array(v if isinstance(v, (list, tuple, np.ndarray)) else [v], dtype=np.float32)
    n = len(f(xi))
    w = np.broadcast_to(f(w), (n,)) if len(f(w)) == 1 else w
    return dict(x_in=f(xi), y_in=f(yi), z_in=f(zi), x_out=f(xo), y_out=f(yo), z_out=f(zo),
                angle_deg=f(ang), wepl=f(w))


G = oracle.make_grid((64, 64, 16), (1.0, 1.0, 2.5), (-32.0, -32.0, -20.0))


def test_zero_angle_is_identity():
    # (x - x0) / dx on exactly representable points, times 1024
    st, qi, qo = oracle.quantize(_hist(-100.0, 3.25, -1.25, 100.0, -7.5, 2.5, 0.0), G)
    assert st[0] == oracle.OK
    assert list(qi[0]) == [(-100 + 32) * Q, int((3.25 + 32) * Q), int((-1.25 + 20) / 2.5 * Q)]
    assert list(qo[0]) == [(100 + 32) * Q, int((-7.5 + 32) * Q), int((2.5 + 20) / 2.5 * Q)]


@pytest.mark.parametrize("ang,expect", [(90.0, lambda x, y: (y, -x)),
                                        (180.0, lambda x, y: (-x, -y)),
                                        (270.0, lambda x, y: (-y, x)),
                                        (-90.0, lambda x, y: (-y, x)),
                                        (450.0, lambda x, y: (y, -x)),
                                        (360.0, lambda x, y: (x, y))])
def test_quarter_turns(ang, expect):
    """Object = R(-theta) lab: a point at lab (x, y) sits at object (y, -x) after
    a 90 degree turn. Exact, since the FP32 cosine of a quarter turn is far below
    half an ulp of the coordinates used."""
    x, y = 12.5, -3.75
    st, qi, _ = oracle.quantize(_hist(x, y, 0.0, x + 1, y, 0.0, ang), G)
    ex, ey = expect(x, y)
    assert st[0] == oracle.OK
    assert qi[0][0] == int(round((ex + 32) * Q)) and qi[0][1] == int(round((ey + 32) * Q))


def test_rotation_preserves_radius_and_angle():
    rng = np.random.default_rng(0)
    n = 2000
    ang = rng.uniform(-720, 720, n).astype(np.float32)
    x = rng.uniform(-90, 90, n).astype(np.float32)
    y = rng.uniform(-90, 90, n).astype(np.float32)
    big = oracle.make_grid((1, 1, 1), (1.0, 1.0, 1.0), (0.0, 0.0, -0.5))
    st, qi, _ = oracle.quantize(_hist(x, y, np.zeros(n), x + 1, y, np.zeros(n), ang), big)
    assert (st == 0).all()
    xo, yo = qi[:, 0] / Q, qi[:, 1] / Q
    # radius preserved (FP32 rounding + 1/1024 rounding)
    assert np.allclose(np.hypot(xo, yo), np.hypot(x, y), atol=2e-3)
    # the object-frame polar angle is the lab angle minus theta
    d = np.angle(np.exp(1j * (np.arctan2(yo, xo) - (np.arctan2(y, x) - np.deg2rad(ang)))))
    r = np.hypot(x, y)
    assert np.all(np.abs(d)[r > 5] < 1e-3)


def test_trig_special_values():
    c, s = oracle.trig_table(np.array([0, 90, 180, 270, 360, -180, 30, 60, 45], dtype=np.float32))
    assert c[0] == 1.0 and s[0] == 0.0
    assert s[1] == 1.0 and abs(c[1]) < 1e-16
    assert c[2] == -1.0 and abs(s[2]) < 1e-15
    assert s[3] == -1.0
    assert c[4] == 1.0 and s[4] == 0.0
    assert c[5] == -1.0
    assert s[6] == np.float32(0.5) and c[7] == np.float32(0.5)
    assert c[8] == s[8] == np.float32(math.sqrt(0.5))


def test_round_half_to_even_on_the_1024_grid():
    # grid origin 0 and 1 mm voxels: q = rint(x * 1024)
    g = oracle.make_grid((8, 8, 8), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    xs = np.array([0.5 / Q, 1.5 / Q, 2.5 / Q, 3.0 / Q + 0.49 / Q], dtype=np.float32)
    st, qi, _ = oracle.quantize(_hist(xs, np.ones(4), np.ones(4), xs + 1, np.ones(4),
                                      np.ones(4), np.zeros(4)), g)
    assert list(qi[:, 0]) == [0, 2, 2, 3]


def test_skip_reasons():
    nan = float("nan")
    h = _hist([1.0, nan, 1e9, 1.0, 0.0], [0.0, 0.0, 0.0, 0.0, 0.0], [0.0] * 5,
              [2.0, 2.0, 2.0, 1.0 + 1e-9, 0.0], [0.0] * 5, [0.0] * 5, [0.0] * 5,
              [0.5, 0.5, 0.5, 0.5, float("inf")])
    st, _, _ = oracle.quantize(h, G)
    assert list(st) == [oracle.OK, oracle.SKIP_NONFINITE, oracle.SKIP_RANGE,
                        oracle.SKIP_DEGENERATE, oracle.SKIP_NONFINITE]


def test_range_limit_is_2_pow_16_voxels():
    g = oracle.make_grid((8, 8, 8), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    st, _, _ = oracle.quantize(_hist([65535.5, 65536.0], [0, 0], [0, 0], [0, 0], [0, 0],
                                     [0, 0], [0, 0]), g)
    assert list(st) == [oracle.OK, oracle.SKIP_RANGE]
