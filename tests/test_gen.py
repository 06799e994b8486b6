"""Pins for the synthetic scan generator (inputs only): closed-form chords,
quadrature of nested ellipsoids, beam geometry and determinism."""
import math

import numpy as np
import pytest

import gen


def test_sphere_chord_closed_form():
    rng = np.random.default_rng(0)
    R, rho = 37.0, 1.3
    ell = gen.sphere_phantom(R, rho)[0]
    for _ in range(200):
        p = rng.uniform(-60, 60, 3)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        # distance from the centre to the line
        d = np.linalg.norm(p - np.dot(p, u) * u)
        want = 2 * math.sqrt(R * R - d * d) if d < R else 0.0
        assert abs(gen.chord(ell, p, u) - want) < 1e-9 * max(1.0, want)


def test_scan_wepl_of_a_centred_sphere():
    """A sphere at the isocentre is rotation invariant: WEPL = rho * 2 sqrt(R^2 - d^2)
    with d the distance from the lab-frame line to the origin."""
    g = gen.Grid((64, 64, 16), (1.0, 1.0, 2.5))
    R, rho = 18.0, 1.04
    spec = gen.ScanSpec(g, 5000, 90, gen.sphere_phantom(R, rho), seed=99)
    h = gen.generate(spec, with_true=True)
    pin = np.stack([h["x_in"], h["y_in"], h["z_in"]], 1).astype(np.float64)
    pout = np.stack([h["x_out"], h["y_out"], h["z_out"]], 1).astype(np.float64)
    u = pout - pin
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    d = np.linalg.norm(pin - (pin * u).sum(1, keepdims=True) * u, axis=1)
    want = rho * 2 * np.sqrt(np.clip(R * R - d * d, 0, None))
    assert np.allclose(h["wepl_true"], want, atol=1e-9)
    assert np.array_equal(h["wepl"], want.astype(np.float32)) or np.allclose(h["wepl"], want, atol=1e-5)


@pytest.mark.parametrize("kind", ["inserts", "ventricles"])
def test_nested_ellipsoids_match_quadrature(kind):
    g = gen.Grid((200, 200, 32), (1.0, 1.0, 3.0))
    ph = gen.head_phantom(g, inserts=kind == "inserts", ventricles=kind == "ventricles")
    spec = gen.ScanSpec(g, 400, 180, ph, seed=5)
    h = gen.generate(spec, with_true=True)
    for i in range(0, 400, 7):
        th = np.deg2rad(float(h["angle_deg"][i]))
        c, s = math.cos(th), math.sin(th)
        a = np.array([h["x_in"][i], h["y_in"][i], h["z_in"][i]], dtype=np.float64)
        b = np.array([h["x_out"][i], h["y_out"][i], h["z_out"][i]], dtype=np.float64)
        rot = lambda p: np.array([c * p[0] + s * p[1], -s * p[0] + c * p[1], p[2]])
        a, b = rot(a), rot(b)
        # the phantom lies well inside the trackers, so the segment carries all of it
        t = (np.arange(200000) + 0.5) / 200000
        pts = a[None, :] + t[:, None] * (b - a)[None, :]
        q = gen.phantom_rsp(ph, pts).sum() * np.linalg.norm(b - a) / len(t)
        assert abs(q - h["wepl_true"][i]) < 2e-2, (i, q, h["wepl_true"][i])


def test_beam_geometry_and_ordering():
    spec = gen.config_spec(1)
    h = gen.generate(spec)
    assert (h["x_in"] == -100.0).all() and (h["x_out"] == 100.0).all()
    # every ray points back at the source (-2000, 0, 0)
    S = np.array([-2000.0, 0.0, 0.0])
    a = np.stack([h["x_in"], h["y_in"], h["z_in"]], 1).astype(np.float64) - S
    b = np.stack([h["x_out"], h["y_out"], h["z_out"]], 1).astype(np.float64) - S
    cross = np.cross(a, b)
    assert np.abs(cross).max() / (np.linalg.norm(a, axis=1) * np.linalg.norm(b, axis=1)).min() < 1e-6
    ang = h["angle_deg"]
    assert (np.diff(ang) >= 0).all()
    vals = np.unique(ang)
    assert len(vals) == 90 and np.allclose(np.diff(vals), 4.0)
    assert abs(np.bincount(np.searchsorted(vals, ang)).std()) < 1.0


def test_ranges_are_slices_of_the_whole_scan():
    spec = gen.config_spec(2, n_hist=50_000)
    full = gen.generate(spec)
    part = gen.generate(spec, 12_345, 20_000)
    for k in gen.FIELDS:
        assert np.array_equal(full[k][12_345:20_000], part[k])
    again = gen.generate(spec)
    assert all(np.array_equal(full[k], again[k]) for k in gen.FIELDS)


def test_noise_and_outliers_statistics():
    from dataclasses import replace
    spec = gen.config_spec(3, n_hist=400_000)
    noisy = gen.generate(replace(spec, outlier_frac=0.0), with_true=True)
    r = noisy["wepl"].astype(np.float64) - noisy["wepl_true"]
    assert abs(r.std() - 3.0) < 0.02 and abs(r.mean()) < 0.02
    out = gen.generate(replace(spec, sigma=0.0), with_true=True)
    moved = np.abs(out["wepl"].astype(np.float64) - out["wepl_true"]) > 1e-3
    assert abs(moved.mean() - 0.02) < 0.002
    assert out["wepl"][moved].min() >= 0.0 and out["wepl"][moved].max() < 300.0


def test_phantom_slice_area_near_paper():
    """Skull cross-section at a 200 mm field: pi * 62 * 78 = 15,193 mm^2, within 1%
    of the paper's 15,336-voxel phantom slice (Section 4.1)."""
    g = gen.Grid((200, 200, 32), (1.0, 1.0, 3.0))
    skull = gen.head_phantom(g)[0]
    area = math.pi * skull.semi[0] * skull.semi[1]
    assert abs(area - 15336) / 15336 < 0.01


def test_ventricle_phantom_chords_in_closed_form():
    """Lines parallel to x through the centre height of the ventricles: the
    WEPL is a sum of axis-aligned chords, 2 a sqrt(1 - (y/b)^2 - (z/c)^2) per
    ellipsoid weighted by its RSP step (skull 1.6, brain 1.04 - 1.6, each
    ventricle 0.9 - 1.04). Checked against the generator's own chords and
    against the RSP the phantom assigns to points: the ventricles' centres
    hold 0.9, the brain between them 1.04, the skull 1.6."""
    g = gen.Grid((200, 200, 32), (1.0, 1.0, 3.0))
    ph = gen.head_phantom(g, ventricles=True)
    assert len(ph) == 4
    skull, brain, v1, v2 = ph
    assert abs(v1.drho - (0.9 - 1.04)) < 1e-12 and v1.centre[0] == -v2.centre[0] > 0
    y, z = v1.centre[1], v1.centre[2]

    def closed(e):
        r = 1 - ((y - e.centre[1]) / e.semi[1]) ** 2 - ((z - e.centre[2]) / e.semi[2]) ** 2
        return 2 * e.semi[0] * math.sqrt(r) if r > 0 else 0.0

    want = sum(e.drho * closed(e) for e in ph)
    got = sum(e.drho * gen.chord(e, (-150.0, y, z), (1.0, 0.0, 0.0)) for e in ph)
    assert abs(got - want) < 1e-9
    # both ventricles lie on this line, fully inside the brain
    assert closed(v1) > 0 and closed(v2) > 0
    assert closed(brain) > 2 * (abs(v1.centre[0]) + v1.semi[0])
    rsp = gen.phantom_rsp(ph, np.array([v1.centre, v2.centre, (0.0, y, z),
                                        (0.0, brain.semi[1] + 1.0, 0.0)]))
    assert np.allclose(rsp, [0.9, 0.9, 1.04, 1.6])
