"""Pins for the oracle's voxel set A_i (Sections 3.2-3.4) and its counts.

The oracle enumerates A_i from a candidate set and an exact integer test; here
it is checked against an independent brute force over every voxel with exact
fractions, against hand-derived cases, and against geometric invariants.
"""
import os

import numpy as np
import pytest

import oracle
from tests.walk_ref import (Q, brute_cells, load_golden, random_lines, tie_lines)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "walk_cases.txt")


def _grid(n):
    return oracle.make_grid(n, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))


@pytest.mark.parametrize("case", load_golden(GOLDEN), ids=lambda c: c[0])
def test_hand_derived_cases(case):
    name, n, qin, qout, cells = case
    g = _grid(n)
    assert list(oracle.line_cells(qin, qout, g)) == cells
    assert list(oracle.line_cells(qin, qout, g, all_voxels=True)) == cells
    assert brute_cells(qin, qout, n) == cells


@pytest.mark.parametrize("n", [(3, 2, 2), (5, 4, 3), (7, 6, 4), (16, 16, 8)])
def test_against_brute_force_tie_rich(n):
    rng = np.random.default_rng(1000 + n[0])
    g = _grid(n)
    count = 300 if n[0] < 16 else 60
    for qin, qout in tie_lines(rng, n, count):
        ref = brute_cells(qin, qout, n)
        got = list(oracle.line_cells(qin, qout, g))
        assert got == ref, (qin, qout)


@pytest.mark.parametrize("n", [(4, 3, 2), (9, 7, 5), (16, 12, 6)])
def test_against_brute_force_generic(n):
    rng = np.random.default_rng(2000 + n[0])
    g = _grid(n)
    for qin, qout in random_lines(rng, n, 150 if n[0] < 16 else 50):
        assert list(oracle.line_cells(qin, qout, g)) == brute_cells(qin, qout, n), (qin, qout)


def test_candidate_pruning_equals_full_scan():
    """The pruned enumeration returns exactly what testing every voxel returns."""
    n = (24, 20, 6)
    g = _grid(n)
    rng = np.random.default_rng(7)
    for qin, qout in tie_lines(rng, n, 150) + random_lines(rng, n, 150):
        assert np.array_equal(oracle.line_cells(qin, qout, g),
                              oracle.line_cells(qin, qout, g, all_voxels=True))


def _trace_order(qin, qout, cells, n):
    """Orders cells along the line by the parameter of a point inside each."""
    from fractions import Fraction
    P0 = np.array(qin, dtype=object)
    D = np.array(qout, dtype=object) - P0
    keyed = []
    for c in cells:
        v = (c % n[0], (c // n[0]) % n[1], c // (n[0] * n[1]))
        lo = None
        for a in range(3):
            if D[a] == 0:
                continue
            t0 = Fraction(int(Q * v[a] - P0[a]), int(D[a]))
            t1 = Fraction(int(Q * (v[a] + 1) - P0[a]), int(D[a]))
            m = min(t0, t1)
            lo = m if lo is None else max(lo, m)
        keyed.append((lo, v))
    keyed.sort(key=lambda kv: kv[0])
    return [v for _, v in keyed]


def test_invariants_connectivity_monotone_reversal():
    n = (12, 10, 5)
    g = _grid(n)
    rng = np.random.default_rng(11)
    for qin, qout in random_lines(rng, n, 200):
        a = oracle.line_cells(qin, qout, g)
        b = oracle.line_cells(qout, qin, g)
        assert np.array_equal(a, b)                      # direction does not matter
        if len(a) == 0:
            continue
        seq = _trace_order(qin, qout, a, n)
        D = [qo - qi for qi, qo in zip(qin, qout)]
        for p, q in zip(seq, seq[1:]):
            step = [q[k] - p[k] for k in range(3)]
            assert all(abs(s) <= 1 for s in step) and any(step)   # 26-connected, no repeats
            for k in range(3):                                     # monotone per axis
                assert step[k] == 0 or np.sign(step[k]) == np.sign(D[k])
        # generic lines (no exact tie): |A| = 1 + sum |index change|
        span = [abs(seq[-1][k] - seq[0][k]) for k in range(3)]
        if all(D[k] % Q for k in range(3)):
            assert len(a) <= 1 + sum(span)


def test_tie_free_count_formula():
    """Lines through no edge or corner visit 1 + sum |delta index| cells."""
    n = (20, 20, 6)
    g = _grid(n)
    rng = np.random.default_rng(5)
    checked = 0
    for _ in range(300):
        qin = [int(rng.integers(-2 * Q, n[a] * Q + 2 * Q)) * 2 + 1 for a in range(3)]
        qout = [int(rng.integers(-2 * Q, n[a] * Q + 2 * Q)) * 2 + 1 for a in range(3)]
        cells = oracle.line_cells(qin, qout, g)
        if len(cells) == 0:
            continue
        seq = _trace_order(qin, qout, cells, n)
        steps = [max(abs(q[k] - p[k]) for k in range(3)) for p, q in zip(seq, seq[1:])]
        diag = sum(1 for p, q in zip(seq, seq[1:]) if sum(abs(q[k] - p[k]) for k in range(3)) > 1)
        if diag == 0:
            span = sum(abs(seq[-1][k] - seq[0][k]) for k in range(3))
            assert len(cells) == 1 + span
            checked += 1
        assert all(s == 1 for s in steps)
    assert checked > 50


def test_fp64_slab_cross_check():
    """Against a floating-point slab test on the same line, the exact set differs
    only for lines passing within a hair of a voxel edge or corner."""
    n = (16, 16, 8)
    g = _grid(n)
    rng = np.random.default_rng(3)
    diff_lines = 0
    total = 400
    centres = np.stack(np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]),
                                   indexing="ij"), -1).reshape(-1, 3)
    lin = centres[:, 0] + n[0] * (centres[:, 1] + n[1] * centres[:, 2])
    for qin, qout in random_lines(rng, n, total):
        p0 = np.array(qin, dtype=np.float64) / Q
        d = (np.array(qout, dtype=np.float64) - np.array(qin, dtype=np.float64)) / Q
        with np.errstate(divide="ignore", invalid="ignore"):
            ta = (centres - p0) / d
            tb = (centres + 1 - p0) / d
        lo = np.where(d == 0, np.where((p0 >= centres) & (p0 < centres + 1), -np.inf, np.inf),
                      np.minimum(ta, tb)).max(axis=1)
        hi = np.where(d == 0, np.where((p0 >= centres) & (p0 < centres + 1), np.inf, -np.inf),
                      np.maximum(ta, tb)).min(axis=1)
        fp = np.sort(lin[lo < hi])
        ex = oracle.line_cells(qin, qout, g)
        if not np.array_equal(fp, ex):
            diff_lines += 1
    assert diff_lines <= total // 50


def test_count_lines_is_sum_of_indicators():
    n = (10, 9, 4)
    g = _grid(n)
    rng = np.random.default_rng(21)
    lines = tie_lines(rng, n, 60) + random_lines(rng, n, 60)
    qin = np.array([l[0] for l in lines], dtype=np.int32)
    qout = np.array([l[1] for l in lines], dtype=np.int32)
    counts = oracle.count_lines(qin, qout, g)
    ref = np.zeros(n[0] * n[1] * n[2], dtype=np.int64)
    for a, b in lines:
        for c in brute_cells(a, b, n):
            ref[c] += 1
    assert np.array_equal(counts, ref)
