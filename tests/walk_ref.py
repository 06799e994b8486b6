"""Independent exact references for the voxel set A_i of a line.

Written directly from the set definition A_i = { v : d(L_i, v) <= d0 }
(Sections 3.2 and 3.4) under the half-open reading: v is in A_i when some point
of the infinite line P(t) = P0 + t D lies in the box [1024 v, 1024 (v + 1)) on
every axis. Python fractions make every comparison exact. Used only to pin the
oracle and to describe the GPU parity cases; not used by either implementation.
"""
from fractions import Fraction
from typing import List, Sequence, Tuple

Q = 1024


def brute_cells(qin: Sequence[int], qout: Sequence[int], n: Sequence[int]) -> List[int]:
    """Every voxel of the grid tested against the line (Algorithm 1's inner
    loop): the intersection of the per-axis parameter intervals must be
    non-empty. Returns sorted linear indices (x fastest)."""
    P0 = [int(v) for v in qin]
    D = [int(b) - int(a) for a, b in zip(qin, qout)]
    assert any(D)
    out = []
    for k in range(n[2]):
        for j in range(n[1]):
            for i in range(n[0]):
                if _meets((i, j, k), P0, D):
                    out.append(i + n[0] * (j + n[1] * k))
    return out


def _meets(v, P0, D) -> bool:
    lo, lo_closed = None, True   # None = -infinity
    hi, hi_closed = None, True   # None = +infinity
    for a in range(3):
        base = Q * v[a]
        if D[a] == 0:
            if not (base <= P0[a] < base + Q):
                return False
            continue
        t_at_low_face = Fraction(base - P0[a], D[a])
        t_at_high_face = Fraction(base + Q - P0[a], D[a])
        if D[a] > 0:   # [t_low, t_high)
            l, lc, h, hc = t_at_low_face, True, t_at_high_face, False
        else:          # (t_high, t_low]
            l, lc, h, hc = t_at_high_face, False, t_at_low_face, True
        if lo is None or l > lo:
            lo, lo_closed = l, lc
        elif l == lo:
            lo_closed = lo_closed and lc
        if hi is None or h < hi:
            hi, hi_closed = h, hc
        elif h == hi:
            hi_closed = hi_closed and hc
    if lo is None or hi is None:
        return True
    return lo < hi or (lo == hi and lo_closed and hi_closed)


def cells_from_text(spec: str, n: Sequence[int]) -> List[int]:
    if spec.strip() == "none":
        return []
    out = []
    for tri in spec.split(";"):
        i, j, k = (int(x) for x in tri.split(","))
        out.append(i + n[0] * (j + n[1] * k))
    return sorted(out)


def load_golden(path: str) -> List[Tuple[str, Tuple[int, int, int], Tuple[int, ...], Tuple[int, ...], List[int]]]:
    cases = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, n, qin, qout, cells = (p.strip() for p in line.split("|"))
            n = tuple(int(x) for x in n.split())
            qin = tuple(int(x) for x in qin.split())
            qout = tuple(int(x) for x in qout.split())
            cases.append((name, n, qin, qout, cells_from_text(cells, n)))
    return cases


def tie_lines(rng, n: Sequence[int], count: int):
    """Random lines rich in exact ties: endpoints on a coarse lattice (multiples
    of 256 or 1024 in 1/1024-voxel units, some exactly on grid faces, edges and
    corners), fixed axes, and points inside or outside the grid."""
    lines = []
    for _ in range(count):
        step = int(rng.choice([1024, 512, 256]))
        lo = [-(2 * Q) // step for _ in range(3)]
        qin = [int(rng.integers(lo[a], (n[a] * Q + 2 * Q) // step + 1)) * step for a in range(3)]
        qout = [int(rng.integers(lo[a], (n[a] * Q + 2 * Q) // step + 1)) * step for a in range(3)]
        # sometimes freeze an axis, or two
        for a in range(3):
            if rng.random() < 0.2:
                qout[a] = qin[a]
        if qin == qout:
            qout[0] += step
        lines.append((qin, qout))
    return lines


def random_lines(rng, n: Sequence[int], count: int):
    """Generic lines with arbitrary 1/1024 endpoints around the grid."""
    lines = []
    for _ in range(count):
        qin = [int(rng.integers(-3 * Q, n[a] * Q + 3 * Q)) for a in range(3)]
        qout = [int(rng.integers(-3 * Q, n[a] * Q + 3 * Q)) for a in range(3)]
        if qin == qout:
            qout[2] += 1
        lines.append((qin, qout))
    return lines
