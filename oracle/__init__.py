"""CPU oracle for proton-CT hull detection -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It wraps ``hull_oracle.c`` (plain C,
FP64 where the paper leaves the precision open) with numpy arrays and shares no
code with the GPU library in ``paper_1402_1720_amd``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hull_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# x86-64 baseline (SSE2) scalar FP32/FP64: one rounding per operation, no FMA,
# no fast-math.
ORACLE_CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                 "-fno-fast-math"]

OK, SKIP_NONFINITE, SKIP_RANGE, SKIP_DEGENERATE = 0, 1, 2, 3
MSC_COUNT, MSC_NEIGHBOR_DIFF = 0, 1
SM_FRACTION, SM_MAX_SLOPE, SM_EDGE = 0, 1, 2
SCOPE_VOLUME, SCOPE_SLICE = 0, 1
NBR_INPLANE4, NBR_SPATIAL6 = 0, 1


def build(force: bool = True) -> str:
    """Compiles ``liboracle.so`` next to its source with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *ORACLE_CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class OrGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_float), ("dy", ctypes.c_float), ("dz", ctypes.c_float),
                ("x0", ctypes.c_float), ("y0", ctypes.c_float), ("z0", ctypes.c_float)]


_FP = ctypes.POINTER(ctypes.c_float)


class OrHist(ctypes.Structure):
    _fields_ = [("x_in", _FP), ("y_in", _FP), ("z_in", _FP), ("x_out", _FP), ("y_out", _FP),
                ("z_out", _FP), ("angle_deg", _FP), ("wepl", _FP), ("n", ctypes.c_int64)]


class OrStats(ctypes.Structure):
    _fields_ = [("n_low", ctypes.c_int64), ("n_high", ctypes.c_int64),
                ("n_skipped", ctypes.c_int64), ("n_missed_grid", ctypes.c_int64),
                ("n_visits_low", ctypes.c_int64), ("n_visits_high", ctypes.c_int64)]

    def as_dict(self) -> Dict[str, int]:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class OrParams(ctypes.Structure):
    """Thresholds and modes of the one-pass call (the GPU library's
    ``hullmi_params`` layout)."""
    _fields_ = [("wepl_low", ctypes.c_float), ("wepl_high", ctypes.c_float),
                ("msc_n_t", ctypes.c_int32), ("msc_mode", ctypes.c_int32),
                ("sm_frac_num", ctypes.c_int32), ("sm_frac_den", ctypes.c_int32),
                ("sm_mode", ctypes.c_int32), ("sm_scope", ctypes.c_int32), ("nbr", ctypes.c_int32)]


class OrFbpParams(ctypes.Structure):
    _fields_ = [("src_dist_mm", ctypes.c_float), ("du_mm", ctypes.c_float),
                ("dv_mm", ctypes.c_float), ("u0_mm", ctypes.c_float), ("v0_mm", ctypes.c_float),
                ("nu", ctypes.c_int32), ("nv", ctypes.c_int32), ("n_angles", ctypes.c_int32),
                ("angle0_deg", ctypes.c_float), ("dangle_deg", ctypes.c_float),
                ("filter", ctypes.c_int32), ("threshold", ctypes.c_float)]


class OrBscParams(ctypes.Structure):
    """Binned SC: cutoff E_L (mm), data cut at k standard deviations (0 = off),
    averaging window W (odd) and the keep threshold num/den."""
    _fields_ = [("wepl_low", ctypes.c_float), ("cut_sigmas", ctypes.c_int32),
                ("window", ctypes.c_int32), ("thr_num", ctypes.c_int32),
                ("thr_den", ctypes.c_int32)]


class OrBscStats(ctypes.Structure):
    _fields_ = [("n_binned", ctypes.c_int64), ("n_cut", ctypes.c_int64),
                ("n_bins_used", ctypes.c_int64), ("n_bins_carved", ctypes.c_int64),
                ("n_lines_skipped", ctypes.c_int64), ("n_visits", ctypes.c_int64)]

    def as_dict(self) -> Dict[str, int]:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_handle = None


def _lib():
    global _handle
    if _handle is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        sig = {
            "or_abi": ([], ctypes.c_int),
            "or_trig_table": ([P, i64, P, P], None),
            "or_quantize_all": ([P, P, P, P, P], None),
            "or_line_meets_cell": ([P, P, P], ctypes.c_int),
            "or_line_cells": ([P, P, P, ctypes.c_int, P, i64], i64),
            "or_count_lines": ([P, P, i64, P, P], None),
            "or_counts": ([P, P, ctypes.c_float, ctypes.c_float, P, P, P], None),
            "or_sc": ([P, i64, P], None),
            "or_msc": ([P, P, i32, ctypes.c_int, ctypes.c_int, P], ctypes.c_int),
            "or_sm": ([P, P, i32, i32, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P], ctypes.c_int),
            "or_fbp_bin": ([P, P, P], i64),
            "or_fbp_filter": ([P, P], None),
            "or_fbp_backproject": ([P, P, P, P], None),
            "or_fbp": ([P, P, P, P, P, P], i64),
            "oracle_hull_sc": ([P, P, ctypes.c_float, P, P, P], ctypes.c_int),
            "oracle_hull_msc": ([P, P, ctypes.c_float, i32, ctypes.c_int, ctypes.c_int, P, P, P],
                                ctypes.c_int),
            "oracle_hull_sm": ([P, P, ctypes.c_float, i32, i32, ctypes.c_int, ctypes.c_int,
                                ctypes.c_int, P, P, P], ctypes.c_int),
            "oracle_hull_all": ([P, P, P, P, P, P, P, P, P], ctypes.c_int),
            "oracle_hull_fbp": ([P, P, P, P, P], ctypes.c_int),
            "or_bsc_line": ([P, P, i32, i32, i32, P, P], ctypes.c_int),
            "or_bsc_cut": ([P, P, i32, P, P, P, P], None),
            "or_fbp_cut": ([P, P, P, i32, P, P, P], i64),
            "or_bsc_blur": ([P, P, i32, i32, i32, P], None),
            "or_bsc": ([P, P, P, P, P, P, P, P, P], ctypes.c_int),
            "oracle_hull_sc_binned": ([P, P, P, P, P, P, P, P, P], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _handle = L
    return _handle


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def make_grid(n, d, origin) -> OrGrid:
    return OrGrid(int(n[0]), int(n[1]), int(n[2]), float(d[0]), float(d[1]), float(d[2]),
                  float(origin[0]), float(origin[1]), float(origin[2]))


def grid_of(g) -> OrGrid:
    """``OrGrid`` from a ``gen.Grid`` (or anything with n, d, origin)."""
    return make_grid(g.n, g.d, g.origin)


class _HistView:
    """Keeps contiguous FP32 copies of the eight history arrays alive."""

    FIELDS = ("x_in", "y_in", "z_in", "x_out", "y_out", "z_out", "angle_deg", "wepl")

    def __init__(self, hist: Dict[str, np.ndarray]):
        self.arrs = [np.ascontiguousarray(hist[k], dtype=np.float32) for k in self.FIELDS]
        n = len(self.arrs[0])
        assert all(len(a) == n for a in self.arrs)
        self.c = OrHist(*[a.ctypes.data_as(_FP) for a in self.arrs], n)


def abi() -> int:
    return _lib().or_abi()


def trig_table(angles: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    a = np.ascontiguousarray(angles, dtype=np.float32)
    c = np.empty_like(a)
    s = np.empty_like(a)
    _lib().or_trig_table(_ptr(a), len(a), _ptr(c), _ptr(s))
    return c, s


def quantize(hist: Dict[str, np.ndarray], grid: OrGrid):
    """Per history: status (OK or skip reason) and quantised endpoints [n,3]."""
    hv = _HistView(hist)
    n = hv.c.n
    st = np.empty(n, dtype=np.int32)
    qin = np.zeros((n, 3), dtype=np.int32)
    qout = np.zeros((n, 3), dtype=np.int32)
    _lib().or_quantize_all(ctypes.byref(hv.c), ctypes.byref(grid), _ptr(st), _ptr(qin), _ptr(qout))
    return st, qin, qout


def line_meets_cell(p0, d, v) -> bool:
    a = np.asarray(p0, dtype=np.int64)
    b = np.asarray(d, dtype=np.int64)
    c = np.asarray(v, dtype=np.int32)
    return bool(_lib().or_line_meets_cell(_ptr(a), _ptr(b), _ptr(c)))


def line_cells(qin, qout, grid: OrGrid, all_voxels: bool = False) -> np.ndarray:
    """A_i of one quantised line: sorted linear voxel indices (x fastest)."""
    a = np.ascontiguousarray(qin, dtype=np.int32)
    b = np.ascontiguousarray(qout, dtype=np.int32)
    cap = int(grid.nx) + int(grid.ny) + int(grid.nz) + 8
    if all_voxels:
        cap = int(grid.nx) * int(grid.ny) * int(grid.nz)
    out = np.empty(cap, dtype=np.int32)
    n = _lib().or_line_cells(_ptr(a), _ptr(b), ctypes.byref(grid), int(all_voxels), _ptr(out), cap)
    assert n <= cap
    return out[:n].copy()


def count_lines(qin: np.ndarray, qout: np.ndarray, grid: OrGrid,
                counts: Optional[np.ndarray] = None) -> np.ndarray:
    a = np.ascontiguousarray(qin, dtype=np.int32).reshape(-1, 3)
    b = np.ascontiguousarray(qout, dtype=np.int32).reshape(-1, 3)
    V = int(grid.nx) * int(grid.ny) * int(grid.nz)
    if counts is None:
        counts = np.zeros(V, dtype=np.int32)
    _lib().or_count_lines(_ptr(a), _ptr(b), len(a), ctypes.byref(grid), _ptr(counts))
    return counts


def counts(hist: Dict[str, np.ndarray], grid: OrGrid, e_low: float = 1.0, e_high: float = 5.0,
           want_n: bool = True, want_m: bool = True):
    """(N, M, stats): low/high crossing counts per voxel, int32, x fastest."""
    hv = _HistView(hist)
    V = int(grid.nx) * int(grid.ny) * int(grid.nz)
    N = np.zeros(V, dtype=np.int32) if want_n else None
    M = np.zeros(V, dtype=np.int32) if want_m else None
    st = OrStats()
    _lib().or_counts(ctypes.byref(hv.c), ctypes.byref(grid), float(e_low), float(e_high),
                     _ptr(N), _ptr(M), ctypes.byref(st))
    return N, M, st.as_dict()


def sc(N: np.ndarray) -> np.ndarray:
    N = np.ascontiguousarray(N, dtype=np.int32)
    mask = np.empty(N.size, dtype=np.uint8)
    _lib().or_sc(_ptr(N), N.size, _ptr(mask))
    return mask


def msc(N: np.ndarray, grid: OrGrid, n_t: int, mode: int = MSC_COUNT,
        nbr: int = NBR_INPLANE4) -> np.ndarray:
    N = np.ascontiguousarray(N, dtype=np.int32).reshape(-1)
    mask = np.empty(N.size, dtype=np.uint8)
    rc = _lib().or_msc(_ptr(N), ctypes.byref(grid), int(n_t), int(mode), int(nbr), _ptr(mask))
    if rc != 0:
        raise ValueError("bad MSC mode")
    return mask


def sm(M: np.ndarray, grid: OrGrid, num: int = 3, den: int = 5, mode: int = SM_FRACTION,
       scope: int = SCOPE_VOLUME, nbr: int = NBR_INPLANE4):
    """(mask, thresholds): thresholds are max M (FRACTION) or M_t (MAX_SLOPE),
    one per slice for scope SLICE."""
    M = np.ascontiguousarray(M, dtype=np.int32).reshape(-1)
    mask = np.empty(M.size, dtype=np.uint8)
    mt = np.zeros(int(grid.nz) if scope == SCOPE_SLICE else 1, dtype=np.int64)
    rc = _lib().or_sm(_ptr(M), ctypes.byref(grid), int(num), int(den), int(mode), int(scope),
                      int(nbr), _ptr(mask), _ptr(mt))
    if rc != 0:
        raise ValueError("bad SM mode/scope")
    return mask, mt


def fbp_params(geo) -> OrFbpParams:
    """``OrFbpParams`` from a ``gen.FbpGeometry``."""
    return OrFbpParams(geo.src_dist, geo.du, geo.dv, geo.u0, geo.v0, geo.nu, geo.nv,
                       geo.n_angles, geo.angle0, geo.dangle, 0, geo.threshold)


def fbp_bin(hist, p: OrFbpParams) -> Tuple[np.ndarray, int]:
    hv = _HistView(hist)
    proj = np.zeros(int(p.n_angles) * int(p.nv) * int(p.nu), dtype=np.float64)
    used = _lib().or_fbp_bin(ctypes.byref(hv.c), ctypes.byref(p), _ptr(proj))
    return proj, int(used)


def fbp_filter(p: OrFbpParams, proj: np.ndarray) -> np.ndarray:
    q = np.ascontiguousarray(proj, dtype=np.float64).copy()
    _lib().or_fbp_filter(ctypes.byref(p), _ptr(q))
    return q


def fbp_backproject(grid: OrGrid, p: OrFbpParams, q: np.ndarray) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.float64)
    img = np.zeros(int(grid.nx) * int(grid.ny) * int(grid.nz), dtype=np.float64)
    _lib().or_fbp_backproject(ctypes.byref(grid), ctypes.byref(p), _ptr(q), _ptr(img))
    return img


def fbp(hist, grid: OrGrid, p: OrFbpParams):
    """(image FP64, mask uint8, filtered projections, histories binned)."""
    hv = _HistView(hist)
    V = int(grid.nx) * int(grid.ny) * int(grid.nz)
    proj = np.zeros(int(p.n_angles) * int(p.nv) * int(p.nu), dtype=np.float64)
    img = np.zeros(V, dtype=np.float64)
    mask = np.zeros(V, dtype=np.uint8)
    used = _lib().or_fbp(ctypes.byref(hv.c), ctypes.byref(grid), ctypes.byref(p), _ptr(proj),
                         _ptr(img), _ptr(mask))
    return img, mask, proj, int(used)


def bsc_params(wepl_low: float = 1.0, cut_sigmas: int = 3, window: int = 5, thr_num: int = 2,
               thr_den: int = 5) -> OrBscParams:
    """Binned SC parameters; the defaults are the paper's (Sections 2.2, 3.2):
    E_L = 1.0 mm, 3-sigma cuts, 5 x 5 averaging, threshold 0.4."""
    return OrBscParams(wepl_low, cut_sigmas, window, thr_num, thr_den)


def bsc_line(p: OrFbpParams, grid: OrGrid, k: int, iu: int, iv: int):
    """(status, qin, qout): the quantised carve line of bin (k, iu, iv)."""
    qin = np.zeros(3, np.int32)
    qout = np.zeros(3, np.int32)
    st = _lib().or_bsc_line(ctypes.byref(p), ctypes.byref(grid), int(k), int(iu), int(iv),
                            _ptr(qin), _ptr(qout))
    return int(st), qin, qout


def bsc_blur(carved: np.ndarray, grid: OrGrid, window: int = 5, thr_num: int = 2,
             thr_den: int = 5) -> np.ndarray:
    c = np.ascontiguousarray(carved, dtype=np.uint8).reshape(-1)
    mask = np.empty(c.size, np.uint8)
    _lib().or_bsc_blur(_ptr(c), ctypes.byref(grid), int(window), int(thr_num), int(thr_den),
                       _ptr(mask))
    return mask


def bsc_cut(hist, p: OrFbpParams, k: int = 3):
    """(bin, keep, binned, cut): per history its bin (-1 when not binned) and
    whether the data cut at k standard deviations keeps it."""
    hv = _HistView(hist)
    n = hv.c.n
    b = np.empty(max(n, 1), np.int64)
    keep = np.empty(max(n, 1), np.uint8)
    nb, nc = ctypes.c_int64(0), ctypes.c_int64(0)
    _lib().or_bsc_cut(ctypes.byref(hv.c), ctypes.byref(p), int(k), _ptr(b), _ptr(keep),
                      ctypes.byref(nb), ctypes.byref(nc))
    return b[:n], keep[:n].astype(bool), int(nb.value), int(nc.value)


def fbp_cut(hist, grid: OrGrid, p: OrFbpParams, k: int = 3):
    """FDK hull after the data cuts: (image FP64, mask, kept bin means, kept)."""
    hv = _HistView(hist)
    V = _vox(grid)
    nb = int(p.n_angles) * int(p.nv) * int(p.nu)
    proj, img, mask = np.zeros(nb), np.zeros(V), np.zeros(V, np.uint8)
    kept = _lib().or_fbp_cut(ctypes.byref(hv.c), ctypes.byref(grid), ctypes.byref(p), int(k),
                             _ptr(proj), _ptr(img), _ptr(mask))
    if kept < 0:
        raise ValueError("FDK after cuts rejected its arguments")
    return img, mask, proj, int(kept)


def sc_binned(hist, grid: OrGrid, p: OrFbpParams, bp: Optional[OrBscParams] = None):
    """Binned SC: dict with kept_n, kept_sum (per bin, 1/1024 mm), carved,
    mask and stats."""
    bp = bp if bp is not None else bsc_params()
    hv = _HistView(hist)
    V = _vox(grid)
    nb = int(p.n_angles) * int(p.nv) * int(p.nu)
    kn, ks = np.empty(nb, np.uint32), np.empty(nb, np.int64)
    carved, mask, st = np.empty(V, np.uint8), np.empty(V, np.uint8), OrBscStats()
    if _lib().or_bsc(ctypes.byref(hv.c), ctypes.byref(grid), ctypes.byref(p), ctypes.byref(bp),
                     _ptr(kn), _ptr(ks), _ptr(carved), _ptr(mask), ctypes.byref(st)) != 0:
        raise ValueError("binned SC rejected its arguments")
    return dict(kept_n=kn, kept_sum=ks, carved=carved, mask=mask, stats=st.as_dict())


# ---------------------------------------------------------------------------
# whole-call mirrors of the GPU library's per-scan calls (host arrays)

def _vox(grid: OrGrid) -> int:
    return int(grid.nx) * int(grid.ny) * int(grid.nz)


def hull_sc(hist, grid: OrGrid, wepl_low: float = 1.0):
    """(N, SC mask, stats)."""
    hv = _HistView(hist)
    V = _vox(grid)
    N, mask, st = np.empty(V, np.int32), np.empty(V, np.uint8), OrStats()
    if _lib().oracle_hull_sc(ctypes.byref(hv.c), ctypes.byref(grid), float(wepl_low), _ptr(N),
                             _ptr(mask), ctypes.byref(st)) != 0:
        raise ValueError("oracle_hull_sc rejected its arguments")
    return N, mask, st.as_dict()


def hull_msc(hist, grid: OrGrid, wepl_low: float, n_t: int, mode: int, nbr: int):
    """(N, MSC mask, stats)."""
    hv = _HistView(hist)
    V = _vox(grid)
    N, mask, st = np.empty(V, np.int32), np.empty(V, np.uint8), OrStats()
    if _lib().oracle_hull_msc(ctypes.byref(hv.c), ctypes.byref(grid), float(wepl_low), int(n_t),
                              int(mode), int(nbr), _ptr(N), _ptr(mask), ctypes.byref(st)) != 0:
        raise ValueError("oracle_hull_msc rejected its arguments")
    return N, mask, st.as_dict()


def hull_sm(hist, grid: OrGrid, wepl_high: float, num: int, den: int, mode: int, scope: int,
            nbr: int):
    """(M, SM mask, stats)."""
    hv = _HistView(hist)
    V = _vox(grid)
    M, mask, st = np.empty(V, np.int32), np.empty(V, np.uint8), OrStats()
    if _lib().oracle_hull_sm(ctypes.byref(hv.c), ctypes.byref(grid), float(wepl_high), int(num),
                             int(den), int(mode), int(scope), int(nbr), _ptr(M), _ptr(mask),
                             ctypes.byref(st)) != 0:
        raise ValueError("oracle_hull_sm rejected its arguments")
    return M, mask, st.as_dict()


def hull_all(hist, grid: OrGrid, p: OrParams):
    """(N, M, SC mask, MSC mask, SM mask, stats)."""
    hv = _HistView(hist)
    V = _vox(grid)
    N, M = np.empty(V, np.int32), np.empty(V, np.int32)
    m1, m2, m3 = (np.empty(V, np.uint8) for _ in range(3))
    st = OrStats()
    if _lib().oracle_hull_all(ctypes.byref(hv.c), ctypes.byref(grid), ctypes.byref(p), _ptr(N),
                              _ptr(M), _ptr(m1), _ptr(m2), _ptr(m3), ctypes.byref(st)) != 0:
        raise ValueError("oracle_hull_all rejected its arguments")
    return N, M, m1, m2, m3, st.as_dict()


def hull_fbp(hist, grid: OrGrid, p: OrFbpParams):
    """(image FP64, mask)."""
    hv = _HistView(hist)
    V = _vox(grid)
    img, mask = np.empty(V, np.float64), np.empty(V, np.uint8)
    if _lib().oracle_hull_fbp(ctypes.byref(hv.c), ctypes.byref(grid), ctypes.byref(p), _ptr(img),
                              _ptr(mask)) != 0:
        raise ValueError("oracle_hull_fbp rejected its arguments")
    return img, mask


def hull_sc_binned(hist, grid: OrGrid, p: OrFbpParams, bp: OrBscParams):
    """(kept_n, kept_sum, carved, mask, stats) through the mirror call."""
    hv = _HistView(hist)
    V = _vox(grid)
    nb = int(p.n_angles) * int(p.nv) * int(p.nu)
    kn, ks = np.empty(nb, np.uint32), np.empty(nb, np.int64)
    carved, mask, st = np.empty(V, np.uint8), np.empty(V, np.uint8), OrBscStats()
    if _lib().oracle_hull_sc_binned(ctypes.byref(hv.c), ctypes.byref(grid), ctypes.byref(p),
                                    ctypes.byref(bp), _ptr(kn), _ptr(ks), _ptr(carved), _ptr(mask),
                                    ctypes.byref(st)) != 0:
        raise ValueError("oracle_hull_sc_binned rejected its arguments")
    return kn, ks, carved, mask, st.as_dict()
