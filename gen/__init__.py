"""Seeded synthetic proton-CT scans for the hull-detection path.

Inputs only: this package builds head phantoms out of nested ellipsoids and
simulates cone-beam proton histories through them (see ``scan_gen.c``). It
holds none of the hull-detection arithmetic; the CPU oracle and the GPU library
both consume what it produces.

The paper's data sets (a simulated NEO digital head phantom with 11,796,480
histories, Section 2.1, and a scanned pediatric head phantom, Section 2.2) are
not available; the scans made here stand in for them with the same shapes: a
200 mm field, 3 mm slices, head-sized nested ellipsoids with the paper's RSP
values (skull 1.6, brain 1.04, Section 2.1) and about 1e7 histories.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field, replace
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "scan_gen.c")
_LIB = os.path.join(_HERE, "libscangen.so")

# FP64 physics, reproducible rounding: no contraction, no fast-math.
GEN_CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off"]


def build(force: bool = True) -> str:
    """Compiles ``libscangen.so`` next to its source with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *GEN_CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Ellipsoid(ctypes.Structure):
    _fields_ = [("cx", ctypes.c_double), ("cy", ctypes.c_double), ("cz", ctypes.c_double),
                ("a", ctypes.c_double), ("b", ctypes.c_double), ("c", ctypes.c_double),
                ("drho", ctypes.c_double)]


class _ScanConfig(ctypes.Structure):
    _fields_ = [("n_hist", ctypes.c_int64), ("n_angles", ctypes.c_int32),
                ("n_ellipsoids", ctypes.c_int32), ("angle0_deg", ctypes.c_double),
                ("src_dist", ctypes.c_double), ("tracker_x", ctypes.c_double),
                ("fan_y", ctypes.c_double), ("fan_z", ctypes.c_double),
                ("sigma", ctypes.c_double), ("outlier_frac", ctypes.c_double),
                ("outlier_max", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("ell", ctypes.POINTER(_Ellipsoid))]


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        fp = ctypes.POINTER(ctypes.c_float)
        lib.gen_scan.argtypes = [ctypes.POINTER(_ScanConfig), ctypes.c_int64, ctypes.c_int64,
                                 fp, fp, fp, fp, fp, fp, fp, fp, ctypes.POINTER(ctypes.c_double)]
        lib.gen_scan.restype = ctypes.c_int
        lib.gen_chord.argtypes = [ctypes.POINTER(_Ellipsoid), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)]
        lib.gen_chord.restype = ctypes.c_double
        _lib_handle = lib
    return _lib_handle


@dataclass(frozen=True)
class Ellipsoid:
    """Axis-aligned ellipsoid in the object frame (mm) adding ``drho`` RSP inside."""
    centre: Tuple[float, float, float]
    semi: Tuple[float, float, float]
    drho: float

    def _c(self) -> _Ellipsoid:
        return _Ellipsoid(*self.centre, *self.semi, self.drho)


@dataclass(frozen=True)
class Grid:
    """Voxel grid in the object frame: ``n`` voxels of size ``d`` mm per axis,
    centred on the isocentre; ``origin`` is the lower corner of voxel (0,0,0)."""
    n: Tuple[int, int, int]
    d: Tuple[float, float, float]

    @property
    def origin(self) -> Tuple[float, float, float]:
        return tuple(-0.5 * n * d for n, d in zip(self.n, self.d))

    @property
    def half(self) -> Tuple[float, float, float]:
        return tuple(0.5 * n * d for n, d in zip(self.n, self.d))

    @property
    def voxels(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]


@dataclass(frozen=True)
class FbpGeometry:
    """Virtual detector at the isocentre plane for the FDK baseline."""
    src_dist: float
    du: float
    dv: float
    nu: int
    nv: int
    u0: float
    v0: float
    n_angles: int
    angle0: float
    dangle: float
    threshold: float = 0.6


@dataclass(frozen=True)
class ScanSpec:
    grid: Grid
    n_hist: int
    n_angles: int
    phantom: Tuple[Ellipsoid, ...]
    seed: int
    sigma: float = 0.0
    outlier_frac: float = 0.0
    outlier_max: float = 300.0
    src_dist: float = 2000.0
    tracker_x: float = 100.0
    angle0: float = 0.0
    fan: Optional[Tuple[float, float]] = None

    @property
    def fan_yz(self) -> Tuple[float, float]:
        if self.fan is not None:
            return self.fan
        hx, hy, hz = self.grid.half
        return (1.05 * math.hypot(hx, hy), 1.05 * hz)

    def fbp_geometry(self, du: float = 1.0, dv: float = 5.0) -> FbpGeometry:
        fy, fz = self.fan_yz
        nu = 2 * int(math.ceil(fy / du))
        nv = 2 * int(math.ceil(fz / dv))
        return FbpGeometry(src_dist=self.src_dist, du=du, dv=dv, nu=nu, nv=nv,
                           u0=-0.5 * nu * du, v0=-0.5 * nv * dv, n_angles=self.n_angles,
                           angle0=self.angle0, dangle=360.0 / self.n_angles)


def head_phantom(grid: Grid, inserts: bool = False,
                 scale: Tuple[float, float, float] = (1.0, 1.0, 1.0),
                 ventricles: bool = False) -> Tuple[Ellipsoid, ...]:
    """Nested-ellipsoid head: skull shell (RSP 1.6) around brain (RSP 1.04), the
    paper's tissue values (Section 2.1). Skull semi-axes are (0.62, 0.78, 0.90)
    of the grid half-extents; at a 200 mm field that is a 15,193 mm^2 central
    slice, within 1% of the paper's 15,336-voxel phantom slice (Section 4.1).
    Optional inserts: three 1 cm ellipsoids of RSP 0.3, 1.1 and 1.8 in the brain.
    Optional ventricles: the paper's phantom also holds two fluid-filled
    ventricles of RSP 0.9 inside the brain (Section 2.1; their size and place
    are not given): ellipsoids of semi-axes (0.12, 0.30, 0.30) of the brain's,
    centred at (+-0.22 a, 0.08 b, 0.05 c) of the brain semi-axes (a, b, c),
    elongated front to back like lateral ventricles and apart from each other.
    Ventricles and inserts are meant to be used one at a time (they would
    overlap)."""
    hx, hy, hz = grid.half
    sx, sy, sz = scale
    a, b, c = 0.62 * hx * sx, 0.78 * hy * sy, 0.90 * hz * sz
    t = 0.06 * min(hx, hy)
    ab, bb, cb = a - t, b - t, c - t
    ells = [Ellipsoid((0.0, 0.0, 0.0), (a, b, c), 1.6),
            Ellipsoid((0.0, 0.0, 0.0), (ab, bb, cb), 1.04 - 1.6)]
    if inserts:
        for (cx, cy), rho in (((0.35 * ab, 0.25 * bb), 0.3), ((-0.35 * ab, 0.25 * bb), 1.1),
                              ((0.0, -0.35 * bb), 1.8)):
            ells.append(Ellipsoid((cx, cy, 0.0), (5.0, 4.0, 5.0), rho - 1.04))
    if ventricles:
        for side in (1.0, -1.0):
            ells.append(Ellipsoid((side * 0.22 * ab, 0.08 * bb, 0.05 * cb),
                                  (0.12 * ab, 0.30 * bb, 0.30 * cb), 0.9 - 1.04))
    return tuple(ells)


def ventricle_spec(n_hist: int = 10_000_000, seed_offset: int = 0) -> ScanSpec:
    """The paper's simulated head (skull, brain, two ventricles of RSP 0.9,
    Section 2.1) on the 200x200x32 grid of 1x1x3 mm voxels (the paper's FDK
    volume, Section 3.1), 180 gantry angles, WEPL noise 3 mm; seed 0x5EED0006."""
    g = Grid((200, 200, 32), (1.0, 1.0, 3.0))
    return ScanSpec(g, int(n_hist), 180, head_phantom(g, ventricles=True),
                    0x5EED0006 + seed_offset, sigma=3.0)


def sphere_phantom(radius: float, rho: float = 1.0,
                   centre: Tuple[float, float, float] = (0.0, 0.0, 0.0)) -> Tuple[Ellipsoid, ...]:
    return (Ellipsoid(centre, (radius, radius, radius), rho),)


def config_spec(config: int, seed_offset: int = 0, n_hist: Optional[int] = None) -> ScanSpec:
    """The three single-scan workloads (small SC case, the 200x200x32 mixed case,
    the full-scale 256x256x64 case) with seed 0x5EED0000 + config (+ offset)."""
    seed = 0x5EED0000 + config + seed_offset
    if config == 1:
        g = Grid((64, 64, 16), (1.0, 1.0, 2.5))
        spec = ScanSpec(g, 100_000, 90, head_phantom(g), seed)
    elif config == 2:
        g = Grid((200, 200, 32), (1.0, 1.0, 3.0))
        spec = ScanSpec(g, 10_000_000, 180, head_phantom(g, inserts=True), seed, sigma=3.0)
    elif config == 3:
        g = Grid((256, 256, 64), (0.78125, 0.78125, 2.5))
        spec = ScanSpec(g, 200_000_000, 360, head_phantom(g, inserts=True), seed, sigma=3.0,
                        outlier_frac=0.02)
    else:
        raise ValueError(f"no single-scan config {config}")
    if n_hist is not None:
        spec = replace(spec, n_hist=int(n_hist))
    return spec


FIELDS = ("x_in", "y_in", "z_in", "x_out", "y_out", "z_out", "angle_deg", "wepl")


def generate(spec: ScanSpec, h0: int = 0, h1: Optional[int] = None,
             with_true: bool = False) -> Dict[str, np.ndarray]:
    """Histories ``[h0, h1)`` of the scan as FP32 SoA numpy arrays (plus
    ``wepl_true`` in FP64 when asked)."""
    if h1 is None:
        h1 = spec.n_hist
    n = h1 - h0
    out = {k: np.empty(n, dtype=np.float32) for k in FIELDS}
    wt = np.empty(n, dtype=np.float64) if with_true else None
    ells = (_Ellipsoid * max(1, len(spec.phantom)))(*[e._c() for e in spec.phantom])
    fy, fz = spec.fan_yz
    cfg = _ScanConfig(spec.n_hist, spec.n_angles, len(spec.phantom), spec.angle0,
                      spec.src_dist, spec.tracker_x, fy, fz, spec.sigma, spec.outlier_frac,
                      spec.outlier_max, spec.seed & 0xFFFFFFFFFFFFFFFF,
                      ctypes.cast(ells, ctypes.POINTER(_Ellipsoid)))
    fp = ctypes.POINTER(ctypes.c_float)
    args = [out[k].ctypes.data_as(fp) for k in FIELDS]
    rc = _lib().gen_scan(ctypes.byref(cfg), h0, h1, *args,
                         wt.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if wt is not None else None)
    if rc != 0:
        raise ValueError("gen_scan rejected its arguments")
    if wt is not None:
        out["wepl_true"] = wt
    return out


def chord(ell: Ellipsoid, p: Sequence[float], u: Sequence[float]) -> float:
    """Chord length of the line p + t*u (u a unit vector) through ``ell``."""
    pa = (ctypes.c_double * 3)(*p)
    ua = (ctypes.c_double * 3)(*u)
    e = ell._c()
    return _lib().gen_chord(ctypes.byref(e), pa, ua)


def phantom_rsp(phantom: Sequence[Ellipsoid], pts: np.ndarray) -> np.ndarray:
    """RSP at object-frame points ``pts`` [..., 3] (truth for hull quality)."""
    rsp = np.zeros(pts.shape[:-1], dtype=np.float64)
    for e in phantom:
        r = sum(((pts[..., i] - e.centre[i]) / e.semi[i]) ** 2 for i in range(3))
        rsp += np.where(r <= 1.0, e.drho, 0.0)
    return rsp


def voxel_centres(grid: Grid) -> np.ndarray:
    """Object-frame voxel centres, shape [nz, ny, nx, 3] (x fastest)."""
    (nx, ny, nz), (dx, dy, dz), (x0, y0, z0) = grid.n, grid.d, grid.origin
    x = x0 + (np.arange(nx) + 0.5) * dx
    y = y0 + (np.arange(ny) + 0.5) * dy
    z = z0 + (np.arange(nz) + 0.5) * dz
    zz, yy, xx = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([xx, yy, zz], axis=-1)


# ---------------------------------------------------------------------------
# Batched and served workloads: many scans of uneven size on several grids.

BATCH_GRIDS = (Grid((64, 64, 16), (1.0, 1.0, 2.5)), Grid((128, 128, 32), (1.0, 1.0, 2.5)),
               Grid((200, 200, 32), (1.0, 1.0, 2.5)), Grid((256, 256, 64), (0.78125, 0.78125, 2.5)))


def batch_specs(n_scans: int = 16, h_lo: float = 1e5, h_hi: float = 5e7, seed: int = 0x5EED0004,
                grids: Sequence[Grid] = BATCH_GRIDS, hist_scale: float = 1.0) -> List[ScanSpec]:
    """Scans with log-uniform history counts, grids drawn from ``grids``,
    ellipsoid sizes jittered by +-15% and noise sigma U[1, 5] mm."""
    rng = np.random.default_rng(seed)
    specs = []
    for s in range(n_scans):
        g = grids[int(rng.integers(len(grids)))]
        h = int(round(math.exp(rng.uniform(math.log(h_lo), math.log(h_hi))) * hist_scale))
        h = max(h, 1)
        scale = tuple(float(v) for v in rng.uniform(0.85, 1.15, size=3))
        sigma = float(rng.uniform(1.0, 5.0))
        n_ang = 90 if g.n[0] <= 64 else 180
        specs.append(ScanSpec(g, h, n_ang, head_phantom(g, inserts=g.n[0] >= 200, scale=scale),
                              seed + 1000 * (s + 1), sigma=sigma))
    return specs
