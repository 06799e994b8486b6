"""ctypes binding of ``libhullmi.so`` (C ABI in ``include/hullmi.h``).

Argument marshalling only: every step of the hull path runs in the HIP
library. torch tensors provide device memory and streams. Sizes, dtypes and
devices are checked here, because the C ABI takes bare pointers.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Dict, Optional, Sequence

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhullmi.so")

HULL_OK, HULL_EINVAL, HULL_ENOMEM, HULL_EDEVICE, HULL_EBUSY, HULL_ENOTSUP, HULL_ETIMEDOUT = range(7)
HULL_ACCUMULATE = 1
HULL_MSC_COUNT, HULL_MSC_NEIGHBOR_DIFF = 0, 1
HULL_SM_FRACTION, HULL_SM_MAX_SLOPE, HULL_SM_EDGE = 0, 1, 2
HULL_SCOPE_VOLUME, HULL_SCOPE_SLICE = 0, 1
HULL_NBR_INPLANE4, HULL_NBR_SPATIAL6 = 0, 1
(HULL_OP_SC, HULL_OP_MSC, HULL_OP_SM, HULL_OP_ALL, HULL_OP_FBP, HULL_OP_COUNT_LINES,
 HULL_OP_SC_BINNED, HULL_OP_FBP_CUT) = range(8)

ABI_VERSION = 3          # the struct layouts below
FIELDS = ("x_in", "y_in", "z_in", "x_out", "y_out", "z_out", "angle_deg", "wepl")


class hullmi_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_float), ("dy", ctypes.c_float), ("dz", ctypes.c_float),
                ("x0", ctypes.c_float), ("y0", ctypes.c_float), ("z0", ctypes.c_float)]


class hullmi_histories(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in FIELDS] + [("n", ctypes.c_int64)]


class hullmi_params(ctypes.Structure):
    _fields_ = [("wepl_low", ctypes.c_float), ("wepl_high", ctypes.c_float),
                ("msc_n_t", ctypes.c_int32), ("msc_mode", ctypes.c_int32),
                ("sm_frac_num", ctypes.c_int32), ("sm_frac_den", ctypes.c_int32),
                ("sm_mode", ctypes.c_int32), ("sm_scope", ctypes.c_int32), ("nbr", ctypes.c_int32)]


class hullmi_fbp_params(ctypes.Structure):
    _fields_ = [("src_dist_mm", ctypes.c_float), ("du_mm", ctypes.c_float),
                ("dv_mm", ctypes.c_float), ("u0_mm", ctypes.c_float), ("v0_mm", ctypes.c_float),
                ("nu", ctypes.c_int32), ("nv", ctypes.c_int32), ("n_angles", ctypes.c_int32),
                ("angle0_deg", ctypes.c_float), ("dangle_deg", ctypes.c_float),
                ("filter", ctypes.c_int32), ("threshold", ctypes.c_float)]


class hullmi_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("n_low", "n_high", "n_skipped", "n_missed_grid",
                                               "n_visits_low", "n_visits_high")]


class hullmi_bsc_params(ctypes.Structure):
    _fields_ = [("wepl_low", ctypes.c_float), ("cut_sigmas", ctypes.c_int32),
                ("window", ctypes.c_int32), ("thr_num", ctypes.c_int32), ("thr_den", ctypes.c_int32)]


BSC_STATS_FIELDS = ("n_binned", "n_cut", "n_bins_used", "n_bins_carved", "n_lines_skipped",
                    "n_visits")


_OUT_FIELDS = [("N", ctypes.c_void_p), ("M", ctypes.c_void_p), ("sc_mask", ctypes.c_void_p),
               ("msc_mask", ctypes.c_void_p), ("sm_mask", ctypes.c_void_p),
               ("image", ctypes.c_void_p), ("fbp_mask", ctypes.c_void_p)]


class hullmi_job(ctypes.Structure):
    _fields_ = ([("op", ctypes.c_int32), ("flags", ctypes.c_uint32), ("hist", hullmi_histories),
                 ("grid", hullmi_grid), ("params", hullmi_params), ("fbp", hullmi_fbp_params)]
                + _OUT_FIELDS + [("stats", ctypes.c_void_p), ("bsc", hullmi_bsc_params),
                                 ("bsc_mask", ctypes.c_void_p), ("bsc_stats", ctypes.c_void_p)])


class hullmi_tuning(ctypes.Structure):
    _fields_ = [("streams", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("walk_blocks", ctypes.c_int32), ("ranges_per_group", ctypes.c_int32),
                ("length_classes", ctypes.c_int32), ("run_stride", ctypes.c_int32)]

    def as_dict(self) -> Dict[str, int]:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class hullmi_request(ctypes.Structure):
    _fields_ = ([("op", ctypes.c_int32), ("hist", hullmi_histories), ("grid", hullmi_grid),
                 ("params", hullmi_params), ("fbp", hullmi_fbp_params)] + _OUT_FIELDS
                + [("bsc", hullmi_bsc_params), ("bsc_mask", ctypes.c_void_p)])


class hullmi_bsc_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in BSC_STATS_FIELDS]


class hullmi_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("stats", hullmi_stats),
                ("bsc_stats", hullmi_bsc_stats),
                ("t_arrive_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64), ("device_ms", ctypes.c_float),
                ("h2d_ms", ctypes.c_float), ("compute_ms", ctypes.c_float),
                ("d2h_ms", ctypes.c_float)]


class hullmi_server_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "completed", "failed", "queued",
                                               "running", "histories_done")] + \
               [(k, ctypes.c_uint64) for k in ("bytes_budget", "bytes_in_use", "bytes_peak")]


# every symbol the header declares, with its ctypes signature
_P, _I32, _I64, _U32, _F, _SZ = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                 ctypes.c_float, ctypes.c_size_t)
SIGNATURES = {
    "hull_abi_version": ([], ctypes.c_int),
    "hull_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "hull_workspace_bytes": ([ctypes.c_int, _P, _I64, _P], _SZ),
    "hull_sc": ([_P, _P, _F, _P, _P, _U32, _P, _P, _SZ, _P], ctypes.c_int),
    "hull_msc": ([_P, _P, _F, _I32, ctypes.c_int, ctypes.c_int, _P, _P, _U32, _P, _P, _SZ, _P],
                 ctypes.c_int),
    "hull_sm": ([_P, _P, _F, _I32, _I32, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P, _U32,
                 _P, _P, _SZ, _P], ctypes.c_int),
    "hull_all": ([_P, _P, _P, _P, _P, _P, _P, _P, _U32, _P, _P, _SZ, _P], ctypes.c_int),
    "hull_fbp": ([_P, _P, _P, _P, _P, _P, _SZ, _P], ctypes.c_int),
    "hull_sc_binned": ([_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _SZ, _P], ctypes.c_int),
    "hull_fbp_cut": ([_P, _P, _P, _I32, _P, _P, _P, _SZ, _P], ctypes.c_int),
    "hull_count_lines": ([_P, _P, _I64, _P, _P, _U32, _P, _P, _SZ, _P], ctypes.c_int),
    "hull_quantize": ([_P, _P, _P, _P, _P, _P], ctypes.c_int),
    "hull_count_profile": ([_P, _P, _P, _P, _P, _U32, _P, _P, _SZ, _P, _P, _P], ctypes.c_int),
    "hull_fbp_profile": ([_P, _P, _P, _P, _P, _P, _SZ, _P, _P, _P], ctypes.c_int),
    "hull_fbp_noalloc": ([_P, _P, _P, _P, _P, _P], ctypes.c_int),
    "hull_footprint_bytes": ([ctypes.c_int, _P, _I64, _P], _SZ),
    "hull_batch_plan": ([_P, ctypes.c_int, _P, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "hull_batch_launch": ([_P, _P], ctypes.c_int),
    "hull_batch_tuning": ([_P, _P], ctypes.c_int),
    "hull_batch_destroy": ([_P], ctypes.c_int),
    "hull_server_create": ([_SZ, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)],
                           ctypes.c_int),
    "hull_server_submit": ([_P, _P, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "hull_server_wait": ([_P, ctypes.c_uint64, _P, _I64], ctypes.c_int),
    "hull_server_stats": ([_P, _P], ctypes.c_int),
    "hull_server_destroy": ([_P], ctypes.c_int),
    "hull_session_create": ([_P, _P, _I64, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)],
                            ctypes.c_int),
    "hull_session_push": ([_P, _P, ctypes.c_int], ctypes.c_int),
    "hull_session_read": ([_P, _P, _P, _P, _P, _P, _P, ctypes.c_int], ctypes.c_int),
    "hull_session_reset": ([_P], ctypes.c_int),
    "hull_session_destroy": ([_P], ctypes.c_int),
}

_lib_handle = None


def lib():
    """The loaded HIP library. Raises if it has not been built: there is no
    other implementation to fall back to."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1402_1720_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        if L.hull_abi_version() != ABI_VERSION:
            raise ImportError(f"{LIB_PATH} has ABI version {L.hull_abi_version()}, this binding "
                              f"expects {ABI_VERSION}: rebuild it")
        _lib_handle = L
    return _lib_handle


class HullError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {hull_strerror(status)} (status {status})")


def _check(rc: int, where: str) -> None:
    if rc != HULL_OK:
        raise HullError(rc, where)


def hull_abi_version() -> int:
    return lib().hull_abi_version()


def hull_strerror(status: int) -> str:
    return lib().hull_strerror(int(status)).decode()


# ---------------------------------------------------------------------------
# marshalling helpers

def make_grid(g) -> hullmi_grid:
    """``hullmi_grid`` from a ``hullmi_grid`` or any object with ``n``, ``d`` and
    ``origin`` triples (lower corner of voxel (0,0,0))."""
    if isinstance(g, hullmi_grid):
        return g
    return hullmi_grid(int(g.n[0]), int(g.n[1]), int(g.n[2]), float(g.d[0]), float(g.d[1]),
                       float(g.d[2]), float(g.origin[0]), float(g.origin[1]), float(g.origin[2]))


def _voxels(g: hullmi_grid) -> int:
    return int(g.nx) * int(g.ny) * int(g.nz)


def _dev_ptr(t: Optional[torch.Tensor], dtype: torch.dtype, numel: Optional[int], name: str,
             device: Optional[torch.device] = None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must hold {numel} elements, got {t.numel()}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    return ctypes.c_void_p(t.data_ptr())


class Histories:
    """Eight FP32 device arrays of one length (SoA), as ``hullmi_histories``."""

    def __init__(self, arrays: Dict[str, torch.Tensor]):
        self.arrays = {k: arrays[k] for k in FIELDS}
        n = self.arrays["wepl"].numel()
        dev = self.arrays["wepl"].device
        ptrs = {k: _dev_ptr(v, torch.float32, n, k, dev) for k, v in self.arrays.items()}
        self.n = n
        self.device = dev
        self.c = hullmi_histories(*[ptrs[k].value if n else None for k in FIELDS], n)

    @classmethod
    def from_numpy(cls, arrays, device="cuda") -> "Histories":
        return cls({k: torch.from_numpy(arrays[k]).to(device) for k in FIELDS})

    def slice(self, a: int, b: int) -> "Histories":
        return Histories({k: v[a:b] for k, v in self.arrays.items()})


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def hull_workspace_bytes(op: int, grid, n: int, fbp: Optional[hullmi_fbp_params] = None) -> int:
    g = make_grid(grid)
    r = lib().hull_workspace_bytes(int(op), ctypes.byref(g), int(n),
                                   ctypes.byref(fbp) if fbp is not None else None)
    if r == ctypes.c_size_t(-1).value:
        raise HullError(HULL_EINVAL, "hull_workspace_bytes")
    return int(r)


def workspace(op: int, grid, n: int, device, fbp=None) -> Optional[torch.Tensor]:
    nbytes = hull_workspace_bytes(op, grid, n, fbp)
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device) if nbytes else None


def _ws(ws: Optional[torch.Tensor]):
    if ws is None:
        return None, 0
    return _dev_ptr(ws, torch.uint8, None, "ws"), ws.numel()


def _stats_ptr(stats):
    return _dev_ptr(stats, torch.int64, 6, "stats")


STATS_FIELDS = ("n_low", "n_high", "n_skipped", "n_missed_grid", "n_visits_low", "n_visits_high")


def stats_dict(stats: torch.Tensor) -> Dict[str, int]:
    v = stats.cpu().tolist()
    return dict(zip(STATS_FIELDS, (int(x) for x in v)))


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)

def hull_sc(hist: Histories, grid, wepl_low: float, N: torch.Tensor,
            mask: Optional[torch.Tensor] = None, flags: int = 0,
            stats: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None, stream=None):
    g = make_grid(grid)
    V = _voxels(g)
    if ws is None:
        ws = workspace(HULL_OP_SC, g, hist.n, hist.device)
    wp, wn = _ws(ws)
    rc = lib().hull_sc(ctypes.byref(hist.c), ctypes.byref(g), float(wepl_low),
                       _dev_ptr(N, torch.int32, V, "N", hist.device),
                       _dev_ptr(mask, torch.uint8, V, "mask", hist.device), int(flags),
                       _stats_ptr(stats), wp, wn, _stream(stream))
    _check(rc, "hull_sc")


def hull_msc(hist: Histories, grid, wepl_low: float, n_t: int, mode: int, nbr: int,
             N: torch.Tensor, mask: Optional[torch.Tensor] = None, flags: int = 0,
             stats: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None, stream=None):
    g = make_grid(grid)
    V = _voxels(g)
    if ws is None:
        ws = workspace(HULL_OP_MSC, g, hist.n, hist.device)
    wp, wn = _ws(ws)
    rc = lib().hull_msc(ctypes.byref(hist.c), ctypes.byref(g), float(wepl_low), int(n_t), int(mode),
                        int(nbr), _dev_ptr(N, torch.int32, V, "N", hist.device),
                        _dev_ptr(mask, torch.uint8, V, "mask", hist.device), int(flags),
                        _stats_ptr(stats), wp, wn, _stream(stream))
    _check(rc, "hull_msc")


def hull_sm(hist: Histories, grid, wepl_high: float, frac_num: int, frac_den: int, mode: int,
            scope: int, nbr: int, M: torch.Tensor, mask: Optional[torch.Tensor] = None,
            flags: int = 0, stats: Optional[torch.Tensor] = None,
            ws: Optional[torch.Tensor] = None, stream=None):
    g = make_grid(grid)
    V = _voxels(g)
    if ws is None:
        ws = workspace(HULL_OP_SM, g, hist.n, hist.device)
    wp, wn = _ws(ws)
    rc = lib().hull_sm(ctypes.byref(hist.c), ctypes.byref(g), float(wepl_high), int(frac_num),
                       int(frac_den), int(mode), int(scope), int(nbr),
                       _dev_ptr(M, torch.int32, V, "M", hist.device),
                       _dev_ptr(mask, torch.uint8, V, "mask", hist.device), int(flags),
                       _stats_ptr(stats), wp, wn, _stream(stream))
    _check(rc, "hull_sm")


def make_params(wepl_low=1.0, wepl_high=5.0, msc_n_t=5, msc_mode=HULL_MSC_COUNT, sm_frac_num=3,
                sm_frac_den=5, sm_mode=HULL_SM_FRACTION, sm_scope=HULL_SCOPE_VOLUME,
                nbr=HULL_NBR_INPLANE4) -> hullmi_params:
    return hullmi_params(wepl_low, wepl_high, msc_n_t, msc_mode, sm_frac_num, sm_frac_den, sm_mode,
                         sm_scope, nbr)


def hull_all(hist: Histories, grid, params: hullmi_params, N: torch.Tensor, M: torch.Tensor,
             sc_mask=None, msc_mask=None, sm_mask=None, flags: int = 0, stats=None, ws=None,
             stream=None):
    g = make_grid(grid)
    V = _voxels(g)
    if ws is None:
        ws = workspace(HULL_OP_ALL, g, hist.n, hist.device)
    wp, wn = _ws(ws)
    d = hist.device
    rc = lib().hull_all(ctypes.byref(hist.c), ctypes.byref(g), ctypes.byref(params),
                        _dev_ptr(N, torch.int32, V, "N", d), _dev_ptr(M, torch.int32, V, "M", d),
                        _dev_ptr(sc_mask, torch.uint8, V, "sc_mask", d),
                        _dev_ptr(msc_mask, torch.uint8, V, "msc_mask", d),
                        _dev_ptr(sm_mask, torch.uint8, V, "sm_mask", d), int(flags),
                        _stats_ptr(stats), wp, wn, _stream(stream))
    _check(rc, "hull_all")


# hull_prof_kernel entries: counting pass, then the FDK hull
PROF_KERNELS = ("classify", "scan", "plan", "scatter", "setup", "walk", "reduce", "overflow",
                "fbp_clear", "fbp_bin", "fbp_filter", "fbp_geometry", "fbp_backproject")
PROF_KERNEL_NAMES = ("k_bin_classify", "k_bin_scan_groups + k_bin_scan_sums", "k_bin_plan",
                     "k_bin_scatter",
                     "k_item_setup", "k_walk_tiles", "k_reduce_tiles", "k_walk_overflow",
                     "k_fill_u64 + k_fill_u32", "k_fbp_bin_lds", "k_fill_u32 + k_fbp_filter",
                     "k_fbp_trig + k_fbp_footprint", "k_fbp_backproject_tiles")


def _prof_result(ms, n, keys):
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(PROF_KERNELS) if k in keys}


def hull_count_profile(hist: Histories, grid, params: hullmi_params, N: torch.Tensor,
                       M: torch.Tensor, flags: int = 0, stats=None, ws=None, stream=None):
    """The counting pass of hull_all with an event pair around every kernel
    launch; waits for the stream and returns {kernel: (ms summed over its
    launches, launches)}."""
    g = make_grid(grid)
    V = _voxels(g)
    if ws is None:
        ws = workspace(HULL_OP_ALL, g, hist.n, hist.device)
    wp, wn = _ws(ws)
    d = hist.device
    K = len(PROF_KERNELS)
    ms = (ctypes.c_float * K)()
    n = (ctypes.c_int32 * K)()
    rc = lib().hull_count_profile(ctypes.byref(hist.c), ctypes.byref(g), ctypes.byref(params),
                                  _dev_ptr(N, torch.int32, V, "N", d),
                                  _dev_ptr(M, torch.int32, V, "M", d), int(flags),
                                  _stats_ptr(stats), wp, wn, _stream(stream), ms, n)
    _check(rc, "hull_count_profile")
    return _prof_result(ms, n, PROF_KERNELS[:8])


def hull_fbp_profile(hist: Histories, grid, fbp: "hullmi_fbp_params", image: torch.Tensor,
                     mask: Optional[torch.Tensor] = None, ws=None, stream=None):
    """hull_fbp with an event pair around every kernel launch; waits for the
    stream and returns {kernel: (ms summed over its launches, launches)}."""
    g = make_grid(grid)
    V = _voxels(g)
    if ws is None:
        ws = workspace(HULL_OP_FBP, g, hist.n, hist.device, fbp)
    wp, wn = _ws(ws)
    d = hist.device
    K = len(PROF_KERNELS)
    ms = (ctypes.c_float * K)()
    n = (ctypes.c_int32 * K)()
    rc = lib().hull_fbp_profile(ctypes.byref(hist.c), ctypes.byref(g), ctypes.byref(fbp),
                                _dev_ptr(image, torch.float32, V, "image", d),
                                _dev_ptr(mask, torch.uint8, V, "mask", d), wp, wn,
                                _stream(stream), ms, n)
    _check(rc, "hull_fbp_profile")
    return _prof_result(ms, n, PROF_KERNELS[8:])


def make_fbp_params(geo) -> hullmi_fbp_params:
    """``hullmi_fbp_params`` from an object with src_dist, du, dv, u0, v0, nu, nv,
    n_angles, angle0, dangle and threshold attributes."""
    return hullmi_fbp_params(geo.src_dist, geo.du, geo.dv, geo.u0, geo.v0, geo.nu, geo.nv,
                             geo.n_angles, geo.angle0, geo.dangle, 0, geo.threshold)


def hull_fbp(hist: Histories, grid, fbp: hullmi_fbp_params, image: torch.Tensor,
             mask: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None, stream=None):
    g = make_grid(grid)
    V = _voxels(g)
    if ws is None:
        ws = workspace(HULL_OP_FBP, g, hist.n, hist.device, fbp)
    wp, wn = _ws(ws)
    d = hist.device
    rc = lib().hull_fbp(ctypes.byref(hist.c), ctypes.byref(g), ctypes.byref(fbp),
                        _dev_ptr(image, torch.float32, V, "image", d),
                        _dev_ptr(mask, torch.uint8, V, "mask", d), wp, wn, _stream(stream))
    _check(rc, "hull_fbp")


NOALLOC_SCRATCH_BYTES = 256 << 20   # HULLMI_NOALLOC_SCRATCH_BYTES


def hull_fbp_noalloc(hist: Histories, grid, fbp: hullmi_fbp_params, image: torch.Tensor,
                     mask: Optional[torch.Tensor] = None, stream=None):
    """hull_fbp with its workspace in the library's fixed device array (no
    allocation in the call; calls overlapping on one device race)."""
    g = make_grid(grid)
    V = _voxels(g)
    d = hist.device
    rc = lib().hull_fbp_noalloc(ctypes.byref(hist.c), ctypes.byref(g), ctypes.byref(fbp),
                                _dev_ptr(image, torch.float32, V, "image", d),
                                _dev_ptr(mask, torch.uint8, V, "mask", d), _stream(stream))
    _check(rc, "hull_fbp_noalloc")


def hull_fbp_cut(hist: Histories, grid, fbp: hullmi_fbp_params, cut_sigmas: int,
                 image: torch.Tensor, mask: Optional[torch.Tensor] = None,
                 ws: Optional[torch.Tensor] = None, stream=None):
    g = make_grid(grid)
    V = _voxels(g)
    if ws is None:
        ws = workspace(HULL_OP_FBP_CUT, g, hist.n, hist.device, fbp)
    wp, wn = _ws(ws)
    d = hist.device
    rc = lib().hull_fbp_cut(ctypes.byref(hist.c), ctypes.byref(g), ctypes.byref(fbp),
                            int(cut_sigmas), _dev_ptr(image, torch.float32, V, "image", d),
                            _dev_ptr(mask, torch.uint8, V, "mask", d), wp, wn, _stream(stream))
    _check(rc, "hull_fbp_cut")


def make_bsc_params(wepl_low=1.0, cut_sigmas=3, window=5, thr_num=2, thr_den=5) -> hullmi_bsc_params:
    """Binned SC parameters; the defaults are the paper's (Sections 2.2, 3.2)."""
    return hullmi_bsc_params(wepl_low, cut_sigmas, window, thr_num, thr_den)


def bsc_stats_dict(stats: torch.Tensor) -> Dict[str, int]:
    return dict(zip(BSC_STATS_FIELDS, (int(x) for x in stats.cpu().tolist())))


def hull_sc_binned(hist: Histories, grid, bins: hullmi_fbp_params, params: hullmi_bsc_params,
                   mask: torch.Tensor, kept_n: Optional[torch.Tensor] = None,
                   kept_sum: Optional[torch.Tensor] = None, carved: Optional[torch.Tensor] = None,
                   stats: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
                   stream=None):
    g = make_grid(grid)
    V = _voxels(g)
    nb = int(bins.nu) * int(bins.nv) * int(bins.n_angles)
    if ws is None:
        ws = workspace(HULL_OP_SC_BINNED, g, hist.n, hist.device, bins)
    wp, wn = _ws(ws)
    d = hist.device
    # kept counts are uint32 in the ABI; below 2^31 (n < 2^31) they read alike as int32
    kn = _dev_ptr(kept_n, torch.int32, nb, "kept_n", d)
    rc = lib().hull_sc_binned(ctypes.byref(hist.c), ctypes.byref(g), ctypes.byref(bins),
                              ctypes.byref(params), kn,
                              _dev_ptr(kept_sum, torch.int64, nb, "kept_sum", d),
                              _dev_ptr(carved, torch.uint8, V, "carved", d),
                              _dev_ptr(mask, torch.uint8, V, "mask", d),
                              _dev_ptr(stats, torch.int64, 6, "stats", d), wp, wn, _stream(stream))
    _check(rc, "hull_sc_binned")


def hull_count_lines(q_in: torch.Tensor, q_out: torch.Tensor, grid, counts: torch.Tensor,
                     flags: int = 0, stats=None, ws=None, stream=None):
    g = make_grid(grid)
    n = q_in.numel() // 3
    if q_in.numel() != 3 * n or q_out.numel() != 3 * n:
        raise ValueError("q_in and q_out must be [n, 3]")
    d = counts.device
    wp, wn = _ws(ws)
    rc = lib().hull_count_lines(_dev_ptr(q_in, torch.int32, 3 * n, "q_in", d),
                                _dev_ptr(q_out, torch.int32, 3 * n, "q_out", d), n,
                                ctypes.byref(g), _dev_ptr(counts, torch.int32, _voxels(g), "counts", d),
                                int(flags), _stats_ptr(stats), wp, wn, _stream(stream))
    _check(rc, "hull_count_lines")


def hull_quantize(hist: Histories, grid, status: torch.Tensor, q_in: torch.Tensor,
                  q_out: torch.Tensor, stream=None):
    g = make_grid(grid)
    n = hist.n
    d = hist.device
    rc = lib().hull_quantize(ctypes.byref(hist.c), ctypes.byref(g),
                             _dev_ptr(status, torch.int32, n, "status", d),
                             _dev_ptr(q_in, torch.int32, 3 * n, "q_in", d),
                             _dev_ptr(q_out, torch.int32, 3 * n, "q_out", d), _stream(stream))
    _check(rc, "hull_quantize")


def hull_footprint_bytes(op: int, grid, n: int, fbp: Optional[hullmi_fbp_params] = None) -> int:
    g = make_grid(grid)
    r = lib().hull_footprint_bytes(int(op), ctypes.byref(g), int(n),
                                   ctypes.byref(fbp) if fbp is not None else None)
    if r == ctypes.c_size_t(-1).value:
        raise HullError(HULL_EINVAL, "hull_footprint_bytes")
    return int(r)


# ---------------------------------------------------------------------------
# batches

_OP_OUTPUTS = {
    HULL_OP_SC: ("N", "sc_mask"), HULL_OP_MSC: ("N", "msc_mask"), HULL_OP_SM: ("M", "sm_mask"),
    HULL_OP_ALL: ("N", "M", "sc_mask", "msc_mask", "sm_mask"), HULL_OP_FBP: ("image", "fbp_mask"),
    HULL_OP_FBP_CUT: ("image", "fbp_mask"), HULL_OP_SC_BINNED: ("bsc_mask",),
}
_OUT_DTYPES = {"N": torch.int32, "M": torch.int32, "sc_mask": torch.uint8,
               "msc_mask": torch.uint8, "sm_mask": torch.uint8, "image": torch.float32,
               "fbp_mask": torch.uint8, "bsc_mask": torch.uint8}


def make_job(op: int, hist: Histories, grid, params: Optional[hullmi_params] = None,
             fbp: Optional[hullmi_fbp_params] = None, flags: int = 0, stats=None,
             bsc: Optional[hullmi_bsc_params] = None, bsc_stats=None, **outputs) -> hullmi_job:
    """``hullmi_job`` for one scan; outputs are device tensors named as the
    struct fields (N, M, sc_mask, msc_mask, sm_mask, image, fbp_mask,
    bsc_mask). ``bsc`` defaults to the paper's binned SC parameters;
    ``bsc_stats`` is an int64[6] device tensor."""
    g = make_grid(grid)
    V = _voxels(g)
    j = hullmi_job()
    j.op, j.flags, j.hist, j.grid = int(op), int(flags), hist.c, g
    j.params = params if params is not None else make_params()
    j.bsc = bsc if bsc is not None else make_bsc_params()
    if fbp is not None:
        j.fbp = fbp
    bp = _dev_ptr(bsc_stats, torch.int64, 6, "bsc_stats", hist.device)
    j.bsc_stats = bp.value if bp is not None else None
    for k, t in outputs.items():
        if k not in _OUT_DTYPES:
            raise ValueError(f"unknown output {k}")
        p = _dev_ptr(t, _OUT_DTYPES[k], V, k, hist.device)
        setattr(j, k, p.value if p is not None else None)
    sp = _stats_ptr(stats)
    j.stats = sp.value if sp is not None else None
    return j


class BatchPlan:
    """``hull_batch_plan`` over jobs; keeps the tensors the jobs point to
    alive as long as the plan."""

    def __init__(self, jobs: Sequence[hullmi_job], keep=(), tuning: Optional[hullmi_tuning] = None):
        self._keep = list(keep)
        arr = (hullmi_job * max(1, len(jobs)))(*jobs)
        h = ctypes.c_void_p()
        rc = lib().hull_batch_plan(arr, len(jobs), ctypes.byref(tuning) if tuning else None,
                                   ctypes.byref(h))
        _check(rc, "hull_batch_plan")
        self._h = h

    @property
    def tuning(self) -> hullmi_tuning:
        t = hullmi_tuning()
        _check(lib().hull_batch_tuning(self._h, ctypes.byref(t)), "hull_batch_tuning")
        return t

    def launch(self, stream=None) -> None:
        _check(lib().hull_batch_launch(self._h, _stream(stream)), "hull_batch_launch")

    def close(self) -> None:
        if self._h:
            lib().hull_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# serving

def _host_ptr(a, dtype, numel, name):
    import numpy as np
    if a is None:
        return None
    if not isinstance(a, np.ndarray) or a.dtype != dtype or not a.flags["C_CONTIGUOUS"]:
        raise ValueError(f"{name} must be a C-contiguous numpy array of {dtype}")
    if numel is not None and a.size != numel:
        raise ValueError(f"{name} must hold {numel} elements, got {a.size}")
    return a.ctypes.data


class Server:
    """``hull_server_*``: host histories in, host masks out. Submitted arrays
    are kept alive until their ticket has been waited for."""

    def __init__(self, hbm_budget: int, max_slots: int = 4, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().hull_server_create(int(hbm_budget), int(max_slots), int(device),
                                        ctypes.byref(h)), "hull_server_create")
        self._h = h
        self._keep = {}

    def submit(self, op: int, hist: Dict[str, "np.ndarray"], grid,
               params: Optional[hullmi_params] = None, fbp: Optional[hullmi_fbp_params] = None,
               bsc: Optional[hullmi_bsc_params] = None, **outputs) -> int:
        """Queues one request; outputs are host numpy arrays named as the
        struct fields. Returns the ticket."""
        import numpy as np
        g = make_grid(grid)
        V = _voxels(g)
        n = int(hist["wepl"].size)
        r = hullmi_request()
        r.op, r.grid = int(op), g
        r.hist = hullmi_histories(*[_host_ptr(hist[k], np.float32, n, k) if n else None
                                    for k in FIELDS], n)
        r.params = params if params is not None else make_params()
        r.bsc = bsc if bsc is not None else make_bsc_params()
        if fbp is not None:
            r.fbp = fbp
        np_types = {torch.int32: np.int32, torch.uint8: np.uint8, torch.float32: np.float32}
        for k, a in outputs.items():
            if k not in _OUT_DTYPES:
                raise ValueError(f"unknown output {k}")
            setattr(r, k, _host_ptr(a, np_types[_OUT_DTYPES[k]], V, k))
        t = ctypes.c_uint64()
        _check(lib().hull_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)),
               "hull_server_submit")
        self._keep[t.value] = (hist, outputs)
        return t.value

    def wait(self, ticket: int, timeout_us: int = -1) -> Optional[Dict]:
        """Result of a ticket as a dict, or None on time-out."""
        res = hullmi_result()
        rc = lib().hull_server_wait(self._h, int(ticket), ctypes.byref(res), int(timeout_us))
        if rc == HULL_ETIMEDOUT:
            return None
        _check(rc, "hull_server_wait")
        self._keep.pop(int(ticket), None)
        out = {k: getattr(res, k) for k, _ in hullmi_result._fields_
               if k not in ("stats", "bsc_stats")}
        out["stats"] = {k: getattr(res.stats, k) for k, _ in hullmi_stats._fields_}
        out["bsc_stats"] = {k: getattr(res.bsc_stats, k) for k in BSC_STATS_FIELDS}
        return out

    def stats(self) -> Dict[str, int]:
        st = hullmi_server_stats()
        _check(lib().hull_server_stats(self._h, ctypes.byref(st)), "hull_server_stats")
        return {k: int(getattr(st, k)) for k, _ in hullmi_server_stats._fields_}

    def close(self) -> None:
        if self._h:
            lib().hull_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Session:
    """Online accumulation (``hull_session_*``): counts resident on the device,
    chunks pushed as they arrive, masks read on demand."""

    def __init__(self, grid, params: hullmi_params, max_chunk: int, device: int = 0):
        self.grid = make_grid(grid)
        self.V = _voxels(self.grid)
        self.params = params
        self.max_chunk = int(max_chunk)
        h = ctypes.c_void_p()
        _check(lib().hull_session_create(ctypes.byref(self.grid), ctypes.byref(params),
                                         self.max_chunk, int(device), ctypes.byref(h)),
               "hull_session_create")
        self._h = h

    def push(self, chunk) -> None:
        """``chunk``: a ``Histories`` (device) or a dict of eight host arrays
        (numpy float32, or CPU torch tensors, ideally pinned)."""
        if isinstance(chunk, Histories):
            _check(lib().hull_session_push(self._h, ctypes.byref(chunk.c), 0), "hull_session_push")
            return
        arrs = {}
        for k in FIELDS:
            a = chunk[k]
            if isinstance(a, torch.Tensor):
                if a.is_cuda or a.dtype != torch.float32 or not a.is_contiguous():
                    raise ValueError(f"{k}: host float32 contiguous tensor expected")
                arrs[k] = (a, a.data_ptr(), a.numel())
            else:
                import numpy as np
                a = np.ascontiguousarray(a, dtype=np.float32)
                arrs[k] = (a, a.ctypes.data, a.size)
        n = arrs["wepl"][2]
        if any(v[2] != n for v in arrs.values()):
            raise ValueError("chunk arrays differ in length")
        c = hullmi_histories(*[arrs[k][1] if n else None for k in FIELDS], n)
        _check(lib().hull_session_push(self._h, ctypes.byref(c), 1), "hull_session_push")

    def read(self, counts: bool = True, masks: bool = True) -> Dict[str, object]:
        """Host copies of N, M, the three masks and the counters so far."""
        import numpy as np
        V = self.V
        N = np.empty(V, np.int32) if counts else None
        M = np.empty(V, np.int32) if counts else None
        m = [np.empty(V, np.uint8) if masks else None for _ in range(3)]
        st = hullmi_stats()
        p = lambda a: None if a is None else ctypes.c_void_p(a.ctypes.data)
        _check(lib().hull_session_read(self._h, p(N), p(M), p(m[0]), p(m[1]), p(m[2]),
                                       ctypes.byref(st), 1), "hull_session_read")
        return dict(N=N, M=M, sc=m[0], msc=m[1], sm=m[2],
                    stats={k: int(getattr(st, k)) for k in STATS_FIELDS})

    def reset(self) -> None:
        _check(lib().hull_session_reset(self._h), "hull_session_reset")

    def close(self) -> None:
        if self._h:
            lib().hull_session_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
