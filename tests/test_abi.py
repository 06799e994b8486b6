"""Host-only checks of the C ABI library: it loads, exports every symbol the
header declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_1402_1720_amd import hullmi as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hullmi.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hull_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported_and_bound():
    L = H.lib()
    syms = declared_symbols()
    assert len(syms) >= 10
    for s in syms:
        assert hasattr(L, s), s
        assert s in H.SIGNATURES, f"binding lacks {s}"


def test_version_and_strerror():
    assert H.hull_abi_version() == H.ABI_VERSION == 3
    assert H.hull_strerror(H.HULL_OK) == "ok"
    assert H.hull_strerror(H.HULL_EINVAL) == "invalid argument"
    assert H.hull_strerror(12345) == "unknown status"


def _grid(nx=8, ny=8, nz=4, d=1.0):
    return H.hullmi_grid(nx, ny, nz, d, d, d, -4.0, -4.0, -2.0)


def test_workspace_sizes():
    g = _grid()
    assert H.hull_workspace_bytes(H.HULL_OP_COUNT_LINES, g, 100) == 0
    sc = H.hull_workspace_bytes(H.HULL_OP_SC, g, 100)
    assert sc > 100 * 24                       # quantised endpoints at least
    assert H.hull_workspace_bytes(H.HULL_OP_MSC, g, 100) == sc
    assert H.hull_workspace_bytes(H.HULL_OP_ALL, g, 100) >= sc + 8 * 4
    # up to 2^26 histories, one internal batch of all of them
    big = H.hull_workspace_bytes(H.HULL_OP_SC, g, 2 ** 26)
    assert H.hull_workspace_bytes(H.HULL_OP_SC, g, 2 ** 26 - 2 ** 16) < big
    # above, two halves, each for a batch of n / k histories in whole blocks of
    # 8192, k the smallest even number of batches of at most 2^25
    def half(b):
        return (H.hull_workspace_bytes(H.HULL_OP_SC, g, b) + 255) // 256 * 256
    assert H.hull_workspace_bytes(H.HULL_OP_SC, g, 2 ** 31 - 1) == 2 * half(2 ** 25) + 256   # k = 64
    assert H.hull_workspace_bytes(H.HULL_OP_SC, g, 3 * 2 ** 25) == 2 * half(3 * 2 ** 23) + 256   # k = 4
    assert H.hull_workspace_bytes(H.HULL_OP_SC, g, 2 ** 26 + 1) == 2 * half(2 ** 24 + 8192) + 256   # k = 4
    assert H.hull_workspace_bytes(H.HULL_OP_SC, g, 2 ** 31 - 1) < 2 * big
    f = H.hullmi_fbp_params(2000.0, 1.0, 5.0, -150.0, -55.0, 300, 22, 180, 0.0, 2.0, 0, 0.6)
    nb = 300 * 22 * 180
    assert H.hull_workspace_bytes(H.HULL_OP_FBP, g, 100, f) >= nb * 16
    with pytest.raises(H.HullError):
        H.hull_workspace_bytes(H.HULL_OP_FBP, g, 100, None)
    with pytest.raises(H.HullError):
        H.hull_workspace_bytes(99, g, 100)
    with pytest.raises(H.HullError):
        H.hull_workspace_bytes(H.HULL_OP_SC, _grid(nx=0), 100)


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first


def _hist(n=10, null=None):
    ptrs = [None if k == null else FAKE.value for k in H.FIELDS]
    return H.hullmi_histories(*ptrs, n)


@pytest.mark.parametrize("case", ["neg_n", "big_n", "null_field", "bad_grid", "big_axis",
                                  "nan_voxel", "nan_thr", "null_out"])
def test_sc_rejects_bad_arguments(case):
    L = H.lib()
    h, g, thr, N = _hist(), _grid(), 1.0, FAKE
    if case == "neg_n":
        h = _hist(-1)
    elif case == "big_n":
        h = _hist(2 ** 31)
    elif case == "null_field":
        h = _hist(null="angle_deg")
    elif case == "bad_grid":
        g = _grid(nz=0)
    elif case == "big_axis":
        g = _grid(nx=4096)
    elif case == "nan_voxel":
        g = _grid(d=float("nan"))
    elif case == "nan_thr":
        thr = float("inf")
    elif case == "null_out":
        N = None
    rc = L.hull_sc(ctypes.byref(h), ctypes.byref(g), thr, N, None, 0, None, FAKE, 1 << 40, None)
    assert rc == H.HULL_EINVAL


def test_mode_and_threshold_checks():
    L = H.lib()
    h, g = _hist(), _grid()
    args = lambda nt, mode, nbr: (ctypes.byref(h), ctypes.byref(g), 1.0, nt, mode, nbr, FAKE, FAKE,
                                  0, None, FAKE, 1 << 40, None)
    assert L.hull_msc(*args(0, 0, 0)) == H.HULL_EINVAL
    assert L.hull_msc(*args(5, 7, 0)) == H.HULL_EINVAL
    assert L.hull_msc(*args(5, 0, 3)) == H.HULL_EINVAL
    smargs = lambda num, den, mode, scope, ws, wsn: (
        ctypes.byref(h), ctypes.byref(g), 5.0, num, den, mode, scope, 0, FAKE, FAKE, 0, None, ws,
        wsn, None)
    assert L.hull_sm(*smargs(3, 0, 0, 0, FAKE, 1 << 20)) == H.HULL_EINVAL
    assert L.hull_sm(*smargs(-1, 5, 0, 0, FAKE, 1 << 20)) == H.HULL_EINVAL
    assert L.hull_sm(*smargs(3, 5, 2, 0, FAKE, 1 << 20)) == H.HULL_EINVAL
    assert L.hull_sm(*smargs(3, 5, 0, 2, FAKE, 1 << 20)) == H.HULL_EINVAL
    # a mask needs the workspace
    assert L.hull_sm(*smargs(3, 5, 0, 0, None, 0)) == H.HULL_ENOMEM
    assert L.hull_sm(*smargs(3, 5, 0, 0, FAKE, 64)) == H.HULL_ENOMEM
    sc_args = (ctypes.byref(h), ctypes.byref(g), 1.0, FAKE, None, 0, None, FAKE, 64, None)
    assert L.hull_sc(*sc_args) == H.HULL_ENOMEM
    # the counting ops run in any workspace down to that of a 2^16-history
    # batch: one byte less is refused before anything is enqueued
    big = _hist(n=1_000_000)
    least = H.hull_workspace_bytes(H.HULL_OP_SC, g, 1 << 16)
    assert least < H.hull_workspace_bytes(H.HULL_OP_SC, g, big.n)
    assert L.hull_sc(ctypes.byref(big), ctypes.byref(g), 1.0, FAKE, None, 0, None, FAKE, least - 1,
                     None) == H.HULL_ENOMEM
    rules = H.hull_workspace_bytes(H.HULL_OP_SM, g, 1 << 16) - least
    assert L.hull_sm(ctypes.byref(big), ctypes.byref(g), 5.0, 3, 5, 0, 0, 0, FAKE, FAKE, 0, None,
                     FAKE, rules + least - 1, None) == H.HULL_ENOMEM
    f = H.hullmi_fbp_params(2000.0, 1.0, 5.0, -150.0, -55.0, 300, 22, 180, 0.0, 2.0, 0, 0.6)
    assert L.hull_fbp(ctypes.byref(h), ctypes.byref(g), ctypes.byref(f), FAKE, None, FAKE, 16,
                      None) == H.HULL_ENOMEM
    f.filter = 3
    assert L.hull_fbp(ctypes.byref(h), ctypes.byref(g), ctypes.byref(f), FAKE, None, FAKE, 1 << 30,
                      None) == H.HULL_EINVAL


def test_binding_checks_tensors_before_calling():
    import torch
    with pytest.raises(ValueError):
        H.Histories({k: torch.zeros(4) for k in H.FIELDS})   # host tensors


def test_footprint_counts_inputs_outputs_and_workspace():
    g = _grid()
    V = 8 * 8 * 4
    n = 1000
    al = lambda b: (b + 255) // 256 * 256
    for op, outs in ((H.HULL_OP_SC, [4 * V, V]), (H.HULL_OP_MSC, [4 * V, V]),
                     (H.HULL_OP_SM, [4 * V, V]), (H.HULL_OP_ALL, [4 * V, 4 * V, V, V, V])):
        ws = H.hull_workspace_bytes(op, g, n)
        # two counter blocks of 48 bytes: the counting ops' and the binned SC's
        want = 8 * al(4 * n) + sum(al(b) for b in outs) + 2 * al(48) + al(ws)
        assert H.hull_footprint_bytes(op, g, n) == want, op
    f = H.hullmi_fbp_params(2000.0, 1.0, 5.0, -150.0, -55.0, 300, 22, 180, 0.0, 2.0, 0, 0.6)
    for op, outs in ((H.HULL_OP_FBP, [4 * V, V]), (H.HULL_OP_FBP_CUT, [4 * V, V]),
                     (H.HULL_OP_SC_BINNED, [V])):
        ws = H.hull_workspace_bytes(op, g, n, f)
        want = 8 * al(4 * n) + sum(al(b) for b in outs) + 2 * al(48) + al(ws)
        assert H.hull_footprint_bytes(op, g, n, f) == want, op
    for bad in ((H.HULL_OP_COUNT_LINES, g, n), (H.HULL_OP_SC, g, -1), (H.HULL_OP_SC, g, 2 ** 31),
                (H.HULL_OP_SC, _grid(ny=0), n), (H.HULL_OP_FBP, g, n), (H.HULL_OP_FBP_CUT, g, n),
                (H.HULL_OP_SC_BINNED, g, n), (8, g, n)):
        with pytest.raises(H.HullError):
            H.hull_footprint_bytes(*bad)


def _bins(src=2000.0):
    return H.hullmi_fbp_params(src, 1.0, 5.0, -150.0, -55.0, 300, 22, 180, 0.0, 2.0, 0, 0.6)


def _job(at=0, **kw):
    """A job whose fake device pointers lie at their own addresses (`at`
    selects a 16 MiB window), so that jobs made with different `at` values
    share no memory."""
    base = FAKE.value + at * (16 << 20)
    j = H.hullmi_job()
    j.op = H.HULL_OP_SC
    j.hist = H.hullmi_histories(*[base + k * (1 << 20) for k in range(8)], 10)
    j.grid = _grid()
    j.params = H.make_params()
    j.N = base + 8 * (1 << 20)
    for k, v in kw.items():
        setattr(j, k, v)
    return j


def test_batch_plan_rejects_bad_jobs_before_touching_the_device():
    L = H.lib()
    out = ctypes.c_void_p()
    assert L.hull_batch_plan(None, 1, None, ctypes.byref(out)) == H.HULL_EINVAL
    assert L.hull_batch_plan(None, -1, None, ctypes.byref(out)) == H.HULL_EINVAL
    jobs = (H.hullmi_job * 2)(_job(0), _job(1))
    assert L.hull_batch_plan(jobs, 2, None, None) == H.HULL_EINVAL
    bad = [_job(N=None), _job(op=9), _job(op=H.HULL_OP_SM), _job(grid=_grid(nx=0)),
           _job(hist=_hist(null="wepl")), _job(op=H.HULL_OP_MSC, params=H.make_params(msc_n_t=0)),
           _job(op=H.HULL_OP_FBP, image=FAKE.value),
           # binned SC and FDK after cuts: bad bins, a missing output, bad parameters
           _job(op=H.HULL_OP_SC_BINNED, fbp=_bins(), bsc=H.make_bsc_params()),
           _job(op=H.HULL_OP_SC_BINNED, fbp=_bins(src=0.0), bsc_mask=FAKE.value,
                bsc=H.make_bsc_params()),
           _job(op=H.HULL_OP_SC_BINNED, fbp=_bins(), bsc_mask=FAKE.value,
                bsc=H.make_bsc_params(window=4)),
           _job(op=H.HULL_OP_FBP_CUT, fbp=_bins(), bsc=H.make_bsc_params()),
           _job(op=H.HULL_OP_FBP_CUT, fbp=_bins(), image=FAKE.value,
                bsc=H.make_bsc_params(cut_sigmas=65))]
    for b in bad:
        arr = (H.hullmi_job * 2)(_job(1), b)
        assert L.hull_batch_plan(arr, 2, None, ctypes.byref(out)) == H.HULL_EINVAL
        assert out.value is None
    # bad tuning
    for t in (H.hullmi_tuning(0, 1, 0), H.hullmi_tuning(17, 1, 0), H.hullmi_tuning(2, 2, 0),
              H.hullmi_tuning(2, 1, -1), H.hullmi_tuning(2, 1, 0, -1), H.hullmi_tuning(2, 1, 0, 65),
              H.hullmi_tuning(2, 1, 0, 2, 17), H.hullmi_tuning(2, 1, 0, 2, -1),
              H.hullmi_tuning(2, 1, 0, 2, 8, 257), H.hullmi_tuning(2, 1, 0, 2, 8, -1)):
        assert L.hull_batch_plan(jobs, 2, ctypes.byref(t), ctypes.byref(out)) == H.HULL_EINVAL
    assert L.hull_batch_launch(None, None) == H.HULL_EINVAL
    assert L.hull_batch_tuning(None, None) == H.HULL_EINVAL
    assert L.hull_batch_destroy(None) == H.HULL_OK


def test_profile_calls_reject_bad_arguments():
    L = H.lib()
    ms = (ctypes.c_float * 13)()
    n = (ctypes.c_int32 * 13)()
    p = H.make_params()
    g = _grid()
    f = _bins()
    # no place for the timings; a bad grid; a missing output; a short workspace
    assert L.hull_count_profile(ctypes.byref(_hist()), ctypes.byref(g), ctypes.byref(p), FAKE,
                                FAKE, 0, None, FAKE, 1 << 30, None, None, n) == H.HULL_EINVAL
    assert L.hull_count_profile(ctypes.byref(_hist()), ctypes.byref(_grid(nx=0)), ctypes.byref(p),
                                FAKE, FAKE, 0, None, FAKE, 1 << 30, None, ms, n) == H.HULL_EINVAL
    assert L.hull_count_profile(ctypes.byref(_hist()), ctypes.byref(g), ctypes.byref(p), FAKE,
                                None, 0, None, FAKE, 1 << 30, None, ms, n) == H.HULL_EINVAL
    assert L.hull_count_profile(ctypes.byref(_hist()), ctypes.byref(g), ctypes.byref(p), FAKE,
                                FAKE, 0, None, FAKE, 16, None, ms, n) == H.HULL_ENOMEM
    assert L.hull_fbp_profile(ctypes.byref(_hist()), ctypes.byref(g), ctypes.byref(f), FAKE, None,
                              FAKE, 1 << 30, None, None, n) == H.HULL_EINVAL
    assert L.hull_fbp_profile(ctypes.byref(_hist()), ctypes.byref(g), None, FAKE, None,
                              FAKE, 1 << 30, None, ms, n) == H.HULL_EINVAL
    assert L.hull_fbp_profile(ctypes.byref(_hist()), ctypes.byref(g), ctypes.byref(f), FAKE, None,
                              FAKE, 16, None, ms, n) == H.HULL_ENOMEM


def test_noalloc_fbp_rejects_bad_arguments_and_oversized_geometry():
    """hull_fbp_noalloc checks its arguments as hull_fbp does, and refuses a
    detector whose workspace exceeds the library's fixed array, before it
    touches the device."""
    L = H.lib()
    g = _grid()
    f = _bins()
    assert L.hull_fbp_noalloc(None, ctypes.byref(g), ctypes.byref(f), FAKE, None, None) == H.HULL_EINVAL
    assert L.hull_fbp_noalloc(ctypes.byref(_hist()), ctypes.byref(g), ctypes.byref(f), None, None,
                              None) == H.HULL_EINVAL
    assert L.hull_fbp_noalloc(ctypes.byref(_hist()), ctypes.byref(_grid(nx=0)), ctypes.byref(f),
                              FAKE, None, None) == H.HULL_EINVAL
    assert L.hull_fbp_noalloc(ctypes.byref(_hist()), ctypes.byref(g), None, FAKE, None,
                              None) == H.HULL_EINVAL
    big = H.hullmi_fbp_params(2000.0, 0.1, 0.1, -100.0, -50.0, 2000, 1000, 360, 0.0, 1.0, 0, 0.6)
    assert H.hull_workspace_bytes(H.HULL_OP_FBP, g, 10, big) > H.NOALLOC_SCRATCH_BYTES
    assert L.hull_fbp_noalloc(ctypes.byref(_hist()), ctypes.byref(g), ctypes.byref(big), FAKE,
                              None, None) == H.HULL_EINVAL


def test_batch_plan_rejects_jobs_that_would_race():
    """The jobs of a plan run on several streams: two jobs writing the same
    counts (for example chunks of one scan accumulating into one volume), a
    job writing another's histories, or overlapping masks or counters are
    refused before anything touches the device. The byte-range check itself
    is also covered host-side in tests/host/runtime_host_check.cpp."""
    L = H.lib()
    out = ctypes.c_void_p()
    V = 8 * 8 * 4
    a = _job(0)
    racing = [
        _job(1, N=a.N, flags=H.HULL_ACCUMULATE),               # the same N
        _job(1, N=a.N + 4 * V - 4),                             # its last word
        _job(1, N=a.hist.wepl),                                 # writes a's WEPL
        _job(1, op=H.HULL_OP_ALL, M=a.N, N=FAKE.value + (40 << 20)),
        _job(1, sc_mask=a.N + 100),                             # mask inside a's N
    ]
    for b in racing:
        arr = (H.hullmi_job * 2)(a, b)
        assert L.hull_batch_plan(arr, 2, None, ctypes.byref(out)) == H.HULL_EINVAL
        assert out.value is None
    # the same tuning is valid; only the overlap makes it fail
    t = H.hullmi_tuning(2, 1, 0)
    arr = (H.hullmi_job * 2)(a, _job(1, N=a.N))
    assert L.hull_batch_plan(arr, 2, ctypes.byref(t), ctypes.byref(out)) == H.HULL_EINVAL


def test_server_argument_checks():
    L = H.lib()
    out = ctypes.c_void_p()
    assert L.hull_server_create(0, 4, 0, ctypes.byref(out)) == H.HULL_EINVAL
    assert L.hull_server_create(1 << 30, 0, 0, ctypes.byref(out)) == H.HULL_EINVAL
    assert L.hull_server_create(1 << 30, 65, 0, ctypes.byref(out)) == H.HULL_EINVAL
    assert L.hull_server_create(1 << 30, 4, -1, ctypes.byref(out)) == H.HULL_EINVAL
    assert L.hull_server_create(1 << 30, 4, 0, None) == H.HULL_EINVAL
    t = ctypes.c_uint64()
    r = H.hullmi_request()
    assert L.hull_server_submit(None, ctypes.byref(r), ctypes.byref(t)) == H.HULL_EINVAL
    assert L.hull_server_wait(None, 1, None, 0) == H.HULL_EINVAL
    assert L.hull_server_stats(None, None) == H.HULL_EINVAL
    assert L.hull_server_destroy(None) == H.HULL_OK


def test_binned_sc_workspace_and_argument_checks():
    L = H.lib()
    g = _grid()
    f = H.hullmi_fbp_params(2000.0, 1.0, 5.0, -150.0, -55.0, 300, 22, 180, 0.0, 2.0, 0, 0.6)
    nb = 300 * 22 * 180
    ws = H.hull_workspace_bytes(H.HULL_OP_SC_BINNED, g, 1024, f)
    # records, per-bin sums, ranges, kept sums, carve list, the carved bits
    assert ws >= 8 * 1024 + nb * (4 + 8 + 8 + 8 + 8 + 4 + 8 + 4) + 8 * 8 * 4 // 8
    assert H.hull_workspace_bytes(H.HULL_OP_SC_BINNED, g, 2048, f) - ws == 8 * 1024
    with pytest.raises(H.HullError):
        H.hull_workspace_bytes(H.HULL_OP_SC_BINNED, g, 100, None)
    h = _hist()
    good = H.make_bsc_params()

    def call(p=good, mask=FAKE, wsn=1 << 40, hist=h, bins=f):
        return L.hull_sc_binned(ctypes.byref(hist), ctypes.byref(g), ctypes.byref(bins),
                                ctypes.byref(p), None, None, None, mask, None, FAKE, wsn, None)

    assert call(wsn=H.hull_workspace_bytes(H.HULL_OP_SC_BINNED, g, 10, f) - 1) == H.HULL_ENOMEM
    assert call(mask=None) == H.HULL_EINVAL
    for bad in (H.make_bsc_params(window=4), H.make_bsc_params(window=33),
                H.make_bsc_params(thr_den=0), H.make_bsc_params(thr_num=-1),
                H.make_bsc_params(cut_sigmas=-1), H.make_bsc_params(cut_sigmas=65),
                H.make_bsc_params(wepl_low=float("nan")), H.make_bsc_params(wepl_low=65536.0)):
        assert call(p=bad) == H.HULL_EINVAL
    assert call(hist=_hist(-1)) == H.HULL_EINVAL
    bad_bins = H.hullmi_fbp_params(0.0, 1.0, 5.0, -150.0, -55.0, 300, 22, 180, 0.0, 2.0, 0, 0.6)
    assert call(bins=bad_bins) == H.HULL_EINVAL


def test_fbp_cut_workspace_and_argument_checks():
    L = H.lib()
    g = _grid()
    f = H.hullmi_fbp_params(2000.0, 1.0, 5.0, -150.0, -55.0, 300, 22, 180, 0.0, 2.0, 0, 0.6)
    ws = H.hull_workspace_bytes(H.HULL_OP_FBP_CUT, g, 1024, f)
    assert ws >= H.hull_workspace_bytes(H.HULL_OP_FBP, g, 1024, f) + 8 * 1024
    h = _hist()

    def call(k=3, image=FAKE, wsn=1 << 40):
        return L.hull_fbp_cut(ctypes.byref(h), ctypes.byref(g), ctypes.byref(f), k, image, None,
                              FAKE, wsn, None)

    assert call(k=-1) == H.HULL_EINVAL and call(k=65) == H.HULL_EINVAL
    assert call(image=None) == H.HULL_EINVAL
    assert call(wsn=H.hull_workspace_bytes(H.HULL_OP_FBP_CUT, g, 10, f) - 1) == H.HULL_ENOMEM


def test_session_argument_checks():
    L = H.lib()
    g, p = _grid(), H.make_params()
    out = ctypes.c_void_p()
    assert L.hull_session_create(ctypes.byref(g), ctypes.byref(p), 1000, 0, None) == H.HULL_EINVAL
    assert L.hull_session_create(ctypes.byref(_grid(nx=0)), ctypes.byref(p), 1000, 0,
                                 ctypes.byref(out)) == H.HULL_EINVAL
    assert L.hull_session_create(ctypes.byref(g), ctypes.byref(p), 0, 0,
                                 ctypes.byref(out)) == H.HULL_EINVAL
    bad = H.make_params(msc_n_t=0)
    assert L.hull_session_create(ctypes.byref(g), ctypes.byref(bad), 1000, 0,
                                 ctypes.byref(out)) == H.HULL_EINVAL
    assert not out.value
    h = _hist()
    assert L.hull_session_push(None, ctypes.byref(h), 1) == H.HULL_EINVAL
    assert L.hull_session_read(None, None, None, None, None, None, None, 1) == H.HULL_EINVAL
    assert L.hull_session_reset(None) == H.HULL_EINVAL
    assert L.hull_session_destroy(None) == H.HULL_EINVAL


def test_library_resolves_every_symbol_at_load():
    """Loading with RTLD_NOW fails on any symbol the library uses but does not
    define (a kernel declared in one namespace and defined in another links
    into a shared library and only fails when called)."""
    ctypes.CDLL(H.LIB_PATH, mode=os.RTLD_NOW | os.RTLD_LOCAL)
