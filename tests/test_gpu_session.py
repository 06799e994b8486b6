"""GPU parity of online accumulation (sessions): after every push the counts,
masks and counters equal the oracle's for all histories pushed so far; host
and device chunks, uneven and empty chunks, reset and independent sessions."""
import sys

import numpy as np
import pytest
import torch

import gen
import oracle
from paper_1402_1720_amd import hullmi as H

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def expect(h, grid, params):
    G = oracle.grid_of(grid)
    N, M, st = oracle.counts(h, G, params.wepl_low, params.wepl_high)
    return dict(N=N, M=M, sc=oracle.sc(N), msc=oracle.msc(N, G, params.msc_n_t, params.msc_mode,
                                                          params.nbr),
                sm=oracle.sm(M, G, params.sm_frac_num, params.sm_frac_den, params.sm_mode,
                             params.sm_scope, params.nbr)[0], stats=st)


def check(got, exp, what):
    for k in ("N", "M", "sc", "msc", "sm"):
        assert np.array_equal(got[k], exp[k]), (what, k)
    assert got["stats"] == exp["stats"], (what, got["stats"], exp["stats"])


def test_config2_scan_pushed_angle_by_angle():
    """The 200x200x32 scan as it is acquired: one host chunk per gantry angle
    (180 of about 55,600 histories); reads after the first angle, half way
    and at the end."""
    spec = gen.config_spec(2)
    h = gen.generate(spec)
    params = H.make_params()
    n = spec.n_hist
    edges = [(k * n) // spec.n_angles for k in range(spec.n_angles + 1)]
    s = H.Session(spec.grid, params, max_chunk=max(np.diff(edges)))
    try:
        for k in range(spec.n_angles):
            s.push({f: h[f][edges[k]:edges[k + 1]] for f in gen.FIELDS})
            if k + 1 in (1, 90, 180):
                say("read after angle", k + 1)
                pre = {f: h[f][:edges[k + 1]] for f in gen.FIELDS}
                check(s.read(), expect(pre, spec.grid, params), f"after {k + 1} angles")
    finally:
        s.close()


def test_host_and_device_chunks_uneven_empty_reset():
    spec = gen.config_spec(1, n_hist=200_000)
    h = gen.generate(spec)
    h = {k: v.copy() for k, v in h.items()}
    h["wepl"] += np.random.default_rng(4).normal(0, 4.0, h["wepl"].size).astype(np.float32)
    params = H.make_params(msc_mode=H.HULL_MSC_NEIGHBOR_DIFF, msc_n_t=50,
                           sm_mode=H.HULL_SM_MAX_SLOPE, sm_scope=H.HULL_SCOPE_SLICE)
    cuts = [0, 1, 1, 4097, 60_000, 60_000, 123_457, 190_000, 200_000]
    s = H.Session(spec.grid, params, max_chunk=70_000)
    try:
        for rep in range(2):
            for i, (a, b) in enumerate(zip(cuts[:-1], cuts[1:])):
                part = {f: h[f][a:b] for f in gen.FIELDS}
                if i % 3 == 1:     # device arrays: one append kernel
                    part = H.Histories.from_numpy(part, DEV)
                elif i % 3 == 2:   # pinned host arrays: the kernel reads them over PCIe
                    part = {f: torch.from_numpy(v.copy()).pin_memory() for f, v in part.items()}
                s.push(part)       # else pageable host arrays: copies
            check(s.read(), expect(h, spec.grid, params), f"pass {rep}")
            s.reset()
        got = s.read()
        assert not got["N"].any() and not got["M"].any() and got["sc"].all()
        with pytest.raises(H.HullError):
            s.push({f: h[f][:70_001] for f in gen.FIELDS})
    finally:
        s.close()


def test_sessions_are_independent():
    spec = gen.config_spec(1, n_hist=100_000)
    h = gen.generate(spec)
    params = H.make_params()
    a = H.Session(spec.grid, params, max_chunk=25_000)
    b = H.Session(spec.grid, params, max_chunk=25_000)
    try:
        for k in range(4):
            part = {f: h[f][k * 25_000:(k + 1) * 25_000] for f in gen.FIELDS}
            a.push(part)
            if k < 2:
                b.push(part)
        check(a.read(), expect(h, spec.grid, params), "a")
        check(b.read(), expect({f: h[f][:50_000] for f in gen.FIELDS}, spec.grid, params), "b")
    finally:
        a.close()
        b.close()
