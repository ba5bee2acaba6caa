"""Property-based checks of the C ABI's argument validation on a host-only context (no
device): random geometries, precisions, flags, step counts, widths and slice lists.  Every
call returns one of the documented status codes, a call that passes validation reports
TL_ERR_DEVICE (it would need a device), no plan is returned, and the process survives.
Host arrays always hold the number of entries their counts say (the interface cannot check
that); device pointers are never dereferenced by a host-only context."""
import ctypes
import math

import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

from paper_2301_05518_amd import _lib

CODES = {0, -1, -2, -3, -4, -5, -6, -7}
FAKE_W, FAKE_PSI = 0x10000, 0x4000000

extent = st.one_of(st.integers(-3, 70), st.sampled_from([0, 1, 2, 4, 4095, 4096, 1 << 20, -(1 << 30)]))
prec = st.one_of(st.integers(-2, 64), st.sampled_from([0, 1, 2, 3, 16, 17, 18, 19, 32, 33, 48, 51]))
sigma = st.one_of(st.floats(-2.0, 80.0), st.sampled_from([0.0, float("nan"), float("inf"), -0.0]))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


@pytest.fixture(scope="module")
def hctx(lib):
    h = ctypes.c_void_p()
    assert lib.tl_create(ctypes.byref(h), -1, None) == 0
    yield h
    assert lib.tl_destroy(h) == 0


def geom(L):
    g = _lib.Geom()
    for i, v in enumerate(L):
        g.L[i] = v
    return g


job_spec = st.tuples(st.tuples(extent, extent, extent, extent),          # geometry
                     st.lists(st.integers(-2, 9), max_size=6),            # t_of_rhs
                     st.one_of(st.none(), st.lists(st.integers(-2, 9), max_size=4)))   # w_slices


def make_jobs(specs):
    jobs = (_lib.Job * max(len(specs), 1))()
    keep = []
    for j, (L, ts, ws) in enumerate(specs):
        jobs[j].g = geom(L)
        jobs[j].W = FAKE_W
        jobs[j].psi = FAKE_PSI + 0x1000000 * j
        arr = (ctypes.c_int32 * max(len(ts), 1))(*ts)
        jobs[j].n_rhs = len(ts)
        jobs[j].t_of_rhs = arr
        keep.append(arr)
        if ws is not None:
            w = (ctypes.c_int32 * max(len(ws), 1))(*ws)
            jobs[j].w_slices = w
            jobs[j].n_w_slices = len(ws)
            keep.append(w)
    return jobs, keep


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(specs=st.lists(job_spec, min_size=0, max_size=3), n_steps=st.integers(-3, 200), sig=sigma, p=prec,
       flags=st.integers(0, 40))
def test_plan_and_smear_validation(lib, hctx, specs, n_steps, sig, p, flags):
    jobs, keep = make_jobs(specs)
    out = ctypes.c_void_p()
    rc = lib.tl_plan_create(hctx, jobs, len(specs), n_steps, ctypes.c_double(sig), p, flags, ctypes.byref(out))
    assert rc in CODES and rc != 0 and out.value is None
    if not math.isfinite(sig) or n_steps < 0 or not specs or flags >= 16:
        assert rc in (-1, -2, -3)   # refused by validation (which check fires first may vary)
    rc2 = lib.tl_smear(hctx, jobs, len(specs), n_steps, ctypes.c_double(sig), p, flags)
    assert rc2 == rc
    assert lib.tl_last_error(hctx) is not None


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(L=st.tuples(extent, extent, extent, extent), p=prec, slices=st.one_of(st.none(), st.lists(st.integers(-2, 9), max_size=5)),
       t=st.integers(-2, 9))
def test_build_and_laplacian_validation(lib, hctx, L, p, slices, t):
    g = geom(L)
    arr = (ctypes.c_int32 * max(len(slices or []), 1))(*(slices or []))
    n = len(slices) if slices is not None else 0
    ptr = arr if slices is not None else None
    ok_geom = lib.tl_check_geom(ctypes.byref(g))
    assert ok_geom in (0, -2)
    nbytes = lib.tl_twolinks_bytes(ctypes.byref(g), p, max(n, 1))
    assert nbytes >= 0
    if ok_geom != 0:
        assert nbytes == 0
    rc = lib.tl_build_twolinks(hctx, ctypes.byref(g), ctypes.c_void_p(FAKE_W), ptr, n, p, ctypes.c_void_p(FAKE_PSI))
    assert rc in CODES and rc != 0
    if ok_geom != 0:
        assert rc in (-2, -1, -3)
    rc = lib.tl_pack_links(hctx, ctypes.byref(g), ctypes.c_void_p(FAKE_W), ptr, n, p, ctypes.c_void_p(FAKE_PSI))
    assert rc in CODES and rc != 0
    a, b = ctypes.c_void_p(0x10000000), ctypes.c_void_p(0x30000000)
    rc = lib.tl_laplacian(hctx, ctypes.byref(g), ctypes.c_void_p(FAKE_W), ptr, n, p, t, a, b)
    assert rc in CODES and rc != 0


@settings(max_examples=200, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(kind=st.integers(-2, 5), n_sites=st.one_of(st.integers(-3, 1 << 20), st.just(1 << 40)),
       n_rhs=st.integers(-3, 5000), phi=st.booleans())
def test_reduce_validation(lib, hctx, kind, n_sites, n_rhs, phi):
    out = (ctypes.c_double * 4)()
    psi = ctypes.c_void_p(0x10000000)
    ph = ctypes.c_void_p(0x50000000) if phi else None
    for fn in (lib.tl_reduce, lib.tl_reduce_noalloc):
        rc = fn(hctx, kind, ctypes.c_int64(n_sites), n_rhs, psi, ph, out)
        assert rc in CODES and rc != 0
        if kind not in (0, 1, 2) or n_rhs <= 0 or n_sites <= 0:
            assert rc in (-1, -2)
