"""sesm_rayleigh_noalloc (the entry point that allocates no device memory)
against sesm_rayleigh through the C ABI: two calls in a row, the second on a
smaller input, equal bit for bit; sizes beyond the fixed array rejected."""
import ctypes
import math

import numpy as np
import pytest

import workloads as W
from oracle import dense

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _noalloc(s):
    f = s.lib.sesm_rayleigh_noalloc
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_void_p]
    return f


def _call(s, f, mu, orders):
    o = np.ascontiguousarray(orders, dtype=np.int32)
    B = np.full(len(o), np.nan + 1j * np.nan, dtype=np.complex128)
    rc = f(s.h, ctypes.c_void_p(mu.data_ptr()), o.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(o),
           ctypes.c_void_p(B.ctypes.data))
    return rc, B


def test_noalloc_matches_rayleigh_twice(torch):
    import paper_1707_04950_amd as lib
    from gpu_util import set_surface, to_dev
    s = lib.Solver(0)
    try:
        f = _noalloc(s)
        # call 1: accelerated random surface, N = 400, 41 orders (propagating and evanescent)
        a, b = W.gaussian_surface(5.0, 0.5, 1.0, W.SEED_BASE + 5)
        wl = W.Workload(name="gauss-d5", d=5.0, k=2 * math.pi, theta_deg=30.0, N=400, j=8, h=0.85, A=40.0,
                        a_coef=a, b_coef=b, L=0.5)
        set_surface(s, wl, dense.Discretization(wl), mode=lib.MODE_ACCEL)
        mu = to_dev(torch, W.random_density(400, 11))
        orders = list(range(-20, 21))
        ref = s.rayleigh(mu, orders)
        rc, got = _call(s, f, mu, orders)
        print("call 1: rc %d, max|B - B_ref| %.1e" % (rc, np.max(np.abs(got - ref))))
        assert rc == 0 and np.array_equal(got, ref)
        # call 2: a smaller input (dense sinusoid, N = 64, 3 orders); the
        # array keeps the first call's 41 entries, only 3 are rewritten
        wl2 = W.config_dense_sinusoid(64)
        set_surface(s, wl2, dense.Discretization(wl2))
        mu2 = to_dev(torch, W.random_density(64, 12))
        orders2 = [-2, 0, 1]
        ref2 = s.rayleigh(mu2, orders2)
        rc, got2 = _call(s, f, mu2, orders2)
        print("call 2: rc %d, max|B - B_ref| %.1e" % (rc, np.max(np.abs(got2 - ref2))))
        assert rc == 0 and np.array_equal(got2, ref2)
        # beyond the fixed array: rejected before any device work
        big = np.zeros(4097, dtype=np.int32)
        rc, _ = _call(s, f, mu2, big)
        assert rc == lib.SESM_EINVAL and b"at most" in s.lib.sesm_last_error(s.h)
    finally:
        s.close()
