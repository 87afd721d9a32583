"""Host side of relative binning: gw_rb_edges (a host computation of the
library) gives exactly the oracle's edges (integer output, compared bit for
bit) for grids up to the 5 Hz / 8192 s neutron-star band, and its argument
checks reject bad input without a device."""
import ctypes

import numpy as np
import pytest

import synth
from oracle import relbin as rb


@pytest.fixture(scope="module")
def gw():
    import os
    import paper_1904_02863_amd as gw
    if not os.path.exists(gw.LIB_PATH):
        from paper_1904_02863_amd import build
        build.build()
    gw.load_library()
    return gw


@pytest.mark.parametrize("grid,chi,eps", [((20.0, 0.25, 3000), 1.0, 0.5), ((30.0, 1 / 16, 20000), 1.0, 0.1),
                                          ((10.0, 1.0, 500), 2.0, 0.05), ((40.0, 0.25, 2), 1.0, 0.5),
                                          ((25.0, 1 / 128, 259585), 0.5, 0.01)])
def test_edges_match_oracle(gw, grid, chi, eps):
    got = gw.rb_edges(grid, chi, eps)
    want = rb.edges(*grid, chi, eps)
    assert got.dtype == np.int64
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("f_low,duration", [(30.0, 64.0), (15.0, 512.0), (5.0, 8192.0)])
def test_edges_match_oracle_long_bands(gw, f_low, duration):
    g = synth.make_grid(f_low, 2048.0, duration)
    for eps in (0.5, 0.03):
        np.testing.assert_array_equal(gw.rb_edges(g, 1.0, eps), rb.edges(g.f_low, g.delta_f, g.n_bins, 1.0, eps))


def test_edge_arguments_are_checked(gw):
    lib = gw.load_library()
    n = ctypes.c_int64(-1)
    g = gw.GwGrid(20.0, 0.25, 1)
    assert lib.gw_rb_edges(ctypes.byref(g), 1.0, 0.5, None, 0, ctypes.byref(n)) == gw.GW_EINVAL
    g = gw.GwGrid(20.0, 0.25, 4000)
    for chi, eps in ((0.0, 0.5), (1.0, 0.0), (1.0, float("nan")), (float("inf"), 0.5)):
        assert lib.gw_rb_edges(ctypes.byref(g), chi, eps, None, 0, ctypes.byref(n)) == gw.GW_EINVAL
    assert lib.gw_rb_edges(ctypes.byref(g), 1.0, 0.5, None, 0, ctypes.byref(n)) == gw.GW_OK
    small = np.empty(max(1, n.value - 1), dtype=np.int64)
    m = ctypes.c_int64()
    rc = lib.gw_rb_edges(ctypes.byref(g), 1.0, 0.5, small.ctypes.data_as(ctypes.c_void_p), small.size,
                         ctypes.byref(m))
    assert rc == gw.GW_EINVAL and m.value == n.value


def test_create_rejects_bad_arguments_without_a_device(gw):
    lib = gw.load_library()
    g = gw.GwGrid(20.0, 0.25, 100)
    h = ctypes.c_void_p()
    edges = np.array([0, 50, 99], dtype=np.int64)
    th = np.array([30.0, 0.8, 400.0, 0.0, 0.0])
    rc = lib.gw_rb_create(None, ctypes.byref(g), 1, None, None, None, th.ctypes.data_as(ctypes.c_void_p), 5,
                          edges.ctypes.data_as(ctypes.c_void_p), 3, 0, ctypes.byref(h), None)
    assert rc == gw.GW_EINVAL and not h.value
    assert lib.gw_rb_lnl(None, None, None, 1, None, 0, None) == gw.GW_EINVAL
    assert lib.gw_rb_destroy(None) == gw.GW_OK
