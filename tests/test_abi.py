"""The C-ABI library without a GPU: it loads, exports every function that
include/coag.h declares, builds the same mass grid as the oracle, and rejects
bad arguments on the host before any device work."""
import ctypes as ct

import numpy as np
import pytest


@pytest.fixture(scope="module")
def L():
    from paper_2402_18471_amd import _lib
    return _lib


def test_library_exports_every_declared_symbol(L):
    lib = L.load()
    names = L.header_symbols()
    assert set(names) == {"coag_mass_grid", "coag_create", "coag_destroy", "coag_last_error",
                          "coag_rates", "coag_rates_blocked", "coag_rhs", "coag_step",
                          "coag_step_noalloc", "coag_step_backward"}
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.parametrize("args", [(100, 1e-5, 0.5, False), (135, 1e-5, 20.0, False),
                                  (40, 1e-12, 1e-3, True), (150, 1e-5, 10.0, False),
                                  (200, 1e-5, 100.0, False), (2, 1e-4, 2e-4, False)])
def test_mass_grid_matches_oracle(L, O, args):
    from paper_2402_18471_amd.coag import coag_mass_grid
    n, lo, hi, by_mass = args
    m, me, s = coag_mass_grid(n, lo, hi, by_mass=by_mass, rho_m=1.67)
    om, ome, os_ = O.mass_grid(n, lo, hi, by_mass=by_mass, rho_m=1.67)
    # both evaluate the same definition with the host libm: identical bits, so
    # the two sides of every parity test see the same grid
    assert np.array_equal(m, om) and np.array_equal(me, ome) and np.array_equal(s, os_)


def test_mass_grid_rejects_bad_arguments(L):
    lib = L.load()
    buf = (ct.c_double * 16)()
    p = ct.cast(buf, L._dp)
    assert lib.coag_mass_grid(1, 1e-5, 1.0, 0, 1.67, p, p, p) == L.COAG_EINVAL
    assert lib.coag_mass_grid(8, 0.0, 1.0, 0, 1.67, p, p, p) == L.COAG_EINVAL
    assert lib.coag_mass_grid(8, 1.0, 0.5, 0, 1.67, p, p, p) == L.COAG_EINVAL
    assert lib.coag_mass_grid(8, 1e-5, 1.0, 0, 1.67, None, p, p) == L.COAG_EINVAL
    assert b"coag_mass_grid" in lib.coag_last_error(None)


def _grid(L, m, me, s, eta=11 / 6, chi=1.0, split=0, n=None):
    dp = lambda a: a.ctypes.data_as(L._dp)
    return L.Grid(len(m) if n is None else n, split, dp(m), dp(me), dp(s), 1.67, eta, chi)


def test_create_rejects_bad_grids_on_host(L):
    from paper_2402_18471_amd.coag import coag_mass_grid
    lib = L.load()
    m, me, s = coag_mass_grid(10, 1e-5, 1.0)
    out = ct.c_void_p()
    cases = [
        (_grid(L, m[::-1].copy(), me, s), b"strictly increasing"),
        (_grid(L, m, me[::-1].copy(), s), b"bracket"),
        (_grid(L, m, me, s, eta=2.0), b"eta"),
        (_grid(L, m, me, s, chi=0.0), b"chi"),
        (_grid(L, m, me, s, split=7), b"split"),
        (_grid(L, m, me, s, n=1), b"n_bins"),
        (_grid(L, m, me, s, n=2000), b"n_bins"),
    ]
    for g, msg in cases:
        assert lib.coag_create(ct.byref(g), ct.byref(out)) == L.COAG_EINVAL
        assert msg in lib.coag_last_error(None), lib.coag_last_error(None)
        assert not out.value
    assert lib.coag_create(None, ct.byref(out)) == L.COAG_EINVAL


def test_calls_reject_null_context(L):
    lib = L.load()
    tol = L.Tol(1e-2, 1e-10, 0.0, 10, 0, 0, 0, 0)
    assert lib.coag_rhs(None, 1, None, None, None, None, None) == L.COAG_EINVAL
    assert lib.coag_step(None, 1, None, None, None, 1.0, None, ct.byref(tol), None, None, None,
                         None, None) == L.COAG_EINVAL
    assert lib.coag_rates(None, 1, None, None, None, None, None, None) == L.COAG_EINVAL
    assert lib.coag_rates_blocked(None, 1, None, None, None, 1, None, None) == L.COAG_EINVAL
    assert lib.coag_step_backward(None, 1, None, None, None, None, None, 1, None, None, None,
                                  None, None, 0, None) == L.COAG_EINVAL
    lib.coag_destroy(None)


def test_binding_refuses_host_tensors(L):
    import torch
    from paper_2402_18471_amd.coag import _dev
    with pytest.raises(ValueError):
        _dev(torch.zeros(3, dtype=torch.float64))
