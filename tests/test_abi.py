"""The C-ABI library without a GPU: it loads, exports every function that
include/coag.h and include/coag_transport.h declare, builds the same mass grid as the oracle, and rejects
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
                          "coag_step_noalloc", "coag_step_backward", "coag_transport_create",
                          "coag_transport_destroy", "coag_transport_last_error",
                          "coag_transport_dt", "coag_transport_step", "coag_evolve"}
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


def test_transport_create_rejects_bad_grids_on_the_host(L):
    """Every check of coag_transport_create runs before any device call."""
    lib = L.load()
    dp = lambda a: a.ctypes.data_as(L._dp)
    R = np.array([1.0, 2.0, 3.0])
    t = np.array([0.0, 0.1])
    s = np.array([1e-4, 1e-3])
    h = ct.c_void_p()

    def create(R_, t_, s_=s, N=2, rho_m=1.6, GM=1.0, Sc=1.0, ca=0.4, cd=0.2, nr=None, nz=None,
               ef=0.0):
        g = L.TGrid(len(R_) - 1 if nr is None else nr, len(t_) - 1 if nz is None else nz,
                    dp(R_), dp(t_), GM, Sc, ca, cd, ef)
        return lib.coag_transport_create(ct.byref(g), N, dp(s_), rho_m, ct.byref(h))

    bad = [dict(R_=np.array([1.0, 1.0, 3.0]), t_=t),          # R not increasing
           dict(R_=np.array([0.0, 1.0, 3.0]), t_=t),          # R_edge[0] = 0
           dict(R_=R, t_=np.array([0.05, 0.1])),               # no midplane
           dict(R_=R, t_=np.array([0.0, 0.0])),                # t not increasing
           dict(R_=R, t_=t, s_=np.array([1e-4, 0.0])),         # a radius of 0
           dict(R_=R, t_=t, N=0), dict(R_=R, t_=t, N=1024),
           dict(R_=R, t_=t, rho_m=0.0), dict(R_=R, t_=t, GM=-1.0), dict(R_=R, t_=t, Sc=0.0),
           dict(R_=R, t_=t, ca=0.0), dict(R_=R, t_=t, cd=-1.0), dict(R_=R, t_=t, nr=0),
           dict(R_=R, t_=t, nz=0), dict(R_=R, t_=t, ef=-1e-20), dict(R_=R, t_=t, ef=np.inf),
           dict(R_=R, t_=t, ef=np.nan)]
    for kw in bad:
        assert create(**kw) == L.COAG_EINVAL, kw
        assert h.value is None
        assert lib.coag_transport_last_error(None).decode().startswith("coag_transport_create")
    assert lib.coag_transport_create(None, 2, dp(s), 1.6, ct.byref(h)) == L.COAG_EINVAL
