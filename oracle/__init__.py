"""CPU oracle of the coagulation-fragmentation update (plain C, FP64).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library ``paper_2402_18471_amd``: the two meet only through
the seeded inputs of ``paper_2402_18471_amd.disc``.

Every function follows Robinson, Booth & Owen (cuDisc), Sec. 5 (dust growth and
fragmentation): eqs. ``smol``, ``ngain``, ``kernel``, ``vbrown``, ``OCVrel``,
``p_frag``, ``Cijk``, ``Rijk``, ``Nijk``, ``fragrem`` and the Bogacki-Shampine
3(2) integrator with the tolerances of that section; the sub-cycling rule is
Sec. 6.  Where the paper is silent or ambiguous the reading taken is stated at
the function that takes it (grid edges, the two-bin split, the loss indices,
the step-size controller).

Packed pair index: p(i, j) = i (i + 1) / 2 + j for j <= i.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")

SPLIT_MASS, SPLIT_NUMBER = 0, 1
ADAPTIVE, FIXED, REPLAY = 0, 1, 2
CELL_OK, CELL_HMIN, CELL_MAXSUB, CELL_NONFINITE = 0, 1, 2, 3

_dp = ct.POINTER(ct.c_double)
_ip = ct.POINTER(ct.c_int32)


class _Grid(ct.Structure):
    _fields_ = [("N", ct.c_int32), ("split", ct.c_int32), ("m", _dp), ("m_edge", _dp),
                ("s", _dp), ("rho_m", ct.c_double), ("eta", ct.c_double), ("chi", ct.c_double),
                ("vertical", ct.c_int32)]


class _Cells(ct.Structure):
    _fields_ = [(k, _dp) for k in ("T", "rho_g", "c_s", "Omega", "H", "nu_mol", "alpha")]


class _Tol(ct.Structure):
    _fields_ = [("rtol", ct.c_double), ("atol_rel", ct.c_double), ("h_min_rel", ct.c_double),
                ("max_sub", ct.c_int32), ("mode", ct.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            from . import build as _b
            _b.build()
        lib = ct.CDLL(_LIBPATH)
        G, Cl, Tl = ct.POINTER(_Grid), ct.POINTER(_Cells), ct.POINTER(_Tol)
        L = ct.c_long
        sig = {
            "oracle_mass_grid": (ct.c_int, [ct.c_int, ct.c_double, ct.c_double, ct.c_int, ct.c_double, _dp, _dp, _dp]),
            "oracle_redistribution_dense": (ct.c_int, [G, _dp]),
            "oracle_redistribution_sparse": (ct.c_int, [G, _ip, _dp, _ip, _dp, _ip, _dp, _dp]),
            "oracle_rates": (ct.c_int, [G, L, Cl, _dp, _dp, _dp, _dp]),
            "oracle_rates_deriv": (ct.c_int, [G, L, Cl, _dp, _dp, _dp, _dp, _dp, _dp]),
            "oracle_rhs": (ct.c_int, [G, L, _dp, _dp, _dp, _dp, _dp, _dp]),
            "oracle_rhs_dense": (ct.c_int, [G, L, _dp, _dp, _dp, _dp]),
            "oracle_rhs_vjp": (ct.c_int, [G, L, _dp, _dp, _dp, _dp, _dp, _dp, _dp]),
            "oracle_step": (ct.c_int, [G, L, _dp, _dp, _dp, ct.c_double, _dp, Tl, _ip, _ip, _dp, _ip]),
            "oracle_step_backward": (ct.c_int, [G, L, Cl, _dp, _dp, _dp, ct.c_double, _dp, _ip,
                                                ct.c_int32, _dp, _dp, _dp, _dp]),
            "oracle_cs_step_grad": (ct.c_double, [G, L, Cl, _dp, _dp, _dp, _dp, _ip, ct.c_int32,
                                                  _dp, ct.c_int, L, ct.c_double]),
            "oracle_cs_rhs_grad": (ct.c_double, [G, _dp, _dp, _dp, _dp, ct.c_int, L, ct.c_double]),
            "oracle_num_threads": (ct.c_int, []),
            "oracle_set_num_threads": (None, [ct.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype, f.argtypes = res, args
        _lib = lib
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _i(a):
    return a.ctypes.data_as(_ip) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle: {what} failed (rc={rc})")


def npairs(N: int) -> int:
    return N * (N + 1) // 2


def pair_index(i, j):
    """Packed index of the unordered pair (i, j), j <= i."""
    return i * (i + 1) // 2 + j


@dataclass
class Grid:
    """Mass grid plus collision-outcome parameters (eta: fragment power law
    exponent, eq. ``fragdist``; chi: impactor excavation factor, eq.
    ``fragrem``; split: two-bin split reading of eq. ``Cijk``; vertical: 1
    for the vertically integrated kernel of Sec. 5.1, whose state is a column
    density and whose cells give the midplane gas density)."""
    m: np.ndarray
    m_edge: np.ndarray
    s: np.ndarray
    rho_m: float
    eta: float = 11.0 / 6.0
    chi: float = 1.0
    split: int = SPLIT_MASS
    vertical: int = 0

    @property
    def N(self) -> int:
        return int(self.m.shape[0])

    @property
    def P(self) -> int:
        return npairs(self.N)

    def _struct(self):
        self.m, self.m_edge, self.s = _f64(self.m), _f64(self.m_edge), _f64(self.s)
        return _Grid(self.N, self.split, _d(self.m), _d(self.m_edge), _d(self.s),
                     self.rho_m, self.eta, self.chi, int(self.vertical))


def mass_grid(N, lo, hi, by_mass=False, rho_m=1.67):
    """N log-spaced bins whose outer edges are lo and hi (radius range in cm,
    or mass range in g if ``by_mass``); returns (m, m_edge, s)."""
    m, me, s = np.empty(N), np.empty(N + 1), np.empty(N)
    _check(_load().oracle_mass_grid(N, lo, hi, 1 if by_mass else 0, rho_m, _d(m), _d(me), _d(s)),
           "mass_grid")
    return m, me, s


def make_grid(N, lo, hi, by_mass=False, rho_m=1.67, eta=11.0 / 6.0, chi=1.0, split=SPLIT_MASS,
              vertical=0):
    m, me, s = mass_grid(N, lo, hi, by_mass, rho_m)
    return Grid(m, me, s, rho_m, eta, chi, split, vertical)


def redistribution_dense(g: Grid):
    D = np.empty((2 * g.P, g.N))
    gs = g._struct()
    _check(_load().oracle_redistribution_dense(ct.byref(gs), _d(D)), "redistribution_dense")
    return D


def redistribution_sparse(g: Grid):
    P, N = g.P, g.N
    ci, ri, fl = (np.empty(P, np.int32) for _ in range(3))
    cw, rw = np.empty((P, 2)), np.empty((P, 2))
    fm, Nf = np.empty(P), np.empty((N, N))
    gs = g._struct()
    _check(_load().oracle_redistribution_sparse(ct.byref(gs), _i(ci), _d(cw), _i(ri), _d(rw),
                                                _i(fl), _d(fm), _d(Nf)), "redistribution_sparse")
    return dict(ci=ci, cw=cw, ri=ri, rw=rw, fl=fl, fm=fm, Nfrac=Nf)


_CELL_KEYS = ("T", "rho_g", "c_s", "Omega", "H", "nu_mol", "alpha")


def _cells_struct(cells):
    arrs = {k: _f64(cells[k]) for k in _CELL_KEYS}
    return _Cells(*[_d(arrs[k]) for k in _CELL_KEYS]), arrs


def rates(g: Grid, cells, v_dust, v_frag):
    """Kc, Kf of shape [C][P] (eqs. ``kernel``, ``p_frag``)."""
    C = int(np.asarray(cells["T"]).shape[0])
    v_dust, v_frag = _f64(v_dust), _f64(np.broadcast_to(v_frag, (C,)))
    Kc, Kf = np.empty((C, g.P)), np.empty((C, g.P))
    cs, keep = _cells_struct(cells)
    gs = g._struct()
    _check(_load().oracle_rates(ct.byref(gs), C, ct.byref(cs), _d(v_dust), _d(v_frag), _d(Kc), _d(Kf)),
           "rates")
    return Kc, Kf


def rates_deriv(g: Grid, cells, v_dust, v_frag):
    C = int(np.asarray(cells["T"]).shape[0])
    v_dust, v_frag = _f64(v_dust), _f64(np.broadcast_to(v_frag, (C,)))
    out = [np.empty((C, g.P)) for _ in range(4)]
    cs, keep = _cells_struct(cells)
    gs = g._struct()
    _check(_load().oracle_rates_deriv(ct.byref(gs), C, ct.byref(cs), _d(v_dust), _d(v_frag),
                                      *[_d(o) for o in out]), "rates_deriv")
    return dict(dKc_dalpha=out[0], dKf_dalpha=out[1], dKc_dvfrag=out[2], dKf_dvfrag=out[3])


def rhs(g: Grid, rho, Kc, Kf, parts=False):
    rho = _f64(np.atleast_2d(rho))
    C = rho.shape[0]
    Kc, Kf = _f64(Kc).reshape(C, g.P), _f64(Kf).reshape(C, g.P)
    out, gain, loss = np.empty_like(rho), np.empty_like(rho), np.empty_like(rho)
    gs = g._struct()
    _check(_load().oracle_rhs(ct.byref(gs), C, _d(rho), _d(Kc), _d(Kf), _d(out), _d(gain), _d(loss)),
           "rhs")
    return (out, gain, loss) if parts else out


def rhs_dense(g: Grid, rho, Kc, Kf):
    rho = _f64(np.atleast_2d(rho))
    C = rho.shape[0]
    Kc, Kf = _f64(Kc).reshape(C, g.P), _f64(Kf).reshape(C, g.P)
    out = np.empty_like(rho)
    gs = g._struct()
    _check(_load().oracle_rhs_dense(ct.byref(gs), C, _d(rho), _d(Kc), _d(Kf), _d(out)), "rhs_dense")
    return out


def rhs_vjp(g: Grid, rho, Kc, Kf, mu):
    rho, mu = _f64(np.atleast_2d(rho)), _f64(np.atleast_2d(mu))
    C = rho.shape[0]
    Kc, Kf = _f64(Kc).reshape(C, g.P), _f64(Kf).reshape(C, g.P)
    gy, gKc, gKf = np.empty_like(rho), np.empty_like(Kc), np.empty_like(Kf)
    gs = g._struct()
    _check(_load().oracle_rhs_vjp(ct.byref(gs), C, _d(rho), _d(Kc), _d(Kf), _d(mu), _d(gy),
                                  _d(gKc), _d(gKf)), "rhs_vjp")
    return gy, gKc, gKf


def step(g: Grid, rho, Kc, Kf, dt, h=None, rtol=1e-2, atol_rel=1e-10, h_min_rel=1e-12,
         max_sub=10000, mode=ADAPTIVE, nsub=None, h_log=None):
    """Sub-cycled BS3(2) integration of every cell over dt.  Returns a dict
    with rho (new state), h, nsub (accepted), nrej, h_log, status."""
    rho = _f64(np.atleast_2d(rho)).copy()
    C = rho.shape[0]
    Kc, Kf = _f64(Kc).reshape(C, g.P), _f64(Kf).reshape(C, g.P)
    h = np.zeros(C) if h is None else _f64(np.broadcast_to(h, (C,))).copy()
    ns = np.zeros(C, np.int32) if nsub is None else np.ascontiguousarray(
        np.broadcast_to(nsub, (C,)), dtype=np.int32).copy()
    nrej = np.zeros(C, np.int32)
    status = np.zeros(C, np.int32)
    if mode == REPLAY:
        log = _f64(h_log).reshape(C, -1).copy()
        max_sub = log.shape[1]
    else:
        log = np.zeros((C, max_sub))
    tol = _Tol(rtol, atol_rel, h_min_rel, max_sub, mode)
    gs = g._struct()
    _check(_load().oracle_step(ct.byref(gs), C, _d(rho), _d(Kc), _d(Kf), float(dt), _d(h),
                               ct.byref(tol), _i(ns), _i(nrej), _d(log), _i(status)), "step")
    return dict(rho=rho, h=h, nsub=ns, nrej=nrej, h_log=log, status=status)


def step_backward(g: Grid, cells, v_dust, v_frag, rho_in, dt, h_log, nsub, g_out):
    """Adjoint of a frozen step sequence; returns (g_in, g_alpha, g_vfrag)."""
    rho_in = _f64(np.atleast_2d(rho_in))
    C = rho_in.shape[0]
    v_dust, v_frag = _f64(v_dust), _f64(np.broadcast_to(v_frag, (C,)))
    h_log = _f64(h_log).reshape(C, -1)
    nsub = np.ascontiguousarray(np.broadcast_to(nsub, (C,)), dtype=np.int32)
    g_out = _f64(g_out).reshape(C, g.N)
    g_in, ga, gv = np.empty_like(rho_in), np.empty(C), np.empty(C)
    cs, keep = _cells_struct(cells)
    gs = g._struct()
    _check(_load().oracle_step_backward(ct.byref(gs), C, ct.byref(cs), _d(v_dust), _d(v_frag),
                                        _d(rho_in), float(dt), _d(h_log), _i(nsub), h_log.shape[1],
                                        _d(g_out), _d(g_in), _d(ga), _d(gv)), "step_backward")
    return g_in, ga, gv


def cs_step_grad(g: Grid, cells, v_dust, v_frag, rho_in, h_log, nsub, g_out, which, index,
                 hcs=1e-30):
    """Complex-step dJ/dx of J = g_out . rho_final; which: 'rho', 'alpha', 'vfrag'."""
    rho_in = _f64(np.atleast_2d(rho_in))
    C = rho_in.shape[0]
    v_dust, v_frag = _f64(v_dust), _f64(np.broadcast_to(v_frag, (C,)))
    h_log = _f64(h_log).reshape(C, -1)
    nsub = np.ascontiguousarray(np.broadcast_to(nsub, (C,)), dtype=np.int32)
    g_out = _f64(g_out).reshape(C, g.N)
    w = {"rho": 0, "alpha": 1, "vfrag": 2}[which]
    cs, keep = _cells_struct(cells)
    gs = g._struct()
    return _load().oracle_cs_step_grad(ct.byref(gs), C, ct.byref(cs), _d(v_dust), _d(v_frag),
                                       _d(rho_in), _d(h_log), _i(nsub), h_log.shape[1], _d(g_out),
                                       w, int(index), hcs)


def cs_rhs_grad(g: Grid, rho, Kc, Kf, mu, which, index, hcs=1e-30):
    """Complex-step d(mu . f)/dx for one cell; which: 'rho', 'Kc', 'Kf'."""
    rho, Kc, Kf, mu = _f64(rho).ravel(), _f64(Kc).ravel(), _f64(Kf).ravel(), _f64(mu).ravel()
    w = {"rho": 0, "Kc": 3, "Kf": 4}[which]
    gs = g._struct()
    return _load().oracle_cs_rhs_grad(ct.byref(gs), _d(rho), _d(Kc), _d(Kf), _d(mu), w, int(index), hcs)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's loops over cells from now on."""
    _load().oracle_set_num_threads(int(n))
