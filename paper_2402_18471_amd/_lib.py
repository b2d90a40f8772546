"""ctypes binding of libcoag (include/coag.h): argument marshalling only.

Every numerical step runs in the HIP kernels of the library; this module
checks tensor shapes, dtypes and devices, passes raw device pointers and the
current torch stream, and turns error codes into exceptions.  It refuses to
run without the compiled library (there is no fallback path).
"""
from __future__ import annotations

import ctypes as ct
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libcoag.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "coag.h")
HEADERS = [HEADER, os.path.join(os.path.dirname(HERE), "include", "coag_transport.h")]

COAG_OK, COAG_EINVAL, COAG_ENOMEM, COAG_EHIP, COAG_ENOTSUP = 0, -1, -2, -3, -4
CELL_OK, CELL_HMIN, CELL_MAXSUB, CELL_NONFINITE = 0, 1, 2, 3
SPLIT_MASS, SPLIT_NUMBER = 0, 1
PREC_FP64, PREC_SPLIT_BF16 = 0, 1
ADAPTIVE, FIXED, REPLAY = 0, 1, 2
RATES_CP64, RATES_BLK32, RATES_BLK64 = 0, 1, 2

_dp = ct.POINTER(ct.c_double)
_vp = ct.c_void_p


class Grid(ct.Structure):
    _fields_ = [("n_bins", ct.c_int32), ("split", ct.c_int32), ("m", _dp), ("m_edge", _dp),
                ("s", _dp), ("rho_m", ct.c_double), ("eta", ct.c_double), ("chi", ct.c_double),
                ("vertical", ct.c_int32)]


class Cells(ct.Structure):
    _fields_ = [(k, _vp) for k in ("T", "rho_g", "c_s", "Omega", "H", "nu_mol", "alpha")]


class Tol(ct.Structure):
    _fields_ = [("rtol", ct.c_double), ("atol_rel", ct.c_double), ("h_min_rel", ct.c_double),
                ("max_sub", ct.c_int32), ("mode", ct.c_int32), ("prec", ct.c_int32),
                ("renorm", ct.c_int32), ("rates_layout", ct.c_int32)]


class TGrid(ct.Structure):
    _fields_ = [("n_r", ct.c_int32), ("n_z", ct.c_int32), ("R_edge", _dp), ("t_edge", _dp),
                ("GM", ct.c_double), ("Sc", ct.c_double), ("c_adv", ct.c_double),
                ("c_diff", ct.c_double), ("eps_floor", ct.c_double)]


class EvolveStats(ct.Structure):
    _fields_ = [("transport_steps", ct.c_int64), ("coag_calls", ct.c_int64),
                ("t_reached", ct.c_double), ("cells_failed", ct.c_int32)]


class CoagError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libcoag error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libcoag.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError(f"{LIBPATH} is missing: build it with "
                           "`python -m paper_2402_18471_amd.build` (hipcc, gfx950)")
    lib = ct.CDLL(LIBPATH)
    i32, i64 = ct.c_int32, ct.c_int64
    P = ct.POINTER
    sig = {
        "coag_mass_grid": (ct.c_int, [i32, ct.c_double, ct.c_double, i32, ct.c_double, _dp, _dp, _dp]),
        "coag_create": (ct.c_int, [P(Grid), P(_vp)]),
        "coag_destroy": (None, [_vp]),
        "coag_last_error": (ct.c_char_p, [_vp]),
        "coag_rates": (ct.c_int, [_vp, i64, P(Cells), _vp, _vp, _vp, _vp, _vp]),
        "coag_rates_blocked": (ct.c_int, [_vp, i64, P(Cells), _vp, _vp, i32, _vp, _vp]),
        "coag_rhs": (ct.c_int, [_vp, i64, _vp, _vp, _vp, _vp, _vp]),
        "coag_step": (ct.c_int, [_vp, i64, _vp, _vp, _vp, ct.c_double, _vp, P(Tol), _vp, _vp,
                                 _vp, _vp, _vp]),
        "coag_step_noalloc": (ct.c_int, [_vp, i64, _vp, _vp, _vp, ct.c_double, _vp, P(Tol), _vp,
                                         _vp, _vp, _vp, _vp]),
        "coag_step_backward": (ct.c_int, [_vp, i64, _vp, P(Cells), _vp, _vp, _vp, i32, _vp, _vp,
                                          _vp, _vp, _vp, i32, _vp]),
        "coag_transport_create": (ct.c_int, [P(TGrid), i32, _dp, ct.c_double, P(_vp)]),
        "coag_transport_destroy": (None, [_vp]),
        "coag_transport_last_error": (ct.c_char_p, [_vp]),
        "coag_transport_dt": (ct.c_int, [_vp, P(Cells), _vp, P(ct.c_double), _vp]),
        "coag_transport_step": (ct.c_int, [_vp, P(Cells), _vp, _vp, _vp, ct.c_double, _vp]),
        "coag_evolve": (ct.c_int, [_vp, _vp, i64, P(Cells), _vp, _vp, _vp, _vp, _vp, ct.c_double,
                                   i64, P(Tol), P(EvolveStats), _vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype, f.argtypes = res, args
    _lib = lib
    return lib


def header_symbols():
    """Function names declared in include/coag.h and include/coag_transport.h."""
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"\b(coag_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


class CoagCellError(CoagError):
    """Some cells of a coag_step call did not complete (per-cell status)."""

    def __init__(self, counts):
        names = {CELL_HMIN: "HMIN", CELL_MAXSUB: "MAXSUB", CELL_NONFINITE: "NONFINITE"}
        what = ", ".join(f"{n} {names.get(k, k)}" for k, n in sorted(counts.items()))
        super().__init__(0, f"coag_step: cells failed ({what})")
        self.counts = counts


def check_cells(status):
    """Raise CoagCellError if any entry of the per-cell status tensor is not
    CELL_OK (waits for the stream that wrote it)."""
    bad = status[status != CELL_OK]
    if bad.numel():
        vals, cnt = bad.unique(return_counts=True)
        raise CoagCellError({int(v): int(c) for v, c in zip(vals.tolist(), cnt.tolist())})


def check(rc, ctx=None):
    if rc != COAG_OK:
        msg = load().coag_last_error(ctx)
        raise CoagError(rc, msg.decode() if msg else "")


def check_t(rc, tctx=None):
    """check() for the transport calls (their messages live in the transport context)."""
    if rc != COAG_OK:
        msg = load().coag_transport_last_error(tctx)
        raise CoagError(rc, msg.decode() if msg else "")
