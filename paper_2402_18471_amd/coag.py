"""Python face of libcoag with the C ABI's names (coag_mass_grid, coag_create,
coag_rates, coag_rates_blocked, coag_rhs, coag_step, coag_step_backward;
coag_step_noalloc through coag_step(..., noalloc=True)).

Tensors are torch CUDA (HIP) tensors, float64 (int32 for counters), contiguous;
torch supplies device memory and the current stream, nothing else.
"""
from __future__ import annotations

import ctypes as ct

import numpy as np
import torch

from . import _lib as L

CELL_KEYS = ("T", "rho_g", "c_s", "Omega", "H", "nu_mol", "alpha")


def coag_mass_grid(n_bins, lo, hi, by_mass=False, rho_m=1.67):
    """Host mass grid: N bins with outer edges lo, hi (radius in cm, or mass in
    g if by_mass).  Returns numpy (m, m_edge, s)."""
    m, me, s = np.empty(n_bins), np.empty(n_bins + 1), np.empty(n_bins)
    dp = lambda a: a.ctypes.data_as(L._dp)
    L.check(L.load().coag_mass_grid(n_bins, lo, hi, 1 if by_mass else 0, rho_m, dp(m), dp(me), dp(s)))
    return m, me, s


def _dev(t, dtype=torch.float64, shape=None, name="tensor"):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def _ptr(t):
    return ct.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


class CoagContext:
    """coag_create / coag_destroy around one mass grid on the current device.
    vertical=True selects the vertically integrated kernel (states are
    surface densities, cells are columns; see coag_grid in include/coag.h)."""

    def __init__(self, m, m_edge, s, rho_m=1.67, eta=11.0 / 6.0, chi=1.0, split=L.SPLIT_MASS,
                 vertical=False):
        self.m = np.ascontiguousarray(m, dtype=np.float64)
        self.m_edge = np.ascontiguousarray(m_edge, dtype=np.float64)
        self.s = np.ascontiguousarray(s, dtype=np.float64)
        self.N = int(self.m.shape[0])
        self.P = self.N * (self.N + 1) // 2
        self.rho_m, self.eta, self.chi, self.split = rho_m, eta, chi, split
        self.vertical = bool(vertical)
        dp = lambda a: a.ctypes.data_as(L._dp)
        g = L.Grid(self.N, split, dp(self.m), dp(self.m_edge), dp(self.s), rho_m, eta, chi,
                   int(self.vertical))
        h = ct.c_void_p()
        self._lib = L.load()
        L.check(self._lib.coag_create(ct.byref(g), ct.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.coag_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        L.check(rc, self._h)

    def _cells(self, cells, C):
        arrs = [_dev(cells[k], shape=(C,), name=k) for k in CELL_KEYS]
        return L.Cells(*[a.data_ptr() for a in arrs]), arrs

    # ------------------------------------------------------------------ calls
    def coag_rates(self, cells, v_dust, v_frag, Kc=None, Kf=None):
        C = int(v_frag.shape[0])
        cs, keep = self._cells(cells, C)
        _dev(v_dust, shape=(C, self.N, 3), name="v_dust")
        _dev(v_frag, shape=(C,), name="v_frag")
        dev = v_frag.device
        Kc = torch.empty((C, self.P), dtype=torch.float64, device=dev) if Kc is None else _dev(Kc, shape=(C, self.P), name="Kc")
        Kf = torch.empty((C, self.P), dtype=torch.float64, device=dev) if Kf is None else _dev(Kf, shape=(C, self.P), name="Kf")
        self._check(self._lib.coag_rates(self._h, C, ct.byref(cs), _ptr(v_dust), _ptr(v_frag),
                                         _ptr(Kc), _ptr(Kf), _stream()))
        return Kc, Kf

    def blocked_shape(self, C):
        """Shape of the 16-cell-blocked rates of C cells (both kinds in one
        array; the layout of COAG_RATES_BLK32 / BLK64 in include/coag.h):
        [ceil(C / 16)][slots][64]."""
        return ((C + 15) // 16, pair_slots(self.N), 64)

    def coag_rates_blocked(self, cells, v_dust, v_frag, dtype=torch.float32, K=None):
        """The rates in the 16-cell-blocked layout (blocked_shape(C)), both
        kinds in one tensor, float32 (for split-precision steps) or float64
        (for the batched FP64 step); coag_step takes it as Kc with Kf None."""
        if dtype not in (torch.float32, torch.float64):
            raise TypeError("dtype must be torch.float32 or torch.float64")
        C = int(v_frag.shape[0])
        cs, keep = self._cells(cells, C)
        _dev(v_dust, shape=(C, self.N, 3), name="v_dust")
        _dev(v_frag, shape=(C,), name="v_frag")
        dev, shp = v_frag.device, self.blocked_shape(C)
        K = torch.empty(shp, dtype=dtype, device=dev) if K is None else _dev(K, dtype, shp, "K")
        self._check(self._lib.coag_rates_blocked(self._h, C, ct.byref(cs), _ptr(v_dust), _ptr(v_frag),
                                                 1 if dtype == torch.float32 else 0, _ptr(K),
                                                 _stream()))
        return K

    def coag_rhs(self, rho, Kc, Kf, out=None):
        C = int(rho.shape[0])
        _dev(rho, shape=(C, self.N), name="rho")
        _dev(Kc, shape=(C, self.P), name="Kc")
        _dev(Kf, shape=(C, self.P), name="Kf")
        out = torch.empty_like(rho) if out is None else _dev(out, shape=(C, self.N), name="out")
        self._check(self._lib.coag_rhs(self._h, C, _ptr(rho), _ptr(Kc), _ptr(Kf), _ptr(out), _stream()))
        return out

    def coag_step(self, rho, Kc, Kf, dt, h=None, mode=L.ADAPTIVE, prec=L.PREC_FP64, rtol=1e-2,
                  atol_rel=1e-10, h_min_rel=1e-12, max_sub=10000, renorm=False, nsub=None,
                  h_log=None, log=True, check_status=True, noalloc=False):
        """Advances rho (in place) by dt; returns dict(rho, h, nsub, nrej, h_log, status).
        Kc, Kf: float64 [C][P] from coag_rates, or the 16-cell-blocked rates
        of coag_rates_blocked as Kc with Kf None (float32: split precision
        only; float64: FP64 only).  check_status: wait for the call and raise CoagCellError if any
        cell's status is not COAG_CELL_OK (the failed cells keep the state
        the call left them in); False returns at once, with the per-cell
        status for the caller to inspect.  noalloc: call coag_step_noalloc,
        which takes the batched step's workspace from the library's static
        per-device scratch array instead of allocating it."""
        C = int(rho.shape[0])
        dev = rho.device
        _dev(rho, shape=(C, self.N), name="rho")
        if Kc.dim() == 3:
            layout = L.RATES_BLK32 if Kc.dtype == torch.float32 else L.RATES_BLK64
            _dev(Kc, dtype=Kc.dtype, shape=self.blocked_shape(C), name="K")
            if Kf is not None:
                raise ValueError("blocked rates hold both kinds: pass Kf=None")
        else:
            layout = L.RATES_CP64
            _dev(Kc, shape=(C, self.P), name="Kc")
            _dev(Kf, shape=(C, self.P), name="Kf")
        if h is None:
            h = torch.zeros(C, dtype=torch.float64, device=dev)
        _dev(h, shape=(C,), name="h")
        if nsub is None:
            nsub = torch.zeros(C, dtype=torch.int32, device=dev)
        _dev(nsub, dtype=torch.int32, shape=(C,), name="nsub")
        if mode == L.REPLAY:
            if h_log is None:
                raise ValueError("REPLAY needs h_log")
            max_sub = int(h_log.shape[1])
        if h_log is None and log:
            h_log = torch.zeros((C, max_sub), dtype=torch.float64, device=dev)
        if h_log is not None:
            _dev(h_log, shape=(C, max_sub), name="h_log")
        nrej = torch.zeros(C, dtype=torch.int32, device=dev)
        status = torch.zeros(C, dtype=torch.int32, device=dev)
        tol = L.Tol(rtol, atol_rel, h_min_rel, max_sub, mode, prec, 1 if renorm else 0, layout)
        fn = self._lib.coag_step_noalloc if noalloc else self._lib.coag_step
        self._check(fn(self._h, C, _ptr(rho), _ptr(Kc), _ptr(Kf), float(dt), _ptr(h),
                       ct.byref(tol), _ptr(nsub), _ptr(nrej), _ptr(h_log), _ptr(status),
                       _stream()))
        out = dict(rho=rho, h=h, nsub=nsub, nrej=nrej, h_log=h_log, status=status)
        if check_status:
            L.check_cells(status)
        return out

    def coag_step_backward(self, rho_in, cells, v_dust, v_frag, h_log, nsub, g_out,
                           prec=L.PREC_FP64):
        C = int(rho_in.shape[0])
        _dev(rho_in, shape=(C, self.N), name="rho_in")
        cs, keep = self._cells(cells, C)
        _dev(v_dust, shape=(C, self.N, 3), name="v_dust")
        _dev(v_frag, shape=(C,), name="v_frag")
        _dev(h_log, name="h_log")
        _dev(nsub, dtype=torch.int32, shape=(C,), name="nsub")
        _dev(g_out, shape=(C, self.N), name="g_out")
        g_in = torch.empty_like(rho_in)
        g_alpha = torch.empty(C, dtype=torch.float64, device=rho_in.device)
        g_vfrag = torch.empty(C, dtype=torch.float64, device=rho_in.device)
        self._check(self._lib.coag_step_backward(self._h, C, _ptr(rho_in), ct.byref(cs),
                                                 _ptr(v_dust), _ptr(v_frag), _ptr(h_log),
                                                 int(h_log.shape[1]), _ptr(nsub), _ptr(g_out),
                                                 _ptr(g_in), _ptr(g_alpha), _ptr(g_vfrag),
                                                 prec, _stream()))
        return g_in, g_alpha, g_vfrag


def coag_create(m, m_edge, s, **kw) -> CoagContext:
    return CoagContext(m, m_edge, s, **kw)


def pair_slots(N):
    """Slots of two pairs per 16-cell block of the blocked rate layout:
    rows taken two pairs at a time, S(N) = m (m + 1) for N = 2m, (m + 1)^2
    for N = 2m + 1."""
    m = N >> 1
    return (m + 1) ** 2 if N & 1 else m * (m + 1)


def _blocked_index(N, f32):
    """[P][16]: the position, within a block of the blocked layout, of the
    coagulating rate (kind 0; kind 1 follows it) of pair p, cell c."""
    i = np.repeat(np.arange(N), np.arange(1, N + 1))
    j = np.concatenate([np.arange(k + 1) for k in range(N)])
    m = i >> 1
    sl = np.where(i & 1, (m + 1) ** 2, m * (m + 1)) + (j >> 1)
    u, c = (j & 1)[:, None], np.arange(16)[None, :]
    if f32:
        return ((sl[:, None] * 16 + c) * 2 + u) * 2
    return ((sl[:, None] * 2 + u) * 16 + c) * 2


def unblock(K, C):
    """Host copies of blocked rates as (Kc, Kf) [C][P] numpy arrays, and the
    values the layout holds besides them (padding cells, zero entries)."""
    x = K.detach().cpu().numpy() if isinstance(K, torch.Tensor) else np.asarray(K)
    nb, S = x.shape[0], x.shape[1]
    N = next(n for n in range(1, 1024) if pair_slots(n) == S)
    idx = _blocked_index(N, x.dtype == np.float32)
    flat = x.reshape(nb, -1)
    kc = flat[:, idx].transpose(0, 2, 1).reshape(nb * 16, -1)
    kf = flat[:, idx + 1].transpose(0, 2, 1).reshape(nb * 16, -1)
    used = np.zeros(flat.shape[1], bool)
    used[idx.ravel()] = True
    used[idx.ravel() + 1] = True
    rest = np.concatenate([kc[C:].ravel(), kf[C:].ravel(), flat[:, ~used].ravel()])
    return kc[:C], kf[:C], rest


def block(Kc, Kf, dtype=torch.float64, device="cuda:0"):
    """Blocked rates (zero padding) from [C][P] arrays (host or device)."""
    kc = Kc.detach().cpu().numpy() if isinstance(Kc, torch.Tensor) else np.asarray(Kc)
    kf = Kf.detach().cpu().numpy() if isinstance(Kf, torch.Tensor) else np.asarray(Kf)
    C, P = kc.shape
    N = int(round((np.sqrt(8 * P + 1) - 1) / 2))
    f32 = dtype == torch.float32
    nb = (C + 15) // 16
    idx = _blocked_index(N, f32)
    flat = np.zeros((nb, 64 * pair_slots(N)), np.float32 if f32 else np.float64)
    pad = lambda a: np.concatenate([a, np.zeros((nb * 16 - C, P))]).reshape(nb, 16, P)
    flat[:, idx] = pad(kc).transpose(0, 2, 1)
    flat[:, idx + 1] = pad(kf).transpose(0, 2, 1)
    return torch.as_tensor(flat.reshape(nb, pair_slots(N), 64), device=device)


class TransportContext:
    """coag_transport_create / destroy (include/coag_transport.h): the dust
    transport step of the dynamics solver on an (R, t = Z/R) grid of n_r x n_z
    cells for the N species of radii s, and the scheduler coupling it to a
    CoagContext.  Marshalling only: the step runs in the library's kernels.
    eps_floor: the dust-to-gas floor of each species (0: none)."""

    def __init__(self, R_edge, t_edge, s, rho_m=1.67, GM=0.0, Sc=1.0, c_adv=0.4, c_diff=0.2,
                 eps_floor=0.0):
        self.R_edge = np.ascontiguousarray(R_edge, dtype=np.float64)
        self.t_edge = np.ascontiguousarray(t_edge, dtype=np.float64)
        self.s = np.ascontiguousarray(s, dtype=np.float64)
        self.n_r, self.n_z, self.N = len(self.R_edge) - 1, len(self.t_edge) - 1, len(self.s)
        self.C = self.n_r * self.n_z
        dp = lambda a: a.ctypes.data_as(L._dp)
        g = L.TGrid(self.n_r, self.n_z, dp(self.R_edge), dp(self.t_edge), GM, Sc, c_adv, c_diff,
                    eps_floor)
        h = ct.c_void_p()
        self._lib = L.load()
        L.check_t(self._lib.coag_transport_create(ct.byref(g), self.N, dp(self.s), rho_m,
                                                   ct.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.coag_transport_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _cells(self, cells):
        arrs = [_dev(cells[k], shape=(self.C,), name=k) for k in CELL_KEYS]
        return L.Cells(*[a.data_ptr() for a in arrs]), arrs

    def dt(self, cells, v):
        """CFL time step (a host float; synchronises the current stream)."""
        cs, keep = self._cells(cells)
        _dev(v, shape=(self.C, self.N, 3), name="v")
        out = ct.c_double()
        L.check_t(self._lib.coag_transport_dt(self._h, ct.byref(cs), _ptr(v), ct.byref(out),
                                               _stream()), self._h)
        return out.value

    def step(self, cells, v_gas, rho, v, dt):
        """One transport step of dt in place on rho [C][N] and v [C][N][3]."""
        cs, keep = self._cells(cells)
        _dev(v_gas, shape=(self.C, 3), name="v_gas")
        _dev(rho, shape=(self.C, self.N), name="rho")
        _dev(v, shape=(self.C, self.N, 3), name="v")
        L.check_t(self._lib.coag_transport_step(self._h, ct.byref(cs), _ptr(v_gas), _ptr(rho),
                                                 _ptr(v), float(dt), _stream()), self._h)

    def evolve(self, ctx: "CoagContext", cells, v_gas, v_frag, rho, v, h, t_end, max_steps=1 << 40,
               prec=L.PREC_FP64, rtol=1e-2, atol_rel=1e-10, h_min_rel=1e-12, max_sub=256):
        """Transport steps at the CFL time step up to t_end, with the
        coagulation update triggered by the scheduler rule; rho, v, h in
        place.  Returns the scheduler statistics as a dict."""
        cs, keep = self._cells(cells)
        _dev(v_gas, shape=(self.C, 3), name="v_gas")
        _dev(v_frag, shape=(self.C,), name="v_frag")
        _dev(rho, shape=(self.C, self.N), name="rho")
        _dev(v, shape=(self.C, self.N, 3), name="v")
        _dev(h, shape=(self.C,), name="h")
        tol = L.Tol(rtol, atol_rel, h_min_rel, max_sub, L.ADAPTIVE, prec, 0, 0)
        st = L.EvolveStats()
        L.check_t(self._lib.coag_evolve(ctx._h, self._h, self.C, ct.byref(cs), _ptr(v_gas),
                                         _ptr(v_frag), _ptr(rho), _ptr(v), _ptr(h), float(t_end),
                                         int(max_steps), ct.byref(tol), ct.byref(st), _stream()),
                  self._h)
        return {"transport_steps": st.transport_steps, "coag_calls": st.coag_calls,
                "t_reached": st.t_reached, "cells_failed": st.cells_failed}
