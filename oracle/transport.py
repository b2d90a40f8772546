"""CPU oracle of the dust transport step (Robinson, Booth & Owen, cuDisc, Sec. 3,
"Dynamics solver"), plain numpy, FP64.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
use it, and it shares no code with the GPU library.

Each dust species is a pressureless fluid with conserved quantities
Q = (rho, rho v_R, rho v_phi R, rho v_Z) (eq. `quants`), advective flux Q v.n
plus a diffusive flux (eqs. `dynfluxes`, `diffflux`, `Fdiffmom`) and explicit
sources (curvature and gravity, eq. `sources`), with drag toward the gas
velocity solved implicitly (eq. `dragforce`, stopping time eq. `t_stop`).
One step follows the eight stages listed after eq. `t_stop` (first-order
fluxes at t^n, half update, half source and drag; second-order fluxes at
t^{n+1/2}, full update from Q^n, full source and drag); the Riemann flux is
eq. `riemann` with the Roe-averaged speed of eq. `roeav`; the time step is the
CFL rule, eqs. `dtCFL`, `dt_adv`, `dt_diff`.

Readings where the paper leaves the discretisation open:

* Grid (Sec. 7's poloidal grid): cells bounded by cylinders R = const and
  cones Z = t R (t = tan of the angle above the midplane), cell (i, j) at
  R in [R_e[i], R_e[i+1]], t in [t_e[j], t_e[j+1]], t_e[0] = 0 the
  midplane.  Volume (2 pi / 3)(R+^3 - R-^3)(t+ - t-); a cylinder face at R_f
  has area 2 pi R_f^2 (t+ - t-) and normal +R; a cone face at t has area
  pi (R+^2 - R-^2) sqrt(1 + t^2) and unit normal (-t, 1) / sqrt(1 + t^2).
  Cell centre R_c = sqrt(R- R+), t_c = (t- + t+) / 2, Z_c = t_c R_c.
* The angular momentum per unit mass is v_phi R with R = R_c in a cell,
  R_f on a cylinder face and the area-weighted mean radius
  (2/3)(R+^3 - R-^3)/(R+^2 - R-^2) on a cone face.
* Boundaries: zero-gradient copies at both radial edges and the top; the
  midplane mirrors the first cell with v_Z reversed.
* Riemann flux: a diverging pair (v_l.n < 0 < v_r.n) carries no flux whatever
  the Roe average says; the Roe average of two empty states is 0.
* Second-order reconstruction: piecewise linear in each primitive (rho, v_R,
  v_phi, v_Z) along each grid direction (coordinate R, resp. t), slope the van
  Leer harmonic mean 2 a b / (a + b) of the two one-sided gradients (0 where
  they differ in sign), the non-uniform-grid form of the limiter.
* Diffusion: flux -(rho_g nu / Sc)_f (eps_r - eps_l) / d with eps = rho / rho_g,
  (rho_g nu)_f the mean of the two cells, d = n . (x_r - x_l) the normal
  distance of the two cell centres; zero through every boundary face.  The
  momentum components carry it with the advected quantity per unit mass of
  the left or right state by its sign (eq. `Fdiffmom` read as F_diff times
  v_R, v_phi R, v_Z).
* Primitives of an empty cell (rho <= 0): velocity 0.
* Dust floor (optional, off by default): a species below eps_floor rho_g in
  a cell at the end of either stage takes the gas velocity; its density is
  kept, so mass stays conserved (`at_floor`).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SQRT_8_OVER_PI = np.sqrt(8.0 / np.pi)


@dataclass
class Geometry:
    """Cell and face geometry of the (R, t) grid (see the module docstring)."""
    R_e: np.ndarray        # [nr + 1]
    t_e: np.ndarray        # [nz + 1]
    Rc: np.ndarray         # [nr]
    tc: np.ndarray         # [nz]
    Zc: np.ndarray         # [nr, nz]
    V: np.ndarray          # [nr, nz]
    AR: np.ndarray         # [nr + 1, nz] cylinder faces
    At: np.ndarray         # [nr, nz + 1] cone faces
    Rcone: np.ndarray      # [nr] area-weighted radius of the cone faces of ring i

    @property
    def nr(self):
        return self.Rc.shape[0]

    @property
    def nz(self):
        return self.tc.shape[0]


def geometry(R_e, t_e) -> Geometry:
    R_e = np.asarray(R_e, dtype=np.float64)
    t_e = np.asarray(t_e, dtype=np.float64)
    Rm, Rp = R_e[:-1], R_e[1:]
    tm, tp = t_e[:-1], t_e[1:]
    Rc = np.sqrt(Rm * Rp)
    tc = 0.5 * (tm + tp)
    V = (2.0 * np.pi / 3.0) * (Rp ** 3 - Rm ** 3)[:, None] * (tp - tm)[None, :]
    AR = 2.0 * np.pi * (R_e ** 2)[:, None] * (tp - tm)[None, :]
    At = np.pi * (Rp ** 2 - Rm ** 2)[:, None] * np.sqrt(1.0 + t_e ** 2)[None, :]
    Rcone = (2.0 / 3.0) * (Rp ** 3 - Rm ** 3) / (Rp ** 2 - Rm ** 2)
    return Geometry(R_e, t_e, Rc, tc, tc[None, :] * Rc[:, None], V, AR, At, Rcone)


@dataclass
class Gas:
    """Gas state per cell [nr, nz]: density, sound speed, viscosity
    nu = alpha c_s H, velocity [nr, nz, 3] (v_R, v_phi, v_Z); G M_*."""
    rho_g: np.ndarray
    c_s: np.ndarray
    nu: np.ndarray
    v_g: np.ndarray
    GM: float
    Sc: float = 1.0


# ---------------------------------------------------------------------------
# primitives <-> conserved (eq. `quants`)
# ---------------------------------------------------------------------------
def conserved(rho, v, R):
    """Q [..., 4] from rho [...] and v [..., 3] with the radius R of the
    angular momentum (broadcast against rho)."""
    return np.stack([rho, rho * v[..., 0], rho * v[..., 1] * R, rho * v[..., 2]], axis=-1)


def primitive(Q, R):
    rho = Q[..., 0]
    v = np.zeros(Q.shape[:-1] + (3,))
    pos = rho > 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        v[..., 0] = np.where(pos, Q[..., 1] / rho, 0.0)
        v[..., 1] = np.where(pos, Q[..., 2] / (rho * R), 0.0)
        v[..., 2] = np.where(pos, Q[..., 3] / rho, 0.0)
    return rho, v


# ---------------------------------------------------------------------------
# Riemann flux of a pressureless fluid (eqs. `roeav`, `riemann`)
# ---------------------------------------------------------------------------
def riemann(Ql, Qr, vl, vr, rl, rr):
    """Advective flux [..., 4] through a face from the left and right
    conserved states Q, their normal velocities v and densities r."""
    sl, sr = np.sqrt(np.maximum(rl, 0.0)), np.sqrt(np.maximum(rr, 0.0))
    den = sl + sr
    with np.errstate(divide="ignore", invalid="ignore"):
        vhat = np.where(den > 0.0, (sl * vl + sr * vr) / den, 0.0)
    Fl = Ql * vl[..., None]
    Fr = Qr * vr[..., None]
    F = np.where((vhat > 0.0)[..., None], Fl, np.where((vhat < 0.0)[..., None], Fr, 0.5 * (Fl + Fr)))
    diverging = (vl < 0.0) & (vr > 0.0)
    return np.where(diverging[..., None], 0.0, F)


# ---------------------------------------------------------------------------
# neighbours with the boundary rules
# ---------------------------------------------------------------------------
def _padded(g: Geometry, rho, v):
    """rho, v with two ghost layers on every side: [nr + 4, nz + 4, N(, 3)]."""
    nr, nz = g.nr, g.nz
    ri = np.clip(np.arange(-2, nr + 2), 0, nr - 1)
    rj = np.arange(-2, nz + 2)
    mirror = rj < 0
    rj_src = np.where(mirror, np.minimum(-rj - 1, nz - 1), np.minimum(rj, nz - 1))
    rho_p = rho[ri][:, rj_src]
    v_p = v[ri][:, rj_src].copy()
    v_p[:, mirror, :, 2] *= -1.0
    return rho_p, v_p


def _coords(g: Geometry):
    """Cell coordinates along each direction including ghosts: R [nr + 4]
    (ghosts mirrored about the edge faces), t [nz + 4] (ghosts mirrored about
    the midplane below and the top face above)."""
    nr, nz = g.nr, g.nz
    R = np.empty(nr + 4)
    R[2:-2] = g.Rc
    R[1] = 2 * g.R_e[0] - g.Rc[0]
    R[0] = 2 * g.R_e[0] - g.Rc[1] if nr > 1 else 2 * g.R_e[0] - g.Rc[0] - (g.R_e[1] - g.R_e[0])
    R[-2] = 2 * g.R_e[-1] - g.Rc[-1]
    R[-1] = 2 * g.R_e[-1] - g.Rc[-2] if nr > 1 else R[-2] + (g.R_e[1] - g.R_e[0])
    t = np.empty(nz + 4)
    t[2:-2] = g.tc
    t[1] = -g.tc[0]
    t[0] = -g.tc[1] if nz > 1 else -g.tc[0] - (g.t_e[1] - g.t_e[0])
    t[-2] = 2 * g.t_e[-1] - g.tc[-1]
    t[-1] = 2 * g.t_e[-1] - g.tc[-2] if nz > 1 else t[-2] + (g.t_e[1] - g.t_e[0])
    return R, t


def _vanleer(a, b):
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(a * b > 0.0, 2.0 * a * b / (a + b), 0.0)


# ---------------------------------------------------------------------------
# total outward flux x area of every cell (the (FA) of eq. `fluxarea`)
# ---------------------------------------------------------------------------
def flux_area(g: Geometry, gas: Gas, rho, v, order):
    """(FA) [nr, nz, N, 4]: advective (order 1: donor cell; order 2:
    piecewise-linear states) plus diffusive fluxes, times face areas, summed
    over each cell's four faces, outward positive."""
    nr, nz, N = rho.shape
    rp, vp = _padded(g, rho, v)
    Rx, tx = _coords(g)
    prim = np.concatenate([rp[..., None], vp], axis=-1)        # [nr+4, nz+4, N, 4]
    if order == 2:
        # limited slopes along R (per unit R) and t (per unit t), cells incl. one ghost ring
        dR_l = (prim[1:-1] - prim[:-2]) / (Rx[1:-1] - Rx[:-2])[:, None, None, None]
        dR_r = (prim[2:] - prim[1:-1]) / (Rx[2:] - Rx[1:-1])[:, None, None, None]
        gR = np.zeros_like(prim)
        gR[1:-1] = _vanleer(dR_l, dR_r)
        dt_l = (prim[:, 1:-1] - prim[:, :-2]) / (tx[1:-1] - tx[:-2])[None, :, None, None]
        dt_r = (prim[:, 2:] - prim[:, 1:-1]) / (tx[2:] - tx[1:-1])[None, :, None, None]
        gt = np.zeros_like(prim)
        gt[:, 1:-1] = _vanleer(dt_l, dt_r)
    eps = rho / gas.rho_g[..., None]
    Dg = gas.rho_g * gas.nu / gas.Sc                             # [nr, nz]
    FA = np.zeros((nr, nz, N, 4))

    def face_flux(PL, PR, vnL, vnR, Rq, Fd):
        """total flux through one face (per unit area) from the left/right
        primitive states, their normal velocities, the face's angular
        momentum radius and the diffusive mass flux Fd."""
        QL = conserved(PL[..., 0], PL[..., 1:], Rq)
        QR = conserved(PR[..., 0], PR[..., 1:], Rq)
        F = riemann(QL, QR, vnL, vnR, PL[..., 0], PR[..., 0])
        wL = np.stack([np.ones_like(vnL), PL[..., 1], PL[..., 2] * Rq, PL[..., 3]], axis=-1)
        wR = np.stack([np.ones_like(vnR), PR[..., 1], PR[..., 2] * Rq, PR[..., 3]], axis=-1)
        return F + Fd[..., None] * np.where((Fd > 0.0)[..., None], wL, wR)

    # cylinder faces: face f between padded cells f + 1 (left) and f + 2 (right)
    for f in range(nr + 1):
        il, ir = f + 1, f + 2
        for j in range(nz):
            jj = j + 2
            PL = prim[il, jj].copy()
            PR = prim[ir, jj].copy()
            if order == 2:
                PL = PL + gR[il, jj] * (g.R_e[f] - Rx[il])
                PR = PR + gR[ir, jj] * (g.R_e[f] - Rx[ir])
            vnL, vnR = PL[..., 1], PR[..., 1]
            if 0 < f < nr:
                d = g.Rc[f] - g.Rc[f - 1]
                Dm = 0.5 * (Dg[f - 1, j] + Dg[f, j])
                Fd = -Dm * (eps[f, j] - eps[f - 1, j]) / d
            else:
                Fd = np.zeros(N)
            F = face_flux(PL, PR, vnL, vnR, g.R_e[f], Fd) * g.AR[f, j]
            if f > 0:
                FA[f - 1, j] += F
            if f < nr:
                FA[f, j] -= F
    # cone faces: face f between padded cells f + 1 (below) and f + 2 (above)
    for f in range(nz + 1):
        jl, jr = f + 1, f + 2
        t = g.t_e[f]
        nrm = np.array([-t, 1.0]) / np.sqrt(1.0 + t * t)
        for i in range(nr):
            ii = i + 2
            PL = prim[ii, jl].copy()
            PR = prim[ii, jr].copy()
            if order == 2:
                PL = PL + gt[ii, jl] * (t - tx[jl])
                PR = PR + gt[ii, jr] * (t - tx[jr])
            vnL = nrm[0] * PL[..., 1] + nrm[1] * PL[..., 3]
            vnR = nrm[0] * PR[..., 1] + nrm[1] * PR[..., 3]
            if 0 < f < nz:
                # normal distance of the two cell centres (same R_c, Z = t R_c)
                d = nrm[1] * g.Rc[i] * (g.tc[f] - g.tc[f - 1])
                Dm = 0.5 * (Dg[i, f - 1] + Dg[i, f])
                Fd = -Dm * (eps[i, f] - eps[i, f - 1]) / d
            else:
                Fd = np.zeros(N)
            F = face_flux(PL, PR, vnL, vnR, g.Rcone[i], Fd) * g.At[i, f]
            if f > 0:
                FA[i, f - 1] += F
            if f < nz:
                FA[i, f] -= F
    return FA


# ---------------------------------------------------------------------------
# sources and drag (eqs. `sources`, `dragforce`, `t_stop`)
# ---------------------------------------------------------------------------
def sources(g: Geometry, gas: Gas, rho, v):
    """Explicit sources [nr, nz, N, 4]: curvature and gravity (no external
    force; drag is implicit)."""
    R = g.Rc[:, None]
    Z = g.Zc
    om2 = gas.GM / (R * R + Z * Z) ** 1.5                       # [nr, nz]
    S = np.zeros(rho.shape + (4,))
    S[..., 1] = rho * v[..., 1] ** 2 / R[..., None] - rho * (om2 * R)[..., None]
    S[..., 3] = -rho * (om2 * Z)[..., None]
    return S


def stopping_time(gas: Gas, s, rho_m):
    """Epstein stopping time [nr, nz, N] of grains of radius s (eq. `t_stop`)."""
    v_th = SQRT_8_OVER_PI * gas.c_s
    return rho_m * np.asarray(s)[None, None, :] / (gas.rho_g * v_th)[..., None]


def drag(v, v_g, ts, h):
    """Implicit drag over h: v - h / (h + t_s) (v - v_g)."""
    return v - (h / (h + ts))[..., None] * (v - v_g[:, :, None, :])


# ---------------------------------------------------------------------------
# one step and the CFL time step
# ---------------------------------------------------------------------------
def at_floor(gas: Gas, rho, v, eps_floor):
    """The dust floor (a reading: Sec. 2 and Sec. 7 speak of floor values of
    the dust density and dust-to-gas ratio without giving them): a species
    whose density in a cell is below eps_floor rho_g moves with the gas; its
    density is kept.  eps_floor = 0: no floor."""
    if eps_floor <= 0.0:
        return v
    low = rho < eps_floor * gas.rho_g[..., None]
    return np.where(low[..., None], gas.v_g[:, :, None, :], v)


def step(g: Geometry, gas: Gas, s, rho_m, rho, v, dt, eps_floor=0.0):
    """One transport step of dt from (rho [nr, nz, N], v [nr, nz, N, 3]);
    returns the new (rho, v).  With eps_floor > 0 the floor applies to the
    state each of the two stages ends with."""
    Rq = g.Rc[:, None, None]
    ts = stopping_time(gas, s, rho_m)
    Q0 = conserved(rho, v, Rq)
    V = g.V[..., None, None]
    # (i)-(iv): first-order fluxes at t^n, half update, half source, drag
    Qs = Q0 - 0.5 * dt / V * flux_area(g, gas, rho, v, order=1)
    Qss = Qs + 0.5 * dt * sources(g, gas, rho, v)
    r_h, v_ss = primitive(Qss, Rq)
    v_h = at_floor(gas, r_h, drag(v_ss, gas.v_g, ts, 0.5 * dt), eps_floor)
    # (v)-(viii): second-order fluxes at t^{n+1/2}, full update from Q^n
    Qd = Q0 - dt / V * flux_area(g, gas, r_h, v_h, order=2)
    Qdd = Qd + dt * sources(g, gas, r_h, v_h)
    r1, v_dd = primitive(Qdd, Rq)
    v1 = at_floor(gas, r1, drag(v_dd, gas.v_g, ts, dt), eps_floor)
    return r1, v1


def cfl_dt(g: Geometry, gas: Gas, v, c_adv=0.4, c_diff=0.2):
    """eqs. `dtCFL`, `dt_adv`, `dt_diff`: dR the cell's radial width, dZ its
    height at R_c; velocities that are zero impose no limit."""
    dR = (g.R_e[1:] - g.R_e[:-1])[:, None]                       # [nr, 1]
    dZ = g.Rc[:, None] * (g.t_e[1:] - g.t_e[:-1])[None, :]        # [nr, nz]
    with np.errstate(divide="ignore"):
        a = np.minimum(np.abs(dR[..., None] / v[..., 0]), np.abs(dZ[..., None] / v[..., 2]))
        k = gas.nu / gas.Sc
        d = np.minimum(dR ** 2 / k, dZ ** 2 / k)
    return float(min(c_adv * np.min(a), c_diff * np.min(d)))
