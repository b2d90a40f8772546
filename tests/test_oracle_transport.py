"""Pins of the transport oracle (Sec. 3, dynamics solver) against what the
mathematics fixes: the Riemann flux's special cases (upwinding, the Roe
average of eq. `roeav`, a diverging pair), exact conservation of mass, the
closed form of the implicit drag over a full two-stage step, second-order
convergence to the exact solution of radial advection in cylindrical
geometry, the spreading of a diffusing ring at the rate its viscosity sets,
the sign and size of gravity and curvature from rest, and the CFL rule's
limits."""
import numpy as np
import pytest

from oracle import transport as T


def _grid(nr, nz, R0=1.0, R1=2.0, t1=0.2, log=False):
    R_e = np.geomspace(R0, R1, nr + 1) if log else np.linspace(R0, R1, nr + 1)
    t_e = np.linspace(0.0, t1, nz + 1)
    return T.geometry(R_e, t_e)


def _gas(g, rho_g=1.0, c_s=1.0, nu=0.0, v_g=(0.0, 0.0, 0.0), GM=0.0):
    shape = (g.nr, g.nz)
    vg = np.zeros(shape + (3,))
    vg[...] = v_g
    return T.Gas(np.full(shape, rho_g), np.full(shape, c_s), np.full(shape, nu), vg, GM)


# ---------------------------------------------------------------------------
# Riemann flux (eqs. `roeav`, `riemann`)
# ---------------------------------------------------------------------------
def _riemann(rl, vl, rr, vr):
    Ql = np.array([[rl, 2.0 * rl, 3.0 * rl, 4.0 * rl]])
    Qr = np.array([[rr, 5.0 * rr, 6.0 * rr, 7.0 * rr]])
    return T.riemann(Ql, Qr, np.array([vl]), np.array([vr]), np.array([rl]), np.array([rr]))[0]


def test_riemann_upwinds_with_the_roe_average():
    # both moving right: the left state's flux; both left: the right state's
    assert np.array_equal(_riemann(2.0, 1.0, 3.0, 0.5), 2.0 * np.array([1, 2, 3, 4.0]) * 1.0)
    assert np.array_equal(_riemann(2.0, -1.0, 3.0, -0.5), 3.0 * np.array([1, 5, 6, 7.0]) * -0.5)
    # converging: the Roe speed weights by sqrt(rho), not rho.  rho_l = 4,
    # rho_r = 1, v_l = 1: v_r = -1.5 gives (2 - 1.5) / 3 > 0 (left state),
    # v_r = -2.5 gives (2 - 2.5) / 3 < 0 (right), where a rho-weighted mean
    # (4 - 2.5) / 5 would still say left
    assert np.array_equal(_riemann(4.0, 1.0, 1.0, -1.5), 4.0 * np.array([1, 2, 3, 4.0]))
    assert np.array_equal(_riemann(4.0, 1.0, 1.0, -2.5), 1.0 * np.array([1, 5, 6, 7.0]) * -2.5)
    # symmetric collision: the Roe speed is 0, the mean of the two fluxes
    f = _riemann(1.0, 1.0, 1.0, -1.0)
    assert np.allclose(f, 0.5 * (np.array([1, 2, 3, 4.0]) - np.array([1, 5, 6, 7.0])), rtol=0, atol=0)
    # diverging (vacuum opens): no flux, whatever the Roe speed
    assert np.array_equal(_riemann(4.0, -0.1, 1.0, 3.0), np.zeros(4))
    # two empty states
    assert np.array_equal(_riemann(0.0, 1.0, 0.0, -1.0), np.zeros(4))


# ---------------------------------------------------------------------------
# conservation and uniform states
# ---------------------------------------------------------------------------
def test_uniform_state_at_rest_is_unchanged():
    g = _grid(6, 4)
    gas = _gas(g, nu=0.3)
    rho = np.full((6, 4, 3), 2.5)
    v = np.zeros((6, 4, 3, 3))
    r1, v1 = T.step(g, gas, np.array([1e-4, 1e-3, 1e-2]), 1.6, rho, v, 0.01)
    assert np.array_equal(r1, rho) and np.array_equal(v1, v)


def test_mass_is_conserved_when_nothing_reaches_the_edges():
    """Random flow and diffusion inside a disc whose outer two rings and top
    two layers are empty: the midplane mirror passes no mass, so sum V rho is
    constant to rounding over several steps (a flux added to one cell and not
    taken from its neighbour, or with a different area, breaks this)."""
    rng = np.random.default_rng(7)
    nr, nz, N = 14, 9, 3
    g = _grid(nr, nz, log=True)
    gas = _gas(g, nu=0.05, GM=0.5)
    gas.rho_g = rng.uniform(0.5, 2.0, (nr, nz))
    gas.c_s = rng.uniform(0.5, 1.0, (nr, nz))
    rho = rng.uniform(0.0, 1.0, (nr, nz, N))
    # mass spreads by at most two cells a step (first-order half step, then
    # the full step's fluxes of the half-stepped state)
    rho[:5] = rho[-5:] = 0.0
    rho[:, -5:] = 0.0
    v = rng.normal(0.0, 0.3, (nr, nz, N, 3))
    s = np.array([1e-3, 1e-2, 1e-1])
    m0 = np.sum(g.V[..., None] * rho)
    for _ in range(2):
        dt = 0.2 * T.cfl_dt(g, gas, v)
        rho, v = T.step(g, gas, s, 1.6, rho, v, dt)
    assert np.all(rho[0] == 0.0) and np.all(rho[-1] == 0.0) and np.all(rho[:, -1] == 0.0)
    assert np.any(rho[1:-1, 0] > 0.0)
    assert abs(np.sum(g.V[..., None] * rho) - m0) <= 1e-14 * m0


# ---------------------------------------------------------------------------
# drag (eqs. `dragforce`, `t_stop`) over the full step
# ---------------------------------------------------------------------------
def test_drag_over_a_step_is_implicit_euler_from_the_old_state():
    """Uniform density and radial velocity far from the axis (R ~ 1e6, where
    the geometric divergence U / R of a uniform flow is 1e-6), no gravity:
    every flux of momentum is the velocity times the mass flux, so the
    velocity stays uniform through the fluxes to ~1e-8 and the step reduces to
    the drag, v1 - v_g = (v0 - v_g) t_s / (dt + t_s) with t_s = rho_m s /
    (rho_g v_th), v_th = sqrt(8 / pi) c_s.  Restarting the second stage from
    the half-stepped state instead of Q^n would apply the drag one and a half
    times; an explicit drag, or h / t_s, would miss by O(1)."""
    g = T.geometry(np.linspace(1e6, 1e6 + 5.0, 6), np.linspace(0.0, 3e-6, 4))
    v_g = np.array([0.2, 0.3, 0.0])
    gas = _gas(g, rho_g=3.0, c_s=2.0, v_g=v_g)
    s = np.array([0.5, 2.0, 8.0])
    rho_m = 1.5
    rho = np.full((5, 3, 3), 1.0)
    v0 = np.array([1.0, 0.0, 0.0])
    v = np.broadcast_to(v0, (5, 3, 3, 3)).copy()
    dt = 0.05
    r1, v1 = T.step(g, gas, s, rho_m, rho, v, dt)
    ts = rho_m * s / (3.0 * np.sqrt(8.0 / np.pi) * 2.0)
    want = v_g[None, :] + (v0 - v_g)[None, :] * (ts / (dt + ts))[:, None]      # [N, 3]
    assert np.allclose(v1, np.broadcast_to(want, v1.shape), rtol=1e-7, atol=1e-9)


# ---------------------------------------------------------------------------
# advection: second-order convergence to the exact cylindrical solution
# ---------------------------------------------------------------------------
def _advect_error(nr):
    """Radial advection at constant speed U, no Z motion, no forces or
    diffusion: d rho / dt + (1/R) d(R rho U)/dR = 0 has the exact solution
    rho(R, t) = rho0(R - U t) (R - U t) / R for any Z, which the cone faces
    must reproduce too (their normals see v_R)."""
    U, t_end = 1.0, 0.25
    g = _grid(nr, 2, R0=1.0, R1=2.0, t1=0.1)
    gas = _gas(g, v_g=(U, 0.0, 0.0))           # drag toward U: a no-op
    rho0 = lambda R: np.exp(-0.5 * ((R - 1.35) / 0.07) ** 2)
    rho = np.repeat(rho0(g.Rc)[:, None, None], 2, axis=1)
    v = np.zeros((nr, 2, 1, 3))
    v[..., 0] = U
    n = int(round(t_end / (0.4 * (g.R_e[1] - g.R_e[0]) / U)))
    dt = t_end / n
    for _ in range(n):
        rho, v = T.step(g, gas, np.array([1.0]), 1.0, rho, v, dt)
    exact = rho0(g.Rc - U * t_end) * (g.Rc - U * t_end) / g.Rc
    return np.sqrt(np.mean((rho[:, :, 0] - exact[:, None]) ** 2))


def test_radial_advection_converges_at_second_order():
    e = [_advect_error(n) for n in (40, 80, 160)]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert r2 > 3.0 and r1 > 2.5, (e, r1, r2)
    assert e[2] < 3e-3


# ---------------------------------------------------------------------------
# diffusion (eq. `diffflux`)
# ---------------------------------------------------------------------------
def test_a_ring_diffuses_at_the_rate_nu_sets():
    """A narrow Gaussian ring far from the axis (width / R = 0.2 %) in a
    uniform gas at rest: the radial variance grows by 2 nu t (Sc = 1), to the
    few per cent that the ring's curvature and the grid leave."""
    nu = 0.02
    g = _grid(200, 1, R0=100.0, R1=104.0, t1=0.01)
    gas = _gas(g, nu=nu, rho_g=2.0)
    sig0 = 0.2
    rho = np.exp(-0.5 * ((g.Rc - 102.0) / sig0) ** 2)[:, None, None]
    v = np.zeros((200, 1, 1, 3))
    w = g.V[:, 0]

    def var(r):
        m = np.sum(w * r[:, 0, 0])
        mu = np.sum(w * r[:, 0, 0] * g.Rc) / m
        return np.sum(w * r[:, 0, 0] * (g.Rc - mu) ** 2) / m

    v0 = var(rho)
    t, t_end = 0.0, 1.0
    while t < t_end:
        dt = min(T.cfl_dt(g, gas, v), t_end - t)
        rho, v = T.step(g, gas, np.array([1.0]), 1.0, rho, v, dt)
        t += dt
    assert abs((var(rho) - v0) / (2.0 * nu * t_end) - 1.0) < 0.03
    assert np.all(rho >= 0.0)


def test_dust_in_step_with_the_gas_does_not_diffuse():
    """rho proportional to rho_g (uniform dust-to-gas ratio) has no diffusive
    flux, however rho_g varies; at rest and without gravity it stays put."""
    rng = np.random.default_rng(3)
    g = _grid(6, 5, log=True)
    gas = _gas(g, nu=0.7)
    gas.rho_g = rng.uniform(0.5, 3.0, (6, 5))
    rho = 0.01 * gas.rho_g[..., None] * np.array([1.0, 2.0])[None, None, :]
    v = np.zeros((6, 5, 2, 3))
    r1, v1 = T.step(g, gas, np.array([0.1, 0.2]), 1.0, rho, v, 0.01)
    assert np.array_equal(r1, rho) and np.array_equal(v1, v)


# ---------------------------------------------------------------------------
# gravity and curvature (eq. `sources`)
# ---------------------------------------------------------------------------
def test_gravity_from_rest_and_keplerian_balance():
    """From rest, without drag, the first step gives dv = -dt Omega^2 (R, Z)
    at the cell centre, Omega^2 = G M / (R^2 + Z^2)^{3/2}, up to O(dt^2); with
    v_phi^2 / R = Omega^2 R the radial kick vanishes to the same order."""
    g = _grid(4, 3, R0=1.0, R1=1.4, t1=0.15)
    GM = 2.0
    gas = _gas(g, rho_g=1e-30, c_s=1.0, GM=GM)           # t_s huge: no drag
    rho = np.ones((4, 3, 1))
    v = np.zeros((4, 3, 1, 3))
    R, Z = g.Rc[:, None], g.Zc
    om2 = GM / (R ** 2 + Z ** 2) ** 1.5
    for dt in (1e-3, 1e-4):
        _, v1 = T.step(g, gas, np.array([1.0]), 1.0, rho, v, dt)
        assert np.allclose(v1[..., 0, 0] / (-dt * om2 * R), 1.0, atol=20 * dt)
        assert np.allclose(v1[..., 0, 2] / (-dt * om2 * Z), 1.0, atol=20 * dt)
    vk = v.copy()
    vk[..., 0, 1] = np.sqrt(om2) * R
    dt = 1e-3
    _, v1 = T.step(g, gas, np.array([1.0]), 1.0, rho, vk, dt)
    assert np.all(np.abs(v1[..., 0, 0]) < 20 * dt * dt * om2 * R)


# ---------------------------------------------------------------------------
# CFL (eqs. `dtCFL`, `dt_adv`, `dt_diff`)
# ---------------------------------------------------------------------------
def test_cfl_limits():
    g = _grid(4, 2, R0=1.0, R1=2.0, t1=0.2)        # dR = 0.25; dZ = 0.1 R_c
    gas = _gas(g, nu=0.0)
    v = np.zeros((4, 2, 1, 3))
    v[1, 1, 0, 0] = -5.0
    assert T.cfl_dt(g, gas, v) == pytest.approx(0.4 * 0.25 / 5.0, rel=1e-15)
    v[2, 0, 0, 2] = 100.0
    assert T.cfl_dt(g, gas, v) == pytest.approx(0.4 * 0.1 * g.Rc[2] / 100.0, rel=1e-15)
    gas = _gas(g, nu=3.0)
    v[...] = 0.0
    assert T.cfl_dt(g, gas, v) == pytest.approx(0.2 * (0.1 * g.Rc[0]) ** 2 / 3.0, rel=1e-15)


# ---------------------------------------------------------------------------
# the dust floor (a reading: floor values are mentioned, not specified)
# ---------------------------------------------------------------------------
def test_floor_species_move_with_the_gas_and_stop_limiting_the_step():
    """A near-empty large-grain species (1e-30 of the gas density) with
    meaningless speeds: without a floor it keeps limiting the CFL step;
    with eps_floor = 1e-20 it ends each stage with the gas velocity, the
    species above the floor are untouched wherever their stencil (two cells
    each way) holds no floored cell (species do not interact in the transport
    step; floored neighbours change the limited slopes), mass is still
    conserved, and the next CFL step is set by the physical species.
    eps_floor = 0 is the step without a floor."""
    rng = np.random.default_rng(19)
    nr, nz, N = 20, 12, 4
    g = _grid(nr, nz, log=True)
    gas = _gas(g, nu=0.05, GM=0.5)
    gas.rho_g = rng.uniform(0.5, 2.0, (nr, nz))
    gas.c_s = rng.uniform(0.5, 1.0, (nr, nz))
    gas.v_g = rng.normal(0.0, 0.1, (nr, nz, 3))
    s = np.array([1e-3, 1e-2, 1e-1, 1.0])
    rho = rng.uniform(0.1, 1.0, (nr, nz, N))
    rho[..., 3] = 1e-30 * gas.rho_g
    rho[:5] = rho[-5:] = 0.0
    rho[:, -5:] = 0.0
    v = rng.normal(0.0, 0.3, (nr, nz, N, 3))
    v[..., 3, :] = rng.normal(0.0, 1e3, (nr, nz, 3))
    eps = 1e-20
    m0 = np.sum(g.V[..., None] * rho)
    dt = T.cfl_dt(g, gas, v)
    r0, v0 = T.step(g, gas, s, 1.6, rho, v, dt)
    r00, v00 = T.step(g, gas, s, 1.6, rho, v, dt, eps_floor=0.0)
    assert np.array_equal(r0, r00) and np.array_equal(v0, v00)
    r1, v1 = T.step(g, gas, s, 1.6, rho, v, dt, eps_floor=eps)
    low = r1 < eps * gas.rho_g[..., None]
    assert np.all(low[..., 3]) and not np.all(low[..., :3])
    assert np.array_equal(v1[low], np.broadcast_to(gas.v_g[:, :, None, :], v1.shape)[low])
    # cells 7..12 in R, 0..4 in Z: every cell within two of them is filled
    inner = (slice(7, 13), slice(0, 5), slice(0, 3))
    assert np.all(rho[5:15, :7, :3] > 0.0)
    assert np.array_equal(r1[inner], r0[inner]) and np.array_equal(v1[inner], v0[inner])
    assert np.all(r1 >= 0.0)
    assert abs(np.sum(g.V[..., None] * r1) - m0) <= 1e-14 * m0
    # the next step: limited by the near-empty species without the floor only
    assert T.cfl_dt(g, gas, v1) > 100.0 * T.cfl_dt(g, gas, v0)
    phys = T.cfl_dt(g, gas, np.where(low[..., None], 0.0, v1))
    assert T.cfl_dt(g, gas, v1) == pytest.approx(phys, rel=0.5)
