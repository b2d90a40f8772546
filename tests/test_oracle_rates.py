"""Pins of the oracle's pair rates (Sec. 5, eqs. `kernel`, `vbrown`, `OCVrel`,
`p_frag`; Stokes number from the Epstein stopping time, eq. `t_stop`).

The pins are independent of the oracle's code: a Monte-Carlo estimate of the
mean relative speed of two Maxwellian grains, the published asymptotes of the
Ormel & Cuzzi relative velocity, and the Gamma(2) survival function from scipy
for the Maxwellian fragmentation probability.
"""
import os

import numpy as np
import pytest
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
YSTAR = 1.6
K_B = 1.380649e-16


def _unit_cells(C, T=0.0, alpha=1e-3, Re=1e8):
    """Cells where St_k equals the grain radius s_k (rho_m = rho_g = Omega =
    v_th = 1) and Re is chosen directly."""
    c_s = np.sqrt(np.pi / 8.0)
    H = 1.0
    nu = alpha * c_s * H / Re
    one = np.ones(C)
    return dict(T=T * one, rho_g=one, c_s=c_s * one, Omega=one, H=H * one,
                nu_mol=nu * one, alpha=alpha * one)


def _stokes_grid(O, lo, hi, N=16):
    m, me, s = O.mass_grid(N, lo, hi, rho_m=1.0)
    return O.Grid(m, me, s, 1.0)


def _vrel2(O, g, Re, alpha=1e-3):
    """V_rel^2 recovered from K with T = 0, no laminar motion, v_frag = 0."""
    cells = _unit_cells(1, 0.0, alpha, Re)
    Kc, Kf = O.rates(g, cells, np.zeros((1, g.N, 3)), 0.0)
    assert np.all(Kc == 0)
    out = {}
    for i in range(g.N):
        for j in range(i + 1):
            p = i * (i + 1) // 2 + j
            w = 0.5 if i == j else 1.0
            sig = np.pi * (g.s[i] + g.s[j]) ** 2
            dv = Kf[0, p] / (w * sig)
            out[(i, j)] = dv * dv / (alpha * cells["c_s"][0] ** 2)
    return out


def test_golden_file_lists_three_limits():
    names = [l.split()[0] for l in open(os.path.join(GOLDEN, "ormel_cuzzi_limits.txt"))
             if l.strip() and not l.startswith("#")]
    assert names == ["tiny", "intermediate_eq", "heavy"]


def test_oc_tiny_grains(O):
    """St_1, St_2 << Re^-1/2: V_rel^2 -> (St_1 - St_2)^2 Re^1/2."""
    Re = 1e8
    delta = Re ** -0.5
    g = _stokes_grid(O, 1e-9 * delta * 1e3, 1e-3 * delta)
    v = _vrel2(O, g, Re)
    for (i, j), val in v.items():
        if i == j:
            assert val == 0.0
            continue
        lim = (g.s[i] - g.s[j]) ** 2 / delta
        np.testing.assert_allclose(val, lim, rtol=3e-3)


def test_oc_intermediate_equal_sizes(O):
    """delta << St << 1, equal sizes: V_rel^2 -> (2y* - 2 + 2/(1+y*)) St."""
    Re = 1e14
    g = _stokes_grid(O, 1e-4, 1e-2)
    v = _vrel2(O, g, Re)
    coef = 2 * YSTAR - 2 + 2 / (1 + YSTAR)
    assert abs(coef - 1.9692307692307693) < 1e-15
    for i in range(g.N):
        np.testing.assert_allclose(v[(i, i)], coef * g.s[i], rtol=1e-5)


def test_oc_heavy_grains(O):
    """St_1, St_2 >> 1: V_rel^2 -> 1/(1+St_1) + 1/(1+St_2)."""
    Re = 1e14
    g = _stokes_grid(O, 1e2, 1e5)
    v = _vrel2(O, g, Re)
    for (i, j), val in v.items():
        lim = 1 / (1 + g.s[i]) + 1 / (1 + g.s[j])
        np.testing.assert_allclose(val, lim, rtol=1e-6)


def _two_bin_grid(O, st2, st1):
    s = np.array([st2, st1])
    m = 4 / 3 * np.pi * s ** 3
    r = m[1] / m[0]
    me = np.array([m[0] / np.sqrt(r), np.sqrt(m[0] * m[1]), m[1] * np.sqrt(r)])
    return O.Grid(m, me, s, 1.0)


@pytest.mark.parametrize("which", ["lower", "upper"])
def test_oc_continuous_across_clamps(O, which):
    """St* = clamp(y* St_1, Re^-1/2, 1) is continuous, so V_rel^2 is continuous
    where the clamp switches: approach y* St_1 = delta and y* St_1 = 1 from
    both sides and watch the difference vanish linearly."""
    Re = 1e6
    delta = Re ** -0.5
    edge = (delta if which == "lower" else 1.0) / YSTAR
    prev = None
    for eps in (1e-4, 1e-6, 1e-8):
        lo = _vrel2(O, _two_bin_grid(O, 0.3 * edge, edge * (1 - eps)), Re)[(1, 0)]
        hi = _vrel2(O, _two_bin_grid(O, 0.3 * edge, edge * (1 + eps)), Re)[(1, 0)]
        d = abs(hi - lo) / hi
        if prev is not None:
            assert d < prev * 0.05          # shrinks ~ eps
        prev = d
    assert prev < 1e-6


def test_brownian_matches_maxwellian_monte_carlo(O):
    """alpha = 0, no laminar motion: Delta v is the mean relative speed of two
    Maxwellian grains of masses m_i, m_j at temperature T, estimated here by
    sampling (4e6 pairs; standard error ~2e-4)."""
    T = 50.0
    N = 6
    m, me, s = O.mass_grid(N, 1e-6, 1e-4, rho_m=1.67)
    g = O.Grid(m, me, s, 1.67)
    cells = _unit_cells(1, T=T, alpha=0.0)
    Kc, Kf = O.rates(g, cells, np.zeros((1, N, 3)), 1e30)   # v_frag huge: p_coag = 1
    assert np.all(Kf == 0)
    rng = np.random.default_rng(11)
    for (i, j) in [(0, 0), (3, 1), (5, 0), (5, 5)]:
        p = i * (i + 1) // 2 + j
        w = 0.5 if i == j else 1.0
        dv = Kc[0, p] / (w * np.pi * (s[i] + s[j]) ** 2)
        n = 4_000_000
        vi = rng.normal(0, np.sqrt(K_B * T / m[i]), (n, 3))
        vj = rng.normal(0, np.sqrt(K_B * T / m[j]), (n, 3))
        mc = np.linalg.norm(vi - vj, axis=1).mean()
        np.testing.assert_allclose(dv, mc, rtol=1.5e-3)


def test_pfrag_is_gamma2_survival(O):
    """p_frag = (1 + y) e^-y with y = 1.5 (v_frag/Delta v)^2 is the survival
    function of Gamma(2, 1) at y; p_coag = 1 - p_frag is its CDF (this pins
    the small-y series branch too).  At Delta v = v_frag, p_frag = 2.5 e^-1.5."""
    g = O.make_grid(30, 1e-5, 10.0)
    rng = np.random.default_rng(3)
    C = 4
    cells = dict(T=np.full(C, 30.0), rho_g=np.full(C, 1e-11), c_s=np.full(C, 4e4),
                 Omega=np.full(C, 1e-8), H=np.full(C, 1e13), nu_mol=np.full(C, 1e5),
                 alpha=np.full(C, 1e-3))
    v = rng.normal(0, 50, (C, g.N, 3))
    vfrag = np.array([1.0, 100.0, 1000.0, 1e5])
    Kc, Kf = O.rates(g, cells, v, vfrag)
    K = Kc + Kf
    pf = Kf / K
    w = np.array([0.5 if i == j else 1.0 for i in range(g.N) for j in range(i + 1)])
    sig = np.array([np.pi * (g.s[i] + g.s[j]) ** 2 for i in range(g.N) for j in range(i + 1)])
    dv = K / (w * sig)
    y = 1.5 * (vfrag[:, None] / dv) ** 2
    # y is rebuilt here from K with a relative error of a few ulp, which the
    # exponential turns into ~y ulp of p_frag
    sf = stats.gamma.sf(y, 2)
    assert np.all(np.abs(pf - sf) <= 1e-14 * (1 + y) * sf + 1e-300)
    pc = Kc / K
    big = pc > 1e-280
    np.testing.assert_allclose(pc[big], stats.gamma.cdf(y, 2)[big], rtol=5e-12)
    assert np.all((pf >= 0) & (pf <= 1) & (pc >= 0) & (pc <= 1))
    assert abs(stats.gamma.sf(1.5, 2) - 2.5 * np.exp(-1.5)) < 4e-16
    # special point Delta v = v_frag: re-run cell 1 with v_frag set to one pair's speed
    p0 = 37
    Kc1, Kf1 = O.rates(g, {k: v_[1:2] for k, v_ in cells.items()}, v[1:2], dv[1, p0])
    np.testing.assert_allclose(Kf1[0, p0] / (Kc1[0, p0] + Kf1[0, p0]), 2.5 * np.exp(-1.5),
                               rtol=4e-15)
    # series and direct branch agree across the switch at y = 1e-2 within the
    # cancellation error of 1 - p_frag there (~ eps / (y^2/2))
    near = (y > 0.5e-2) & (y < 2e-2)
    if near.any():
        np.testing.assert_allclose(pc[near], stats.gamma.cdf(y[near], 2), rtol=2e-11)


def test_rates_nonnegative_and_finite_on_disc(O):
    from paper_2402_18471_amd import disc
    cfg = disc.scaled(disc.CONFIGS["disc512x256_n200"], 8, 4, 40)
    g = O.make_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    d = disc.make_disc(cfg, g.s)
    Kc, Kf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    assert np.all(np.isfinite(Kc)) and np.all(np.isfinite(Kf))
    assert np.all(Kc >= 0) and np.all(Kf >= 0) and np.all(Kc + Kf > 0)


# A cell whose gas state has no unit values and no two equal ones, so that a
# factor put in the wrong place (rho_m for rho_g, Omega divided instead of
# multiplied, c_s missing from v_th, H missing from Re) changes the Stokes or
# Reynolds number by orders of magnitude.
_RHO_M, _RHO_G, _OMEGA, _C_S, _H = 3.3, 2.1e-2, 0.13, 23.0, 2.3


def _physical_cell(alpha, Re):
    """One cell with the distinct values above; nu_mol set so that
    Re = alpha c_s H / nu_mol (Sec. 7.1) takes the requested value."""
    nu = alpha * _C_S * _H / Re
    one = np.ones(1)
    return dict(T=0.0 * one, rho_g=_RHO_G * one, c_s=_C_S * one, Omega=_OMEGA * one,
                H=_H * one, nu_mol=nu * one, alpha=alpha * one)


def _stokes(s):
    """St = t_s Omega with the Epstein stopping time of eq. `t_stop` (Sec. 3.1),
    t_s = rho_m s / (rho_g v_th), v_th = (8/pi)^1/2 c_s; written out here,
    independently of the oracle."""
    v_th = np.sqrt(8.0 / np.pi) * _C_S
    return _RHO_M * s / (_RHO_G * v_th) * _OMEGA


def _grid_for_stokes(O, st_lo, st_hi, N=16):
    """Grid whose bins span the Stokes numbers [st_lo, st_hi] in the cell above."""
    per_cm = _stokes(1.0)
    m, me, s = O.mass_grid(N, st_lo / per_cm, st_hi / per_cm, rho_m=_RHO_M)
    return O.Grid(m, me, s, _RHO_M)


def _vrel2_physical(O, g, alpha, Re):
    """V_rel^2 recovered from K (T = 0, no laminar motion, v_frag = 0 so that
    every collision fragments and K = w sigma sqrt(alpha) c_s V_rel)."""
    cells = _physical_cell(alpha, Re)
    Kc, Kf = O.rates(g, cells, np.zeros((1, g.N, 3)), 0.0)
    assert np.all(Kc == 0)
    out = {}
    for i in range(g.N):
        for j in range(i + 1):
            p = i * (i + 1) // 2 + j
            w = 0.5 if i == j else 1.0
            dv = Kf[0, p] / (w * np.pi * (g.s[i] + g.s[j]) ** 2)
            out[(i, j)] = dv * dv / (alpha * _C_S ** 2)
    return out


def test_stokes_and_reynolds_numbers_in_a_physical_cell(O):
    """The Ormel & Cuzzi limits at Stokes and Reynolds numbers computed here
    from the cell's rho_m, rho_g, Omega, c_s, H and nu_mol (eq. `t_stop`,
    Re = nu_t / nu_mol with nu_t = alpha c_s H): tiny grains give
    V_rel^2 -> Re^1/2 (St_1 - St_2)^2, equal intermediate grains
    V_rel^2 -> (2 y* - 2 + 2/(1 + y*)) St, heavy grains 1/(1+St_1) + 1/(1+St_2).
    Swapping rho_m and rho_g, or dropping c_s, Omega or H, moves St or Re by
    a factor of 10 or more and fails these by far more than their tolerance."""
    alpha = 2.7e-3
    # tiny: St << Re^-1/2 (Re = 1e8, delta = 1e-4)
    Re = 1e8
    delta = Re ** -0.5
    g = _grid_for_stokes(O, 1e-6 * delta, 1e-3 * delta)
    st = _stokes(g.s)
    v = _vrel2_physical(O, g, alpha, Re)
    for (i, j), val in v.items():
        if i != j:
            np.testing.assert_allclose(val, (st[i] - st[j]) ** 2 / delta, rtol=3e-3)
    # intermediate, equal sizes: delta << St << 1 (Re = 1e14)
    Re = 1e14
    g = _grid_for_stokes(O, 1e-4, 1e-2)
    st = _stokes(g.s)
    v = _vrel2_physical(O, g, alpha, Re)
    coef = 2 * YSTAR - 2 + 2 / (1 + YSTAR)
    for i in range(g.N):
        np.testing.assert_allclose(v[(i, i)], coef * st[i], rtol=1e-5)
    # heavy: St >> 1
    g = _grid_for_stokes(O, 1e2, 1e5)
    st = _stokes(g.s)
    v = _vrel2_physical(O, g, alpha, Re)
    for (i, j), val in v.items():
        np.testing.assert_allclose(val, 1 / (1 + st[i]) + 1 / (1 + st[j]), rtol=1e-6)
    # the chosen values really separate the factors: each misplacement moves
    # St by at least a factor 10
    base = _stokes(1.0)
    v_th = np.sqrt(8 / np.pi) * _C_S
    for wrong in (_RHO_G * 1.0 / (_RHO_M * v_th) * _OMEGA,      # rho_m <-> rho_g
                  _RHO_M / (_RHO_G * v_th) / _OMEGA,              # Omega divided
                  _RHO_M / (_RHO_G * np.sqrt(8 / np.pi)) * _OMEGA):  # c_s dropped
        assert max(wrong / base, base / wrong) > 10


def test_reynolds_number_sets_the_smallest_eddy(O):
    """Tiny-grain limit at two Reynolds numbers 100 apart in the same cell
    (only nu_mol changes): V_rel^2 scales as Re^1/2, i.e. by 10."""
    alpha = 2.7e-3
    g = _grid_for_stokes(O, 1e-12, 1e-9)
    a = _vrel2_physical(O, g, alpha, 1e8)
    b = _vrel2_physical(O, g, alpha, 1e10)
    for key in a:
        if key[0] != key[1]:
            np.testing.assert_allclose(b[key] / a[key], 10.0, rtol=1e-3)
