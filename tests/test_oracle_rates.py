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
