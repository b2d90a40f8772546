"""Pins of the oracle's vertically integrated kernel (Sec. 5.1: the kernel of
the single-radius comparison with DustPy, for surface densities).

Each species has a Gaussian vertical profile of scale height h_k; the column
collision rate is the volume rate integrated over height, so K is divided by
sqrt(2 pi (h_i^2 + h_j^2)), and the vertical relative velocity is the
difference of the terminal settling speeds St Omega Z at Z = h_k.  Pinned by:
  - the reduction to the volume kernel: the vertically integrated rates equal
    the oracle's volume rates, fed settling speeds as vertical velocities,
    over the overlap factor, both written out here from eq. `t_stop` and the
    scale-height formula h = H sqrt(alpha / (alpha + St));
  - the overlap factor against numerical quadrature of n_i(z) n_j(z);
  - well mixed grains (St << alpha): every h -> H, no settling, and the
    rates -> volume rates / sqrt(4 pi) H;
  - the midplane Stokes number of a column equals (pi / 2) rho_m s / Sigma_g;
  - the hand derivatives and the step adjoint against the complex step of
    the same forward formulas.
"""
import numpy as np
import pytest


def _columns(O, n_r=3, n_bins=12, s_min=3e-3, s_max=3e-2, r=(10.0, 40.0), drift=True,
             alpha=1e-3):
    from paper_2402_18471_amd import disc
    cfg = disc.ColumnConfig("t", n_r, n_bins, s_min, s_max, r[0], r[1], alpha=alpha,
                            drift=drift)
    gv = O.make_grid(n_bins, s_min, s_max, rho_m=cfg.rho_m, vertical=1)
    g3 = O.make_grid(n_bins, s_min, s_max, rho_m=cfg.rho_m, vertical=0)
    d = disc.make_columns(cfg, gv.s)
    return cfg, gv, g3, d


def _written_out(cfg, g, d):
    """St, h, settling speed per (column, bin), from eq. `t_stop` (Epstein,
    midplane) and h = H sqrt(alpha / (alpha + St))."""
    c = d["cells"]
    v_th = np.sqrt(8.0 / np.pi) * c["c_s"]
    St = cfg.rho_m * g.s[None, :] / (c["rho_g"] * v_th)[:, None] * c["Omega"][:, None]
    h = c["H"][:, None] * np.sqrt(c["alpha"][:, None] / (c["alpha"][:, None] + St))
    return St, h, St * c["Omega"][:, None] * h


def _pairs(N):
    i = np.repeat(np.arange(N), np.arange(1, N + 1))
    j = np.concatenate([np.arange(k + 1) for k in range(N)])
    return i, j


@pytest.mark.parametrize("case", ["0d", "drift", "wide"])
def test_vertical_rates_are_volume_rates_with_settling_over_the_overlap(O, case):
    if case == "0d":
        cfg, gv, g3, d = _columns(O, 1, 24, 1e-5, 100.0, (20.0, 20.0), drift=False)
    elif case == "drift":
        cfg, gv, g3, d = _columns(O)
    else:
        cfg, gv, g3, d = _columns(O, 4, 40, 1e-5, 100.0, (5.0, 100.0), alpha=3e-3)
    St, h, vset = _written_out(cfg, gv, d)
    v = d["v_dust"].copy()
    v[:, :, 2] = vset
    Kc3, Kf3 = O.rates(g3, d["cells"], v, d["v_frag"])
    Kc, Kf = O.rates(gv, d["cells"], d["v_dust"], d["v_frag"])
    i, j = _pairs(gv.N)
    G = 1.0 / np.sqrt(2.0 * np.pi * (h[:, i] ** 2 + h[:, j] ** 2))
    for got, vol in ((Kc, Kc3), (Kf, Kf3)):
        want = vol * G
        assert np.all(np.abs(got - want) <= 1e-13 * np.abs(want) + 1e-300), case
    assert Kc.max() > 0 and np.all(np.isfinite(Kc)) and np.all(np.isfinite(Kf))
    if case == "wide":
        assert Kf.max() > 0      # both outcomes present on the wide grid


def test_overlap_factor_against_quadrature(O):
    """int n_i(z) n_j(z) dz / (N_i N_j) for Gaussian columns of unit surface
    density, by adaptive quadrature, equals the factor the rates carry."""
    from scipy.integrate import quad
    cfg, gv, g3, d = _columns(O, 1, 30, 1e-5, 100.0, (20.0, 20.0), drift=False)
    St, h, vset = _written_out(cfg, gv, d)
    h = h[0]
    assert h.max() / h.min() > 30.0           # from well mixed to settled
    prof = lambda z, hk: np.exp(-0.5 * (z / hk) ** 2) / (np.sqrt(2.0 * np.pi) * hk)
    Kc, _ = O.rates(gv, d["cells"], d["v_dust"], d["v_frag"])
    v = d["v_dust"].copy()
    v[:, :, 2] = vset
    Kc3, _ = O.rates(g3, d["cells"], v, d["v_frag"])
    for a, b in ((0, 0), (29, 0), (29, 29), (20, 7), (15, 14)):
        hi, hj = h[a], h[b]
        L = 12.0 * max(hi, hj)
        val, err = quad(lambda z: prof(z, hi) * prof(z, hj), -L, L, epsabs=0.0, epsrel=1e-13,
                        limit=400, points=[0.0])
        p = a * (a + 1) // 2 + b
        np.testing.assert_allclose(Kc[0, p] / Kc3[0, p], val, rtol=1e-9)


def test_well_mixed_grains_reduce_to_the_volume_kernel(O):
    """St << alpha for every bin: h_k -> H and the settling speeds vanish, so
    the rates approach the volume rates (no vertical relative velocity)
    divided by sqrt(4 pi) H, to O(St / alpha) and the settling speeds
    against Brownian motion (1e-4 here)."""
    cfg, gv, g3, d = _columns(O, 2, 16, 1e-6, 1e-5, (10.0, 30.0), drift=True, alpha=0.3)
    St, h, vset = _written_out(cfg, gv, d)
    assert St.max() / 0.3 < 1e-5
    v = d["v_dust"].copy()
    v[:, :, 2] = 0.0
    Kc3, Kf3 = O.rates(g3, d["cells"], v, d["v_frag"])
    Kc, Kf = O.rates(gv, d["cells"], d["v_dust"], d["v_frag"])
    H = d["cells"]["H"][:, None]
    np.testing.assert_allclose(Kc, Kc3 / (np.sqrt(4.0 * np.pi) * H), rtol=1e-4)


def test_midplane_stokes_number_of_a_column(O):
    """With rho_g = Sigma_g / (sqrt(2 pi) H) and H = c_s / Omega, the Stokes
    number of eq. `t_stop` is (pi / 2) rho_m s / Sigma_g."""
    cfg, gv, g3, d = _columns(O, 5, 20, 1e-5, 100.0, (5.0, 100.0))
    St, h, vset = _written_out(cfg, gv, d)
    want = 0.5 * np.pi * cfg.rho_m * gv.s[None, :] / d["cells"]["Sigma_g"][:, None]
    np.testing.assert_allclose(St, want, rtol=1e-13)


def test_vertical_rate_derivatives_against_complex_step_chain(O):
    """The hand dK/dalpha (through v_turb, Re, the scale heights, the
    settling speeds and the overlap factor) and dK/dv_frag, in the step
    adjoint, against the complex step of the forward; the rate derivatives
    alone against central differences."""
    cfg, gv, g3, d = _columns(O)
    der = O.rates_deriv(gv, d["cells"], d["v_dust"], d["v_frag"])
    for key in ("alpha", "vfrag"):
        base = d["cells"]["alpha"] if key == "alpha" else d["v_frag"]
        hh = 1e-6 * base

        def K(x):
            cells = dict(d["cells"])
            if key == "alpha":
                cells["alpha"] = x
                return O.rates(gv, cells, d["v_dust"], d["v_frag"])
            return O.rates(gv, cells, d["v_dust"], x)
        Kcp, Kfp = K(base + hh)
        Kcm, Kfm = K(base - hh)
        sfx = "dalpha" if key == "alpha" else "dvfrag"
        for fd, hand in (((Kcp - Kcm) / (2 * hh[:, None]), der["dKc_" + sfx]),
                         ((Kfp - Kfm) / (2 * hh[:, None]), der["dKf_" + sfx])):
            scale = np.abs(hand).max(axis=1, keepdims=True)
            assert np.all(np.abs(fd - hand) <= 1e-6 * scale + 1e-8 * np.abs(hand)), key
    # the chain through a frozen step sequence, against the complex step
    rng = np.random.default_rng(11)
    rho = 0.01 * d["cells"]["Sigma_g"][:, None] * rng.uniform(0.2, 1.0, d["rho"].shape) / gv.N
    Kc, Kf = O.rates(gv, d["cells"], d["v_dust"], d["v_frag"])
    a = O.step(gv, rho, Kc, Kf, d["dt"] * 30, max_sub=64)
    assert np.all(a["status"] == 0) and np.all(a["nsub"] >= 2)
    g_out = rng.normal(size=rho.shape) / rho.sum(1, keepdims=True)
    g_in, ga, gvf = O.step_backward(gv, d["cells"], d["v_dust"], d["v_frag"], rho, 1.0,
                                    a["h_log"], a["nsub"], g_out)
    args = (gv, d["cells"], d["v_dust"], d["v_frag"], rho, a["h_log"], a["nsub"], g_out)
    for q in range(rho.shape[0]):
        np.testing.assert_allclose(ga[q], O.cs_step_grad(*args, "alpha", q), rtol=1e-11)
        np.testing.assert_allclose(gvf[q], O.cs_step_grad(*args, "vfrag", q), rtol=1e-11)
        for k in range(0, gv.N, 3):
            np.testing.assert_allclose(g_in[q, k], O.cs_step_grad(*args, "rho", q * gv.N + k),
                                       rtol=1e-11, atol=1e-13 * np.abs(g_in[q]).max())
