"""Pins of the oracle's hand-written adjoint of the coagulation step.

The adjoint (oracle_step_backward / oracle_rhs_vjp) is checked against the
complex-step derivative of the forward arithmetic (a perturbation i*1e-30 of
one input carried through the complex instantiation of the same formulas,
exact to rounding and independent of the hand derivation), and against
central finite differences of the FP64 forward with a frozen step sequence
(relative step 1e-6).

The grids here span three decades of mass.  The adjoint with respect to the
density of a light bin i is a sum of terms of the size of the heavy partners'
masses that cancel down to terms of size m_i (a collision adds m_i to a heavy
bin that also loses its own m_j), so on grids spanning many decades every FP64
evaluation of it, by any method, carries a rounding error of order
eps * m_max / m_min relative to its value; narrow grids keep the comparison at
the 1e-12 level.
"""
import numpy as np
import pytest


def _problem(O, n_bins=12, cells=(2, 1), steps=3):
    from paper_2402_18471_amd import disc
    cfg = disc.scaled(disc.CONFIGS["disc64x32_n100"], cells[0], cells[1], n_bins)
    g = O.make_grid(cfg.n_bins, 3e-4, 3e-3, rho_m=cfg.rho_m)
    d = disc.make_disc(cfg, g.s)
    # a spread distribution so every bin takes part
    rng = np.random.default_rng(9)
    rho = 0.01 * d["cells"]["rho_g"][:, None] * rng.uniform(0.2, 1.0, (cfg.n_cells, g.N)) / g.N
    Kc, Kf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    a = O.step(g, rho, Kc, Kf, d["dt"] * steps, max_sub=64)
    assert np.all(a["status"] == 0)
    rng = np.random.default_rng(5)
    g_out = rng.normal(size=rho.shape) / rho.sum(1, keepdims=True)
    return g, d, rho, a, g_out


def _fwd_J(O, g, d, rho, a, g_out, alpha=None, vfrag=None):
    cells = dict(d["cells"])
    if alpha is not None:
        cells["alpha"] = alpha
    vf = d["v_frag"] if vfrag is None else vfrag
    Kc, Kf = O.rates(g, cells, d["v_dust"], vf)
    r = O.step(g, rho, Kc, Kf, 1.0, mode=O.REPLAY, nsub=a["nsub"], h_log=a["h_log"])
    return float((g_out * r["rho"]).sum())


def test_rhs_vjp_against_complex_step(O):
    g = O.make_grid(10, 1e-4, 1e-3, chi=1.0)
    rng = np.random.default_rng(2)
    rho = rng.uniform(0.1, 1, g.N) * g.m * 1e3
    Kc, Kf = rng.uniform(0, 1, g.P) * 1e-8, rng.uniform(0, 1, g.P) * 1e-8
    mu = rng.normal(size=g.N)
    gy, gKc, gKf = O.rhs_vjp(g, rho, Kc, Kf, mu)
    for k in range(g.N):
        cs = O.cs_rhs_grad(g, rho, Kc, Kf, mu, "rho", k)
        np.testing.assert_allclose(gy[0, k], cs, rtol=1e-12, atol=1e-14 * np.abs(gy).max())
    for p in range(0, g.P, 5):
        np.testing.assert_allclose(gKc[0, p], O.cs_rhs_grad(g, rho, Kc, Kf, mu, "Kc", p),
                                   rtol=1e-12, atol=1e-14 * np.abs(gKc).max())
        np.testing.assert_allclose(gKf[0, p], O.cs_rhs_grad(g, rho, Kc, Kf, mu, "Kf", p),
                                   rtol=1e-12, atol=1e-14 * np.abs(gKf).max())


def test_rate_derivatives_against_central_differences(O):
    """The hand dK/dalpha, dK/dv_frag against central differences of the
    rates (the full chain is checked by complex step below)."""
    g, d, rho, a, g_out = _problem(O)
    der = O.rates_deriv(g, d["cells"], d["v_dust"], d["v_frag"])
    for key, name in (("alpha", "alpha"), ("vfrag", "v_frag")):
        base = d["cells"]["alpha"] if key == "alpha" else d["v_frag"]
        h = 1e-6 * base
        def K(x):
            cells = dict(d["cells"])
            if key == "alpha":
                cells["alpha"] = x
                return O.rates(g, cells, d["v_dust"], d["v_frag"])
            return O.rates(g, cells, d["v_dust"], x)
        Kcp, Kfp = K(base + h)
        Kcm, Kfm = K(base - h)
        fdc = (Kcp - Kcm) / (2 * h[:, None])
        fdf = (Kfp - Kfm) / (2 * h[:, None])
        sfx = "dalpha" if key == "alpha" else "dvfrag"
        for fd, hand in ((fdc, der["dKc_" + sfx]), (fdf, der["dKf_" + sfx])):
            scale = np.abs(hand).max(axis=1, keepdims=True)
            assert np.all(np.abs(fd - hand) <= 1e-6 * scale + 1e-8 * np.abs(hand))


@pytest.mark.parametrize("chi", [1.0])
def test_step_adjoint_against_complex_step(O, chi):
    g, d, rho, a, g_out = _problem(O)
    g_in, ga, gv = O.step_backward(g, d["cells"], d["v_dust"], d["v_frag"], rho, 1.0,
                                   a["h_log"], a["nsub"], g_out)
    C = rho.shape[0]
    args = (g, d["cells"], d["v_dust"], d["v_frag"], rho, a["h_log"], a["nsub"], g_out)
    for q in range(C):
        for k in range(g.N):
            cs = O.cs_step_grad(*args, "rho", q * g.N + k)
            np.testing.assert_allclose(g_in[q, k], cs, rtol=1e-11,
                                       atol=1e-13 * np.abs(g_in[q]).max())
        np.testing.assert_allclose(ga[q], O.cs_step_grad(*args, "alpha", q), rtol=1e-11)
        np.testing.assert_allclose(gv[q], O.cs_step_grad(*args, "vfrag", q), rtol=1e-11)


def test_step_adjoint_against_central_differences(O):
    """Central differences (relative step 1e-6) of the FP64 forward with the
    step sequence frozen, for alpha, v_frag and a few initial-state
    directions."""
    g, d, rho, a, g_out = _problem(O)
    g_in, ga, gv = O.step_backward(g, d["cells"], d["v_dust"], d["v_frag"], rho, 1.0,
                                   a["h_log"], a["nsub"], g_out)
    C = rho.shape[0]
    for q in range(C):
        for name, base, grad in (("alpha", d["cells"]["alpha"], ga), ("vfrag", d["v_frag"], gv)):
            h = 1e-6 * base[q]
            xp, xm = base.copy(), base.copy()
            xp[q] += h
            xm[q] -= h
            Jp = _fwd_J(O, g, d, rho, a, g_out, **{("alpha" if name == "alpha" else "vfrag"): xp})
            Jm = _fwd_J(O, g, d, rho, a, g_out, **{("alpha" if name == "alpha" else "vfrag"): xm})
            np.testing.assert_allclose((Jp - Jm) / (2 * h), grad[q], rtol=1e-6)
    rng = np.random.default_rng(240218472)
    for _ in range(4):
        dirn = rng.normal(size=rho.shape) * rho
        eps = 1e-6
        Jp = _fwd_J(O, g, d, rho + eps * dirn, a, g_out)
        Jm = _fwd_J(O, g, d, rho - eps * dirn, a, g_out)
        np.testing.assert_allclose((Jp - Jm) / (2 * eps), (g_in * dirn).sum(), rtol=1e-6)
