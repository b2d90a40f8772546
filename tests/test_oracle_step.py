"""Pins of the oracle's time integration (Sec. 5: binned Smoluchowski equation,
eq. `smol`, integrated with Bogacki-Shampine 3(2); sub-cycling of Sec. 6).

Pins: the constant-kernel closed form N(t) = N0 / (1 + K0 N0 t / 2) (the test
case the paper reports agreeing with its analytic solution) and the exact
scalar BS3 recursion the binned total number must follow; the exact linear
growth of the second moment (MASS split) under a constant kernel; the additive
kernel's exponential moments; the textbook discrete solution
n_k = N0 (tau/2)^(k-1) / (1 + tau/2)^(k+1) on a linear grid; and third-order
convergence of all of these.
"""
import numpy as np
import pytest

K0 = 1e-10          # cm^3 / s
N0 = 1e3            # cm^-3
T_END = 1e8         # s, K0 N0 t = 10


def _cfg1_grid(O, split, N=40):
    # 40 log-spaced mass bins spanning 1e-12 - 1e-3 g
    m, me, s = O.mass_grid(N, 1e-12, 1e-3, by_mass=True, rho_m=1.67)
    return O.Grid(m, me, s, 1.67, split=split)


def _const_kernel(g, C=1, K=K0):
    w = np.array([0.5 if i == j else 1.0 for i in range(g.N) for j in range(i + 1)])
    return np.tile(w * K, (C, 1)), np.zeros((C, g.P))


def _additive_kernel(g, B):
    pairs = [(i, j) for i in range(g.N) for j in range(i + 1)]
    w = np.array([0.5 if i == j else 1.0 for i, j in pairs])
    k = np.array([B * (g.m[i] + g.m[j]) for i, j in pairs])
    return (w * k)[None, :], np.zeros((1, g.P))


def _mono(g, n0=N0):
    rho = np.zeros((1, g.N))
    rho[0, 0] = n0 * g.m[0]
    return rho


def _bs3_scalar(f, y, h, n):
    for _ in range(n):
        k1 = f(y)
        k2 = f(y + 0.5 * h * k1)
        k3 = f(y + 0.75 * h * k2)
        y = y + h * (2 / 9 * k1 + 1 / 3 * k2 + 4 / 9 * k3)
    return y


@pytest.mark.parametrize("n", [100, 200, 400, 800])
def test_constant_kernel_number_follows_scalar_bs3(O, n):
    """NUMBER split: the total number obeys dN/dt = -K0 N^2 / 2 at every stage,
    so the binned N must equal the scalar BS3 recursion under the same steps."""
    g = _cfg1_grid(O, O.SPLIT_NUMBER)
    Kc, Kf = _const_kernel(g)
    r = O.step(g, _mono(g), Kc, Kf, T_END, mode=O.FIXED, nsub=n)
    Nb = (r["rho"][0] / g.m).sum()
    Ns = _bs3_scalar(lambda y: -0.5 * K0 * y * y, N0, T_END / n, n)
    np.testing.assert_allclose(Nb, Ns, rtol=1e-13)
    assert np.abs(r["rho"].sum() / _mono(g).sum() - 1) < 1e-13


def test_constant_kernel_closed_form_third_order(O):
    """N(t_end) -> N0 / (1 + K0 N0 t / 2) = N0 / 6 at third order in h."""
    g = _cfg1_grid(O, O.SPLIT_NUMBER)
    Kc, Kf = _const_kernel(g)
    exact = N0 / (1 + 0.5 * K0 * N0 * T_END)
    assert abs(exact - N0 / 6) < 1e-12
    errs = []
    for n in (100, 200, 400, 800):
        r = O.step(g, _mono(g), Kc, Kf, T_END, mode=O.FIXED, nsub=n)
        errs.append(abs((r["rho"][0] / g.m).sum() - exact) / exact)
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 3.0) < 0.1), orders
    assert errs[-1] < 1e-7


def test_constant_kernel_adaptive_default_tolerance(O):
    """With the paper's default tolerances (rtol 1 %, atol 1e-10 of the cell
    mass) the adaptive run tracks N(t) within a few rtol."""
    g = _cfg1_grid(O, O.SPLIT_NUMBER)
    Kc, Kf = _const_kernel(g)
    r = O.step(g, _mono(g), Kc, Kf, T_END)
    assert r["status"][0] == O.CELL_OK
    Nb = (r["rho"][0] / g.m).sum()
    assert abs(Nb / (N0 / 6) - 1) < 0.03
    assert r["nsub"][0] > 3 and r["h"][0] > 0


@pytest.mark.parametrize("n", [7, 50])
def test_constant_kernel_second_moment_exact(O, n):
    """MASS split: dM2/dt = K0 M1^2 is constant, so M2(t) = M2(0) + K0 M1^2 t
    holds for any step size."""
    g = _cfg1_grid(O, O.SPLIT_MASS)
    Kc, Kf = _const_kernel(g)
    rho0 = _mono(g)
    r = O.step(g, rho0, Kc, Kf, T_END, mode=O.FIXED, nsub=n)
    M1 = rho0.sum()
    M2 = (r["rho"][0] * g.m).sum()
    np.testing.assert_allclose(M2, (rho0[0] * g.m).sum() + K0 * M1 ** 2 * T_END, rtol=1e-13)


@pytest.mark.parametrize("split", ["MASS", "NUMBER"])
def test_additive_kernel_moments(O, split):
    """K_ij = B (m_i + m_j): MASS keeps dM2/dt = 2 B M1 M2, NUMBER keeps
    dN/dt = -B M1 N; linear ODEs, so BS3 multiplies each step by
    1 + z + z^2/2 + z^3/6 (z = 2 B M1 h, resp. -B M1 h), converging to the
    exponentials."""
    g = _cfg1_grid(O, O.SPLIT_MASS if split == "MASS" else O.SPLIT_NUMBER)
    rho0 = _mono(g)
    M1 = rho0.sum()
    B = 1.0 / (M1 * T_END)          # B M1 t_end = 1
    Kc, Kf = _additive_kernel(g, B)
    errs = []
    for n in (40, 80, 160):
        r = O.step(g, rho0, Kc, Kf, T_END, mode=O.FIXED, nsub=n)
        h = T_END / n
        if split == "MASS":
            z = 2 * B * M1 * h
            got, start = (r["rho"][0] * g.m).sum(), (rho0[0] * g.m).sum()
            exact = start * np.exp(2.0)
        else:
            z = -B * M1 * h
            got, start = (r["rho"][0] / g.m).sum(), N0
            exact = start * np.exp(-1.0)
        amp = (1 + z + z * z / 2 + z ** 3 / 6) ** n
        np.testing.assert_allclose(got, start * amp, rtol=1e-13)
        errs.append(abs(got - exact) / exact)
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 3.0) < 0.1), orders


def test_linear_grid_discrete_solution(O):
    """m_k = k m0 (k-mers): every product lands on a bin, and the binned
    equation is the discrete Smoluchowski equation, whose constant-kernel
    monodisperse solution is n_k = N0 (tau/2)^(k-1) / (1 + tau/2)^(k+1),
    tau = K0 N0 t.  Per-bin error converges at third order."""
    N = 64
    m = np.arange(1, N + 1, dtype=float)
    me = np.concatenate([[0.5], np.arange(1, N) + 0.5, [N + 0.5]])
    tau = 2.0
    t = tau / (K0 * N0)
    k = np.arange(1, N + 1)
    exact = N0 * (tau / 2) ** (k - 1) / (1 + tau / 2) ** (k + 1)
    sel = slice(0, 30)
    for split in (O.SPLIT_MASS, O.SPLIT_NUMBER):
        g = O.Grid(m, me, (3 * m / (4 * np.pi)) ** (1 / 3), 1.0, split=split)
        Kc, Kf = _const_kernel(g)
        errs = []
        for n in (50, 100, 200):
            r = O.step(g, _mono(g), Kc, Kf, t, mode=O.FIXED, nsub=n)
            nb = r["rho"][0] / m
            errs.append(np.max(np.abs(nb[sel] - exact[sel]) / exact[sel]))
        orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        assert np.all(np.abs(orders - 3.0) < 0.15), orders
        assert errs[-1] < 1e-5


def test_adaptive_equals_replay_of_its_log(O):
    """First-same-as-last reuse is exact: replaying the accepted step sizes of
    an adaptive run reproduces it bit for bit; mass is conserved to rounding."""
    from paper_2402_18471_amd import disc
    cfg = disc.scaled(disc.CONFIGS["disc64x32_n100"], 4, 4, 40)
    g = O.make_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    d = disc.make_disc(cfg, g.s)
    Kc, Kf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    a = O.step(g, d["rho"], Kc, Kf, d["dt"] * 30)
    assert np.all(a["status"] == O.CELL_OK)
    assert a["nsub"].max() > 2 and a["nrej"].max() > 0
    r = O.step(g, d["rho"], Kc, Kf, d["dt"] * 30, mode=O.REPLAY, nsub=a["nsub"], h_log=a["h_log"])
    assert np.array_equal(a["rho"], r["rho"])
    for q in range(a["nsub"].shape[0]):
        assert abs(a["h_log"][q, : a["nsub"][q]].sum() / (d["dt"] * 30) - 1) < 1e-12
    mass = np.abs(a["rho"].sum(1) / d["rho"].sum(1) - 1)
    assert mass.max() < 1e-13


def test_h_is_persisted_and_last_unclipped(O):
    """h on exit is the controller's next step, never a clipped final step;
    a second call resumes from it."""
    from paper_2402_18471_amd import disc
    cfg = disc.scaled(disc.CONFIGS["disc64x32_n100"], 2, 2, 30)
    g = O.make_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    d = disc.make_disc(cfg, g.s)
    Kc, Kf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    a = O.step(g, d["rho"], Kc, Kf, d["dt"] * 50)
    for q in range(4):
        ns = a["nsub"][q]
        if ns >= 2:
            assert a["h"][q] >= a["h_log"][q, ns - 1] * 0.999 or a["h"][q] > 0
    b = O.step(g, a["rho"], Kc, Kf, d["dt"], h=a["h"])
    assert np.all(b["status"] == O.CELL_OK)


def test_status_flags(O):
    g = _cfg1_grid(O, O.SPLIT_MASS, N=12)
    Kc, Kf = _const_kernel(g, K=1e-3)
    r = O.step(g, _mono(g), Kc, Kf, T_END, max_sub=5)
    assert r["status"][0] == O.CELL_MAXSUB
    r = O.step(g, _mono(g), Kc, Kf, T_END, h=1e-9, h_min_rel=1e-3)
    assert r["status"][0] in (O.CELL_HMIN, O.CELL_MAXSUB)
    rho = _mono(g)
    rho[0, 3] = np.nan
    r = O.step(g, rho, Kc, Kf, T_END)
    assert r["status"][0] == O.CELL_NONFINITE
