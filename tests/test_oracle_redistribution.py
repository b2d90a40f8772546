"""Pins of the oracle's mass grid and redistribution tables (Sec. 5, eqs.
`Cijk`, `Rijk`, `fragdist`, `Nijk`, `fragrem`; grid of Sec. 7).

Each check compares the oracle with something other than itself: numbers the
paper prints, exact invariants of the two-bin split, numerical integration of
the fragment power law, and the second formulation of the fragment gain.
"""
import os

import numpy as np
import pytest
from scipy import integrate

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _pairs(N):
    return [(i, j) for i in range(N) for j in range(i + 1)]


def test_paper_grid_ratio(O):
    """Sec. 7: 100 bins over 0.1 um - 0.5 cm and 135 over 0.1 um - 20 cm both
    give m_{n+1}/m_n = 1.38 (printed to two decimals)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "paper_grid_ratio.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 2
    for n, lo, hi, ratio, dec in rows:
        m, me, s = O.mass_grid(int(n), float(lo), float(hi))
        r = m[1:] / m[:-1]
        assert np.allclose(r, r[0], rtol=1e-12, atol=0)          # constant ratio
        assert round(float(r[0]), int(dec)) == float(ratio)
        assert np.log10(r[0]) < 1 / 7                              # > 7 bins per decade
        # edges bracket the centres and are their geometric midpoints
        assert np.all(me[:-1] < m) and np.all(m < me[1:])
        np.testing.assert_allclose(me[1:-1], np.sqrt(m[:-1] * m[1:]), rtol=1e-13)
        # radius range is the outer edge range; m = 4/3 pi rho_m s^3
        np.testing.assert_allclose(m, 4 / 3 * np.pi * 1.67 * s ** 3, rtol=1e-14)
        np.testing.assert_allclose([me[0], me[-1]],
                                   4 / 3 * np.pi * 1.67 * np.array([float(lo), float(hi)]) ** 3,
                                   rtol=1e-13)


@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("chi", [0.5, 1.0, 2.0])
def test_rows_conserve_mass_and_bracket(O, split, chi):
    """Every coag and frag row of D deposits exactly m_i + m_j; the two-bin
    split brackets the product; MASS rows keep the second moment, NUMBER rows
    keep the particle count."""
    g = O.make_grid(24, 1e-5, 1.0, chi=chi, split=split)
    D = O.redistribution_dense(g)
    sp = O.redistribution_sparse(g)
    P, m = g.P, g.m
    tot = np.array([m[i] + m[j] for i, j in _pairs(g.N)])
    np.testing.assert_allclose(D[:P].sum(1), tot, rtol=4e-16 * 4)
    np.testing.assert_allclose(D[P:].sum(1), tot, rtol=4e-16 * 8)
    assert np.all(D >= 0)
    for p, (i, j) in enumerate(_pairs(g.N)):
        M = m[i] + m[j]
        k = sp["ci"][p]
        w0, w1 = sp["cw"][p]
        if M < m[-1]:
            assert m[k] <= M < m[k + 1]
            # second moment of the split
            if split == 0:
                np.testing.assert_allclose(w0 * m[k] + w1 * m[k + 1], M * M, rtol=1e-14)
            else:
                np.testing.assert_allclose(w0 / m[k] + w1 / m[k + 1], 1.0, rtol=1e-14)
        else:
            assert k == g.N - 1 and w1 == 0.0
        # remnant: eq. `fragrem`
        mrem = m[i] - chi * m[j] if chi * m[j] < m[i] else 0.0
        r0, r1 = sp["rw"][p]
        np.testing.assert_allclose(r0 + r1, mrem, rtol=1e-15, atol=0)
        np.testing.assert_allclose(sp["fm"][p], M - mrem, rtol=1e-14)
        # top fragment bin: m^e_l <= largest fragment < m^e_{l+1}
        mfmax = min(chi * m[j], m[i])
        l = sp["fl"][p]
        assert g.m_edge[l + 1] > mfmax and (l == 0 or g.m_edge[l] <= mfmax)


def test_exact_hit_goes_to_one_bin(O):
    """Linear grid m_k = k+1: m_i + m_j is a bin mass, which receives it whole
    (the tie-break that makes the discrete Smoluchowski equation exact)."""
    N = 16
    m = np.arange(1, N + 1, dtype=float)
    me = np.concatenate([[0.5], np.arange(1, N) + 0.5, [N + 0.5]])
    g = O.Grid(m, me, (3 * m / (4 * np.pi)) ** (1 / 3), 1.0)
    sp = O.redistribution_sparse(g)
    for p, (i, j) in enumerate(_pairs(N)):
        if i + j + 1 < N:
            assert sp["ci"][p] == i + j + 1 and sp["cw"][p][1] == 0.0
            assert sp["cw"][p][0] == m[i] + m[j]


@pytest.mark.parametrize("eta", [11 / 6, 1.5, 2.5])
def test_fragment_fractions_are_power_law_integrals(O, eta):
    """N_k(m^e_{l+1}) is the share of fragment mass in bin k for n(m) ~ m^-eta
    between m^e_0 and m^e_{l+1} (eqs. `fragdist`, `Nijk`); checked by
    quadrature of m^(1-eta) and the telescoping sum to 1."""
    g = O.make_grid(12, 1e-5, 1e-2, eta=eta)
    Nf = O.redistribution_sparse(g)["Nfrac"]
    me = g.m_edge
    for l in range(g.N):
        np.testing.assert_allclose(Nf[l, : l + 1].sum(), 1.0, rtol=1e-14)
        assert np.all(Nf[l, l + 1:] == 0)
        # integrate in log m to keep quad well conditioned
        f = lambda x: np.exp((2 - eta) * x)
        tot = integrate.quad(f, np.log(me[0]), np.log(me[l + 1]), epsabs=0, epsrel=1e-13)[0]
        for k in range(l + 1):
            part = integrate.quad(f, np.log(me[k]), np.log(me[k + 1]), epsabs=0, epsrel=1e-13)[0]
            np.testing.assert_allclose(Nf[l, k], part / tot, rtol=1e-10)


@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("chi", [0.5, 1.0, 2.0])
def test_rafikov_accumulation_equals_per_pair_fragments(O, split, chi):
    """Sec. 5: accumulating fragment mass per top bin, then distributing it,
    gives the same gain as the per-pair F_ijk written out densely."""
    rng = np.random.default_rng(7)
    for grid in ("log", "linear"):
        if grid == "log":
            g = O.make_grid(14, 1e-5, 1.0, chi=chi, split=split)
        else:
            N = 10
            m = np.arange(1, N + 1, dtype=float)
            me = np.concatenate([[0.5], np.arange(1, N) + 0.5, [N + 0.5]])
            g = O.Grid(m, me, (3 * m / (4 * np.pi)) ** (1 / 3), 1.0, chi=chi, split=split)
        C, P = 3, g.P
        rho = rng.uniform(0.1, 1.0, (C, g.N)) * g.m
        Kc, Kf = rng.uniform(0, 1, (C, P)), rng.uniform(0, 1, (C, P))
        f, gain, loss = O.rhs(g, rho, Kc, Kf, parts=True)
        fd = O.rhs_dense(g, rho, Kc, Kf)
        np.testing.assert_allclose(f, fd, rtol=0, atol=1e-14 * (gain + loss).max())
        # mass conservation of the full right-hand side
        assert np.all(np.abs(f.sum(1)) <= 1e-14 * gain.sum(1))


def test_bad_grid_rejected(O):
    g = O.make_grid(8, 1e-5, 1.0)
    g.m = g.m[::-1].copy()
    with pytest.raises(ValueError):
        O.redistribution_dense(g)
    g = O.make_grid(8, 1e-5, 1.0, eta=2.0)
    with pytest.raises(ValueError):
        O.redistribution_dense(g)


@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("n", [2, 3, 5])
def test_rows_conserve_mass_on_coarse_grids(O, split, n):
    """Very coarse grids (up to 18 decades of mass per bin): the split must
    still deposit exactly m_i + m_j (1 - eps is evaluated without the
    cancellation of 1 - (m_u - M)/(m_u - m_l))."""
    for chi in (0.5, 1.0, 2.0):
        g = O.make_grid(n, 1e-5, 10.0, chi=chi, split=split)
        D = O.redistribution_dense(g)
        tot = np.array([g.m[i] + g.m[j] for i, j in _pairs(g.N)])
        np.testing.assert_allclose(D[: g.P].sum(1), tot, rtol=1e-15)
        np.testing.assert_allclose(D[g.P:].sum(1), tot, rtol=1e-15)
