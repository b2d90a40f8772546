"""Brute-force pin of the oracle's right-hand side (Sec. 5, eqs. `smol`,
`ngain`, `Cijk`, `Rijk`, `fragrem`, `fragdist`, `Nijk`).

The right-hand side is evaluated here a second time, literally: for every
bin k a sum over every pair (i, j <= i) of n_i n_j K_ij [p_coag (m_i + m_j)
C_ijk + p_frag (m_rem R_ijk + m_frag F_ijk)], with the per-pair fragment
fractions F_ijk = N_k(m^e_{l+1}) of eq. `Nijk` (no accumulation per top bin),
minus sum_i m_k n_i n_k K_ik (p_coag + p_frag).  Nothing here comes from the
oracle: the bracketing bins, the split fractions, the remnant, the top
fragment bin and the fragment fractions are all recomputed from the
equations, with the readings the oracle documents (an exact hit goes wholly
to its bin, products beyond the grid to the end bins, the largest fragment
min(chi m_im, m_tar) sets the top bin and total minus remnant is the
fragment mass, the loss kernel is not halved).  Random symmetric kernels
K >= 0, probabilities p in [0, 1], chi in {0.5, 1, 2}, both split readings,
linear and logarithmic grids of 6-16 bins.
"""
import numpy as np
import pytest


def _lower_upper(m, M):
    """l(M), u(M) and eps(M) (eqs. `Cijk`, `Rijk`): l the largest bin with
    m_l <= M, u = l + 1, eps = (m_u - M) / (m_u - m_l); None for u when M lies
    at or beyond the top bin, or below bin 0 (then everything goes to the end
    bin)."""
    N = len(m)
    if M >= m[N - 1]:
        return N - 1, None, 1.0
    if M < m[0]:
        return 0, None, 1.0
    lo = max(k for k in range(N) if m[k] <= M)
    up = lo + 1
    return lo, up, (m[up] - M) / (m[up] - m[lo])


def _two_bin(m, M, split, k):
    """Mass fraction of a product of mass M that lands in bin k: eps to l and
    1 - eps to u read as mass fractions (split 0), or one particle split by
    number, eps m_l / M and (1 - eps) m_u / M (split 1)."""
    if M <= 0:
        return 0.0
    lo, up, eps = _lower_upper(m, M)
    if up is None:
        return 1.0 if k == lo else 0.0
    if split == 0:
        return eps if k == lo else (1.0 - eps if k == up else 0.0)
    return eps * m[lo] / M if k == lo else ((1.0 - eps) * m[up] / M if k == up else 0.0)


def _fragment_fraction(me, eta, m_largest, k):
    """F_ijk = N_k(m_max) of eq. `Nijk` with m_max = m^e_{l+1} and l the
    smallest index with m^e_{l+1} > m_largest (the top bin, clipped to the
    grid)."""
    N = len(me) - 1
    l = next((q for q in range(N) if me[q + 1] > m_largest), N - 1)
    if k > l:
        return 0.0
    e = 2.0 - eta
    return (me[k + 1] ** e - me[k] ** e) / (me[l + 1] ** e - me[0] ** e)


def _literal_rhs(m, me, eta, chi, split, rho, K, pf):
    """Eq. `smol` for one cell, term by term; K, pf symmetric N x N."""
    N = len(m)
    n = rho / m
    out = np.zeros(N)
    scale = np.zeros(N)               # sum of |terms| per bin, for the tolerance
    for k in range(N):
        for i in range(N):
            for j in range(i + 1):
                Kij = 0.5 * K[i, j] if i == j else K[i, j]
                pc, pfr = 1.0 - pf[i, j], pf[i, j]
                tar, im = (m[i], m[j])                   # i >= j: i is the target
                if chi * im < tar:                        # eq. `fragrem`
                    m_rem, m_largest = tar - chi * im, chi * im
                else:
                    m_rem, m_largest = 0.0, tar
                m_frag = (m[i] + m[j]) - m_rem
                gain = n[i] * n[j] * Kij * (
                    pc * (m[i] + m[j]) * _two_bin(m, m[i] + m[j], split, k)
                    + pfr * (m_rem * _two_bin(m, m_rem, split, k)
                             + m_frag * _fragment_fraction(me, eta, m_largest, k)))
                out[k] += gain
                scale[k] += abs(gain)
        for i in range(N):
            loss = m[k] * n[i] * n[k] * K[i, k] * ((1.0 - pf[i, k]) + pf[i, k])
            out[k] -= loss
            scale[k] += abs(loss)
    return out, scale


def _grids(N):
    m_lin = np.arange(1, N + 1, dtype=float) * 2.5e-12
    me_lin = np.concatenate([[0.5 * m_lin[0]], 0.5 * (m_lin[:-1] + m_lin[1:]),
                             [m_lin[-1] + 0.5 * m_lin[0]]])
    r = 10.0 ** (9.0 / N)                                 # 9 decades of mass
    m_log = 1e-14 * r ** (np.arange(N) + 0.5)
    me_log = 1e-14 * r ** np.arange(N + 1)
    return {"linear": (m_lin, me_lin), "log": (m_log, me_log)}


@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("chi", [0.5, 1.0, 2.0])
@pytest.mark.parametrize("N", [6, 11, 16])
def test_literal_rhs_matches_oracle(O, N, chi, split):
    rng = np.random.default_rng(1000 * N + int(10 * chi) + split)
    eta = 11.0 / 6.0
    for name, (m, me) in _grids(N).items():
        s = (3 * m / (4 * np.pi * 1.6)) ** (1.0 / 3.0)
        g = O.Grid(m.copy(), me.copy(), s, 1.6, eta=eta, chi=chi, split=split)
        for _ in range(2):
            A = rng.uniform(0.0, 1.0, (N, N))
            K = A + A.T                                    # symmetric, >= 0
            B = rng.uniform(0.0, 1.0, (N, N))
            pf = np.tril(B) + np.tril(B, -1).T             # symmetric, in [0, 1]
            K[rng.uniform(size=(N, N)) < 0.1] = 0.0
            K = np.tril(K) + np.tril(K, -1).T
            rho = rng.uniform(0.05, 1.0, N) * m * 1e9
            w = np.array([0.5 if i == j else 1.0 for i in range(N) for j in range(i + 1)])
            Kp = np.array([K[i, j] for i in range(N) for j in range(i + 1)])
            pp = np.array([pf[i, j] for i in range(N) for j in range(i + 1)])
            Kc, Kf = w * Kp * (1.0 - pp), w * Kp * pp
            got = O.rhs(g, rho, Kc[None], Kf[None])[0]
            ref, scale = _literal_rhs(m, me, eta, chi, split, rho, K, pf)
            assert np.all(np.abs(got - ref) <= 1e-14 * scale), (name, np.max(np.abs(got - ref) / scale))
            # and the dense per-pair form of the oracle, for good measure
            dense = O.rhs_dense(g, rho, Kc[None], Kf[None])[0]
            assert np.all(np.abs(dense - ref) <= 1e-14 * scale)


def test_literal_rhs_sees_a_dropped_fragment_term(O):
    """The literal sum is sensitive to what it pins: without the fragment
    term it no longer matches the oracle (so a dropped term in either would
    be caught)."""
    N, chi, split = 8, 1.0, 0
    m, me = _grids(N)["log"]
    s = (3 * m / (4 * np.pi * 1.6)) ** (1.0 / 3.0)
    g = O.Grid(m.copy(), me.copy(), s, 1.6, chi=chi, split=split)
    rng = np.random.default_rng(5)
    A = rng.uniform(0.5, 1.0, (N, N))
    K = A + A.T
    pf = np.full((N, N), 0.5)
    rho = rng.uniform(0.1, 1.0, N) * m * 1e9
    w = np.array([0.5 if i == j else 1.0 for i in range(N) for j in range(i + 1)])
    Kp = np.array([K[i, j] for i in range(N) for j in range(i + 1)])
    got = O.rhs(g, rho, (w * Kp * 0.5)[None], (w * Kp * 0.5)[None])[0]
    ref, scale = _literal_rhs(m, me, 11 / 6, chi, split, rho, K, pf)
    assert np.all(np.abs(got - ref) <= 1e-14 * scale)
    orig = _fragment_fraction
    try:
        globals()["_fragment_fraction"] = lambda *a: 0.0
        bad, _ = _literal_rhs(m, me, 11 / 6, chi, split, rho, K, pf)
    finally:
        globals()["_fragment_fraction"] = orig
    assert np.max(np.abs(got - bad) / scale) > 1e-3
