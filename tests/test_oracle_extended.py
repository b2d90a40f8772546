"""Pins of the oracle's extended-precision evaluation (oracle/extended.py),
the reference the GPU tests hold FP64 results to where FP64 rounding is
amplified (heavy bins whose gain and loss nearly cancel; adjoint components
in bins empty at the start).

It is a second implementation of the oracle's own definitions (numpy, its own
order of summation) on the oracle's FP64 tables and rates:
  - in float64 it reproduces the C oracle to rounding (right-hand side, steps
    of a given sequence, adjoint and rate chain rule);
  - in long double it agrees with the C oracle wherever FP64 is well
    conditioned (populated bins of the adjoint, alpha, v_frag, the state);
  - in long double its right-hand side's total equals the mass defect of the
    FP64 tables to long-double rounding;
  - its long-double adjoint moves by ~4e-8 of the largest component when the
    order of summation changes (pairs shuffled), where the FP64 evaluations
    in two orders differ by ~1e-3 of it: it resolves what FP64 cannot.
"""
import numpy as np
import pytest

LD = np.longdouble


@pytest.fixture(scope="module")
def E():
    from oracle import extended
    return extended


def _case(O, nr=4, nz=2, nb=None):
    from paper_2402_18471_amd import disc
    cfg = disc.scaled(disc.CONFIGS["disc64x32_n100"], nr, nz, nb)
    g = O.make_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    d = disc.make_disc(cfg, g.s)
    Kc, Kf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    return g, d, Kc, Kf


def _loss_grad(g, r):
    lns = np.log(g.s)
    M = r.sum(1, keepdims=True)
    return (lns[None, :] - (r * lns).sum(1, keepdims=True) / M) / M


def test_long_double_is_extended():
    if np.finfo(LD).nmant < 63:
        pytest.skip("numpy long double is not the x87 extended format here")
    assert np.finfo(LD).eps < 1.1e-19


@pytest.mark.parametrize("dtype", [np.float64, LD], ids=["f64", "ld"])
def test_rhs_and_steps_against_the_c_oracle(O, E, dtype):
    g, d, Kc, Kf = _case(O)
    rho = d["rho"]
    e = E.Extended(g, Kc, Kf, dtype)
    f = e.rhs(rho).astype(np.float64)
    fo, gain, loss = O.rhs(g, rho, Kc, Kf, parts=True)
    assert np.all(np.abs(f - fo) <= 1e-14 * (gain + loss) + 1e-300)
    a = O.step(g, rho, Kc, Kf, d["dt"] * 5, max_sub=64)
    y = e.step(rho, a["h_log"], a["nsub"]).astype(np.float64)
    M = rho.sum(1, keepdims=True)
    assert np.all(np.abs(y - a["rho"]) <= 1e-13 * np.abs(a["rho"]) + 1e-15 * M)


@pytest.mark.parametrize("dtype", [np.float64, LD], ids=["f64", "ld"])
def test_adjoint_against_the_c_oracle_where_fp64_is_well_conditioned(O, E, dtype):
    g, d, Kc, Kf = _case(O)
    rho = d["rho"]
    a = O.step(g, rho, Kc, Kf, d["dt"] * 5, max_sub=64)
    g_out = _loss_grad(g, a["rho"])
    og, oa, ov = O.step_backward(g, d["cells"], d["v_dust"], d["v_frag"], rho, 0.0, a["h_log"],
                                 a["nsub"], g_out)
    r = E.step_backward(g, d["cells"], d["v_dust"], d["v_frag"], rho, a["h_log"], a["nsub"],
                        g_out, Kc, Kf, dtype)
    gi = r["g_in"].astype(np.float64)
    held = rho >= 1e-12 * rho.sum(1, keepdims=True)
    sc = np.abs(og).max(1, keepdims=True)
    assert np.all((np.abs(gi - og) <= 1e-13 * sc)[held])
    al, vf = d["cells"]["alpha"], d["v_frag"]
    S = np.maximum(np.abs(al * oa), np.abs(vf * ov))
    assert np.all(np.abs(al * (r["g_alpha"].astype(np.float64) - oa)) <= 1e-12 * S)
    assert np.all(np.abs(vf * (r["g_vfrag"].astype(np.float64) - ov)) <= 1e-12 * S)


def test_long_double_rhs_conserves_mass_up_to_the_tables(O, E):
    """The FP64 tables conserve each pair's mass only to their own rounding
    (cw0 + cw1 and rw0 + rw1 + m_frag sum_k N_k differ from m_i + m_j by an
    ulp or so); in long double the right-hand side's total equals the defect
    those tables predict, sum_p R_p (sum_k D_pk - m_i - m_j), to long-double
    rounding of the gross flux."""
    g, d, Kc, Kf = _case(O, 2, 2, 40)
    rng = np.random.default_rng(4)
    rho = 0.01 * d["cells"]["rho_g"][:, None] * rng.uniform(0.1, 1.0, (4, g.N)) / g.N
    e = E.Extended(g, Kc, Kf)
    f = e.rhs(rho.astype(LD))
    n = rho.astype(LD) / e.m
    nn = n[:, e.pi] * n[:, e.pj]
    M = e.m[e.pi] + e.m[e.pj]
    fsum = e.Nf.sum(1)[e.fl]                       # sum_k N_k(m^e_{l+1}) of the pair's l
    defect = (nn * e.Kc * (e.cw0 + e.cw1 - M) +
              nn * e.Kf * (e.rw0 + e.rw1 + e.fm * fsum - M)).sum(1)
    _, gain, loss = O.rhs(g, rho, Kc, Kf, parts=True)
    assert np.all(np.abs(f.sum(1) - defect) <= 1e-17 * gain.sum(1))
    # and that defect is FP64 rounding of the tables: <= 1e-15 of the gross flux
    assert np.all(np.abs(defect) <= 1e-15 * gain.sum(1))


def test_long_double_adjoint_does_not_depend_on_the_summation_order(O, E):
    """Pairs visited in a shuffled order change the FP64 adjoint in bins empty
    at the start by ~1e-3 of the cell's largest component, the long-double
    one by a thousand times less (~4e-8)."""
    g, d, Kc, Kf = _case(O, 4, 2)
    rho = d["rho"]
    a = O.step(g, rho, Kc, Kf, d["dt"] * 5, max_sub=64)
    g_out = _loss_grad(g, a["rho"])
    held = rho >= 1e-12 * rho.sum(1, keepdims=True)
    perm = np.random.default_rng(7).permutation(g.P)
    out = {}
    for dtype in (np.float64, LD):
        runs = []
        for shuffle in (False, True):
            e = E.Extended(g, Kc, Kf, dtype)
            if shuffle:
                for k in ("pi", "pj", "ci", "ci1", "cw0", "cw1", "ri", "ri1", "rw0", "rw1", "fl",
                          "fm", "w", "offdiag"):
                    setattr(e, k, getattr(e, k)[perm])
                e.Kc, e.Kf = e.Kc[:, perm], e.Kf[:, perm]
                for k, idx in (("_ci", e.ci), ("_ci1", e.ci1), ("_ri", e.ri), ("_ri1", e.ri1),
                               ("_fl", e.fl), ("_i", e.pi), ("_j", e.pj)):
                    setattr(e, k, E._Scatter(idx, g.N))
            runs.append(e.step_backward(rho, a["h_log"], a["nsub"], g_out)["g_in"].astype(np.float64))
        sc = np.abs(runs[0]).max(1, keepdims=True)
        out[dtype] = np.max((np.abs(runs[0] - runs[1]) / sc)[~held])
    print(f"order sensitivity, bins empty at the start: FP64 {out[np.float64]:.2e}, "
          f"long double {out[LD]:.2e} of the largest component")
    assert out[np.float64] > 1e-5
    assert out[LD] < 1e-6 and out[LD] < 1e-3 * out[np.float64]
