"""GPU parity of the FP64 path against the CPU oracle, through the C ABI.

Inputs are seeded synthetic discs (paper_2402_18471_amd.disc) on the
configuration grids; both sides get the same grid (identical bits, see
test_abi.py) and the same rates where a call takes rates as input.

Tolerances (FP64): both sides evaluate the same formulas in a different
order (atomics, fused multiply-adds, the suffix-sum form of the fragment
distribution, device exp/sqrt vs libm), so results agree to a few ulp of the
gross terms that make them up:
  rates        |dK| <= 1e-12 (Kc + Kf)
  rhs          |df_k| <= 1e-12 (gain_k + loss_k)
  step         against the oracle's extended-precision evaluation of the same
               steps (oracle/extended.py: the oracle's tables and rates, long
               double arithmetic), with
                 base = 1e-12 |rho_k| + 1e-13 dt (gain_k + loss_k) + 1e-14 atol
               (atol = 1e-10 sum rho; gain, loss at the start state): the
               rounding bound of evaluating gain - loss, which nearly cancel in
               heavy bins sweeping up light grains.
                 batched kernel   |rho_gpu - rho_ld| <= 0.05 base
                 per-cell kernel  |rho_gpu - rho_ld| <= base + |rho_oracle - rho_ld|
               The batched kernel folds the heavier grain's loss into the
               redistribution entries before any product (an exact FP64
               difference), so it carries far less of that rounding than the
               oracle's literal order (measured: <= 0.0023 base, where the
               oracle reaches 7 base on a start populated in every bin); the
               per-cell kernels sum in the oracle's way and are held to be no
               farther from the exact-arithmetic result than the oracle is.
  adjoint      |dg| <= 1e-9 max|g| on a well-conditioned grid
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _np(t):
    return t.detach().cpu().numpy()


def make_ctx(m, me, s, kernel=None, **kw):
    """A context whose FP64 steps take the given kernel ("batch": 16 cells per
    workgroup on the matrix cores, "cell": one workgroup per cell)."""
    from paper_2402_18471_amd.coag import coag_create
    old = os.environ.get("COAG_STEP_KERNEL")
    if kernel is not None:
        os.environ["COAG_STEP_KERNEL"] = kernel
    try:
        return coag_create(m, me, s, **kw)
    finally:
        if old is None:
            os.environ.pop("COAG_STEP_KERNEL", None)
        else:
            os.environ["COAG_STEP_KERNEL"] = old


def _case(O, cfg_name, n_r, n_z, n_bins=None, seed_cells=None, kernel=None):
    from paper_2402_18471_amd import disc
    from paper_2402_18471_amd.coag import coag_mass_grid
    cfg = disc.CONFIGS[cfg_name]
    if (n_r, n_z) != (cfg.n_r, cfg.n_z) or n_bins is not None:
        cfg = disc.scaled(cfg, n_r, n_z, n_bins)
    m, me, s = coag_mass_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    g = O.make_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    d = disc.make_disc(cfg, g.s)
    ctx = make_ctx(m, me, s, kernel, rho_m=cfg.rho_m)
    cells_t = {k: _t(v) for k, v in d["cells"].items()}
    return cfg, g, d, ctx, cells_t


def _rates_tol(gpu, ora, tot):
    return np.all(np.abs(gpu - ora) <= 1e-12 * tot)


@pytest.mark.parametrize("case", [("disc64x32_n100", 8, 4, None),
                                  ("disc256x128_n150", 4, 4, None),
                                  ("disc512x256_n200", 4, 2, None),
                                  ("disc64x32_n100", 3, 1, 2),
                                  ("disc64x32_n100", 2, 1, 1023)])
def test_rates_parity(O, case):
    cfg, g, d, ctx, cells = _case(O, *case)
    Kc, Kf = ctx.coag_rates(cells, _t(d["v_dust"]), _t(d["v_frag"]))
    torch.cuda.synchronize()
    oKc, oKf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    tot = oKc + oKf
    assert _rates_tol(_np(Kc), oKc, tot) and _rates_tol(_np(Kf), oKf, tot), (
        np.max(np.abs(_np(Kc) - oKc) / tot), np.max(np.abs(_np(Kf) - oKf) / tot))


def _spread_rho(d, g, seed=1):
    """A distribution populated in every bin (the MRN start is empty above
    1 um), so that every pair contributes."""
    rng = np.random.default_rng(seed)
    C = d["rho"].shape[0]
    w = rng.uniform(0.1, 1.0, (C, g.N)) * (g.s / g.s[0]) ** -0.5
    return 0.01 * d["cells"]["rho_g"][:, None] * w / w.sum(1, keepdims=True)


@pytest.mark.parametrize("case", [("disc64x32_n100", 8, 4, None),
                                  ("disc256x128_n150", 4, 4, None),
                                  ("disc512x256_n200", 2, 2, None),
                                  ("disc64x32_n100", 3, 1, 2),
                                  ("disc64x32_n100", 1, 1, 1023)])
@pytest.mark.parametrize("chi_split", [(1.0, 0), (2.0, 1), (0.5, 0)])
def test_rhs_parity(O, case, chi_split):
    from paper_2402_18471_amd.coag import coag_create
    chi, split = chi_split
    cfg, g, d, ctx, cells = _case(O, *case)
    g.chi, g.split = chi, split
    ctx = coag_create(ctx.m, ctx.m_edge, ctx.s, rho_m=cfg.rho_m, chi=chi, split=split)
    oKc, oKf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    for rho in (d["rho"], _spread_rho(d, g)):
        f = ctx.coag_rhs(_t(rho), _t(oKc), _t(oKf))
        torch.cuda.synchronize()
        of, gain, loss = O.rhs(g, rho, oKc, oKf, parts=True)
        err = np.abs(_np(f) - of)
        assert np.all(err <= 1e-12 * (gain + loss) + 1e-300), np.max(err / (gain + loss + 1e-300))
        # mass conservation of the GPU right-hand side
        assert np.all(np.abs(_np(f).sum(1)) <= 1e-13 * gain.sum(1))


def _ld_steps(g, Kc, Kf, rho0, h_log, nsub):
    """The same steps in the oracle's extended-precision evaluation."""
    from oracle import extended
    return extended.Extended(g, Kc, Kf).step(rho0, h_log, nsub).astype(np.float64)


def _step_ok(gpu, ora, ld, rho0, gl_dt, kernel):
    """Per-bin step bar against the extended-precision result (module
    docstring); returns the boolean array."""
    atol = 1e-10 * rho0.sum(1, keepdims=True)
    base = 1e-12 * np.abs(ld) + 1e-13 * gl_dt + 1e-14 * atol
    if kernel == "batch":
        return np.abs(gpu - ld) <= 0.05 * base
    return np.abs(gpu - ld) <= base + np.abs(ora - ld)


def _gl_dt(O, g, rho0, Kc, Kf, dt):
    _, gain, loss = O.rhs(g, rho0, Kc, Kf, parts=True)
    return dt * (gain + loss)


KERNELS = ["batch", "cell"]


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("case", [("disc64x32_n100", 8, 4, None),
                                  ("disc256x128_n150", 4, 2, None),
                                  ("disc64x32_n100", 5, 7, None),
                                  # 20 batches of 16 cells: two whole groups of eight
                                  # workgroups (the second dealt to the XCDs rotated)
                                  # and a group of four
                                  ("disc64x32_n100", 20, 16, None)])
def test_step_fixed_parity(O, case, kernel):
    cfg, g, d, ctx, cells = _case(O, *case, kernel=kernel)
    oKc, oKf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    C = d["rho"].shape[0]
    # the populated-everywhere start takes shorter steps: with a full dt and three
    # fixed steps its heaviest bins are outside the integrator's stability region
    # and the result (oracle included) amplifies 1e-15 input noise to 20 %
    for rho0, dt, n in ((d["rho"], d["dt"], 4), (_spread_rho(d, g), d["dt"] / 1000, 3)):
        rho = _t(rho0)
        nsub = _t(np.full(C, n), torch.int32)
        r = ctx.coag_step(rho, _t(oKc), _t(oKf), dt, mode=1, nsub=nsub, max_sub=8)
        torch.cuda.synchronize()
        o = O.step(g, rho0, oKc, oKf, dt, mode=O.FIXED, nsub=n)
        ld = _ld_steps(g, oKc, oKf, rho0, o["h_log"], o["nsub"])
        ok = _step_ok(_np(r["rho"]), o["rho"], ld, rho0, _gl_dt(O, g, rho0, oKc, oKf, dt), kernel)
        assert np.all(ok), np.max(np.abs(_np(r["rho"]) - ld) / (np.abs(ld) + 1e-300))
        assert np.all(_np(r["status"]) == 0)
        np.testing.assert_array_equal(_np(r["h_log"])[:, :n], o["h_log"][:, :n])


@pytest.mark.parametrize("chi", [2.0, 0.5])
def test_batched_step_other_crater_yields(O, chi):
    """The batched FP64 step with chi = 2 (destroyed targets below the
    diagonal) and chi = 1/2 (every collision craters)."""
    cfg, g, d, ctx, cells = _case(O, "disc256x128_n150", 8, 4, kernel="batch")
    g.chi = chi
    ctx = make_ctx(ctx.m, ctx.m_edge, ctx.s, "batch", rho_m=cfg.rho_m, chi=chi)
    oKc, oKf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    C, n, dt = d["rho"].shape[0], 3, d["dt"] * 4
    rho0 = d["rho"]

    from paper_2402_18471_amd.coag import block
    # the blocked layout is one only the batched kernel takes (COAG_ENOTSUP,
    # raised, if this grid and chi did not allow it)
    r = ctx.coag_step(_t(rho0), block(oKc, oKf), None, dt, mode=1,
                      nsub=_t(np.full(C, n), torch.int32), max_sub=8)
    torch.cuda.synchronize()
    o = O.step(g, rho0, oKc, oKf, dt, mode=O.FIXED, nsub=n)
    ld = _ld_steps(g, oKc, oKf, rho0, o["h_log"], o["nsub"])
    assert np.all(_np(r["status"]) == 0)
    assert np.all(_step_ok(_np(r["rho"]), o["rho"], ld, rho0, _gl_dt(O, g, rho0, oKc, oKf, dt),
                           "batch"))


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("case", [("disc64x32_n100", 16, 8, None),
                                  ("disc256x128_n150", 8, 4, None),
                                  ("disc512x256_n200", 4, 2, None)])
def test_step_adaptive_parity_by_replay(O, case, kernel):
    """ADAPTIVE on the GPU, then the oracle replays the GPU's accepted steps:
    states agree per bin; the accept/reject counts agree with the oracle's
    own adaptive run in nearly every cell (rounding can flip a borderline
    decision)."""
    cfg, g, d, ctx, cells = _case(O, *case, kernel=kernel)
    oKc, oKf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    rho0 = d["rho"]
    dt = d["dt"] * 20
    r = ctx.coag_step(_t(rho0), _t(oKc), _t(oKf), dt, max_sub=256)
    torch.cuda.synchronize()
    st, ns, hl = _np(r["status"]), _np(r["nsub"]), _np(r["h_log"])
    assert np.all(st == 0)
    o = O.step(g, rho0, oKc, oKf, dt, mode=O.REPLAY, nsub=ns, h_log=hl)["rho"]
    ld = _ld_steps(g, oKc, oKf, rho0, hl, ns)
    assert np.all(_step_ok(_np(r["rho"]), o, ld, rho0, _gl_dt(O, g, rho0, oKc, oKf, dt), kernel))
    oa = O.step(g, rho0, oKc, oKf, dt, max_sub=256)
    same = (oa["nsub"] == ns) & (oa["nrej"] == _np(r["nrej"]))
    assert same.mean() >= 0.99
    # sub-steps tile dt exactly and h is the next unclipped proposal
    for q in range(len(ns)):
        assert abs(hl[q, : ns[q]].sum() / dt - 1) < 1e-12
    # mass conservation
    m0, m1 = rho0.sum(1), _np(r["rho"]).sum(1)
    assert np.max(np.abs(m1 / m0 - 1)) < 1e-13


def test_all_cells_of_the_64x32_disc_over_calls_replayed_by_oracle(O):
    """The whole 64x32-cell, 100-bin disc (2048 cells), three ADAPTIVE calls
    of dt = 10 yr on the batched FP64 step, the state carried from call to
    call; the oracle replays the GPU's step sequence of each call from its own
    state at the call's start.  Every cell: GPU within the rounding bar of
    the oracle's FP64 result; every eighth cell (256): GPU within the batched
    kernel's bar of the oracle's extended-precision chain."""
    cfg, g, d, ctx, cells = _case(O, "disc64x32_n100", 64, 32, None, kernel="batch")
    oKc, oKf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    dt = d["dt"]
    rho_g = _t(d["rho"])
    h = torch.zeros(cfg.n_cells, dtype=torch.float64, device=DEV)
    logs, gpu_states = [], []
    for _ in range(3):
        r = ctx.coag_step(rho_g, _t(oKc), _t(oKf), dt, h=h, max_sub=256)
        torch.cuda.synchronize()
        assert np.all(_np(r["status"]) == 0)
        logs.append((_np(r["nsub"]).copy(), _np(r["h_log"]).copy()))
        gpu_states.append(_np(rho_g).copy())
    from oracle import extended
    sel = np.arange(0, cfg.n_cells, 8)
    ext = extended.Extended(g, oKc[sel], oKf[sel])
    x, xl = d["rho"], d["rho"][sel].astype(np.longdouble)
    for k, (ns, hl) in enumerate(logs):
        xo = O.step(g, x, oKc, oKf, dt, mode=O.REPLAY, nsub=ns, h_log=hl)["rho"]
        xl = ext.step(xl, hl[sel], ns[sel])
        gl = _gl_dt(O, g, x, oKc, oKf, dt)
        base = 1e-12 * np.abs(xo) + 1e-13 * gl + 1e-14 * 1e-10 * x.sum(1, keepdims=True)
        ok = np.abs(gpu_states[k] - xo) <= base
        assert np.all(ok), (k, np.argwhere(~ok)[:5])
        ld = xl.astype(np.float64)
        assert np.all(_step_ok(gpu_states[k][sel], xo[sel], ld, x[sel], gl[sel], "batch")), k
        x = xo
    assert sum(int(ns.sum()) for ns, _ in logs) > 2 * cfg.n_cells


@pytest.mark.parametrize("kernel", KERNELS)
def test_step_renorm_and_status(O, kernel):
    cfg, g, d, ctx, cells = _case(O, "disc64x32_n100", 4, 2, None, kernel=kernel)
    oKc, oKf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    rho0 = d["rho"].copy()
    rho0[1, 5] = np.nan
    r = ctx.coag_step(_t(rho0), _t(oKc), _t(oKf), d["dt"], renorm=True, check_status=False)
    torch.cuda.synchronize()
    st = _np(r["status"])
    assert st[1] == 3 and np.all(np.delete(st, 1) == 0)
    ok = np.delete(np.arange(rho0.shape[0]), 1)
    m0, m1 = rho0[ok].sum(1), _np(r["rho"])[ok].sum(1)
    assert np.max(np.abs(m1 / m0 - 1)) < 1e-15
    # max_sub exhausted
    r = ctx.coag_step(_t(d["rho"]), _t(oKc), _t(oKf), d["dt"] * 1e4, max_sub=2, check_status=False)
    torch.cuda.synchronize()
    assert np.any(_np(r["status"]) == 2)
    # by default the binding raises on the failed cells
    from paper_2402_18471_amd import _lib as L
    with pytest.raises(L.CoagCellError) as ei:
        ctx.coag_step(_t(d["rho"]), _t(oKc), _t(oKf), d["dt"] * 1e4, max_sub=2)
    assert ei.value.counts.get(L.CELL_MAXSUB, 0) > 0


def test_zero_cells_is_a_no_op(O):
    cfg, g, d, ctx, cells = _case(O, "disc64x32_n100", 1, 1, None)
    e = torch.empty((0, g.N), dtype=torch.float64, device=DEV)
    k = torch.empty((0, g.P), dtype=torch.float64, device=DEV)
    out = ctx.coag_rhs(e, k, k)
    r = ctx.coag_step(e, k, k, 1.0)
    torch.cuda.synchronize()
    assert out.shape == (0, g.N) and r["rho"].shape == (0, g.N)


def test_host_errors_leave_outputs_untouched(O):
    from paper_2402_18471_amd._lib import CoagError
    cfg, g, d, ctx, cells = _case(O, "disc64x32_n100", 1, 2, None)
    oKc, oKf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    rho = _t(d["rho"])
    before = rho.clone()
    with pytest.raises(CoagError):
        ctx.coag_step(rho, _t(oKc), _t(oKf), -1.0)
    with pytest.raises(CoagError):
        ctx.coag_step(rho, _t(oKc), _t(oKf), 1.0, rtol=0.0)
    torch.cuda.synchronize()
    assert torch.equal(rho, before)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("cells_rz", [(4, 2), (5, 7)])
def test_backward_parity(O, kernel, cells_rz):
    """Adjoint on a well-conditioned grid (3 decades of mass): GPU vs oracle,
    with the forward replay on the batched step (REPLAY mode, keeping the
    stage states) or inside the adjoint kernel (per-cell contexts); 8 cells
    (one partial batch of 16) and 35 (two whole batches and a ragged one)."""
    from paper_2402_18471_amd import disc
    from paper_2402_18471_amd.coag import coag_mass_grid
    cfg = disc.scaled(disc.CONFIGS["disc64x32_n100"], *cells_rz, 24)
    m, me, s = coag_mass_grid(24, 3e-4, 3e-3, rho_m=cfg.rho_m)
    g = O.make_grid(24, 3e-4, 3e-3, rho_m=cfg.rho_m)
    d = disc.make_disc(cfg, g.s)
    rng = np.random.default_rng(9)
    rho = 0.01 * d["cells"]["rho_g"][:, None] * rng.uniform(0.2, 1.0, (cfg.n_cells, g.N)) / g.N
    ctx = make_ctx(m, me, s, kernel, rho_m=cfg.rho_m)
    oKc, oKf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    a = O.step(g, rho, oKc, oKf, d["dt"] * 5, max_sub=32)
    g_out = rng.normal(size=rho.shape) / rho.sum(1, keepdims=True)
    og, oa, ov = O.step_backward(g, d["cells"], d["v_dust"], d["v_frag"], rho, 0.0,
                                 a["h_log"], a["nsub"], g_out)
    cells = {k: _t(v) for k, v in d["cells"].items()}
    gi, ga, gv = ctx.coag_step_backward(_t(rho), cells, _t(d["v_dust"]), _t(d["v_frag"]),
                                        _t(a["h_log"]), _t(a["nsub"], torch.int32), _t(g_out))
    torch.cuda.synchronize()
    gi, ga, gv = _np(gi), _np(ga), _np(gv)
    scale = np.abs(og).max(axis=1, keepdims=True)
    assert np.all(np.abs(gi - og) <= 1e-9 * scale), np.max(np.abs(gi - og) / scale)
    np.testing.assert_allclose(ga, oa, rtol=1e-9)
    np.testing.assert_allclose(gv, ov, rtol=1e-9)
