"""The batched adjoint of coag_step (coag_step_backward, FP64 and split BF16)
against the oracle's hand-written FP64 adjoint, through the C ABI.

One coagulation call per case: the oracle's own ADAPTIVE step over 5 dt gives
the step sequence (h_log), both sides differentiate J = sum over cells of the
mass-weighted mean ln s after that call, with respect to the state at its
start, alpha and v_frag.  The GPU replays the steps in its own precision (the
split form along its own split-precision trajectory) and compares with the
oracle's FP64 gradient.

Bars, per cell:
  bins populated at the start (rho_k >= 1e-12 sum rho):
      FP64   |dg_k| <= 1e-12 |g_k| + 1e-15 max|g|
      split  |dg_k| <= 1e-6 max(|g_k|, 0.05 max|g|)   (relative per bin; the
             gradient of a mean log size changes sign across the bins, so
             relative errors are taken against at least 5 % of the cell's
             largest component), and |dg| <= 1e-7 max|g| everywhere there
  bins empty at the start: dJ/drho_k there is ill-conditioned (its terms
      cancel to 13 digits): the FP64 oracle is 1e-3 .. 4e-3 of the cell's
      largest component away from the exact-arithmetic value, so both sides
      are held to the oracle's extended-precision adjoint (oracle/extended.py)
      instead, per cell over those bins:
        batched kernels   max|g - g_ld| <= 0.1 max|g_oracle - g_ld| + 1e-12 max|g|
      (they fold the heavier grain's loss into the redistribution entries
      before any product and are measured 60 .. 1000x closer than the
      oracle); the per-cell kernel, which sums in the oracle's order, within
      5x the oracle's largest distance over the cells
  alpha, v_frag: with S = max(|alpha dJ/dalpha|, |v_frag dJ/dv_frag|) the
      cell's largest logarithmic sensitivity, |x d(dJ/dx)| <= tol S, tol =
      1e-12 (FP64), 1e-6 (split).  (Where fragmentation is off, dJ/dv_frag is
      10^-30 .. 10^-250 of S: below the range of the split form's FP32 rates.)
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
CASES = [("disc64x32_n100", 8, 4, None), ("disc256x128_n150", 4, 4, None),
         ("disc512x256_n200", 4, 4, None)]


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _ctx(m, me, s, rho_m, slab=None):
    from paper_2402_18471_amd.coag import coag_create
    old = os.environ.get("COAG_ADJ_SLAB_CELLS")
    if slab is not None:
        os.environ["COAG_ADJ_SLAB_CELLS"] = str(slab)
    try:
        return coag_create(m, me, s, rho_m=rho_m)
    finally:
        if old is None:
            os.environ.pop("COAG_ADJ_SLAB_CELLS", None)
        else:
            os.environ["COAG_ADJ_SLAB_CELLS"] = old


def _setup(O, case):
    from paper_2402_18471_amd import disc
    from paper_2402_18471_amd.coag import coag_mass_grid
    name, nr, nz, nb = case
    cfg = disc.scaled(disc.CONFIGS[name], nr, nz, nb)
    m, me, s = coag_mass_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    g = O.make_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    d = disc.make_disc(cfg, g.s)
    return cfg, g, d, (m, me, s)


def _loss_grad(g, rho_end):
    lns = np.log(g.s)
    M = rho_end.sum(1, keepdims=True)
    return (lns[None, :] - (rho_end * lns).sum(1, keepdims=True) / M) / M


def _oracle_call(O, g, d, rho, dt):
    oKc, oKf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    a = O.step(g, rho, oKc, oKf, dt, max_sub=64)
    assert np.all(a["status"] == 0)
    g_out = _loss_grad(g, a["rho"])
    og, oa, ov = O.step_backward(g, d["cells"], d["v_dust"], d["v_frag"], rho, 0.0,
                                 a["h_log"], a["nsub"], g_out)
    return a, g_out, og, oa, ov


def _ld_adjoint(g, d, rho, a, g_out):
    """The oracle's adjoint of the same call in extended precision."""
    from oracle import extended
    oKc, oKf = _oracle_rates(g, d)
    r = extended.step_backward(g, d["cells"], d["v_dust"], d["v_frag"], rho, a["h_log"],
                               a["nsub"], g_out, oKc, oKf)
    return r["g_in"].astype(np.float64)


def _oracle_rates(g, d):
    import oracle as O
    return O.rates(g, d["cells"], d["v_dust"], d["v_frag"])


def _empty_bound(rho, og, ld, factor):
    """Per-cell bound over the bins empty at the start: factor times the
    oracle's own largest distance from the extended-precision adjoint there,
    plus 1e-12 of the cell's largest component."""
    empty = rho < 1e-12 * rho.sum(1, keepdims=True)
    scale = np.abs(ld).max(1)
    return factor * np.where(empty, np.abs(og - ld), 0.0).max(1) + 1e-12 * scale, empty


def _gpu_backward(ctx, d, rho, a, g_out, prec):
    cells = {k: _t(v) for k, v in d["cells"].items()}
    gi, ga, gv = ctx.coag_step_backward(_t(rho), cells, _t(d["v_dust"]), _t(d["v_frag"]),
                                        _t(a["h_log"]), _t(a["nsub"], torch.int32), _t(g_out),
                                        prec=prec)
    torch.cuda.synchronize()
    return gi.cpu().numpy(), ga.cpu().numpy(), gv.cpu().numpy()


def _check(d, rho, og, oa, ov, ld, gi, ga, gv, split):
    scale = np.abs(og).max(1, keepdims=True)
    res = rho >= 1e-12 * rho.sum(1, keepdims=True)
    err = np.abs(gi - og)
    if split:
        bound = 1e-6 * np.maximum(np.abs(og), 0.05 * scale)
        assert np.all((err <= 1e-7 * scale)[res]), np.max((err / scale)[res])
    else:
        bound = 1e-12 * np.abs(og) + 1e-15 * scale
    assert np.all(err[res] <= bound[res]), np.max((err / np.maximum(np.abs(og), 1e-300))[res])
    if ld is not None:
        eb, empty = _empty_bound(rho, og, ld, 0.1)
        got = np.where(empty, np.abs(gi - ld), 0.0).max(1)
        assert np.all(got <= eb), np.max(got / eb)
    al, vf = d["cells"]["alpha"], d["v_frag"]
    S = np.maximum(np.abs(al * oa), np.abs(vf * ov))
    tol = 1e-6 if split else 1e-12
    assert np.all(np.abs(al * (ga - oa)) <= tol * S), np.max(np.abs(al * (ga - oa)) / S)
    assert np.all(np.abs(vf * (gv - ov)) <= tol * S), np.max(np.abs(vf * (gv - ov)) / S)
    return np.max((err / scale)[res])


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "split"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_adjoint_one_call_against_oracle(O, case, prec):
    cfg, g, d, (m, me, s) = _setup(O, case)
    rho = d["rho"]
    a, g_out, og, oa, ov = _oracle_call(O, g, d, rho, d["dt"] * 5)
    ld = _ld_adjoint(g, d, rho, a, g_out)
    ctx = _ctx(m, me, s, cfg.rho_m)
    gi, ga, gv = _gpu_backward(ctx, d, rho, a, g_out, prec)
    _check(d, rho, og, oa, ov, ld, gi, ga, gv, prec == 1)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "split"])
def test_adjoint_ragged_batches_well_conditioned(O, prec):
    """35 cells (two whole batches of 16 and a ragged one) on a 24-bin grid
    spanning one decade of size, a random g_out: every bin populated."""
    from paper_2402_18471_amd import disc
    from paper_2402_18471_amd.coag import coag_mass_grid
    cfg = disc.scaled(disc.CONFIGS["disc64x32_n100"], 5, 7, 24)
    m, me, s = coag_mass_grid(24, 3e-4, 3e-3, rho_m=cfg.rho_m)
    g = O.make_grid(24, 3e-4, 3e-3, rho_m=cfg.rho_m)
    d = disc.make_disc(cfg, g.s)
    rng = np.random.default_rng(9)
    rho = 0.01 * d["cells"]["rho_g"][:, None] * rng.uniform(0.2, 1.0, (cfg.n_cells, g.N)) / g.N
    oKc, oKf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    a = O.step(g, rho, oKc, oKf, d["dt"] * 5, max_sub=32)
    g_out = rng.normal(size=rho.shape) / rho.sum(1, keepdims=True)
    og, oa, ov = O.step_backward(g, d["cells"], d["v_dust"], d["v_frag"], rho, 0.0,
                                 a["h_log"], a["nsub"], g_out)
    ctx = _ctx(m, me, s, cfg.rho_m)
    gi, ga, gv = _gpu_backward(ctx, d, rho, a, g_out, prec)
    _check(d, rho, og, oa, ov, None, gi, ga, gv, prec == 1)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "split"])
def test_slabs_give_the_same_gradients(O, prec):
    """The adjoint's workspace holds a slab of cells at a time: slabs of 16
    and 48 cells (the 70-cell disc in 5 and 2 slabs, the last ragged) give
    what one slab of all cells gives, up to the order of LDS atomics."""
    cfg, g, d, (m, me, s) = _setup(O, ("disc64x32_n100", 10, 7, 40))
    rho = d["rho"]
    a, g_out, og, oa, ov = _oracle_call(O, g, d, rho, d["dt"] * 5)
    ref = _gpu_backward(_ctx(m, me, s, cfg.rho_m), d, rho, a, g_out, prec)
    for slab in (16, 48):
        got = _gpu_backward(_ctx(m, me, s, cfg.rho_m, slab=slab), d, rho, a, g_out, prec)
        for x, y in zip(got, ref):
            sc = np.abs(y).max()
            assert np.all(np.abs(x - y) <= 1e-12 * sc), (slab, np.max(np.abs(x - y)) / sc)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "split"])
def test_invalid_step_counts_give_nan_for_those_cells_only(O, prec):
    cfg, g, d, (m, me, s) = _setup(O, ("disc64x32_n100", 4, 5, 40))
    rho = d["rho"]
    a, g_out, og, oa, ov = _oracle_call(O, g, d, rho, d["dt"] * 2)
    ns = a["nsub"].copy()
    ns[3] = -1
    ns[17] = a["h_log"].shape[1] + 1
    bad = dict(a, nsub=ns)
    ctx = _ctx(m, me, s, cfg.rho_m)
    gi, ga, gv = _gpu_backward(ctx, d, rho, bad, g_out, prec)
    gi2, ga2, gv2 = _gpu_backward(ctx, d, rho, a, g_out, prec)
    for c in (3, 17):
        assert np.all(np.isnan(gi[c])) and np.isnan(ga[c]) and np.isnan(gv[c])
    ok = np.ones(len(rho), bool)
    ok[[3, 17]] = False
    assert np.all(np.isfinite(gi[ok])) and np.all(np.isfinite(ga[ok]))
    sc = np.abs(gi2[ok]).max()
    assert np.all(np.abs(gi[ok] - gi2[ok]) <= 1e-12 * sc)


def test_zero_steps_pass_the_cotangent_through(O):
    """nsub = 0: the call is the identity, g_in = g_out, no alpha / v_frag
    dependence; in place (g_in aliasing g_out) through the C ABI."""
    import ctypes as ct
    from paper_2402_18471_amd import _lib as L
    cfg, g, d, (m, me, s) = _setup(O, ("disc64x32_n100", 2, 9, 40))
    ctx = _ctx(m, me, s, cfg.rho_m)
    C = cfg.n_cells
    cells = {k: _t(v) for k, v in d["cells"].items()}
    cs = L.Cells(*[cells[k].data_ptr() for k in ("T", "rho_g", "c_s", "Omega", "H", "nu_mol",
                                                 "alpha")])
    rng = np.random.default_rng(2)
    gbuf = _t(rng.normal(size=(C, g.N)))
    g0 = gbuf.clone()
    ga = torch.full((C,), 7.0, dtype=torch.float64, device=DEV)
    gv = torch.full((C,), 7.0, dtype=torch.float64, device=DEV)
    hl = torch.zeros((C, 4), dtype=torch.float64, device=DEV)
    ns = torch.zeros(C, dtype=torch.int32, device=DEV)
    p = lambda x: ct.c_void_p(x.data_ptr())
    for prec in (0, 1):
        L.check(ctx._lib.coag_step_backward(ctx._h, C, p(_t(d["rho"])), ct.byref(cs),
                                            p(_t(d["v_dust"])), p(_t(d["v_frag"])), p(hl), 4,
                                            p(ns), p(gbuf), p(gbuf), p(ga), p(gv), prec,
                                            ct.c_void_p(torch.cuda.current_stream().cuda_stream)),
                ctx._h)
        torch.cuda.synchronize()
        assert torch.equal(gbuf, g0)
        assert torch.all(ga == 0) and torch.all(gv == 0)


def test_batched_and_per_cell_adjoints_agree_on_the_100_bin_grid(O):
    """The batched adjoint (16 cells per workgroup, matrix cores) and the
    per-cell one (COAG_STEP_KERNEL=cell: one workgroup per cell, its own
    replay, dJ/dK per pair) on 35 cells of the 100-bin disc (two whole
    batches and a ragged one), one call: populated bins to 1e-12 relative;
    bins empty at the start against the extended-precision adjoint, the
    batched kernel within 0.1x the oracle's own distance from it per cell,
    the per-cell one within 5x its largest distance over the cells."""
    from paper_2402_18471_amd.coag import coag_create
    cfg, g, d, (m, me, s) = _setup(O, ("disc64x32_n100", 5, 7, None))
    rho = d["rho"]
    a, g_out, og, oa, ov = _oracle_call(O, g, d, rho, d["dt"] * 5)
    ld = _ld_adjoint(g, d, rho, a, g_out)
    old = os.environ.get("COAG_STEP_KERNEL")
    os.environ["COAG_STEP_KERNEL"] = "cell"
    try:
        cell_ctx = coag_create(m, me, s, rho_m=cfg.rho_m)
    finally:
        if old is None:
            os.environ.pop("COAG_STEP_KERNEL", None)
        else:
            os.environ["COAG_STEP_KERNEL"] = old
    gb, ab, vb = _gpu_backward(_ctx(m, me, s, cfg.rho_m), d, rho, a, g_out, 0)
    gc, ac, vc = _gpu_backward(cell_ctx, d, rho, a, g_out, 0)
    scale = np.abs(gc).max(1, keepdims=True)
    res = rho >= 1e-12 * rho.sum(1, keepdims=True)
    err = np.abs(gb - gc)
    assert np.all((err <= 1e-12 * np.abs(gc) + 1e-15 * scale)[res])
    eb, empty = _empty_bound(rho, og, ld, 0.1)
    e = np.where(empty, np.abs(gb - ld), 0.0).max(1)
    assert np.all(e <= eb), np.max(e / eb)
    # the per-cell kernel: within 5x the oracle's largest distance over the cells
    # (its error and the oracle's are of one kind, FP64 in the literal order, so
    # a single cell can find the oracle luckier than itself)
    e_cell = np.where(empty, np.abs(gc - ld), 0.0).max()
    e_ora = np.where(empty, np.abs(og - ld), 0.0).max()
    assert e_cell <= 5.0 * e_ora, e_cell / e_ora
    al, vf = d["cells"]["alpha"], d["v_frag"]
    S = np.maximum(np.abs(al * ac), np.abs(vf * vc))
    assert np.all(np.abs(al * (ab - ac)) <= 1e-12 * S)
    assert np.all(np.abs(vf * (vb - vc)) <= 1e-12 * S)
