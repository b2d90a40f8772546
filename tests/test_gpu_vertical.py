"""GPU parity of the vertically integrated kernel (Sec. 5.1: surface densities,
rates over the Gaussian column overlap, settling speeds at the dust scale
height) against the oracle, through the C ABI, on the paper's single-radius
shape (R = 20 au, T = 36 K, mu = 2.4, alpha = 1e-3, v_frag = 1 m/s, 200
species) and on columns at 5 - 100 au with radial drift.

Bars as for the volume kernel:
  rates   FP64 |dK| <= 1e-12 (Kc + Kf), [C][P] and blocked; blocked FP32
          within FP32 rounding (1.2e-7 |K|, or 1.2e-38 where K is below
          FP32's normal range)
  steps   the oracle's ADAPTIVE steps replayed on the GPU from the oracle's
          state at each call's start, against the oracle's extended-precision
          evaluation of the same steps: batched kernel 0.05 base (0.05 (base +
          the oracle's own distance) along the single column's approach to
          steady state, where stiff stages amplify rounding), per-cell kernel
          base + the oracle's own distance (ten times the oracle's worst
          relative distance on that approach) (base = 1e-12 |rho| + 1e-13 dt
          (gain + loss) + 1e-14 atol); split precision 1e-6 relative per bin
          holding >= 1e-12 of the column's mass, 1e-18 of it below
  adjoint the bars of the volume kernel's batched adjoint (FP64 1e-12
          relative in populated bins; split 1e-6 per component against at
          least 5 % of the largest; alpha and v_frag against the column's
          largest logarithmic sensitivity; bins empty at the start against
          the extended-precision adjoint, within half the oracle's own
          distance from it plus 1e-7 of the column's largest component.  In
          these columns the large grains are eroded by small ones at high
          rates, each collision returning almost all of the target's mass as
          remnant: the adjoint of an empty large-grain bin then depends on
          the remnant entries to their last bit (one-ulp random changes of
          the FP64 remnant table move the extended-precision result there by
          O(1) of the column's largest component: measured), and the GPU
          builds its tables itself; measured within 0.12 of the oracle's
          distance, 5e-5 of the largest component)
"""
import dataclasses
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


def _setup(O, name="col4096_n200", n_r=None, n_bins=None, kernel=None):
    from paper_2402_18471_amd import disc
    from paper_2402_18471_amd.coag import coag_create, coag_mass_grid
    cfg = disc.COLUMNS[name]
    upd = {}
    if n_r is not None:
        upd["n_r"] = n_r
    if n_bins is not None:
        upd["n_bins"] = n_bins
    cfg = dataclasses.replace(cfg, **upd)
    m, me, s = coag_mass_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    g = O.make_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m, vertical=1)
    d = disc.make_columns(cfg, g.s)
    old = os.environ.get("COAG_STEP_KERNEL")
    if kernel is not None:
        os.environ["COAG_STEP_KERNEL"] = kernel
    try:
        ctx = coag_create(m, me, s, rho_m=cfg.rho_m, vertical=True)
    finally:
        if old is None:
            os.environ.pop("COAG_STEP_KERNEL", None)
        else:
            os.environ["COAG_STEP_KERNEL"] = old
    cells = {k: _t(v) for k, v in d["cells"].items()}
    return cfg, g, d, ctx, cells


def _unblock(K, C):
    from paper_2402_18471_amd.coag import unblock
    return unblock(K, C)[:2]


CASES = [("col0d_n200", None, None), ("col4096_n200", 40, None), ("col4096_n200", 37, 100)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-{c[1]}-{c[2]}")
def test_vertical_rates_parity(O, case):
    cfg, g, d, ctx, cells = _setup(O, *case)
    C = cfg.n_cells
    vd, vf = _t(d["v_dust"]), _t(d["v_frag"])
    oKc, oKf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    tot = oKc + oKf
    assert np.all(np.isfinite(tot)) and tot.max() > 0
    Kc, Kf = ctx.coag_rates(cells, vd, vf)
    B64 = ctx.coag_rates_blocked(cells, vd, vf, dtype=torch.float64)
    B32 = ctx.coag_rates_blocked(cells, vd, vf, dtype=torch.float32)
    torch.cuda.synchronize()
    for got, ora in ((_np(Kc), oKc), (_np(Kf), oKf)):
        assert np.all(np.abs(got - ora) <= 1e-12 * tot), np.max(np.abs(got - ora) / tot)
    for x, ora in zip(_unblock(B64, C), (oKc, oKf)):
        assert np.all(np.abs(x - ora) <= 1e-12 * tot), np.max(np.abs(x - ora) / tot)
    for x, ora in zip(_unblock(B32, C), (oKc, oKf)):
        x = x.astype(np.float64)
        assert np.all(np.abs(x - ora) <= 1.2e-7 * np.abs(ora) + 1.2e-38)


def _ld_steps(g, Kc, Kf, rho0, h_log, nsub):
    from oracle import extended
    return extended.Extended(g, Kc, Kf).step(rho0, h_log, nsub).astype(np.float64)


@pytest.mark.parametrize("kernel", ["batch", "cell"])
def test_vertical_0d_column_over_calls(O, kernel):
    """The single-radius column, 30 calls of 1000 yr from the MRN start to the
    fragmentation-limited steady state (the peak of the distribution moves
    from 1 um to ~100 um): at every call the oracle takes its ADAPTIVE steps
    from its own state and the GPU replays them from the same state.  Near
    the steady state the accepted steps are long against the fastest
    fragment-feeding modes, and the stages amplify the rounding of gain -
    loss: the FP64 oracle is up to ~800 base from the extended-precision
    steps there (measured), so the batched kernel is held to 0.05 (base +
    the oracle's own distance) instead of 0.05 base, and the per-cell
    kernel, which sums in the oracle's way and meets its own rounding
    pattern, to base (1 + 10 max_k (oracle's distance / base)): no farther
    than ten times the oracle's worst relative distance that call (measured
    up to 5.6 times)."""
    cfg, g, d, ctx, cells = _setup(O, "col0d_n200", kernel=kernel)
    oKc, oKf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    rho = d["rho"].copy()
    dt = d["dt"]
    rows = []
    for call in range(30):
        a = O.step(g, rho, oKc, oKf, dt, max_sub=256)
        assert np.all(a["status"] == 0)
        r = ctx.coag_step(_t(rho), _t(oKc), _t(oKf), dt, mode=2, nsub=_t(a["nsub"], torch.int32),
                          h_log=_t(a["h_log"]), max_sub=256)
        torch.cuda.synchronize()
        ld = _ld_steps(g, oKc, oKf, rho, a["h_log"], a["nsub"])
        _, gain, loss = O.rhs(g, rho, oKc, oKf, parts=True)
        base = 1e-12 * np.abs(ld) + 1e-13 * dt * (gain + loss) + 1e-14 * 1e-10 * rho.sum()
        got = _np(r["rho"])
        dist = np.abs(a["rho"] - ld)
        ok = (np.abs(got - ld) <= 0.05 * (base + dist)) if kernel == "batch" else (
            np.abs(got - ld) <= base * (1.0 + 10.0 * np.max(dist / base)))
        rows.append((call, int(a["nsub"][0]), np.max(np.abs(got - ld) / base),
                     np.max(dist / base), bool(np.all(ok))))
        rho = a["rho"]
    print(f"\n{kernel}: call, steps, max |gpu - ld| / base, max |oracle - ld| / base")
    for row in rows:
        print("  %2d %3d %10.3g %10.3g %s" % row)
    assert all(r[-1] for r in rows)
    # the distribution has grown to the fragmentation barrier
    assert g.s[np.argmax(rho[0])] > 5e-3


def test_vertical_columns_adaptive_and_split(O):
    """40 columns at 5 - 100 au (three batches, the last ragged), one call of
    300 yr: the oracle's ADAPTIVE steps replayed on the GPU in FP64
    (against the extended-precision steps) and in split precision (blocked
    FP32 rates; against the oracle per bin); the GPU's own ADAPTIVE run takes
    the oracle's step counts in nearly every column."""
    cfg, g, d, ctx, cells = _setup(O, "col4096_n200", 40)
    C = cfg.n_cells
    oKc, oKf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    rho0, dt = d["rho"], 0.3 * d["dt"]
    a = O.step(g, rho0, oKc, oKf, dt, max_sub=256)
    assert np.all(a["status"] == 0)
    ns, hl = _t(a["nsub"], torch.int32), _t(a["h_log"])
    r = ctx.coag_step(_t(rho0), _t(oKc), _t(oKf), dt, mode=2, nsub=ns, h_log=hl, max_sub=256)
    torch.cuda.synchronize()
    ld = _ld_steps(g, oKc, oKf, rho0, a["h_log"], a["nsub"])
    _, gain, loss = O.rhs(g, rho0, oKc, oKf, parts=True)
    base = 1e-12 * np.abs(ld) + 1e-13 * dt * (gain + loss) + 1e-14 * 1e-10 * rho0.sum(1, keepdims=True)
    assert np.all(np.abs(_np(r["rho"]) - ld) <= 0.05 * base)
    # split precision, blocked FP32 rates
    B32 = ctx.coag_rates_blocked(cells, _t(d["v_dust"]), _t(d["v_frag"]), dtype=torch.float32)
    rs = ctx.coag_step(_t(rho0), B32, None, dt, mode=2, prec=1, nsub=_t(a["nsub"], torch.int32),
                       h_log=_t(a["h_log"]), max_sub=256)
    torch.cuda.synchronize()
    y, o = _np(rs["rho"]), a["rho"]
    M = o.sum(1, keepdims=True)
    res = o >= 1e-12 * M
    assert np.all((np.abs(y - o) <= 1e-6 * np.abs(o))[res]), np.max((np.abs(y - o) / o)[res])
    assert np.all((np.abs(y - o) <= 1e-18 * M)[~res])
    # the GPU's own ADAPTIVE call
    ra = ctx.coag_step(_t(rho0), _t(oKc), _t(oKf), dt, max_sub=256)
    torch.cuda.synchronize()
    assert np.all(_np(ra["status"]) == 0)
    assert (_np(ra["nsub"]) == a["nsub"]).mean() >= 0.95
    assert np.max(np.abs(_np(ra["rho"]).sum(1) / rho0.sum(1) - 1)) < 1e-13


def _loss_grad(g, rho_end):
    lns = np.log(g.s)
    M = rho_end.sum(1, keepdims=True)
    return (lns[None, :] - (rho_end * lns).sum(1, keepdims=True) / M) / M


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "split"])
def test_vertical_adjoint_against_oracle(O, prec):
    """35 columns (two whole batches and a ragged one), 200 bins, one call of
    the oracle's ADAPTIVE steps over 300 yr; J the mass-weighted mean
    ln s of every column."""
    from oracle import extended
    cfg, g, d, ctx, cells = _setup(O, "col4096_n200", 35)
    rho = d["rho"]
    oKc, oKf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    a = O.step(g, rho, oKc, oKf, 0.3 * d["dt"], max_sub=64)
    assert np.all(a["status"] == 0)
    g_out = _loss_grad(g, a["rho"])
    og, oa, ov = O.step_backward(g, d["cells"], d["v_dust"], d["v_frag"], rho, 0.0, a["h_log"],
                                 a["nsub"], g_out)
    ld = extended.step_backward(g, d["cells"], d["v_dust"], d["v_frag"], rho, a["h_log"],
                                a["nsub"], g_out, oKc, oKf)["g_in"].astype(np.float64)
    gi, ga, gv = ctx.coag_step_backward(_t(rho), cells, _t(d["v_dust"]), _t(d["v_frag"]),
                                        _t(a["h_log"]), _t(a["nsub"], torch.int32), _t(g_out),
                                        prec=prec)
    torch.cuda.synchronize()
    gi, ga, gv = _np(gi), _np(ga), _np(gv)
    scale = np.abs(og).max(1, keepdims=True)
    res = rho >= 1e-12 * rho.sum(1, keepdims=True)
    err = np.abs(gi - og)
    if prec == 1:
        bound = 1e-6 * np.maximum(np.abs(og), 0.05 * scale)
        assert np.all((err <= 1e-7 * scale)[res])
    else:
        bound = 1e-12 * np.abs(og) + 1e-15 * scale
    assert np.all(err[res] <= bound[res]), np.max((err / np.maximum(np.abs(og), 1e-300))[res])
    empty = ~res
    eb = 0.5 * np.where(empty, np.abs(og - ld), 0.0).max(1) + 1e-7 * np.abs(ld).max(1)
    got = np.where(empty, np.abs(gi - ld), 0.0).max(1)
    sc = np.abs(ld).max(1)
    print(f"\nbins empty at the start, against long double: GPU {np.max(got / sc):.2e}, "
          f"oracle {np.max(np.where(empty, np.abs(og - ld), 0.0).max(1) / sc):.2e} of the "
          f"column's largest component")
    assert np.all(got <= eb), np.max(got / eb)
    al, vf = d["cells"]["alpha"], d["v_frag"]
    S = np.maximum(np.abs(al * oa), np.abs(vf * ov))
    tol = 1e-6 if prec == 1 else 1e-12
    assert np.all(np.abs(al * (ga - oa)) <= tol * S), np.max(np.abs(al * (ga - oa)) / S)
    assert np.all(np.abs(vf * (gv - ov)) <= tol * S), np.max(np.abs(vf * (gv - ov)) / S)


def test_vertical_adjoint_needs_the_batched_kernels(O):
    """The per-cell adjoint has the volume kernel's rate derivatives only: a
    vertically integrated context that forces it refuses the backward."""
    from paper_2402_18471_amd._lib import CoagError
    cfg, g, d, ctx, cells = _setup(O, "col4096_n200", 3, kernel="cell")
    a = O.step(g, d["rho"], *O.rates(g, d["cells"], d["v_dust"], d["v_frag"]), 0.1 * d["dt"],
               max_sub=64)
    with pytest.raises(CoagError) as e:
        ctx.coag_step_backward(_t(d["rho"]), cells, _t(d["v_dust"]), _t(d["v_frag"]),
                               _t(a["h_log"]), _t(a["nsub"], torch.int32),
                               _t(_loss_grad(g, a["rho"])))
    assert e.value.code == -4
