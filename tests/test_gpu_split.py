"""Split-BF16 step (COAG_PREC_SPLIT_BF16) and blocked FP32 rates against the FP64 oracle.

The split arithmetic perturbs every right-hand side by a few 2^-24 of the
gain terms of each bin (the gain contraction runs on three-limb BF16 products
with FP32 accumulation; losses, fragments, stage states, control and update
stay FP64).  To measure that perturbation and nothing else, the GPU replays a
step sequence the oracle also takes (REPLAY of the oracle's adaptive steps,
or the split step's own adaptive steps replayed by the oracle).  Bar, per bin
of every cell:
    |rho_split - rho_oracle| <= 1e-6 |rho_oracle| + 1e-18 sum_k rho_k
i.e. 1e-6 relative in every bin that holds more than 1e-12 of the cell's mass
("resolved"), with the absolute floor reached only by bins below 1e-12 of it;
and the total mass of every cell conserved to 1e-12 (FP64 bookkeeping at the
end of each call).  Starting states: the MRN start over dt and over 20 dt, and
a state evolved by the oracle for 100 dt (then one call of dt).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _np(t):
    return t.detach().cpu().numpy()


def _case(O, name, n_r, n_z):
    from paper_2402_18471_amd import disc
    from paper_2402_18471_amd.coag import coag_create, coag_mass_grid
    cfg = disc.scaled(disc.CONFIGS[name], n_r, n_z, None)
    m, me, s = coag_mass_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    g = O.make_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    d = disc.make_disc(cfg, g.s)
    ctx = coag_create(m, me, s, rho_m=cfg.rho_m)
    cells = {k: _t(v) for k, v in d["cells"].items()}
    return cfg, g, d, ctx, cells


def _bar(gpu, ora, rho0):
    M = rho0.sum(1, keepdims=True)
    lim = 1e-6 * np.abs(ora) + 1e-18 * M
    return np.abs(gpu - ora) <= lim, np.max(np.abs(gpu - ora) / lim)


def _evolved(O, g, d, Kc, Kf):
    r = O.step(g, d["rho"], Kc, Kf, 100 * d["dt"], max_sub=2048)
    assert np.all(r["status"] == 0)
    return r["rho"]


CASES = [("disc64x32_n100", 8, 4), ("disc256x128_n150", 8, 4), ("disc512x256_n200", 4, 4),
         ("disc256x128_n150", 5, 7)]


def _unblock(K, C):
    """Blocked rates -> Kc, Kf [C][P] (float64), and the padding values."""
    from paper_2402_18471_amd.coag import unblock
    a, b, rest = unblock(K, C)
    return a.astype(np.float64), b.astype(np.float64), rest


# (13, 3) and (5, 7): a ragged last block of 16 cells.  The writer keeps
# fewer per-grain values in LDS as the grid grows: all of them at 100 and 150
# bins, St and the velocity at 200, St alone at 320 bins.
RATE_CASES = CASES[:3] + [("disc64x32_n100", 13, 3), ("disc64x32_n100", 5, 7)]


@pytest.mark.parametrize("case", RATE_CASES + [("disc64x32_n100", 5, 7, 320)])
def test_rates_blocked_f32(O, case):
    if len(case) == 4:
        from paper_2402_18471_amd import disc
        from paper_2402_18471_amd.coag import coag_create, coag_mass_grid
        cfg = disc.scaled(disc.CONFIGS[case[0]], case[1], case[2], case[3])
        m, me, s = coag_mass_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
        g = O.make_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
        d = disc.make_disc(cfg, g.s)
        ctx = coag_create(m, me, s, rho_m=cfg.rho_m)
        cells = {k: _t(v) for k, v in d["cells"].items()}
    else:
        cfg, g, d, ctx, cells = _case(O, *case)
    C = cfg.n_cells
    from paper_2402_18471_amd.coag import pair_slots
    K = ctx.coag_rates_blocked(cells, _t(d["v_dust"]), _t(d["v_frag"]))
    torch.cuda.synchronize()
    assert tuple(K.shape) == ((C + 15) // 16, pair_slots(cfg.n_bins), 64)
    oKc, oKf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    kc, kf, rest = _unblock(K, C)
    for a, b in ((kc, oKc), (kf, oKf)):
        assert np.all(np.abs(a - b) <= 2.0 ** -24 * np.abs(b) + 1e-12 * (oKc + oKf))
    assert np.all(rest == 0.0)


@pytest.mark.parametrize("rates", ["f64", "f32"])
@pytest.mark.parametrize("case", CASES)
def test_split_step_replays_oracle_steps(O, case, rates):
    cfg, g, d, ctx, cells = _case(O, *case)
    oKc, oKf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    if rates == "f32":
        Kc, Kf = ctx.coag_rates_blocked(cells, _t(d["v_dust"]), _t(d["v_frag"])), None
    else:
        Kc, Kf = _t(oKc), _t(oKf)
    for rho0, dt in ((d["rho"], d["dt"]), (d["rho"], 20 * d["dt"]),
                     (_evolved(O, g, d, oKc, oKf), d["dt"])):
        o = O.step(g, rho0, oKc, oKf, dt, max_sub=512)
        assert np.all(o["status"] == 0)
        r = ctx.coag_step(_t(rho0), Kc, Kf, dt, mode=2, prec=1, nsub=_t(o["nsub"], torch.int32),
                          h_log=_t(o["h_log"]))
        torch.cuda.synchronize()
        assert np.all(_np(r["status"]) == 0)
        x = _np(r["rho"])
        ok, worst = _bar(x, o["rho"], rho0)
        assert np.all(ok), worst
        assert np.max(np.abs(x.sum(1) / rho0.sum(1) - 1)) <= 1e-12


@pytest.mark.parametrize("chi", [2.0, 0.5])
def test_split_step_other_crater_yields(O, chi):
    """chi = 2: a projectile destroys targets up to twice its mass, so whole
    chunks below the diagonal mix cratering and destroyed pairs; chi = 1/2:
    every collision craters, the diagonal included."""
    from paper_2402_18471_amd.coag import coag_create
    cfg, g, d, ctx, cells = _case(O, "disc256x128_n150", 8, 4)
    g.chi = chi
    ctx = coag_create(ctx.m, ctx.m_edge, ctx.s, rho_m=cfg.rho_m, chi=chi)
    oKc, oKf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    Kc, Kf = ctx.coag_rates_blocked(cells, _t(d["v_dust"]), _t(d["v_frag"])), None
    for rho0, dt in ((d["rho"], 20 * d["dt"]), (_evolved(O, g, d, oKc, oKf), d["dt"])):
        o = O.step(g, rho0, oKc, oKf, dt, max_sub=512)
        assert np.all(o["status"] == 0)
        r = ctx.coag_step(_t(rho0), Kc, Kf, dt, mode=2, prec=1, nsub=_t(o["nsub"], torch.int32),
                          h_log=_t(o["h_log"]))
        torch.cuda.synchronize()
        assert np.all(_np(r["status"]) == 0)
        x = _np(r["rho"])
        ok, worst = _bar(x, o["rho"], rho0)
        assert np.all(ok), worst
        assert np.max(np.abs(x.sum(1) / rho0.sum(1) - 1)) <= 1e-12


@pytest.mark.parametrize("case", CASES[1:3])
def test_split_adaptive_replayed_by_oracle(O, case):
    """ADAPTIVE split step; the oracle replays its accepted steps."""
    cfg, g, d, ctx, cells = _case(O, *case)
    oKc, oKf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    Kc, Kf = ctx.coag_rates_blocked(cells, _t(d["v_dust"]), _t(d["v_frag"])), None
    rho0, dt = d["rho"], 20 * d["dt"]
    r = ctx.coag_step(_t(rho0), Kc, Kf, dt, prec=1, max_sub=256)
    torch.cuda.synchronize()
    st, ns, hl = _np(r["status"]), _np(r["nsub"]), _np(r["h_log"])
    assert np.all(st == 0)
    for q in range(len(ns)):
        assert abs(hl[q, : ns[q]].sum() / dt - 1) < 1e-12
    o = O.step(g, rho0, oKc, oKf, dt, mode=O.REPLAY, nsub=ns, h_log=hl)
    ok, worst = _bar(_np(r["rho"]), o["rho"], rho0)
    assert np.all(ok), worst
    assert np.max(np.abs(_np(r["rho"]).sum(1) / rho0.sum(1) - 1)) <= 1e-12
    # the step-size controller sees nearly the same errors as in FP64
    oa = O.step(g, rho0, oKc, oKf, dt, max_sub=256)
    assert np.mean(oa["nsub"] == ns) >= 0.95


def test_split_rejections_and_host_errors(O):
    from paper_2402_18471_amd import _lib as L
    from paper_2402_18471_amd.coag import coag_create, coag_mass_grid
    cfg, g, d, ctx, cells = _case(O, "disc64x32_n100", 2, 2)
    oKc, oKf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    Kc32, Kf32 = ctx.coag_rates_blocked(cells, _t(d["v_dust"]), _t(d["v_frag"])), None
    rho = _t(d["rho"])
    before = rho.clone()
    with pytest.raises(L.CoagError) as e:       # FP32 rates with the FP64 step
        ctx.coag_step(rho, Kc32, Kf32, d["dt"], prec=0)
    assert e.value.code == L.COAG_EINVAL
    m, me, s = coag_mass_grid(8, 1e-5, 1e-3)    # fewer bins than the 16-bin window
    small = coag_create(m, me, s)
    z = torch.zeros((1, 36), dtype=torch.float64, device=DEV)
    with pytest.raises(L.CoagError) as e:
        small.coag_step(torch.ones((1, 8), dtype=torch.float64, device=DEV), z, z, 1.0, prec=1)
    assert e.value.code == L.COAG_ENOTSUP
    c1 = {k: v[:1].contiguous() for k, v in cells.items()}
    with pytest.raises(L.CoagError) as e:       # nor the split adjoint
        small.coag_step_backward(torch.ones((1, 8), dtype=torch.float64, device=DEV), c1,
                                 torch.zeros((1, 8, 3), dtype=torch.float64, device=DEV),
                                 _t(d["v_frag"][:1]),
                                 torch.zeros((1, 1), dtype=torch.float64, device=DEV),
                                 torch.zeros(1, dtype=torch.int32, device=DEV),
                                 torch.ones((1, 8), dtype=torch.float64, device=DEV), prec=1)
    assert e.value.code == L.COAG_ENOTSUP
    torch.cuda.synchronize()
    assert torch.equal(rho, before)


@pytest.mark.parametrize("name", ["disc256x128_n150", "disc512x256_n200"])
def test_split_error_on_spread_sample(name):
    """The bench's measurement as a test: 512 cells spread over the full disc
    (cells evolve independently, so the sample alone takes the same path),
    three FP64 calls of dt from the MRN start, then one FP64 call over 20 dt
    that the split step (blocked FP32 rates) replays.  Bar: 1e-6 relative in
    resolved bins (>= 1e-12 of the cell's mass), 1e-18 of the cell's mass in
    the rest, total mass to 1e-12."""
    from paper_2402_18471_amd import _lib as L
    from paper_2402_18471_amd import disc
    from paper_2402_18471_amd.coag import coag_create, coag_mass_grid
    cfg = disc.CONFIGS[name]
    m, me, s = coag_mass_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    d = disc.make_disc(cfg, s)
    idx = np.arange(0, cfg.n_cells, cfg.n_cells // 512)
    sub = disc.subset_cells(d, idx)
    ctx = coag_create(m, me, s, rho_m=cfg.rho_m)
    cells = {k: _t(v) for k, v in sub["cells"].items()}
    vd, vf = _t(sub["v_dust"]), _t(sub["v_frag"])
    K64 = ctx.coag_rates(cells, vd, vf)
    K32 = ctx.coag_rates_blocked(cells, vd, vf)
    rho = _t(sub["rho"])
    h = torch.zeros(len(idx), dtype=torch.float64, device=DEV)
    for _ in range(3):
        r = ctx.coag_step(rho, *K64, d["dt"], h=h, max_sub=512)
        assert np.all(_np(r["status"]) == 0)
    rho0 = rho.clone()
    a = ctx.coag_step(rho0.clone(), *K64, 20 * d["dt"], max_sub=512)
    b = ctx.coag_step(rho0.clone(), K32, None, 20 * d["dt"], mode=L.REPLAY, prec=1,
                      nsub=a["nsub"].clone(), h_log=a["h_log"])
    torch.cuda.synchronize()
    assert np.all(_np(a["status"]) == 0) and np.all(_np(b["status"]) == 0)
    x, ref = _np(b["rho"]), _np(a["rho"])
    M = ref.sum(1, keepdims=True)
    res = ref >= 1e-12 * M
    err = np.abs(x - ref)
    assert np.max(err[res] / ref[res]) <= 1e-6, np.max(err[res] / ref[res])
    assert np.max((err / M)[~res], initial=0.0) <= 1e-18
    assert np.max(np.abs(x.sum(1) / _np(rho0).sum(1) - 1)) <= 1e-12
