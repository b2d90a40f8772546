"""The transport step (coag_transport_dt / coag_transport_step) against the
transport oracle on the same seeded disc inputs, and the scheduler
(coag_evolve) against its rule, through the C ABI.

Bars: the kernels and the oracle evaluate the same expressions in FP64 in
different orders (per-cell sums of the four face fluxes, fused multiply-adds),
so states agree to rounding: each (cell, species) density within 1e-12
relative (of the larger of the densities before and after the step where a
step nearly empties a species) plus 1e-14 of its cell's largest density, each velocity within
1e-12 relative plus 1e-12 of the largest speed of its cell and species row;
the CFL step of the same velocities within 1e-14 relative.  The scheduler test runs the same library
calls in Python by the rule of the header; the FP64 coagulation step deposits
with LDS atomics whose order may differ between launches, so densities agree
to 1e-12 relative (floor 1e-24 of the cell's mass) and the counts exactly.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _inputs(n_r, n_z, n_bins, fill=True):
    from paper_2402_18471_amd import disc
    cfg = disc.scaled(disc.CONFIGS["disc64x32_n100"], n_r, n_z, n_bins)
    s = np.geomspace(cfg.s_min, cfg.s_max, n_bins)
    d = disc.make_transport(cfg, s)
    if fill:
        # mass in every bin (the MRN start fills only the smallest grains)
        d["rho"] = d["rho"] + 1e-3 * d["cells"]["rho_g"][:, None] * np.sqrt(s / s[-1])[None, :]
    return cfg, s, d


def _oracle(cfg, s, d):
    from oracle import transport as T
    g = T.geometry(d["R_edge"], d["t_edge"])
    c = d["cells"]
    sh = (cfg.n_r, cfg.n_z)
    nu = c["alpha"] * c["c_s"] * c["H"]
    gas = T.Gas(c["rho_g"].reshape(sh), c["c_s"].reshape(sh), nu.reshape(sh),
                d["v_gas"].reshape(sh + (3,)), d["GM"])
    return T, g, gas


def _ctx(cfg, s, d):
    from paper_2402_18471_amd.coag import TransportContext
    return TransportContext(d["R_edge"], d["t_edge"], s, rho_m=cfg.rho_m, GM=d["GM"])


def _close(rho_g, v_g, rho_o, v_o, rho_pre=None):
    """the module docstring's bars (with rho_pre: relative to the larger of
    the density before and after the step); returns the largest ratios to
    them"""
    C, N = rho_o.shape
    rfloor = 1e-14 * np.abs(rho_o).max(axis=1, keepdims=True)
    scale = np.abs(rho_o) if rho_pre is None else np.maximum(np.abs(rho_o), np.abs(rho_pre))
    er = np.abs(rho_g - rho_o) / (1e-12 * scale + rfloor + 1e-300)
    vmax = np.abs(v_o).max(axis=2, keepdims=True)
    ev = np.abs(v_g - v_o) / (1e-12 * np.abs(v_o) + 1e-12 * vmax + 1e-300)
    return float(er.max()), float(ev.max())


@pytest.mark.parametrize("shape", [(24, 12, 12), (5, 3, 7), (1, 1, 4), (128, 64, 150)])
def test_transport_steps_match_the_oracle(shape):
    n_r, n_z, N = shape
    cfg, s, d = _inputs(n_r, n_z, N)
    T, g, gas = _oracle(cfg, s, d)
    tc = _ctx(cfg, s, d)
    cells = {k: _t(v) for k, v in d["cells"].items()}
    rho, v, vg = _t(d["rho"]), _t(d["v"]), _t(d["v_gas"])
    ro = d["rho"].reshape(n_r, n_z, N).copy()
    vo = d["v"].reshape(n_r, n_z, N, 3).copy()
    for k in range(2 if N > 100 else 3):
        # the CFL rule on the same velocities (the GPU's): the same minimum
        dt_g = tc.dt(cells, v)
        dt_c = T.cfl_dt(g, gas, v.cpu().numpy().reshape(n_r, n_z, N, 3))
        assert dt_g == pytest.approx(dt_c, rel=1e-14), (k, dt_g, dt_c)
        # both sides step by the oracle's own step size
        dt_o = T.cfl_dt(g, gas, vo)
        tc.step(cells, vg, rho, v, dt_o)
        ro, vo = T.step(g, gas, s, cfg.rho_m, ro, vo, dt_o)
        torch.cuda.synchronize()
        er, ev = _close(rho.cpu().numpy(), v.cpu().numpy().reshape(-1, N, 3),
                        ro.reshape(-1, N), vo.reshape(-1, N, 3))
        print(f"shape {shape} step {k}: density {er:.3g}, velocity {ev:.3g} of the bar")
        assert er <= 1.0 and ev <= 1.0


def test_transport_conserves_mass_on_the_gpu():
    """Empty outer rings and top layers, as in the oracle's pin: the total
    mass sum V rho over the disc stays constant to rounding."""
    n_r, n_z, N = 40, 20, 10
    cfg, s, d = _inputs(n_r, n_z, N)
    rho = d["rho"].reshape(n_r, n_z, N)
    # mass spreads by at most two cells a step
    rho[:8] = rho[-8:] = 0.0
    rho[:, -8:] = 0.0
    T, g, gas = _oracle(cfg, s, d)
    tc = _ctx(cfg, s, d)
    cells = {k: _t(v) for k, v in d["cells"].items()}
    rt, v, vg = _t(rho.reshape(-1, N)), _t(d["v"]), _t(d["v_gas"])
    V = _t(g.V.reshape(-1, 1))
    m0 = float((V * rt).sum())
    for _ in range(3):
        tc.step(cells, vg, rt, v, tc.dt(cells, v))
    torch.cuda.synchronize()
    r = rt.cpu().numpy().reshape(n_r, n_z, N)
    assert np.all(r[0] == 0) and np.all(r[-1] == 0) and np.all(r[:, -1] == 0)
    assert abs(float((V * rt).sum()) - m0) <= 1e-14 * m0


def test_transport_rejects_bad_steps():
    from paper_2402_18471_amd import _lib as L
    cfg, s, d = _inputs(4, 3, 5)
    tc = _ctx(cfg, s, d)
    cells = {k: _t(v) for k, v in d["cells"].items()}
    rho, v, vg = _t(d["rho"]), _t(d["v"]), _t(d["v_gas"])
    before = rho.clone()
    for dt in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(L.CoagError) as e:
            tc.step(cells, vg, rho, v, dt)
        assert e.value.code == L.COAG_EINVAL
    torch.cuda.synchronize()
    assert torch.equal(rho, before)


@pytest.mark.parametrize("prec", ["fp64", "split"])
def test_evolve_follows_the_scheduler_rule(prec):
    """coag_evolve against the rule written out with the library's own calls:
    dt = CFL step clipped to what is left; transport step; when the time since
    the last coagulation update reaches the smallest last sub-step of the
    cells (0 at the start), or at t_end, rates and an ADAPTIVE step over that
    time."""
    from paper_2402_18471_amd import _lib as L
    from paper_2402_18471_amd.coag import coag_create, coag_mass_grid
    n_r, n_z, N = 16, 8, 40
    from paper_2402_18471_amd import disc
    cfg = disc.scaled(disc.CONFIGS["disc64x32_n100"], n_r, n_z, N)
    m, me, s = coag_mass_grid(N, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    d = disc.make_transport(cfg, s)
    ctx = coag_create(m, me, s, rho_m=cfg.rho_m)
    tc = _ctx(cfg, s, d)
    cells = {k: _t(v) for k, v in d["cells"].items()}
    vg, vf = _t(d["v_gas"]), _t(d["v_frag"])
    p = L.PREC_SPLIT_BF16 if prec == "split" else L.PREC_FP64
    C = cfg.n_cells
    # time: a few hundred CFL steps of the inner disc
    dt0 = tc.dt(cells, _t(d["v"]))
    t_end = 40.0 * dt0
    rho_a, v_a, h_a = _t(d["rho"]), _t(d["v"]), torch.zeros(C, dtype=torch.float64, device=DEV)
    st = tc.evolve(ctx, cells, vg, vf, rho_a, v_a, h_a, t_end, prec=p)
    # the rule, step by step
    rho_b, v_b, h_b = _t(d["rho"]), _t(d["v"]), torch.zeros(C, dtype=torch.float64, device=DEV)
    t, since, trig, steps, calls = 0.0, 0.0, 0.0, 0, 0
    dtype = torch.float32 if prec == "split" else torch.float64
    while t < t_end:
        dt = tc.dt(cells, v_b)
        last = not (dt < t_end - t)
        if last:
            dt = t_end - t
        tc.step(cells, vg, rho_b, v_b, dt)
        steps += 1
        t = t_end if last else t + dt
        since += dt
        if since >= trig or last:
            K = ctx.coag_rates_blocked(cells, v_b, vf, dtype=dtype)
            r = ctx.coag_step(rho_b, K, None, since, h=h_b, prec=p, max_sub=256)
            calls += 1
            since = 0.0
            hp = h_b[h_b > 0]
            trig = float(hp.min()) if hp.numel() else 0.0
    torch.cuda.synchronize()
    assert st["transport_steps"] == steps and st["coag_calls"] == calls, (st, steps, calls)
    assert st["t_reached"] == t_end and st["cells_failed"] == 0
    assert calls >= 2
    a, b = rho_a.cpu().numpy(), rho_b.cpu().numpy()
    M = b.sum(1, keepdims=True)
    assert np.all(np.abs(a - b) <= 1e-12 * np.abs(b) + 1e-24 * M)
    assert torch.allclose(v_a, v_b, rtol=1e-12, atol=0.0)
    assert torch.allclose(h_a, h_b, rtol=1e-12, atol=0.0)


def test_transport_and_coagulation_together_match_the_oracles():
    """A dozen global steps of the scheduler's sequence on a small disc, each
    operation checked against the oracle from the GPU's own state at that
    point (so that rounding differences do not compound over the coupled
    run): the transport step against the transport oracle's step on the same
    dt, the CFL step against the oracle's rule on the GPU's velocities, and
    each coagulation update against the coagulation oracle's rates of the
    GPU's velocities and its step replaying the GPU call's sub-steps (the step
    sequence is the GPU's, as in the coagulation parity tests).  Bars: the
    transport bars of this module; coagulation densities within 1e-10
    relative in bins above 1e-20 of the cell's mass, 1e-20 of the cell's mass
    below (the calls here are long, up to centuries, and replay the same steps
    on rates that agree to 1e-12)."""
    import oracle as O
    from paper_2402_18471_amd.coag import coag_create, coag_mass_grid
    from paper_2402_18471_amd import disc
    n_r, n_z, N = 6, 4, 30
    cfg = disc.scaled(disc.CONFIGS["disc64x32_n100"], n_r, n_z, N)
    m, me, s = coag_mass_grid(N, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    og = O.make_grid(N, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    d = disc.make_transport(cfg, s)
    T, g, gas = _oracle(cfg, s, d)
    ctx = coag_create(m, me, s, rho_m=cfg.rho_m)
    tc = _ctx(cfg, s, d)
    cells = {k: _t(v) for k, v in d["cells"].items()}
    vg, vf = _t(d["v_gas"]), _t(d["v_frag"])
    C = cfg.n_cells
    rho_b, v_b, h_b = _t(d["rho"]), _t(d["v"]), torch.zeros(C, dtype=torch.float64, device=DEV)
    sh = (n_r, n_z)
    since, trig, calls = 0.0, 0.0, 0
    for step in range(12):
        r0, v0 = rho_b.cpu().numpy(), v_b.cpu().numpy()
        dt = tc.dt(cells, v_b)
        assert dt == pytest.approx(T.cfl_dt(g, gas, v0.reshape(sh + (N, 3))), rel=1e-14)
        tc.step(cells, vg, rho_b, v_b, dt)
        r3, v3 = T.step(g, gas, s, cfg.rho_m, r0.reshape(sh + (N,)), v0.reshape(sh + (N, 3)), dt)
        torch.cuda.synchronize()
        # after coagulation calls some species are nearly emptied by the flux
        # of a step (the new density the difference of two near-equal
        # terms): their rounding is relative to the density before the step
        et, ev = _close(rho_b.cpu().numpy(), v_b.cpu().numpy(), r3.reshape(C, N),
                        v3.reshape(C, N, 3), rho_pre=r0)
        assert et <= 1.0 and ev <= 1.0, (step, et, ev)
        since += dt
        ec = 0.0
        if since >= trig:
            r1, v1 = rho_b.cpu().numpy(), v_b.cpu().numpy()
            K = ctx.coag_rates_blocked(cells, v_b, vf, dtype=torch.float64)
            r = ctx.coag_step(rho_b, K, None, since, h=h_b, max_sub=256)
            torch.cuda.synchronize()
            ns, hl = r["nsub"].cpu().numpy(), r["h_log"].cpu().numpy()
            Kc, Kf = O.rates(og, d["cells"], v1, d["v_frag"])
            ro = O.step(og, r1, Kc, Kf, since, mode=O.REPLAY, nsub=ns, h_log=hl)["rho"]
            a = rho_b.cpu().numpy()
            M = ro.sum(1, keepdims=True)
            res = np.abs(ro) > 1e-20 * M
            err = np.where(res, np.abs(a - ro) / (1e-10 * np.abs(ro) + 1e-300),
                           np.abs(a - ro) / (1e-20 * M + 1e-300))
            ec = float(err.max())
            calls += 1
            since = 0.0
            hp = h_b[h_b > 0]
            trig = float(hp.min()) if hp.numel() else 0.0
        print(f"global step {step}: dt {dt:.4g} s, coagulation calls {calls}; transport "
              f"{max(et, ev):.3g}, coagulation {ec:.3g} of the bars", flush=True)
        assert ec <= 1.0, (step, ec)
    assert calls >= 3
