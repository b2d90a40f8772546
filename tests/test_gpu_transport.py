"""The transport step (coag_transport_dt / coag_transport_step) against the
transport oracle on the same seeded disc inputs, and the scheduler
(coag_evolve) against its rule, through the C ABI.

Bars: the kernels and the oracle evaluate the same expressions in FP64 in
different orders (per-cell sums of the four face fluxes, fused multiply-adds),
so states agree to rounding: each (cell, species) density within 1e-12
relative plus 1e-14 of its cell's largest density, each velocity within
1e-12 relative plus 1e-12 of the largest speed of its cell and species row;
the CFL step within 1e-14 relative from the same inputs (1e-9 after steps,
each side from its own velocities).  The scheduler test runs the same library
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


def _inputs(n_r, n_z, n_bins, fill=True, base="disc64x32_n100"):
    from paper_2402_18471_amd import disc
    cfg = disc.scaled(disc.CONFIGS[base], n_r, n_z, n_bins)
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


def _ctx(cfg, s, d, eps_floor=0.0):
    from paper_2402_18471_amd.coag import TransportContext
    return TransportContext(d["R_edge"], d["t_edge"], s, rho_m=cfg.rho_m, GM=d["GM"],
                            eps_floor=eps_floor)


def _close(rho_g, v_g, rho_o, v_o):
    """the module docstring's bars; returns the largest ratios to them"""
    C, N = rho_o.shape
    rfloor = 1e-14 * np.abs(rho_o).max(axis=1, keepdims=True)
    er = np.abs(rho_g - rho_o) / (1e-12 * np.abs(rho_o) + rfloor + 1e-300)
    vmax = np.abs(v_o).max(axis=2, keepdims=True)
    ev = np.abs(v_g - v_o) / (1e-12 * np.abs(v_o) + 1e-12 * vmax + 1e-300)
    return float(er.max()), float(ev.max())


@pytest.mark.parametrize("shape", [(24, 12, 12), (5, 3, 7), (1, 1, 4), (128, 64, 150),
                                   (2, 3, 1023)])
def test_transport_steps_match_the_oracle(shape):
    n_r, n_z, N = shape
    cfg, s, d = _inputs(n_r, n_z, N)
    _parity(shape, cfg, s, d, 2 if N > 100 else 3)


def test_transport_step_matches_the_oracle_at_the_bench_size():
    """One step of the full 256 x 128-cell, 150-species disc the bench times
    (every bin filled), element by element against the oracle (about 16 s
    of numpy)."""
    from paper_2402_18471_amd import disc
    cfg0 = disc.CONFIGS["disc256x128_n150"]
    shape = (cfg0.n_r, cfg0.n_z, cfg0.n_bins)
    cfg, s, d = _inputs(*shape, base="disc256x128_n150")
    assert (cfg.n_r, cfg.n_z, cfg.n_bins) == shape
    _parity(shape, cfg, s, d, 1)


def test_subnormal_densities_match_the_oracle():
    """The coagulation update leaves subnormal densities in the upper bins;
    their velocities (momentum over density) stay finite and within the bars."""
    n_r, n_z, N = 12, 6, 20
    cfg, s, d = _inputs(n_r, n_z, N)
    rng = np.random.default_rng(11)
    rho = d["rho"].reshape(-1, N)
    rho[:, -6:] = rng.uniform(1.0, 4.0, size=(rho.shape[0], 6)) * 1e-310
    assert np.all(rho[:, -6:] < np.finfo(np.float64).tiny)
    _parity((n_r, n_z, N), cfg, s, d, 2)


def test_floor_species_match_the_oracle():
    """The dust floor: three species at 1e-30 of the gas density with
    meaningless speeds (1e7 cm/s), eps_floor = 1e-20: both sides give them
    the gas velocity at the end of each stage, and the later CFL steps come
    from the other species."""
    n_r, n_z, N = 24, 12, 12
    cfg, s, d = _inputs(n_r, n_z, N)
    rng = np.random.default_rng(5)
    rho = d["rho"].reshape(-1, N)
    rho[:, 9:] = 1e-30 * d["cells"]["rho_g"][:, None]
    v = d["v"].reshape(-1, N, 3)
    v[:, 9:, :] = rng.normal(0.0, 1e7, (rho.shape[0], 3, 3))
    v_after = _parity((n_r, n_z, N), cfg, s, d, 3, eps_floor=1e-20)
    vg = d["v_gas"].reshape(-1, 1, 3)
    assert np.array_equal(v_after.reshape(-1, N, 3)[:, 9:, :], np.broadcast_to(vg, (rho.shape[0], 3, 3)))


def _parity(shape, cfg, s, d, n_steps, eps_floor=0.0):
    n_r, n_z, N = shape
    T, g, gas = _oracle(cfg, s, d)
    tc = _ctx(cfg, s, d, eps_floor)
    cells = {k: _t(v) for k, v in d["cells"].items()}
    rho, v, vg = _t(d["rho"]), _t(d["v"]), _t(d["v_gas"])
    ro = d["rho"].reshape(n_r, n_z, N).copy()
    vo = d["v"].reshape(n_r, n_z, N, 3).copy()
    for k in range(n_steps):
        # the CFL rule: the same minimum from the same inputs at the start;
        # later each side from its own velocities (equal to the bars above,
        # the limiting component possibly far below the row's largest)
        dt_g = tc.dt(cells, v)
        dt_o = T.cfl_dt(g, gas, vo)
        assert dt_g == pytest.approx(dt_o, rel=1e-14 if k == 0 else 1e-9), (k, dt_g, dt_o)
        # both sides step by the oracle's step size
        tc.step(cells, vg, rho, v, dt_o)
        ro, vo = T.step(g, gas, s, cfg.rho_m, ro, vo, dt_o, eps_floor=eps_floor)
        torch.cuda.synchronize()
        er, ev = _close(rho.cpu().numpy(), v.cpu().numpy().reshape(-1, N, 3),
                        ro.reshape(-1, N), vo.reshape(-1, N, 3))
        print(f"shape {shape} step {k}: density {er:.3g}, velocity {ev:.3g} of the bar")
        assert bool(torch.isfinite(v).all()) and bool(torch.isfinite(rho).all())
        assert er <= 1.0 and ev <= 1.0
    return v.cpu().numpy()


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


@pytest.mark.parametrize("prec,eps_floor,N", [("fp64", 0.0, 40), ("split", 0.0, 40),
                                              ("fp64", 1e-20, 40), ("fp64", 0.0, 10)])
def test_evolve_follows_the_scheduler_rule(prec, eps_floor, N):
    """coag_evolve against the rule written out with the library's own calls:
    dt = CFL step clipped to what is left; transport step; when the time since
    the last coagulation update reaches the smallest last sub-step of the
    cells (0 at the start), or at t_end, rates and an ADAPTIVE step over that
    time.  With 10 bins the batched step does not apply (it needs 16 or more):
    FP64 [C][P] rates and the per-cell step."""
    from paper_2402_18471_amd import _lib as L
    from paper_2402_18471_amd.coag import coag_create, coag_mass_grid
    n_r, n_z = 16, 8
    from paper_2402_18471_amd import disc
    cfg = disc.scaled(disc.CONFIGS["disc64x32_n100"], n_r, n_z, N)
    m, me, s = coag_mass_grid(N, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    d = disc.make_transport(cfg, s)
    ctx = coag_create(m, me, s, rho_m=cfg.rho_m)
    tc = _ctx(cfg, s, d, eps_floor)
    cells = {k: _t(v) for k, v in d["cells"].items()}
    vg, vf = _t(d["v_gas"]), _t(d["v_frag"])
    p = L.PREC_SPLIT_BF16 if prec == "split" else L.PREC_FP64
    C = cfg.n_cells
    # time: a few hundred CFL steps of the inner disc
    dt0 = tc.dt(cells, _t(d["v"]))
    t_end = 40.0 * dt0
    rho_a, v_a, h_a = _t(d["rho"]), _t(d["v"]), torch.zeros(C, dtype=torch.float64, device=DEV)
    st = tc.evolve(ctx, cells, vg, vf, rho_a, v_a, h_a, t_end, prec=p)
    dtype = torch.float32 if prec == "split" else torch.float64

    def rule():
        """the rule, step by step; returns (rho, v, h, steps, calls)"""
        rho_b, v_b, h_b = _t(d["rho"]), _t(d["v"]), torch.zeros(C, dtype=torch.float64, device=DEV)
        t, since, trig, steps, calls = 0.0, 0.0, 0.0, 0, 0
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
                if N >= 16:
                    K = ctx.coag_rates_blocked(cells, v_b, vf, dtype=dtype)
                    ctx.coag_step(rho_b, K, None, since, h=h_b, prec=p, max_sub=256)
                else:
                    Kc, Kf = ctx.coag_rates(cells, v_b, vf)
                    ctx.coag_step(rho_b, Kc, Kf, since, h=h_b, prec=p, max_sub=256)
                calls += 1
                since = 0.0
                hp = h_b[h_b > 0]
                trig = float(hp.min()) if hp.numel() else 0.0
        torch.cuda.synchronize()
        return rho_b.cpu().numpy(), v_b.cpu().numpy(), h_b.cpu().numpy(), steps, calls

    b_rho, b_v, b_h, steps, calls = rule()
    assert st["transport_steps"] == steps and st["coag_calls"] == calls, (st, steps, calls)
    assert st["t_reached"] == t_end and st["cells_failed"] == 0
    assert calls >= 2
    a_rho, a_v, a_h = rho_a.cpu().numpy(), v_a.cpu().numpy(), h_a.cpu().numpy()
    M = b_rho.sum(1, keepdims=True)
    # largest difference relative to the value (the value at least 1e-24 of
    # the cell's mass), and of h
    e_rho = lambda x, y: float(np.max(np.abs(x - y) / (np.abs(y) + 1e-24 * M)))
    e_h = lambda x, y: float(np.max(np.abs(x - y) / np.maximum(np.abs(y), 1e-300)))
    if N >= 16:
        # the batched step: rounding-level differences only
        assert np.all(np.abs(a_rho - b_rho) <= 1e-12 * np.abs(b_rho) + 1e-24 * M)
        assert e_h(a_h, b_h) <= 1e-12
    else:
        # the per-cell FP64 step accumulates with LDS atomics in an order
        # that varies between launches, and the adaptive control carries the
        # differences on (measured: 5e-8 of a density, 1.6e-10 of h, between
        # two runs of the same calls): coag_evolve is held to ten times the
        # rule's difference from a second run of itself
        c_rho, c_v, c_h, steps2, calls2 = rule()
        assert (steps2, calls2) == (steps, calls)
        assert e_rho(a_rho, b_rho) <= 10.0 * max(e_rho(c_rho, b_rho), 1e-12)
        assert e_h(a_h, b_h) <= 10.0 * max(e_h(c_h, b_h), 1e-12)
    assert np.allclose(a_v, b_v, rtol=1e-12, atol=0.0)


def test_a_disc_at_rest_has_no_cfl_limit():
    """No velocity, no turbulence and no gravity: no component limits the
    step, the CFL step is +inf, and the scheduler covers t_end in one
    transport step (which moves nothing) with one coagulation update over all
    of it."""
    from paper_2402_18471_amd.coag import coag_create, coag_mass_grid
    from paper_2402_18471_amd import disc
    n_r, n_z, N = 4, 3, 20
    cfg = disc.scaled(disc.CONFIGS["disc64x32_n100"], n_r, n_z, N)
    m, me, s = coag_mass_grid(N, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    d = disc.make_transport(cfg, s)
    d["cells"]["alpha"][:] = 0.0
    d["GM"] = 0.0
    tc = _ctx(cfg, s, d)
    cells = {k: _t(v) for k, v in d["cells"].items()}
    v = torch.zeros((cfg.n_cells, N, 3), dtype=torch.float64, device=DEV)
    assert tc.dt(cells, v) == float("inf")
    ctx = coag_create(m, me, s, rho_m=cfg.rho_m)
    rho = _t(d["rho"])
    h = torch.zeros(cfg.n_cells, dtype=torch.float64, device=DEV)
    vg = torch.zeros((cfg.n_cells, 3), dtype=torch.float64, device=DEV)
    st = tc.evolve(ctx, cells, vg, _t(d["v_frag"]), rho, v, h, 100.0 * 3.15576e7, prec=0)
    torch.cuda.synchronize()
    assert st["transport_steps"] == 1 and st["coag_calls"] == 1 and st["cells_failed"] == 0
    assert st["t_reached"] == 100.0 * 3.15576e7
    assert torch.count_nonzero(v) == 0 and bool(torch.all(h > 0))


def test_evolve_rejects_bad_arguments():
    """coag_evolve's checks: t_end and max_steps, a coagulation context with
    another bin count or of the vertically integrated kernel, a precision it
    does not take, split precision on a grid
    the batched step does not cover (all before any work); and the step cap,
    which stops a run that needs more steps with COAG_EINVAL and its state
    finite (10 bins: FP64 runs the per-cell step)."""
    from paper_2402_18471_amd import _lib as L
    from paper_2402_18471_amd.coag import coag_create, coag_mass_grid
    from paper_2402_18471_amd import disc
    n_r, n_z, N = 6, 4, 10
    cfg = disc.scaled(disc.CONFIGS["disc64x32_n100"], n_r, n_z, N)
    m, me, s = coag_mass_grid(N, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    d = disc.make_transport(cfg, s)
    ctx = coag_create(m, me, s, rho_m=cfg.rho_m)
    m2, me2, s2 = coag_mass_grid(N + 2, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    ctx_other = coag_create(m2, me2, s2, rho_m=cfg.rho_m)
    tc = _ctx(cfg, s, d)
    cells = {k: _t(v) for k, v in d["cells"].items()}
    vg, vf = _t(d["v_gas"]), _t(d["v_frag"])
    rho, v = _t(d["rho"]), _t(d["v"])
    h = torch.zeros(cfg.n_cells, dtype=torch.float64, device=DEV)
    dt0 = tc.dt(cells, v)

    def code(**kw):
        args = dict(ctx=ctx, t_end=10.0 * dt0, max_steps=1 << 20, prec=L.PREC_FP64)
        args.update(kw)
        with pytest.raises(L.CoagError) as e:
            tc.evolve(args["ctx"], cells, vg, vf, rho, v, h, args["t_end"],
                      max_steps=args["max_steps"], prec=args["prec"])
        return e.value.code, str(e.value)

    before = rho.clone()
    for t_end in (0.0, -1.0, float("nan"), float("inf")):
        assert code(t_end=t_end)[0] == L.COAG_EINVAL
    assert code(max_steps=0)[0] == L.COAG_EINVAL
    assert code(ctx=ctx_other)[0] == L.COAG_EINVAL
    # a context of the vertically integrated kernel takes surface densities
    assert code(ctx=coag_create(m, me, s, rho_m=cfg.rho_m, vertical=True))[0] == L.COAG_EINVAL
    assert code(prec=7)[0] == L.COAG_EINVAL
    # split precision needs the batched step, which 10 bins do not allow:
    # refused before any transport step
    assert code(prec=L.PREC_SPLIT_BF16)[0] == L.COAG_ENOTSUP
    torch.cuda.synchronize()
    assert torch.equal(rho, before)
    # one step of dt0 leaves 9 dt0 to go
    c, msg = code(max_steps=1)
    assert c == L.COAG_EINVAL and "transport steps reached" in msg
    torch.cuda.synchronize()
    assert bool(torch.isfinite(rho).all()) and not torch.equal(rho, before)
