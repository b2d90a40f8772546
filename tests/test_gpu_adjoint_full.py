"""The differentiation workload at full size: the 64x32-cell, 100-bin disc,
200 coagulation calls (FIXED, 8 sub-steps each), checkpoints every 20 calls,
J = sum over cells of the mass-weighted mean ln s.  Gradients with respect to
alpha, v_frag (per cell) and the initial density from torch.autograd
(coag_step_backward, FP64 and split precision) against central differences of
the FP64 GPU forward with its frozen steps: the two scalars at h = 1e-6
relative, 16 random directions in rho_0 and 32 single components at h = 3e-8
of the cell's mass (the evaluations run as copies of the disc's cells in two
forwards); and, on 16 cells, against the oracle's FP64 adjoint chained over
the same 200 calls.

Bars: every cell's dJ_c/dln x within 1e-6 (split: 1e-5) of the largest
|dJ_c/dln x| over the cells (the central differences carry O(h^2)
truncation, <= 1e-7 of it here, and ~1e-9 rounding); the oracle's final
states to 1e-9 relative (floor 1e-15 of the cell's mass), its alpha and
v_frag gradients to 1e-6 relative, its density gradient to 1e-6 of the
cell's largest component in the bins populated at the start.  In the bins
empty at the start (grains above 1 um) dJ/drho_k is ill-conditioned on the
18-decade grid: the FP64 oracle's chained gradient is up to ~2e-3 of the
cell's largest component away from the exact-arithmetic value there.  On two
of the 16 cells both are compared with the oracle's extended-precision chain
(oracle/extended.py, long double, 200 calls): the GPU within 1e-5 of the
cell's largest component (measured ~1e-6; the long-double chain itself moves
by ~5e-8 when its summation order changes).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
CALLS, NSUB, CKPT = 200, 8, 20


@pytest.fixture(scope="module")
def setup():
    from paper_2402_18471_amd import disc
    from paper_2402_18471_amd.coag import coag_create, coag_mass_grid
    cfg = disc.CONFIGS["disc64x32_n100_adj"]
    m, me, s = coag_mass_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    d = disc.make_disc(cfg, s)
    ctx = coag_create(m, me, s, rho_m=cfg.rho_m)
    return cfg, d, ctx, np.log(s)


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _fwd(ctx, d, rho0, alpha, vfrag, idx=None):
    from paper_2402_18471_amd import disc
    from paper_2402_18471_amd.autograd import coag_evolve
    sub = d if idx is None else disc.subset_cells(d, idx)
    cells = {k: _t(v) for k, v in sub["cells"].items()}
    return coag_evolve(ctx, rho0, alpha, vfrag, cells, _t(sub["v_dust"]), float(d["dt"]), CALLS,
                       ckpt_every=CKPT, fixed_nsub=NSUB, max_sub=NSUB)


def _Jc(out, lns):
    return (out * lns).sum(1) / out.sum(1)


def _copies(d, R):
    """The disc's cells repeated R times (copy r of cell c at r C + c): one
    forward of the copies gives R independent finite-difference evaluations
    per cell, since the cells never interact."""
    from paper_2402_18471_amd import disc
    C = len(d["rho"])
    return disc.subset_cells(d, np.tile(np.arange(C), R))


def _J_copies(ctx, d, rho, al, vf, lns):
    rep = _copies(d, len(rho) // len(d["rho"]))
    with torch.no_grad():
        return _Jc(_fwd(ctx, rep, _t(rho), _t(al), _t(vf)), lns).cpu().numpy()


@pytest.fixture(scope="module")
def fd(setup):
    """Central differences of the FP64 forward with its frozen steps (FIXED):
    dJ_c/dln alpha_c, dJ_c/dln v_frag,c with h = 1e-6 relative; 16 random
    directions in rho_0 (8 over all bins, 8 over the bins empty at the start)
    and 32 single components (every third bin), each scaled by the cell's
    mass, with h = 3e-8: the map is strongly nonlinear in the bins just above
    the MRN range, where the O(h^2) truncation error of a random direction
    is 5e-5 of the largest derivative at h = 1e-6 (5e-3 at 1e-5, 5e-7 .. 1e-6
    at 1e-7: measured), and the rounding of J over 2h stays below 1e-9."""
    cfg, d, ctx, lns_np = setup
    lns = _t(lns_np)
    C, N = d["rho"].shape
    h, hr = 1e-6, 3e-8
    r0, a0, v0 = d["rho"], d["cells"]["alpha"], d["v_frag"]
    M = r0.sum(1, keepdims=True)
    rng = np.random.default_rng(240218473)
    dirs = rng.standard_normal((16, C, N))
    dirs[8:] *= (r0 == 0)[None]
    comps = np.arange(0, 3 * 32, 3)
    # run 1: the two scalars (4 copies) and the 16 directions (32 copies)
    rho, al, vf = [], [], []
    for f in (1 + h, 1 - h):
        rho += [r0, r0]
        al += [a0 * f, a0]
        vf += [v0, v0 * f]
    for k in range(16):
        for sgn in (1, -1):
            rho.append(r0 + sgn * hr * M * dirs[k])
            al.append(a0)
            vf.append(v0)
    J = _J_copies(ctx, d, np.concatenate(rho), np.concatenate(al), np.concatenate(vf),
                  lns).reshape(-1, C)
    out = {"alpha": (J[0] - J[2]) / (2 * h), "vfrag": (J[1] - J[3]) / (2 * h),
           "dirs": dirs, "dir": (J[4::2] - J[5::2]) / (2 * hr), "comps": comps, "M": M[:, 0]}
    # run 2: the 32 single components (64 copies)
    rho = []
    for k in comps:
        for sgn in (1, -1):
            r = r0.copy()
            r[:, k] += sgn * hr * M[:, 0]
            rho.append(r)
    J = _J_copies(ctx, d, np.concatenate(rho), np.tile(a0, 64), np.tile(v0, 64),
                  lns).reshape(-1, C)
    out["comp"] = (J[0::2] - J[1::2]) / (2 * hr)       # [32][C]: dJ_c / d(rho_k / M)
    return out


def _adjoint(setup, prec):
    from paper_2402_18471_amd import _lib as L
    cfg, d, ctx, lns_np = setup
    rho0 = _t(d["rho"]).requires_grad_(True)
    al = _t(d["cells"]["alpha"]).requires_grad_(True)
    vf = _t(d["v_frag"]).requires_grad_(True)
    from paper_2402_18471_amd.autograd import coag_evolve
    cells = {k: _t(v) for k, v in d["cells"].items()}
    out = coag_evolve(ctx, rho0, al, vf, cells, _t(d["v_dust"]), float(d["dt"]), CALLS,
                      ckpt_every=CKPT, fixed_nsub=NSUB, max_sub=NSUB,
                      prec=L.PREC_FP64 if prec == "fp64" else L.PREC_SPLIT_BF16)
    _Jc(out, _t(lns_np)).sum().backward()
    return al.grad.cpu().numpy(), vf.grad.cpu().numpy(), rho0.grad.cpu().numpy()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-6), ("split", 1e-5)])
def test_full_adjoint_against_central_differences(setup, fd, prec, tol):
    """Both adjoints against central differences of the FP64 forward: every
    cell's derivative within tol of the largest over the cells, for alpha,
    v_frag, each of the 16 directions and each of the 32 components.  The
    split adjoint differentiates the split forward, whose states differ from
    the FP64 forward's by ~1e-7 relative: hence 1e-5."""
    cfg, d, ctx, lns = setup
    ga, gv, gr = _adjoint(setup, prec)
    a0, v0, M = d["cells"]["alpha"], d["v_frag"], fd["M"]
    checks = [("alpha", fd["alpha"], ga * a0), ("v_frag", fd["vfrag"], gv * v0)]
    for k in range(16):
        checks.append((f"direction {k}", fd["dir"][k], (gr * fd["dirs"][k]).sum(1) * M))
    for n, k in enumerate(fd["comps"]):
        checks.append((f"component {k}", fd["comp"][n], gr[:, k] * M))
    worst = 0.0
    for name, f, a in checks:
        scale = np.max(np.abs(a))
        if scale == 0.0:
            assert np.max(np.abs(f)) <= 1e-12, name
            continue
        e = np.max(np.abs(f - a)) / scale
        worst = max(worst, e)
        assert e <= tol, (name, e)
    print(f"{prec}: worst error against central differences {worst:.2e} of the largest "
          f"derivative over the cells ({len(checks)} derivatives per cell)")


def test_full_adjoint_against_oracle_on_16_cells(setup, O):
    from paper_2402_18471_amd import disc
    cfg, d, ctx, lns = setup
    idx = np.arange(0, cfg.n_cells, cfg.n_cells // 16)
    sub = disc.subset_cells(d, idx)
    rho0 = _t(sub["rho"]).requires_grad_(True)
    al = _t(sub["cells"]["alpha"]).requires_grad_(True)
    vf = _t(sub["v_frag"]).requires_grad_(True)
    out = _fwd(ctx, d, rho0, al, vf, idx)
    _Jc(out, _t(lns)).sum().backward()
    g = O.make_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    def chain(r0):
        Kc, Kf = O.rates(g, sub["cells"], sub["v_dust"], sub["v_frag"])
        states, logs, r = [], [], r0.copy()
        for _ in range(CALLS):
            states.append(r)
            a = O.step(g, r, Kc, Kf, d["dt"], mode=O.FIXED, nsub=NSUB, max_sub=NSUB)
            r, _ = a["rho"], logs.append(a["h_log"])
        Jc = (r * lns).sum(1) / r.sum(1)
        gr = (lns[None, :] - Jc[:, None]) / r.sum(1, keepdims=True)
        ga, gv = np.zeros(len(idx)), np.zeros(len(idx))
        for s in range(CALLS - 1, -1, -1):
            gr, a_s, v_s = O.step_backward(g, sub["cells"], sub["v_dust"], sub["v_frag"],
                                           states[s], d["dt"], logs[s], np.full(len(idx), NSUB),
                                           gr)
            ga += a_s
            gv += v_s
        return gr, ga, gv, r

    gr, ga, gv, r = chain(sub["rho"])
    x = out.detach().cpu().numpy()
    assert np.all(np.abs(x - r) <= 1e-9 * np.abs(r) + 1e-15 * r.sum(1, keepdims=True))
    np.testing.assert_allclose(al.grad.cpu().numpy(), ga, rtol=1e-6, atol=1e-6 * np.abs(ga).max())
    np.testing.assert_allclose(vf.grad.cpu().numpy(), gv, rtol=1e-6, atol=1e-6 * np.abs(gv).max())
    gi = rho0.grad.cpu().numpy()
    sc = np.abs(gr).max(1, keepdims=True)
    err = np.abs(gi - gr) / sc
    held = sub["rho"] > 0                          # bins populated at the start
    assert np.all(err[held] <= 1e-6), np.max(err[held])
    # bins empty at the start: against the extended-precision chain on two cells
    from oracle import extended
    two = np.array([0, 9])
    cells2 = {k: v[two] for k, v in sub["cells"].items()}
    ext = extended.Extended(g, *O.rates(g, cells2, sub["v_dust"][two], sub["v_frag"][two]))
    steps = np.full((2, CALLS * NSUB), d["dt"] / NSUB)
    y = ext.step(sub["rho"][two], steps, np.full(2, CALLS * NSUB))
    M = y.sum(1, keepdims=True)
    g_end = (lns[None, :] - (y * lns).sum(1, keepdims=True) / M) / M
    ld = ext.step_backward(sub["rho"][two], steps, np.full(2, CALLS * NSUB),
                           g_end)["g_in"].astype(np.float64)
    sc2 = np.abs(ld).max(1, keepdims=True)
    e_gpu = (np.abs(gi[two] - ld) / sc2)[~held[two]]
    e_ora = (np.abs(gr[two] - ld) / sc2)[~held[two]]
    print(f"bins empty at the start, against long double: GPU {e_gpu.max():.2e}, "
          f"oracle {e_ora.max():.2e} of the cell's largest component")
    assert np.all(e_gpu <= 1e-5), e_gpu.max()
