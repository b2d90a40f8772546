"""Edge cases of the step kernels, FP64 (batched and per-cell) and split-BF16.

The batched step advances 16 cells in lockstep, so the cases are built around
batch structure: fewer cells than a batch, a ragged last batch, and cells
within one batch that must not disturb each other (an empty cell, a cell with
a NaN, a cell with one populated bin, an invalid sub-step count).  Valid cells
are compared with the oracle replaying the same steps (FP64: conditioning-
aware bound of test_gpu_parity; split: 1e-6 relative, floor 1e-18 of the
cell's mass).
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
FORMS = [("batch", 0), ("cell", 0), ("batch", 1)]     # (FP64 kernel, prec)


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _np(t):
    return t.detach().cpu().numpy()


def _ctx(m, me, s, kernel, **kw):
    from paper_2402_18471_amd.coag import coag_create
    old = os.environ.get("COAG_STEP_KERNEL")
    os.environ["COAG_STEP_KERNEL"] = kernel
    try:
        return coag_create(m, me, s, **kw)
    finally:
        if old is None:
            os.environ.pop("COAG_STEP_KERNEL", None)
        else:
            os.environ["COAG_STEP_KERNEL"] = old


def _disc(O, n_r, n_z, n_bins=None, lo=None, hi=None):
    from paper_2402_18471_amd import disc
    from paper_2402_18471_amd.coag import coag_mass_grid
    cfg = disc.scaled(disc.CONFIGS["disc64x32_n100"], n_r, n_z, n_bins)
    lo = cfg.s_min if lo is None else lo
    hi = cfg.s_max if hi is None else hi
    m, me, s = coag_mass_grid(cfg.n_bins, lo, hi, rho_m=cfg.rho_m)
    g = O.make_grid(cfg.n_bins, lo, hi, rho_m=cfg.rho_m)
    d = disc.make_disc(cfg, g.s)
    return cfg, (m, me, s), g, d


def _close(O, g, gpu, ora, rho0, Kc, Kf, dt, prec):
    M = rho0.sum(1, keepdims=True)
    if prec == 1:
        return np.abs(gpu - ora) <= 1e-6 * np.abs(ora) + 1e-18 * M
    _, gain, loss = O.rhs(g, rho0, Kc, Kf, parts=True)
    return np.abs(gpu - ora) <= 1e-12 * np.abs(ora) + 1e-13 * dt * (gain + loss) + 1e-24 * M


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("shape", [(3, 1), (19, 1)])
def test_odd_cells_in_a_batch(O, form, shape):
    """An empty cell, a NaN cell, a one-bin cell and an invalid sub-step
    count among ordinary cells; C below one batch and a ragged last batch."""
    kernel, prec = form
    cfg, grid, g, d = _disc(O, *shape)
    ctx = _ctx(*grid, kernel, rho_m=cfg.rho_m)
    C = cfg.n_cells
    Kc, Kf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    rho0 = d["rho"].copy()
    rho0[0] = 0.0                                     # empty cell
    if C > 2:
        rho0[2, 5] = np.nan                           # NaN cell
        rho0[1] = 0.0
        rho0[1, 7] = 1e-14                            # one populated bin
    nsub = np.full(C, 3, np.int32)
    if C > 4:
        nsub[4] = 99                                  # more than max_sub
    dt = d["dt"]
    r = ctx.coag_step(_t(rho0), _t(Kc), _t(Kf), dt, mode=1, prec=prec, nsub=_t(nsub, torch.int32),
                      max_sub=8, check_status=False)
    torch.cuda.synchronize()
    st, x = _np(r["status"]), _np(r["rho"])
    assert st[0] == 0 and np.all(x[0] == 0.0)
    ok = np.ones(C, bool)
    if C > 2:
        assert st[2] == 3
        ok[2] = False
    if C > 4:
        assert st[4] == 2
        np.testing.assert_array_equal(x[4], rho0[4])  # no step taken
        ok[4] = False
    assert np.all(st[ok] == 0)
    o = O.step(g, rho0[ok], Kc[ok], Kf[ok], dt, mode=O.FIXED, nsub=3)
    assert np.all(_close(O, g, x[ok], o["rho"], rho0[ok], Kc[ok], Kf[ok], dt, prec))


@pytest.mark.parametrize("form", FORMS)
def test_minimum_window_grid(O, form):
    """16 bins over a 10x range of sizes: the smallest grid the batched
    step's 16-bin window admits, every product within it."""
    kernel, prec = form
    cfg, grid, g, d = _disc(O, 4, 5, 16, 1e-4, 1e-3)
    ctx = _ctx(*grid, kernel, rho_m=cfg.rho_m)
    Kc, Kf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    rng = np.random.default_rng(5)
    rho0 = 0.01 * d["cells"]["rho_g"][:, None] * rng.uniform(0.1, 1.0, (cfg.n_cells, 16)) / 16
    dt = d["dt"] * 1e-3
    o = O.step(g, rho0, Kc, Kf, dt, max_sub=64)
    assert np.all(o["status"] == 0)
    r = ctx.coag_step(_t(rho0), _t(Kc), _t(Kf), dt, mode=2, prec=prec,
                      nsub=_t(o["nsub"], torch.int32), h_log=_t(o["h_log"]))
    torch.cuda.synchronize()
    assert np.all(_np(r["status"]) == 0)
    assert np.all(_close(O, g, _np(r["rho"]), o["rho"], rho0, Kc, Kf, dt, prec))


@pytest.mark.parametrize("form", FORMS)
def test_replay_of_zero_steps_keeps_the_state(O, form):
    kernel, prec = form
    cfg, grid, g, d = _disc(O, 3, 6)
    ctx = _ctx(*grid, kernel, rho_m=cfg.rho_m)
    Kc, Kf = O.rates(g, d["cells"], d["v_dust"], d["v_frag"])
    C = cfg.n_cells
    rho = _t(d["rho"])
    r = ctx.coag_step(rho, _t(Kc), _t(Kf), d["dt"], mode=2, prec=prec,
                      nsub=torch.zeros(C, dtype=torch.int32, device=DEV),
                      h_log=torch.zeros((C, 4), dtype=torch.float64, device=DEV))
    torch.cuda.synchronize()
    assert np.all(_np(r["status"]) == 0)
    x = _np(r["rho"])
    if prec == 0:
        np.testing.assert_array_equal(x, d["rho"])
    else:           # split precision restores each cell's entry mass, a no-op here
        np.testing.assert_allclose(x, d["rho"], rtol=1e-15, atol=0)
