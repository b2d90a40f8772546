"""16-cell-blocked FP64 rates (coag_rates_blocked, f32 = 0: both kinds in one
array, rows taken two pairs at a time) and the batched FP64 step reading them.

The blocked writer runs the same per-pair arithmetic as coag_rates, so its
values equal coag_rates' after unblocking (to 1e-15 relative, allowing a
different contraction of one expression); the padding cells of the last block
are zeros.  The step reads the same numbers from another address, so with
blocked rates it must reproduce the [C][P] path (itself held to the oracle by
test_gpu_parity): step counts and status exactly, states and step sizes to
rounding, 1e-12 relative with a floor of 1e-15 of the cell's largest bin.  Not
bit for bit: the FP64 step deposits its gain tiles with LDS atomics, whose
order follows the timing of the waves.  Grids: 150 bins (all per-grain values
tabulated), 200 (St and velocity), 320 (St only); cell counts with a ragged
last block of 16.
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


def _case(name, n_r, n_z, n_bins=None, kernel=None):
    from paper_2402_18471_amd import disc
    from paper_2402_18471_amd.coag import coag_create, coag_mass_grid
    cfg = disc.scaled(disc.CONFIGS[name], n_r, n_z, n_bins)
    m, me, s = coag_mass_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    d = disc.make_disc(cfg, s)
    old = os.environ.get("COAG_STEP_KERNEL")
    if kernel:
        os.environ["COAG_STEP_KERNEL"] = kernel
    try:
        ctx = coag_create(m, me, s, rho_m=cfg.rho_m)
    finally:
        if old is None:
            os.environ.pop("COAG_STEP_KERNEL", None)
        else:
            os.environ["COAG_STEP_KERNEL"] = old
    cells = {k: _t(v) for k, v in d["cells"].items()}
    return cfg, d, ctx, cells


def _unblock(K, C):
    from paper_2402_18471_amd.coag import unblock
    return unblock(K, C)


@pytest.mark.parametrize("case", [("disc256x128_n150", 5, 7, None), ("disc512x256_n200", 4, 4, None),
                                  ("disc64x32_n100", 5, 7, 320)])
def test_blocked_f64_rates_equal_cp_rates(case):
    cfg, d, ctx, cells = _case(*case)
    C = cfg.n_cells
    vd, vf = _t(d["v_dust"]), _t(d["v_frag"])
    from paper_2402_18471_amd.coag import pair_slots
    Kc, Kf = ctx.coag_rates(cells, vd, vf)
    B = ctx.coag_rates_blocked(cells, vd, vf, dtype=torch.float64)
    torch.cuda.synchronize()
    assert tuple(B.shape) == ((C + 15) // 16, pair_slots(cfg.n_bins), 64)
    bc, bf, rest = _unblock(B, C)
    for x, K in ((bc, Kc), (bf, Kf)):
        np.testing.assert_allclose(x, _np(K), rtol=1e-15, atol=0)
    # padding cells and the zero entries of rows of odd length
    assert rest.size == 2 * ((-C) % 16) * ctx.P + 2 * 16 * ((cfg.n_bins + 1) // 2) * B.shape[0]
    assert np.all(rest == 0.0)


@pytest.mark.parametrize("case", [("disc256x128_n150", 5, 7), ("disc512x256_n200", 4, 4),
                                  ("disc64x32_n100", 8, 4)])
@pytest.mark.parametrize("mode", ["adaptive", "fixed"])
def test_step_with_blocked_f64_rates_matches_the_cp_step(case, mode):
    from paper_2402_18471_amd import _lib as L
    cfg, d, ctx, cells = _case(*case)
    C = cfg.n_cells
    vd, vf = _t(d["v_dust"]), _t(d["v_frag"])
    K = ctx.coag_rates(cells, vd, vf)
    B = ctx.coag_rates_blocked(cells, vd, vf, dtype=torch.float64)
    # blocked rates hold the same values (within one rounding): step with
    # the [C][P] rates rebuilt from them, so both runs see identical numbers
    x, y, _ = _unblock(B, C)
    K = (_t(x), _t(y))
    for dt in (d["dt"], 20 * d["dt"]):
        kw = dict(max_sub=256) if mode == "adaptive" else dict(
            mode=L.FIXED, nsub=torch.full((C,), 5, dtype=torch.int32, device=DEV), max_sub=8)
        a = ctx.coag_step(_t(d["rho"]), *K, dt, **{k: (v.clone() if torch.is_tensor(v) else v)
                                                    for k, v in kw.items()})
        b = ctx.coag_step(_t(d["rho"]), B, None, dt, **{k: (v.clone() if torch.is_tensor(v) else v)
                                                         for k, v in kw.items()})
        torch.cuda.synchronize()
        assert np.all(_np(a["status"]) == 0)
        for key in ("nsub", "nrej", "status"):
            np.testing.assert_array_equal(_np(b[key]), _np(a[key]), err_msg=key)
        x, y = _np(b["rho"]), _np(a["rho"])
        assert np.all(np.abs(x - y) <= 1e-12 * np.abs(y) + 1e-15 * y.max(1, keepdims=True))
        for key in ("h", "h_log"):
            np.testing.assert_allclose(_np(b[key]), _np(a[key]), rtol=1e-12, atol=0, err_msg=key)


def test_blocked_f64_rate_errors():
    from paper_2402_18471_amd import _lib as L
    cfg, d, ctx, cells = _case("disc64x32_n100", 2, 2)
    vd, vf = _t(d["v_dust"]), _t(d["v_frag"])
    B = ctx.coag_rates_blocked(cells, vd, vf, dtype=torch.float64)
    rho = _t(d["rho"])
    with pytest.raises(L.CoagError) as e:               # double blocked rates, split step
        ctx.coag_step(rho, B, None, d["dt"], prec=1)
    assert e.value.code == L.COAG_EINVAL
    with pytest.raises(ValueError):                     # blocked rates with a Kf
        ctx.coag_step(rho, B, B, d["dt"])
    _, _, cctx, ccells = _case("disc64x32_n100", 2, 2, kernel="cell")
    B = cctx.coag_rates_blocked(ccells, vd, vf, dtype=torch.float64)
    with pytest.raises(L.CoagError) as e:               # per-cell FP64 kernel forced
        cctx.coag_step(rho, B, None, d["dt"])
    assert e.value.code == L.COAG_ENOTSUP
    np.testing.assert_array_equal(_np(rho), d["rho"])   # untouched
    torch.cuda.synchronize()
