"""Closed forms on the GPU: one cell, 40 mass bins over 1e-12 - 1e-3 g, a
constant kernel K0 = 1e-10 cm^3/s (no fragmentation), monodisperse start
N0 = 1e3 cm^-3 in bin 0, integrated to K0 N0 t = 10 with FIXED steps.

  NUMBER split: the binned total number follows the scalar BS3 recursion of
    dN/dt = -K0 N^2 / 2 under the same steps, and converges to the closed form
    N0 / (1 + K0 N0 t / 2) = N0 / 6 at third order in h;
  MASS split: the second moment grows exactly as M2(0) + K0 M1^2 t;
  total mass is conserved.
Each for the batched FP64 step, the per-cell FP64 step and the split-BF16
step (the last to its 1e-6 bar; its mass by the FP64 bookkeeping).
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
K0, N0, T_END = 1e-10, 1e3, 1e8
FORMS = [("batch", 0), ("cell", 0), ("batch", 1)]


def _ctx(split, kernel):
    from paper_2402_18471_amd.coag import coag_create, coag_mass_grid
    m, me, s = coag_mass_grid(40, 1e-12, 1e-3, by_mass=True, rho_m=1.67)
    old = os.environ.get("COAG_STEP_KERNEL")
    os.environ["COAG_STEP_KERNEL"] = kernel
    try:
        return coag_create(m, me, s, rho_m=1.67, split=split), m
    finally:
        if old is None:
            os.environ.pop("COAG_STEP_KERNEL", None)
        else:
            os.environ["COAG_STEP_KERNEL"] = old


def _run(ctx, m, n, prec):
    N = len(m)
    w = np.array([0.5 if i == j else 1.0 for i in range(N) for j in range(i + 1)])
    Kc = torch.as_tensor((w * K0)[None, :], dtype=torch.float64, device=DEV)
    Kf = torch.zeros_like(Kc)
    rho = torch.zeros((1, N), dtype=torch.float64, device=DEV)
    rho[0, 0] = N0 * m[0]
    r = ctx.coag_step(rho, Kc, Kf, T_END, mode=1, prec=prec,
                      nsub=torch.full((1,), n, dtype=torch.int32, device=DEV), max_sub=n)
    torch.cuda.synchronize()
    assert int(r["status"][0]) == 0
    return r["rho"][0].cpu().numpy()


def _bs3_scalar(f, y, h, n):
    for _ in range(n):
        k1 = f(y)
        k2 = f(y + 0.5 * h * k1)
        k3 = f(y + 0.75 * h * k2)
        y = y + h * (2 / 9 * k1 + 1 / 3 * k2 + 4 / 9 * k3)
    return y


@pytest.mark.parametrize("form", FORMS)
def test_number_closed_form(form):
    kernel, prec = form
    ctx, m = _ctx(1, kernel)                    # NUMBER split
    exact = N0 / (1 + 0.5 * K0 * N0 * T_END)
    tol = 1e-13 if prec == 0 else 1e-6
    errs = []
    for n in (100, 200, 400, 800):
        rho = _run(ctx, m, n, prec)
        Nb = (rho / m).sum()
        Ns = _bs3_scalar(lambda y: -0.5 * K0 * y * y, N0, T_END / n, n)
        assert abs(Nb / Ns - 1) < tol, (n, Nb, Ns)
        assert abs(rho.sum() / (N0 * m[0]) - 1) < (1e-13 if prec == 0 else 1e-12)
        errs.append(abs(Nb - exact) / exact)
    if prec == 0:
        orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        assert np.all(np.abs(orders - 3.0) < 0.1), orders
    assert errs[-1] < 1e-6


@pytest.mark.parametrize("form", FORMS)
def test_mass_split_second_moment(form):
    kernel, prec = form
    ctx, m = _ctx(0, kernel)                    # MASS split
    M1 = N0 * m[0]
    for n in (100, 400):
        rho = _run(ctx, m, n, prec)
        M2 = (rho * m).sum()
        expect = M1 * m[0] + K0 * M1 ** 2 * T_END
        assert abs(M2 / expect - 1) < (1e-13 if prec == 0 else 1e-6), (n, M2, expect)
        assert abs(rho.sum() / M1 - 1) < (1e-13 if prec == 0 else 1e-12)
