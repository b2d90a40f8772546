"""Extended-precision evaluation of the oracle's right-hand side, BS3 steps
of a given step sequence, and hand-written adjoint (TEST INFRASTRUCTURE ONLY:
loaded by tests/ alone, like the rest of the oracle).

The same definitions as the C oracle, in the same order of terms: the
right-hand side of the binned Smoluchowski equation (Sec. 5, eqs. `smol`,
`ngain`, the loss term, fragments through eq. `Nijk`), the Bogacki-Shampine
3(2) update (Sec. 5, closing paragraph; tableau of Bogacki & Shampine 1989)
over a frozen sequence of step sizes (FIXED / REPLAY), and the transposed
stage recurrences of its adjoint with dJ/dKc, dJ/dKf per pair.  The
arithmetic is numpy's long double (64-bit significand on x86-64), fed the
oracle's own FP64 redistribution tables, rates and rate derivatives, so it
evaluates exactly the problem the FP64 oracle and the GPU evaluate, with
about 2000x less rounding.

Why: where gain and loss of a bin nearly cancel (a heavy grain sweeping up
light ones keeps almost all of the product's mass), every FP64 evaluation
carries an error of eps (gain + loss), and some outputs amplify it (the
adjoint in bins empty at the start loses up to ~2e-3 of the cell's largest
component over 200 calls in the oracle's order).  There the FP64 oracle is
not precise enough to judge a result; this evaluation is.
"""
from __future__ import annotations

import numpy as np

from . import Grid, redistribution_sparse, rates_deriv

LD = np.longdouble


class _Scatter:
    """Sum of vals[:, q] into out[:, idx[q]] for a fixed index array, by
    sorting once and reducing contiguous runs (np.add.reduceat keeps the
    dtype; np.bincount would round to FP64)."""

    def __init__(self, idx, N):
        self.order = np.argsort(idx, kind="stable")
        s = idx[self.order]
        self.starts = np.flatnonzero(np.r_[True, s[1:] != s[:-1]])
        self.targets = s[self.starts]
        self.N = N

    def __call__(self, vals):
        out = np.zeros((vals.shape[0], self.N), vals.dtype)
        out[:, self.targets] = np.add.reduceat(vals[:, self.order], self.starts, axis=1)
        return out


class Extended:
    """Right-hand side, steps and adjoint of C cells on grid g with pair rates
    Kc, Kf ([C][P] FP64, e.g. from oracle.rates), in dtype (long double by
    default; float64 gives the oracle's arithmetic in numpy's order)."""

    def __init__(self, g: Grid, Kc, Kf, dtype=LD):
        T = self.T = dtype
        t = redistribution_sparse(g)
        N, P = g.N, g.P
        self.N, self.P = N, P
        i = np.repeat(np.arange(N), np.arange(1, N + 1))
        j = np.concatenate([np.arange(k + 1) for k in range(N)])
        self.pi, self.pj = i, j
        self.m = np.asarray(g.m, dtype=T)
        self.ci = t["ci"].astype(np.int64)
        self.ci1 = np.minimum(self.ci + 1, N - 1)
        self.cw0, self.cw1 = t["cw"][:, 0].astype(T), t["cw"][:, 1].astype(T)
        self.ri = t["ri"].astype(np.int64)
        self.ri1 = np.minimum(self.ri + 1, N - 1)
        self.rw0, self.rw1 = t["rw"][:, 0].astype(T), t["rw"][:, 1].astype(T)
        self.fl = t["fl"].astype(np.int64)
        self.fm = t["fm"].astype(T)
        self.Nf = t["Nfrac"].astype(T)                 # [l][k] = N_k(m^e_{l+1})
        self.w = np.where(i == j, T(0.5), T(1.0))
        self.Kc = np.asarray(Kc, dtype=T).reshape(-1, P)
        self.Kf = np.asarray(Kf, dtype=T).reshape(-1, P)
        self.C = self.Kc.shape[0]
        Kt = (self.Kc + self.Kf) / self.w              # un-halved kernel for the loss
        self.Kfull = np.zeros((self.C, N, N), T)
        self.Kfull[:, i, j] = Kt
        self.Kfull[:, j, i] = Kt
        sc = lambda idx: _Scatter(idx, N)
        self._ci, self._ci1, self._ri, self._ri1 = sc(self.ci), sc(self.ci1), sc(self.ri), sc(self.ri1)
        self._fl, self._i, self._j = sc(self.fl), sc(i), sc(j)
        self.offdiag = (i != j).astype(T)

    def rhs(self, y):
        """drho/dt of every cell: gain - loss (eqs. `smol`, `ngain`)."""
        n = y / self.m
        nn = n[:, self.pi] * n[:, self.pj]
        Rc, Rf = nn * self.Kc, nn * self.Kf
        gain = (self._ci(Rc * self.cw0) + self._ci1(Rc * self.cw1) +
                self._ri(Rf * self.rw0) + self._ri1(Rf * self.rw1))
        gain = gain + self._fl(Rf * self.fm) @ self.Nf
        loss = self.m * n * np.einsum("cik,ci->ck", self.Kfull, n)
        return gain - loss

    def vjp(self, y, mu):
        """J(y)^T mu, and the per-pair a sc, a sf (dJ/dKc, dJ/dKf terms)."""
        n = y / self.m
        pi, pj = self.pi, self.pj
        suf = mu @ self.Nf.T                           # sum_{k<=l} mu_k N_k(m^e_{l+1})
        lp = (mu[:, pi] * self.m[pi] + self.offdiag * mu[:, pj] * self.m[pj]) / self.w
        dc = mu[:, self.ci] * self.cw0 + mu[:, self.ci1] * self.cw1
        df = mu[:, self.ri] * self.rw0 + mu[:, self.ri1] * self.rw1 + self.fm * suf[:, self.fl]
        sc, sf = dc - lp, df - lp
        a = n[:, pi] * n[:, pj]
        ga = self.Kc * sc + self.Kf * sf
        gn = self._i(n[:, pj] * ga) + self._j(n[:, pi] * ga)
        return gn / self.m, a * sc, a * sf

    def _steps(self, h_log, nsub):
        h = np.asarray(h_log, dtype=np.float64).reshape(self.C, -1)
        ns = np.asarray(nsub, dtype=np.int64).reshape(self.C)
        return h, ns

    def step(self, rho, h_log, nsub):
        """nsub[c] BS3 steps of sizes h_log[c][:] (REPLAY; FIXED is the same
        with equal sizes).  Cells take their steps in lockstep; a cell whose
        steps are done keeps its state."""
        T = self.T
        y = np.asarray(rho, dtype=T).copy()
        h, ns = self._steps(h_log, nsub)
        for s in range(int(ns.max()) if len(ns) else 0):
            act = ns > s
            hs = np.where(act, h[:, min(s, h.shape[1] - 1)], 0.0).astype(T)[:, None]
            k1 = self.rhs(y)
            k2 = self.rhs(y + T(0.5) * hs * k1)
            k3 = self.rhs(y + T(0.75) * hs * k2)
            yn = y + hs * (T(2.0 / 9.0) * k1 + T(1.0 / 3.0) * k2 + T(4.0 / 9.0) * k3)
            y = np.where(act[:, None], yn, y)
        return y

    def step_backward(self, rho_in, h_log, nsub, g_out, dKc_da=None, dKf_da=None, dKc_dv=None,
                      dKf_dv=None):
        """Adjoint of step(): g_in = dJ/drho_in for g_out = dJ/drho_end, and
        dJ/dKc, dJ/dKf per pair; with the rate derivatives given ([C][P],
        e.g. oracle.rates_deriv), also dJ/dalpha and dJ/dv_frag per cell."""
        T = self.T
        h, ns = self._steps(h_log, nsub)
        y = np.asarray(rho_in, dtype=T).copy()
        starts = []
        for s in range(int(ns.max()) if len(ns) else 0):
            act = ns > s
            hs = np.where(act, h[:, min(s, h.shape[1] - 1)], 0.0).astype(T)[:, None]
            starts.append((y.copy(), hs))
            k1 = self.rhs(y)
            k2 = self.rhs(y + T(0.5) * hs * k1)
            k3 = self.rhs(y + T(0.75) * hs * k2)
            yn = y + hs * (T(2.0 / 9.0) * k1 + T(1.0 / 3.0) * k2 + T(4.0 / 9.0) * k3)
            y = np.where(act[:, None], yn, y)
        lam = np.asarray(g_out, dtype=T).copy()
        gKc, gKf = np.zeros_like(self.Kc), np.zeros_like(self.Kf)
        for ys, hs in reversed(starts):
            # cells without this step have hs = 0: every product below vanishes
            k1 = self.rhs(ys)
            y2 = ys + T(0.5) * hs * k1
            k2 = self.rhs(y2)
            y3 = ys + T(0.75) * hs * k2
            v3, a3, b3 = self.vjp(y3, hs * T(4.0) / T(9.0) * lam)
            v2, a2, b2 = self.vjp(y2, hs / T(3.0) * lam + T(0.75) * hs * v3)
            mu1 = hs * T(2.0) / T(9.0) * lam + T(0.5) * hs * v2
            lam = lam + (v3 + v2)
            v1, a1, b1 = self.vjp(ys, mu1)
            lam = lam + v1
            gKc += a3 + a2 + a1
            gKf += b3 + b2 + b1
        out = {"g_in": lam, "gKc": gKc, "gKf": gKf}
        if dKc_da is not None:
            d = [np.asarray(x, dtype=T).reshape(self.C, self.P)
                 for x in (dKc_da, dKf_da, dKc_dv, dKf_dv)]
            out["g_alpha"] = (gKc * d[0] + gKf * d[1]).sum(1)
            out["g_vfrag"] = (gKc * d[2] + gKf * d[3]).sum(1)
        return out


def step_backward(g: Grid, cells, v_dust, v_frag, rho_in, h_log, nsub, g_out, Kc, Kf,
                  dtype=LD):
    """The oracle's adjoint of one call (as oracle.step_backward) in extended
    precision, on the oracle's own FP64 rates Kc, Kf and rate derivatives.
    Returns dict(g_in, g_alpha, g_vfrag, gKc, gKf) in dtype."""
    e = Extended(g, Kc, Kf, dtype)
    d = rates_deriv(g, cells, v_dust, v_frag)
    return e.step_backward(rho_in, h_log, nsub, g_out, d["dKc_dalpha"], d["dKf_dalpha"],
                           d["dKc_dvfrag"], d["dKf_dvfrag"])
