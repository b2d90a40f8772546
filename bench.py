"""Throughput of the coagulation-fragmentation hot path on one MI355X.

One bench step = one coagulation call on every cell of the synthetic disc:
coag_rates (pair rates from the gas state and dust velocities) followed by
coag_step (adaptive BS3(2) sub-cycling over dt = 10 yr), the state carried
from step to step.  The metric is accepted cell-steps per second, a
cell-step being one accepted BS3 sub-step of one cell (three right-hand-side
evaluations, error estimate and FP64 update).

Prints one JSON line (see the design doc for every field).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector, dense
HBM_PEAK_GBS = 8000.0


def rhs_flops(N: int) -> float:
    """Algorithmic FP64 operations of one cell right-hand side: per pair 3 to
    form the coagulating/fragmenting collision rates, 10 for the five sparse
    gain deposits (coag pair, remnant pair, fragment bin), 4 for the two
    partners' losses; per bin 8 (n = rho/m, fragment suffix sum and the final
    gain - loss)."""
    P = N * (N + 1) // 2
    return 17.0 * P + 8.0 * N


def step_algebra_flops(N: int) -> float:
    """Stage states, update and error estimate of one BS3 attempt per cell."""
    return 20.0 * N


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="disc256x128_n150")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-cells", type=int, default=512)
    ap.add_argument("--prec", choices=("fp64", "split"), default="fp64")
    ap.add_argument("--rates", choices=("f64", "f32"), default="f64")
    ap.add_argument("--kernel", choices=("batch", "cell"), default="batch")
    return ap.parse_args()


def cpu_baseline(cfg, disc_mod, n_cells, target_s=10.0, max_calls=2000):
    """The oracle, untouched, on a bounded sample of the same workload:
    n_cells cells spread evenly over the disc, repeated coagulation calls
    (rates + adaptive step over dt, state carried) until about target_s of
    CPU time has been spent."""
    import oracle as O
    g = O.make_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    d = disc_mod.make_disc(cfg, g.s)
    idx = np.linspace(0, cfg.n_cells - 1, n_cells).astype(np.int64)
    sub = disc_mod.subset_cells(d, idx)
    rho = sub["rho"].copy()
    h = np.zeros(len(idx))
    acc = calls = 0
    t0 = time.perf_counter()
    while calls < max_calls and time.perf_counter() - t0 < target_s:
        Kc, Kf = O.rates(g, sub["cells"], sub["v_dust"], sub["v_frag"])
        r = O.step(g, rho, Kc, Kf, sub["dt"], h=h)
        rho, h = r["rho"], r["h"]
        acc += int(r["nsub"].sum())
        calls += 1
    dt = time.perf_counter() - t0
    return {"value": acc / dt, "unit": "cell-steps/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{len(idx)} cells spread over the {cfg.n_cells}-cell disc, {calls} coagulation "
                      f"calls each (rates + adaptive step), {acc} accepted cell-steps in {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                          "(the cell-parallel path would shard by radial rings, see DESIGN.md)"}))
        sys.exit(2)
    import torch
    from paper_2402_18471_amd import disc
    from paper_2402_18471_amd.coag import coag_create, coag_mass_grid

    cfg = disc.CONFIGS[args.config]
    dev = "cuda:0"
    if args.kernel == "cell":
        os.environ["COAG_STEP_KERNEL"] = "cell"
    split = args.prec == "split"
    f32 = args.rates == "f32"
    if f32 and not split:
        sys.exit("--rates f32 needs --prec split")
    m, me, s = coag_mass_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    d = disc.make_disc(cfg, s)
    C, N = cfg.n_cells, cfg.n_bins
    t = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    ctx = coag_create(m, me, s, rho_m=cfg.rho_m)
    cells = {k: t(v) for k, v in d["cells"].items()}
    v_dust, v_frag = t(d["v_dust"]), t(d["v_frag"])
    rho = t(d["rho"])
    h = torch.zeros(C, dtype=torch.float64, device=dev)
    K = args.steps
    nsub_all = torch.zeros((args.warmup + K, C), dtype=torch.int32, device=dev)
    nrej_all = torch.zeros((args.warmup + K, C), dtype=torch.int32, device=dev)
    status = torch.zeros(C, dtype=torch.int32, device=dev)
    Kc = torch.empty((C, ctx.P), dtype=torch.float32 if f32 else torch.float64, device=dev)
    Kf = torch.empty_like(Kc)
    from paper_2402_18471_amd import _lib as L
    import ctypes as ct
    lib = L.load()
    tol = L.Tol(1e-2, 1e-10, 1e-12, 4096, L.ADAPTIVE,
                L.PREC_SPLIT_BF16 if split else L.PREC_FP64, 0, 1 if f32 else 0)
    rates_fn = lib.coag_rates_f32 if f32 else lib.coag_rates
    cs = L.Cells(*[cells[k].data_ptr() for k in ("T", "rho_g", "c_s", "Omega", "H", "nu_mol", "alpha")])
    stream = torch.cuda.current_stream()
    sp = ct.c_void_p(stream.cuda_stream)
    p = lambda x: ct.c_void_p(x.data_ptr())
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.warmup + K)]

    def one(i):
        e0, e1, e2 = ev[i]
        e0.record(stream)
        L.check(rates_fn(ctx._h, C, ct.byref(cs), p(v_dust), p(v_frag), p(Kc), p(Kf), sp), ctx._h)
        e1.record(stream)
        L.check(lib.coag_step(ctx._h, C, p(rho), p(Kc), p(Kf), float(d["dt"]), p(h), ct.byref(tol),
                              p(nsub_all[i]), p(nrej_all[i]), None, p(status), sp), ctx._h)
        e2.record(stream)

    for i in range(args.warmup):
        one(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup, args.warmup + K):
        one(i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = status.cpu().numpy()
    ns = nsub_all[args.warmup:].cpu().numpy().astype(np.int64)
    nr = nrej_all[args.warmup:].cpu().numpy().astype(np.int64)
    acc, rej = int(ns.sum()), int(nr.sum())
    rates_ms = np.array([ev[i][0].elapsed_time(ev[i][1]) for i in range(args.warmup, args.warmup + K)])
    step_ms = np.array([ev[i][1].elapsed_time(ev[i][2]) for i in range(args.warmup, args.warmup + K)])
    # dominant kernel: the step kernel; algorithmic FP64 work per launch
    attempts_per_step = (ns + nr).sum(axis=1)          # per launch, summed over cells
    calls_per_launch = C                                # one k1 evaluation per cell per call
    flops = (3.0 * attempts_per_step + calls_per_launch) * rhs_flops(N) + \
        attempts_per_step * step_algebra_flops(N)
    achieved_tf = float(np.mean(flops / (step_ms * 1e-3)) / 1e12)
    out = {
        "metric": "coag cell-steps/s (accepted BS3 sub-steps x cells per second), FP64",
        "value": acc / wall,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": wall / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded transition-disc gas state, drift/settling velocities, MRN start)",
        "config": {"workload": cfg.name, "cells": C, "bins": N, "pairs": ctx.P,
                   "dt_yr": cfg.dt / 3.15576e7, "rtol": 1e-2, "atol_rel": 1e-10},
        "attempted_cell_steps_per_s": (acc + rej) / wall,
        "cells_calls_per_s": C * K / wall,
        "rates_ms": float(rates_ms.mean()),
        "step_ms": float(step_ms.mean()),
        "cells_failed": int((st != 0).sum()),
        "roofline": {"bound": "alu", "kernel": "k_step (coag_step, FP64)",
                     "achieved": achieved_tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tf / FP64_PEAK_TFLOPS, "traffic": None},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, disc, args.cpu_sample_cells)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
