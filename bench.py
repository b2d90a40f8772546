"""Throughput of the coagulation-fragmentation hot path on one MI355X.

One bench step = one coagulation call on every cell of the synthetic disc:
coag_rates_blocked (pair rates from the gas state and dust velocities, in the
16-cell-blocked layout the batched step reads) followed by coag_step
(adaptive BS3(2) sub-cycling over dt = 10 yr), the state carried from step to
step.  The metric is accepted cell-steps per second, a
cell-step being one accepted BS3 sub-step of one cell (three right-hand-side
evaluations, error estimate and FP64 update).

Measured on the 256x128-cell, 150-bin disc:
  value          FP64 path (FP64 rates, batched FP64 matrix-core step)
  split_bf16     split-BF16 step with FP32 rates: throughput, speedup over the
                 FP64 path, and its per-bin error against the FP64 oracle
                 (replaying the split call's steps) on a stratified sample of cells
  adjoint        coag_step_backward time over forward (rates + step) time on
                 the 64x32-cell, 100-bin disc, FP64 and split BF16 (and on
                 the bench disc, where the batched adjoint fills the GPU),
                 with the backward's algorithmic HBM bytes over its time
  roofline       the FP64 step kernel against HBM bandwidth: algorithmic
                 bytes = (16 P + 16 N) per cell per right-hand side
  cpu_baseline   the CPU oracle on a sample of the same workload

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes as ct
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
# what the batched step's code object is built from: its sources, the headers
# it includes and the build flags
KERNEL_FILES = [os.path.join("csrc", f) for f in ("coag_batch.hip", "coag_batch.h",
                                                    "coag_batch_common.h", "coag_launch.h",
                                                    "coag_device.h")] + ["build.py"]
COUNTERS = os.path.join(ROOT, "profiles", "kernel_counters.json")
# every file the transport kernels are built from, and their counter summary
TRANSPORT_FILES = [os.path.join("csrc", f) for f in ("coag_transport.hip", "coag_rate.h",
                                                    "coag_launch.h", "coag_device.h")] + [
    os.path.join("..", "include", f) for f in ("coag.h", "coag_transport.h")] + ["build.py"]
TR_COUNTERS = os.path.join(ROOT, "profiles", "transport_counters.json")


def progress(msg):
    """A line on stderr per finished phase (stdout carries only the JSON)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def lockstep_efficiency(attempts, prev):
    """Share of the batched step's cell-slots that do useful work: 16 cells
    advance in lockstep, so a batch costs 16 (1 + 3 max attempts) cell
    right-hand sides.  Also what grouping the cells by the previous call's
    attempts (a stable sort) would give."""
    def eff(a):
        C = a.shape[1]
        pad = (-C) % 16
        b = np.pad(a, ((0, 0), (0, pad)))
        used = (3 * a + 1).sum()
        cost = (16 * (3 * b.reshape(a.shape[0], -1, 16).max(axis=2) + 1)).sum()
        return float(used / cost)
    order = np.argsort(prev, axis=1, kind="stable")
    return {"efficiency": eff(attempts),
            "efficiency_grouped_by_previous_call": eff(np.take_along_axis(attempts, order, axis=1))}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="disc256x128_n150")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-split", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-vertical", action="store_true")
    ap.add_argument("--no-transport", action="store_true")
    ap.add_argument("--cpu-sample-cells", type=int, default=512)
    ap.add_argument("--kernel", choices=("batch", "cell"), default="batch",
                    help="FP64 step kernel (cell: one workgroup per cell)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with one 1 GiB device-to-device copy (counter calibration)")
    ap.add_argument("--evolve", metavar="CONFIG",
                    help="instead of the step benchmark: differentiable coagulation calls "
                         "(torch.autograd, checkpointed) on CONFIG, forward and backward timed")
    ap.add_argument("--evolve-calls", type=int, default=20)
    ap.add_argument("--evolve-ckpt", type=int, default=20)
    ap.add_argument("--evolve-prec", choices=("fp64", "split"), default="split")
    ap.add_argument("--summarize-transport-counters", nargs=3,
                    metavar=("OUT_JSON", "FETCH_CSV", "WRITE_CSV"),
                    help="no GPU work: write the transport kernels' counter summary (the "
                         "transport roofline's traffic is read from it) from a FETCH_SIZE and a "
                         "WRITE_SIZE pass of rocprofv3 over a 'bench.py --steps 1 --warmup 1 "
                         "--no-cpu-baseline --no-adjoint --no-vertical --no-split "
                         "--calibrate-copy' run")
    ap.add_argument("--summarize-counters", nargs="+",
                    metavar="OUT_JSON BENCH_LOG TRACE_CSV PMC_CSV",
                    help="no GPU work: write the per-kernel counter summary (the roofline's "
                         "traffic is read from it) from the output of a 'bench.py --steps 1 "
                         "--warmup 1 --no-cpu-baseline --calibrate-copy' run, a rocprofv3 kernel "
                         "trace of the bench, and the counter_collection.csv files of rocprofv3 "
                         "passes over that run (FETCH_SIZE, WRITE_SIZE, issue counters, FP64 "
                         "instruction counters)")
    return ap.parse_args()


ADJ_BUDGET = 8 << 30        # the library's workspace budget for one adjoint slab


def evolve_memory_plan(C, N, calls, ckpt, width, prec_split):
    """Device bytes the differentiable run holds at its peak (the backward
    pass), on the host from the shapes: the rates of one call (16-cell-blocked
    FP32 for split; FP64 [C][P] plus the step's reordered copy for FP64), the
    step's slope workspace, the adjoint's slab workspace (the library's rule:
    rates, their derivative factors, step starts and stage states of `width`
    steps, replay state, slopes and v3 for the fewest equal slabs of whole
    16-cell batches that fit ADJ_BUDGET, all cells if they fit), checkpoints
    every ckpt calls, the
    compacted step logs (width per call, an upper bound) and step counts,
    one segment's start states, and the state, its gradient and g_out."""
    P = N * (N + 1) // 2
    m = N >> 1
    SL = (m + 1) ** 2 if N & 1 else m * (m + 1)          # pair slots per 16-cell block
    Cb = -(-C // 16) * 16
    al = lambda b: -(-b // 256) * 256
    rates = Cb // 16 * 64 * SL * 4 if prec_split else 2 * C * P * 8 + Cb // 16 * 64 * SL * 8
    slopes = al(Cb * 5 * N * 8)

    def adj(S):
        Sb = -(-S // 16) * 16
        rt, gt = (4, 4) if prec_split else (8, 8)
        return (al(rt * 64 * SL * (Sb // 16)) + 2 * al(gt * P * Sb) + al(8 * N * (width + 1) * S) +
                al(8 * N * 2 * width * S) + al(8 * N * S) + al(Sb * 5 * N * 8) + al(4 * S) +
                al(8 * N * S))
    if adj(C) <= ADJ_BUDGET:
        S = C
    else:
        smax = max(4096, ADJ_BUDGET // adj(16) * 16)
        nslab = -(-C // smax)
        S = min(C, -(-(-(-C // nslab)) // 16) * 16)
    state = C * N * 8
    plan = {"rates_one_call": rates, "step_workspace": slopes, "adjoint_slab_cells": S,
            "adjoint_workspace": adj(S), "checkpoints": -(-calls // ckpt) * state,
            "step_logs_upper_bound": calls * C * width * 8, "step_counts": calls * C * 4,
            "segment_starts": ckpt * state, "state_grads": 4 * state}
    plan["total"] = sum(v for k, v in plan.items() if k != "adjoint_slab_cells")
    return {k: (v / 1e9 if k != "adjoint_slab_cells" else v) for k, v in plan.items()}


def evolve(args):
    """Forward and backward time of n differentiable coagulation calls
    (paper_2402_18471_amd.autograd.coag_evolve: ADAPTIVE, checkpoint every
    ckpt calls; the backward recomputes each segment and runs the adjoint in
    the forward's precision) on one disc, loss = sum over cells of the
    mass-weighted mean ln s; the device memory in use, sampled after every
    checkpoint segment of both passes, beside the plan computed from the
    shapes."""
    import torch
    from paper_2402_18471_amd import disc
    from paper_2402_18471_amd import _lib as L
    from paper_2402_18471_amd.autograd import coag_evolve
    from paper_2402_18471_amd.coag import coag_create, coag_mass_grid
    cfg = disc.CONFIGS[args.evolve]
    m, me, s = coag_mass_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    d = disc.make_disc(cfg, s)
    dev = "cuda:0"
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    ctx = coag_create(m, me, s, rho_m=cfg.rho_m)
    cells = {k: t(v) for k, v in d["cells"].items()}
    rho0 = t(d["rho"]).requires_grad_(True)
    al = t(d["cells"]["alpha"]).requires_grad_(True)
    vf = t(d["v_frag"]).requires_grad_(True)
    lns = t(np.log(s))
    split = args.evolve_prec == "split"
    prec = L.PREC_SPLIT_BF16 if split else L.PREC_FP64
    max_sub = 64
    plan = evolve_memory_plan(cfg.n_cells, cfg.n_bins, args.evolve_calls, args.evolve_ckpt,
                              max_sub, split)
    progress(f"evolve {cfg.name}: {args.evolve_calls} calls, {args.evolve_prec}; planned peak "
             f"<= {plan['total']:.1f} GB (step logs at their {max_sub}-step upper bound)")
    free0, total = torch.cuda.mem_get_info()
    peak = {"forward": 0.0, "backward": 0.0}
    tick = {"t": time.perf_counter()}

    def on_segment(phase, done, n):
        torch.cuda.synchronize()
        used = (total - torch.cuda.mem_get_info()[0]) / 1e9
        peak[phase] = max(peak[phase], used)
        now = time.perf_counter()
        progress(f"{phase}: {done}/{n} calls, {now - tick['t']:.1f} s, device memory {used:.1f} GB")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = coag_evolve(ctx, rho0, al, vf, cells, t(d["v_dust"]), float(d["dt"]), args.evolve_calls,
                      ckpt_every=args.evolve_ckpt, prec=prec, max_sub=max_sub,
                      progress=on_segment)
    J = ((out * lns).sum(1) / out.sum(1)).sum()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    used_fwd = (total - torch.cuda.mem_get_info()[0]) / 1e9
    progress(f"forward {t1 - t0:.2f} s")
    tick["t"] = t1
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    used_bwd = (total - torch.cuda.mem_get_info()[0]) / 1e9
    progress(f"backward {t2 - t1:.2f} s")
    g = [x.grad for x in (rho0, al, vf)]
    print(json.dumps({
        "workload": cfg.name, "cells": cfg.n_cells, "bins": cfg.n_bins, "calls": args.evolve_calls,
        "ckpt_every": args.evolve_ckpt, "forward_precision": args.evolve_prec,
        "adjoint_precision": args.evolve_prec, "forward_s": t1 - t0, "backward_s": t2 - t1,
        "backward_over_forward": (t2 - t1) / (t1 - t0),
        "cell_calls_per_s_forward": cfg.n_cells * args.evolve_calls / (t1 - t0),
        "device_memory_in_use_gb": {"before": (total - free0) / 1e9, "after_forward": used_fwd,
                                    "after_backward": used_bwd,
                                    "max_sampled_forward": peak["forward"],
                                    "max_sampled_backward": peak["backward"]},
        "memory_plan_gb": plan,
        "gradients_finite": bool(all(torch.isfinite(x).all() for x in g)),
        "data": "synthetic disc, forward = coag_rates + ADAPTIVE coag_step per call"}), flush=True)


def _kernel_short(name):
    """Kernel name without return type, namespaces and arguments."""
    import re
    n = name.replace("void ", "").replace("(anonymous namespace)::", "").replace("coag::", "")
    return re.sub(r"\(.*", "", n).strip()


def summarize_counters(out_json, bench_log, trace_csv, *pmc_csvs):
    """Per-kernel counter summary of rocprofv3 passes over one 'bench.py
    --steps 1 --warmup 1 --no-cpu-baseline --calibrate-copy' run (FETCH_SIZE,
    WRITE_SIZE, issue counters, FP64 instruction counters; one pass each), with
    durations from a kernel trace of the bench.  Launches are grouped by
    kernel and grid size (the bench disc's launches, the adjoint's slabs and
    the small samples have different grids); per group the mean per launch,
    and for the step kernels the timed (second) launch.  FETCH_SIZE and
    WRITE_SIZE (KiB) are scaled by what they read for the final 1 GiB device
    copy; busy fractions are per SIMD: cycles = GRBM_GUI_ACTIVE / 8 XCDs,
    1024 SIMDs, 4 cycles per wave64 VALU instruction; FP64 FLOPs =
    64 (ADD + MUL + TRANS + 2 FMA) instructions."""
    import csv
    import hashlib
    counters = {}                   # (kernel, grid) -> list over launches of {counter: value}
    order = {}
    for path in pmc_csvs:
        per = {}
        for r in csv.DictReader(open(path)):
            d = per.setdefault(int(r["Dispatch_Id"]),
                               {"k": (_kernel_short(r["Kernel_Name"]), int(r["Grid_Size"]))})
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        seen = {}
        for did in sorted(per):
            d = per[did]
            key = d.pop("k")
            idx = seen[key] = seen.get(key, -1) + 1
            slot = counters.setdefault(key, [])
            while len(slot) <= idx:
                slot.append({})
            slot[idx].update(d)
            order.setdefault(key, did)
    dur = {}
    for r in csv.DictReader(open(trace_csv)):
        grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        key = (_kernel_short(r["Kernel_Name"]), grid)
        dur.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6)
    copies = [c for (k, gsz), L in counters.items() if k == "__amd_rocclr_copyBuffer" for c in L
              if "FETCH_SIZE" in c]
    cal = max(copies, key=lambda c: c["FETCH_SIZE"])
    f_fac = (1 << 30) / (cal["FETCH_SIZE"] * 1024.0)
    w_cal = max((c for (k, gsz), L in counters.items() if k == "__amd_rocclr_copyBuffer" for c in L
                 if "WRITE_SIZE" in c), key=lambda c: c["WRITE_SIZE"])
    w_fac = (1 << 30) / (w_cal["WRITE_SIZE"] * 1024.0)
    b = json.loads([ln for ln in open(bench_log) if ln.startswith("{")][-1])
    disc_grid = -(-b["config"]["cells"] // 16) * 512          # threads of a step launch
    shas = kernel_shas()
    out = {"kernel_sources_sha256": shas,
           "workload": f"{b['config']['workload']} (bench.py --steps 1 --warmup 1); adjoint "
                       "kernels from its adjoint legs", "calibration": {
               "copy_bytes": 1 << 30, "FETCH_SIZE_KiB": cal["FETCH_SIZE"], "fetch_factor": f_fac,
               "WRITE_SIZE_KiB": w_cal["WRITE_SIZE"], "write_factor": w_fac},
           "groups": []}
    for key in sorted(counters, key=lambda k: order[k]):
        name, grid = key
        if not any(t in name for t in ("k_step_batch", "k_rates", "k_adj", "k_rate_derivs")):
            continue
        L = counters[key]

        def mean(c, sel=None):
            v = [x[c] for x in (L if sel is None else [L[sel]]) if c in x]
            return float(np.mean(v)) if v else None
        g = {"kernel": name, "grid_threads": grid, "launches": len(L),
             "trace_ms_mean": float(np.mean(dur[key])) if key in dur else None}
        # the step on the whole bench disc: the second launch is the timed call
        # (later ones, if any, are the adjoint leg's forward calls)
        sel = 1 if name.startswith("k_step_batch") and grid == disc_grid and len(L) > 1 else None
        g["counted_launch"] = "second (the timed call)" if sel == 1 else "mean over launches"
        if mean("FETCH_SIZE", sel) is not None:
            g["fetch_bytes"] = mean("FETCH_SIZE", sel) * 1024.0 * f_fac
            g["fetch_bytes_mean"] = mean("FETCH_SIZE") * 1024.0 * f_fac
        if mean("WRITE_SIZE", sel) is not None:
            g["write_bytes"] = mean("WRITE_SIZE", sel) * 1024.0 * w_fac
            g["write_bytes_mean"] = mean("WRITE_SIZE") * 1024.0 * w_fac
        grbm = mean("GRBM_GUI_ACTIVE", sel)
        if grbm:
            cyc = grbm / 8.0
            g["counter_ms"] = cyc / 2.4e6
            g["counter_ms_mean"] = mean("GRBM_GUI_ACTIVE") / 8.0 / 2.4e6
            if mean("SQ_INSTS_VALU", sel) is not None:
                g["valu_busy"] = mean("SQ_INSTS_VALU", sel) * 4.0 / (1024.0 * cyc)
                g["mfma_busy"] = mean("SQ_VALU_MFMA_BUSY_CYCLES", sel) / (1024.0 * cyc)
                g["valu_instr"] = mean("SQ_INSTS_VALU", sel)
                g["mfma_instr"] = mean("SQ_INSTS_MFMA", sel)
                g["lds_instr"] = mean("SQ_INSTS_LDS", sel)
            f64 = [mean(c, sel) for c in ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64",
                                           "SQ_INSTS_VALU_TRANS_F64", "SQ_INSTS_VALU_FMA_F64")]
            if all(x is not None for x in f64):
                g["fp64_flop"] = 64.0 * (f64[0] + f64[1] + f64[2] + 2.0 * f64[3])
        out["groups"].append(g)
    out["bench_rhs_per_call"] = {"fp64": b["rhs_per_call"], "split": b["split_bf16"]["rhs_per_call"]}
    with open(out_json, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def kernel_shas(files=None):
    """SHA-256 of every file the batched step's code object (or the files
    given, paths relative to the package) is built from."""
    import hashlib
    pkg = os.path.join(ROOT, "paper_2402_18471_amd")
    return {f: hashlib.sha256(open(os.path.join(pkg, f), "rb").read()).hexdigest()
            for f in (KERNEL_FILES if files is None else files)}


def summarize_transport_counters(out_json, fetch_csv, write_csv):
    """Counter summary of the transport kernels from a FETCH_SIZE and a
    WRITE_SIZE pass of rocprofv3 over one 'bench.py --steps 1 --warmup 1
    --no-cpu-baseline --no-adjoint --no-vertical --no-split --calibrate-copy'
    run: per kernel the mean over its launches (all on the bench disc), in
    bytes, scaled by what the counters read for the final 1 GiB device copy;
    the step's bytes are those of k_tr_prep, k_tr_half and k_tr_full."""
    import csv
    vals = {}
    for path in (fetch_csv, write_csv):
        for r in csv.DictReader(open(path)):
            k = _kernel_short(r["Kernel_Name"])
            if k == "__amd_rocclr_copyBuffer":
                k = (k, int(r["Grid_Size"]))
            vals.setdefault((k, r["Counter_Name"]), []).append(float(r["Counter_Value"]))
    cal = {c: max(max(v) for (k, cn), v in vals.items()
                  if isinstance(k, tuple) and cn == c) for c in ("FETCH_SIZE", "WRITE_SIZE")}
    fac = {c: (1 << 30) / (cal[c] * 1024.0) for c in cal}
    kern = {}
    for (k, cn), v in vals.items():
        if isinstance(k, str) and k.startswith("k_tr_") and cn in fac:
            d = kern.setdefault(k, {"launches": len(v)})
            d["fetch_bytes" if cn == "FETCH_SIZE" else "write_bytes"] = (
                sum(v) / len(v) * 1024.0 * fac[cn])
    step = sum(kern[k][b] for k in ("k_tr_prep", "k_tr_half", "k_tr_full")
               for b in ("fetch_bytes", "write_bytes"))
    out = {"kernel_sources_sha256": kernel_shas(TRANSPORT_FILES),
           "workload": "disc256x128_n150 transport (bench.py --steps 1 --warmup 1 "
                       "--no-cpu-baseline --no-adjoint --no-vertical --no-split --calibrate-copy)",
           "calibration": {"copy_bytes": 1 << 30, "FETCH_SIZE_KiB": cal["FETCH_SIZE"],
                           "WRITE_SIZE_KiB": cal["WRITE_SIZE"], "fetch_factor": fac["FETCH_SIZE"],
                           "write_factor": fac["WRITE_SIZE"]},
           "kernels": kern, "step_bytes": step}
    with open(out_json, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({"step_bytes": step, "kernels": kern}))


def transport_traffic():
    """HBM bytes of one transport step on the bench disc from the committed
    counter summary, or None when there is none or any file the transport
    kernels are built from has changed since the counters were taken."""
    try:
        with open(TR_COUNTERS) as f:
            c = json.load(f)
        shas = kernel_shas(TRANSPORT_FILES)
    except OSError:
        return None
    if c.get("kernel_sources_sha256") != shas:
        return None
    return float(c["step_bytes"])


def profiled_traffic(rhs_per_launch, kind):
    """HBM bytes per launch of the batched step kernel (FP64 or split form) on
    the bench disc from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE of the timed launch, calibrated on a device copy, scaled per
    cell right-hand side), or None when there is none or any file the kernel
    is built from (sources, headers, build flags) has changed since the
    counters were taken."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
        shas = kernel_shas()
    except OSError:
        return None
    if c.get("kernel_sources_sha256") != shas:
        return None
    want = "k_step_batch<0, double, true>" if kind == "fp64" else "k_step_batch<1, float, true>"
    grp = [g for g in c["groups"] if g["kernel"] == want and "fetch_bytes" in g]
    if not grp:
        return None
    g = max(grp, key=lambda x: x["grid_threads"])
    per = (g["fetch_bytes"] + g["write_bytes"]) / c["bench_rhs_per_call"][kind]
    return float(np.mean(rhs_per_launch) * per / 1e9)


def cpu_model():
    """The host CPU's model name (/proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(cfg, disc_mod, n_cells, target_s=10.0, max_calls=2000, one_thread_s=5.0):
    """The oracle, untouched, on a bounded sample of the same workload:
    n_cells cells spread evenly over the disc, repeated coagulation calls
    (rates + adaptive step over dt, state carried) until about target_s of
    CPU time has been spent, on all the host's threads; then the same sample
    from its start again on one thread for about one_thread_s."""
    import oracle as O
    g = O.make_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    d = disc_mod.make_disc(cfg, g.s)
    idx = np.linspace(0, cfg.n_cells - 1, n_cells).astype(np.int64)
    sub = disc_mod.subset_cells(d, idx)

    def run(budget):
        rho = sub["rho"].copy()
        h = np.zeros(len(idx))
        acc = calls = 0
        t0 = time.perf_counter()
        while calls < max_calls and time.perf_counter() - t0 < budget:
            Kc, Kf = O.rates(g, sub["cells"], sub["v_dust"], sub["v_frag"])
            r = O.step(g, rho, Kc, Kf, sub["dt"], h=h)
            rho, h = r["rho"], r["h"]
            acc += int(r["nsub"].sum())
            calls += 1
        return acc, calls, time.perf_counter() - t0

    cores = O.num_threads()
    acc, calls, dt = run(target_s)
    O.set_num_threads(1)
    try:
        acc1, calls1, dt1 = run(one_thread_s)
    finally:
        O.set_num_threads(cores)
    return {"value": acc / dt, "unit": "cell-steps/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "one_thread_value": acc1 / dt1,
            "sample": f"{len(idx)} cells spread over the {cfg.n_cells}-cell disc, {calls} coagulation "
                      f"calls each (rates + adaptive step), {acc} accepted cell-steps in {dt:.1f} s "
                      f"on {cores} threads; one thread: {calls1} calls, {acc1} cell-steps in "
                      f"{dt1:.1f} s (the same calls from the same start, fewer of them)"}


class Disc:
    """A synthetic disc resident on the GPU with its context and buffers."""

    def __init__(self, cfg_name, torch, kernel="batch"):
        from paper_2402_18471_amd import disc
        from paper_2402_18471_amd import _lib as L
        from paper_2402_18471_amd.coag import coag_create, coag_mass_grid
        if kernel == "cell":
            os.environ["COAG_STEP_KERNEL"] = "cell"
        self.torch, self.L = torch, L
        # a disc of (R, Z) cells, or columns of the vertically integrated kernel
        self.vertical = cfg_name in disc.COLUMNS
        self.cfg = cfg = disc.COLUMNS[cfg_name] if self.vertical else disc.CONFIGS[cfg_name]
        dev = self.dev = "cuda:0"
        m, me, s = coag_mass_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
        self.d = d = disc.make_columns(cfg, s) if self.vertical else disc.make_disc(cfg, s)
        self.C, self.N = cfg.n_cells, cfg.n_bins
        self.kernel = kernel
        self.t = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt,
                                                              device=dev)
        self.ctx = coag_create(m, me, s, rho_m=cfg.rho_m, vertical=self.vertical)
        os.environ.pop("COAG_STEP_KERNEL", None)
        self.P = self.ctx.P
        self.cells = {k: self.t(v) for k, v in d["cells"].items()}
        self.v_dust, self.v_frag = self.t(d["v_dust"]), self.t(d["v_frag"])
        self.lib = L.load()
        self.cs = L.Cells(*[self.cells[k].data_ptr() for k in
                            ("T", "rho_g", "c_s", "Omega", "H", "nu_mol", "alpha")])
        self.stream = torch.cuda.current_stream()
        self.sp = ct.c_void_p(self.stream.cuda_stream)

    def p(self, x):
        return ct.c_void_p(x.data_ptr()) if x is not None else None

    def forward(self, steps, warmup, split, rho=None):
        """steps + warmup coagulation calls from rho (default: the initial
        state); per-call HIP-event times of rates and step on the stream."""
        torch, L = self.torch, self.L
        C = self.C
        f32 = split
        # rates layout: 16-cell-blocked (float for split, double for the
        # batched FP64 step); [C][P] for the per-cell FP64 kernel
        blk = split or self.kernel == "batch"
        rho = (self.t(self.d["rho"]) if rho is None else rho.clone())
        h = torch.zeros(C, dtype=torch.float64, device=self.dev)
        n = warmup + steps
        nsub = torch.zeros((n, C), dtype=torch.int32, device=self.dev)
        nrej = torch.zeros((n, C), dtype=torch.int32, device=self.dev)
        status = torch.zeros(C, dtype=torch.int32, device=self.dev)
        max_sub = 4096
        # blocked: both kinds in Kc, Kf unused
        Kc = torch.empty(self.ctx.blocked_shape(C) if blk else (C, self.P),
                         dtype=torch.float32 if f32 else torch.float64, device=self.dev)
        Kf = None if blk else torch.empty_like(Kc)
        tol = L.Tol(1e-2, 1e-10, 1e-12, max_sub, L.ADAPTIVE,
                    L.PREC_SPLIT_BF16 if split else L.PREC_FP64, 0,
                    L.RATES_BLK32 if f32 else (L.RATES_BLK64 if blk else L.RATES_CP64))
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(n)]
        p, sp, h_ = self.p, self.sp, self.ctx._h
        dt = float(self.d["dt"])

        def one(i):
            e = ev[i]
            e[0].record(self.stream)
            if blk:
                L.check(self.lib.coag_rates_blocked(h_, C, ct.byref(self.cs), p(self.v_dust),
                                                    p(self.v_frag), 1 if f32 else 0, p(Kc), sp), h_)
            else:
                L.check(self.lib.coag_rates(h_, C, ct.byref(self.cs), p(self.v_dust),
                                            p(self.v_frag), p(Kc), p(Kf), sp), h_)
            e[1].record(self.stream)
            L.check(self.lib.coag_step(h_, C, p(rho), p(Kc), p(Kf), dt, p(h), ct.byref(tol),
                                       p(nsub[i]), p(nrej[i]), None, p(status), sp), h_)
            e[2].record(self.stream)

        for i in range(warmup):
            one(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(warmup, n):
            one(i)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        sl = slice(warmup, n)
        ns = nsub[sl].cpu().numpy().astype(np.int64)
        nr = nrej[sl].cpu().numpy().astype(np.int64)
        prev = (nsub + nrej)[warmup - 1:n - 1].cpu().numpy() if warmup > 0 else ns + nr
        return dict(wall=wall, acc=int(ns.sum()), rej=int(nr.sum()), ns=ns, nr=nr, prev_attempts=prev,
                    rates_ms=np.array([ev[i][0].elapsed_time(ev[i][1]) for i in range(warmup, n)]),
                    step_ms=np.array([ev[i][1].elapsed_time(ev[i][2]) for i in range(warmup, n)]),
                    failed=int((status.cpu().numpy() != 0).sum()), rho=rho)


def split_error(D, sample, calls=20):
    """Split-BF16 step against the FP64 oracle over the same steps, on a
    sample of cells from the disc's initial state: one split call over
    `calls` dt (ADAPTIVE, FP32 blocked rates, its own steps), then the oracle
    replays those steps in FP64 with its own rates from the same start.
    Resolved bins hold >= 1e-12 of the cell's mass; the rest are reported
    relative to the cell's mass."""
    import oracle as O
    torch, L = D.torch, D.L
    from paper_2402_18471_amd import disc
    idx = np.asarray(sample)
    sub = disc.subset_cells(D.d, idx)
    cells = {k: D.t(v) for k, v in sub["cells"].items()}
    vd, vf = D.t(sub["v_dust"]), D.t(sub["v_frag"])
    rho0 = sub["rho"]
    dt = calls * float(D.d["dt"])
    K32 = D.ctx.coag_rates_blocked(cells, vd, vf)
    b = D.ctx.coag_step(D.t(rho0), K32, None, dt, prec=L.PREC_SPLIT_BF16, max_sub=1024)
    torch.cuda.synchronize()
    x, ns, hl = b["rho"].cpu().numpy(), b["nsub"].cpu().numpy(), b["h_log"].cpu().numpy()
    g = O.make_grid(D.cfg.n_bins, D.cfg.s_min, D.cfg.s_max, rho_m=D.cfg.rho_m,
                    vertical=int(D.vertical))
    oKc, oKf = O.rates(g, sub["cells"], sub["v_dust"], sub["v_frag"])
    ref = O.step(g, rho0, oKc, oKf, dt, mode=O.REPLAY, nsub=ns, h_log=hl)["rho"]
    M = ref.sum(1, keepdims=True)
    res = ref >= 1e-12 * M
    err = np.abs(x - ref)
    return {"sample": f"{len(idx)} cells (every {D.C // len(idx)}th) from the initial state, one "
                      f"split call over {calls} dt ({float(ns.mean()):.1f} accepted sub-steps per "
                      "cell), replayed by the FP64 oracle",
            "max_rel_err_resolved_bins": float(np.max(err[res] / ref[res])),
            "max_abs_err_unresolved_bins_over_cell_mass": float(np.max((err / M)[~res]))
            if np.any(~res) else 0.0,
            "max_total_mass_err": float(np.max(np.abs(x.sum(1) / rho0.sum(1) - 1))),
            "status_ok": bool(np.all(b["status"].cpu().numpy() == 0))}


def adjoint_ratio(torch, workload, reps=3, dt_scale=1.0):
    """Backward / forward time of the same coagulation call on `workload`, in
    FP64 and in split BF16: the first call from the initial state (rates +
    ADAPTIVE step, steps recorded; the split form with FP32 blocked rates),
    then coag_step_backward of that call in the same precision (which
    recomputes the rates and their derivative factors, replays the stage
    states and runs the reverse sweep); HIP events on the stream, mean over
    reps after one warm-up.  Also the backward's algorithmic HBM bytes over
    its time: per cell, the rates and derivative factors written once
    (2 + 2 arrays of P), the replay's 1 + 3 n right-hand sides (rates and
    state read), the sweep's 3 n transposed ones (rates, derivative factors,
    stage state, cotangents), n = accepted steps of the cell."""
    from paper_2402_18471_amd import _lib as L
    D = Disc(workload, torch)
    rho_in = D.t(D.d["rho"])
    dt = float(D.d["dt"]) * dt_scale
    P, N = D.P, D.N
    g_out = torch.ones((D.C, D.N), dtype=torch.float64, device=D.dev) / rho_in.sum(1, keepdim=True)
    out = {"workload": D.cfg.name, "cells": D.C, "dt_yr": dt / 3.15576e7}
    for name, prec in (("fp64", L.PREC_FP64), ("split_bf16", L.PREC_SPLIT_BF16)):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        fwd, bwd = [], []
        for r in range(reps + 1):
            rho = rho_in.clone()
            ev[0].record(D.stream)
            if prec == L.PREC_SPLIT_BF16:
                Kc, Kf = D.ctx.coag_rates_blocked(D.cells, D.v_dust, D.v_frag), None
            else:
                Kc, Kf = D.ctx.coag_rates(D.cells, D.v_dust, D.v_frag)
            a = D.ctx.coag_step(rho, Kc, Kf, dt, max_sub=64, prec=prec, check_status=False)
            ev[1].record(D.stream)
            ev[2].record(D.stream)
            D.ctx.coag_step_backward(rho_in, D.cells, D.v_dust, D.v_frag, a["h_log"], a["nsub"],
                                     g_out, prec=prec)
            ev[3].record(D.stream)
            torch.cuda.synchronize()
            L.check_cells(a["status"])
            del Kc, Kf
            if r:
                fwd.append(ev[0].elapsed_time(ev[1]))
                bwd.append(ev[2].elapsed_time(ev[3]))
        f, b = float(np.mean(fwd)), float(np.mean(bwd))
        n = a["nsub"].cpu().numpy().astype(np.float64)
        rt = 4 if prec == L.PREC_SPLIT_BF16 else 8
        per_cell = (4 * rt * P + (1 + 3 * n) * (2 * rt * P + 16 * N) +
                    3 * n * (4 * rt * P + 40 * N))
        ach = float(per_cell.sum() / (b * 1e-3) / 1e9)
        out[name] = {"backward_ms": b, "forward_ms": f, "adjoint_over_forward": b / f,
                     "accepted_substeps_per_cell": float(n.mean()),
                     "backward_roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                                           "unit": "GB/s", "frac": ach / HBM_PEAK_GBS}}
    out["note"] = ("same call both ways: the first call from the initial state; forward = rates "
                   "+ ADAPTIVE step; backward recomputes the rates, their derivative factors and "
                   "the stage states, then runs the reverse sweep; backward_roofline: the "
                   "backward's algorithmic bytes (see bench.py adjoint_ratio) over its time")
    return out


def vertical_columns(torch, workload, steps=10, warmup=2):
    """The vertically integrated kernel on `workload` (columns, surface
    densities): FP64 and split-BF16 calls with the state carried, the split
    form's error against the FP64 oracle on a sample of columns, and the
    adjoint's backward / forward time in both precisions."""
    D = Disc(workload, torch)
    out = {"workload": D.cfg.name, "columns": D.C, "bins": D.N,
           "dt_yr": D.cfg.dt / 3.15576e7}
    for name, split in (("fp64", False), ("split_bf16", True)):
        r = D.forward(steps, warmup, split)
        out[name] = {"value": r["acc"] / r["wall"], "unit": "cell-steps/s",
                     "ms_per_step": r["wall"] / steps * 1e3,
                     "rates_ms": float(r["rates_ms"].mean()),
                     "step_ms": float(r["step_ms"].mean()), "cells_failed": r["failed"],
                     "accepted_substeps_per_call": r["acc"] / (steps * D.C)}
    out["split_bf16"]["speedup_vs_fp64"] = out["split_bf16"]["value"] / out["fp64"]["value"]
    out["split_bf16"]["error_vs_oracle"] = split_error(D, np.arange(0, D.C, max(1, D.C // 64)),
                                                       calls=1)
    a = adjoint_ratio(torch, workload, reps=1, dt_scale=0.3)
    out["adjoint"] = {"dt_yr": a["dt_yr"], **{k: {"adjoint_over_forward": a[k]["adjoint_over_forward"],
                                                  "backward_ms": a[k]["backward_ms"]}
                                              for k in ("fp64", "split_bf16")}}
    return out


def transport_leg(torch, config, steps=20, warmup=3, evolve_yr=10.0):
    """The transport step of the dynamics solver on `config`'s grid and
    species (Sec. 3): `steps` CFL steps from the disc's initial state, each
    step's two kernels timed with HIP events on the current stream; HBM
    roofline of the step with 160 algorithmic bytes per (cell, species) (the
    state at t^n read twice, the half-step state written once and read once,
    the new state written: 5 x 32 bytes); then the scheduler (coag_evolve,
    FP64 coagulation) over `evolve_yr` years from the disc's initial state."""
    from paper_2402_18471_amd import disc
    from paper_2402_18471_amd.coag import TransportContext, coag_create, coag_mass_grid
    cfg = disc.CONFIGS[config]
    m, me, s = coag_mass_grid(cfg.n_bins, cfg.s_min, cfg.s_max, rho_m=cfg.rho_m)
    d = disc.make_transport(cfg, s)
    dev = "cuda:0"
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    tc = TransportContext(d["R_edge"], d["t_edge"], s, rho_m=cfg.rho_m, GM=d["GM"])
    cells = {k: t(v) for k, v in d["cells"].items()}
    rho, v, vg = t(d["rho"]), t(d["v"]), t(d["v_gas"])
    C, N = cfg.n_cells, cfg.n_bins
    ms, dts = [], []
    for k in range(warmup + steps):
        dt = tc.dt(cells, v)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        tc.step(cells, vg, rho, v, dt)
        e1.record()
        e1.synchronize()
        if k >= warmup:
            ms.append(e0.elapsed_time(e1))
            dts.append(dt)
    step_ms = float(np.mean(ms))
    byts = 160.0 * C * N
    tb = transport_traffic() if config == "disc256x128_n150" else None
    out = {"workload": f"{config} transport", "cells": C, "species": N, "steps": steps,
           "step_ms": step_ms, "cell_species_updates_per_s": C * N / (step_ms * 1e-3),
           "cfl_dt_yr": float(np.mean(dts)) / 3.15576e7,
           "roofline": {"bound": "hbm", "achieved": byts / (step_ms * 1e-3) / 1e9, "peak": 8000.0,
                        "unit": "GB/s", "frac": byts / (step_ms * 1e-3) / 1e9 / 8000.0,
                        "traffic": None if tb is None else tb / 1e9, "traffic_unit": "GB per step",
                        "algorithmic_bytes": "160 B per (cell, species) per step"}}
    ctx = coag_create(m, me, s, rho_m=cfg.rho_m)
    rho, v = t(d["rho"]), t(d["v"])
    h = torch.zeros(C, dtype=torch.float64, device=dev)
    vf = t(d["v_frag"])
    t_end = evolve_yr * 3.15576e7
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    st = tc.evolve(ctx, cells, vg, vf, rho, v, h, t_end)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    out["evolve"] = {"t_end_yr": t_end / 3.15576e7, "wall_s": wall, **st,
                     "note": "coag_evolve: CFL transport steps, FP64 coagulation triggered by the "
                             "scheduler rule; wall time includes one host sync per transport step"}
    # the same run with a dust-to-gas floor of 1e-20 per species: near-empty
    # species move with the gas and stop setting the CFL step
    eps = 1e-20
    tf = TransportContext(d["R_edge"], d["t_edge"], s, rho_m=cfg.rho_m, GM=d["GM"], eps_floor=eps)
    rho, v = t(d["rho"]), t(d["v"])
    h = torch.zeros(C, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    st = tf.evolve(ctx, cells, vg, vf, rho, v, h, t_end)
    torch.cuda.synchronize()
    out["evolve_floor"] = {"eps_floor": eps, "t_end_yr": t_end / 3.15576e7,
                           "wall_s": time.perf_counter() - w0, **st}
    return out


def main():
    args = parse()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
    if args.summarize_transport_counters:
        summarize_transport_counters(*args.summarize_transport_counters)
        return
    if args.evolve:
        evolve(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                          "(cells are independent: the path would shard by radial rings dealt "
                          "cyclically over the GPUs)"}))
        sys.exit(2)
    import torch
    from paper_2402_18471_amd import disc

    D = Disc(args.config, torch, args.kernel)
    progress(f"disc {args.config} ready")
    C, N, P = D.C, D.N, D.P
    K, W = args.steps, args.warmup
    f = D.forward(K, W, False)
    progress(f"fp64: {K} calls, {f['wall'] / K * 1e3:.2f} ms per call")
    attempts = f["ns"] + f["nr"]                              # [steps][C]
    lockstep = lockstep_efficiency(attempts, f["prev_attempts"])
    rhs_per_launch = (3 * attempts + 1).sum(axis=1)            # k1 once per cell per call
    bytes_per_launch = rhs_per_launch * (16.0 * P + 16.0 * N)
    achieved = float(np.mean(bytes_per_launch / (f["step_ms"] * 1e-3)) / 1e9)
    out = {
        "metric": "coag cell-steps/s, FP64 vs split-BF16 at <=1e-6 rel err; adjoint/fwd time",
        "value": f["acc"] / f["wall"],
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": f["wall"] / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded transition-disc gas state, drift/settling velocities, MRN start)",
        "config": {"workload": D.cfg.name, "cells": C, "bins": N, "pairs": P,
                   "dt_yr": D.cfg.dt / 3.15576e7, "rtol": 1e-2, "atol_rel": 1e-10,
                   "fp64_step_kernel": args.kernel},
        "attempted_cell_steps_per_s": (f["acc"] + f["rej"]) / f["wall"],
        "cells_calls_per_s": C * K / f["wall"],
        "rates_ms": float(f["rates_ms"].mean()),
        "step_ms": float(f["step_ms"].mean()),
        "cells_failed": f["failed"],
        "rhs_per_call": float(np.mean(rhs_per_launch)),
        "lockstep": lockstep,
        "roofline": {"bound": "hbm", "kernel": "coag_step FP64 (k_step_batch)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": profiled_traffic(rhs_per_launch, "fp64"),
                     "traffic_unit": "GB per launch",
                     "algorithmic_bytes": "(16 P + 16 N) B per cell per right-hand side; "
                                          "1 + 3 x attempts right-hand sides per cell per call"},
    }
    if not args.no_split:
        s = D.forward(K, W, True)
        progress(f"split: {K} calls, {s['wall'] / K * 1e3:.2f} ms per call")
        s_rhs = (3 * (s["ns"] + s["nr"]) + 1).sum(axis=1)
        s_alg = s_rhs * (8.0 * P + 16.0 * N)          # FP32 rates
        s_ach = float(np.mean(s_alg / (s["step_ms"] * 1e-3)) / 1e9)
        out["split_bf16"] = {
            "rhs_per_call": float(np.mean(s_rhs)),
            "roofline": {"bound": "hbm", "kernel": "coag_step split-BF16 (k_step_batch)",
                         "achieved": s_ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": s_ach / HBM_PEAK_GBS,
                         "traffic": profiled_traffic(s_rhs, "split"),
                         "traffic_unit": "GB per launch",
                         "algorithmic_bytes": "(8 P + 16 N) B per cell per right-hand side"},
            "value": s["acc"] / s["wall"], "unit": "cell-steps/s", "rates": "f32",
            "ms_per_step": s["wall"] / K * 1e3, "rates_ms": float(s["rates_ms"].mean()),
            "step_ms": float(s["step_ms"].mean()), "cells_failed": s["failed"],
            "speedup_vs_fp64": (s["acc"] / s["wall"]) / (f["acc"] / f["wall"]),
            "error_vs_oracle": split_error(D, np.arange(0, C, max(1, C // 512))),
        }
    free, total = torch.cuda.mem_get_info()
    out["device_memory_used_gb"] = (total - free) / 1e9    # rates, workspaces, torch cache
    if not args.no_adjoint:
        out["adjoint"] = adjoint_ratio(torch, "disc64x32_n100_adj")
        progress("adjoint timed on the 64x32 x 100 disc")
        out["adjoint_on_bench_disc"] = adjoint_ratio(torch, args.config, reps=2)
        progress(f"adjoint timed on {args.config}")
    if not args.no_vertical:
        out["vertical"] = vertical_columns(torch, "col4096_n200")
        progress("vertically integrated kernel timed on 4096 columns")
    if not args.no_transport:
        out["transport"] = transport_leg(torch, args.config)
        progress("transport step and scheduler timed")
    if not args.no_cpu_baseline:
        progress("oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(D.cfg, disc, args.cpu_sample_cells)
    if args.calibrate_copy:
        x = torch.ones(1 << 27, dtype=torch.float64, device=D.dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = 1 << 30
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
