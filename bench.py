#!/usr/bin/env python3
"""Throughput of the AGIS simple iteration (S[AC] + frame rotator) on one GPU.

One "step" is one full iteration of the hot path over the whole synthetic
workload: the S block over every source, the A/C accumulation pass over every
observation, the segmented band solves, the calibration solve and the frame
rotator.  Inputs are resident in HBM before the timed region starts.

Prints one JSON line (metric obs/s per AGIS iteration).  The CPU baseline is
the oracle (test infrastructure) timed on a bounded sample of the same
workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


# Algorithmic per-unit figures of the two observation passes (FP64 flops,
# an add, multiply or divide counting 1 and a fused multiply-add 2; bytes
# each pass must move).  The flop counts follow the formulas of the
# observation model as the kernels evaluate them:
#   model (ephemeris, proper direction, aberration, B-splines, attitude,
#   SRS direction, field angle, residual)                          226
#   A/C: attitude partials 29, normal-equation terms 83, the 120 interval
#        sums 240                                                  352
#   S:   source partials 72, weight 2, the 21 source sums 58        132
AC_FLOPS_PER_OBS = 226.0 + 352.0
S_FLOPS_PER_OBS = 226.0 + 132.0
S_FLOPS_PER_SOURCE = 400.0     # 5x5 modified Cholesky, variances, update
AC_BYTES_PER_OBS = 28.0        # t 8, eta 8, sigma 4, cell+fov 4, source 4
AC_BYTES_PER_INTERVAL = 8.0 * (116 + 4) + 8.0 + 4 * 8.0   # sums out, offset, coefficient in
AC_BYTES_PER_SOURCE = 56.0     # r, mu vector, parallax of s^(k+1)
S_BYTES_PER_OBS = 28.0         # t 8, eta 8, sigma 4, cell+fov 4, left index 4
S_BYTES_PER_SOURCE = 40.0 + 40.0 + 64.0 + 40.0 + 8.0 + 4.0 + 8.0   # s in/out, prep, d, Q, defect, offset

KERNEL_SOURCES = ("paper_1112_4139_amd/csrc/hot.hip", "paper_1112_4139_amd/csrc/model.h")
PMC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_gaia1.txt")
KERNEL_SYMBOL = {"ac_pass": "k_ac_pass", "source_update": "k_source_update"}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch of kernel from the committed rocprofv3 PMC
    summary (FETCH_SIZE + WRITE_SIZE scaled by a copy-kernel calibration),
    taken on the FP64 gaia1 workload; None for another workload or
    precision, when no summary exists or when the kernels changed since."""
    if workload != "gaia1" or precision != "fp64" or not os.path.exists(PMC_FILE):
        return None
    vals = {}
    with open(PMC_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha1") != kernel_source_hash():
        return None
    key = KERNEL_SYMBOL[kernel] + " hbm_bytes_per_launch"
    return float(vals[key]) if key in vals else None


def workload_description(name, w):
    sp = w.spec
    return {"workload": name,
            "sources": int(w.src_true.shape[0]), "observations": int(w.n_obs),
            "years": sp.years, "obs_per_transit": sp.ccd_per_transit, "knot_interval_s": sp.knot_dt,
            "attitude_coefficients": int(w.n_att), "cells": int(w.n_cells), "segment_intervals": sp.seg_len,
            "overlap_L": sp.seg_overlap, "lambda": sp.lambda_reg, "sigma_uas": 100.0,
            "outlier_frac": sp.outlier_frac, "robust": bool(sp.robust),
            **({"ac_obs_per_transit": 1, "ac_observations": int((w.cell < 0).sum()),
                "sigma_ac_uas": round(float(w.sigma[w.cell < 0][0]) / 4.8481368e-12, 1)} if sp.ac_obs else {}),
            "law": "Gaia-like: spin 60 arcsec/s, precession 63 d, aspect 45 deg, basic angle 106.5 deg"}


def cpu_baseline(w, frac, log_fn):
    """Time one oracle iteration on a source subset of the same workload."""
    import oracle
    import synth
    oracle.build()
    rng = np.random.default_rng(7)
    n_src = w.src_true.shape[0]
    m = max(1, int(n_src * frac))
    pick = np.sort(rng.choice(n_src, m, replace=False))
    remap = -np.ones(n_src, np.int64)
    remap[pick] = np.arange(m)
    keep = remap[w.src] >= 0
    import copy
    ws = copy.copy(w)
    ws.src_true = w.src_true[pick]
    ws.src_start = w.src_start[pick]
    for name in ("t", "fov", "cell", "sigma", "eps", "eta_nominal"):
        setattr(ws, name, np.ascontiguousarray(getattr(w, name)[keep]))
    ws.src = np.ascontiguousarray(remap[w.src[keep]].astype(np.int32))
    eta = oracle.observed_field_angles(ws)
    pr = oracle.problem_from_world(ws, eta, state="start")
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    log_fn(f"cpu baseline: oracle on {m} sources, {ws.n_obs} obs, {threads} threads")
    t0 = time.perf_counter()
    pr.iterate(s_ref=ws.src_true)
    dt = time.perf_counter() - t0
    return {"value": ws.n_obs / dt, "unit": "obs/s", "cores": threads, "kind": "oracle",
            "sample": f"one S[AC]+frame iteration over {m} of {n_src} sources ({ws.n_obs} obs) and all "
                      f"{w.n_att} attitude coefficients, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="gaia1")
    ap.add_argument("--seg-len", type=int, default=None)
    ap.add_argument("--cpu-frac", type=float, default=0.2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64",
                    help="mixed: FP32 partials and compensated FP32 normal-equation sums")
    ap.add_argument("--scheme", choices=("si", "cg"), default="si",
                    help="si: one simple S[AC] iteration per step; cg: one conjugate-gradient step per step "
                         "(cycles of 40 iterations; an iteration is one pass of the blocks plus p'N p)")
    ap.add_argument("--ac", action="store_true",
                    help="add one across-scan observation per transit (cell -1) to the workload")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the timed steps, run one plain device copy of this many MiB (the reference "
                         "kernel for scaling HBM counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding of this path "
              "is a design note, not a measured configuration", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth.configs as C
    from paper_1112_4139_amd import agis

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    over = {} if args.seg_len is None else {"seg_len": args.seg_len}
    if args.ac:
        over["ac_obs"] = True
    wname = args.workload + ("+ac" if args.ac else "")
    t0 = time.time()
    w = C.make(args.workload, progress=log, **over)
    log(f"workload {args.workload}: {w.src_true.shape[0]} sources, {w.n_obs} obs, {w.n_att} coefficients "
        f"({time.time() - t0:.1f} s)")

    ctx = agis.agis_create(w.consts, w.knots, precision=1 if args.precision == "mixed" else 0, device=0)
    n_src = w.src_true.shape[0]
    # observed field angles of the synthetic world: the library's own model at
    # the true parameters (eta_obs = eta(t | truth) - c_true + noise)
    zeros = np.zeros(w.n_obs)
    agis.agis_load_observations(ctx, w.t, zeros, w.sigma, w.src, w.fov, w.cell, n_src, w.n_cells)
    agis.agis_set_sources(ctx, w.src_true)
    agis.agis_set_attitude(ctx, w.att_true)
    agis.agis_set_calibration(ctx, w.cal_true)
    R = agis.agis_residuals(ctx)                   # = c_true - eta_true
    eta_obs = -R + w.eps
    del R, zeros
    if args.no_cpu_baseline:
        w.eps = w.eta_nominal = None           # not needed any more
    log("observed field angles computed")
    agis.agis_load_observations(ctx, w.t, eta_obs, w.sigma, w.src, w.fov, w.cell, n_src, w.n_cells)
    agis.agis_set_sources(ctx, w.src_start)
    agis.agis_set_attitude(ctx, w.att_start)
    agis.agis_set_calibration(ctx, w.cal_start)
    agis.agis_set_frame_reference(ctx, w.src_true)
    sz = agis.agis_problem_size(ctx)
    log(f"store built: {sz}")

    s_group = agis.agis_autotune(ctx)
    log(f"autotuned: {s_group} lanes per source")

    def step():
        if args.scheme == "cg":
            agis.agis_cg_iterate(ctx, 1, 40, stats=False)
        else:
            agis.agis_iterate(ctx, 1, stats=False)

    for i in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} done")
    kt = {k: [] for k in ("source_update", "ac_pass", "band_solve", "calib_solve", "frame")}
    t_start = time.perf_counter()
    for i in range(args.steps):
        step()
        for k, v in agis.agis_kernel_times(ctx).items():
            kt[k].append(v)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_step = 1000.0 * elapsed / args.steps
    value = w.n_obs / (elapsed / args.steps)
    kavg = {k: float(np.mean(v)) for k, v in kt.items()}
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step, kernels {kavg}")
    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {n * 8} bytes read, {n * 8} bytes written")
        agis.agis_destroy(ctx)
        return
    st = agis.agis_iterate(ctx, 1, stats=True)[0]
    log(f"last iteration stats: S rms {st['s']['rms_update']} A defect {st['a']['defect']}")

    # dominant kernel and its roofline: both observation passes are bound by
    # FP64 arithmetic (their algorithmic HBM traffic needs ~10% of 8 TB/s)
    K = w.n_att - 3
    dom = max(("ac_pass", "source_update"), key=lambda k: kavg[k])
    if dom == "ac_pass":
        alg_flops = AC_FLOPS_PER_OBS * w.n_obs
        alg_bytes = AC_BYTES_PER_OBS * w.n_obs + AC_BYTES_PER_INTERVAL * K + AC_BYTES_PER_SOURCE * n_src
    else:
        alg_flops = S_FLOPS_PER_OBS * w.n_obs + S_FLOPS_PER_SOURCE * n_src
        alg_bytes = S_BYTES_PER_OBS * w.n_obs + S_BYTES_PER_SOURCE * n_src + 32.0 * w.n_att
    sec = kavg[dom] * 1e-3
    tfs = alg_flops / sec / 1e12
    traffic = measured_traffic(dom, wname, args.precision)
    roofline = {"kernel": dom, "bound": "alu", "achieved": round(tfs, 2), "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(tfs / FP64_PEAK_TFLOPS, 4), "traffic": traffic,
                "alg_flops_per_launch": alg_flops, "alg_bytes_per_launch": alg_bytes,
                "alg_hbm_GBs": round(alg_bytes / sec / 1e9, 1),
                "alg_hbm_frac": round(alg_bytes / sec / 1e9 / HBM_PEAK_GBS, 4), "avg_ms": kavg[dom]}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args.cpu_frac, log)
        log(f"cpu baseline {cpu['value']:.3g} obs/s on {cpu['cores']} threads")

    out = {"metric": "obs/s per AGIS iteration", "value": value, "unit": "obs/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if args.precision == "fp64" else "f64 model, f32 partials and sums", "data": "synthetic",
           "config": {**workload_description(wname, w), "lanes_per_source": s_group,
                      **({"scheme": "conjugate gradients"} if args.scheme == "cg" else {})},
           "kernel_ms": kavg, "roofline": roofline,
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)
    agis.agis_destroy(ctx)


if __name__ == "__main__":
    main()
