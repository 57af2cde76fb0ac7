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
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


# Algorithmic work per observation per iteration (a fused multiply-add
# counts 2 flop), the per-unit figures of the hot-path measurement plan:
#   forward model 186, source partials 60, attitude partials 50,
#   source sums 40, attitude sums 290, calibration sums 4;
#   the robust inner iteration's three further solves 240 (4 rounds in all).
# Per kernel:
MODEL_FLOPS = 186.0
S_FLOPS_PER_OBS = MODEL_FLOPS + 60.0 + 40.0              # 286
S_ROBUST_FLOPS_PER_OBS = S_FLOPS_PER_OBS + 240.0          # 526
AC_FLOPS_PER_OBS = MODEL_FLOPS + 50.0 + 290.0 + 4.0       # 530
EPS_FLOPS_PER_OBS = MODEL_FLOPS + 4.0                     # a model pass and R^2 - sigma^2
# Algorithmic HBM bytes: every pass streams 28 B per observation (t 8,
# eta 8, sigma 4, cell+fov 4, left index or source 4) and gathers ~88 B per
# source; the A/C pass writes 62 doubles per attitude coefficient.
BYTES_PER_OBS = 28.0
BYTES_PER_SOURCE = 88.0
BYTES_PER_COEF = 62.0 * 8.0

KERNEL_SOURCES = ("paper_1112_4139_amd/csrc/hot.hip", "paper_1112_4139_amd/csrc/model.h",
                  "paper_1112_4139_amd/csrc/robust.hip", "paper_1112_4139_amd/csrc/source_block.h")
# kernel timer -> symbol prefix of its kernels in the counter summaries
KERNEL_SYMBOL = {"ac_pass": "k_ac_pass", "source_update": "k_source_update", "source_update_robust": "k_s_",
                 "excess_noise": "k_eps_fused"}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def pmc_file(workload):
    return os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.txt")


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch of a kernel (its HIP-event timer's kernels) from
    the committed rocprofv3 counter summary of the workload (FETCH_SIZE +
    WRITE_SIZE scaled by a copy-kernel calibration), taken in FP64; None for
    another precision, when no summary exists or when the kernel sources
    changed since the counters were taken."""
    path = pmc_file(workload)
    if precision != "fp64" or not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha1") != kernel_source_hash():
        return None
    key = kernel + " hbm_bytes_per_launch"
    return float(vals[key].split()[0]) if key in vals else None


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
            **({"calibration": "large-scale along-scan geometric: 3 shifted-Legendre coefficients per cell and CCD",
                "calibration_groups": int(w.n_cells * w.consts["geo_ccds"])} if sp.geo_cal else {}),
            **({"small_scale": f"one value per CCD, {sp.geo_small_days}-day interval and pixel column (eq:cc2)",
                "small_scale_values": int(w.geo_small_true.size)} if sp.geo_cal and sp.geo_small else {}),
            "law": "Gaia-like: spin 60 arcsec/s, precession 63 d, aspect 45 deg, basic angle 106.5 deg"}


def geo_coefficients(w, which):
    """The world's geometric coefficients, AL, then AC and small-scale where
    the world has them (the layout agis_set_geo_calibration takes)."""
    parts = [getattr(w, f"geo_{which}")] + [x for x in (getattr(w, f"geo_ac_{which}", None),
                                                         getattr(w, f"geo_small_{which}", None)) if x is not None]
    return np.concatenate([np.reshape(x, -1) for x in parts])


def host_description():
    model, ram = None, None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.lower().startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal"):
                    ram = round(int(line.split()[1]) / 1024 ** 2, 1)
                    break
    except OSError:
        pass
    return model, ram


def time_slice(w, day0, n_days):
    """The observations of n_days whole days from day day0 of the mission:
    the sources they see (renumbered), the attitude coefficients and knots
    that cover them, the days' calibration cells.  Across-scan records keep
    cell -1."""
    import copy
    DAY = 86400.0
    t0 = w.consts["t_beg"] + day0 * DAY
    t1 = min(t0 + n_days * DAY, w.consts["t_end"])
    keep = (w.t >= t0) & (w.t < t1)
    ws = copy.copy(w)
    src_ids, inv = np.unique(w.src[keep], return_inverse=True)
    ws.src_true, ws.src_start = w.src_true[src_ids], w.src_start[src_ids]
    for name in ("t", "fov", "sigma", "eps"):
        setattr(ws, name, np.ascontiguousarray(getattr(w, name)[keep]))
    ws.src = np.ascontiguousarray(inv.astype(np.int32))
    cell = w.cell[keep]
    ws.cell = np.ascontiguousarray(np.where(cell >= 0, cell - 2 * day0, cell).astype(np.int32))
    nd = int(np.ceil((t1 - t0) / DAY - 1e-9))
    ws.cal_true = w.cal_true[2 * day0:2 * (day0 + nd)]
    ws.cal_start = w.cal_start[2 * day0:2 * (day0 + nd)]
    # knot intervals [l0, l1] hold the slice; coefficients l0 - 3 .. l1
    l0 = int(np.searchsorted(w.knots, t0, side="right") - 1)
    l1 = int(np.searchsorted(w.knots, t1, side="left") - 1)
    ws.knots = np.ascontiguousarray(w.knots[l0 - 3:l1 + 5])
    ws.att_true = w.att_true[l0 - 3:l1 + 1]
    ws.att_start = w.att_start[l0 - 3:l1 + 1]
    ws.consts = dict(w.consts, t_beg=float(ws.knots[3]), t_end=float(ws.knots[-4]))
    return ws


def cpu_baseline(w, days, days_1t, log_fn):
    """The oracle's iteration (S[AC] and the frame rotator) timed on time
    slices of the same workload: all threads of the host share on `days` days
    of observations, one thread on `days_1t` days."""
    import ctypes

    import oracle
    oracle.build()
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    gomp = ctypes.CDLL("libgomp.so.1")
    out = {}
    n_days = int(np.ceil((w.consts["t_end"] - w.consts["t_beg"]) / 86400.0 - 1e-9))
    for nt, nd in ((threads, days), (1, days_1t)):
        day0 = n_days // 2
        ws = time_slice(w, day0, nd)
        eta = oracle.observed_field_angles(ws)
        pr = oracle.problem_from_world(ws, eta, state="start")
        gomp.omp_set_num_threads(nt)
        t0 = time.perf_counter()
        pr.iterate(s_ref=ws.src_true)
        dt = time.perf_counter() - t0
        gomp.omp_set_num_threads(threads)
        out[nt] = (ws.n_obs / dt, ws.n_obs, ws.src_true.shape[0], ws.n_att, dt, nd)
        log_fn(f"cpu baseline: {nt} threads, {nd} days ({ws.n_obs} obs, {ws.src_true.shape[0]} sources), "
               f"{dt:.1f} s, {ws.n_obs / dt:.3g} obs/s")
    model, ram = host_description()
    v, n_obs, n_src, n_att, dt, nd = out[threads]
    v1, n1, s1, a1, dt1, nd1 = out[1]
    return {"value": v, "unit": "obs/s", "cores": threads, "kind": "oracle",
            "sample": f"one S[AC] + frame iteration of the oracle over the observations of {nd} whole days in mid-"
                      f"mission ({n_obs} obs, {n_src} sources, {n_att} attitude coefficients), {dt:.1f} s",
            "one_thread": {"value": v1, "sample": f"{nd1} day(s): {n1} obs, {s1} sources, {dt1:.1f} s"},
            "cpu_model": model, "host_ram_gib": ram}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="gaia5",
                    help="gaia5: 2M sources, 5 yr, robust (the largest single-GPU configuration); gaia1: 1M "
                         "sources, 1 yr")
    ap.add_argument("--seg-len", type=int, default=None)
    ap.add_argument("--cpu-days", type=int, default=48, help="days of observations the oracle iterates over "
                                                            "(all threads of the host share)")
    ap.add_argument("--cpu-days-1t", type=int, default=6, help="... and on one thread")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64",
                    help="mixed: FP32 partials and compensated FP32 normal-equation sums")
    ap.add_argument("--scheme", choices=("si", "cg"), default="si",
                    help="si: one simple S[AC] iteration per step; cg: one conjugate-gradient step per step "
                         "(cycles of 40 iterations; an iteration is one pass of the blocks plus p'N p)")
    ap.add_argument("--ac", action="store_true",
                    help="add one across-scan observation per transit (cell -1) to the workload")
    ap.add_argument("--geo", action="store_true",
                    help="the large-scale geometric calibration (3 coefficients per cell and CCD) in place of one "
                         "offset per cell; with --ac the across-scan term too; no CPU baseline")
    ap.add_argument("--geo-small", action="store_true",
                    help="with --geo: the small-scale along-scan term too (one value per CCD, 30-day interval and "
                         "pixel column)")
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
    if args.geo:
        over["geo_cal"] = True
        over["geo_ac"] = args.ac            # with across-scan records: the AC term too
        over["geo_small"] = args.geo_small
        args.no_cpu_baseline = True
    wname = (args.workload + ("+ac" if args.ac else "") + ("+geo" if args.geo else "")
             + ("+small" if args.geo and args.geo_small else ""))
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
    if args.geo:
        agis.agis_load_geometry(ctx, w.ccd, w.mu, int(w.consts["geo_ccds"]), w.ac_cell,
                                int(w.consts.get("geo_ac_cells", 0)) if w.ac_cell is not None else 0,
                                small_days=int(w.consts.get("geo_small_days", 0)))
        agis.agis_set_geo_calibration(ctx, geo_coefficients(w, "true"))
    R = agis.agis_residuals(ctx)                   # = c_true - eta_true (plus the true geometric terms)
    eta_obs = -R + w.eps
    del R, zeros
    if args.no_cpu_baseline:
        w.eps = w.eta_nominal = None           # not needed any more
    log("observed field angles computed")
    agis.agis_load_observations(ctx, w.t, eta_obs, w.sigma, w.src, w.fov, w.cell, n_src, w.n_cells)
    agis.agis_set_sources(ctx, w.src_start)
    agis.agis_set_attitude(ctx, w.att_start)
    agis.agis_set_calibration(ctx, w.cal_start)
    if args.geo:
        agis.agis_load_geometry(ctx, w.ccd, w.mu, int(w.consts["geo_ccds"]), w.ac_cell,
                                int(w.consts.get("geo_ac_cells", 0)) if w.ac_cell is not None else 0,
                                small_days=int(w.consts.get("geo_small_days", 0)))
        agis.agis_set_geo_calibration(ctx, geo_coefficients(w, "start"))
    agis.agis_set_frame_reference(ctx, w.src_true)
    sz = agis.agis_problem_size(ctx)
    log(f"store built: {sz}")

    s_group = agis.agis_autotune(ctx)
    tuning = agis.agis_get_tuning(ctx)
    log(f"autotuned: {tuning}")

    def step():
        if args.scheme == "cg":
            agis.agis_cg_iterate(ctx, 1, 40, stats=False)
        else:
            agis.agis_iterate(ctx, 1, stats=False)

    for i in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} done")
    kt = {k: [] for k in ("source_update", "ac_pass", "band_solve", "calib_solve", "frame", "excess_noise")}
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

    # the dominant kernel (timer) and its roofline: per-unit algorithmic
    # flops and bytes times the units one launch processes, over the
    # launch's average device time
    robust = bool(w.spec.robust)
    K = w.n_att - 3
    per_launch = {
        "source_update": ((S_ROBUST_FLOPS_PER_OBS if robust else S_FLOPS_PER_OBS) * w.n_obs,
                          BYTES_PER_OBS * w.n_obs + BYTES_PER_SOURCE * n_src),
        "ac_pass": (AC_FLOPS_PER_OBS * w.n_obs,
                    BYTES_PER_OBS * w.n_obs + BYTES_PER_SOURCE * n_src + BYTES_PER_COEF * w.n_att),
        "excess_noise": (EPS_FLOPS_PER_OBS * w.n_obs, BYTES_PER_OBS * w.n_obs + BYTES_PER_SOURCE * n_src),
    }
    dom = max((k for k in per_launch if kavg[k] > 0), key=lambda k: kavg[k])
    alg_flops, alg_bytes = per_launch[dom]
    sec = kavg[dom] * 1e-3
    tfs = alg_flops / sec / 1e12
    sym = "source_update_robust" if dom == "source_update" and robust else dom
    traffic = measured_traffic(sym, wname, args.precision)
    roofline = {"kernel": sym, "bound": "alu", "achieved": round(tfs, 2), "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(tfs / FP64_PEAK_TFLOPS, 4), "traffic": traffic,
                "alg_flops_per_launch": alg_flops, "alg_bytes_per_launch": alg_bytes,
                "alg_hbm_GBs": round(alg_bytes / sec / 1e9, 1),
                "alg_hbm_frac": round(alg_bytes / sec / 1e9 / HBM_PEAK_GBS, 4), "avg_ms": kavg[dom],
                "per_kernel_frac": {k: round(f / (kavg[k] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)
                                    for k, (f, _) in per_launch.items() if kavg[k] > 0}}

    cpu = None
    if not args.no_cpu_baseline:
        agis.agis_destroy(ctx)
        ctx = None
        del eta_obs
        cpu = cpu_baseline(w, args.cpu_days, args.cpu_days_1t, log)

    out = {"metric": "obs/s per AGIS iteration", "value": value, "unit": "obs/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if args.precision == "fp64" else "f64 model, f32 partials and sums", "data": "synthetic",
           "config": {**workload_description(wname, w), "lanes_per_source": s_group,
                      **({"robust_s_path": ["hbm columns", "rows in hbm, solves in lds", "all in lds",
                                         "rows in registers"][
                          tuning["robust_s_path"]],
                          "inner_rounds": ["records re-read each round", "32 lanes per source, first 8 records in "
                                           "registers", "64 lanes per source, first 8 records in registers"][
                              tuning["irls_cache"]]} if w.spec.robust else {}),
                      **({"scheme": "conjugate gradients"} if args.scheme == "cg" else {})},
           "kernel_ms": kavg, "roofline": roofline,
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)
    if ctx is not None:
        agis.agis_destroy(ctx)


if __name__ == "__main__":
    main()
