"""Training and evaluation of the learned extrapolation (driver over the C ABI).

The plain simple iteration (S[AC] and the frame rotator) is run on synthetic
worlds; every ``m`` iterations the library records the parameter change as
one "update" of each source and attitude coefficient.  From the fourth record
on, the library's features (the last four updates normalised by their RMS s,
plus two descriptors) are paired with the target (x_{j+H} - x_j) / s: where
the plain trajectory will be H records later.  The networks output four
coefficients that mix the unit's recorded updates; training fits the mixture
to the target.  A finite horizon keeps the
targets bounded (towards the limit they grow like rho / (1 - rho) with the
slowest contraction rho of the iteration, close to 1).  The two MLPs are
trained on the GPU by the library's own kernels (Adam, the rate lowered in
three stages).  The learned solve tries the candidate x + sum_k c_k u_k
after every record from the fourth one on, through the library's gated
step (one iteration from the candidate against one plain iteration; the
history restarts when the candidate is kept).

Agreement with a reference (the convergence criterion): the largest over the
classes alpha*, delta, parallax, mu_alpha*, mu_delta, the three attitude
rotation axes and the calibration of the RMS difference, in uas.

Usage (GPU):  python -m paper_1112_4139_amd.learned [--world tiny] ...
prints one JSON line with iterations and wall time to agreement.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import agis

UAS = np.pi / 180 / 3600 * 1e-6


def problem(name, seed, precision=agis.AGIS_FP64, **over):
    """A synthetic world (seeded) and a context at its start values; the
    observed field angles are the library's model at the truth plus the
    world's noise."""
    import synth.configs as C
    w = C.make(name, seed_truth=seed, seed_noise=seed + 100, seed_start=seed + 200, **over)
    ctx = agis.agis_create(w.consts, w.knots, precision=precision)
    n_src = w.src_true.shape[0]
    agis.agis_load_observations(ctx, w.t, np.zeros(w.n_obs), w.sigma, w.src, w.fov, w.cell, n_src, w.n_cells)
    agis.agis_set_sources(ctx, w.src_true)
    agis.agis_set_attitude(ctx, w.att_true)
    agis.agis_set_calibration(ctx, w.cal_true)
    eta = -agis.agis_residuals(ctx) + w.eps
    agis.agis_load_observations(ctx, w.t, eta, w.sigma, w.src, w.fov, w.cell, n_src, w.n_cells)
    agis.agis_set_sources(ctx, w.src_start)
    agis.agis_set_attitude(ctx, w.att_start)
    agis.agis_set_calibration(ctx, w.cal_start)
    agis.agis_set_frame_reference(ctx, w.src_true)
    return w, ctx


def state(ctx, w):
    return (agis.agis_get_sources(ctx, w.src_true.shape[0]), agis.agis_get_attitude(ctx, w.n_att),
            agis.agis_get_calibration(ctx, w.n_cells))


def _qmul(a, b):
    ax, ay, az, aw = a.T
    bx, by, bz, bw = b.T
    return np.stack([aw * bx + ax * bw + ay * bz - az * by, aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw, aw * bw - ax * bx - ay * by - az * bz], axis=1)


def disagreement(x, ref):
    """Largest per-class RMS difference (uas) between states x and ref."""
    ds = x[0] - ref[0]
    ds[:, 0] = ((ds[:, 0] + np.pi) % (2 * np.pi) - np.pi) * np.cos(ref[0][:, 1])
    d = _qmul(ref[1] * np.array([-1, -1, -1, 1.0]), x[1])
    d /= np.linalg.norm(d, axis=1)[:, None]
    rot = 2 * d[:, :3] * np.sign(d[:, 3:4])
    rms = list(np.sqrt(np.mean(ds * ds, axis=0))) + list(np.sqrt(np.mean(rot * rot, axis=0)))
    rms.append(np.sqrt(np.mean((x[2] - ref[2]) ** 2)))
    return max(rms) / UAS


def targets(x_ref, x, which):
    """(x_ref - x) in the units of the recorded updates (alpha*: d alpha
    cos delta at x; coefficients: component differences)."""
    if which == 0:
        d = x_ref[0] - x[0]
        d[:, 0] = ((d[:, 0] + np.pi) % (2 * np.pi) - np.pi) * np.cos(x[0][:, 1])
        return d
    return x_ref[1] - x[1]


def collect(ctx, w, m, n_macro, horizon, every=1):
    """Training samples of one plain trajectory of n_macro records: features
    and scales at records 4 .. n_macro - horizon (every `every`-th), targets
    towards the state `horizon` records later."""
    agis.agis_learned_reset(ctx)
    feats, states = {}, {}
    for j in range(1, n_macro + 1):
        agis.agis_iterate(ctx, m, stats=False)
        agis.agis_learned_record(ctx)
        if j >= 4 and (j - 4) % every == 0 and j + horizon <= n_macro:
            feats[j] = (agis.agis_learned_features(ctx, 0), agis.agis_learned_features(ctx, 1))
            states[j] = state(ctx, w)
        if (j - horizon) in feats:
            states[j] = state(ctx, w)
    data = []
    for which in (0, 1):
        X, T = [], []
        for j, f in feats.items():
            X.append(f[which][0])
            T.append((targets(states[j + horizon], states[j], which) /
                      np.maximum(f[which][1], 1e-300)[:, None]).astype(np.float32))
        X, T = np.concatenate(X), np.concatenate(T)
        ok = np.isfinite(T).all(axis=1) & np.isfinite(X).all(axis=1)
        data.append((X[ok], T[ok]))
    return data


def solve_cg(ctx, w, n_iter, ref, tol=1.0, log=None, restart=40):
    """Conjugate gradients (Sect. 4.7) in cycles of restart + 1 evaluations
    (one at the cycle's start point, then restart iterations), until the
    disagreement with ref drops below tol uas.  The frame rotator, which CG
    applies at each cycle start, is applied before each check, as the simple
    iteration applies it after every iteration.  Returns the evaluations
    (each one pass of the three blocks, like one S[AC] iteration), the wall
    time of the library calls, the cycles and breakdowns, and the median
    step length."""
    it = 0
    t_gpu = 0.0
    alphas = []
    cycles = breakdowns = 0
    dis = disagreement(state(ctx, w), ref)
    while it < n_iter and dis > tol:
        t0 = time.perf_counter()
        st = agis.agis_cg_iterate(ctx, restart + 1, restart)
        agis.agis_frame_apply(ctx, agis.agis_frame_fit(ctx))
        t_gpu += time.perf_counter() - t0
        it += restart + 1
        cycles += 1
        breakdowns += sum(x["breakdown"] for x in st)
        alphas += [x["alpha"] for x in st if x["alpha"] > 0]
        dis = disagreement(state(ctx, w), ref)
        if log and cycles % 20 == 0:
            log(f"cg it {it}: disagreement {dis:.3f} uas, breakdowns {breakdowns}")
    return dict(iterations=it if dis <= tol else None, seconds=t_gpu, cycles=cycles, breakdowns=breakdowns,
                disagreement=dis, chi2=agis.agis_chi2(ctx),
                median_alpha=float(np.median(alphas)) if alphas else None)


def solve(ctx, w, m, n_iter, ref, mode, tol=1.0, log=None, asi_stride=16, asi_lambda_max=0.99, cg_restart=40):
    """Iterate in blocks of m iterations until the disagreement with ref
    drops below tol uas.  mode "plain": the simple iteration alone; "asi":
    after each block from the third record of a history on, the accelerated
    step of Sect. 4.7 (factor lambda / (1 - lambda) on the newest update);
    "learned": after each block from the fourth record on, the gated learned
    step.  Returns the S[AC] iterations (the gate's two included), the wall
    time of the library calls, the accept/reject counts (asi: steps taken
    and skipped) and the median q_cand / q_plain of the gate, or the median
    lambda of the accelerated steps."""
    learned = mode == "learned"
    if mode == "cg":
        return solve_cg(ctx, w, n_iter, ref, tol=tol, log=log, restart=cg_restart)
    agis.agis_learned_reset(ctx)
    acc = rej = 0
    it = 0
    count = 0                       # records since the history started
    t_gpu = 0.0
    ratios = []
    blocks = 0
    dis = disagreement(state(ctx, w), ref)
    while it < n_iter and dis > tol:
        t0 = time.perf_counter()          # every library call below returns after its device work
        if learned:
            # m iterations, a record and (from the fourth record on) the gated step
            r = agis.agis_iterate_learned(ctx, 1, m)[0]
            it += r["iterations"]
            if r["gated"]:
                ratios.append(r["q_candidate"] / r["q_plain"])
                acc += int(r["accepted"])
                rej += int(not r["accepted"])
            t_gpu += time.perf_counter() - t0
            blocks += 1
            dis = disagreement(state(ctx, w), ref)
            if log and blocks % 20 == 0:
                log(f"{mode} it {it}: disagreement {dis:.3f} uas, accepted {acc} rejected {rej}")
            continue
        agis.agis_iterate(ctx, m, stats=False)
        agis.agis_learned_record(ctx)
        count += 1
        it += m
        if mode == "asi" and count >= 3:
            r = agis.agis_asi_step(ctx, asi_stride, asi_lambda_max)
            ratios.append(r["lam"])
            if r["factor"] > 0:
                acc += 1
                count = 0
            else:
                rej += 1
        t_gpu += time.perf_counter() - t0
        blocks += 1
        dis = disagreement(state(ctx, w), ref)
        if log and blocks % 20 == 0:
            log(f"{mode} it {it}: disagreement {dis:.3f} uas, "
                f"accepted {acc} rejected {rej}")
    return dict(iterations=it if dis <= tol else None, seconds=t_gpu, accepted=acc, rejected=rej,
                disagreement=dis, chi2=agis.agis_chi2(ctx),
                median_ratio=float(np.median(ratios)) if ratios else None)


def errors_to_truth(ctx, w):
    """Per-class RMS error of the current state against the world's true
    parameters (uas): alpha*, delta, parallax, mu_alpha*, mu_delta, the three
    attitude axes, calibration."""
    x = state(ctx, w)
    ds = x[0] - w.src_true
    ds[:, 0] = ((ds[:, 0] + np.pi) % (2 * np.pi) - np.pi) * np.cos(w.src_true[:, 1])
    d = _qmul(w.att_true * np.array([-1, -1, -1, 1.0]), x[1])
    d /= np.linalg.norm(d, axis=1)[:, None]
    rot = 2 * d[:, :3] * np.sign(d[:, 3:4])
    out = list(np.sqrt(np.mean(ds * ds, axis=0))) + list(np.sqrt(np.mean(rot * rot, axis=0)))
    out.append(np.sqrt(np.mean((x[2] - w.cal_true) ** 2)))
    return [float(v / UAS) for v in out]


def precision_run(world, seed, n, mode, restart=40, log=None):
    """The same scheme (plain or cg) for n block passes in FP64 and in mixed
    precision from the same start: each one's per-class RMS error to the
    truth and the per-class RMS difference between the two final states
    (uas), the measure of whether both reach the same fixed point."""
    states, out = {}, {}
    for name, prec in (("fp64", agis.AGIS_FP64), ("mixed", agis.AGIS_MIXED)):
        w, ctx = problem(world, seed, precision=prec)
        t0 = time.perf_counter()
        if mode == "cg":
            agis.agis_cg_iterate(ctx, n, restart, stats=False)
            agis.agis_frame_apply(ctx, agis.agis_frame_fit(ctx))
        else:
            agis.agis_iterate(ctx, n, stats=False)
        out[name] = {"seconds": time.perf_counter() - t0, "rms_error_uas": errors_to_truth(ctx, w)}
        states[name] = state(ctx, w)
        if log:
            log(f"{mode} {name}: {out[name]}")
        agis.agis_destroy(ctx)
    a, b = states["fp64"], states["mixed"]
    ds = b[0] - a[0]
    ds[:, 0] = ((ds[:, 0] + np.pi) % (2 * np.pi) - np.pi) * np.cos(a[0][:, 1])
    d = _qmul(a[1] * np.array([-1, -1, -1, 1.0]), b[1])
    d /= np.linalg.norm(d, axis=1)[:, None]
    rot = 2 * d[:, :3] * np.sign(d[:, 3:4])
    diff = list(np.sqrt(np.mean(ds * ds, axis=0))) + list(np.sqrt(np.mean(rot * rot, axis=0)))
    diff.append(np.sqrt(np.mean((b[2] - a[2]) ** 2)))
    out["mixed_minus_fp64_rms_uas"] = [float(v / UAS) for v in diff]
    return out


def budget_run(world, seed, n, modes, m=50, restart=40, log=None):
    """Each scheme for the same number of block passes n from the world's
    start values (with the frame rotator): per-class RMS error to the truth
    and the wall time of the library calls.  No reference solution is
    needed, so this runs at any workload size."""
    out = {}
    for mode in modes:
        w, ctx = problem(world, seed)
        t0 = time.perf_counter()
        if mode == "plain":
            agis.agis_iterate(ctx, n, stats=False)
        elif mode == "cg":
            agis.agis_cg_iterate(ctx, n, restart, stats=False)
            agis.agis_frame_apply(ctx, agis.agis_frame_fit(ctx))
        elif mode == "asi":
            agis.agis_learned_reset(ctx)
            count = done = 0
            while done < n:
                k = min(m, n - done)
                agis.agis_iterate(ctx, k, stats=False)
                done += k
                agis.agis_learned_record(ctx)
                count += 1
                if count >= 3 and agis.agis_asi_step(ctx, 16, 0.99)["factor"] > 0:
                    count = 0
        else:
            raise ValueError(f"budget runs take plain, asi and cg, not {mode}")
        sec = time.perf_counter() - t0
        out[mode] = {"evaluations": n, "seconds": sec, "rms_error_uas": errors_to_truth(ctx, w)}
        if log:
            log(f"{mode}: {out[mode]}")
        agis.agis_destroy(ctx)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--world", default="tiny")
    ap.add_argument("--train-seeds", default="1,2,3,4")
    ap.add_argument("--eval-seed", type=int, default=0)
    ap.add_argument("--m", type=int, default=50, help="iterations per recorded update")
    ap.add_argument("--macro", type=int, default=None, help="records per training trajectory (horizon + 100)")
    ap.add_argument("--horizon", type=int, default=160, help="records ahead that the networks predict")
    ap.add_argument("--ref-eval", type=int, default=200000, help="iterations of the evaluation reference run")
    ap.add_argument("--steps", type=int, default=12000, help="Adam steps per network (three rate stages)")
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--max-iter", type=int, default=160000)
    ap.add_argument("--tol", type=float, default=1.0)
    ap.add_argument("--modes", default="plain,asi,learned", help="solves to compare (plain, asi, learned, cg)")
    ap.add_argument("--cg-restart", type=int, default=40, help="CG iterations per cycle")
    ap.add_argument("--ref-file", default=None, help="npz cache of the evaluation reference (read if it matches)")
    ap.add_argument("--compare-precisions", action="store_true",
                    help="with --budget: run the (single) mode in FP64 and in mixed precision and report the "
                         "difference of the final states")
    ap.add_argument("--budget", type=int, default=0,
                    help="instead of the convergence study: run each of --modes (plain, asi, cg) for this many "
                         "block passes and report the errors to the truth")
    args = ap.parse_args(argv)
    if args.macro is None:
        args.macro = args.horizon + 100

    def log(msg):
        print(f"[learned {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)

    if args.budget and args.compare_precisions:
        out = precision_run(args.world, args.eval_seed, args.budget, args.modes.split(",")[0],
                            restart=args.cg_restart, log=log)
        print(json.dumps({"world": args.world, "seed": args.eval_seed, "budget": args.budget,
                          "mode": args.modes.split(",")[0], **out}), flush=True)
        return
    if args.budget:
        out = budget_run(args.world, args.eval_seed, args.budget, args.modes.split(","), m=args.m,
                         restart=args.cg_restart, log=log)
        print(json.dumps({"world": args.world, "seed": args.eval_seed, "budget": args.budget, **out}), flush=True)
        return

    data = [[], []]
    ctx_train = None
    train = "learned" in args.modes.split(",")
    for seed in [int(x) for x in args.train_seeds.split(",") if x and train]:
        w, ctx = problem(args.world, seed)
        d = collect(ctx, w, args.m, args.macro, args.horizon)
        for which in (0, 1):
            data[which].append(d[which])
        log(f"seed {seed}: {d[0][0].shape[0]} source and {d[1][0].shape[0]} coefficient samples")
        if ctx_train is None:
            ctx_train = ctx
        else:
            agis.agis_destroy(ctx)
    weights, losses = [], []
    for which in (0, 1) if train else ():
        X = np.concatenate([d[0] for d in data[which]])
        T = np.concatenate([d[1] for d in data[which]])
        agis.agis_mlp_init(ctx_train, which, 1234 + which)
        t0 = time.perf_counter()
        q = args.steps // 4
        stages = [(2 * q, args.lr), (q, args.lr / 4), (args.steps - 3 * q, args.lr / 16)]
        loss = np.concatenate([agis.agis_mlp_train(ctx_train, which, X, T, n, args.batch, lr, seed=99 + which)
                               for n, lr in stages if n > 0])
        log(f"net {which}: {X.shape[0]} samples, loss {loss[:20].mean():.4g} -> {loss[-200:].mean():.4g} "
            f"({time.perf_counter() - t0:.1f} s)")
        weights.append(agis.agis_mlp_get_weights(ctx_train, which))
        losses.append((float(loss[:20].mean()), float(loss[-200:].mean())))
    if ctx_train is not None:
        agis.agis_destroy(ctx_train)

    w, ctx = problem(args.world, args.eval_seed)
    cached = None
    if args.ref_file and os.path.exists(args.ref_file):
        z = np.load(args.ref_file)
        if (int(z["iterations"]) == args.ref_eval and str(z["world"]) == args.world
                and int(z["seed"]) == args.eval_seed):
            cached = (z["s"], z["a"], z["c"]), float(z["chi2"])
            log(f"evaluation reference from {args.ref_file}")
    if cached is None:
        done = 0
        while done < args.ref_eval:
            n = min(10000, args.ref_eval - done)
            agis.agis_iterate(ctx, n, stats=False)
            done += n
            log(f"evaluation reference: {done} of {args.ref_eval} plain iterations")
        ref, chi2_ref = state(ctx, w), agis.agis_chi2(ctx)
        if args.ref_file:
            np.savez(args.ref_file, s=ref[0], a=ref[1], c=ref[2], chi2=chi2_ref, iterations=args.ref_eval,
                     world=args.world, seed=args.eval_seed)
    else:
        ref, chi2_ref = cached
    agis.agis_destroy(ctx)
    out = {}
    for mode in args.modes.split(","):
        w, ctx = problem(args.world, args.eval_seed)
        for which in range(len(weights)):
            agis.agis_mlp_load(ctx, which, weights[which])
        out[mode] = solve(ctx, w, args.m, args.max_iter, ref, mode, tol=args.tol, log=log,
                          cg_restart=args.cg_restart)
        log(f"{mode}: {out[mode]}")
        agis.agis_destroy(ctx)
    print(json.dumps({"world": args.world, "train_seeds": args.train_seeds, "eval_seed": args.eval_seed,
                      "m": args.m, "horizon": args.horizon, "tol_uas": args.tol, "ref_iterations": args.ref_eval,
                      "chi2_ref": chi2_ref, "train_loss": losses, **out}), flush=True)


if __name__ == "__main__":
    main()
