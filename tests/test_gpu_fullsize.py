"""Parity at the full size of the 1M-source / 1-year / 9-CCD workload
(gaia1, 160,919,875 observations), on sampled outputs.

The GPU updates the whole problem with the same launchers the benchmark
times.  The oracle computes the sampled outputs one by one, each from a
sub-world that holds exactly the observations the output depends on:
residuals of sampled observations; the S update of sampled sources (all of
their observations, Sect. 5.1); the A update of sampled attitude segments
(the observations of the segment's data range with its overlap,
Sect. 5.2.2); the C update of sampled days (both cells, all observations of
the day, Sect. 5.3).  The criterion is the one of the small-world parity
tests: within max(1e-3 uas, the FP64 rounding floor) of the
extended-precision oracle, and per component no less accurate than the FP64
oracle.  The observed field angles come from the oracle's model.  Every
test runs on gaia1 and on gaia1 with one across-scan record per transit
(17.9M more records, cell -1).
"""
import types

import numpy as np
import pytest

import synth.configs as C
from test_gpu_parity import TOL_UAS, agis_mod, check_floor, fp64_floor  # noqa: F401

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

OBS_FIELDS = ("t", "src", "fov", "cell", "sigma", "eps", "ccd", "mu", "ac_cell")


def subworld(w, idx):
    """The world restricted to the observations idx (sorted); sources,
    attitude, calibration, knots and constants unchanged."""
    sub = types.SimpleNamespace(**{k: v for k, v in vars(w).items() if k not in OBS_FIELDS})
    for k in OBS_FIELDS:
        v = getattr(w, k, None)
        setattr(sub, k, None if v is None else v[idx])
    sub.n_obs, sub.n_att, sub.n_cells = idx.size, w.n_att, w.n_cells
    return sub


@pytest.fixture(scope="module", params=["gaia1", "gaia1+ac"])
def full(oracle_lib, agis_mod, request):
    w = C.make("gaia1", ac_obs=request.param.endswith("+ac"))
    eta = oracle_lib.observed_field_angles(w)
    print(f"{request.param}: {w.n_obs} observations, {w.src_true.shape[0]} sources, {w.n_att} coefficients", flush=True)
    ctx = agis_mod.agis_create(w.consts, w.knots)
    agis_mod.agis_load_observations(ctx, w.t, eta, w.sigma, w.src, w.fov, w.cell, w.src_true.shape[0], w.n_cells)
    yield w, eta, ctx
    agis_mod.agis_destroy(ctx)


def _start(agis, ctx, w):
    agis.agis_set_sources(ctx, w.src_start)
    agis.agis_set_attitude(ctx, w.att_start)
    agis.agis_set_calibration(ctx, w.cal_start)


def test_fullsize_residuals(agis_mod, oracle_lib, full):
    w, eta, ctx = full
    _start(agis_mod, ctx, w)
    R = agis_mod.agis_residuals(ctx)
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(w.n_obs, 4096, replace=False))
    sub = subworld(w, idx)
    Ro = oracle_lib.problem_from_world(sub, eta[idx], state="start").observe()["R"]
    d = R[idx] - Ro
    print(f"residuals at {idx.size} sampled observations: max |GPU - oracle| {np.abs(d).max():.2e} rad, "
          f"rms {np.sqrt(np.mean(d * d)):.2e} rad")
    assert np.sqrt(np.mean(d * d)) < 1.5e-16 and np.abs(d).max() < 1e-15


def test_fullsize_source_update(agis_mod, oracle_lib, full):
    w, eta, ctx = full
    _start(agis_mod, ctx, w)
    agis_mod.agis_source_update(ctx)
    G = agis_mod.agis_get_sources(ctx, w.src_true.shape[0])
    rng = np.random.default_rng(11)
    pick = np.sort(rng.choice(w.src_true.shape[0], 2000, replace=False))
    idx = np.flatnonzero(np.isin(w.src, pick))
    sub = subworld(w, idx)

    def run(pr):
        _, _, de = pr.source_update()
        run.defect = de
        return pr.s.copy(), pr.a.copy(), pr.c.copy()

    X, O, tol = fp64_floor(oracle_lib, sub, eta[idx], run)
    run(oracle_lib.problem_from_world(sub, eta[idx], state="start"))
    mask = np.zeros(w.src_true.shape[0], bool)
    mask[pick] = True
    mask &= run.defect == 0
    assert mask.sum() > 1900
    name = "gaia1+ac" if (w.cell < 0).any() else "gaia1"
    dg = check_floor(f"S update, {pick.size} sampled sources of {name} ({idx.size} observations)", X[0], O[0], G,
                     tol[0], 0, mask=mask)
    assert np.mean(np.abs(dg) <= TOL_UAS) > 0.95


def test_fullsize_attitude_calibration_update(agis_mod, oracle_lib, full):
    """One A/C pass and solve at the start values (s, a, c)."""
    w, eta, ctx = full
    _start(agis_mod, ctx, w)
    agis_mod.agis_attitude_calibration_update(ctx)
    Ga = agis_mod.agis_get_attitude(ctx, w.n_att)
    Gc = agis_mod.agis_get_calibration(ctx, w.n_cells)
    knots = w.knots
    S, L = int(w.consts["seg_len"]), int(w.consts["seg_overlap"])
    n_iv = knots.size - 7
    n_seg = (n_iv + S - 1) // S
    rng = np.random.default_rng(13)
    for K in sorted(rng.choice(np.arange(1, n_seg - 1), 3, replace=False)):
        # observations of the segment's intervals and its overlap, with a margin
        lo_iv, hi_iv = max(K * S - L - 4, 0), min((K + 1) * S + L + 4, n_iv)
        t_lo, t_hi = knots[3 + lo_iv], knots[3 + hi_iv]
        idx = np.flatnonzero((w.t >= t_lo) & (w.t < t_hi))
        sub = subworld(w, idx)
        rng_kept = {}

        def run(pr, K=K):
            d, de, lo, hi = pr.attitude_segment(int(K))
            rng_kept["lo"], rng_kept["hi"] = lo, hi
            a = pr.a.copy()
            a[lo:hi + 1] += d[lo:hi + 1]
            return pr.s.copy(), a, pr.c.copy()

        X, O, tol = fp64_floor(oracle_lib, sub, eta[idx], run)
        lo, hi = rng_kept["lo"], rng_kept["hi"]
        assert hi - lo + 1 == S
        sl = slice(lo, hi + 1)
        rd = check_floor(f"A update, segment {K} of {n_seg} (coefficients {lo}..{hi}, {idx.size} observations)",
                         X[1][sl], O[1][sl], Ga[sl], tol[1][sl], 1)
        assert np.mean(np.abs(rd[:, 2]) <= TOL_UAS) > 0.99
    # calibration of two sampled days (cells 2 day, 2 day + 1)
    for day in sorted(rng.choice(np.arange(1, w.n_cells // 2 - 1), 2, replace=False)):
        cells = (2 * day, 2 * day + 1)
        idx = np.flatnonzero((w.cell == cells[0]) | (w.cell == cells[1]))
        sub = subworld(w, idx)

        def run(pr):
            pr.calibration_update()          # applies its update to pr.c
            return pr.s.copy(), pr.a.copy(), pr.c.copy()

        X, O, tol = fp64_floor(oracle_lib, sub, eta[idx], run)
        sel = np.array(cells)
        check_floor(f"C update, day {day} ({idx.size} observations)",
                    X[2][sel], O[2][sel], Gc[sel], tol[2][sel], 2)
