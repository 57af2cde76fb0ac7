"""Parity at the full size of the robust 2M-source / 5-year / 9-CCD workload
(gaia5, ~1.6G observations, 1% outliers), on sampled outputs.

The GPU updates the whole problem with the launchers the benchmark times
(the robust source update with its inner iteration, the excess attitude
noise per bucket, the robustly weighted A/C pass and solves).  The oracle
computes sampled outputs one by one, each from a sub-world that holds
exactly the observations the output depends on: the robust S update of 1,000
random sources and of the 50 with the most observations (Sect. 5.1.2); the
excess attitude noise eps_a^2 of sampled buckets (eq e09, every observation
of the bucket's knot intervals); the robust A update of sampled segments
(Sect. 5.2.2, 5.2.5) and the C update of sampled days (Sect. 5.3), both with
the excess noise the GPU used.  Criterion: as in the small-world parity
tests, within max(1e-3 uas, the FP64 rounding floor) of the
extended-precision oracle, and per component no less accurate than the FP64
oracle; eps_a^2 to the rounding of R^2.  The observed field angles come from
the oracle's model (in chunks).
"""
import numpy as np
import pytest

import synth
import synth.configs as C
from test_gpu_fullsize import subworld
from test_gpu_parity import TOL_UAS, agis_mod, check_floor, fp64_floor  # noqa: F401

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1200)]

UAS = synth.UAS


@pytest.fixture(scope="module")
def full5(oracle_lib, agis_mod):
    w = C.make("gaia5")
    print(f"gaia5: {w.n_obs} observations, {w.src_true.shape[0]} sources, {w.n_att} coefficients", flush=True)
    eta = oracle_lib.observed_field_angles(w)
    print("gaia5: observed field angles from the oracle's model", flush=True)
    ctx = agis_mod.agis_create(w.consts, w.knots)
    agis_mod.agis_load_observations(ctx, w.t, eta, w.sigma, w.src, w.fov, w.cell, w.src_true.shape[0], w.n_cells)
    w.eta_nominal = None                        # not needed; frees host memory
    yield w, eta, ctx
    agis_mod.agis_destroy(ctx)


def _start(agis, ctx, w):
    agis.agis_set_sources(ctx, w.src_start)
    agis.agis_set_attitude(ctx, w.att_start)
    agis.agis_set_calibration(ctx, w.cal_start)
    nb = (w.n_att - 3 + w.consts["eps_bucket"] - 1) // w.consts["eps_bucket"]
    agis.agis_set_excess_noise(ctx, np.full(3 * nb, w.consts["eps_a_init"] ** 2))   # AL, ACP, ACF
    return nb


def _bucket_members(w, buckets, B, K, chunk=1 << 27):
    """Indices of the observations of each sampled bucket's knot intervals
    (the last bucket closed at its right end): one pass of the observation
    times against the buckets' sorted edges, in chunks that print progress."""
    knots = w.knots
    lo = knots[3 + buckets * B]
    hi = knots[3 + np.minimum(buckets * B + B, K)].copy()
    hi[buckets * B + B >= K] = np.nextafter(hi[buckets * B + B >= K], np.inf)
    edges = np.ravel(np.column_stack([lo, hi]))
    assert np.all(np.diff(edges) >= 0)
    found_idx, found_b = [], []
    for c0 in range(0, w.n_obs, chunk):
        pos = np.searchsorted(edges, w.t[c0:c0 + chunk], side="right")
        inside = np.flatnonzero(pos & 1)
        found_idx.append(inside + c0)
        found_b.append((pos[inside] - 1) // 2)
        print(f"bucket membership: {min(c0 + chunk, w.n_obs)} of {w.n_obs} observations", flush=True)
    idx, which = np.concatenate(found_idx), np.concatenate(found_b)
    order = np.argsort(which, kind="stable")
    idx, which = idx[order], which[order]
    cut = np.searchsorted(which, np.arange(buckets.size + 1))
    return [idx[cut[k]:cut[k + 1]] for k in range(buckets.size)]


def test_gaia5_robust_source_update(agis_mod, oracle_lib, full5):
    w, eta, ctx = full5
    _start(agis_mod, ctx, w)
    agis_mod.agis_source_update(ctx)
    G = agis_mod.agis_get_sources(ctx, w.src_true.shape[0])
    nobs = np.bincount(w.src, minlength=w.src_true.shape[0])
    rng = np.random.default_rng(17)
    largest = np.argsort(-nobs, kind="stable")[:50]
    pick = np.unique(np.r_[rng.choice(w.src_true.shape[0], 1000, replace=False), largest])
    idx = np.flatnonzero(np.isin(w.src, pick))
    sub = subworld(w, idx)
    print(f"S sample: {pick.size} sources, {idx.size} observations, {nobs[largest].min()}..{nobs.max()} "
          f"observations for the 50 largest", flush=True)

    def run(pr):
        _, _, de = pr.source_update()
        run.defect = de
        return pr.s.copy(), pr.a.copy(), pr.c.copy()

    X, O, tol = fp64_floor(oracle_lib, sub, eta[idx], run)
    run(oracle_lib.problem_from_world(sub, eta[idx], state="start"))
    mask = np.zeros(w.src_true.shape[0], bool)
    mask[pick] = True
    mask &= run.defect == 0
    assert mask[largest].all() and mask.sum() > 0.99 * pick.size
    dg = check_floor(f"robust S update, {pick.size} sampled sources of gaia5", X[0], O[0], G, tol[0], 0, mask=mask)
    assert np.mean(np.abs(dg) <= TOL_UAS) > 0.95


def test_gaia5_excess_noise(agis_mod, oracle_lib, full5):
    """eps_a^2 of 300 sampled buckets at the start values (attitude 50 mas
    off, so eps_a is large and every bucket has a positive estimate)."""
    w, eta, ctx = full5
    nb = _start(agis_mod, ctx, w)
    agis_mod.agis_excess_noise_update(ctx)
    e_g = agis_mod.agis_get_excess_noise(ctx, 3 * nb)
    # every record along scan: the across-scan components have no values
    assert np.all(e_g[nb:] == 0.0)
    B = int(w.consts["eps_bucket"])
    rng = np.random.default_rng(19)
    buckets = np.sort(rng.choice(nb, 300, replace=False))
    K = w.n_att - 3
    ok_all = []
    for b, idx in zip(buckets, _bucket_members(w, buckets, B, K)):
        pr = oracle_lib.problem_from_world(subworld(w, idx), eta[idx], state="start")
        e_o = pr.excess_attitude_noise()[b]
        ok_all.append((b, idx.size, e_o, e_g[b]))
    e_o = np.array([x[2] for x in ok_all])
    e_gs = np.array([x[3] for x in ok_all])
    d = np.abs(e_gs - e_o)
    print(f"eps_a^2 of {buckets.size} buckets ({np.mean([x[1] for x in ok_all]):.0f} observations on average): "
          f"median eps_a {np.median(np.sqrt(e_o)) / UAS:.1f} uas, max |d eps_a^2| {d.max():.2e} rad^2, "
          f"max relative {np.max(d / np.maximum(e_o, 1e-300)):.2e}")
    assert np.all(e_o > 0)
    # R^2 - sigma^2 carries the residuals' rounding, |d(R^2)| <= 2 |R| |dR|
    # with |dR| < 1e-15 rad (the residual parity at full size) and |R| about
    # (eps_a^2 + sigma^2)^1/2 at the quantile; a factor 2 for the two order
    # statistics it interpolates
    s2 = (100 * UAS) ** 2
    assert np.all(d <= 4e-15 * np.sqrt(e_o + s2) + 2e-24)


def test_gaia5_attitude_calibration_update(agis_mod, oracle_lib, full5):
    """One robust A/C pass and solve at the start values with eps_a at its
    initial value (the weights w(R / sigma~) / sigma~^2 of the outliers)."""
    w, eta, ctx = full5
    _start(agis_mod, ctx, w)
    agis_mod.agis_attitude_calibration_update(ctx)
    Ga = agis_mod.agis_get_attitude(ctx, w.n_att)
    Gc = agis_mod.agis_get_calibration(ctx, w.n_cells)
    knots = w.knots
    S, L = int(w.consts["seg_len"]), int(w.consts["seg_overlap"])
    n_iv = knots.size - 7
    n_seg = (n_iv + S - 1) // S
    rng = np.random.default_rng(23)
    for K in sorted(rng.choice(np.arange(1, n_seg - 1), 3, replace=False)):
        lo_iv, hi_iv = max(K * S - L - 4, 0), min((K + 1) * S + L + 4, n_iv)
        idx = np.flatnonzero((w.t >= knots[3 + lo_iv]) & (w.t < knots[3 + hi_iv]))
        sub = subworld(w, idx)
        kept = {}

        def run(pr, K=K):
            d, de, lo, hi = pr.attitude_segment(int(K))
            kept["lo"], kept["hi"] = lo, hi
            a = pr.a.copy()
            a[lo:hi + 1] += d[lo:hi + 1]
            return pr.s.copy(), a, pr.c.copy()

        X, O, tol = fp64_floor(oracle_lib, sub, eta[idx], run)
        sl = slice(kept["lo"], kept["hi"] + 1)
        rd = check_floor(f"robust A update, gaia5 segment {K} of {n_seg} ({idx.size} observations)",
                         X[1][sl], O[1][sl], Ga[sl], tol[1][sl], 1)
        assert np.mean(np.abs(rd[:, 2]) <= TOL_UAS) > 0.99
    for day in sorted(rng.choice(np.arange(1, w.n_cells // 2 - 1), 2, replace=False)):
        cells = (2 * day, 2 * day + 1)
        idx = np.flatnonzero((w.cell == cells[0]) | (w.cell == cells[1]))
        sub = subworld(w, idx)

        def run(pr):
            pr.calibration_update()
            return pr.s.copy(), pr.a.copy(), pr.c.copy()

        X, O, tol = fp64_floor(oracle_lib, sub, eta[idx], run)
        sel = np.array(cells)
        check_floor(f"robust C update, gaia5 day {day} ({idx.size} observations)", X[2][sel], O[2][sel], Gc[sel],
                    tol[2][sel], 2)
