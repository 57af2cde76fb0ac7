"""Pins of the oracle's large-scale along-scan geometric calibration
(eq:etazeta, Sect. 3.4; the C block of Sect. 5.3 with eq:calCon and the
constraint eq:cc1).

World: the small nine-CCD workload with the geometric model: per
calibration cell (day and field of view) and CCD three coefficients of the
shifted Legendre polynomials L*_0..2 in the across-scan pixel coordinate,
in place of one offset per cell; one pixel coordinate per transit.

* The polynomials: L*_r(x) on [0, 1] are orthogonal with norms 1/(2r+1)
  (Gauss-Legendre quadrature) and take their closed-form end values.
* At the truth the noise-free residuals vanish (to rounding).
* From zero coefficients, sources and attitude at the truth and no noise,
  one C update recovers the true coefficients: the model is linear in them
  and the truth satisfies eq:cc1.
* With noise and offsets, the update equals the plain definition: per cell
  and CCD the weighted least-squares fit of -R on (L*_0, L*_1, L*_2) over
  its records (numpy.linalg.lstsq), then eq:calCon for eq:cc1, i.e. each
  day's mean constant term removed; the constraint then holds.
* The across-scan term (the AC half of eq:etazeta, constraint eq:cc3), on
  the nine-CCD world with one AC record per transit on a CCD line drawn per
  transit: a unit AC coefficient moves exactly its group's AC residuals, by
  L*_r(x); the AC residuals vanish at the truth; one update from zero
  coefficients recovers both terms' truth; with noise the AC part of the
  update is the per-group weighted least squares followed by each cell's
  mean AC constant term removed (eq:calCon for eq:cc3), which then holds.
* The simple iteration S[AC] recovers the coefficients on a noise-free world
  (the tiny workload with one across-scan record per transit and the
  geometric model on its single CCD line; the sparse nine-CCD parity world
  does not support iterating) from start values ~25 mas off: below 5% of
  the start error in every term after 20 iterations.
"""
import numpy as np
import pytest

import synth
import synth.configs as C

UAS, MAS = synth.UAS, synth.MAS


@pytest.fixture(scope="module")
def geo_world(oracle_lib):
    w = C.make("small9", geo_cal=True, noise=False)
    return w, oracle_lib.observed_field_angles(w)


def _legendre(r, x):
    return [np.ones_like(x), 2 * x - 1, 6 * x * x - 6 * x + 1][r]


def _x(w):
    return (w.mu.astype(np.float64) - 13.5) / 1966.0


def test_shifted_legendre_orthogonal():
    """Against the quadrature of the definition: orthogonal on [0, 1] with
    integral of L*_r^2 equal to 1 / (2r + 1); L*_r(0) = (-1)^r, L*_r(1) = 1.
    The polynomials are the model's, evaluated through a one-record world."""
    import oracle
    u, wq = np.polynomial.legendre.leggauss(8)
    x = 0.5 * (u + 1.0)
    w = C.make("small9", geo_cal=True, noise=False)
    # one record per quadrature node: its geometric term with a unit
    # coefficient r is L*_r at the node
    vals = np.zeros((3, x.size))
    for r in range(3):
        geo = np.zeros_like(w.geo_true)
        geo[0, 0, r] = 1.0
        pr = oracle.Problem(w.consts, w.knots, np.full(x.size, w.t[0]), np.zeros(x.size), w.sigma[:x.size],
                            np.full(x.size, w.src[0], np.int32), np.full(x.size, 1, np.int8),
                            np.zeros(x.size, np.int32), w.src_true, w.att_true, np.zeros_like(w.cal_true),
                            ccd=np.zeros(x.size, np.int8), mu=(13.5 + 1966.0 * x).astype(np.float32), geo=geo)
        pr0 = oracle.Problem(w.consts, w.knots, np.full(x.size, w.t[0]), np.zeros(x.size), w.sigma[:x.size],
                             np.full(x.size, w.src[0], np.int32), np.full(x.size, 1, np.int8),
                             np.zeros(x.size, np.int32), w.src_true, w.att_true, np.zeros_like(w.cal_true),
                             ccd=np.zeros(x.size, np.int8), mu=(13.5 + 1966.0 * x).astype(np.float32),
                             geo=np.zeros_like(geo))
        vals[r] = pr.observe()["R"] - pr0.observe()["R"]
    xq = (np.float32(13.5 + 1966.0 * x).astype(np.float64) - 13.5) / 1966.0
    G = 0.5 * (vals * wq) @ vals.T
    np.testing.assert_allclose(G, np.diag([1.0, 1.0 / 3.0, 1.0 / 5.0]), atol=2e-6)
    for r in range(3):
        np.testing.assert_allclose(vals[r], _legendre(r, xq), rtol=0, atol=1e-12)


def test_residuals_vanish_at_the_truth(oracle_lib, geo_world):
    w, eta = geo_world
    R = oracle_lib.problem_from_world(w, eta, state="truth").observe()["R"]
    print(f"noise-free residuals at the truth: max {np.abs(R).max():.2e} rad")
    assert np.abs(R).max() < 1e-15


def test_calibration_update_recovers_the_truth(oracle_lib, geo_world):
    w, eta = geo_world
    pr = oracle_lib.problem_from_world(w, eta, state="truth")
    pr.set_state(geo=np.zeros_like(w.geo_true))
    pr.calibration_update()
    d = (pr.geo.reshape(w.geo_true.shape) - w.geo_true) / UAS
    print(f"recovered geometric calibration: max error {np.abs(d).max():.2e} uas "
          f"(true coefficients up to {np.abs(w.geo_true).max() / UAS:.0f} uas)")
    assert np.abs(d).max() < 1e-6


def test_calibration_update_is_the_weighted_lstsq_with_cc1(oracle_lib):
    w = C.make("small9", geo_cal=True)
    eta = oracle_lib.observed_field_angles(w)
    pr = oracle_lib.problem_from_world(w, eta, state="start")
    o = pr.observe()
    R, x = np.asarray(o["R"]), _x(w)
    W = 1.0 / w.sigma.astype(np.float64) ** 2
    n_ccd = int(w.consts["geo_ccds"])
    g = w.cell.astype(np.int64) * n_ccd + w.ccd
    ref = np.zeros((w.cal_true.size * n_ccd, 3))
    for gi in np.unique(g[w.cell >= 0]):
        sel = g == gi
        A = np.stack([_legendre(r, x[sel]) for r in range(3)], axis=1) * np.sqrt(W[sel])[:, None]
        ref[gi] = np.linalg.lstsq(A, -R[sel] * np.sqrt(W[sel]), rcond=None)[0]
    per_day = 2 * n_ccd
    c0 = ref[:, 0].reshape(-1, per_day)
    ref[:, 0] = (c0 - c0.mean(axis=1, keepdims=True)).reshape(-1)
    d = pr.calibration_update().reshape(-1, 3)
    scale = np.abs(ref).max()
    print(f"C update vs weighted lstsq + eq:cc1: max |diff| {np.abs(d - ref).max() / UAS:.2e} uas "
          f"(update up to {scale / UAS:.0f} uas)")
    np.testing.assert_allclose(d, ref, rtol=0, atol=1e-9 * scale)
    # eq:cc1 holds for the updated coefficients (the start values satisfy it)
    geo = pr.geo.reshape(-1, 3)[:, 0].reshape(-1, per_day)
    assert np.abs(geo.sum(axis=1)).max() < 1e-20 * per_day + 1e-12 * np.abs(geo).max()


def test_iterations_recover_the_calibration(oracle_lib):
    w = C.make("tiny", geo_cal=True, ac_obs=True, noise=False)
    eta = oracle_lib.observed_field_angles(w)
    pr = oracle_lib.problem_from_world(w, eta, state="start")
    e0 = (w.geo_start - w.geo_true) / UAS
    errs = [np.sqrt(np.mean(e0 * e0, axis=(0, 1)))]
    for _ in range(20):
        pr.iterate(s_ref=w.src_true)
        e = (pr.geo.reshape(w.geo_true.shape) - w.geo_true) / UAS
        errs.append(np.sqrt(np.mean(e * e, axis=(0, 1))))
    errs = np.array(errs)
    print("geometric calibration RMS error (r = 0, 1, 2) every 4 iterations [uas]:\n", np.round(errs[::4], 2))
    assert np.all(errs[-1] < 0.05 * errs[0])


@pytest.fixture(scope="module")
def geo_ac_world(oracle_lib):
    w = C.make("small9", geo_cal=True, ac_obs=True, geo_ac=True, noise=False)
    return w, oracle_lib.observed_field_angles(w)


def test_ac_term_moves_its_group_only(oracle_lib, geo_ac_world):
    """Against the definition: a unit coefficient r of one AC group adds
    L*_r(x) to the residuals of that group's AC records and nothing to any
    other record."""
    w, eta = geo_ac_world
    base = oracle_lib.problem_from_world(w, eta, state="truth")
    R0 = np.asarray(base.observe()["R"])
    n_al = w.geo_true.size
    ac = np.flatnonzero(w.cell < 0)
    l = ac[len(ac) // 2]
    gi = int(w.ac_cell[l]) * int(w.consts["geo_ccds"]) + int(w.ccd[l])
    members = (w.cell < 0) & (w.ac_cell.astype(np.int64) * int(w.consts["geo_ccds"]) + w.ccd == gi)
    assert members.sum() > 3
    for r in range(3):
        pr = oracle_lib.problem_from_world(w, eta, state="truth")
        geo = pr.geo.copy()
        geo[n_al + 3 * gi + r] += 1.0
        pr.set_state(geo=geo)
        dR = np.asarray(pr.observe()["R"]) - R0
        np.testing.assert_allclose(dR[members], _legendre(r, _x(w)[members]), rtol=0, atol=1e-12)
        assert np.all(dR[~members] == 0.0)


def test_ac_residuals_vanish_and_update_recovers_both_terms(oracle_lib, geo_ac_world):
    w, eta = geo_ac_world
    pr = oracle_lib.problem_from_world(w, eta, state="truth")
    R = np.asarray(pr.observe()["R"])
    assert np.abs(R).max() < 1e-15
    pr.set_state(geo=np.zeros_like(pr.geo))
    pr.calibration_update()
    d_al = (pr.geo[:w.geo_true.size].reshape(w.geo_true.shape) - w.geo_true) / UAS
    d_ac = (pr.geo[w.geo_true.size:].reshape(w.geo_ac_true.shape) - w.geo_ac_true) / UAS
    print(f"recovered AL / AC terms: max error {np.abs(d_al).max():.2e} / {np.abs(d_ac).max():.2e} uas")
    assert np.abs(d_al).max() < 1e-6 and np.abs(d_ac).max() < 1e-6


def test_ac_update_is_the_weighted_lstsq_with_cc3(oracle_lib):
    w = C.make("small9", geo_cal=True, ac_obs=True, geo_ac=True)
    eta = oracle_lib.observed_field_angles(w)
    pr = oracle_lib.problem_from_world(w, eta, state="start")
    R, x = np.asarray(pr.observe()["R"]), _x(w)
    W = 1.0 / w.sigma.astype(np.float64) ** 2
    n_ccd = int(w.consts["geo_ccds"])
    ac = w.cell < 0
    g = np.where(ac, w.ac_cell.astype(np.int64) * n_ccd + w.ccd, -1)
    ref = np.zeros((int(w.consts["geo_ac_cells"]) * n_ccd, 3))
    for gi in np.unique(g[ac]):
        sel = g == gi
        A = np.stack([_legendre(r, x[sel]) for r in range(3)], axis=1) * np.sqrt(W[sel])[:, None]
        ref[gi] = np.linalg.lstsq(A, -R[sel] * np.sqrt(W[sel]), rcond=None)[0]
    c0 = ref[:, 0].reshape(-1, n_ccd)
    ref[:, 0] = (c0 - c0.mean(axis=1, keepdims=True)).reshape(-1)
    d = pr.calibration_update()[w.geo_true.size:].reshape(-1, 3)
    scale = np.abs(ref).max()
    print(f"AC update vs weighted lstsq + eq:cc3: max |diff| {np.abs(d - ref).max() / UAS:.2e} uas "
          f"(update up to {scale / UAS:.0f} uas)")
    np.testing.assert_allclose(d, ref, rtol=0, atol=1e-9 * scale)
    geo_ac = pr.geo[w.geo_true.size:].reshape(-1, 3)[:, 0].reshape(-1, n_ccd)
    assert np.abs(geo_ac.sum(axis=1)).max() < 1e-12 * np.abs(geo_ac).max()


def test_iterations_recover_both_terms(oracle_lib):
    """The tiny world (one CCD line, so eq:cc3 holds every AC constant term at
    zero) with AC records and both terms: noise-free iterations from start
    values ~25 mas off bring every term of both below 5% of its start error."""
    w = C.make("tiny", geo_cal=True, ac_obs=True, geo_ac=True, noise=False)
    eta = oracle_lib.observed_field_angles(w)
    pr = oracle_lib.problem_from_world(w, eta, state="start")
    n_al = w.geo_true.size

    def err():
        e_al = (pr.geo[:n_al].reshape(w.geo_true.shape) - w.geo_true) / UAS
        e_ac = (pr.geo[n_al:].reshape(w.geo_ac_true.shape) - w.geo_ac_true) / UAS
        return np.array([np.sqrt(np.mean(e * e, axis=(0, 1))) for e in (e_al, e_ac)])    # [AL / AC][r]
    e0 = err()
    for _ in range(20):
        pr.iterate(s_ref=w.src_true)
    e1 = err()
    print("RMS error [uas], AL and AC terms (r = 0, 1, 2): start\n", np.round(e0, 2), "\nafter 20\n", np.round(e1, 3))
    live = e0 > 0
    assert np.all(e1[live] < 0.05 * e0[live]) and np.all(e1[~live] < 1e-9)


def test_basic_angle_monitor_recovers_a_basic_angle_change(oracle_lib):
    """eq:DeltaGamma: observations made with the basic angle Gamma_c + delta
    (the true lines of sight further apart by delta), solved with the model's
    conventional Gamma_c, sources and attitude at the truth and no noise: the
    C update absorbs the change into the AL constant terms with opposite
    signs in the two fields of view, and the monitored offset of every day
    moves by +delta (the offset of the actual basic angle from Gamma_c), to
    1e-6 of delta and the same on every day (the sign and the normalisation
    are what this pins; the model's field angles are not exactly linear in
    the basic angle, which leaves ~6e-9 of delta)."""
    import copy
    w = C.make("small9", geo_cal=True, noise=False)
    delta = 1.0 * MAS
    wd = copy.copy(w)
    wd.consts = dict(w.consts, gamma_c=w.consts["gamma_c"] + delta)
    eta = oracle_lib.observed_field_angles(wd)
    pr = oracle_lib.problem_from_world(w, eta, state="true")
    n_ccd = int(w.consts["geo_ccds"])
    before = oracle_lib.basic_angle(pr.geo, w.n_cells, n_ccd)
    pr.calibration_update()
    moved = oracle_lib.basic_angle(pr.geo, w.n_cells, n_ccd) - before
    seen = np.bincount(w.cell[w.cell >= 0] // 2, minlength=w.n_cells // 2) > 0
    print(f"basic-angle offset moved by {moved[seen].mean() / MAS:.9f} mas (delta 1 mas), "
          f"spread {np.ptp(moved[seen]) / UAS:.2e} uas over {seen.sum()} days")
    assert np.allclose(moved[seen], delta, rtol=1e-6, atol=0)
    assert np.ptp(moved[seen]) < 1e-9 * delta
    assert np.all(moved[~seen] == 0.0)
