"""Pins of the oracle's robust weighting (Sect. 5.1.2, 5.2.5): the
downweighting function eq:dw, the type-7 quantile, the source inner
iteration and the excess attitude noise of eq e09."""
import numpy as np
import pytest

import synth
import synth.configs as C

MAS, UAS = synth.MAS, synth.UAS


def test_weight_function_values_and_smoothness(oracle_lib):
    w = oracle_lib.weight_function
    # values quoted with eq:dw
    assert abs(w(10.0) - 0.036) < 5e-4
    assert 2.5e-15 < w(100.0) < 3.5e-15
    assert w(0.0) == 1.0 and w(2.0) == 1.0 and w(-1.5) == 1.0
    for z in (0.3, 2.4, 3.0, 7.0):
        assert w(z) == w(-z)
    # continuous value and slope at |z| = 2 and 3; non-increasing
    h = 1e-6
    for z0 in (2.0, 3.0):
        assert abs(w(z0 + h) - w(z0 - h)) < 1e-6
        left = (w(z0 - h) - w(z0 - 2 * h)) / h
        right = (w(z0 + 2 * h) - w(z0 + h)) / h
        assert abs(left - right) < 1e-5
    zs = np.linspace(0, 20, 2001)
    ws = np.array([w(z) for z in zs])
    assert np.all(np.diff(ws) <= 0) and np.all(ws > 0)
    # the exponential branch from |z| = 3 on
    assert abs(w(3.0) - np.exp(-1.0)) < 1e-6 and abs(w(6.0) - np.exp(-2.0)) < 1e-15


def test_quantile_is_type7(oracle_lib):
    rng = np.random.default_rng(5)
    for n in (1, 2, 3, 7, 100, 1001):
        x = rng.normal(size=n)
        x[: n // 3] = x[0]                      # ties
        for p in (0.0, 1 / 6, 0.5, 0.68, 5 / 6, 1.0):
            assert oracle_lib.quantile(x, p) == pytest.approx(np.quantile(x, p, method="linear"), abs=1e-15)
    assert oracle_lib.quantile(np.zeros(0), 0.68) == 0.0


@pytest.fixture(scope="module")
def outlier_world(oracle_lib):
    """Noise-free tiny world with 1% gross outliers (20-100 mas)."""
    w = C.make("tiny", noise=False)
    eta = oracle_lib.observed_field_angles(w)
    rng = np.random.default_rng(11)
    bad = rng.random(w.n_obs) < 0.01
    eta_bad = eta + np.where(bad, rng.choice([-1.0, 1.0], w.n_obs) * rng.uniform(20, 100, w.n_obs) * MAS, 0.0)
    return w, eta_bad, bad


def _problem(oracle_lib, w, eta, robust, s0, keep=None):
    consts = dict(w.consts)
    consts["robust"] = int(robust)
    consts["eps_a_init"] = 0.0
    k = slice(None) if keep is None else keep
    return oracle_lib.Problem(consts, w.knots, w.t[k], eta[k], w.sigma[k], w.src[k], w.fov[k], w.cell[k], s0,
                              w.att_true, w.cal_true)


def _sdiff(a, b):
    x = (a - b) / UAS
    x[:, 0] *= np.cos(b[:, 1])
    return x


def test_inner_iteration_rejects_gross_outliers(oracle_lib, outlier_world):
    """Sources 1 mas from the truth: the robust update on data with gross
    outliers equals the plain update on the data without them (every
    outlier ends with a weight of exp(-|z|/3) ~ 0); the plain update on the
    contaminated data is off by mas."""
    w, eta_bad, bad = outlier_world
    rng = np.random.default_rng(12)
    s0 = w.src_true + rng.normal(0, 1.0, w.src_true.shape) * MAS
    pr = _problem(oracle_lib, w, eta_bad, True, s0)
    _, _, de_r = pr.source_update()
    pc = _problem(oracle_lib, w, eta_bad, False, s0, keep=~bad)
    _, _, de_c = pc.source_update()
    pp = _problem(oracle_lib, w, eta_bad, False, s0)
    pp.source_update()
    n_clean = np.bincount(w.src[~bad], minlength=w.src_true.shape[0])
    n_bad = np.bincount(w.src[bad], minlength=w.src_true.shape[0])
    sel = (n_clean >= 10) & (n_bad >= 1) & (de_r == 0) & (de_c == 0)
    assert sel.sum() > 500
    assert np.abs(_sdiff(pr.s, pc.s))[sel].max() < 1e-4
    assert np.median(np.abs(_sdiff(pp.s, pc.s))[sel].max(1)) > 100.0


def test_excess_attitude_noise(oracle_lib, tiny_world):
    """eq e09 per bucket of 8 knot intervals: equals NumPy's 68th percentile
    of R^2 - sigma^2 over the bucket (clipped at 0); recovers an excess
    noise added to the observations of a range of buckets."""
    w = tiny_world
    eta = oracle_lib.observed_field_angles(w)
    rng = np.random.default_rng(21)
    consts = dict(w.consts)
    consts["robust"] = 1
    consts["eps_a_init"] = 0.0
    sig = w.sigma.astype(np.float64)
    # truth state, observation noise sigma plus an excess of 300 uas in a window
    pr0 = oracle_lib.Problem(consts, w.knots, w.t, eta, w.sigma, w.src, w.fov, w.cell, w.src_true, w.att_true,
                             w.cal_true)
    ell = pr0.observe()["ell"]
    bucket = (ell - 3) // 8
    win = (bucket >= 100) & (bucket < 160)
    excess = 300.0 * UAS
    eta2 = eta + rng.normal(0, 1, w.n_obs) * sig + np.where(win, rng.normal(0, excess, w.n_obs), 0.0)
    pr = oracle_lib.Problem(consts, w.knots, w.t, eta2, w.sigma, w.src, w.fov, w.cell, w.src_true, w.att_true,
                            w.cal_true)
    e2 = pr.excess_attitude_noise()
    R = pr.observe()["R"]
    nb = e2.size // 3                                  # along scan; the across-scan components are empty here
    assert np.all(e2[nb:] == 0.0)
    e2 = e2[:nb]
    ref = np.zeros(nb)
    for j in np.unique(bucket):
        v = R[bucket == j] ** 2 - sig[bucket == j] ** 2
        ref[j] = max(0.0, np.quantile(v, 0.68, method="linear"))
    assert np.allclose(e2, ref, rtol=1e-12, atol=1e-30)
    # statistical recovery: for N(0, s^2 + e^2) residuals the 68% point of
    # R^2 - s^2 is 0.989 (s^2 + e^2) - s^2
    inside = np.sqrt(np.median(e2[100:160]))
    expect = np.sqrt(0.989 * (100.0 ** 2 + 300.0 ** 2) - 100.0 ** 2) * UAS
    assert abs(inside / expect - 1) < 0.1
    outside = np.concatenate([e2[:100], e2[160:]])
    assert np.median(np.sqrt(outside)) < 30 * UAS


def test_robust_attitude_update_rejects_outliers(oracle_lib, outlier_world):
    """Sources and calibration at the truth, attitude 1 mas off: after the
    excess attitude noise has been estimated from the residuals (Sect.
    5.2.5, it absorbs the 1 mas attitude error), the robust attitude update
    on contaminated data equals the plain update on the clean data, while
    the plain update on the contaminated data is pulled by the outliers."""
    w, eta_bad, bad = outlier_world
    rng = np.random.default_rng(13)

    def rot_uas(a_ref, a):
        out = []
        for x, y in zip(a_ref, a):
            q = oracle_lib.qmul(oracle_lib.qinv(x), y)
            q = q / np.linalg.norm(q)
            out.append(2 * q[:3] * np.sign(q[3]) / UAS)
        return np.array(out)

    a0 = w.att_true.copy()
    for n in range(a0.shape[0]):
        a0[n] = oracle_lib.qmul(a0[n], oracle_lib.qrot(rng.normal(0, 1.0, 3) * MAS))
    consts = dict(w.consts)
    consts["eps_a_init"] = 0.0

    def run(robust, keep=None):
        consts["robust"] = int(robust)
        k = slice(None) if keep is None else keep
        p = oracle_lib.Problem(consts, w.knots, w.t[k], eta_bad[k], w.sigma[k], w.src[k], w.fov[k], w.cell[k],
                               w.src_true, a0, w.cal_true)
        if robust:
            p.excess_attitude_noise()
        p.attitude_update()
        return p.a

    a_rob, a_clean, a_plain = run(True), run(False, keep=~bad), run(False)
    mid = slice(20, w.n_att - 20)
    # along-scan rotation error of one update against the truth (a single
    # update from 1 mas leaves a few 1e-2 uas whatever the weights)
    e_rob = np.abs(rot_uas(w.att_true[mid], a_rob[mid]))[:, 2]
    e_clean = np.abs(rot_uas(w.att_true[mid], a_clean[mid]))[:, 2]
    e_plain = np.abs(rot_uas(w.att_true[mid], a_plain[mid]))[:, 2]
    print("robust attitude pin: median err rob %.3g clean %.3g plain %.3g uas" % (np.median(e_rob), np.median(e_clean), np.median(e_plain)))
    assert np.median(e_rob) < 1.5 * np.median(e_clean) + 0.01
    assert np.percentile(e_rob, 99) < 1.5 * np.percentile(e_clean, 99) + 0.05
    assert np.median(e_plain) > 50 * np.median(e_rob)


@pytest.fixture(scope="module")
def ac_world(oracle_lib):
    """Noise-free tiny world with one across-scan record per transit."""
    w = C.make("tiny", noise=False, ac_obs=True)
    return w, oracle_lib.observed_field_angles(w)


def test_excess_attitude_noise_components(oracle_lib, ac_world):
    """The three excess-noise functions (Sect. 3.6: along scan, across scan
    in the preceding and in the following field of view), each by eq e09
    over its own observations: every (component, bucket) equals NumPy's 68th
    percentile of R^2 - sigma^2 over that set; an excess of 300 uas added to
    the ACP records of buckets 100-159 and of 200 uas to the AL records of
    buckets 300-359 is recovered in that component and bucket range only."""
    w, eta = ac_world
    rng = np.random.default_rng(31)
    consts = dict(w.consts, robust=1, eps_a_init=0.0)
    sig = w.sigma.astype(np.float64)
    pr0 = oracle_lib.Problem(consts, w.knots, w.t, eta, w.sigma, w.src, w.fov, w.cell, w.src_true, w.att_true,
                             w.cal_true)
    bucket = (pr0.observe()["ell"] - 3) // 8
    comp = np.where(w.cell >= 0, 0, np.where(w.fov > 0, 1, 2))
    acp_win = (comp == 1) & (bucket >= 100) & (bucket < 160)
    al_win = (comp == 0) & (bucket >= 300) & (bucket < 360)
    eta2 = (eta + rng.normal(0, 1, w.n_obs) * sig + np.where(acp_win, rng.normal(0, 300 * UAS, w.n_obs), 0.0)
            + np.where(al_win, rng.normal(0, 200 * UAS, w.n_obs), 0.0))
    pr = oracle_lib.Problem(consts, w.knots, w.t, eta2, w.sigma, w.src, w.fov, w.cell, w.src_true, w.att_true,
                            w.cal_true)
    e2 = pr.excess_attitude_noise()
    nb = e2.size // 3
    R = pr.observe()["R"]
    ref = np.zeros(3 * nb)
    for a in range(3):
        for j in np.unique(bucket[comp == a]):
            sel = (comp == a) & (bucket == j)
            ref[a * nb + j] = max(0.0, np.quantile(R[sel] ** 2 - sig[sel] ** 2, 0.68, method="linear"))
    assert np.allclose(e2, ref, rtol=1e-12, atol=1e-30)
    e = np.sqrt(e2.reshape(3, nb)) / UAS
    s_ac = float(sig[comp == 1][0]) / UAS
    exp_acp = np.sqrt(0.989 * (s_ac ** 2 + 300.0 ** 2) - s_ac ** 2)
    exp_al = np.sqrt(0.989 * (100.0 ** 2 + 200.0 ** 2) - 100.0 ** 2)
    print(f"ACP window {np.median(e[1, 100:160]):.1f} uas (expected {exp_acp:.1f}); AL window "
          f"{np.median(e[0, 300:360]):.1f} (expected {exp_al:.1f}); elsewhere AL {np.median(e[0, :100]):.1f}, "
          f"ACP {np.median(e[1, 200:300]):.1f}, ACF {np.median(e[2]):.1f} uas")
    assert abs(np.median(e[1, 100:160]) / exp_acp - 1) < 0.15
    assert abs(np.median(e[0, 300:360]) / exp_al - 1) < 0.1
    assert np.median(e[1, 300:360]) < 0.3 * exp_acp and np.median(e[2, 100:160]) < 0.3 * exp_acp
    assert np.median(e[0, 100:160]) < 0.3 * exp_al


def test_inner_iteration_with_across_scan_records(oracle_lib, ac_world):
    """Robust S update with along- and across-scan records of one source (a
    scale ratio of 5.65 between their sigmas): the initial downweights take
    varsigma from each kind's own residuals, so gross outliers of either
    kind are rejected: the robust update on contaminated data equals the
    plain update on the clean data to the influence the outliers keep
    (across scan a 20 mas outlier is only 35 sigma, w = exp(-35/3) ~ 1e-5,
    which moves a source by a few 1e-2 uas; along scan w ~ 1e-29), while the
    plain update is pulled off by mas."""
    w, eta = ac_world
    rng = np.random.default_rng(33)
    bad = rng.random(w.n_obs) < 0.01
    eta_bad = eta + np.where(bad, rng.choice([-1.0, 1.0], w.n_obs) * rng.uniform(20, 100, w.n_obs) * MAS, 0.0)
    s0 = w.src_true + rng.normal(0, 1.0, w.src_true.shape) * MAS
    consts = dict(w.consts, robust=1, eps_a_init=0.0)

    def run(robust, keep=slice(None)):
        c = dict(consts, robust=int(robust))
        p = oracle_lib.Problem(c, w.knots, w.t[keep], eta_bad[keep], w.sigma[keep], w.src[keep], w.fov[keep],
                               w.cell[keep], s0, w.att_true, w.cal_true)
        _, _, de = p.source_update()
        return p.s, de

    s_rob, de_r = run(True)
    s_clean, de_c = run(False, ~bad)
    s_plain, _ = run(False)
    n_clean = np.bincount(w.src[~bad], minlength=w.src_true.shape[0])
    n_bad = np.bincount(w.src[bad], minlength=w.src_true.shape[0])
    n_ac_bad = np.bincount(w.src[bad & (w.cell < 0)], minlength=w.src_true.shape[0])
    sel = (n_clean >= 20) & (n_bad >= 1) & (de_r == 0) & (de_c == 0)
    assert sel.sum() > 500 and (sel & (n_ac_bad >= 1)).sum() > 100
    d_rob = np.abs(_sdiff(s_rob, s_clean)).max(1)
    print(f"robust - clean: AL-only outliers max {d_rob[sel & (n_ac_bad == 0)].max():.2e} uas, "
          f"with AC outliers max {d_rob[sel & (n_ac_bad >= 1)].max():.2e} uas")
    assert d_rob[sel & (n_ac_bad == 0)].max() < 1e-4
    assert d_rob[sel].max() < 0.1
    assert np.median(np.abs(_sdiff(s_plain, s_clean))[sel].max(1)) > 100.0
