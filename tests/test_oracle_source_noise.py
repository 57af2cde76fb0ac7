"""Pins of the oracle's excess source noise (robust mode 2, Sect. 5.1.2,
eq:epsi and eq:D).

World: the noise-free tiny world with Gaussian noise of the formal sigma
(100 uas, the same for every observation) added to every observation and a
further 200 uas to every fourth source's; attitude and calibration at the
truth, sources 50 mas off, no excess attitude noise.

* Closed form: with equal sigma and all w_l = 1, W_l = 1 / (sigma^2 + y) is
  one common factor, the solution does not depend on y and Q(y) = Q(0)
  sigma^2 / (sigma^2 + y); the rational step matches exactly that form, so
  its first step lands on Q(eps_i^2) = nu = n_i - 5 to rounding.
* eps_i = 0 exactly when Q(0) <= nu; D = (Q(0) - nu) / sqrt(2 nu).
* Statistics: the noisy sources' eps_i recovers the injected 200 uas in the
  median; the clean sources' D has mean ~0 and spread ~1 (Q(0) ~ chi^2_nu).
"""
import numpy as np
import pytest

import synth
import synth.configs as C

MAS, UAS = synth.MAS, synth.UAS


@pytest.fixture(scope="module")
def noisy(oracle_lib):
    w = C.make("tiny", noise=False)
    eta = oracle_lib.observed_field_angles(w)
    rng = np.random.default_rng(21)
    sig = w.sigma.astype(np.float64)
    extra = (w.src % 4 == 0)
    eta = eta + rng.normal(size=eta.size) * sig + np.where(extra, rng.normal(size=eta.size) * 200 * UAS, 0.0)
    consts = dict(w.consts)
    consts["robust"] = 2
    consts["eps_a_init"] = 0.0
    pr = oracle_lib.Problem(consts, w.knots, w.t, eta, w.sigma, w.src, w.fov, w.cell, w.src_start, w.att_true,
                            w.cal_true)
    s0 = pr.s.copy()
    d, Q, de = pr.source_update()
    return w, pr, s0, Q, extra


def test_rational_step_is_exact_for_equal_weights(oracle_lib, noisy):
    w, pr, s0, Q, extra = noisy
    # all final weights 1: every |R| / sqrt(sigma^2 + eps_i^2) <= 2 at the solution
    R = pr.observe()["R"]
    sig2 = w.sigma.astype(np.float64) ** 2
    z = np.abs(R) / np.sqrt(sig2 + pr.src_eps2[w.src])
    n_src = w.src_true.shape[0]
    all_one = np.bincount(w.src, weights=(z > 2.0).astype(float), minlength=n_src) == 0
    n = np.bincount(w.src, minlength=n_src)
    nu = n - 5.0
    pos = all_one & (pr.src_eps2 > 0)
    assert pos.sum() > 500
    assert np.abs(Q[pos] / nu[pos] - 1).max() < 1e-9
    # eps_i^2 = sigma^2 (Q(0) / nu - 1), Q(0) = Q(eps_i^2) (sigma^2 + eps_i^2) / sigma^2
    s2 = float(sig2[0])
    q0 = Q[pos] * (s2 + pr.src_eps2[pos]) / s2
    np.testing.assert_allclose(pr.src_eps2[pos], s2 * (q0 / nu[pos] - 1), rtol=1e-8)
    np.testing.assert_allclose(pr.src_D[pos], (q0 - nu[pos]) / np.sqrt(2 * nu[pos]), rtol=1e-8)


def test_zero_when_chi2_below_nu_and_statistics(oracle_lib, noisy):
    w, pr, s0, Q, extra = noisy
    n_src = w.src_true.shape[0]
    src_extra = np.zeros(n_src, bool)
    src_extra[np.unique(w.src[extra])] = True
    eps = np.sqrt(pr.src_eps2) / UAS
    D = pr.src_D
    # eps_i = 0 exactly where D <= 0 (Q(0) <= nu), positive where D > 0
    assert np.all(eps[D <= 0] == 0.0) and np.all(eps[D > 0] > 0.0)
    med = np.median(eps[src_extra])
    print(f"noisy sources: median eps_i {med:.1f} uas (injected 200); clean: mean D {D[~src_extra].mean():.3f}, "
          f"std {D[~src_extra].std():.3f}, {np.mean(eps[~src_extra] == 0):.2f} with eps_i = 0")
    assert 170 < med < 230
    assert abs(D[~src_extra].mean()) < 0.25 and 0.7 < D[~src_extra].std() < 1.4
    assert np.median(D[src_extra]) > 4.0
    assert 0.4 < np.mean(eps[~src_extra] == 0) < 0.8
