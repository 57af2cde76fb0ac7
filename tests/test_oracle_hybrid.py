"""Pins of the oracle's frozen weights, the switch of the hybrid scheme
(Sect. 4.7; Problem.frozen_sigma, oracle.cg.freeze).

* At the state where they are frozen, the fixed weights reproduce the robust
  A and C updates (whose weights they are) to the rounding of sigma_eff =
  W^-1/2 (FP64), and the robust weight function: sigma_eff = sigma~ for
  residuals within 2 sigma~, much larger for gross outliers.
* CG on the frozen problem lowers the frozen objective sum W R^2 below what
  the robust simple iteration reaches in the same number of evaluations.
"""
import numpy as np
import pytest

import synth
import synth.configs as C
from test_oracle_robust import _problem, outlier_world  # noqa: F401

MAS, UAS = synth.MAS, synth.UAS


def test_frozen_weights_reproduce_the_robust_ac_updates(oracle_lib, outlier_world):
    from oracle import cg as ocg
    w, eta, bad = outlier_world
    pr = _problem(oracle_lib, w, eta, True, w.src_start.copy())
    pr.iterate_sac()                                   # sources near their solution, eps_a estimated
    x = (pr.s.copy(), pr.a.copy(), pr.c.copy())
    fr = ocg.freeze(pr)
    o = pr.observe()
    s2 = w.sigma.astype(np.float64) ** 2 + pr.eps_a2[(o["ell"] - 3) // int(pr.consts["eps_bucket"])]
    z = np.abs(o["R"]) / np.sqrt(s2)
    sig = fr.sigma_eff
    inlier = z <= 2.0                                  # eq:dw: w = 1
    np.testing.assert_allclose(sig[inlier], np.sqrt(s2[inlier]), rtol=1e-15)
    assert np.all(sig[~inlier] >= np.sqrt(s2[~inlier]) * (1 - 1e-15))
    assert np.median(sig[bad] / np.sqrt(s2[bad])) > 10.0
    # the A and C updates at the freezing state
    for name in ("attitude_update", "calibration_update"):
        pr.set_state(*x)
        fr.set_state(*x)
        d_ref, d_got = getattr(pr, name)(), getattr(fr, name)()
        d_ref = d_ref[0] if isinstance(d_ref, tuple) else d_ref
        d_got = d_got[0] if isinstance(d_got, tuple) else d_got
        rel = np.abs(d_got - d_ref).max() / np.abs(d_ref).max()
        print(f"{name}: max |frozen - robust| / max |update| = {rel:.1e}")
        assert rel <= 1e-10


def test_hybrid_lowers_the_frozen_objective(oracle_lib, outlier_world):
    from oracle import cg as ocg
    w, eta, bad = outlier_world
    pr = _problem(oracle_lib, w, eta, True, w.src_start.copy())
    for _ in range(3):
        pr.iterate(w.src_true)
    fr = ocg.freeze(pr)
    W = 1.0 / fr.sigma_eff ** 2

    def objective(p):
        return float(np.sum(W * p.observe()["R"] ** 2))

    q0 = objective(fr)
    si = ocg.freeze(pr)                                  # the same frozen problem, simple iteration
    for _ in range(12):
        si.iterate(w.src_true)
    it = ocg.CG(fr, restart=40, s_ref=w.src_true)
    it.run(12)
    q_si, q_cg = objective(si), objective(fr)
    print(f"frozen objective: start {q0:.6g}, 12 SI iterations {q_si:.6g}, 12 CG steps {q_cg:.6g}")
    assert q_cg < q_si < q0
