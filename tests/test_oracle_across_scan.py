"""Pins of the oracle's across-scan (AC) observations (eq:synth, eq:resAC;
Sect. 5.1.3 and 5.2.3 for their partials).

World: the tiny workload with one AC observation per transit (AC
uncertainty 520/92 of the AL one, the paper's bright-star ratio), marked by
cell = -1; every other recipe as for the along-scan pins.

* S block: with AC rows in the design matrix the 5x5 solution is still the
  weighted least-squares solution (numpy.linalg.lstsq).
* A block: one segment's solve equals dense regularised least squares over
  its AL and AC observations.
* C block: the closed form over the AL observations only (AC observations
  carry no calibration parameter).
* Geometry (Sect. 7.2.3): the AC attitude is fixed by the AC observations;
  the errors about the SRS y and x axes then stand in the ratio
  tan(Gamma_c / 2) the paper prints (224 / 167 uas).
"""

import numpy as np
import pytest

import synth
import synth.configs as C
from test_oracle_blocks import _rot_err, _segment_rows

UAS = synth.UAS


@pytest.fixture(scope="module")
def ac_world(oracle_lib):
    w = C.make("tiny", ac_obs=True)
    return w, oracle_lib.observed_field_angles(w)


def test_source_block_is_weighted_lstsq_with_ac(ac_world, oracle_lib):
    w, eta = ac_world
    pr = oracle_lib.problem_from_world(w, eta, state="start")
    o = pr.observe(partials=True)
    d, Q, defect = pr.source_update()
    order = np.argsort(w.src, kind="stable")
    off = np.searchsorted(w.src[order], np.arange(w.src_true.shape[0] + 1))
    ac = w.cell < 0
    n_checked = 0
    for i in range(0, w.src_true.shape[0], 499):
        rows = order[off[i]:off[i + 1]]
        assert ac[rows].any() and (~ac[rows]).any()
        sw = 1.0 / w.sigma[rows].astype(np.float64)
        A = o["dsrc"][rows] * sw[:, None]
        h = o["R"][rows] * sw
        if np.linalg.matrix_rank(A) < 5:
            continue
        x = np.linalg.lstsq(A, h, rcond=None)[0]
        cond = np.linalg.cond(A)
        assert np.abs(d[i] - x).max() <= 1e-14 * cond**2 * np.abs(x).max() + 1e-20
        Rpost = h - A @ d[i]
        assert abs(Q[i] - Rpost @ Rpost) <= 1e-8 * max(Q[i], 1e-30) + 1e-12
        n_checked += 1
    assert n_checked >= 30


def test_attitude_segment_is_regularised_lstsq_with_ac(ac_world, oracle_lib):
    w, eta = ac_world
    pr = oracle_lib.problem_from_world(w, eta, state="start")
    o = pr.observe(partials=True)
    K = 5
    d, defect, keep_lo, keep_hi = pr.attitude_segment(K)
    S, L = pr.consts["seg_len"], pr.consts["seg_overlap"]
    x0, x1 = 3 + K * S, 3 + (K + 1) * S
    J, r, n_lo = _segment_rows(pr, o, w, x0 - L, x1 + L, False)
    x = np.linalg.lstsq(J, -r, rcond=None)[0].reshape(-1, 4)
    ref = x[keep_lo - n_lo:keep_hi - n_lo + 1]
    got = d[keep_lo:keep_hi + 1]
    assert np.abs(got - ref).max() < 1e-6 * np.abs(ref).max()


def test_calibration_block_ignores_ac(ac_world, oracle_lib):
    w, eta = ac_world
    pr = oracle_lib.problem_from_world(w, eta, state="truth")
    pr.set_state(c=w.cal_start)
    R = pr.observe()["R"]
    d = pr.calibration_update()
    al = w.cell >= 0
    W = 1.0 / w.sigma[al].astype(np.float64) ** 2
    sw = np.bincount(w.cell[al], weights=W, minlength=w.n_cells)
    swr = np.bincount(w.cell[al], weights=W * R[al], minlength=w.n_cells)
    dt = np.where(sw > 0, -swr / np.where(sw > 0, sw, 1), 0.0)
    m = 0.5 * (dt[0::2] + dt[1::2])
    ref = dt.copy()
    ref[0::2] -= m
    ref[1::2] -= m
    np.testing.assert_allclose(d, ref, rtol=1e-12, atol=1e-22)


def test_ac_attitude_error_ratio(oracle_lib):
    """Sources and calibration at the truth, attitude from its start values,
    two attitude updates (the linearised solution): without AC data the
    errors about x and y are large; with them they drop several-fold and
    the y / x ratio of their RMS is tan(Gamma_c / 2) = 1.34 (the printed
    224 / 167), while the AL axis z hardly changes."""
    from test_golden import _values
    paper = _values()
    rms = {}
    for ac in (False, True):
        w = C.make("tiny", ac_obs=ac, lambda_reg=1e-3)
        eta = oracle_lib.observed_field_angles(w)
        pr = oracle_lib.problem_from_world(w, eta, state="truth")
        pr.set_state(a=w.att_start)
        for _ in range(2):
            pr.attitude_update()
        e = _rot_err(oracle_lib, pr.a, w.att_true, np.arange(40, w.n_att - 40, 3))
        rms[ac] = np.sqrt(np.mean(e ** 2, axis=0))
    ratio = rms[True][1] / rms[True][0]
    printed = paper["attitude_error_y_uas"] / paper["attitude_error_x_uas"]
    tan_half = np.tan(0.5 * w.consts["gamma_c"])
    print(f"attitude RMS errors (x, y, z) uas: AL only {np.round(rms[False], 1)}, AL + AC {np.round(rms[True], 1)}; "
          f"y / x {ratio:.3f} (printed {printed:.3f}, tan(Gamma_c/2) {tan_half:.3f})")
    assert abs(printed - tan_half) < 0.01
    assert abs(ratio - printed) < 0.1
    assert np.all(rms[True][:2] < rms[False][:2] / 4)
    assert abs(rms[True][2] / rms[False][2] - 1) < 0.1


def test_robust_weighting_takes_ac(oracle_lib, ac_world):
    """A robust problem with AC records holds the three excess attitude
    noise components of Sect. 3.6 (along scan, across scan in the preceding
    and in the following field of view) per bucket of knot intervals."""
    w, eta = ac_world
    consts = dict(w.consts)
    consts["robust"] = 1
    pr = oracle_lib.Problem(consts, w.knots, w.t, eta, w.sigma, w.src, w.fov, w.cell, w.src_start, w.att_start,
                            w.cal_start)
    nb = (w.n_att - 3 + consts["eps_bucket"] - 1) // consts["eps_bucket"]
    assert pr.eps_a2.size == 3 * nb
