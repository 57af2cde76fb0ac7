"""Pins of the oracle's small-scale along-scan geometric calibration
(eq:etazeta's delta-eta, Sect. 3.4, with the constraint eq:cc2; the C block
of Sect. 5.3).

World: the 60-day nine-CCD workload with the geometric model and the
small-scale term: one value per CCD, 30-day long interval and pixel column
m = round(mu) (1966 columns, ~15 records each), beside the large-scale
coefficients of each cell and CCD.

* A unit small-scale value moves exactly the along-scan residuals of its
  CCD, interval and column, by one; nothing else.
* At the truth the noise-free residuals vanish; from the large-scale
  coefficients ~25 mas off and the small-scale values at zero (sources and
  attitude at the truth, no noise) one C update recovers every coefficient:
  the truth is a zero-residual point that satisfies eq:cc1 and eq:cc2, and
  the constrained problem has no other.  Also with the across-scan term.
* With noise and offsets the update is the plain definition, assembled here
  from the records independently of the oracle: per CCD and interval the
  weighted least squares of -R on the columns' indicators and the cells'
  L*_r(x), subject to eq:cc2 (for r = 0, 1, 2 the update's values times
  L*_r at the column centres sum to zero), written as its Lagrange system
  (constraint rows scaled to the normal matrix's diagonal) and solved by
  scipy's sparse LU; unknowns without records stay zero; then
  eq:calCon for eq:cc1 (each day's mean constant term removed).
* eq:cc2 holds for the updated values.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
import synth.configs as C

UAS, MAS = synth.UAS, synth.MAS
COLS = 1966


def _columns(w):
    """Each record's pixel column m = round(mu), as 0..1965."""
    return np.minimum(np.floor(w.mu.astype(np.float64) + 0.5), 1979).astype(np.int64) - 14


def _legendre(x):
    return np.stack([np.ones_like(x), 2.0 * x - 1.0, 6.0 * x * x - 6.0 * x + 1.0], axis=1)


@pytest.fixture(scope="module")
def small_world(oracle_lib):
    w = C.make("geo9", geo_small=True, noise=False)
    return w, oracle_lib.observed_field_angles(w)


def test_small_value_moves_its_column_only(oracle_lib, small_world):
    w, eta = small_world
    pr = oracle_lib.problem_from_world(w, eta, state="true")
    R0 = np.asarray(pr.observe()["R"]).copy()
    nl = w.geo_true.size
    k, n, m = 1, 4, 777
    g = pr.geo.copy()
    g[nl + (k * 9 + n) * COLS + m] += 1.0
    pr.set_state(geo=g)
    dR = np.asarray(pr.observe()["R"]) - R0
    mine = (w.cell >= 0) & (w.ccd == n) & ((w.cell // 2) // 30 == k) & (_columns(w) == m)
    assert mine.sum() > 0
    assert np.allclose(dR[mine], 1.0, rtol=0, atol=1e-15)
    assert np.array_equal(dR[~mine], np.zeros((~mine).sum()))


def _start_small_zero(oracle_lib, w, eta):
    """Sources and attitude at the truth, large-scale terms at their start
    values, small-scale values zero."""
    pr = oracle_lib.problem_from_world(w, eta, state="true")
    g = oracle_lib.world_geo(w, "start").copy()
    pr.set_state(geo=g)
    return pr


def test_residuals_vanish_and_update_recovers_the_truth(oracle_lib, small_world):
    w, eta = small_world
    pr = oracle_lib.problem_from_world(w, eta, state="true")
    assert np.abs(np.asarray(pr.observe()["R"])).max() < 1e-18
    pr = _start_small_zero(oracle_lib, w, eta)
    tru = oracle_lib.world_geo(w, "true")
    assert np.abs(pr.geo - tru).max() > 10 * MAS
    pr.calibration_update()
    err = np.abs(pr.geo - tru)
    print(f"after one C update: max |coefficient - truth| {err.max() / UAS:.2e} uas")
    assert err.max() < 1e-5 * UAS


def test_update_recovers_the_truth_with_the_ac_term(oracle_lib):
    w = C.make("geo9", geo_small=True, noise=False, ac_obs=True, geo_ac=True)
    eta = oracle_lib.observed_field_angles(w)
    pr = _start_small_zero(oracle_lib, w, eta)
    tru = oracle_lib.world_geo(w, "true")
    pr.calibration_update()
    err = np.abs(pr.geo - tru)
    print(f"with the AC term: max |coefficient - truth| {err.max() / UAS:.2e} uas")
    assert err.max() < 1e-5 * UAS


def _plain_update(w, R, W):
    """The constrained weighted least squares per CCD and interval (Lagrange
    system, sparse LU), then eq:calCon for eq:cc1."""
    nl = w.geo_true.size
    K = w.geo_small_true.shape[0]
    d = np.zeros(nl + w.geo_small_true.size)
    al = w.cell >= 0
    col = _columns(w)
    L = _legendre((w.mu.astype(np.float64) - 13.5) / 1966.0)
    Lm = _legendre((np.arange(14, 1980) - 13.5) / 1966.0)
    for k in range(K):
        c0, c1 = 60 * k, min(60 * (k + 1), w.n_cells)
        for n in range(9):
            sel = np.flatnonzero(al & (w.ccd == n) & (w.cell >= c0) & (w.cell < c1))
            nu = COLS + 3 * (c1 - c0)
            rows = np.repeat(np.arange(sel.size), 4)
            cols = np.stack([col[sel]] + [COLS + 3 * (w.cell[sel] - c0) + r for r in range(3)], 1).reshape(-1)
            vals = np.concatenate([np.ones((sel.size, 1)), L[sel]], 1).reshape(-1)
            J = sp.csr_matrix((vals, (rows, cols)), shape=(sel.size, nu))
            act = np.flatnonzero(np.asarray(J.getnnz(axis=0)) > 0)
            Ja = J[:, act]
            Nm = (Ja.T @ sp.diags(W[sel]) @ Ja).tocsc()
            b = -(Ja.T @ (W[sel] * R[sel]))
            Cm = np.zeros((act.size, 3))
            is_col = act < COLS
            # the constraint rows scaled to the normal matrix's diagonal (the
            # same solution; the multipliers scale by 1 / s)
            Cm[is_col] = Lm[act[is_col]] * np.median(Nm.diagonal())
            KKT = sp.bmat([[Nm, sp.csr_matrix(Cm)], [sp.csr_matrix(Cm.T), None]]).tocsc()
            x = spla.spsolve(KKT, np.concatenate([b, np.zeros(3)]))[: act.size]
            full = np.zeros(nu)
            full[act] = x
            d[nl + (k * 9 + n) * COLS: nl + (k * 9 + n + 1) * COLS] = full[:COLS]
            dl = d[:nl].reshape(w.n_cells, 9, 3)
            dl[c0:c1, n, :] = full[COLS:].reshape(-1, 3)
    dl = d[:nl].reshape(w.n_cells // 2, 18, 3)
    dl[:, :, 0] -= dl[:, :, 0].mean(axis=1)[:, None]
    return d


def test_update_is_the_constrained_lstsq_with_cc1(oracle_lib):
    w = C.make("geo9", geo_small=True)
    eta = oracle_lib.observed_field_angles(w)
    pr = oracle_lib.problem_from_world(w, eta, state="start")
    R = np.asarray(pr.observe()["R"])
    W = 1.0 / w.sigma.astype(np.float64) ** 2
    d = np.asarray(pr.calibration_update())
    ref = _plain_update(w, R, W)
    diff = np.abs(d - ref).max()
    print(f"oracle update vs the sparse Lagrange solve: max diff {diff / UAS:.2e} uas "
          f"(max |update| {np.abs(ref).max() / UAS:.3g} uas)")
    assert diff < 1e-9 * np.abs(ref).max()
    # eq:cc2 for the updated values (zero at the start)
    Lm = _legendre((np.arange(14, 1980) - 13.5) / 1966.0)
    small = np.asarray(pr.geo[w.geo_true.size:]).reshape(-1, COLS)
    scale = np.abs(small).sum(axis=1)
    assert np.all(np.abs(small @ Lm) <= 1e-12 * scale[:, None])
