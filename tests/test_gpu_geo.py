"""Parity of the large-scale geometric calibration (eq:etazeta, Sect. 3.4;
the C block of Sect. 5.3 with eq:calCon for eq:cc1 and, with the across-scan
term, eq:cc3) of the HIP library with the oracle, through the C ABI, on
worlds with the along-scan term alone and with both terms.

* Residuals at the start values with the geometric terms (the observed
  angles the library stores carry them): within the residual bound of the
  plain parity test.
* One C update on the small nine-CCD world with noise and offsets: every
  coefficient within the FP64-floor criterion of the other parity tests
  (extended-precision oracle as reference), and eq:cc1 holds.
* Two S[AC] iterations with the frame rotator on the tiny world with
  across-scan records and the geometric model: sources, attitude and
  coefficients within the criterion.
* The graph-replayed iteration is bitwise the eager one, and device-memory
  inputs give the same residuals as host ones, bit for bit.
* The calls it refuses, and a bad CCD index or coordinate.
* The basic-angle monitor (eq:DeltaGamma) after a change of the basic
  angle in the observations.
"""
import numpy as np
import pytest

import synth
import synth.configs as C
from test_gpu_parity import agis_mod, check_floor, fp64_floor  # noqa: F401

pytestmark = pytest.mark.gpu

UAS = synth.UAS


def _ctx(agis, w, eta, pr):
    """A context holding the oracle problem pr's state, with the geometry."""
    ctx = agis.agis_create(w.consts, w.knots)
    agis.agis_load_observations(ctx, w.t, eta, w.sigma, w.src, w.fov, w.cell, w.src_true.shape[0], w.n_cells)
    agis.agis_load_geometry(ctx, w.ccd, w.mu, int(w.consts["geo_ccds"]), w.ac_cell,
                            int(w.consts.get("geo_ac_cells", 0)) if w.ac_cell is not None else 0)
    agis.agis_set_sources(ctx, pr.s)
    agis.agis_set_attitude(ctx, pr.a)
    agis.agis_set_geo_calibration(ctx, pr.geo)
    return ctx


@pytest.fixture(scope="module", params=["AL term", "AL and AC terms"])
def small9_geo(oracle_lib, request):
    both = request.param == "AL and AC terms"
    w = C.make("small9", geo_cal=True, ac_obs=both, geo_ac=both)
    return w, oracle_lib.observed_field_angles(w)


def test_geo_residuals(agis_mod, oracle_lib, small9_geo):
    w, eta = small9_geo
    pr = oracle_lib.problem_from_world(w, eta, state="start")
    ctx = _ctx(agis_mod, w, eta, pr)
    R = agis_mod.agis_residuals(ctx)
    d = R - np.asarray(pr.observe()["R"])
    print(f"geometric residuals: max |GPU - oracle| {np.abs(d).max():.2e} rad, rms {np.sqrt(np.mean(d * d)):.2e}")
    assert np.abs(d).max() < 1e-15 and np.sqrt(np.mean(d * d)) < 1.5e-16
    agis_mod.agis_destroy(ctx)


def test_geo_calibration_update_parity(agis_mod, oracle_lib, small9_geo):
    w, eta = small9_geo

    def run(pr):
        pr.calibration_update()
        return pr.s.copy(), pr.a.copy(), pr.geo.copy()

    X, O, tol = fp64_floor(oracle_lib, w, eta, run)
    pr = oracle_lib.problem_from_world(w, eta, state="start")
    ctx = _ctx(agis_mod, w, eta, pr)
    agis_mod.agis_calibration_update(ctx)
    G = agis_mod.agis_get_geo_calibration(ctx, pr.geo.size)
    check_floor("geometric C update", X[2], O[2], G, tol[2], 2)
    n_ccd = int(w.consts["geo_ccds"])
    n_al = w.geo_true.size // 3
    c0 = G.reshape(-1, 3)[:n_al, 0].reshape(-1, 2 * n_ccd)
    assert np.abs(c0.sum(axis=1)).max() < 1e-12 * np.abs(c0).max()              # eq:cc1
    if w.ac_cell is not None:
        a0 = G.reshape(-1, 3)[n_al:, 0].reshape(-1, n_ccd)
        assert np.abs(a0.sum(axis=1)).max() < 1e-12 * np.abs(a0).max()          # eq:cc3
    agis_mod.agis_destroy(ctx)


@pytest.mark.parametrize("both", [False, True], ids=["AL term", "AL and AC terms"])
def test_geo_iterations_parity(agis_mod, oracle_lib, both):
    w = C.make("tiny", geo_cal=True, ac_obs=True, geo_ac=both)
    eta = oracle_lib.observed_field_angles(w)
    n_it = 2

    def run(pr):
        for _ in range(n_it):
            pr.iterate(s_ref=w.src_true)
        return pr.s.copy(), pr.a.copy(), pr.geo.copy()

    X, O, tol = fp64_floor(oracle_lib, w, eta, run)
    pr = oracle_lib.problem_from_world(w, eta, state="start")
    ctx = _ctx(agis_mod, w, eta, pr)
    agis_mod.agis_set_frame_reference(ctx, w.src_true)
    agis_mod.agis_iterate(ctx, n_it, stats=False)
    G = (agis_mod.agis_get_sources(ctx, w.src_true.shape[0]), agis_mod.agis_get_attitude(ctx, w.n_att),
         agis_mod.agis_get_geo_calibration(ctx, pr.geo.size))
    check_floor("geometric iterations: sources", X[0], O[0], G[0], tol[0], 0)
    check_floor("geometric iterations: attitude", X[1], O[1], G[1], tol[1], 1)
    check_floor("geometric iterations: coefficients", X[2], O[2], G[2], tol[2], 2)
    # the cell offsets stay zero
    assert np.all(agis_mod.agis_get_calibration(ctx, w.n_cells) == 0.0)
    agis_mod.agis_destroy(ctx)


def test_geo_graph_and_device_inputs(agis_mod, oracle_lib):
    import torch
    w = C.make("tiny", geo_cal=True, ac_obs=True)
    eta = oracle_lib.observed_field_angles(w)
    pr = oracle_lib.problem_from_world(w, eta, state="start")
    e, g = _ctx(agis_mod, w, eta, pr), _ctx(agis_mod, w, eta, pr)
    for c in (e, g):
        agis_mod.agis_set_frame_reference(c, w.src_true)
    agis_mod.agis_iterate(e, 4, stats=False)
    agis_mod.agis_iterate_graph(g, 2)
    agis_mod.agis_iterate(g, 1, stats=False)             # eager work between replays
    agis_mod.agis_iterate_graph(g, 1)

    def state(c):
        return (agis_mod.agis_get_sources(c, w.src_true.shape[0]), agis_mod.agis_get_attitude(c, w.n_att),
                agis_mod.agis_get_geo_calibration(c, pr.geo.size))
    for x, y, what in zip(state(e), state(g), ("sources", "attitude", "coefficients")):
        assert np.array_equal(x, y), what
    # the geometry from device memory
    d = agis_mod.agis_create(w.consts, w.knots)
    agis_mod.agis_load_observations(d, w.t, eta, w.sigma, w.src, w.fov, w.cell, w.src_true.shape[0], w.n_cells)
    agis_mod.agis_load_geometry(d, torch.from_numpy(w.ccd).cuda(), torch.from_numpy(w.mu).cuda(),
                                int(w.consts["geo_ccds"]))
    h = _ctx(agis_mod, w, eta, pr)
    for c in (d, h):
        agis_mod.agis_set_sources(c, pr.s)
        agis_mod.agis_set_attitude(c, pr.a)
        agis_mod.agis_set_geo_calibration(c, w.geo_true)
    assert np.array_equal(agis_mod.agis_residuals(d), agis_mod.agis_residuals(h))
    for c in (e, g, d, h):
        agis_mod.agis_destroy(c)


def test_geo_refusals(agis_mod, oracle_lib, small9_geo):
    w, eta = small9_geo
    pr = oracle_lib.problem_from_world(w, eta, state="start")
    ctx = _ctx(agis_mod, w, eta, pr)
    for call in (lambda: agis_mod.agis_set_calibration(ctx, np.zeros(w.n_cells)),
                 lambda: agis_mod.agis_cg_iterate(ctx, 1, 40),
                 lambda: agis_mod.agis_learned_reset(ctx)):
        with pytest.raises(agis_mod.AgisError) as e:
            call()
        assert e.value.code == -7
    with pytest.raises(agis_mod.AgisError):
        agis_mod.agis_get_geo_calibration(ctx, pr.geo.size + 1)
    bad = w.ccd.copy()
    bad[np.flatnonzero(w.cell >= 0)[0]] = 9
    with pytest.raises(agis_mod.AgisError):
        agis_mod.agis_load_geometry(ctx, bad, w.mu, 9)
    mu = w.mu.copy()
    mu[np.flatnonzero(w.cell >= 0)[0]] = 2000.0
    with pytest.raises(agis_mod.AgisError):
        agis_mod.agis_load_geometry(ctx, w.ccd, mu, 9)
    if w.ac_cell is not None:
        ac = w.ac_cell.copy()
        ac[np.flatnonzero(w.cell < 0)[0]] = int(w.consts["geo_ac_cells"])
        with pytest.raises(agis_mod.AgisError):
            agis_mod.agis_load_geometry(ctx, w.ccd, w.mu, 9, ac, int(w.consts["geo_ac_cells"]))
    # a rejected geometry leaves the cell offsets in use, at zero, and the
    # observed angles as loaded
    assert np.all(agis_mod.agis_get_calibration(ctx, w.n_cells) == 0.0)
    agis_mod.agis_set_calibration(ctx, np.zeros(w.n_cells))
    plain = oracle_lib.problem_from_world(w, eta, state="start")
    plain.set_state(c=np.zeros(w.n_cells), geo=np.zeros_like(pr.geo))
    R = agis_mod.agis_residuals(ctx)
    assert np.abs(R - np.asarray(plain.observe()["R"])).max() < 1e-15
    agis_mod.agis_destroy(ctx)


def test_basic_angle_monitor(agis_mod, oracle_lib):
    """eq:DeltaGamma through the C ABI: observations made with the basic angle
    Gamma_c + 1 mas, one C update by the library at the truth: the library's
    monitor equals the oracle's formula applied to the library's own
    coefficients (to rounding), and it moved by +1 mas on every day (to 1e-6,
    as the oracle's pin)."""
    import copy
    w = C.make("small9", geo_cal=True, noise=False)
    delta = 1.0 * synth.MAS
    wd = copy.copy(w)
    wd.consts = dict(w.consts, gamma_c=w.consts["gamma_c"] + delta)
    eta = oracle_lib.observed_field_angles(wd)
    pr = oracle_lib.problem_from_world(w, eta, state="true")
    ctx = _ctx(agis_mod, w, eta, pr)
    n_days, n_ccd = w.n_cells // 2, int(w.consts["geo_ccds"])
    before = agis_mod.agis_basic_angle(ctx, n_days)
    agis_mod.agis_calibration_update(ctx)
    after = agis_mod.agis_basic_angle(ctx, n_days)
    G = agis_mod.agis_get_geo_calibration(ctx, pr.geo.size)
    ref = oracle_lib.basic_angle(G, w.n_cells, n_ccd)
    print(f"monitor vs the formula on the library's coefficients: max diff {np.abs(after - ref).max():.2e} rad; "
          f"moved by {np.mean(after - before) / synth.MAS:.9f} mas")
    assert np.abs(after - ref).max() <= 1e-15 * max(np.abs(ref).max(), 1e-30)
    seen = np.bincount(w.cell[w.cell >= 0] // 2, minlength=n_days) > 0
    assert np.allclose((after - before)[seen], delta, rtol=1e-6, atol=0)
    with pytest.raises(agis_mod.AgisError) as e:
        agis_mod.agis_basic_angle(ctx, n_days + 1)
    assert e.value.code == -2
    agis_mod.agis_destroy(ctx)
