"""Parity of the small-scale along-scan geometric calibration (eq:etazeta's
delta-eta with eq:cc2, Sect. 3.4; the C block of Sect. 5.3) of the HIP
library with the oracle, through the C ABI, on the 60-day nine-CCD world
(two 30-day long intervals, ~15 records per pixel column, CCD and interval).

* Residuals with non-zero small-scale values: within the residual bound of
  the plain parity test.
* One C update from the start values (large-scale terms ~25 mas off,
  small-scale values zero), with noise, with the along-scan terms, with the
  across-scan term too, and in robust mode with 1% outliers (the A/C
  weights downweight them): every coefficient within the FP64-floor
  criterion of the other parity tests (extended-precision oracle as
  reference); eq:cc1 and eq:cc2 hold.
* Two S[AC] iterations with the frame rotator, with across-scan records and
  all three terms, on the tiny world cut to 360 days (twelve whole 30-day
  intervals, ~15 records per column; its stars have at least six transits,
  which the 60-day world's do not: there the S block is ill-posed and the
  iteration diverges in the oracle as well): sources, attitude and
  coefficients within the criterion.
* The graph-replayed iteration is bitwise the eager one (same world).
* The arguments it refuses.
* With the Sun's light deflection and the global block too: two S[ACG]
  iterations on the same world, g0 included.
* A mixed-precision context's C update equals the FP64 context's.
"""
import numpy as np
import pytest

import synth
import synth.configs as C
from test_gpu_parity import agis_mod, check_floor, fp64_floor  # noqa: F401

pytestmark = pytest.mark.gpu

COLS = 1966
DAYS = 30


def _ctx(agis, w, eta, pr):
    """A context holding the oracle problem pr's state, with the geometry and
    the small-scale term."""
    ctx = agis.agis_create(w.consts, w.knots)
    agis.agis_load_observations(ctx, w.t, eta, w.sigma, w.src, w.fov, w.cell, w.src_true.shape[0], w.n_cells)
    agis.agis_load_geometry(ctx, w.ccd, w.mu, int(w.consts["geo_ccds"]), w.ac_cell,
                            int(w.consts.get("geo_ac_cells", 0)) if w.ac_cell is not None else 0,
                            small_days=int(w.consts["geo_small_days"]))
    agis.agis_set_sources(ctx, pr.s)
    agis.agis_set_attitude(ctx, pr.a)
    agis.agis_set_geo_calibration(ctx, pr.geo)
    return ctx


def _legendre_columns():
    x = (np.arange(14, 1980) - 13.5) / 1966.0
    return np.stack([np.ones_like(x), 2.0 * x - 1.0, 6.0 * x * x - 6.0 * x + 1.0], axis=1)


@pytest.fixture(scope="module", params=["AL terms", "AL and AC terms", "robust, AL and AC terms"])
def geo9_small(oracle_lib, request):
    both = "AC" in request.param
    robust = {"robust": True, "outlier_frac": 0.01} if request.param.startswith("robust") else {}
    w = C.make("geo9", geo_small=True, ac_obs=both, geo_ac=both, **robust)
    return w, oracle_lib.observed_field_angles(w)


def test_small_residuals(agis_mod, oracle_lib, geo9_small):
    w, eta = geo9_small
    pr = oracle_lib.problem_from_world(w, eta, state="start")
    pr.set_state(geo=oracle_lib.world_geo(w, "true"))        # non-zero small-scale values
    ctx = _ctx(agis_mod, w, eta, pr)
    R = agis_mod.agis_residuals(ctx)
    d = R - np.asarray(pr.observe()["R"])
    print(f"residuals with the small-scale term: max |GPU - oracle| {np.abs(d).max():.2e} rad, "
          f"rms {np.sqrt(np.mean(d * d)):.2e}")
    assert np.abs(d).max() < 1e-15 and np.sqrt(np.mean(d * d)) < 1.5e-16
    agis_mod.agis_destroy(ctx)


def test_small_calibration_update_parity(agis_mod, oracle_lib, geo9_small):
    w, eta = geo9_small

    def run(pr):
        pr.calibration_update()
        return pr.s.copy(), pr.a.copy(), pr.geo.copy()

    X, O, tol = fp64_floor(oracle_lib, w, eta, run)
    pr = oracle_lib.problem_from_world(w, eta, state="start")
    ctx = _ctx(agis_mod, w, eta, pr)
    agis_mod.agis_calibration_update(ctx)
    G = agis_mod.agis_get_geo_calibration(ctx, pr.geo.size)
    nl = pr.geo.size - w.geo_small_true.size
    check_floor("small-scale C update: large-scale coefficients", X[2][:nl], O[2][:nl], G[:nl], tol[2][:nl], 2)
    check_floor("small-scale C update: small-scale values", X[2][nl:], O[2][nl:], G[nl:], tol[2][nl:], 2)
    n_ccd = int(w.consts["geo_ccds"])
    n_al = w.geo_true.size // 3
    c0 = G[:nl].reshape(-1, 3)[:n_al, 0].reshape(-1, 2 * n_ccd)
    assert np.abs(c0.sum(axis=1)).max() < 1e-12 * np.abs(c0).max()              # eq:cc1
    small = G[nl:].reshape(-1, COLS)
    assert np.all(np.abs(small @ _legendre_columns()) <= 1e-12 * np.abs(small).sum(axis=1)[:, None])   # eq:cc2
    agis_mod.agis_destroy(ctx)


def _iter_world():
    return C.make("tiny", years=360 / 365.25, geo_cal=True, geo_small=True, ac_obs=True, geo_ac=True)


@pytest.fixture(scope="module")
def tiny_small(oracle_lib):
    w = _iter_world()
    return w, oracle_lib.observed_field_angles(w)


def test_small_iterations_parity(agis_mod, oracle_lib, tiny_small):
    w, eta = tiny_small
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
    check_floor("small-scale iterations: sources", X[0], O[0], G[0], tol[0], 0)
    check_floor("small-scale iterations: attitude", X[1], O[1], G[1], tol[1], 1)
    check_floor("small-scale iterations: coefficients", X[2], O[2], G[2], tol[2], 2)
    agis_mod.agis_destroy(ctx)


def test_small_graph_bitwise_and_refusals(agis_mod, oracle_lib, tiny_small):
    w, eta = tiny_small
    pr = oracle_lib.problem_from_world(w, eta, state="start")
    e, g = _ctx(agis_mod, w, eta, pr), _ctx(agis_mod, w, eta, pr)
    for c in (e, g):
        agis_mod.agis_set_frame_reference(c, w.src_true)
    agis_mod.agis_iterate(e, 4, stats=False)
    agis_mod.agis_iterate_graph(g, 2)
    agis_mod.agis_iterate(g, 1, stats=False)             # eager work between replays
    agis_mod.agis_iterate_graph(g, 1)
    for c in (e, g):
        assert np.all(np.isfinite(agis_mod.agis_get_geo_calibration(c, pr.geo.size)))
    for x, y, what in zip((agis_mod.agis_get_sources(e, w.src_true.shape[0]), agis_mod.agis_get_attitude(e, w.n_att),
                           agis_mod.agis_get_geo_calibration(e, pr.geo.size)),
                          (agis_mod.agis_get_sources(g, w.src_true.shape[0]), agis_mod.agis_get_attitude(g, w.n_att),
                           agis_mod.agis_get_geo_calibration(g, pr.geo.size)),
                          ("sources", "attitude", "coefficients")):
        assert np.array_equal(x, y), what
    n_ac = int(w.consts["geo_ac_cells"])
    for days in (-1, DAYS + 1):
        with pytest.raises(agis_mod.AgisError) as err:
            agis_mod.agis_load_geometry(e, w.ccd, w.mu, int(w.consts["geo_ccds"]), w.ac_cell, n_ac,
                                        small_days=days)
        assert err.value.code == -1
    # a refused argument changes nothing: the context still iterates with
    # the geometry it had, as its twin does
    agis_mod.agis_iterate(e, 1, stats=False)
    agis_mod.agis_iterate(g, 1, stats=False)
    assert np.array_equal(agis_mod.agis_get_geo_calibration(e, pr.geo.size),
                          agis_mod.agis_get_geo_calibration(g, pr.geo.size))
    with pytest.raises(agis_mod.AgisError):
        agis_mod.agis_set_geo_calibration(e, np.zeros(pr.geo.size - COLS))
    for c in (e, g):
        agis_mod.agis_destroy(c)


def test_small_with_global_block_parity(agis_mod, oracle_lib):
    """All three geometric terms with the Sun's light deflection and the
    global block (S[ACG], Sect. 5.4): two iterations with the frame rotator on
    the 360-day tiny world; sources, attitude, coefficients and g0 within the
    criterion (g0 by its per-parameter bound alone, as in the global-block
    tests)."""
    from test_gpu_ppn import check_g0
    w = C.make("tiny", years=360 / 365.25, geo_cal=True, geo_small=True, ac_obs=True, geo_ac=True, ppn=True)
    eta = oracle_lib.observed_field_angles(w)
    n_it = 2

    def run(pr):
        for _ in range(n_it):
            pr.iterate(s_ref=w.src_true)
        return pr.s.copy(), pr.a.copy(), np.concatenate([pr.geo, [pr.g0]])

    X, O, tol = fp64_floor(oracle_lib, w, eta, run)
    pr = oracle_lib.problem_from_world(w, eta, state="start")
    ctx = _ctx(agis_mod, w, eta, pr)
    agis_mod.agis_set_global(ctx, w.g0_start)
    agis_mod.agis_set_frame_reference(ctx, w.src_true)
    agis_mod.agis_iterate(ctx, n_it, stats=False)
    G = (agis_mod.agis_get_sources(ctx, w.src_true.shape[0]), agis_mod.agis_get_attitude(ctx, w.n_att),
         agis_mod.agis_get_geo_calibration(ctx, pr.geo.size))
    g0 = agis_mod.agis_get_global(ctx)[0]
    check_floor("geometric terms with S[ACG]: sources", X[0], O[0], G[0], tol[0], 0)
    check_floor("geometric terms with S[ACG]: attitude", X[1], O[1], G[1], tol[1], 1)
    check_floor("geometric terms with S[ACG]: coefficients", X[2][:-1], O[2][:-1], G[2], tol[2][:-1], 2)
    check_g0("geometric terms with S[ACG]: g0", float(X[2][-1]), float(O[2][-1]), g0, float(tol[2][-1]))
    agis_mod.agis_destroy(ctx)


def test_small_calibration_update_mixed_precision(agis_mod, oracle_lib):
    """The mixed-precision mode forms the attitude sums of the A/C pass in
    FP32 and keeps the model and the calibration's weights in FP64: one C
    update with all three geometric terms in a mixed context equals the FP64
    context's to rounding (1e-6 uas; the FP64 path itself is held to the
    oracle by the tests above)."""
    w = C.make("geo9", geo_small=True, ac_obs=True, geo_ac=True)
    eta = oracle_lib.observed_field_angles(w)
    pr = oracle_lib.problem_from_world(w, eta, state="start")
    out = []
    for prec in (agis_mod.AGIS_FP64, agis_mod.AGIS_MIXED):
        ctx = agis_mod.agis_create(w.consts, w.knots, precision=prec)
        agis_mod.agis_load_observations(ctx, w.t, eta, w.sigma, w.src, w.fov, w.cell, w.src_true.shape[0],
                                        w.n_cells)
        agis_mod.agis_load_geometry(ctx, w.ccd, w.mu, int(w.consts["geo_ccds"]), w.ac_cell,
                                    int(w.consts["geo_ac_cells"]), small_days=int(w.consts["geo_small_days"]))
        agis_mod.agis_set_sources(ctx, pr.s)
        agis_mod.agis_set_attitude(ctx, pr.a)
        agis_mod.agis_set_geo_calibration(ctx, pr.geo)
        agis_mod.agis_calibration_update(ctx)
        out.append(agis_mod.agis_get_geo_calibration(ctx, pr.geo.size))
        agis_mod.agis_destroy(ctx)
    d = np.abs(out[1] - out[0]).max() / synth.UAS
    print(f"geometric C update, mixed vs FP64 context: max diff {d:.2e} uas")
    assert d < 1e-6
