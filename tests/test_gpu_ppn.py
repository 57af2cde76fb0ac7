"""Parity of the global block (Sect. 5.4, eq:normG) with the PPN parameter
gamma = 1 + g0 (eq:gammaPPN) and the Sun's light deflection in the model
(eq:astro), of the HIP library with the oracle, through the C ABI.

* Residuals with the deflection at the start values (g0 = 1e-3): within the
  residual bound of the plain parity test.
* One global update (g0 with the pseudo-parameter g1): g0 within the
  FP64-floor criterion of the other parity tests (extended-precision oracle
  as the reference).
* Two S[ACG] + frame iterations on the tiny world, plain and robust (1%
  outliers): sources, attitude, calibration and g0 within the criterion.
* The graph-replayed iteration is bitwise the eager one; the refused calls
  and configurations.
"""
import numpy as np
import pytest

import synth.configs as C
from test_gpu_parity import Pair, agis_mod, check_floor, fp64_floor, report  # noqa: F401

pytestmark = pytest.mark.gpu


def check_g0(name, x, o, g, tol):
    """g0 against the extended-precision reference x: within its FP64-floor
    tolerance (24 times the estimated sensitivity, as for every parameter);
    the RMS comparison with the FP64 oracle is a statistic over many
    parameters and is not applied to this single one."""
    dg, do = np.array([(g - x) / 4.8481368e-12]), np.array([(o - x) / 4.8481368e-12])
    report(f"{name} (GPU - ext)", dg, np.array([tol]))
    report(f"{name} (FP64 oracle - ext)", do, np.array([tol]))
    assert abs(dg[0]) <= tol


@pytest.fixture(scope="module", params=["tiny", "tiny_robust"])
def ppn_world(oracle_lib, request):
    w = C.make(request.param, ppn=True)
    return w, oracle_lib.observed_field_angles(w)


def _pair(agis, oracle_lib, w, eta):
    p = Pair(agis, oracle_lib, w, eta)
    agis.agis_set_global(p.ctx, w.g0_start)
    return p


def test_ppn_residuals(agis_mod, oracle_lib, ppn_world):
    w, eta = ppn_world
    p = _pair(agis_mod, oracle_lib, w, eta)
    assert agis_mod.agis_get_global(p.ctx)[0] == w.g0_start == p.pr.g0
    d = agis_mod.agis_residuals(p.ctx) - np.asarray(p.pr.observe()["R"])
    print(f"residuals with the deflection: max |GPU - oracle| {np.abs(d).max():.2e} rad, "
          f"rms {np.sqrt(np.mean(d * d)):.2e}")
    assert np.abs(d).max() < 1e-15 and np.sqrt(np.mean(d * d)) < 1.5e-16
    p.close()


def test_ppn_global_update_parity(agis_mod, oracle_lib, ppn_world):
    w, eta = ppn_world

    def run(pr):
        pr.global_update()
        return pr.s.copy(), pr.a.copy(), np.array([pr.g0])

    X, O, tol = fp64_floor(oracle_lib, w, eta, run)
    p = _pair(agis_mod, oracle_lib, w, eta)
    dg0, g1 = agis_mod.agis_global_update(p.ctx)
    g0 = agis_mod.agis_get_global(p.ctx)[0]
    print(f"global update: d g0 {dg0:.6e}, g1 {g1:.3e}, g0 {g0:.6e} (extended oracle {float(X[2][0]):.6e})")
    check_g0("g0 after one global update", float(X[2][0]), float(O[2][0]), g0, float(tol[2][0]))
    p.close()


def test_ppn_iterations_parity(agis_mod, oracle_lib, ppn_world):
    w, eta = ppn_world
    n_it = 2

    def run(pr):
        for _ in range(n_it):
            pr.iterate(s_ref=w.src_true)
        run.g0 = pr.g0
        return pr.s.copy(), pr.a.copy(), np.concatenate([pr.c, [pr.g0]])

    X, O, tol = fp64_floor(oracle_lib, w, eta, run)
    p = _pair(agis_mod, oracle_lib, w, eta)
    agis_mod.agis_set_frame_reference(p.ctx, w.src_true)
    agis_mod.agis_iterate(p.ctx, n_it, stats=False)
    G = p.gpu_state()
    g0 = agis_mod.agis_get_global(p.ctx)[0]
    print(f"g0 after {n_it} S[ACG] iterations: GPU {g0:.6e}, extended oracle {float(X[2][-1]):.6e}")
    check_floor("S[ACG] iterations: sources", X[0], O[0], G[0], tol[0], 0)
    check_floor("S[ACG] iterations: attitude", X[1], O[1], G[1], tol[1], 1)
    check_floor("S[ACG] iterations: calibration", X[2][:-1], O[2][:-1], G[2], tol[2][:-1], 2)
    check_g0("S[ACG] iterations: g0", float(X[2][-1]), float(O[2][-1]), g0, float(tol[2][-1]))
    p.close()


def test_ppn_graph_and_refusals(agis_mod, oracle_lib):
    w = C.make("tiny", ppn=True)
    eta = oracle_lib.observed_field_angles(w)
    e, g = _pair(agis_mod, oracle_lib, w, eta), _pair(agis_mod, oracle_lib, w, eta)
    for p in (e, g):
        agis_mod.agis_set_frame_reference(p.ctx, w.src_true)
    agis_mod.agis_iterate(e.ctx, 3, stats=False)
    agis_mod.agis_iterate_graph(g.ctx, 2)
    agis_mod.agis_iterate(g.ctx, 1, stats=False)
    for x, y in zip(e.gpu_state(), g.gpu_state()):
        assert np.array_equal(x, y)
    assert agis_mod.agis_get_global(e.ctx) == agis_mod.agis_get_global(g.ctx)
    for call in (lambda: agis_mod.agis_cg_iterate(e.ctx, 1, 40), lambda: agis_mod.agis_learned_reset(e.ctx)):
        with pytest.raises(agis_mod.AgisError) as err:
            call()
        assert err.value.code == -7
    e.close()
    g.close()
    # the global block needs the deflection; the deflection runs in FP64 only
    for over, prec in (({"ppn": 1, "defl": 0.0}, 0), ({}, 1)):
        consts = dict(w.consts)
        consts.update(over)
        with pytest.raises(agis_mod.AgisError):
            agis_mod.agis_create(consts, w.knots, precision=prec)
    # a robust context with the deflection refuses to freeze its weights
    wr = C.make("tiny_robust", ppn=True)
    r = agis_mod.agis_create(wr.consts, wr.knots)
    agis_mod.agis_load_observations(r, wr.t, np.zeros(wr.n_obs), wr.sigma, wr.src, wr.fov, wr.cell,
                                    wr.src_true.shape[0], wr.n_cells)
    with pytest.raises(agis_mod.AgisError):
        agis_mod.agis_freeze_weights(r, 1)
    agis_mod.agis_destroy(r)
