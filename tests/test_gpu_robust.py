"""Parity of the robust mode (Sect. 5.1.2, 5.2.5) of the HIP library with the
oracle: excess attitude noise per bucket, the source inner iteration, and
iterations with robust attitude and calibration weights, on the tiny world
with 1% gross outliers (noise N(0, 50 mas)).  Same criterion as the plain
parity tests: the extended-precision oracle is the reference."""
import types

import numpy as np
import pytest

import synth
import synth.configs as C
from test_gpu_parity import Pair, agis_mod, check_floor, fp64_floor, report  # noqa: F401

pytestmark = pytest.mark.gpu

UAS = synth.UAS


@pytest.fixture(scope="module")
def tiny_robust(oracle_lib):
    w = C.make("tiny_robust")
    return w, oracle_lib.observed_field_angles(w)


def test_excess_noise_parity(agis_mod, oracle_lib, tiny_robust):
    w, eta = tiny_robust
    p = Pair(agis_mod, oracle_lib, w, eta, state="truth")
    agis_mod.agis_set_sources(p.ctx, w.src_true)
    agis_mod.agis_set_attitude(p.ctx, w.att_true)
    agis_mod.agis_set_calibration(p.ctx, w.cal_true)
    e_o = p.pr.excess_attitude_noise()
    agis_mod.agis_excess_noise_update(p.ctx)
    e_g = agis_mod.agis_get_excess_noise(p.ctx, e_o.size)
    d = np.sqrt(np.abs(e_g - e_o)) / UAS
    print(f"eps_a: buckets {e_o.size}, nonzero {np.mean(e_o > 0):.2f}, median {np.median(np.sqrt(e_o)) / UAS:.2f} uas, "
          f"max |d eps_a^2|^(1/2) {d.max():.2e} uas")
    # R^2 - sigma^2 with |R| ~ 100 uas carries the residuals' rounding
    # (|dR| < 1e-15 rad): |d(R^2)| < 2 |R| |dR| ~ 1e-24 rad^2
    assert np.all(np.abs(e_g - e_o) <= 2e-24)
    p.close()


def test_robust_source_update_parity(agis_mod, oracle_lib, tiny_robust):
    w, eta = tiny_robust

    def run(pr):
        _, _, de = pr.source_update()
        run.defect = de
        return pr.s.copy(), pr.a.copy(), pr.c.copy()

    X, O, tol = fp64_floor(oracle_lib, w, eta, run)
    run(oracle_lib.problem_from_world(w, eta, state="start"))
    good = run.defect == 0
    p = Pair(agis_mod, oracle_lib, w, eta)
    agis_mod.agis_source_update(p.ctx)
    G = p.gpu_state()
    dg = check_floor("robust S update", X[0], O[0], G[0], tol[0], 0, mask=good)
    assert np.mean(np.abs(dg) <= 1e-3) > 0.95
    p.close()


def test_robust_iterations_parity(agis_mod, oracle_lib, tiny_robust):
    """Two robust S[AC] iterations with the frame rotator: sources, attitude,
    calibration and the excess attitude noise."""
    w, eta = tiny_robust
    n_it = 2

    def run(pr):
        for _ in range(n_it):
            pr.iterate(s_ref=w.src_true)
        run.eps = np.asarray(pr.eps_a2, np.float64).copy()
        return pr.s.copy(), pr.a.copy(), pr.c.copy()

    X, O, tol = fp64_floor(oracle_lib, w, eta, run)
    run(oracle_lib.problem_from_world(w, eta, state="start"))
    e_o = run.eps
    p = Pair(agis_mod, oracle_lib, w, eta)
    agis_mod.agis_set_frame_reference(p.ctx, w.src_true)
    agis_mod.agis_iterate(p.ctx, n_it)
    G = p.gpu_state()
    check_floor("robust iterations: sources", X[0], O[0], G[0], tol[0], 0)
    check_floor("robust iterations: attitude", X[1], O[1], G[1], tol[1], 1)
    check_floor("robust iterations: calibration", X[2], O[2], G[2], tol[2], 2)
    e_g = agis_mod.agis_get_excess_noise(p.ctx, e_o.size)
    rel = np.abs(np.sqrt(e_g) - np.sqrt(e_o)) / UAS
    print(f"robust iterations: eps_a median {np.median(np.sqrt(e_o)) / UAS:.3f} uas, max diff {rel.max():.2e} uas")
    assert rel.max() < 1e-2
    p.close()


def test_robust_mode_calls(agis_mod, oracle_lib, tiny_robust):
    w, eta = tiny_robust
    plain = C.make("small")
    ctx = agis_mod.agis_create(plain.consts, plain.knots)
    with pytest.raises(agis_mod.AgisError) as e:
        agis_mod.agis_excess_noise_update(ctx)
    assert e.value.code == -7
    agis_mod.agis_destroy(ctx)
    bad = dict(w.consts)
    bad["eps_bucket"] = 0
    with pytest.raises(agis_mod.AgisError):
        agis_mod.agis_create(bad, w.knots)
    ctx = agis_mod.agis_create(w.consts, w.knots)
    nb = (w.knots.size - 7 + 7) // 8
    with pytest.raises(agis_mod.AgisError) as e:
        agis_mod.agis_set_excess_noise(ctx, np.zeros(nb + 1))
    assert e.value.code == -2
    agis_mod.agis_set_excess_noise(ctx, np.full(nb, 1e-20))
    assert np.all(agis_mod.agis_get_excess_noise(ctx, nb) == 1e-20)
    agis_mod.agis_destroy(ctx)


@pytest.mark.parametrize("eps_bucket", [8, 100, 200])
def test_quantile_paths_agree(agis_mod, oracle_lib, tiny_robust, eps_bucket, monkeypatch):
    """The exact quantiles from register-held keys (sets up to 2,048, in the
    register kernel) and from keys re-read on every radix pass (larger sets,
    and every set in the lean kernel) are the same numbers: with the default
    kernel choice, the lean kernel forced everywhere and the register kernel
    forced everywhere, the robust S update and the excess noise agree bit
    for bit, and the noise agrees with the oracle.
    Buckets of 8, 100 and 200 intervals hold ~100, ~1,300 and ~2,600
    observations (the last beyond the register capacity)."""
    w, eta = tiny_robust
    consts = dict(w.consts)
    consts["eps_bucket"] = eps_bucket
    wb = types.SimpleNamespace(**{**vars(w), "consts": consts, "n_cells": w.n_cells, "n_att": w.n_att,
                                  "n_obs": w.n_obs})
    out = []
    # default choice; the lean kernel everywhere; the register kernel everywhere
    for env in ({}, {"AGIS_SELECT_REG_LIMIT": "0"}, {"AGIS_SELECT_REG_MIN_MEAN": "0"}):
        for k in ("AGIS_SELECT_REG_LIMIT", "AGIS_SELECT_REG_MIN_MEAN"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        p = Pair(agis_mod, oracle_lib, wb, eta, state="truth")
        agis_mod.agis_excess_noise_update(p.ctx)
        e_g = agis_mod.agis_get_excess_noise(p.ctx, p.pr.eps_a2.size)
        agis_mod.agis_set_sources(p.ctx, w.src_start)
        agis_mod.agis_source_update(p.ctx)
        out.append((e_g, p.gpu_state()[0]))
        if not env:
            e_o = p.pr.excess_attitude_noise()
        p.close()
    for k in ("AGIS_SELECT_REG_LIMIT", "AGIS_SELECT_REG_MIN_MEAN"):
        monkeypatch.delenv(k, raising=False)
    print(f"eps_bucket {eps_bucket}: {e_o.size} buckets; max |eps^2 GPU - oracle| {np.abs(out[0][0] - e_o).max():.2e}")
    for o in out[1:]:
        assert np.array_equal(out[0][0], o[0]) and np.array_equal(out[0][1], o[1])
    assert np.all(np.abs(out[0][0] - e_o) <= 2e-24)
