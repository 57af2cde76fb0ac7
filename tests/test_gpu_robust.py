"""Parity of the robust mode (Sect. 5.1.2, 5.2.5) of the HIP library with the
oracle: excess attitude noise per bucket, the source inner iteration, and
iterations with robust attitude and calibration weights, on the tiny world
with 1% gross outliers (noise N(0, 50 mas)), with and without across-scan
records (then three excess-noise components per bucket and the initial
downweights per kind of record).  Same criterion as the plain parity tests:
the extended-precision oracle is the reference."""
import types

import numpy as np
import pytest

import synth
import synth.configs as C
from test_gpu_parity import Pair, agis_mod, check_floor, fp64_floor, report  # noqa: F401

pytestmark = pytest.mark.gpu

UAS = synth.UAS


@pytest.fixture(scope="module", params=["tiny_robust", "tiny_robust+ac"])
def tiny_robust(oracle_lib, request):
    w = C.make("tiny_robust", ac_obs=request.param.endswith("+ac"))
    return w, oracle_lib.observed_field_angles(w)


def eps_bound(w, e_o):
    """Bound on |GPU - oracle| of eps_a^2 per component and bucket: R^2 -
    sigma^2 carries the residuals' rounding, |d(R^2)| <= 2 |R| |dR| with
    |dR| < 1e-15 rad and |R| about (eps_a^2 + sigma^2)^1/2 at the quantile,
    times 2 for the two order statistics it interpolates; sigma of the
    component's records (along or across scan)."""
    nb = e_o.size // 3
    al = w.sigma[w.cell >= 0]
    ac = w.sigma[w.cell < 0]
    s = np.repeat([al.max() if al.size else 0.0, ac.max() if ac.size else 0.0, ac.max() if ac.size else 0.0], nb)
    return 4e-15 * np.sqrt(e_o + s.astype(np.float64) ** 2) + 2e-24


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
    nb = e_o.size // 3
    for c, name in enumerate(("AL", "ACP", "ACF")):
        ec = e_o[c * nb:(c + 1) * nb]
        print(f"eps_a {name}: buckets {nb}, nonzero {np.mean(ec > 0):.2f}, median {np.median(np.sqrt(ec)) / UAS:.2f} "
              f"uas, max |d eps_a^2|^(1/2) {d[c * nb:(c + 1) * nb].max():.2e} uas")
    assert np.all(np.abs(e_g - e_o) <= eps_bound(w, e_o))
    if not (w.cell < 0).any():
        assert np.all(e_g[nb:] == 0.0)
    p.close()


PATH_ENV = {"one kernel": {"AGIS_ROBUST_FUSED": "2"}, "columns": {"AGIS_ROBUST_FUSED": "0"},
            "rows then LDS": {"AGIS_ROBUST_FUSED": "3"}, "registers": {"AGIS_ROBUST_FUSED": "4"},
            "mixed": {"AGIS_ROBUST_FUSED": "2", "AGIS_ROBUST_MAX_CAP": "32"},
            "rows then LDS, mixed": {"AGIS_ROBUST_FUSED": "3", "AGIS_ROBUST_MAX_CAP": "32"},
            "registers, mixed": {"AGIS_ROBUST_FUSED": "4", "AGIS_ROBUST_MAX_CAP": "32"},
            "registers, one row per lane": {"AGIS_ROBUST_FUSED": "4", "AGIS_SREG_ROWS": "1",
                                            "AGIS_ROBUST_MAX_CAP": "300"},
            "columns, 32 lanes": {"AGIS_ROBUST_FUSED": "1", "AGIS_S_GROUP": "32"},
            "columns, 32 lanes, cached": {"AGIS_ROBUST_FUSED": "1", "AGIS_IRLS_CACHE": "1"},
            "columns, 64 lanes": {"AGIS_ROBUST_FUSED": "1", "AGIS_S_GROUP": "64"},
            "columns, 64 lanes, cached": {"AGIS_ROBUST_FUSED": "1", "AGIS_IRLS_CACHE": "2"}}
PATH_VARS = ("AGIS_ROBUST_FUSED", "AGIS_ROBUST_MAX_CAP", "AGIS_SREG_ROWS", "AGIS_S_GROUP", "AGIS_IRLS_CACHE")


@pytest.mark.parametrize("path", ["one kernel", "columns", "rows then LDS", "registers", "mixed",
                                  "rows then LDS, mixed", "registers, mixed"])
def test_robust_source_update_parity(agis_mod, oracle_lib, tiny_robust, path, monkeypatch):
    """The robust S update on its paths: every source in the one-kernel path
    (model, varsigma and solves per source in LDS), every source through HBM
    columns (three kernels; the default), the rows to HBM columns and then
    varsigma and the solves per source in LDS, every source with its rows
    in registers, and each of the on-chip paths with the sources of more
    than 32 observations on the column kernels."""
    w, eta = tiny_robust
    env = PATH_ENV[path]
    for k in PATH_VARS:
        monkeypatch.delenv(k, raising=False)
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    if path.endswith("mixed"):
        nobs = np.bincount(w.src, minlength=w.src_true.shape[0])
        assert (nobs > 32).any() and (nobs <= 32).any()

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


@pytest.fixture(scope="module")
def small9_robust(oracle_lib):
    w = C.make("small9", robust=True, outlier_frac=0.01, years=1.0, min_transits=6)
    return w, oracle_lib.observed_field_angles(w)


def test_irls_register_cache_is_bitwise(agis_mod, oracle_lib, small9_robust, monkeypatch):
    """The inner rounds with each lane's first eight records kept in
    registers take the records in the same order as the rounds that re-read
    them: 32 and 64 lanes per source, cached and not, the same sources bit
    for bit (the nine-CCD world: 54-351 records per source, so records
    beyond the cache at 32 lanes)."""
    w, eta = small9_robust
    out = {}
    for path in ("columns, 32 lanes", "columns, 32 lanes, cached", "columns, 64 lanes", "columns, 64 lanes, cached"):
        for k in PATH_VARS:
            monkeypatch.delenv(k, raising=False)
        for k, v in PATH_ENV[path].items():
            monkeypatch.setenv(k, v)
        p = Pair(agis_mod, oracle_lib, w, eta)
        agis_mod.agis_source_update(p.ctx)
        out[path] = p.gpu_state()[0]
        p.close()
    for k in PATH_VARS:
        monkeypatch.delenv(k, raising=False)
    assert np.array_equal(out["columns, 32 lanes"], out["columns, 32 lanes, cached"])
    assert np.array_equal(out["columns, 64 lanes"], out["columns, 64 lanes, cached"])


@pytest.mark.parametrize("path", ["registers, one row per lane", "columns", "columns, 64 lanes, cached"])
def test_robust_source_update_several_wavefronts(agis_mod, oracle_lib, small9_robust, path, monkeypatch):
    """The register path with a source spread over several wavefronts
    (one row per lane: 64 rows a wavefront; the nine-CCD world over one year
    with 1% outliers, stars with at least six transits, has 54-351
    observations per source, so up to five wavefronts a source, and the
    sources above 300 observations on the column kernels): the block-wide
    selection of varsigma and the block-wide sums of the inner rounds,
    against the oracle; and the column path on the same world, with and
    without the register cache of its inner rounds."""
    w, eta = small9_robust
    nobs = np.bincount(w.src, minlength=w.src_true.shape[0])
    assert (nobs > 300).any() and (nobs > 256).sum() > 100 and (nobs <= 64).any()
    for k in PATH_VARS:
        monkeypatch.delenv(k, raising=False)
    for k, v in PATH_ENV[path].items():
        monkeypatch.setenv(k, v)

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
    dg = check_floor(f"robust S update, {path}", X[0], O[0], G[0], tol[0], 0, mask=good)
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
    nb = 3 * ((w.knots.size - 7 + 7) // 8)      # buckets of 8 intervals, per AL, ACP, ACF
    for wrong in (nb // 3, nb + 1):
        with pytest.raises(agis_mod.AgisError) as e:
            agis_mod.agis_set_excess_noise(ctx, np.zeros(wrong))
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
    # the HBM-column kernels with the default choice, the lean kernel
    # everywhere and the register kernel everywhere; then the default paths
    # (the excess-noise estimate in one kernel, values and selection in LDS)
    names = ("AGIS_SELECT_REG_LIMIT", "AGIS_SELECT_REG_MIN_MEAN", "AGIS_ROBUST_FUSED")
    for env in ({"AGIS_ROBUST_FUSED": "0"}, {"AGIS_SELECT_REG_LIMIT": "0", "AGIS_ROBUST_FUSED": "0"},
                {"AGIS_SELECT_REG_MIN_MEAN": "0", "AGIS_ROBUST_FUSED": "0"}, {}):
        for k in names:
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
    for k in names:
        monkeypatch.delenv(k, raising=False)
    print(f"eps_bucket {eps_bucket}: {e_o.size} buckets; max |eps^2 GPU - oracle| {np.abs(out[0][0] - e_o).max():.2e}")
    for o in out[1:3]:
        assert np.array_equal(out[0][0], o[0]) and np.array_equal(out[0][1], o[1])
    # the same values and exact order statistics on the one-kernel path
    assert np.array_equal(out[0][0], out[3][0])
    assert np.all(np.abs(out[0][0] - e_o) <= eps_bound(w, e_o))
