"""Parity at full size of the geometric calibration (eq:etazeta, Sect. 3.4;
the C block of Sect. 5.3 with eq:calCon for eq:cc1 and eq:cc3, and eq:cc2):
the 1M-source / 1-year / 9-CCD workload with one across-scan record per
transit and all three terms (3 coefficients per cell and CCD along scan, the
small-scale values per CCD, 30-day interval and pixel column, 3 coefficients
per AC cell of 30 days and CCD across scan; 178.8M records), loaded as the
benchmark's --geo --geo-small --ac run loads it, on sampled outputs.

The oracle computes each sampled output from a sub-world that holds exactly
the records it depends on: residuals at 4,096 sampled records; the C update
at the start values of two sampled (CCD, interval) blocks (the block's
along-scan records: its 1966 small-scale values and its cells' linear and
quadratic coefficients, which eq:cc1's day means over all CCDs do not
touch) and of the AC groups of two sampled AC cells (the AC records of the
cell).  With the plain weights W = 1 / sigma^2 a block's (group's) update
depends on its own records only, and eq:cc3 couples only the groups of one
AC cell.  Criterion: as in the small-world parity tests, the FP64 floor of
the extended-precision oracle.
"""
import numpy as np
import pytest

import synth.configs as C
from oracle import world_geo
from test_gpu_fullsize import subworld
from test_gpu_parity import agis_mod, check_floor, fp64_floor  # noqa: F401

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1200)]


@pytest.fixture(scope="module")
def full_geo(oracle_lib, agis_mod):
    w = C.make("gaia1", ac_obs=True, geo_cal=True, geo_ac=True, geo_small=True)
    print(f"gaia1+ac+geo: {w.n_obs} records, {w.n_cells} cells, {int(w.consts['geo_ac_cells'])} AC cells, "
          f"{w.geo_small_true.size} small-scale values", flush=True)
    eta = oracle_lib.observed_field_angles(w)
    print("gaia1+ac+geo: observed angles from the oracle's model", flush=True)
    ctx = agis_mod.agis_create(w.consts, w.knots)
    agis_mod.agis_load_observations(ctx, w.t, eta, w.sigma, w.src, w.fov, w.cell, w.src_true.shape[0], w.n_cells)
    agis_mod.agis_load_geometry(ctx, w.ccd, w.mu, int(w.consts["geo_ccds"]), w.ac_cell,
                                int(w.consts["geo_ac_cells"]), small_days=int(w.consts["geo_small_days"]))
    w.eta_nominal = None
    yield w, eta, ctx
    agis_mod.agis_destroy(ctx)


def _start(agis, ctx, w):
    agis.agis_set_sources(ctx, w.src_start)
    agis.agis_set_attitude(ctx, w.att_start)
    agis.agis_set_geo_calibration(ctx, world_geo(w, "start"))


def test_fullsize_geo_residuals(agis_mod, oracle_lib, full_geo):
    w, eta, ctx = full_geo
    _start(agis_mod, ctx, w)
    R = agis_mod.agis_residuals(ctx)
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(w.n_obs, 4096, replace=False))
    sub = subworld(w, idx)
    Ro = oracle_lib.problem_from_world(sub, eta[idx], state="start").observe()["R"]
    d = R[idx] - Ro
    print(f"residuals at {idx.size} sampled records ({(w.cell[idx] < 0).sum()} across scan): "
          f"max |GPU - oracle| {np.abs(d).max():.2e} rad, rms {np.sqrt(np.mean(d * d)):.2e} rad")
    assert np.sqrt(np.mean(d * d)) < 1.5e-16 and np.abs(d).max() < 1e-15


def test_fullsize_geo_calibration_update(agis_mod, oracle_lib, full_geo):
    w, eta, ctx = full_geo
    _start(agis_mod, ctx, w)
    agis_mod.agis_calibration_update(ctx)
    n_ccd, n_ac = int(w.consts["geo_ccds"]), int(w.consts["geo_ac_cells"])
    n_small = w.geo_small_true.size
    G = agis_mod.agis_get_geo_calibration(ctx, 3 * (w.n_cells + n_ac) * n_ccd + n_small)
    n_al = 3 * w.n_cells * n_ccd
    small0 = 3 * (w.n_cells + n_ac) * n_ccd
    days = int(w.consts["geo_small_days"])
    rng = np.random.default_rng(19)

    def run(pr):
        pr.calibration_update()
        return pr.s.copy(), pr.a.copy(), pr.geo.copy()

    # eq:cc1 over every day
    c0 = G[:n_al].reshape(-1, 2 * n_ccd, 3)[:, :, 0]
    assert np.abs(c0.sum(axis=1)).max() < 1e-12 * np.abs(c0).max()
    # two sampled (CCD, interval) blocks, whole intervals
    n_k = (w.n_cells // 2) // days
    for k, n in zip(sorted(rng.choice(np.arange(n_k), 2, replace=False)), rng.choice(n_ccd, 2, replace=False)):
        c_lo, c_hi = 2 * days * k, 2 * days * (k + 1)
        idx = np.flatnonzero((w.cell >= c_lo) & (w.cell < c_hi) & (w.ccd == n))
        X, O, tol = fp64_floor(oracle_lib, subworld(w, idx), eta[idx], run)
        sel = small0 + (k * n_ccd + n) * 1966 + np.arange(1966)
        check_floor(f"small-scale C update, CCD {n}, interval {k} ({idx.size} records)",
                    X[2][sel], O[2][sel], G[sel], tol[2][sel], 2)
        lq = (3 * (np.arange(c_lo, c_hi)[:, None] * n_ccd + n) + np.array([1, 2])[None, :]).reshape(-1)
        check_floor(f"its cells' linear and quadratic coefficients ({lq.size})",
                    X[2][lq], O[2][lq], G[lq], tol[2][lq], 2)
    # the AC groups of two sampled AC cells
    for cell in sorted(rng.choice(np.arange(1, n_ac - 1), 2, replace=False)):
        idx = np.flatnonzero(w.ac_cell == cell)
        X, O, tol = fp64_floor(oracle_lib, subworld(w, idx), eta[idx], run)
        sel = n_al + np.arange(3 * cell * n_ccd, 3 * (cell + 1) * n_ccd)
        check_floor(f"AC geometric C update, AC cell {cell} ({idx.size} records, {sel.size} coefficients)",
                    X[2][sel], O[2][sel], G[sel], tol[2][sel], 2)
        c0 = G[sel].reshape(-1, 3)[:, 0]
        assert abs(c0.sum()) < 1e-12 * np.abs(c0).max()                       # eq:cc3
