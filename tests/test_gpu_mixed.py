"""Mixed precision (FP32 partials and compensated FP32 normal-matrix sums;
FP64 right-hand sides, model and solves) against FP64: one source update against the FP64 oracle, and
the iterate after many S[AC] + frame iterations against the FP64 path (itself
at parity with the oracle).  The error is reported in uas per class."""
import numpy as np
import pytest

import synth
import synth.configs as C
from test_gpu_parity import agis_mod, rot_diff_uas, src_diff_uas  # noqa: F401

pytestmark = pytest.mark.gpu

UAS = synth.UAS
AGIS_MIXED = 1


@pytest.fixture(scope="module")
def tiny(oracle_lib):
    w = C.make("tiny")
    return w, oracle_lib.observed_field_angles(w)


def _ctx(agis, w, eta, precision, s, a, c):
    ctx = agis.agis_create(w.consts, w.knots, precision=precision)
    agis.agis_load_observations(ctx, w.t, eta, w.sigma, w.src, w.fov, w.cell, w.src_true.shape[0], w.n_cells)
    agis.agis_set_sources(ctx, s)
    agis.agis_set_attitude(ctx, a)
    agis.agis_set_calibration(ctx, c)
    return ctx


def _state(agis, ctx, w):
    return (agis.agis_get_sources(ctx, w.src_true.shape[0]), agis.agis_get_attitude(ctx, w.n_att),
            agis.agis_get_calibration(ctx, w.n_cells))


def _summary(name, ds, da, dc):
    rs, ra = np.sqrt(np.mean(ds * ds, axis=0)), np.sqrt(np.mean(da * da, axis=0))
    print(f"{name}: sources rms {np.array2string(rs, precision=3)} max {np.abs(ds).max():.3e} uas; "
          f"attitude rms {np.array2string(ra, precision=3)} max {np.abs(da).max():.3e} uas; "
          f"calibration max {np.abs(dc).max():.3e} uas")


def test_mixed_source_update_vs_oracle(agis_mod, oracle_lib, tiny):
    """One update of sources 50 mas from the truth: the FP32 normal matrix
    carries ~6e-8 relative rounding per entry, amplified by the condition
    of the source's 5x5 system; the error is a small fraction of the update
    (the iteration then refines it)."""
    w, eta = tiny
    pr = oracle_lib.problem_from_world(w, eta, state="start")
    d_o, _, de = pr.source_update()
    ctx = _ctx(agis_mod, w, eta, AGIS_MIXED, w.src_start, w.att_start, w.cal_start)
    agis_mod.agis_source_update(ctx)
    s_g, _, _ = _state(agis_mod, ctx, w)
    good = de == 0
    ds = src_diff_uas(pr.s, s_g)[good]
    upd = np.abs(d_o[good]).max(axis=1) / UAS
    _summary("mixed S update vs FP64 oracle", ds, np.zeros((1, 3)), np.zeros(1))
    rel = np.abs(ds).max(axis=1) / upd
    print(f"error / update: median {np.median(rel):.2e}, 99% {np.percentile(rel, 99):.2e}, max {rel.max():.2e}")
    # the right-hand side is summed in FP64 (measured: median 9e-8, 99% 5e-5)
    assert np.median(rel) < 1e-6 and np.percentile(rel, 99) < 1e-3
    agis_mod.agis_destroy(ctx)


def test_mixed_iterations_track_fp64(agis_mod, oracle_lib, tiny):
    """The outer iteration refines the mixed iterate: after 1 iteration it
    differs from FP64 by a fraction of the update, after 1000 iterations
    (S[AC] + frame rotator) by a small fraction of the total correction
    applied since the start (RMS per class below 1e-3 of it; the along-scan
    attitude axis and the calibration below 0.5 uas).  The plain iteration
    has not converged then: its slowest modes (across-scan attitude, weakly
    fixed by along-scan data alone) contract by ~0.999 per iteration, and the
    FP32 rounding perturbs exactly those."""
    w, eta = tiny
    ctxs = {}
    for prec in (0, AGIS_MIXED):
        ctxs[prec] = _ctx(agis_mod, w, eta, prec, w.src_start, w.att_start, w.cal_start)
        agis_mod.agis_set_frame_reference(ctxs[prec], w.src_true)
        agis_mod.agis_iterate(ctxs[prec], 1, stats=False)
    f0, f1 = _state(agis_mod, ctxs[0], w), _state(agis_mod, ctxs[AGIS_MIXED], w)
    d1 = (src_diff_uas(f0[0], f1[0]), rot_diff_uas(f0[1], f1[1]), (f1[2] - f0[2]) / UAS)
    _summary("mixed vs FP64 after 1 iteration", *d1)
    st0 = agis_mod.agis_iterate(ctxs[0], 999)[-1]
    agis_mod.agis_iterate(ctxs[AGIS_MIXED], 999, stats=False)
    print(f"after 1000 iterations: FP64 source update rms "
          f"{np.array2string(np.array(st0['s']['rms_update']) / UAS, precision=3)} uas")
    l0, l1 = _state(agis_mod, ctxs[0], w), _state(agis_mod, ctxs[AGIS_MIXED], w)
    dn = (src_diff_uas(l0[0], l1[0]), rot_diff_uas(l0[1], l1[1]), (l1[2] - l0[2]) / UAS)
    _summary("mixed vs FP64 after 1000 iterations", *dn)
    for c in ctxs.values():
        agis_mod.agis_destroy(c)
    moved_s = np.sqrt(np.mean(src_diff_uas(w.src_start, l0[0]) ** 2, axis=0))
    moved_a = np.sqrt(np.mean(rot_diff_uas(w.att_start, l0[1]) ** 2, axis=0))
    # The FP32 normal matrices change the path to the common fixed point
    # (the right-hand sides are FP64), and the slow across-scan modes have
    # not converged after 1000 iterations: measured 0.26 uas (alpha*) and
    # 1.8 uas (attitude x) RMS; with FP32 right-hand sides two equally valid
    # orders of the A/C sums had given 0.26-1.1 and 1.9-16.6 uas.
    assert np.all(np.sqrt(np.mean(dn[0] ** 2, axis=0)) <= 1e-3 * moved_s)
    assert np.all(np.sqrt(np.mean(dn[1] ** 2, axis=0)) <= 1e-3 * moved_a)
    # along-scan attitude and calibration, which the iteration determines
    # well, within 0.05 uas (measured 0.007 uas RMS and 0.027 uas max)
    assert np.sqrt(np.mean(dn[1][:, 2] ** 2)) <= 0.05 and np.abs(dn[2]).max() <= 0.05


def test_mixed_converges_to_the_fp64_point(agis_mod, oracle_lib):
    """On the tiny world with one across-scan record per transit (every
    attitude axis well determined), FP64 and mixed precision each run 1,200
    S[AC] + frame iterations from the start values, by which both have
    converged (their last 200 iterations move no parameter class by more
    than 1e-3 uas RMS); the two limits agree within 0.05 uas in every class,
    RMS and maximum (the mixed path's right-hand sides are FP64, so its
    fixed point is the FP64 one; its FP32 normal matrices only change the
    path to it)."""
    w = C.make("tiny", ac_obs=True)
    eta = oracle_lib.observed_field_angles(w)
    limits = {}
    for prec in (0, AGIS_MIXED):
        ctx = _ctx(agis_mod, w, eta, prec, w.src_start, w.att_start, w.cal_start)
        agis_mod.agis_set_frame_reference(ctx, w.src_true)
        agis_mod.agis_iterate_graph(ctx, 1000)
        before = _state(agis_mod, ctx, w)
        agis_mod.agis_iterate_graph(ctx, 200)
        after = _state(agis_mod, ctx, w)
        ds, da = src_diff_uas(before[0], after[0]), rot_diff_uas(before[1], after[1])
        dc = (after[2] - before[2]) / UAS
        _summary(f"precision {prec}: change over the last 200 iterations", ds, da, dc)
        assert np.sqrt(np.mean(ds * ds, axis=0)).max() < 1e-3 and np.sqrt(np.mean(da * da, axis=0)).max() < 1e-3
        limits[prec] = after
        agis_mod.agis_destroy(ctx)
    a, b = limits[0], limits[AGIS_MIXED]
    ds, da, dc = src_diff_uas(a[0], b[0]), rot_diff_uas(a[1], b[1]), (b[2] - a[2]) / UAS
    _summary("mixed - FP64 at convergence", ds, da, dc)
    for d in (ds, da, dc[:, None]):
        assert np.sqrt(np.mean(d * d, axis=0)).max() <= 0.05 and np.abs(d).max() <= 0.05
