"""The graph-captured iteration (agis_iterate_graph) against the eager one
(agis_iterate): the same kernels on the same stream, so the iterates agree
bit for bit, also when graph replays and eager iterations alternate, after
the captured configuration changes (frame reference cleared, observations
reloaded: the graph is captured again), and in the robust mode."""
import time

import numpy as np
import pytest

import synth.configs as C
from test_gpu_parity import agis_mod  # noqa: F401

pytestmark = pytest.mark.gpu


def _ctx(agis, w, eta):
    ctx = agis.agis_create(w.consts, w.knots)
    agis.agis_load_observations(ctx, w.t, eta, w.sigma, w.src, w.fov, w.cell, w.src_true.shape[0], w.n_cells)
    agis.agis_set_sources(ctx, w.src_start)
    agis.agis_set_attitude(ctx, w.att_start)
    agis.agis_set_calibration(ctx, w.cal_start)
    agis.agis_set_frame_reference(ctx, w.src_true)
    return ctx


def _state(agis, ctx, w, robust=False):
    out = [agis.agis_get_sources(ctx, w.src_true.shape[0]), agis.agis_get_attitude(ctx, w.n_att),
           agis.agis_get_calibration(ctx, w.n_cells)]
    if robust:
        nb = (w.knots.size - 7 + int(w.consts["eps_bucket"]) - 1) // int(w.consts["eps_bucket"])
        out.append(agis.agis_get_excess_noise(ctx, 3 * nb))   # AL, ACP, ACF
    return out


def _same(x, y):
    return all(np.array_equal(a, b) for a, b in zip(x, y))


@pytest.fixture(scope="module")
def tiny(oracle_lib):
    w = C.make("tiny")
    return w, oracle_lib.observed_field_angles(w)


def test_graph_equals_eager(agis_mod, tiny):
    w, eta = tiny
    e, g = _ctx(agis_mod, w, eta), _ctx(agis_mod, w, eta)
    agis_mod.agis_iterate(e, 6, stats=False)
    agis_mod.agis_iterate_graph(g, 3)
    agis_mod.agis_iterate(g, 1, stats=False)             # eager work between replays
    agis_mod.agis_iterate_graph(g, 2)
    assert _same(_state(agis_mod, e, w), _state(agis_mod, g, w))
    # without the frame rotator (captured again)
    for c in (e, g):
        agis_mod.agis_set_frame_reference(c, None)
    agis_mod.agis_iterate(e, 2, stats=False)
    agis_mod.agis_iterate_graph(g, 2)
    assert _same(_state(agis_mod, e, w), _state(agis_mod, g, w))
    # observations reloaded (new buffers; sources and calibration start from
    # zero, so set again): captured again
    s0, a0, c0 = _state(agis_mod, e, w)
    for c in (e, g):
        agis_mod.agis_load_observations(c, w.t, eta, w.sigma, w.src, w.fov, w.cell, w.src_true.shape[0],
                                        w.n_cells)
        agis_mod.agis_set_sources(c, s0)
        agis_mod.agis_set_attitude(c, a0)
        agis_mod.agis_set_calibration(c, c0)
        agis_mod.agis_set_frame_reference(c, w.src_true)
    agis_mod.agis_iterate(e, 2, stats=False)
    agis_mod.agis_iterate_graph(g, 2)
    assert _same(_state(agis_mod, e, w), _state(agis_mod, g, w))
    agis_mod.agis_iterate_graph(g, 0)
    with pytest.raises(RuntimeError):
        agis_mod.agis_iterate_graph(g, -1)
    agis_mod.agis_destroy(e)
    agis_mod.agis_destroy(g)


def test_graph_equals_eager_robust(agis_mod, oracle_lib):
    w = C.make("tiny_robust")
    eta = oracle_lib.observed_field_angles(w)
    e, g = _ctx(agis_mod, w, eta), _ctx(agis_mod, w, eta)
    agis_mod.agis_iterate(e, 4, stats=False)
    agis_mod.agis_iterate_graph(g, 2)
    agis_mod.agis_iterate(g, 1, stats=False)
    agis_mod.agis_iterate_graph(g, 1)
    assert _same(_state(agis_mod, e, w, True), _state(agis_mod, g, w, True))
    agis_mod.agis_destroy(e)
    agis_mod.agis_destroy(g)


def test_graph_timing(agis_mod, tiny):
    """Per-iteration wall time of the two paths on the tiny world (short
    kernels): reported; the graph must not be slower than the eager path."""
    w, eta = tiny
    ctx = _ctx(agis_mod, w, eta)
    agis_mod.agis_iterate(ctx, 5, stats=False)
    agis_mod.agis_iterate_graph(ctx, 5)
    n = 200
    t0 = time.perf_counter()
    agis_mod.agis_iterate(ctx, n, stats=False)
    t_e = (time.perf_counter() - t0) / n
    t0 = time.perf_counter()
    agis_mod.agis_iterate_graph(ctx, n)
    t_g = (time.perf_counter() - t0) / n
    print(f"tiny world: eager {1e3 * t_e:.3f} ms, graph {1e3 * t_g:.3f} ms per iteration")
    assert t_g <= 1.1 * t_e
    agis_mod.agis_destroy(ctx)


def test_autotune_keeps_state(agis_mod, tiny, monkeypatch):
    """agis_autotune times the S pass per group size from the current state
    and restores it: every state array is bitwise unchanged, the chosen size
    is one of the candidates, and a following source update equals that of a
    context fixed to the chosen size."""
    w, eta = tiny
    ctx = _ctx(agis_mod, w, eta)
    agis_mod.agis_iterate(ctx, 3, stats=False)
    before = _state(agis_mod, ctx, w)
    g = agis_mod.agis_autotune(ctx)
    print(f"autotuned lanes per source: {g}")
    assert g in (8, 16, 32)
    assert _same(before, _state(agis_mod, ctx, w))
    monkeypatch.setenv("AGIS_S_GROUP", str(g))
    ref = _ctx(agis_mod, w, eta)
    monkeypatch.delenv("AGIS_S_GROUP")
    for c in (ctx, ref):
        agis_mod.agis_set_sources(c, before[0])
        agis_mod.agis_set_attitude(c, before[1])
        agis_mod.agis_set_calibration(c, before[2])
        agis_mod.agis_source_update(c)
    assert _same(_state(agis_mod, ctx, w), _state(agis_mod, ref, w))
    agis_mod.agis_destroy(ctx)
    agis_mod.agis_destroy(ref)


@pytest.mark.parametrize("ac", [False, True])
def test_autotune_robust_path_keeps_state(agis_mod, oracle_lib, ac, monkeypatch):
    """In robust mode 1 the autotuner also picks the S block's path: the
    state is restored bit for bit, the choice is reported by
    agis_get_tuning, and a following robust source update equals that of a
    context fixed to the same lanes per source, path and quantile kernel."""
    w = C.make("tiny_robust", ac_obs=ac)
    eta = oracle_lib.observed_field_angles(w)
    ctx = _ctx(agis_mod, w, eta)
    agis_mod.agis_iterate(ctx, 2, stats=False)
    before = _state(agis_mod, ctx, w, robust=True)
    g = agis_mod.agis_autotune(ctx)
    tun = agis_mod.agis_get_tuning(ctx)
    print(f"autotuned (tiny_robust{'+ac' if ac else ''}): {tun}")
    assert tun["lanes_per_source"] == g and tun["robust_s_path"] in (0, 1, 2)
    assert _same(before, _state(agis_mod, ctx, w, robust=True))
    env = {"AGIS_S_GROUP": str(g), "AGIS_SELECT_PAIR": "1" if tun["paired_selection"] else "0",
           "AGIS_ROBUST_FUSED": {0: "1", 1: "3", 2: "2"}[tun["robust_s_path"]]}
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    ref = _ctx(agis_mod, w, eta)
    for k in env:
        monkeypatch.delenv(k)
    assert agis_mod.agis_get_tuning(ref) == tun
    for c in (ctx, ref):
        agis_mod.agis_set_sources(c, before[0])
        agis_mod.agis_set_attitude(c, before[1])
        agis_mod.agis_set_calibration(c, before[2])
        agis_mod.agis_set_excess_noise(c, before[3])
        agis_mod.agis_source_update(c)
    assert _same(_state(agis_mod, ctx, w), _state(agis_mod, ref, w))
    agis_mod.agis_destroy(ctx)
    agis_mod.agis_destroy(ref)
