"""Degenerate inputs on the GPU: no observations at all (plain and robust).
Every normal-equation block is then zero: Algorithm C1 skips every pivot
(App. C.3), so each source and attitude segment reports defects, every
update is zero and an iteration with the frame rotator leaves all
parameters as they were."""
import numpy as np
import pytest

import synth.configs as C
from test_gpu_parity import agis_mod  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["tiny", "tiny_robust"])
def test_no_observations(agis_mod, name):
    w = C.make(name)
    n_src = w.src_true.shape[0]
    ctx = agis_mod.agis_create(w.consts, w.knots)
    e = np.zeros(0)
    agis_mod.agis_load_observations(ctx, e, e, np.zeros(0, np.float32), np.zeros(0, np.int32),
                                    np.zeros(0, np.int8), np.zeros(0, np.int32), n_src, w.n_cells)
    size = agis_mod.agis_problem_size(ctx)
    assert size["n_obs"] == 0 and size["n_src"] == n_src
    agis_mod.agis_set_sources(ctx, w.src_start)
    agis_mod.agis_set_attitude(ctx, w.att_start)
    agis_mod.agis_set_calibration(ctx, w.cal_start)
    assert agis_mod.agis_residuals(ctx).size == 0
    st = agis_mod.agis_iterate(ctx, 2)
    agis_mod.agis_iterate_graph(ctx, 1)
    print(f"{name}: S defects {st[-1]['s']['defect']}, A defects {st[-1]['a']['defect']}")
    assert st[-1]["s"]["defect"] >= n_src and st[-1]["a"]["defect"] > 0
    s = agis_mod.agis_get_sources(ctx, n_src)
    a = agis_mod.agis_get_attitude(ctx, w.n_att)
    c = agis_mod.agis_get_calibration(ctx, w.n_cells)
    assert np.array_equal(s, w.src_start) and np.array_equal(a, w.att_start) and np.array_equal(c, w.cal_start)
    assert agis_mod.agis_chi2(ctx) == 0.0
    # with the frame rotator: its fit has no weight, so the rotation is the
    # identity and the rigorous transform moves the sources by rounding only
    agis_mod.agis_set_frame_reference(ctx, w.src_true)
    agis_mod.agis_iterate(ctx, 1, stats=False)
    s = agis_mod.agis_get_sources(ctx, n_src)
    a = agis_mod.agis_get_attitude(ctx, w.n_att)
    assert np.all(np.isfinite(s)) and np.all(np.isfinite(a))
    ds = s - w.src_start
    ds[:, 0] = (ds[:, 0] + np.pi) % (2 * np.pi) - np.pi        # alpha comes back in (-pi, pi]
    assert np.abs(ds).max() < 1e-14 and np.abs(a - w.att_start).max() < 1e-14
    agis_mod.agis_destroy(ctx)
