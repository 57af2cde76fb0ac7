"""Resuming an iteration from its saved state (the paper's runs persist the
parameters between iterations, Sect. 7.1): ten S[AC] + frame iterations in
one context equal five, then the state read out (sources, attitude,
calibration and, in the robust mode, the excess attitude noise), a new
context loaded with the same observations and set to that state, and five
more, bit for bit."""
import numpy as np
import pytest

import synth.configs as C
from test_gpu_parity import agis_mod  # noqa: F401

pytestmark = pytest.mark.gpu


def _fresh(agis, w, eta):
    ctx = agis.agis_create(w.consts, w.knots)
    agis.agis_load_observations(ctx, w.t, eta, w.sigma, w.src, w.fov, w.cell, w.src_true.shape[0], w.n_cells)
    agis.agis_set_frame_reference(ctx, w.src_true)
    return ctx


def _state(agis, ctx, w, robust, nb):
    out = [agis.agis_get_sources(ctx, w.src_true.shape[0]), agis.agis_get_attitude(ctx, w.n_att),
           agis.agis_get_calibration(ctx, w.n_cells)]
    if robust:
        out.append(agis.agis_get_excess_noise(ctx, nb))
    return out


@pytest.mark.parametrize("name", ["tiny", "tiny_robust", "tiny_robust+ac"])
def test_resume_equals_continuous(agis_mod, oracle_lib, name):
    w = C.make(name.split("+")[0], ac_obs=name.endswith("+ac"))
    eta = oracle_lib.observed_field_angles(w)
    robust = bool(w.consts["robust"])
    nb = 3 * ((w.n_att - 3 + w.consts["eps_bucket"] - 1) // w.consts["eps_bucket"])   # AL, ACP, ACF
    ref = _fresh(agis_mod, w, eta)
    agis_mod.agis_set_sources(ref, w.src_start)
    agis_mod.agis_set_attitude(ref, w.att_start)
    agis_mod.agis_set_calibration(ref, w.cal_start)
    agis_mod.agis_iterate(ref, 10, stats=False)
    full = _state(agis_mod, ref, w, robust, nb)
    agis_mod.agis_destroy(ref)

    first = _fresh(agis_mod, w, eta)
    agis_mod.agis_set_sources(first, w.src_start)
    agis_mod.agis_set_attitude(first, w.att_start)
    agis_mod.agis_set_calibration(first, w.cal_start)
    agis_mod.agis_iterate(first, 5, stats=False)
    saved = _state(agis_mod, first, w, robust, nb)
    agis_mod.agis_destroy(first)

    second = _fresh(agis_mod, w, eta)
    agis_mod.agis_set_sources(second, saved[0])
    agis_mod.agis_set_attitude(second, saved[1])
    agis_mod.agis_set_calibration(second, saved[2])
    if robust:
        agis_mod.agis_set_excess_noise(second, saved[3])
    agis_mod.agis_iterate(second, 5, stats=False)
    resumed = _state(agis_mod, second, w, robust, nb)
    agis_mod.agis_destroy(second)
    for x, y, what in zip(full, resumed, ("sources", "attitude", "calibration", "excess attitude noise")):
        assert np.array_equal(x, y), what
