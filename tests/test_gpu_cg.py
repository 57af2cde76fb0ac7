"""Conjugate gradients on the GPU (agis_cg_iterate, Sect. 4.7) against the
oracle's scheme (oracle/cg.py): the same cycles of steps, compared
parameter by parameter with the FP64-floor criterion of
the other parity tests (extended-precision oracle as reference); the step
lengths and direction coefficients agree to rounding.  Also: the cycle
restarts after any outside change of the state, the robust mode is refused,
and CG lowers the objective faster than the simple iteration."""
import numpy as np
import pytest

import synth.configs as C
from test_gpu_parity import Pair, check_floor, fp64_floor, src_diff_uas, agis_mod  # noqa: F401

pytestmark = pytest.mark.gpu

N_EVAL, RESTART = 6, 3          # cycle start, 3 iterations, cycle start (frame rotator), 1 iteration


@pytest.fixture(scope="module")
def tiny(oracle_lib):
    w = C.make("tiny")
    return w, oracle_lib.observed_field_angles(w)


def test_cg_parity(agis_mod, oracle_lib, tiny):
    from oracle import cg as ocg
    w, eta = tiny
    steps = {}

    def run(pr):
        it = ocg.CG(pr, restart=RESTART, s_ref=w.src_true)
        ab = []
        for _ in range(N_EVAL):
            it.step()
            ab.append((float(it.alpha), float(it.beta)))
        steps.setdefault(pr.precision, ab)
        return pr.s.copy(), pr.a.copy(), pr.c.copy()

    X, O, tol = fp64_floor(oracle_lib, w, eta, run)
    p = Pair(agis_mod, oracle_lib, w, eta)
    agis_mod.agis_set_frame_reference(p.ctx, w.src_true)
    st = agis_mod.agis_cg_iterate(p.ctx, N_EVAL, RESTART)
    G = p.gpu_state()
    assert [x["cycle_start"] for x in st] == [1, 0, 0, 0, 1, 0]
    assert not any(x["breakdown"] for x in st)
    ref = steps["extended"]
    for k, x in enumerate(st):
        print(f"evaluation {k}: alpha {x['alpha']:.12g} (oracle {ref[k][0]:.12g}), "
              f"beta {x['beta']:.12g} (oracle {ref[k][1]:.12g}), {x['ms']:.3f} ms")
        assert abs(x["alpha"] - ref[k][0]) <= 1e-9 * max(abs(ref[k][0]), 1e-300)
        assert abs(x["beta"] - ref[k][1]) <= 1e-7 * max(abs(ref[k][1]), 1e-12)
    check_floor("CG: sources", X[0], O[0], G[0], tol[0], 0)
    check_floor("CG: attitude", X[1], O[1], G[1], tol[1], 1)
    check_floor("CG: calibration", X[2], O[2], G[2], tol[2], 2)
    p.close()


def test_cg_cycle_restarts_after_outside_change(agis_mod, oracle_lib, tiny):
    w, eta = tiny
    p = Pair(agis_mod, oracle_lib, w, eta)
    st = agis_mod.agis_cg_iterate(p.ctx, 3, 10)
    assert [x["cycle_start"] for x in st] == [1, 0, 0]
    s, a, c = p.gpu_state()                              # reading does not disturb the cycle
    st = agis_mod.agis_cg_iterate(p.ctx, 1, 10)
    assert st[0]["cycle_start"] == 0
    agis_mod.agis_set_sources(p.ctx, s)                  # writing does
    st = agis_mod.agis_cg_iterate(p.ctx, 2, 10)
    assert [x["cycle_start"] for x in st] == [1, 0]
    agis_mod.agis_iterate(p.ctx, 1, stats=False)
    assert agis_mod.agis_cg_iterate(p.ctx, 1, 10)[0]["cycle_start"] == 1
    # a cycle of restart iterations, then a new start
    st = agis_mod.agis_cg_iterate(p.ctx, 5, 2)
    assert [x["cycle_start"] for x in st] == [0, 0, 1, 0, 0]
    with pytest.raises(RuntimeError):
        agis_mod.agis_cg_iterate(p.ctx, 1, 0)
    agis_mod.agis_cg_iterate(p.ctx, 0, 5)
    p.close()


def test_cg_refused_in_robust_mode(agis_mod, oracle_lib):
    w = C.make("tiny_robust")
    eta = oracle_lib.observed_field_angles(w)
    p = Pair(agis_mod, oracle_lib, w, eta)
    with pytest.raises(RuntimeError, match="robust"):
        agis_mod.agis_cg_iterate(p.ctx, 1, 10)
    p.close()


def test_cg_lowers_the_objective_faster(agis_mod, oracle_lib, tiny):
    """From the start values, with the frame rotator: after the same number
    of evaluations (each one pass of the three blocks) CG reaches a lower
    sum of W R^2 and a smaller parallax error than the simple iteration."""
    w, eta = tiny
    n = 200
    out = {}
    for mode in ("si", "cg"):
        p = Pair(agis_mod, oracle_lib, w, eta)
        agis_mod.agis_set_frame_reference(p.ctx, w.src_true)
        if mode == "si":
            agis_mod.agis_iterate(p.ctx, n, stats=False)
        else:
            agis_mod.agis_cg_iterate(p.ctx, n, 40, stats=False)
        s = p.gpu_state()[0]
        out[mode] = (agis_mod.agis_chi2(p.ctx), np.sqrt(np.mean((s[:, 2] - w.src_true[:, 2]) ** 2)))
        p.close()
    print(f"after {n} evaluations: chi2 SI {out['si'][0]:.6f}, CG {out['cg'][0]:.6f}; "
          f"parallax RMS error SI {out['si'][1] / 4.8481368e-12:.2f} uas, CG {out['cg'][1] / 4.8481368e-12:.2f} uas")
    assert out["cg"][0] < out["si"][0]
    assert out["cg"][1] < 0.7 * out["si"][1]
