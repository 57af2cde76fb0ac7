"""The hybrid scheme on the GPU (Sect. 4.7): robust simple iterations, then
the weights frozen (agis_freeze_weights) and conjugate gradients on the
fixed problem, against the oracle's same sequence (oracle.cg.freeze) with
the FP64-floor criterion of the other parity tests.  Thawing returns to the
robust weighting without touching the state; a plain context refuses to
freeze."""
import numpy as np
import pytest

import synth.configs as C
from test_gpu_parity import DIFFS, Pair, fp64_floor, agis_mod  # noqa: F401

pytestmark = pytest.mark.gpu

N_SI, N_CG, RESTART = 2, 4, 3        # robust S[AC] + frame twice; CG: cycle start and 3 iterations


@pytest.fixture(scope="module")
def tiny_robust(oracle_lib):
    w = C.make("tiny_robust")
    return w, oracle_lib.observed_field_angles(w)


def test_hybrid_parity(agis_mod, oracle_lib, tiny_robust):
    from oracle import cg as ocg
    w, eta = tiny_robust

    def run(pr):
        for _ in range(N_SI):
            pr.iterate(s_ref=w.src_true)
        fr = ocg.freeze(pr)
        ocg.CG(fr, restart=RESTART, s_ref=w.src_true).run(N_CG)
        return fr.s.copy(), fr.a.copy(), fr.c.copy()

    X, O, tol = fp64_floor(oracle_lib, w, eta, run)
    p = Pair(agis_mod, oracle_lib, w, eta)
    agis_mod.agis_set_frame_reference(p.ctx, w.src_true)
    agis_mod.agis_iterate(p.ctx, N_SI, stats=False)
    with pytest.raises(RuntimeError, match="freeze"):
        agis_mod.agis_cg_iterate(p.ctx, 1, RESTART)
    agis_mod.agis_freeze_weights(p.ctx, True)
    st = agis_mod.agis_cg_iterate(p.ctx, N_CG, RESTART)
    assert [x["cycle_start"] for x in st] == [1, 0, 0, 0] and not any(x["breakdown"] for x in st)
    G = p.gpu_state()
    # The sequence compounds the rounding of the robust inner iterations, the
    # weights frozen from the residuals and the CG steps; the FP64 oracle
    # itself is then only 48% within 1e-3 uas for the across-scan attitude.
    # Criterion: per class, the GPU's largest and RMS deviation from the
    # extended-precision oracle at most twice the FP64 oracle's, and at least
    # 99.5% of the parameters within the per-parameter FP64-floor tolerance
    # (measured: single sources and coefficients reached 3x and 1.8x it).
    for name, which in (("sources", 0), ("attitude", 1), ("calibration", 2)):
        f = DIFFS[which]
        dg, do = np.abs(f(X[which], G[which])), np.abs(f(X[which], O[which]))
        within = float(np.mean(dg <= tol[which]))
        rms_g, rms_o = np.sqrt(np.mean(dg * dg, axis=0)), np.sqrt(np.mean(do * do, axis=0))
        print(f"hybrid {name}: max |GPU - ext| {dg.max():.2e} (FP64 oracle {do.max():.2e}) uas, "
              f"rms {np.array2string(np.atleast_1d(rms_g), precision=6)} "
              f"(oracle {np.array2string(np.atleast_1d(rms_o), precision=6)}), "
              f"{100 * within:.3f}% within tolerance, worst ratio {(dg / tol[which]).max():.2f}")
        assert dg.max() <= 2.0 * do.max() + 1e-6
        assert np.all(rms_g <= 2.0 * rms_o + 1e-6)
        assert within >= 0.995
    p.close()


def test_thaw_returns_to_robust(agis_mod, oracle_lib, tiny_robust):
    w, eta = tiny_robust
    a, b = Pair(agis_mod, oracle_lib, w, eta), Pair(agis_mod, oracle_lib, w, eta)
    for p in (a, b):
        agis_mod.agis_set_frame_reference(p.ctx, w.src_true)
        agis_mod.agis_iterate(p.ctx, 1, stats=False)
    agis_mod.agis_freeze_weights(a.ctx, True)
    agis_mod.agis_freeze_weights(a.ctx, False)
    for p in (a, b):
        agis_mod.agis_iterate(p.ctx, 2, stats=False)
    nb = (w.knots.size - 7 + int(w.consts["eps_bucket"]) - 1) // int(w.consts["eps_bucket"])
    for x, y in zip(a.gpu_state() + (agis_mod.agis_get_excess_noise(a.ctx, nb),),
                    b.gpu_state() + (agis_mod.agis_get_excess_noise(b.ctx, nb),)):
        assert np.array_equal(x, y)
    a.close()
    b.close()


def test_plain_context_refuses_to_freeze(agis_mod, oracle_lib):
    w = C.make("tiny")
    eta = oracle_lib.observed_field_angles(w)
    p = Pair(agis_mod, oracle_lib, w, eta)
    with pytest.raises(RuntimeError, match="not robust"):
        agis_mod.agis_freeze_weights(p.ctx, True)
    p.close()


def test_hybrid_converges_faster_than_robust_si(agis_mod, oracle_lib, tiny_robust):
    """From the start values with the frame rotator: 20 robust iterations,
    then 200 more evaluations either as robust simple iterations or as CG on
    weights frozen at the start of every cycle of 40 (the paper's hybrid, with
    its weights refreshed at each return to SI).  The hybrid ends with the
    smaller parallax error (median and RMS over the sources; the RMS is set by
    a few poorly observed sources)."""
    w, eta = tiny_robust
    n_warm, n = 20, 200
    out = {}
    for mode in ("si", "hybrid"):
        p = Pair(agis_mod, oracle_lib, w, eta)
        agis_mod.agis_set_frame_reference(p.ctx, w.src_true)
        agis_mod.agis_iterate(p.ctx, n_warm, stats=False)
        if mode == "si":
            agis_mod.agis_iterate(p.ctx, n, stats=False)
        else:
            for _ in range(n // 40):
                agis_mod.agis_freeze_weights(p.ctx, True)
                agis_mod.agis_cg_iterate(p.ctx, 40, 40, stats=False)
                agis_mod.agis_freeze_weights(p.ctx, False)
        s = p.gpu_state()[0]
        e = np.abs(s[:, 2] - w.src_true[:, 2]) / 4.8481368e-12
        out[mode] = (float(np.median(e)), float(np.sqrt(np.mean(e * e))))
        p.close()
    print(f"parallax error after {n_warm} + {n} evaluations (median, RMS): robust SI {out['si'][0]:.2f}, "
          f"{out['si'][1]:.2f} uas; hybrid {out['hybrid'][0]:.2f}, {out['hybrid'][1]:.2f} uas")
    assert out["hybrid"][0] < out["si"][0] and out["hybrid"][1] < out["si"][1]
