"""Parity of the HIP library (through its C ABI) with the CPU oracle.

Same seeded inputs on both sides; the observed field angles come from the
oracle's observation model at the true parameters.  Updated parameters are
compared with the oracle built in extended precision: each within
max(1e-3 uas, its FP64 rounding floor), and per component no less accurate
than the FP64 oracle itself (attitude compared as rotations,
eq:diffrot2-3, since the coefficients' scale is unobservable).  Sources whose 5x5 system is singular
(too few observations) are compared through their defect flag only, because
"any valid solution" is acceptable there (Appendix C.3).
"""
import types

import numpy as np
import pytest
from scipy.ndimage import maximum_filter1d

import synth
import synth.configs as C

pytestmark = pytest.mark.gpu

UAS = synth.UAS
TOL_UAS = 1e-3


@pytest.fixture(scope="module")
def agis_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1112_4139_amd import agis
    return agis


def _qmul(a, b):
    ax, ay, az, aw = a.T
    bx, by, bz, bw = b.T
    return np.stack([aw * bx + ax * bw + ay * bz - az * by, aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw, aw * bw - ax * bx - ay * by - az * bz], axis=1)


def rot_diff_uas(a_ref, a):
    """Rotation angles (x, y, z) from a_ref to a per coefficient [uas]."""
    conj = a_ref * np.array([-1, -1, -1, 1.0])
    d = _qmul(conj, a)
    d /= np.linalg.norm(d, axis=1)[:, None]
    return 2 * d[:, :3] * np.sign(d[:, 3:4]) / UAS


def src_diff_uas(s_ref, s):
    ds = s - s_ref
    ds[:, 0] = ((ds[:, 0] + np.pi) % (2 * np.pi) - np.pi) * np.cos(s_ref[:, 1])
    return ds / UAS


# The per-parameter bound.  An FP64 implementation's rounding error in a
# parameter p is modelled as e_p = c s_p g_p, g_p ~ N(0, 1): s_p is the
# parameter's sensitivity to the two kinds of rounding in which FP64
# implementations differ -- rounding-level noise in the residuals, and the
# order in which the sums over observations are taken (which perturbs the
# normal matrices in proportion to the update, so that it dominates for
# ill-conditioned sources with large updates) -- and c the implementation's
# noise level in those units.  s_p is estimated as the RMS of the
# parameter's responses to N_DRAWS independent draws, each of which adds
# N(0, (3e-16 rad)^2) to every residual (~2x the measured RMS difference of
# the GPU's and the oracle's residuals) and feeds the oracle its
# observations in a random order (the oracle sums a source's and a cell's
# observations in input order).  With c <= 1,
# e_p / s_hat_p then follows Student's t with N_DRAWS degrees of freedom,
# and FLOOR_FACTOR is its two-sided quantile for a false alarm of 1e-3 over
# 1e5 parameters (scipy.stats.t.ppf(1 - 5e-9, 8) = 23.9).  An attitude
# coefficient's bound is also at least REF_FACTOR x the largest deviation of
# the FP64 oracle among the 33 coefficients around it (a pooled sample of the
# local floor, which follows the band system's conditioning: the largest of
# 33 Gaussian deviations is ~2.4 sigma, so the bound is ~10 sigma).
N_DRAWS = 8
FLOOR_FACTOR = 24.0
REF_FACTOR = 4.0
ULP_NOISE = 3e-16


def fp64_floor(oracle_lib, world, eta, run, n_draws=N_DRAWS, ulp_noise=ULP_NOISE, factor=FLOOR_FACTOR,
               factor_ref=REF_FACTOR):
    """Reference result X, FP64 oracle result O and per-parameter tolerances.

    X is the oracle built in x87 extended precision (64-bit significand): the
    exact answer to ~1e-19 relative.  An FP64 implementation cannot do better
    than the FP64 rounding floor of each parameter; the tolerance is
    max(1e-3 uas, factor x s_hat_p) with s_hat_p the RMS response of the
    parameter to n_draws perturbations of every residual by N(0, ulp_noise^2),
    each with the observations in a random order (see FLOOR_FACTOR above),
    and for attitude coefficients also factor_ref x
    the FP64 oracle's largest deviation |O - X| among the 16 coefficients on
    either side.  run(problem) -> (s, a, c)."""
    X = [np.asarray(v, np.float64) for v in run(oracle_lib.problem_from_world(world, eta, "start", "extended"))]
    O = run(oracle_lib.problem_from_world(world, eta, state="start"))
    ss = [np.zeros_like(src_diff_uas(O[0], O[0])), np.zeros((O[1].shape[0], 3)), np.zeros_like(O[2])]
    for k in range(n_draws):
        rng = np.random.default_rng(100 + k)
        noisy = eta + rng.normal(0, ulp_noise, eta.shape)
        perm = rng.permutation(eta.size)
        out = run(oracle_lib.problem_from_world(reordered(world, perm), noisy[perm], state="start"))
        for i, f in enumerate(DIFFS):
            ss[i] += f(O[i], out[i]) ** 2
    sens = [np.sqrt(x / n_draws) for x in ss]
    tol = [np.maximum(TOL_UAS, factor * sens[i]) for i in range(3)]
    # the floor of an attitude coefficient is set by the conditioning of the
    # local band system, which varies slowly along the mission: the largest
    # FP64 deviation among the 16 coefficients on either side
    ref_a = maximum_filter1d(np.abs(DIFFS[1](X[1], O[1])), size=33, axis=0, mode="nearest")
    tol[1] = np.maximum(tol[1], factor_ref * ref_a)
    return X, O, tol


OBS_FIELDS = ("t", "src", "fov", "cell", "sigma", "eps", "ccd", "mu", "ac_cell")


def reordered(w, perm):
    """The world with its observations taken in the order perm (sources,
    attitude, calibration, knots and constants unchanged)."""
    out = types.SimpleNamespace(**{k: v for k, v in vars(w).items() if k not in OBS_FIELDS})
    for k in OBS_FIELDS:
        if getattr(w, k, None) is not None:
            setattr(out, k, getattr(w, k)[perm])
    return out


def cal_diff_uas(c_ref, c):
    return (c - c_ref) / UAS


DIFFS = (src_diff_uas, rot_diff_uas, cal_diff_uas)


def check_floor(name, X, O, G, tol, which, mask=None, rms_factor=2.0):
    """GPU result G against the extended-precision reference X: every
    parameter within its FP64-floor tolerance, and per component an RMS error
    no larger than rms_factor x that of the FP64 oracle O."""
    f = DIFFS[which]
    dg, do = f(X, G), f(X, O)
    if mask is not None:
        dg, do, tol = dg[mask], do[mask], tol[mask]
    report(f"{name} (GPU - ext)", dg, tol)
    report(f"{name} (FP64 oracle - ext)", do, tol)
    assert np.all(np.abs(dg) <= tol)
    rms_g = np.sqrt(np.mean(dg * dg, axis=0))
    rms_o = np.sqrt(np.mean(do * do, axis=0))
    assert np.all(rms_g <= rms_factor * rms_o + 1e-5), (rms_g, rms_o)
    return dg


def report(name, diff, tol):
    within = float(np.mean(np.abs(diff) <= TOL_UAS))
    ratio = np.abs(diff) / tol
    worst = np.unravel_index(np.argmax(ratio), ratio.shape)
    rms = np.sqrt(np.mean(diff * diff, axis=0))
    print(f"{name}: max {np.abs(diff).max():.2e} uas, rms {np.array2string(np.atleast_1d(rms), precision=2)}, "
          f"{100 * within:.2f}% within 1e-3 uas, worst diff/tol {ratio.max():.2f} at "
          f"{tuple(int(x) for x in worst)} (diff {np.abs(diff)[worst]:.2e}, tol {tol[worst]:.2e})")


class Pair:
    """The same problem held by the oracle and by a GPU context."""

    def __init__(self, agis, oracle_lib, world, eta, state="start"):
        self.w = world
        self.pr = oracle_lib.problem_from_world(world, eta, state=state)
        self.agis = agis
        self.ctx = agis.agis_create(world.consts, world.knots)
        agis.agis_load_observations(self.ctx, world.t, eta, world.sigma, world.src, world.fov, world.cell,
                                    world.src_true.shape[0], world.n_cells)
        agis.agis_set_sources(self.ctx, self.pr.s)
        agis.agis_set_attitude(self.ctx, self.pr.a)
        agis.agis_set_calibration(self.ctx, self.pr.c)

    def gpu_state(self):
        a = self.agis
        n = self.w.src_true.shape[0]
        return (a.agis_get_sources(self.ctx, n), a.agis_get_attitude(self.ctx, self.w.n_att),
                a.agis_get_calibration(self.ctx, self.w.n_cells))

    def close(self):
        self.agis.agis_destroy(self.ctx)


@pytest.fixture(scope="module")
def small(oracle_lib):
    w = C.make("small")
    return w, oracle_lib.observed_field_angles(w)


@pytest.fixture(scope="module")
def tiny(oracle_lib):
    w = C.make("tiny")
    return w, oracle_lib.observed_field_angles(w)


def test_library_loads_and_reports_sizes(agis_mod, small, oracle_lib):
    w, eta = small
    p = Pair(agis_mod, oracle_lib, w, eta)
    sz = agis_mod.agis_problem_size(p.ctx)
    assert sz["n_obs"] == w.n_obs and sz["n_att"] == w.n_att and sz["n_cells"] == w.n_cells
    assert sz["n_segments"] == p.pr.num_segments()
    p.close()


def test_residuals_match(agis_mod, small, oracle_lib):
    w, eta = small
    p = Pair(agis_mod, oracle_lib, w, eta)
    Rg = agis_mod.agis_residuals(p.ctx)
    Ro = p.pr.observe()["R"]
    d = Rg - Ro
    print(f"residuals: max |diff| {np.abs(d).max():.2e} rad, rms {np.sqrt(np.mean(d * d)):.2e} rad")
    assert np.abs(d).max() / UAS < TOL_UAS
    # the premise of fp64_floor: the two models differ by rounding only,
    # well inside the 3e-16 rad noise it propagates through the oracle
    assert np.sqrt(np.mean(d * d)) < 1.5e-16
    p.close()


@pytest.mark.parametrize("world", ["small", "tiny"])
def test_source_update_parity(agis_mod, oracle_lib, world, request):
    w, eta = request.getfixturevalue(world)

    def run(pr):
        _, _, de = pr.source_update()
        run.defect = de
        return pr.s.copy(), pr.a.copy(), pr.c.copy()

    X, O, tol = fp64_floor(oracle_lib, w, eta, run)
    run(oracle_lib.problem_from_world(w, eta, state="start"))
    good = run.defect == 0          # singular sources: any valid solution (App. C.3)
    p = Pair(agis_mod, oracle_lib, w, eta)
    st = agis_mod.agis_source_update(p.ctx)
    G = p.gpu_state()
    assert good.mean() > 0.95
    dg = check_floor(f"S update [{world}]", X[0], O[0], G[0], tol[0], 0, mask=good)
    assert np.mean(np.abs(dg) <= TOL_UAS) > 0.95
    assert st["n_units"] == w.src_true.shape[0]
    p.close()


@pytest.mark.parametrize("world", ["tiny"])
def test_attitude_calibration_update_parity(agis_mod, oracle_lib, world, request):
    """One S[AC] iteration without the frame rotator."""
    w, eta = request.getfixturevalue(world)

    def run(pr):
        pr.iterate_sac()
        return pr.s.copy(), pr.a.copy(), pr.c.copy()

    X, O, tol = fp64_floor(oracle_lib, w, eta, run)
    p = Pair(agis_mod, oracle_lib, w, eta)
    agis_mod.agis_source_update(p.ctx)
    st_a, st_c = agis_mod.agis_attitude_calibration_update(p.ctx)
    G = p.gpu_state()
    rd = check_floor("A update rotation", X[1], O[1], G[1], tol[1], 1)
    assert np.mean(np.abs(rd[:, 2]) <= TOL_UAS) > 0.99        # along-scan axis
    scale = np.abs(np.linalg.norm(G[1], axis=1) / np.linalg.norm(O[1], axis=1) - 1)
    assert scale.max() < 1e-10
    check_floor("C update", X[2], O[2], G[2], tol[2], 2)
    assert np.all(np.abs(G[2][0::2] + G[2][1::2]) < 1e-18)
    p.close()


def test_frame_rotator_parity(agis_mod, small, oracle_lib):
    w, eta = small
    p = Pair(agis_mod, oracle_lib, w, eta)
    agis_mod.agis_set_frame_reference(p.ctx, w.src_true)
    eo_g = agis_mod.agis_frame_fit(p.ctx)
    eo_o = p.pr.frame_fit(w.src_true)
    assert np.abs(eo_g - eo_o).max() / UAS < 1e-5
    eo = np.array([3.0, -7.0, 5.0, 2.0, 4.0, -6.0]) * synth.MAS
    agis_mod.agis_frame_apply(p.ctx, eo)
    p.pr.frame_apply(eo)
    s_g, a_g, _ = p.gpu_state()
    assert np.abs(src_diff_uas(p.pr.s, s_g)).max() < TOL_UAS
    assert np.abs(rot_diff_uas(p.pr.a, a_g)).max() < TOL_UAS
    p.close()


def test_iterations_with_frame_rotator_parity(agis_mod, tiny, oracle_lib):
    w, eta = tiny
    n_it = 3

    def run(pr):
        for _ in range(n_it):
            pr.iterate(s_ref=w.src_true)
        return pr.s.copy(), pr.a.copy(), pr.c.copy()

    X, O, tol = fp64_floor(oracle_lib, w, eta, run)
    p = Pair(agis_mod, oracle_lib, w, eta)
    agis_mod.agis_set_frame_reference(p.ctx, w.src_true)
    stats = agis_mod.agis_iterate(p.ctx, n_it)
    G = p.gpu_state()
    check_floor("3 iterations: sources", X[0], O[0], G[0], tol[0], 0)
    check_floor("3 iterations: attitude", X[1], O[1], G[1], tol[1], 1)
    check_floor("3 iterations: calibration", X[2], O[2], G[2], tol[2], 2)
    assert len(stats) == n_it and all(np.isfinite(x["ms"]) for x in stats)
    p.close()


def test_bitwise_reproducible(agis_mod, small, oracle_lib):
    w, eta = small
    outs = []
    for _ in range(2):
        p = Pair(agis_mod, oracle_lib, w, eta)
        agis_mod.agis_set_frame_reference(p.ctx, w.src_true)
        agis_mod.agis_iterate(p.ctx, 2, stats=False)
        outs.append(p.gpu_state())
        p.close()
    for x, y in zip(*outs):
        assert np.array_equal(x, y)


def test_data_gap_natural_break(agis_mod, oracle_lib):
    """Observations removed over more than M knot intervals: the attitude
    system there is singular (Sect. 5.2.2 natural break); C1 counts the
    defect, the solution stays finite and matches the oracle."""
    w = C.make("tiny")
    t0, t1 = w.knots[3 + 500], w.knots[3 + 512]
    keep = ~((w.t >= t0) & (w.t < t1))
    for name in ("t", "src", "fov", "cell", "sigma", "eps", "eta_nominal"):
        setattr(w, name, np.ascontiguousarray(getattr(w, name)[keep]))
    eta = oracle_lib.observed_field_angles(w)

    def run(pr):
        pr.iterate_sac()
        return pr.s.copy(), pr.a.copy(), pr.c.copy()

    X, O, tol = fp64_floor(oracle_lib, w, eta, run)
    p = Pair(agis_mod, oracle_lib, w, eta)
    agis_mod.agis_source_update(p.ctx)
    st_a, st_c = agis_mod.agis_attitude_calibration_update(p.ctx)
    assert st_a["defect"] > 0
    G = p.gpu_state()
    assert np.all(np.isfinite(G[1]))
    # coefficients whose support lies entirely inside the gap get no update
    inside = np.arange(500 + 3, 512 - 3)
    np.testing.assert_array_equal(G[1][inside], w.att_start[inside])
    check_floor("A update with a data gap", X[1], O[1], G[1], tol[1], 1)
    p.close()


def test_invalid_inputs_rejected(agis_mod, small, oracle_lib):
    w, eta = small
    ctx = agis_mod.agis_create(w.consts, w.knots)
    n_src = w.src_true.shape[0]
    bad_src = w.src.copy()
    bad_src[10] = n_src
    with pytest.raises(agis_mod.AgisError) as e:
        agis_mod.agis_load_observations(ctx, w.t, eta, w.sigma, bad_src, w.fov, w.cell, n_src, w.n_cells)
    assert e.value.code == -3
    bad_t = w.t.copy()
    bad_t[5] = w.knots[-1] + 10.0
    with pytest.raises(agis_mod.AgisError) as e:
        agis_mod.agis_load_observations(ctx, bad_t, eta, w.sigma, w.src, w.fov, w.cell, n_src, w.n_cells)
    assert e.value.code == -3
    bad_fov = w.fov.copy()
    bad_fov[3] = 0
    with pytest.raises(agis_mod.AgisError):
        agis_mod.agis_load_observations(ctx, w.t, eta, w.sigma, w.src, bad_fov, w.cell, n_src, w.n_cells)
    with pytest.raises(agis_mod.AgisError) as e:
        agis_mod.agis_source_update(ctx)
    assert e.value.code == -7
    agis_mod.agis_destroy(ctx)


def test_device_pointer_inputs(agis_mod, small, oracle_lib):
    import torch
    w, eta = small
    dev = torch.device("cuda:0")
    ctx = agis_mod.agis_create(w.consts, w.knots)
    cols = [torch.from_numpy(x).to(dev) for x in (w.t, eta, w.sigma, w.src, w.fov, w.cell)]
    agis_mod.agis_load_observations(ctx, *cols, w.src_true.shape[0], w.n_cells)
    agis_mod.agis_set_sources(ctx, torch.from_numpy(w.src_start).to(dev))
    agis_mod.agis_set_attitude(ctx, torch.from_numpy(w.att_start).to(dev))
    agis_mod.agis_set_calibration(ctx, torch.from_numpy(w.cal_start).to(dev))
    torch.cuda.synchronize()
    R = torch.empty(w.n_obs, dtype=torch.float64, device=dev)
    agis_mod.agis_residuals(ctx, R)
    pr = oracle_lib.problem_from_world(w, eta, state="start")
    assert np.abs(R.cpu().numpy() - pr.observe()["R"]).max() / UAS < TOL_UAS
    agis_mod.agis_destroy(ctx)
