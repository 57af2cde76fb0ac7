"""Learned extrapolation on the GPU: the MLP forward and gradient kernels
against the FP64 NumPy network (same bfloat16-rounded weights), training,
the update history and features against values computed on the host from
the recorded states, the candidate arithmetic, and the gate of the learned
step (a rejected candidate leaves exactly the plain iterate; a linear
extrapolation along the slow mode is accepted)."""
import numpy as np
import pytest

import synth.configs as C
from oracle import mlp
from test_gpu_parity import agis_mod  # noqa: F401

pytestmark = pytest.mark.gpu

F_IN = (22, 18)
F_OUT = (4, 4)                 # mixing coefficients
NC = (5, 4)                    # update components (target columns)


@pytest.fixture(scope="module")
def tiny(oracle_lib):
    w = C.make("tiny")
    return w, oracle_lib.observed_field_angles(w)


def _ctx(agis, w, eta, with_ref=True):
    ctx = agis.agis_create(w.consts, w.knots)
    agis.agis_load_observations(ctx, w.t, eta, w.sigma, w.src, w.fov, w.cell, w.src_true.shape[0], w.n_cells)
    agis.agis_set_sources(ctx, w.src_start)
    agis.agis_set_attitude(ctx, w.att_start)
    agis.agis_set_calibration(ctx, w.cal_start)
    if with_ref:
        agis.agis_set_frame_reference(ctx, w.src_true)
    return ctx


def _state(agis, ctx, w):
    return (agis.agis_get_sources(ctx, w.src_true.shape[0]), agis.agis_get_attitude(ctx, w.n_att),
            agis.agis_get_calibration(ctx, w.n_cells))


def _weights(which, **parts):
    p = {name: np.zeros(s) for name, s in mlp.shapes(F_IN[which], F_OUT[which])}
    p.update(parts)
    return mlp.pack(p, F_IN[which], F_OUT[which]).astype(np.float32)


@pytest.mark.parametrize("which", [0, 1])
def test_mlp_forward_vs_reference(agis_mod, tiny, which):
    """FP32 accumulation over at most 64 terms of O(1): a few 1e-6."""
    w, eta = tiny
    ctx = _ctx(agis_mod, w, eta)
    agis_mod.agis_mlp_init(ctx, which, 7 + which)
    wt = agis_mod.agis_mlp_get_weights(ctx, which)
    rng = np.random.default_rng(11 + which)
    n = 3 * 256 + 77                                   # several blocks and a ragged tail
    X = rng.normal(size=(n, F_IN[which])).astype(np.float32)
    Yg = agis_mod.agis_mlp_forward(ctx, which, X)
    Yr = mlp.forward(wt, X, F_IN[which], F_OUT[which])
    err = np.abs(Yg - Yr).max()
    print(f"net {which}: max |Y_gpu - Y_ref| = {err:.2e} (max |Y| {np.abs(Yr).max():.2f})")
    assert err < 2e-5 * max(1.0, np.abs(Yr).max())
    assert agis_mod.agis_mlp_forward(ctx, which, X[:0]).shape == (0, F_OUT[which])
    agis_mod.agis_destroy(ctx)


@pytest.mark.parametrize("which", [0, 1])
def test_mlp_gradient_vs_reference(agis_mod, tiny, which):
    w, eta = tiny
    ctx = _ctx(agis_mod, w, eta)
    agis_mod.agis_mlp_init(ctx, which, 3)
    wt = agis_mod.agis_mlp_get_weights(ctx, which)
    rng = np.random.default_rng(21 + which)
    n = 7 * 128 + 45                                   # ragged gradient block
    X = rng.normal(size=(n, F_IN[which])).astype(np.float32)
    T = rng.normal(size=(n, NC[which])).astype(np.float32)
    g, L = agis_mod.agis_mlp_gradient(ctx, which, X, T)
    Lr, gr = mlp.loss_and_gradient(wt, X, T, F_IN[which], F_OUT[which], NC[which])
    rel = np.abs(g - gr).max() / np.abs(gr).max()
    print(f"net {which}: loss {L:.6g} vs {Lr:.6g}; max gradient error / max |gradient| = {rel:.2e}")
    assert abs(L - Lr) <= 1e-5 * Lr
    assert rel < 1e-4
    # one block's worth and a single sample
    for m in (128, 1):
        g, L = agis_mod.agis_mlp_gradient(ctx, which, X[:m], T[:m])
        Lr, gr = mlp.loss_and_gradient(wt, X[:m], T[:m], F_IN[which], F_OUT[which], NC[which])
        assert abs(L - Lr) <= 1e-5 * Lr and np.abs(g - gr).max() < 1e-4 * np.abs(gr).max()
    agis_mod.agis_destroy(ctx)


def test_mlp_training(agis_mod, tiny):
    """Adam on a smooth target lowers the loss; the same seeds give the
    same weights bit for bit (fixed-order reductions)."""
    w, eta = tiny
    rng = np.random.default_rng(5)
    X = rng.normal(size=(5000, 22)).astype(np.float32)
    M = rng.normal(scale=0.3, size=(22, 4))
    T = mlp.mix(np.tanh(X @ M), X, 5).astype(np.float32)
    runs = []
    for _ in range(2):
        ctx = _ctx(agis_mod, w, eta)
        agis_mod.agis_mlp_init(ctx, 0, 1)
        loss = agis_mod.agis_mlp_train(ctx, 0, X, T, 400, 256, 3e-3, seed=9)
        runs.append((loss, agis_mod.agis_mlp_get_weights(ctx, 0)))
        L_full = mlp.loss_and_gradient(runs[-1][1], X, T, 22, 4, 5)[0]
        agis_mod.agis_destroy(ctx)
    loss = runs[0][0]
    print(f"loss {loss[:10].mean():.4f} -> {loss[-50:].mean():.4f}; full-set loss of the result {L_full:.4f}")
    assert loss[-50:].mean() < 0.2 * loss[:10].mean()
    assert np.array_equal(runs[0][1], runs[1][1]) and np.array_equal(runs[0][0], runs[1][0])


def test_history_and_features(agis_mod, tiny):
    w, eta = tiny
    ctx = _ctx(agis_mod, w, eta)
    agis_mod.agis_iterate(ctx, 5, stats=False)
    agis_mod.agis_learned_reset(ctx)
    prev = _state(agis_mod, ctx, w)
    ups_s, ups_a = [], []
    for r in range(6):                                 # ring of four wraps around
        agis_mod.agis_iterate(ctx, 2 + r, stats=False)
        agis_mod.agis_learned_record(ctx)
        cur = _state(agis_mod, ctx, w)
        d = cur[0] - prev[0]
        d[:, 0] *= np.cos(cur[0][:, 1])
        ups_s.append(d)
        ups_a.append(cur[1] - prev[1])
        prev = cur
        if r < 3:
            with pytest.raises(RuntimeError):
                agis_mod.agis_learned_features(ctx, 0)
    s, a, _ = prev
    nobs = np.bincount(w.src, minlength=s.shape[0])
    eps = w.consts["eps_obl"]
    for which, ups, nc in ((0, ups_s, 5), (1, ups_a, 4)):
        H = np.concatenate(ups[::-1][:4], axis=1)        # newest first
        sc = np.sqrt(np.mean(H * H, axis=1))
        Xh = H / np.where(sc > 0, sc, np.inf)[:, None]
        Xg, scg = agis_mod.agis_learned_features(ctx, which)
        np.testing.assert_allclose(scg, sc.astype(np.float32), rtol=2e-7, atol=0)
        np.testing.assert_allclose(Xg[:, :4 * nc], Xh.astype(np.float32), rtol=2e-7, atol=1e-7)
        if which == 0:
            desc = np.stack([np.log(nobs + 1.0) / 5,
                             -np.sin(eps) * np.cos(s[:, 1]) * np.sin(s[:, 0]) + np.cos(eps) * np.sin(s[:, 1])], 1)
        else:
            ph = 2 * np.arctan2(a[:, 2], a[:, 3])
            desc = np.stack([np.sin(ph), np.cos(ph)], 1)
        np.testing.assert_allclose(Xg[:, 4 * nc:], desc.astype(np.float32), rtol=0, atol=2e-7)
    agis_mod.agis_destroy(ctx)


def test_candidate_arithmetic(agis_mod, tiny):
    """With W3 = 0 the networks output b3; learned_apply then moves every
    unit by sum_k b3_k u_k over its recorded updates (newest first; for
    sources d alpha* converted to d alpha), and starts a new history."""
    w, eta = tiny
    ctx = _ctx(agis_mod, w, eta)
    agis_mod.agis_learned_reset(ctx)
    prev = _state(agis_mod, ctx, w)
    ups_s, ups_a = [], []
    for r in range(5):
        agis_mod.agis_iterate(ctx, 3 + r, stats=False)
        agis_mod.agis_learned_record(ctx)
        cur = _state(agis_mod, ctx, w)
        d = cur[0] - prev[0]
        d[:, 0] *= np.cos(cur[0][:, 1])
        ups_s.append(d)
        ups_a.append(cur[1] - prev[1])
        prev = cur
    b_s = np.array([0.5, -1.25, 2.0, 0.75])
    b_a = np.array([1.5, -0.5, 0.25, -2.0])
    agis_mod.agis_mlp_load(ctx, 0, _weights(0, b3=b_s, W1=np.ones((64, 22))))
    agis_mod.agis_mlp_load(ctx, 1, _weights(1, b3=b_a, W1=np.ones((64, 18))))
    s0, a0, c0 = _state(agis_mod, ctx, w)
    agis_mod.agis_learned_apply(ctx)
    s1, a1, c1 = _state(agis_mod, ctx, w)
    ds = sum(b * u for b, u in zip(b_s, ups_s[::-1]))
    ds[:, 0] /= np.cos(s0[:, 1])
    da = sum(b * u for b, u in zip(b_a, ups_a[::-1]))
    # x + d rounds once in FP64: within one unit in the last place of x
    # (and d itself carries the rounding of the recorded differences)
    tol_s = np.spacing(np.abs(s0)) + 1e-12 * np.abs(ds) + 8 * np.spacing(np.abs(s0)).max(axis=0)
    assert np.all(np.abs(s1 - (s0 + ds)) <= tol_s)
    assert np.all(np.abs(a1 - (a0 + da)) <= 8 * np.spacing(np.abs(a0)) + 1e-12 * np.abs(da))
    assert np.abs(ds).max() > 0 and np.abs(da).max() > 0
    assert np.array_equal(c1, c0)
    with pytest.raises(RuntimeError):                  # history restarted
        agis_mod.agis_learned_features(ctx, 0)
    agis_mod.agis_destroy(ctx)


def _twins(agis, w, eta, n_pre, m):
    """Two contexts on the same trajectory: n_pre plain iterations, then a
    history of four records m iterations apart."""
    out = []
    for _ in range(2):
        ctx = _ctx(agis, w, eta)
        agis.agis_iterate(ctx, n_pre, stats=False)
        agis.agis_learned_reset(ctx)
        for _ in range(4):
            agis.agis_iterate(ctx, m, stats=False)
            agis.agis_learned_record(ctx)
        out.append(ctx)
    return out


@pytest.mark.parametrize("b3", [0.0, 1.0e3])
def test_rejected_candidate_is_the_plain_iterate(agis_mod, tiny, b3):
    """Zero output: the candidate iteration repeats the plain one (the source
    data recomputed from the restored parameters), q_cand equals q_plain to
    rounding, and the strict test rejects it or not.  A large shift: rejected.  Either way the state is
    the plain iterate one iteration on, bit for bit."""
    w, eta = tiny
    ctx, twin = _twins(agis_mod, w, eta, 10, 5)
    agis_mod.agis_mlp_load(ctx, 0, _weights(0, b3=np.full(4, b3)))
    agis_mod.agis_mlp_load(ctx, 1, _weights(1, b3=np.full(4, b3)))
    r = agis_mod.agis_learned_step(ctx)
    agis_mod.agis_iterate(twin, 1, stats=False)
    print(r)
    assert r["q_plain"] == agis_mod.agis_chi2(twin)
    if b3 == 0.0:
        assert abs(r["q_candidate"] - r["q_plain"]) <= 1e-12 * r["q_plain"]
        if r["accepted"]:
            return
    else:
        assert not r["accepted"] and r["q_candidate"] > r["q_plain"]
    for x, y in zip(_state(agis_mod, ctx, w), _state(agis_mod, twin, w)):
        assert np.array_equal(x, y)
    agis_mod.agis_learned_record(ctx)                 # the history goes on
    agis_mod.agis_learned_features(ctx, 0)
    agis_mod.agis_destroy(ctx)
    agis_mod.agis_destroy(twin)


def test_linear_extrapolation_is_accepted(agis_mod, tiny):
    """Once the simple iteration decays geometrically, k times the newest
    update ahead is closer to the solution: networks that output the
    coefficients (k, 0, 0, 0) give a candidate that the gate keeps, and the
    state is one iteration on from x0 + k (newest update)."""
    w, eta = tiny
    ctx, twin = _twins(agis_mod, w, eta, 2000, 20)
    for which in (0, 1):
        agis_mod.agis_mlp_load(ctx, which, _weights(which, b3=np.array([4.0, 0.0, 0.0, 0.0])))
    q0 = agis_mod.agis_chi2(ctx)
    r = agis_mod.agis_learned_step(ctx)
    print(r, "chi2 before", q0)
    assert r["accepted"] and r["q_candidate"] < r["q_plain"] < q0
    with pytest.raises(RuntimeError):                  # new history
        agis_mod.agis_learned_features(ctx, 0)
    # the twin takes the same candidate without the gate, then one iteration
    for which in (0, 1):
        agis_mod.agis_mlp_load(twin, which, agis_mod.agis_mlp_get_weights(ctx, which))
    agis_mod.agis_learned_apply(twin)
    agis_mod.agis_iterate(twin, 1, stats=False)
    for x, y in zip(_state(agis_mod, ctx, w), _state(agis_mod, twin, w)):
        assert np.array_equal(x, y)
    agis_mod.agis_destroy(ctx)
    agis_mod.agis_destroy(twin)


@pytest.mark.parametrize("stride,lambda_max", [(1, 0.99), (7, 0.99), (3, 0.5)])
def test_asi_step(agis_mod, tiny, stride, lambda_max):
    """Accelerated step: lambda is the least-squares ratio of the two newest
    parallax updates over every stride-th source (clamped), and sources,
    attitude and calibration move by lambda / (1 - lambda) times their
    newest update; a new history starts."""
    w, eta = tiny
    ctx = _ctx(agis_mod, w, eta)
    agis_mod.agis_iterate(ctx, 200, stats=False)
    agis_mod.agis_learned_reset(ctx)
    prev = _state(agis_mod, ctx, w)
    ups = []
    for r in range(3):
        agis_mod.agis_iterate(ctx, 10, stats=False)
        agis_mod.agis_learned_record(ctx)
        cur = _state(agis_mod, ctx, w)
        d = [cur[0] - prev[0], cur[1] - prev[1], cur[2] - prev[2]]
        d[0][:, 0] *= np.cos(cur[0][:, 1])
        ups.append(d)
        prev = cur
    u1, u2 = ups[-1][0][::stride, 2], ups[-2][0][::stride, 2]
    lam = min(max(np.sum(u1 * u2) / np.sum(u2 * u2), 0.0), lambda_max)
    f = lam / (1 - lam)
    s0, a0, c0 = prev
    r = agis_mod.agis_asi_step(ctx, stride, lambda_max)
    print(r, "host lambda", lam)
    assert abs(r["lam"] - lam) <= 1e-12 and abs(r["factor"] - f) <= 1e-12 * f
    assert f > 0
    s1, a1, c1 = _state(agis_mod, ctx, w)
    ds = r["factor"] * ups[-1][0]
    ds[:, 0] /= np.cos(s0[:, 1])
    assert np.all(np.abs(s1 - (s0 + ds)) <= 2 * np.spacing(np.abs(s0)) + 1e-12 * np.abs(ds))
    for x1, x0, u in ((a1, a0, ups[-1][1]), (c1, c0, ups[-1][2])):
        assert np.all(np.abs(x1 - (x0 + r["factor"] * u)) <= 2 * np.spacing(np.abs(x0)) + 1e-12 * np.abs(u) * f)
    with pytest.raises(RuntimeError):                  # new history: fewer than two records
        agis_mod.agis_asi_step(ctx, stride, lambda_max)
    with pytest.raises(RuntimeError):                  # invalid stride
        agis_mod.agis_asi_step(ctx, 0, 0.9)
    agis_mod.agis_destroy(ctx)


def test_learned_solve_beats_plain(agis_mod):
    """Train both networks on one plain trajectory of the tiny world (seed
    1), then iterate seed 0 with and without the gated learned step for the
    same number of S[AC] iterations (the gate's included): the learned
    iterate has the lower sum W R^2, i.e. it is closer to the solution in the
    norm of the normal matrix, and the gate kept some of its candidates."""
    from paper_1112_4139_amd import learned

    m, horizon = 50, 20
    w1, ctx1 = learned.problem("tiny", 1)
    data = learned.collect(ctx1, w1, m, 60, horizon)
    for which in (0, 1):
        X, T = data[which]
        agis_mod.agis_mlp_init(ctx1, which, 5 + which)
        loss = np.concatenate([agis_mod.agis_mlp_train(ctx1, which, X, T, n, 1024, lr, seed=3 + which)
                               for n, lr in ((2000, 1e-3), (1000, 2.5e-4))])
        print(f"net {which}: {X.shape[0]} samples, loss {loss[:20].mean():.3g} -> {loss[-100:].mean():.3g}")
        assert loss[-100:].mean() < 0.3 * loss[:20].mean()
    weights = [agis_mod.agis_mlp_get_weights(ctx1, which) for which in (0, 1)]
    agis_mod.agis_destroy(ctx1)
    chi2 = {}
    for mode in ("learned", "plain"):
        w0, ctx = learned.problem("tiny", 0)
        for which in (0, 1):
            agis_mod.agis_mlp_load(ctx, which, weights[which])
        agis_mod.agis_learned_reset(ctx)
        it, count, acc = 0, 0, 0
        if mode == "learned":
            while it < 4000:
                agis_mod.agis_iterate(ctx, m, stats=False)
                agis_mod.agis_learned_record(ctx)
                it, count = it + m, count + 1
                if count >= 4:
                    r = agis_mod.agis_learned_step(ctx)
                    it += 2
                    if r["accepted"]:
                        acc, count = acc + 1, 0
        else:
            # as many S[AC] iterations as the learned run took
            it = chi2["learned"][1]
            agis_mod.agis_iterate(ctx, it, stats=False)
        chi2[mode] = (agis_mod.agis_chi2(ctx), it, acc)
        agis_mod.agis_destroy(ctx)
    print(chi2)
    assert chi2["learned"][2] > 0
    assert chi2["learned"][0] < chi2["plain"][0]


def test_mlp_train_step(agis_mod, tiny):
    """One Adam step on a whole batch: the returned loss is the batch loss at
    the weights before the step (as agis_mlp_gradient gives it), and the
    first Adam step moves every weight with a gradient well above Adam's
    epsilon by lr against its gradient's sign (m_hat = g, v_hat = g^2)."""
    w, eta = tiny
    rng = np.random.default_rng(11)
    X = rng.normal(size=(700, 22)).astype(np.float32)
    T = rng.normal(size=(700, 5)).astype(np.float32)
    ctx = _ctx(agis_mod, w, eta)
    agis_mod.agis_mlp_init(ctx, 0, 21)
    w0 = agis_mod.agis_mlp_get_weights(ctx, 0)
    g, L = agis_mod.agis_mlp_gradient(ctx, 0, X, T)
    lr = 1e-3
    L1 = agis_mod.agis_mlp_train_step(ctx, 0, X, T, lr)
    w1 = agis_mod.agis_mlp_get_weights(ctx, 0)
    assert L1 == L
    big = np.abs(g) > 1e-4
    assert big.sum() > 1000
    np.testing.assert_allclose(w1[big] - w0[big], -lr * np.sign(g[big]), rtol=2e-3, atol=2e-9)
    assert np.all(np.abs(w1 - w0) <= lr * (1 + 1e-3))
    agis_mod.agis_destroy(ctx)


def test_iterate_learned_is_the_block_loop(agis_mod, tiny):
    """agis_iterate_learned runs, per block, m iterations, a record and from
    the fourth record on the gated step: the same state bit for bit as those
    calls made one by one, with the same gate decisions (networks that
    extrapolate along the newest update, whose candidates the gate keeps;
    after a kept one the history needs four new records)."""
    w, eta = tiny
    m, n_blocks = 20, 9
    weights = [_weights(which, b3=np.array([4.0, 0.0, 0.0, 0.0])) for which in (0, 1)]
    ctx, twin = (_ctx(agis_mod, w, eta) for _ in range(2))
    for c in (ctx, twin):
        agis_mod.agis_iterate(c, 1000, stats=False)
        for which in (0, 1):
            agis_mod.agis_mlp_load(c, which, weights[which])
    st = agis_mod.agis_iterate_learned(ctx, n_blocks, m)
    agis_mod.agis_learned_reset(twin)
    count, manual = 0, []
    for b in range(n_blocks):
        agis_mod.agis_iterate(twin, m, stats=False)
        agis_mod.agis_learned_record(twin)
        count += 1
        if count >= 4:
            r = agis_mod.agis_learned_step(twin)
            manual.append((m + 2, True, r["accepted"], r["q_plain"], r["q_candidate"]))
            if r["accepted"]:
                count = 0
        else:
            manual.append((m, False, False, 0.0, 0.0))
    got = [(x["iterations"], x["gated"], x["accepted"], x["q_plain"], x["q_candidate"]) for x in st]
    print(got)
    assert got == manual
    assert sum(x[2] for x in got) >= 2 and sum(x[1] for x in got) >= 2
    for x, y in zip(_state(agis_mod, ctx, w), _state(agis_mod, twin, w)):
        assert np.array_equal(x, y)
    with pytest.raises(RuntimeError):
        agis_mod.agis_iterate_learned(ctx, 1, 0)
    agis_mod.agis_destroy(ctx)
    agis_mod.agis_destroy(twin)


def test_asi_trajectory_parity(agis_mod, oracle_lib, tiny):
    """Accelerated simple iteration (Sect. 4.7) from the start values: nine
    records of two iterations with the frame rotator and an accelerated step
    from every third record, on the GPU and in the oracle's own scheme
    (oracle.asi, extended precision as the reference).  The same three
    steps are taken with the same lambda, and every parameter ends within the
    FP64-floor tolerance of the other parity tests, which here carries the
    rounding of the recorded updates through factors lambda / (1 - lambda)
    of up to ~16."""
    from oracle.asi import AcceleratedIteration
    from test_gpu_parity import check_floor, fp64_floor

    w, eta = tiny
    m, n_blocks, stride = 2, 9, 16

    def run(pr):
        acc = AcceleratedIteration(pr, w.src_true, stride=stride, lambda_max=0.99)
        run.steps.append(acc.run(n_blocks, m))
        return pr.s.copy(), pr.a.copy(), pr.c.copy()

    run.steps = []
    X, O, tol = fp64_floor(oracle_lib, w, eta, run)
    steps_x, steps_o = run.steps[0], run.steps[1]
    ctx = _ctx(agis_mod, w, eta)
    agis_mod.agis_learned_reset(ctx)
    count, steps_g = 0, []
    for _ in range(n_blocks):
        agis_mod.agis_iterate(ctx, m, stats=False)
        agis_mod.agis_learned_record(ctx)
        count += 1
        if count >= 3:
            r = agis_mod.agis_asi_step(ctx, stride, 0.99)
            steps_g.append((r["lam"], r["factor"]))
            if r["factor"] > 0:
                count = 0
    G = _state(agis_mod, ctx, w)
    print("lambda (GPU, extended, FP64 oracle):", [(g[0], float(x[0]), o[0])
                                                   for g, x, o in zip(steps_g, steps_x, steps_o)])
    assert len(steps_g) == len(steps_x) == 3 and all(f > 0 for _, f in steps_g)
    # lambda's own floor, by the rule of the parameters: its response to the
    # 3e-16 rad perturbations of the residuals (fp64_floor's draws) and the
    # FP64 oracle's deviation
    from test_gpu_parity import FLOOR_FACTOR
    for k, (g, x, o) in enumerate(zip(steps_g, steps_x, steps_o)):
        sens = np.sqrt(np.mean([(p[k][0] - o[0]) ** 2 for p in run.steps[2:]]))
        tol_lam = max(1e-10, FLOOR_FACTOR * sens)
        print(f"step {k}: |lambda GPU - ext| {abs(g[0] - float(x[0])):.2e}, tolerance {tol_lam:.2e}")
        assert abs(g[0] - float(x[0])) <= tol_lam
    check_floor("ASI: sources", X[0], O[0], G[0], tol[0], 0)
    check_floor("ASI: attitude", X[1], O[1], G[1], tol[1], 1)
    check_floor("ASI: calibration", X[2], O[2], G[2], tol[2], 2)
    agis_mod.agis_destroy(ctx)
