"""Pins of the FP64 MLP reference: bfloat16 rounding, a closed-form special
case, the mixing head against a brute-force sum, and central finite
differences of a loss written out independently."""
import numpy as np

from oracle import mlp


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 0.0, 3.0e-30], np.float32)
    r = mlp.bf16_round(x)
    # 8 significand bits: 1 + 2^-8 is halfway (ties to even -> 1), 1 + 3 2^-8 -> 1 + 2^-6
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == np.float32(1.0 + 2 ** -7)
    assert r[3] == np.float32(1.0 + 2 ** -6) and r[4] == -2.5 and r[5] == 0.0
    assert abs(r[6] / 3.0e-30 - 1) < 2 ** -8
    assert np.all(mlp.bf16_round(r) == r)


def test_forward_special_case():
    F, O = 22, 4
    rng = np.random.default_rng(1)
    p = {name: np.zeros(s) for name, s in mlp.shapes(F, O)}
    p["b3"] = np.array([0.5, -1.0, 2.0, 0.25])
    p["W1"] = rng.normal(size=(64, F))
    w = mlp.pack(p, F, O)
    X = rng.normal(size=(7, F))
    # W2 = 0, b2 = 0 => h2 = 0 => y = b3 for any input
    assert np.array_equal(mlp.forward(w, X, F, O), np.tile(p["b3"], (7, 1)))


def test_mixing_head():
    """c = e_k mixes in exactly the k-th group of inputs."""
    rng = np.random.default_rng(3)
    X = rng.normal(size=(5, 22))
    for k in range(4):
        c = np.zeros((5, 4))
        c[:, k] = 1.0
        assert np.array_equal(mlp.mix(c, X, 5), X[:, 5 * k:5 * k + 5])
    c = rng.normal(size=(5, 4))
    brute = np.array([[sum(c[i, k] * X[i, 5 * k + j] for k in range(4)) for j in range(5)] for i in range(5)])
    assert np.allclose(mlp.mix(c, X, 5), brute, rtol=1e-14, atol=1e-14)


def test_gradient_finite_differences():
    for F, O, nc, seed in ((18, 4, 4, 2), (22, 4, 5, 4)):
        rng = np.random.default_rng(seed)
        # weights already on the bfloat16 grid, so that rounding is the identity
        w = mlp.bf16_round(rng.normal(scale=0.3, size=mlp.n_weights(F, O)).astype(np.float32)).astype(np.float64)
        X = rng.normal(size=(16, F))
        T = rng.normal(size=(16, nc))
        L, g = mlp.loss_and_gradient(w, X, T, F, O, nc)

        def loss_exact(wv):
            p = mlp.unpack(wv, F, O)
            h1 = np.tanh(X @ p["W1"].T + p["b1"])
            h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
            c = h2 @ p["W3"].T + p["b3"]
            yh = np.stack([sum(c[:, k] * X[:, k * nc + j] for k in range(O)) for j in range(nc)], axis=1)
            return 0.5 * np.sum((yh - T) ** 2) / X.shape[0]

        assert abs(loss_exact(w) - L) < 1e-13 * max(1.0, L)
        idx = rng.choice(w.size, 60, replace=False)
        for k in idx:
            e = np.zeros_like(w)
            e[k] = 1e-6
            fd = (loss_exact(w + e) - loss_exact(w - e)) / 2e-6
            assert abs(fd - g[k]) < 1e-7 * max(1.0, abs(g[k]))
