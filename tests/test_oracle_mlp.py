"""Pins of the oracle MLP: SplitMix64 reference output, finite-difference
gradients, the closed-form first Adam step, bfloat16 rounding."""
import numpy as np

from oracle import mlp


def test_splitmix64_reference_value():
    # Vigna's SplitMix64 seeded with 0: first output 0xE220A8397B1DCDAF
    assert mlp.splitmix64(0, 0) == 0xE220A8397B1DCDAF


def test_init_range_and_determinism():
    n, H = 9, 6
    th = mlp.init_params(n, H, seed=7)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(th, n, H)
    assert np.all(np.abs(W1) <= np.sqrt(6 / n)) and np.all(b1 == 0)
    assert np.all(np.abs(W3) <= np.sqrt(6 / H))
    assert np.array_equal(th, mlp.init_params(n, H, seed=7))
    assert not np.array_equal(th, mlp.init_params(n, H, seed=8))


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    n, H, B = 7, 5, 6
    th = mlp.init_params(n, H, seed=3) + 0.05 * rng.standard_normal(mlp.n_params(n, H))
    X = rng.standard_normal((B, n))
    T = rng.standard_normal((B, n))
    L, g = mlp.loss_and_grad(th, X, T, n, H)
    h = 1e-6
    for i in range(len(th)):
        e = np.zeros_like(th)
        e[i] = h
        Lp, _ = mlp.loss_and_grad(th + e, X, T, n, H)
        Lm, _ = mlp.loss_and_grad(th - e, X, T, n, H)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_first_adam_step_closed_form():
    # from zero moments the first step is theta - lr g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th = np.array([1.0, 2.0, 3.0, 4.0])
    opt = mlp.Adam(4, lr=0.01)
    new = opt.step(th, g)
    np.testing.assert_allclose(new, th - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=1e-15)


def test_bf16_rounding():
    x = np.array([1.0, 1.00390625, 1.005859375, 3.0e38, -2.5], dtype=np.float32)
    r = mlp.bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                 # halfway (1 + 2^-8) ties to even: 1.0
    assert r[2] == np.float32(1.0078125)  # above halfway rounds up
    assert r[4] == -2.5
    # every result has a zero low half-word
    assert np.all((r.view(np.uint32) & 0xFFFF) == 0)
