"""Pins of the scorer reference: bf16 rounding against hand-worked cases,
and the backward pass against central finite differences of the exact
(unrounded) float64 model.  CPU only."""
import numpy as np

from oracle import mlp_ref


def test_bf16_rounding_cases():
    eps = 2.0 ** -7                     # bf16 spacing just above 1.0
    cases = [
        (1.0, 1.0),
        (1.0 + eps / 2, 1.0),           # tie -> even (mantissa 0)
        (1.0 + 3 * eps / 2, 1.0 + 2 * eps),   # tie -> even (mantissa 2)
        (1.0 + eps / 4, 1.0),
        (1.0 + 3 * eps / 4, 1.0 + eps),
        (-2.5, -2.5),
        (3.0e38, 1.765625 * 2.0 ** 127),   # 3e38 = 1.7632 * 2^127 -> 98/128
        (0.0, 0.0),
    ]
    for x, want in cases:
        got = float(mlp_ref.bf16_round(np.float32(x)))
        assert np.isclose(got, want, rtol=0, atol=abs(want) * 1e-7), (x, got, want)
    bits = mlp_ref.bf16_bits(np.array([1.0, -2.0, 0.5], np.float32))
    assert list(bits) == [0x3F80, 0xC000, 0x3F00]
    assert list(mlp_ref.from_bf16_bits(bits)) == [1.0, -2.0, 0.5]


def test_gradients_match_finite_differences():
    rng = np.random.Generator(np.random.PCG64(31))
    F, H, B = 6, 10, 9
    p = {k: v.astype(np.float64) for k, v in mlp_ref.init_params(rng, F, H).items()}
    p["b1"] = rng.standard_normal(H) * 0.1
    p["b2"] = rng.standard_normal(H) * 0.1
    X = rng.standard_normal((B, F))
    t = rng.standard_normal(B)
    g, _ = mlp_ref.backward(p, X, t, rounding=False)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for i in range(0, flat.size, max(1, flat.size // 7)):
            old = flat[i]
            flat[i] = old + h
            lp = mlp_ref.loss(p, X, t, rounding=False)
            flat[i] = old - h
            lm = mlp_ref.loss(p, X, t, rounding=False)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-7, (k, i, fd, an)


def test_rounded_forward_is_close_to_exact():
    rng = np.random.Generator(np.random.PCG64(32))
    p = mlp_ref.init_params(rng)
    X = rng.standard_normal((50, 16))
    y_r, _ = mlp_ref.forward(p, X, True)
    y_e, _ = mlp_ref.forward(p, X, False)
    assert np.max(np.abs(y_r - y_e)) < 0.05 * (np.max(np.abs(y_e)) + 1)


def test_adam_decreases_loss():
    rng = np.random.Generator(np.random.PCG64(33))
    p = mlp_ref.init_params(rng, 8, 32)
    X = rng.standard_normal((64, 8))
    t = X[:, 0] * 0.5 - X[:, 1]
    m = {k: np.zeros_like(v, np.float64) for k, v in p.items()}
    v = {k: np.zeros_like(x, np.float64) for k, x in p.items()}
    l0 = mlp_ref.loss(p, X, t)
    for s in range(1, 200):
        g, _ = mlp_ref.backward(p, X, t)
        mlp_ref.adam_step(p, g, m, v, s, lr=3e-3)
    assert mlp_ref.loss(p, X, t) < 0.2 * l0
