"""Pins of the float64 network reference: bfloat16 rounding against hand
values, and the analytic gradient against central finite differences."""
import numpy as np

from oracle import mlp


def test_bf16_rounding_hand_values():
    # representable neighbours of 1 in bfloat16 are 1 and 1 + 2^-7
    assert mlp.bf16(1.0) == 1.0
    assert mlp.bf16(1.0 + 2.0 ** -7) == 1.0 + 2.0 ** -7
    assert mlp.bf16(1.0 + 2.0 ** -8) == 1.0                 # tie -> even (1.0)
    assert mlp.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6  # tie -> even
    assert mlp.bf16(1.0 + 2.0 ** -8 + 2.0 ** -12) == 1.0 + 2.0 ** -7
    assert mlp.bf16(-2.5) == -2.5
    assert mlp.bf16(0.0) == 0.0


def test_gradient_matches_finite_differences():
    g = np.random.default_rng(0)
    X = g.normal(size=(24, 32))
    T = g.normal(size=24)
    p = np.concatenate([g.normal(0, 0.25, 128 * 32), g.normal(0, 0.1, 128),
                        g.normal(0, 0.1, 128 * 128), g.normal(0, 0.1, 128),
                        g.normal(0, 0.3, 128), [0.2]])
    G, L = mlp.grad(X, T, p, emulate=False)
    assert abs(L - mlp.loss(X, T, p)) < 1e-15
    idx = np.concatenate([g.choice(np.arange(mlp.OW1, mlp.OB1), 12),
                          g.choice(np.arange(mlp.OB1, mlp.OW2), 6),
                          g.choice(np.arange(mlp.OW2, mlp.OB2), 12),
                          g.choice(np.arange(mlp.OB2, mlp.OW3), 6),
                          g.choice(np.arange(mlp.OW3, mlp.OB3), 6), [mlp.OB3]])
    eps = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        fd = (mlp.loss(X, T, pp) - mlp.loss(X, T, pm)) / (2 * eps)
        assert abs(fd - G[i]) <= 1e-6 * max(1.0, abs(G[i])), (i, fd, G[i])


def test_emulated_forward_close_to_exact():
    g = np.random.default_rng(1)
    X = g.normal(size=(40, 32))
    p = g.normal(0, 0.1, mlp.NPARAMS)
    a, _ = mlp.forward(X, p, emulate=False)
    b, _ = mlp.forward(X, p, emulate=True)
    assert np.max(np.abs(a - b)) <= 2e-2 * np.max(np.abs(a))
