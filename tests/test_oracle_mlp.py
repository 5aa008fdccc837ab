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


def _bf16_exact_problem():
    """A batch, parameters and targets for which every value the emulation
    rounds (inputs, W1, W2, first activations, the two propagated errors) is
    already a bfloat16 number: small integers times powers of two with at
    most eight significant bits."""
    g = np.random.default_rng(3)
    B = 8
    X = g.integers(-1, 2, size=(B, 32)).astype(float)
    W1 = g.integers(-1, 2, size=(128, 32)) * 0.25
    b1 = g.integers(-2, 3, size=128) * 0.25
    W2 = g.integers(-1, 2, size=(128, 128)) * (g.random((128, 128)) < 0.12) * 2.0 ** -4
    b2 = g.integers(-2, 3, size=128) * 2.0 ** -6
    w3 = g.integers(-1, 2, size=128) * 2.0 ** -3
    p = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [0.125]])
    out, _ = mlp.forward(X, p, emulate=False)
    # targets that make out - T a power of two: g = 2 (out - T) / B is dyadic
    T = out - np.array([0.5, -0.25, 1.0, -0.5, 0.25, -1.0, 0.5, 0.125])
    return X, T, p


def test_emulation_changes_nothing_on_bf16_exact_values():
    """Where every rounded operand is already a bfloat16 number, the emulated
    forward and gradient equal the exact float64 ones bit for bit: the
    emulation only rounds, at the matrix-product operands."""
    X, T, p = _bf16_exact_problem()
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p)
    # the construction really is bf16-exact at every rounding point
    z1 = X @ W1.T + b1
    a1 = np.maximum(z1, 0.0)
    out, c = mlp.forward(X, p, emulate=False)
    gq = 2.0 * (out - T) / X.shape[0]
    dz2 = gq[:, None] * w3[None, :] * (c["a2"] > 0)
    dz1 = (dz2 @ W2) * (a1 > 0)
    for v in (X, W1, W2, a1, dz2, dz1):
        np.testing.assert_array_equal(mlp.bf16(v), v)
    oe, _ = mlp.forward(X, p, emulate=True)
    np.testing.assert_array_equal(oe, out)
    Ge, Le = mlp.grad(X, T, p, emulate=True)
    Gx, Lx = mlp.grad(X, T, p, emulate=False)
    np.testing.assert_array_equal(Ge, Gx)
    assert Le == Lx


def test_emulated_rounding_points_hand_case():
    """One row, everything zero except one path through unit 0 of both hidden
    layers.  b1[0] = 1 + 2^-9 makes a1[0] non-representable in bfloat16
    (spacing 2^-7 at 1): the emulation feeds 1.0 to the second product.
    w3[0] = 1 + 2^-9 is not a product operand, so the output is
    a2[0] w3[0] = 1 + 2^-9.  With T = 0 and B = 1, g = 2 out = 2 + 2^-8;
    dZ2[0] = g w3[0] = 2 (1 + 2^-9)^2 = 2 + 2^-7 + 2^-17 rounds up to 2 + 2^-6
    before the products gW2 = dZ2^T a1 and dA1 = dZ2 W2; the bias gradients
    take the unrounded errors."""
    P = np.zeros(mlp.NPARAMS)
    e9 = 2.0 ** -9
    P[mlp.OB1 + 0] = 1.0 + e9
    P[mlp.OW2 + 0] = 1.0          # W2[0][0]
    P[mlp.OW3 + 0] = 1.0 + e9
    X = np.zeros((1, 32))
    X[0, 0] = 1.0
    T = np.zeros(1)
    out, _ = mlp.forward(X, P, emulate=True)
    assert out[0] == 1.0 + e9
    G, L = mlp.grad(X, T, P, emulate=True)
    assert L == (1.0 + e9) ** 2
    want = np.zeros(mlp.NPARAMS)
    dz2b = 2.0 + 2.0 ** -6
    want[mlp.OW2 + 0] = dz2b * 1.0              # gW2[0][0] = dZ2b * a1b
    want[mlp.OB2 + 0] = 2.0 * (1.0 + e9) ** 2   # gb2[0] = dZ2, unrounded
    want[mlp.OW3 + 0] = 1.0 * (2.0 + 2.0 ** -8)  # gw3[0] = a2[0] g
    want[mlp.OB3] = 2.0 + 2.0 ** -8
    want[mlp.OB1 + 0] = dz2b                    # dZ1[0] = dA1[0] = dZ2b W2b[0][0]
    # gW1[0][j] = dZ1b[0] X[j]: only X[0] = 1 is nonzero (gW1 row 0 is W1[0][:])
    want[mlp.OW1 + 0] = dz2b
    np.testing.assert_array_equal(G, want)
    # without the emulation every one of those values moves
    Gx, _ = mlp.grad(X, T, P, emulate=False)
    for i in (mlp.OW2, mlp.OB1, mlp.OW1, mlp.OW3, mlp.OB3):
        assert Gx[i] != G[i]
