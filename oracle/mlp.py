"""Float64 reference of the bandwidth network (test infrastructure only).

32 -> 128 -> 128 -> 1 with ReLU, parameters in one vector laid out as
W1[128][32], b1[128], W2[128][128], b2[128], w3[128], b3 (the layout of the
C ABI).  ``emulate=True`` rounds the operands of the three matrix products
(inputs, W1, first activations, W2, and in the backward pass the two
propagated errors) to bfloat16 with round-to-nearest-even, exactly where the
GPU kernels feed their matrix cores; everything else is float64.  The
gradient is the analytic backward pass of the mean squared error, written
from the chain rule; tests pin it with central finite differences.
"""
import numpy as np

IN, H = 32, 128
OW1 = 0
OB1 = OW1 + H * IN
OW2 = OB1 + H
OB2 = OW2 + H * H
OW3 = OB2 + H
OB3 = OW3 + H
NPARAMS = OB3 + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return (p[OW1:OB1].reshape(H, IN), p[OB1:OW2], p[OW2:OB2].reshape(H, H),
            p[OB2:OW3], p[OW3:OB3], p[OB3])


def bf16(a):
    """Round to bfloat16 (nearest, ties to even) through float32."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(X, p, emulate=True):
    W1, b1, W2, b2, w3, b3 = unpack(p)
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    Xb, W1b, W2b = r(X), r(W1), r(W2)
    z1 = Xb @ W1b.T + b1
    a1 = np.maximum(z1, 0.0)
    a1b = r(a1)
    z2 = a1b @ W2b.T + b2
    a2 = np.maximum(z2, 0.0)
    out = a2 @ w3 + b3
    return out, dict(Xb=Xb, W1b=W1b, W2b=W2b, a1=a1, a1b=a1b, a2=a2)


def loss(X, T, p, emulate=False):
    out, _ = forward(X, p, emulate)
    return float(np.mean((out - np.asarray(T, dtype=np.float64)) ** 2))


def grad(X, T, p, emulate=True):
    """Gradient of (1/B) sum (out - T)^2 in the parameter layout, and the loss."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    out, c = forward(X, p, emulate)
    T = np.asarray(T, dtype=np.float64)
    B = out.shape[0]
    g = 2.0 * (out - T) / B
    gw3 = c["a2"].T @ g
    gb3 = g.sum()
    dZ2 = g[:, None] * w3[None, :] * (c["a2"] > 0)
    dZ2b = r(dZ2)
    dA1 = dZ2b @ c["W2b"]
    dZ1 = dA1 * (c["a1"] > 0)
    dZ1b = r(dZ1)
    gW2 = dZ2b.T @ c["a1b"]
    gb2 = dZ2.sum(0)
    gW1 = dZ1b.T @ c["Xb"]
    gb1 = dZ1.sum(0)
    G = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gw3, [gb3]])
    return G, float(np.mean((out - T) ** 2))
