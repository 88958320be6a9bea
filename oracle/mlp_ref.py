"""CPU reference of the cost model's network (test infrastructure only).

Plain fp64 numpy forward pass and hand-written backward pass of the
16-64-64-1 ReLU network with mean-squared-error loss, using the same
parameter layout as the library (W1[64][16], b1[64], W2[64][64], b2[64],
w3[64], b3) and the same bf16 rounding of weights (round to nearest even).
Pinned by central finite differences in the tests.
"""
import numpy as np

IN, H = 16, 64
NPARAM = H * IN + H + H * H + H + H + 1


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even)."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    special = (u & 0x7F800000) == 0x7F800000
    r = np.where(special, u.astype(np.uint32), r)
    return r.view(np.float32).reshape(a.shape)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * IN].reshape(H, IN); o += H * IN
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def standardise(X, stats):
    stats = np.asarray(stats, dtype=np.float64)
    return (np.asarray(X, dtype=np.float64) - stats[:IN]) / stats[IN:2 * IN]


def forward(p, stats, X):
    W1, b1, W2, b2, w3, b3 = unpack(p)
    x = standardise(X, stats)
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    return y, (x, z1, h1, z2, h2)


def loss(p, stats, X, Y):
    y, _ = forward(p, stats, X)
    return float(np.mean((y - np.asarray(Y, dtype=np.float64)) ** 2))


def gradient(p, stats, X, Y):
    """d loss / d p by the chain rule, layer by layer."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    y, (x, z1, h1, z2, h2) = forward(p, stats, X)
    n = len(y)
    dy = 2.0 * (y - np.asarray(Y, dtype=np.float64)) / n          # d loss / d y
    g_w3 = h2.T @ dy
    g_b3 = dy.sum()
    dz2 = np.outer(dy, w3) * (z2 > 0)
    g_W2 = dz2.T @ h1
    g_b2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    g_W1 = dz1.T @ x
    g_b1 = dz1.sum(0)
    return np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, [g_b3]])
