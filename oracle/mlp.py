"""Plain NumPy reference of the surrogate MLP -- TEST INFRASTRUCTURE.

The surrogate maps the 4 n_s pulse coefficients to the standardised log10 of the pair yield:
n_in -> depth x (width, GELU) -> 1.  Only the test-suite imports this module.

Arithmetic is float64.  With bf16=True the values the GPU rounds to bfloat16 are rounded here too
(round to nearest even, through float32): the network input, every weight matrix used as a
matrix operand, every hidden activation, and every back-propagated pre-activation gradient used
as a matrix operand.  Biases, pre-activations, gradients of weights and the optimiser state stay
unrounded.  With bf16=False the network is plain float64 (used to pin this code against
automatic differentiation and finite differences).

Parameter vector layout (float): for each hidden layer l: W_l [k_in][width] (row k, column n),
b_l [width]; then the output w [width], b [1].
GELU is the erf form, gelu(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2.
Adam: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2, p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)


def bf16(x):
    """Round to bfloat16 (nearest even) through float32; returns float64 values."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def shapes(n_in, width, depth):
    out, k = [], n_in
    for _ in range(depth):
        out.append(((k, width), (width,)))
        k = width
    out.append(((width,), (1,)))
    return out


def unpack(params, n_in, width, depth):
    p = np.asarray(params, dtype=np.float64)
    Ws, bs, o = [], [], 0
    for wshape, bshape in shapes(n_in, width, depth):
        nw, nb = int(np.prod(wshape)), int(np.prod(bshape))
        Ws.append(p[o:o + nw].reshape(wshape))
        o += nw
        bs.append(p[o:o + nb].reshape(bshape))
        o += nb
    assert o == p.size
    return Ws, bs


def pack(Ws, bs):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in zip(Ws, bs)])


def forward(params, x, n_in, width, depth, bf=True):
    """Returns (y [B], cache)."""
    r = bf16 if bf else (lambda v: np.asarray(v, dtype=np.float64))
    Ws, bs = unpack(params, n_in, width, depth)
    h = r(x)
    hs, zs = [h], []
    for l in range(depth):
        z = h @ r(Ws[l]) + bs[l]
        h = r(gelu(z))
        zs.append(z)
        hs.append(h)
    y = h @ r(Ws[depth]) + bs[depth][0]
    return y, (hs, zs)


def loss_grad(params, x, t, n_in, width, depth, bf=True):
    """Mean squared error and its gradient with respect to the parameter vector."""
    r = bf16 if bf else (lambda v: np.asarray(v, dtype=np.float64))
    Ws, bs = unpack(params, n_in, width, depth)
    y, (hs, zs) = forward(params, x, n_in, width, depth, bf)
    B = y.shape[0]
    d = y - t
    loss = float(np.mean(d * d))
    dy = 2.0 * d / B
    gW, gb = [None] * (depth + 1), [None] * (depth + 1)
    gW[depth] = hs[depth].T @ dy
    gb[depth] = np.array([dy.sum()])
    dh = np.outer(dy, r(Ws[depth]))
    for l in range(depth - 1, -1, -1):
        dz = dh * gelu_grad(zs[l])
        gb[l] = dz.sum(axis=0)
        dzr = r(dz)
        gW[l] = hs[l].T @ dzr
        if l > 0:
            dh = dzr @ r(Ws[l]).T
    return loss, pack(gW, gb)


def adam(params, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (params, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
