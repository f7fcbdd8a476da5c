"""FP64 references for the learned initial guess (network and POD).

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module; it never imports the GPU
package.

Network: 10 -> 256 -> 256 -> 32 with GELU(z) = z/2 (1 + erf(z / sqrt 2))
after the hidden layers; loss = mean over batch and outputs of (y - t)^2.
Parameter vector layout: W1 [256][10], b1 [256], W2 [256][256], b2 [256],
W3 [32][256], b3 [32].

`forward_backward(..., bf16=True)` evaluates in FP64 but rounds to BF16
(round to nearest even) exactly where the GPU path feeds BF16 operands to
its matrix products: inputs, weights, the two hidden activations, and the
back-propagated dY, dZ2, dZ1.  With bf16=False it is the plain FP64
network (used for finite-difference pins).

`adam_step` is one step of Adam (Kingma and Ba, "Adam: a method for
stochastic optimization", ICLR 2015, Algorithm 1) in FP64.

POD by the method of snapshots: G = S^T S, eigenpairs of G (numpy eigh, a
library routine), Phi = S V diag(lambda)^(-1/2), largest-magnitude entry of
each column positive.
"""
from __future__ import annotations

import math

import numpy as np

IN, HID, OUT = 10, 256, 32
SIZES = [("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (OUT, HID)), ("b3", (OUT,))]
P = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    out, off = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = np.asarray(p[off:off + k], dtype=np.float64).reshape(shape)
        off += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SIZES])


def bf16(a):
    """Round to the nearest BF16 value (ties to even), via FP32."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


_erf = np.vectorize(math.erf)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward_backward(p, X, T=None, bf16_points=True):
    """Returns (Y, loss, grad) -- loss and grad only when targets T given."""
    w = unpack(p)
    r = bf16 if bf16_points else (lambda a: np.asarray(a, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    Xb, W1, W2, W3 = r(X), r(w["W1"]), r(w["W2"]), r(w["W3"])
    Z1 = Xb @ W1.T + w["b1"]
    H1 = r(gelu(Z1))
    Z2 = H1 @ W2.T + w["b2"]
    H2 = r(gelu(Z2))
    Y = H2 @ W3.T + w["b3"]
    if T is None:
        return Y, None, None
    B = X.shape[0]
    D = Y - np.asarray(T, dtype=np.float64)
    loss = float(np.mean(D * D))
    dY = 2.0 * D / (B * OUT)
    dYb = r(dY)
    g = {"W3": dYb.T @ H2, "b3": dY.sum(0)}
    dZ2 = (dYb @ W3) * gelu_grad(Z2)
    dZ2b = r(dZ2)
    g["W2"] = dZ2b.T @ H1
    g["b2"] = dZ2.sum(0)
    dZ1 = (dZ2b @ W2) * gelu_grad(Z1)
    dZ1b = r(dZ1)
    g["W1"] = dZ1b.T @ Xb
    g["b1"] = dZ1.sum(0)
    return Y, loss, pack(g)


def loss_fp64(p, X, T):
    Y, _, _ = forward_backward(p, X, None, bf16_points=False)
    D = Y - T
    return float(np.mean(D * D))


def init_params(seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in SIZES:
        fan_in = {"W1": IN, "b1": IN, "W2": HID, "b2": HID, "W3": HID, "b3": HID}[name]
        b = 1.0 / math.sqrt(fan_in)
        d[name] = rng.uniform(-b, b, size=shape)
    return pack(d)


# ------------------------------------------------------------------ Adam


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Step t (1-based) of Adam on parameters p with gradient g and moments
    m, v (all FP64); returns the new (p, m, v).  The moments are exponential
    moving averages of g and g^2, divided by 1 - b^t to remove their bias
    towards the zero start; the step is lr * mhat / (sqrt(vhat) + eps)."""
    p, g, m, v = (np.asarray(a, dtype=np.float64) for a in (p, g, m, v))
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ------------------------------------------------------------------ POD


def pod(S, r):
    """(Phi [n][r], lambda [r] descending, G) of the snapshot matrix S [n][m]."""
    S = np.asarray(S, dtype=np.float64)
    G = S.T @ S
    lam, V = np.linalg.eigh(G)
    order = np.argsort(lam)[::-1][:r]
    lam = lam[order]
    V = V[:, order]
    Phi = (S @ V) / np.sqrt(lam)
    for j in range(r):
        i = int(np.argmax(np.abs(Phi[:, j])))
        if Phi[i, j] < 0:
            Phi[:, j] = -Phi[:, j]
    return Phi, lam, G
