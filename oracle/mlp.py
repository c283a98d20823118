"""Plain fp64 reference of the learned screener's network.

TEST INFRASTRUCTURE ONLY.  Imported by the test suite, ``__graft_entry__.smoke``
and the benchmark's CPU-baseline leg; the product package never imports it.

The screener is an extension of the method (the paper has no learned
component): a multilayer perceptron 8 -> 64 -> 64 -> 1 with ReLU hidden
layers and a sigmoid output, scoring the vertices a batch touches from the
eight features of ``dc_oracle.h``, trained with binary cross-entropy (a
positive-class weight) and Adam.

Parameters are one flat fp32 vector of 4801 entries:
    W1 [64][8] | b1 [64] | W2 [64][64] | b2 [64] | w3 [64] | b3 [1]
(row = output unit).  Compute follows the device recipe: every parameter and
every activation or back-propagated signal that feeds a matrix product is
rounded to bfloat16 (round to nearest even, through fp32), sums are exact here
(fp64) where the device accumulates in fp32.  ``mirror=False`` drops every
rounding and gives the exact fp64 network, which the finite-difference pins
use.
"""
from __future__ import annotations

import numpy as np

IN, HID = 8, 64
OFF_W1 = 0
OFF_B1 = OFF_W1 + HID * IN
OFF_W2 = OFF_B1 + HID
OFF_B2 = OFF_W2 + HID * HID
OFF_W3 = OFF_B2 + HID
OFF_B3 = OFF_W3 + HID
NPARAM = OFF_B3 + 1  # 4801

BF16_ULP = 2.0 ** -7   # bound on the relative gap between two adjacent bf16 values
FP32_ACC = 2.0 ** -16  # bound on the relative error of a <= 64-term fp32 sum


def bf16_bits(x) -> np.ndarray:
    """bfloat16 bit patterns of x: fp64 -> fp32 (nearest even), then the top
    16 bits with round to nearest even on the 16 dropped bits."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def from_bits(b) -> np.ndarray:
    """fp64 values of bfloat16 bit patterns."""
    u = (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16)
    return np.ascontiguousarray(u).view(np.float32).astype(np.float64)


def bf16(x) -> np.ndarray:
    return from_bits(bf16_bits(x))


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    return (w[OFF_W1:OFF_B1].reshape(HID, IN), w[OFF_B1:OFF_W2],
            w[OFF_W2:OFF_B2].reshape(HID, HID), w[OFF_B2:OFF_W3],
            w[OFF_W3:OFF_B3], w[OFF_B3])


def init_weights(seed: int) -> np.ndarray:
    """He-uniform hidden layers, small output layer, zero biases (fp32)."""
    rng = np.random.default_rng(np.random.SeedSequence((seed, 0x5C12)))
    w = np.zeros(NPARAM, np.float64)
    w[OFF_W1:OFF_B1] = rng.uniform(-1, 1, HID * IN) * np.sqrt(6.0 / IN)
    w[OFF_W2:OFF_B2] = rng.uniform(-1, 1, HID * HID) * np.sqrt(6.0 / HID)
    w[OFF_W3:OFF_B3] = rng.uniform(-1, 1, HID) * np.sqrt(1.0 / HID)
    return w.astype(np.float32)


def _round(x, mirror):
    return bf16(x) if mirror else x


def forward(w, X, mirror=True):
    """Logits z3 [n] of inputs X [n, 8] (fp64 values, bf16-representable when
    mirroring) and the intermediate values of the pass."""
    W1, b1, W2, b2, w3, b3 = (_round(p, mirror) for p in unpack(w))
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = _round(np.maximum(z1, 0.0), mirror)
    z2 = h1 @ W2.T + b2
    h2 = _round(np.maximum(z2, 0.0), mirror)
    z3 = h2 @ w3 + b3
    return z3, dict(W1=W1, b1=b1, W2=W2, b2=b2, w3=w3, b3=b3, X=X, z1=z1, h1=h1,
                    z2=z2, h2=h2)


def forward_bound(w, X):
    """Per-sample bound on |z3(device) - z3(this reference)|: each side rounds
    h1, h2 to bf16 (the two results differ by at most one bf16 step where the
    device's fp32 sum and this fp64 sum straddle a rounding boundary), and
    the device's fp32 sums add at most FP32_ACC of the absolute terms."""
    z3, c = forward(w, X, mirror=True)
    aW1, ab1, aW2, ab2 = np.abs(c["W1"]), np.abs(c["b1"]), np.abs(c["W2"]), np.abs(c["b2"])
    aw3, ab3 = np.abs(c["w3"]), abs(c["b3"])
    e1 = BF16_ULP * np.abs(c["h1"]) + FP32_ACC * (np.abs(c["X"]) @ aW1.T + ab1)
    e2 = BF16_ULP * np.abs(c["h2"]) + e1 @ aW2.T + FP32_ACC * (np.abs(c["h1"]) @ aW2.T + ab2)
    e3 = e2 @ aw3 + FP32_ACC * (np.abs(c["h2"]) @ aw3 + ab3)
    return e3


def softplus(x):
    return np.maximum(x, 0.0) + np.log1p(np.exp(-np.abs(x)))


def sigmoid(x):
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def loss_of(z3, y, pos_weight):
    """Mean binary cross-entropy with logits and a weight on the positives."""
    y = np.asarray(y, dtype=np.float64)
    return float(np.mean(pos_weight * y * softplus(-z3) + (1.0 - y) * softplus(z3)))


def loss_grad(w, X, y, pos_weight, mirror=True):
    """Loss and gradient (flat, NPARAM) of the mean weighted BCE.  With
    mirror=True also the per-entry bound on the device's deviation: the sum
    of the absolute contributions times 2^-5 (one bf16 step on each of the
    two operands of every term, compounded over the two back-propagated
    layers, plus fp32 accumulation)."""
    z3, c = forward(w, X, mirror)
    y = np.asarray(y, dtype=np.float64)
    n = len(y)
    p = sigmoid(z3)
    dz3 = ((pos_weight * y + 1.0 - y) * p - pos_weight * y) / max(n, 1)
    g = np.zeros(NPARAM, np.float64)
    bnd = np.zeros(NPARAM, np.float64)
    h2, h1, X = c["h2"], c["h1"], c["X"]
    g[OFF_W3:OFF_B3] = dz3 @ h2
    g[OFF_B3] = dz3.sum()
    dz2 = _round(np.outer(dz3, c["w3"]) * (c["z2"] > 0), mirror)
    g[OFF_W2:OFF_B2] = (dz2.T @ h1).ravel()
    g[OFF_B2:OFF_W3] = dz2.sum(axis=0)
    dh1 = dz2 @ c["W2"]
    dz1 = _round(dh1 * (c["z1"] > 0), mirror)
    g[OFF_W1:OFF_B1] = (dz1.T @ X).ravel()
    g[OFF_B1:OFF_W2] = dz1.sum(axis=0)
    if mirror:
        a3, a2, a1 = np.abs(dz3), np.abs(dz2), np.abs(dz1)
        bnd[OFF_W3:OFF_B3] = a3 @ np.abs(h2)
        bnd[OFF_B3] = a3.sum()
        bnd[OFF_W2:OFF_B2] = (a2.T @ np.abs(h1)).ravel()
        bnd[OFF_B2:OFF_W3] = a2.sum(axis=0)
        bnd[OFF_W1:OFF_B1] = (a1.T @ np.abs(X)).ravel()
        bnd[OFF_B1:OFF_W2] = a1.sum(axis=0)
        bnd *= 2.0 ** -5
    return loss_of(z3, y, pos_weight), g, bnd


def adam(w, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba 2015) at step number t >= 1; returns new
    (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def recall_threshold(z, y, recall):
    """Largest logit threshold theta such that {z >= theta} keeps at least the
    given fraction of the positives (all vertices when there are none)."""
    pos = np.sort(np.asarray(z, dtype=np.float64)[np.asarray(y) != 0])
    if len(pos) == 0:
        return -np.inf
    drop = int(np.floor((1.0 - recall) * len(pos) + 1e-9))
    return float(pos[drop])
