"""Pins of the screener network's fp64 reference (oracle/mlp.py).

Each is fixed by something other than the reference itself: torch's CPU
bfloat16 conversion (round to nearest even), torch's
binary_cross_entropy_with_logits and Adam in float64, closed forms of
special weights, and central finite differences of the exact network."""
import numpy as np
import pytest
import torch

from oracle import mlp as M


def rand_X(n, seed):
    rng = np.random.default_rng(seed)
    X = np.column_stack([rng.uniform(0, 1, n), rng.uniform(-1, 1, n), rng.uniform(0, 1, n),
                         rng.uniform(0, 1, n), rng.uniform(-2, 1, n), rng.uniform(-2, 1, n),
                         rng.integers(0, 2, n), rng.uniform(0, 0.2, n)])
    return M.bf16(X)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000),
                        [1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 1 + 2 ** -9,
                         1 - 2 ** -9, 0.0, -0.0, 3.0, 65504.0, 1e-30]])
    want = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).view(torch.int16)
    got = M.bf16_bits(x).astype(np.int16)
    assert np.array_equal(got, want.numpy())
    # ties go to even
    assert M.bf16(1 + 2 ** -8)[()] == 1.0 and M.bf16(1 + 3 * 2 ** -8)[()] == 1 + 2 ** -6


def test_zero_weights_closed_form():
    X = rand_X(50, 2)
    y = (np.arange(50) % 3 == 0).astype(np.uint8)
    w = np.zeros(M.NPARAM)
    w[M.OFF_B3] = 0.75
    z, _ = M.forward(w, X)
    assert np.all(z == 0.75)
    loss, g, _ = M.loss_grad(w, X, y, pos_weight=2.0)
    p = 1 / (1 + np.exp(-0.75))
    ym = y.mean()
    assert loss == pytest.approx(-(2 * ym * np.log(p) + (1 - ym) * np.log(1 - p)), rel=1e-12)
    assert g[M.OFF_B3] == pytest.approx(np.mean((2 * y + 1 - y) * p - 2 * y), rel=1e-12)
    assert np.all(g[:M.OFF_B3] == 0)


def test_relu_network_closed_form():
    """W1 copies feature j to unit j (and -x_j to unit 8+j), W2 passes units
    through, w3 = +1/-1: the logit is sum_j |x_j| = sum relu(x) + relu(-x)."""
    w = np.zeros(M.NPARAM)
    W1, W2, w3 = np.zeros((64, 8)), np.zeros((64, 64)), np.zeros(64)
    for j in range(8):
        W1[j, j], W1[8 + j, j] = 1.0, -1.0
        W2[j, j], W2[8 + j, 8 + j] = 1.0, 1.0
        w3[j] = w3[8 + j] = 1.0
    w[M.OFF_W1:M.OFF_B1] = W1.ravel()
    w[M.OFF_W2:M.OFF_B2] = W2.ravel()
    w[M.OFF_W3:M.OFF_B3] = w3
    X = rand_X(40, 3)
    z, _ = M.forward(w, X, mirror=False)
    assert np.allclose(z, np.abs(X).sum(axis=1), rtol=0, atol=1e-15)


def test_loss_matches_torch():
    X = rand_X(300, 4)
    w = M.init_weights(5).astype(np.float64)
    y = (np.random.default_rng(6).uniform(size=300) < 0.2).astype(np.uint8)
    z, _ = M.forward(w, X, mirror=False)
    want = torch.nn.functional.binary_cross_entropy_with_logits(
        torch.from_numpy(z), torch.from_numpy(y.astype(np.float64)),
        pos_weight=torch.tensor(3.5, dtype=torch.float64)).item()
    assert M.loss_of(z, y, 3.5) == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_finite_differences(seed):
    X = rand_X(64, 10 + seed)
    y = (np.random.default_rng(seed).uniform(size=64) < 0.3).astype(np.uint8)
    w = M.init_weights(seed).astype(np.float64)
    w[M.OFF_B1:M.OFF_W2] = 0.05  # keep most units away from the ReLU kink
    w[M.OFF_B2:M.OFF_W3] = 0.05
    loss, g, _ = M.loss_grad(w, X, y, 2.0, mirror=False)
    rng = np.random.default_rng(100 + seed)
    idx = np.concatenate([rng.choice(M.NPARAM, 120, replace=False),
                          [M.OFF_B3, M.OFF_W3, M.OFF_B2, M.OFF_B1, 0]])
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        zp, _ = M.forward(wp, X, mirror=False)
        zm, _ = M.forward(wm, X, mirror=False)
        fd = (M.loss_of(zp, y, 2.0) - M.loss_of(zm, y, 2.0)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(g[i]), (i, fd, g[i])


def test_mirrored_gradient_close_to_exact():
    X = rand_X(256, 20)
    y = (np.random.default_rng(21).uniform(size=256) < 0.3).astype(np.uint8)
    w = M.init_weights(22)
    _, ge, _ = M.loss_grad(w, X, y, 2.0, mirror=False)
    _, gm, bnd = M.loss_grad(w, X, y, 2.0, mirror=True)
    assert np.linalg.norm(gm - ge) <= 0.05 * np.linalg.norm(ge)
    assert np.all(bnd >= 0)


def test_adam_matches_torch():
    rng = np.random.default_rng(30)
    w0 = rng.standard_normal(M.NPARAM)
    grads = [rng.standard_normal(M.NPARAM) * 10.0 ** -s for s in range(5)]
    p = torch.nn.Parameter(torch.from_numpy(w0.copy()))
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    w, m, v = w0.copy(), np.zeros(M.NPARAM), np.zeros(M.NPARAM)
    for t, g in enumerate(grads, 1):
        p.grad = torch.from_numpy(g.copy())
        opt.step()
        w, m, v = M.adam(w, m, v, g, t, 1e-3)
    assert np.allclose(w, p.detach().numpy(), rtol=0, atol=1e-14)


def test_recall_threshold():
    z = np.array([5.0, 1.0, 3.0, -2.0, 0.5, 4.0])
    y = np.array([1, 1, 1, 0, 1, 0])
    assert M.recall_threshold(z, y, 1.0) == 0.5
    assert M.recall_threshold(z, y, 0.75) == 1.0
    assert M.recall_threshold(z, np.zeros(6), 0.99) == -np.inf
