"""dc_mlp_grad_noalloc (the screener gradient with its scratch in the
library's fixed device array, for callers that cannot allocate) against
dc_mlp_grad (allocated scratch), through the C ABI: two calls in a row, the
second on fewer samples, so the second reads a scratch array that still
holds the first call's partial sums.  Both run the same kernels in the same
order, so the gradient and the loss must be equal bit for bit; both are also
checked against the oracle's fp64 gradient within the bound the oracle
derives from the bf16 / fp32 arithmetic."""
import numpy as np
import pytest
import torch

from oracle import mlp as M
from paper_1904_08553_amd import dc

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    X = np.column_stack([rng.uniform(0, 1, n), rng.uniform(-1, 1, n), rng.uniform(0, 1, n),
                         rng.uniform(0, 1, n), rng.uniform(-2, 1, n), rng.uniform(-2, 1, n),
                         rng.integers(0, 2, n), rng.uniform(0, 0.2, n)])
    bits = M.bf16_bits(X).reshape(n, 8)
    y = (rng.uniform(size=n) < 0.3).astype(np.uint8)
    return bits, y


def test_grad_noalloc_equals_grad_two_calls():
    w = M.init_weights(31)
    w[M.OFF_B1:M.OFF_W2] = 0.05
    net = dc.MLP(w)
    for n, seed in ((50_021, 1), (1_003, 2)):  # the second call is smaller
        _log(f"case: dc_mlp_grad_noalloc n={n}")
        bits, y = _inputs(n, seed)
        Xd = torch.from_numpy(bits.astype(np.uint16).view(np.int16)).cuda().contiguous()
        yd = torch.from_numpy(y).cuda().contiguous()
        loss_a, g_a = net.grad(Xd, yd, 2.5)
        loss_b, g_b = net.grad_noalloc(Xd, yd, 2.5)
        assert loss_a == loss_b
        assert np.array_equal(g_a.view(np.uint32), g_b.view(np.uint32))
        lo, go, bnd = M.loss_grad(w, M.from_bits(bits), y, 2.5)
        assert loss_b == pytest.approx(lo, rel=1e-4, abs=1e-6)
        dev = np.abs(g_b.astype(np.float64) - go)
        assert np.all(dev <= bnd + 1e-7 * np.max(np.abs(go)))
    net.close()
