"""GPU parity of the smart local moving levels (dSLM-DS and dSLM-base: the
paper's second host method, Sec. 3.4) against the CPU oracle, through the C
ABI: C_t bit for bit, R_t, every sweep of every level including the
refinement sweeps (phase 1) with their exact Delta N, N and 2m."""
import numpy as np
import pytest

from gpu_common import compare, make_pair, step_pair
from paper_1904_08553_amd import workloads as W

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("mode", ["delta", "all", "static"])
@pytest.mark.parametrize("seed", range(6))
def test_slm_small_random(mode, seed):
    n = 10 + seed % 6
    _log(f"case: slm random n={n} seed={seed} mode={mode}")
    (u, v, w), batches = W.random_dynamic(n, 2 * n + 3, 3, 4, 2, seed=2000 + seed)
    o, g = make_pair(n, u, v, w, mode=mode, slm=True)
    compare(o, g, "init")
    for t, b in enumerate(batches):
        step_pair(o, g, b)
        compare(o, g, f"step {t}")
    g.close()


@pytest.mark.parametrize("opts", [dict(max_levels=1), dict(guard=0), dict(max_levels=2),
                                  dict(del_rule=1)])
def test_slm_options(opts):
    _log(f"case: slm options {opts}")
    (u, v, w), batches = W.random_dynamic(60, 180, 3, 12, 6, seed=41)
    o, g = make_pair(60, u, v, w, slm=True, **opts)
    compare(o, g, "init")
    for t, b in enumerate(batches):
        step_pair(o, g, b)
        compare(o, g, f"step {t}")
    g.close()


def test_slm_planted_partition():
    pp = W.PlantedPartition(n=2000, blocks=20, p_in=0.05, p_out=0.001, seed=0)
    _log("case: slm planted partition 2000")
    (u, v, w), batches = pp.batches(steps=4, n_ins=500, n_del=200)
    o, g = make_pair(pp.n, u, v, w, slm=True)
    compare(o, g, "init")
    for t, b in enumerate(batches):
        step_pair(o, g, b)
        compare(o, g, f"step {t}")
    g.close()


@pytest.mark.parametrize("mode", ["delta", "all"])
def test_slm_dcsbm_hub_rows(mode):
    """20K vertices with rows of thousands of entries (every evaluation bin,
    the hub-row bin included, in local moving and in refinement)."""
    _log(f"case: slm dcsbm 20K mode={mode}")
    gen = W.DCSBM(n=20000, m=200000, blocks=40, dmax=20000, seed=4)
    (u, v, w), it = gen.stream(3, frac=0.02)
    o, g = make_pair(gen.n, u, v, w, mode=mode, slm=True)
    compare(o, g, "init")
    for t, b in enumerate(it):
        step_pair(o, g, b)
        compare(o, g, f"step {t}")
    g.close()
