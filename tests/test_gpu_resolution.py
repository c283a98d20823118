"""The temporal-resolution study on the GPU: cuts of one event stream into
2 and 8 steps run bit-exact with the oracle (labels, R_t, sweep trace, exact
modularity); cuts of 4 and 8 steps reach the same graph at their common
boundaries; the driver reports sane averages and times."""
import numpy as np
import pytest

from gpu_common import compare, make_pair
from paper_1904_08553_amd import dc
from paper_1904_08553_amd import resolution as RS
from paper_1904_08553_amd import workloads as W

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def stream():
    return W.temporal_events(n=31_250, events=246_000, slices=12, blocks=31, dmax=31_250 // 8,
                             seed=5)


@pytest.mark.parametrize("steps", [2, 8])
def test_cut_matches_oracle(stream, steps):
    _log(f"case: resolution cut steps={steps}")
    (u, v, w), it = W.rebin(stream, steps)
    o, g = make_pair(stream.n, u, v, w)
    compare(o, g, "init")
    for j, b in enumerate(it, start=2):
        o.apply_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)
        g.apply_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)
        compare(o, g, f"step {j} of {steps}")


def test_nested_cuts_reach_the_same_graphs(stream):
    _log("case: nested cuts 4 / 8")
    graphs = {}
    for steps in (4, 8):
        (u, v, w), it = W.rebin(stream, steps)
        g = dc.DynamicCommunities(stream.n, u, v, w)
        states = [g.csr()]
        for b in it:
            g.apply_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)
            states.append(g.csr())
        graphs[steps] = states
        g.close()
    for j in range(4):
        a, b = graphs[4][j], graphs[8][2 * j + 1]
        assert all(np.array_equal(x, y) for x, y in zip(a, b)), f"boundary {j + 1} of 4"


def test_study_driver(stream):
    _log("case: resolution driver")
    rows = RS.study(stream, (2, 4))
    assert [r["steps"] for r in rows] == [2, 4]
    for r in rows:
        assert 0.0 < r["avg_q_delta"] < 1.0 and 0.0 < r["avg_q_all"] < 1.0
        assert abs(r["avg_q_delta"] - r["avg_q_all"]) < 0.02
        assert r["total_s_delta"] > 0 and r["total_s_all"] > 0
        assert r["batch_changes"] > 0
