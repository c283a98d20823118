"""GPU parity of the cascade-aware screening (an extension of Alg. 2 for the
indirect effect noted after the proof of Lemma 3.2): R_t, labels, sweep
traces, exact modularity and the cascade counters equal the oracle's, step
by step, on planted partitions and on a power-law graph with hubs."""
import numpy as np
import pytest

from gpu_common import compare, make_pair, step_pair
from paper_1904_08553_amd import workloads as W

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def _check_counts(o, g, where):
    st = g.last_stats()
    assert (st.cascade_candidates, st.cascade_expanded) == \
        (o.info.cascade_candidates, o.info.cascade_expanded), where
    assert st.ds_accepted == o.info.ds_accepted, where


@pytest.mark.parametrize("theta", [(1, 20), (1, 4)])
def test_cascade_planted_partition(theta):
    _log(f"case: cascade planted partition theta={theta}")
    pp = W.PlantedPartition()
    (u, v, w), batches = pp.batches()
    o, g = make_pair(pp.n, u, v, w, cascade=theta)
    total = 0
    for t, b in enumerate(batches):
        step_pair(o, g, b)
        compare(o, g, f"step {t}")
        _check_counts(o, g, f"step {t}")
        total += o.info.cascade_expanded
    assert total > 0


def test_cascade_screener_graph():
    _log("case: cascade screener-style graph")
    n, (u, v, w), batches = W.screener_graph(3, n=20000)
    o, g = make_pair(n, u, v, w, cascade=(1, 20))
    for t, b in enumerate(batches):
        step_pair(o, g, b)
        compare(o, g, f"step {t}")
        _check_counts(o, g, f"step {t}")
    assert o.info.cascade_candidates > 0


def test_cascade_with_hubs():
    _log("case: cascade dcsbm hubs")
    gen = W.DCSBM(n=20000, m=200000, blocks=40, dmax=20000, seed=7)
    (u, v, w), it = gen.stream(3, frac=0.01)
    o, g = make_pair(gen.n, u, v, w, cascade=(1, 10))
    for t, b in enumerate(it):
        step_pair(o, g, b)
        compare(o, g, f"step {t}")
        _check_counts(o, g, f"step {t}")


def test_cascade_with_conservative_deletion_rule():
    """The conservative deletion rule keeps separate screening passes; the
    cascade runs on the accepted insertion sources there too."""
    _log("case: cascade + conservative deletions")
    pp = W.PlantedPartition()
    (u, v, w), batches = pp.batches()
    o, g = make_pair(pp.n, u, v, w, cascade=(1, 4), del_rule=1)
    for t, b in enumerate(batches):
        step_pair(o, g, b)
        compare(o, g, f"step {t}")
        _check_counts(o, g, f"step {t}")
