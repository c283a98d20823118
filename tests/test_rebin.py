"""Host logic of the temporal-resolution study: one event stream cut into
different numbers of time steps.  Every cut, applied batch by batch, must
reproduce the graph that replaying the events one at a time gives at each
bin boundary; insertions must be absent before their bin and deletions
present; bins of s steps nest in those of 2s steps."""
import numpy as np
import pytest

from paper_1904_08553_amd import workloads as W


@pytest.fixture(scope="module")
def stream():
    return W.temporal_events(n=3000, events=24000, slices=12, blocks=30, dmax=300, seed=3)


def _replay(stream, bounds):
    alive = set()
    states = []
    e = 0
    for b in bounds[1:]:
        while e < b:
            p = (int(min(stream.u[e], stream.v[e])), int(max(stream.u[e], stream.v[e])))
            if stream.op[e] > 0:
                assert p not in alive
                alive.add(p)
            else:
                assert p in alive
                alive.remove(p)
            e += 1
        states.append(set(alive))
    return states


def test_stream_shape(stream):
    assert len(stream) == 24000
    assert (stream.op[:2000] == 1).all()             # slice 1 builds G_1
    assert 0.1 < (stream.op == -1).mean() < 0.2      # later slices: 15% deletions
    assert (stream.u != stream.v).all()


@pytest.mark.parametrize("steps", [1, 2, 3, 4, 8, 12, 16, 28])
def test_rebin_matches_event_replay(stream, steps):
    bounds = W.bin_bounds(len(stream), steps)
    states = _replay(stream, bounds)
    (u, v, w), it = W.rebin(stream, steps)
    cur = {(int(a), int(b)) for a, b in zip(u, v)}
    assert (u < v).all() and (w == 1).all()
    assert cur == states[0]
    for j, b in enumerate(it, start=1):
        ins = {(int(a), int(c)) for a, c in zip(b.add_u, b.add_v)}
        dele = {(int(a), int(c)) for a, c in zip(b.del_u, b.del_v)}
        assert not (ins & cur), f"bin {j}: insertion of a present pair"
        assert dele <= cur, f"bin {j}: deletion of an absent pair"
        assert len(ins) == len(b.add_u) and len(dele) == len(b.del_u)
        cur = (cur - dele) | ins
        assert cur == states[j], f"bin {j}"


def test_bins_nest():
    for s in (2, 4, 6, 8, 12, 14):
        coarse = W.bin_bounds(63_000_000, s)
        fine = W.bin_bounds(63_000_000, 2 * s)
        assert coarse == fine[::2]
