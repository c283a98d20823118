"""GPU tests of checkpoint/resume and of the serving loop (through
include/dc.h): every graph's results in the server's mix (merged level-0
sweeps, eviction to host memory under a small budget) equal those of the
graph's own context run alone, and the single-graph path equals the CPU
oracle."""
import numpy as np
import pytest

from gpu_common import compare, make_pair
from oracle import oracle as O
from paper_1904_08553_amd import dc
from paper_1904_08553_amd import workloads as W

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def _streams(sizes, steps, seed0=900):
    out = []
    for j, n in enumerate(sizes):
        gen = W.DCSBM(n=n, m=10 * n, blocks=max(10, n // 500), dmax=max(64, n // 4),
                      seed=seed0 + j)
        (u, v, w), it = gen.stream(steps, frac=0.02)
        out.append((n, (u, v, w), list(it)))
    return out


def _alone(streams):
    res = []
    for n, (u, v, w), batches in streams:
        g = dc.DynamicCommunities(n, u, v, w)
        cs = []
        for b in batches:
            cs.append(g.apply_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v).copy())
        res.append(cs)
        g.close()
    return res


def _mix(streams, budget, max_inflight, order_seed):
    srv = dc.Server(budget_bytes=budget, max_inflight=max_inflight)
    gids = [srv.add_graph(n, u, v, w) for n, (u, v, w), _ in streams]
    # interleave the graphs' batches in a shuffled order that keeps each
    # graph's own order
    rng = np.random.default_rng(order_seed)
    cursor = [0] * len(streams)
    tickets = []
    while any(c < len(s[2]) for c, s in zip(cursor, streams)):
        j = int(rng.choice([i for i, s in enumerate(streams) if cursor[i] < len(s[2])]))
        b = streams[j][2][cursor[j]]
        tickets.append((j, cursor[j], srv.submit(gids[j], b.add_u, b.add_v, b.add_w, b.del_u,
                                                 b.del_v)))
        cursor[j] += 1
    out = [[None] * len(s[2]) for s in streams]
    for j, t, tk in tickets:
        C, st, times = srv.poll(tk, gids[j])
        assert times[0] <= times[1] <= times[2]
        out[j][t] = C
    stats = srv.stats()
    srv.close()
    return out, stats


def test_checkpoint_resume_matches_oracle(tmp_path):
    _log("case: checkpoint and resume")
    gen = W.DCSBM(n=20000, m=200000, blocks=40, dmax=20000, seed=4)
    (u, v, w), it = gen.stream(3, frac=0.01)
    batches = list(it)
    o, g = make_pair(gen.n, u, v, w)
    b = batches[0]
    o.apply_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)
    g.apply_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)
    off, col, wt, C = g.export_state()
    oo, oc, ow = o.csr()
    assert np.array_equal(off, oo) and np.array_equal(col, oc) and np.array_equal(wt, ow)
    assert np.array_equal(C, o.C)
    # through a checkpoint file
    dc.save_checkpoint(g, tmp_path / "g.npz")
    r = dc.load_checkpoint(tmp_path / "g.npz")
    assert r.modularity() == g.modularity()
    for t, b in enumerate(batches[1:]):
        o.apply_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)
        r.apply_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)
        compare(o, r, f"resumed step {t}")


def test_server_mix_equals_alone():
    sizes = [3000, 12000, 5000, 20000, 8000, 4000]
    _log(f"case: server mix sizes={sizes}")
    streams = _streams(sizes, 3)
    alone = _alone(streams)
    mix, stats = _mix(streams, 0, 4, order_seed=1)
    _log(f"  stats {stats}")
    for j in range(len(streams)):
        for t in range(3):
            assert np.array_equal(mix[j][t], alone[j][t]), f"graph {j} batch {t}"
    assert stats["batches"] == 18 and stats["merged_rounds"] > 0
    assert stats["evictions"] == 0


def test_server_small_budget_evicts_and_matches():
    sizes = [6000, 15000, 9000, 12000]
    _log(f"case: server small budget sizes={sizes}")
    streams = _streams(sizes, 3, seed0=950)
    alone = _alone(streams)
    _, full = _mix(streams, 0, 4, order_seed=2)
    budget = int(0.55 * full["peak_resident_bytes"])
    mix, stats = _mix(streams, budget, 4, order_seed=3)
    _log(f"  budget {budget} stats {stats}")
    for j in range(len(streams)):
        for t in range(3):
            assert np.array_equal(mix[j][t], alone[j][t]), f"graph {j} batch {t}"
    assert stats["evictions"] > 0 and stats["restores"] > 0


def _oracle_labels(streams):
    """Every graph's C_t after each batch, from the CPU oracle alone."""
    res = []
    for n, (u, v, w), batches in streams:
        o = O.Oracle(n, u, v, w)
        cs = []
        for b in batches:
            o.apply_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)
            cs.append(o.C.copy())
        o.close()
        res.append(cs)
    return res


@pytest.mark.parametrize("budget_frac", [0.0, 0.5])
def test_server_matches_oracle(budget_frac):
    """Every graph of a merged mix (several graphs' level-0 sweeps in one
    launch per bin, and with a small budget also evicted and restored)
    equals the oracle batch by batch."""
    sizes = [2500, 6000, 4000, 9000, 3000]
    _log(f"case: server vs oracle, every graph, budget fraction {budget_frac}")
    streams = _streams(sizes, 3, seed0=970)
    budget = 0
    if budget_frac > 0:
        _, full = _mix(streams, 0, 5, order_seed=5)
        budget = int(budget_frac * full["peak_resident_bytes"])
    mix, stats = _mix(streams, budget, 5, order_seed=4)
    _log(f"  stats {stats}")
    want = _oracle_labels(streams)
    for j in range(len(streams)):
        for t in range(3):
            assert np.array_equal(mix[j][t], want[j][t]), f"graph {j} batch {t}"
    assert stats["merged_rounds"] > 0
    if budget > 0:
        assert stats["evictions"] > 0 and stats["restores"] > 0
        assert stats["peak_resident_bytes"] <= budget


def test_server_batch_error_and_recovery():
    _log("case: server errors")
    streams = _streams([3000, 3000], 2, seed0=990)
    srv = dc.Server(max_inflight=2)
    gids = [srv.add_graph(n, u, v, w) for n, (u, v, w), _ in streams]
    bad = srv.submit(gids[0], [5], [5], [1])  # self-loop
    with pytest.raises(dc.DCError) as e:
        srv.poll(bad, gids[0])
    assert e.value.status == -3
    with pytest.raises(dc.DCError):
        srv.submit(99, [0], [1], [1])
    # the graph continues as if the bad batch had not been sent
    alone = _alone(streams)
    for t in range(2):
        tk = [srv.submit(gids[j], *(lambda b: (b.add_u, b.add_v, b.add_w, b.del_u, b.del_v))(
            streams[j][2][t])) for j in range(2)]
        for j in range(2):
            C, _, _ = srv.poll(tk[j], gids[j])
            assert np.array_equal(C, alone[j][t])
    srv.close()
