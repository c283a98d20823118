"""Pins of the oracle's screener samples and of its two-half step.

The samples (touched set, integer quantities, features, move labels) are
recomputed here from the exact-rational spec-literal reading: gains by
recomputing Eq. (1) (Sec. 3.1), Delta-screening as Python sets (Alg. 2,
Sec. 3.5), labels by a literal rerun of the level-0 sweeps (Alg. 1) with
every vertex active.  The features must equal the correctly rounded value of
their exact rational (Python's Fraction -> float rounds correctly)."""
from fractions import Fraction

import numpy as np
import pytest

import spec_literal as L
from oracle import oracle as O
from paper_1904_08553_amd import workloads as W


def literal_samples(adj_prev, adj, C, add_pairs, del_pairs, guard=True, max_sweeps=100,
                    tau_den=10 ** 6):
    n = len(adj)
    tm = L.two_m(adj)
    pairs = {(min(a, b), max(a, b)) for a, b in list(add_pairs) + list(del_pairs)}
    touch = {i: 0 for i in range(n)}
    for a, b in pairs:
        touch[a] += 1
        touch[b] += 1
    src = {x for p in pairs for x in p}
    Rds = L.screen(adj, C, add_pairs, del_pairs)
    T = set(src) | Rds
    for s in src:
        T |= set(adj[s])
    a = {}
    for v in range(n):
        a[C[v]] = a.get(C[v], 0) + L.degree(adj, v)
    # labels: level 0 rerun from C with every vertex active
    Cl = dict(C)
    Tthr = (tm * tm) // tau_den if tau_den else 0
    L.sweeps(adj, Cl, set(range(n)), max_sweeps, Tthr, guard, 0, [])
    out = []
    for i in sorted(T):
        c = C[i]
        k = L.degree(adj, i)
        e_own = sum(x for j, x in adj[i].items() if j != i and C[j] == c)
        cands = sorted({C[j] for j in adj[i] if j != i} - {c})
        gs = []
        for D in cands:
            g = L.gain(adj, C, i, D) * tm * tm / 2
            assert g.denominator == 1
            gs.append((-int(g), D))
        gs.sort()
        G1 = -gs[0][0] if len(gs) > 0 else None
        G2 = -gs[1][0] if len(gs) > 1 else None
        raw = [k, L.degree(adj_prev, i), touch[i], e_own, G1, G2, a[c], int(i in Rds)]
        out.append((i, raw, int(Cl[i] != c)))
    return out


def exact_features(raw, tm):
    k, kp, t, e_own, G1, G2, ac, ds = raw
    mx = max(k, kp)
    f = [
        Fraction(k, k + 16),
        Fraction(k - kp, mx) if mx > 0 else Fraction(0),
        Fraction(t, t + 4),
        Fraction(e_own, k) if k > 0 else Fraction(0),
        Fraction(G1, tm * k) if (k > 0 and G1 is not None) else Fraction(-3),
        Fraction(G2, tm * k) if (k > 0 and G2 is not None) else Fraction(-3),
        Fraction(ds),
        Fraction(ac, tm) if tm > 0 else Fraction(0),
    ]
    return [float(x) for x in f]


@pytest.mark.parametrize("seed", range(10))
def test_samples_match_literal(seed):
    n = 10 + seed % 5
    (u, v, w), batches = W.random_dynamic(n, 2 * n, 4, 5, 3, seed=7100 + seed)
    o = O.Oracle(n, u, v, w, collect=1)
    adj = L.adjacency(n, u, v, w)
    for b in batches:
        C = {i: int(x) for i, x in enumerate(o.C)}
        adj_prev = {i: dict(r) for i, r in adj.items()}
        for a_, b_ in zip(b.del_u, b.del_v):
            del adj[int(a_)][int(b_)]
            del adj[int(b_)][int(a_)]
        for a_, b_, x in zip(b.add_u, b.add_v, b.add_w):
            a_, b_, x = int(a_), int(b_), int(x)
            adj[a_][b_] = adj[a_].get(b_, 0) + x
            adj[b_][a_] = adj[b_].get(a_, 0) + x
        o.apply_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)
        s = o.samples()
        lit = literal_samples(adj_prev, adj, C,
                              list(zip(map(int, b.add_u), map(int, b.add_v))),
                              list(zip(map(int, b.del_u), map(int, b.del_v))))
        assert [x[0] for x in lit] == list(s["ids"])
        tm = L.two_m(adj)
        for q, (i, raw, y) in enumerate(lit):
            got = [None if r == O.NO_GAIN else int(r) for r in s["raw"][q]]
            assert got == raw, (i, got, raw)
            assert int(s["y"][q]) == y, i
            assert list(s["X"][q]) == exact_features(raw, tm), i


def test_samples_special_cases():
    """A deletion that isolates a vertex, a pair deleted and re-added (one
    changed pair), and a vertex with no foreign neighbour community."""
    # path 0-1-2 plus triangle 3-4-5 joined by 2-3
    u, v, w = [0, 1, 3, 4, 5, 2], [1, 2, 4, 5, 3, 3], [1, 1, 1, 1, 1, 1]
    o = O.Oracle(6, u, v, w, collect=1)
    o.apply_batch([4], [5], [2], [0, 4], [1, 5])  # 0 isolated; (4,5) replaced
    s = o.samples()
    rows = {int(i): (list(r), list(x)) for i, r, x in zip(s["ids"], s["raw"], s["X"])}
    raw0, x0 = rows[0]
    assert raw0[0] == 0 and raw0[1] == 1 and raw0[2] == 1
    assert x0[:6] == [0.0, -1.0, 0.2, 0.0, -3.0, -3.0]
    raw4, x4 = rows[4]
    assert raw4[2] == 1 and raw4[0] == 3 and raw4[1] == 2  # replace counts once
    assert x4[1] == float(Fraction(1, 3))


def test_finish_override_all_equals_mode_all():
    """Finishing a screened step over every vertex is the ALL step."""
    pp = W.PlantedPartition(n=300, blocks=6, p_in=0.15, p_out=0.01, seed=3)
    (u, v, w), batches = pp.batches(steps=2, n_ins=80, n_del=30)
    a = O.Oracle(pp.n, u, v, w, mode=O.MODE_ALL)
    d = O.Oracle(pp.n, u, v, w, mode=O.MODE_DELTA)
    b = batches[0]
    a.apply_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)
    d.stage_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)
    d.finish_batch(np.ones(pp.n, np.uint8))
    assert np.array_equal(a.C, d.C)
    assert a.trace == d.trace
    assert a.modularity() == d.modularity()


def test_stage_finish_equals_apply():
    pp = W.PlantedPartition(n=300, blocks=6, p_in=0.15, p_out=0.01, seed=4)
    (u, v, w), batches = pp.batches(steps=3, n_ins=80, n_del=30)
    x = O.Oracle(pp.n, u, v, w)
    y = O.Oracle(pp.n, u, v, w, mode=O.MODE_LEARNED)
    for b in batches:
        x.apply_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)
        y.stage_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)
        assert len(y.samples()["ids"]) > 0
        y.finish_batch()  # no override: the screened set
        assert np.array_equal(x.C, y.C) and np.array_equal(x.R, y.R)
        assert x.trace == y.trace


def test_stage_protocol_errors():
    o = O.Oracle(4, [0, 2], [1, 3], [1, 1])
    with pytest.raises(O.OracleError) as e:
        o.finish_batch()
    assert e.value.status == -1
    o.stage_batch([0], [2], [1])
    with pytest.raises(O.OracleError):
        o.stage_batch([1], [3], [1])
    o.finish_batch()
    assert o.samples()["ids"].size == 0  # not collecting
