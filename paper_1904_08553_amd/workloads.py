"""Seeded synthetic dynamic-graph workloads.

This module only draws inputs: graphs and per-step batches of edge additions
and deletions.  It holds none of the community-detection arithmetic, and both
the HIP path and the CPU oracle consume exactly the arrays it returns.

The shapes follow the paper's inputs (Sec. 4.1, Table 1): streaming
stochastic-block-model graphs with random edge sampling, and a long temporal
interaction stream with mostly intra-community, localised growth.  Those
datasets are not reproduced; every input here is drawn from
``numpy.random.Generator(PCG64)`` seeded by ``SeedSequence((seed, tag, step))``.

Edges are canonical undirected pairs ``u < v`` with int32 ids and weights.
A batch is ``Batch(add_u, add_v, add_w, del_u, del_v)``: deletions remove
existing edges of the previous graph, insertions add edges absent from it.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def _rng(seed: int, *tags: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence((int(seed),) + tuple(int(t) for t in tags))))


def _searchsorted(a, x, side="left"):
    """np.searchsorted(a, x, side) for unsorted queries x, issued in sorted
    order (the binary searches then walk the table in one direction, far
    faster on large tables); the result is the same array."""
    x = np.asarray(x)
    if len(x) < 4096:
        return np.searchsorted(a, x, side=side)
    order = np.argsort(x, kind="stable")
    out = np.empty(len(x), np.intp)
    out[order] = np.searchsorted(a, x[order], side=side)
    return out


def _key(u, v):
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    return (lo << 32) | hi


def _unkey(k):
    k = np.asarray(k, np.int64)
    return (k >> 32).astype(np.int32), (k & 0xFFFFFFFF).astype(np.int32)


@dataclass
class Batch:
    add_u: np.ndarray
    add_v: np.ndarray
    add_w: np.ndarray
    del_u: np.ndarray
    del_v: np.ndarray

    @property
    def size(self) -> int:
        return int(len(self.add_u) + len(self.del_u))


@dataclass
class EdgeSet:
    """Sorted canonical keys of the current graph with aligned weights."""
    keys: np.ndarray
    w: np.ndarray

    @staticmethod
    def from_edges(u, v, w):
        k = _key(u, v)
        order = np.argsort(k, kind="stable")
        return EdgeSet(k[order], np.asarray(w, np.int32)[order])

    def __len__(self):
        return len(self.keys)

    def contains(self, k):
        k = np.asarray(k, np.int64)
        if len(self.keys) == 0:
            return np.zeros(len(k), bool)
        order = np.argsort(k, kind="stable")  # sorted queries search far faster
        ks = k[order]
        pos = np.minimum(np.searchsorted(self.keys, ks), len(self.keys) - 1)
        out = np.empty(len(k), bool)
        out[order] = self.keys[pos] == ks
        return out

    def apply(self, b: Batch):
        if len(b.del_u):
            dk = np.sort(_key(b.del_u, b.del_v))
            pos = np.searchsorted(self.keys, dk)
            keep = np.ones(len(self.keys), bool)
            keep[pos] = False
            self.keys, self.w = self.keys[keep], self.w[keep]
        if len(b.add_u):
            ak = _key(b.add_u, b.add_v)
            order = np.argsort(ak, kind="stable")
            ak, aw = ak[order], np.asarray(b.add_w, np.int32)[order]
            pos = np.searchsorted(self.keys, ak)
            self.keys = np.insert(self.keys, pos, ak)
            self.w = np.insert(self.w, pos, aw)

    def edges(self):
        u, v = _unkey(self.keys)
        return u, v, self.w.copy()


def _fresh_pairs(sampler, count, existing: EdgeSet, rng, max_rounds=64):
    """Draw ``count`` distinct canonical non-self-loop pairs absent from
    ``existing``; ``sampler(rng, k)`` returns candidate (u, v) arrays."""
    got = np.empty(0, np.int64)
    for _ in range(max_rounds):
        need = count - len(got)
        if need <= 0:
            break
        u, v = sampler(rng, int(need * 1.25) + 16)
        ok = u != v
        k = _key(u[ok], v[ok])
        k = k[~existing.contains(k)]
        k = k[~np.isin(k, got)]
        _, first = np.unique(k, return_index=True)
        k = k[np.sort(first)]
        got = np.concatenate([got, k[:need]])
    if len(got) < count:
        raise RuntimeError("could not draw enough distinct new pairs")
    return got


def _pick_deletions(es: EdgeSet, count, rng):
    count = min(int(count), len(es))
    idx = rng.choice(len(es), size=count, replace=False)
    return _unkey(es.keys[np.sort(idx)])


# ---------------------------------------------------------------------------
# Planted partition (equal blocks), the small stand-in for the streaming SBM
# inputs.


@dataclass
class PlantedPartition:
    n: int = 2000
    blocks: int = 20
    p_in: float = 0.05
    p_out: float = 0.001
    seed: int = 0
    block_of: np.ndarray = field(default=None, repr=False)

    def __post_init__(self):
        rng = _rng(self.seed, 1)
        perm = rng.permutation(self.n)
        bsz = self.n // self.blocks
        self.block_of = np.minimum(perm // bsz, self.blocks - 1).astype(np.int32)
        self.order = np.argsort(self.block_of, kind="stable").astype(np.int32)
        counts = np.bincount(self.block_of, minlength=self.blocks)
        self.bstart = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        self.members = [self.order[self.bstart[b]:self.bstart[b + 1]] for b in range(self.blocks)]

    def graph(self):
        rng = _rng(self.seed, 2)
        keys = []
        tri = {}
        for b in range(self.blocks):
            mem = self.members[b]
            if len(mem) not in tri:
                tri[len(mem)] = np.triu_indices(len(mem), 1)
            iu, ju = tri[len(mem)]
            m = rng.random(len(iu)) < self.p_in
            keys.append(_key(mem[iu[m]], mem[ju[m]]))
        sizes = np.array([len(m) for m in self.members], np.int64)
        inter_pairs = (self.n * (self.n - 1)) // 2 - int((sizes * (sizes - 1) // 2).sum())
        n_inter = rng.binomial(inter_pairs, self.p_out)
        intra = np.concatenate(keys) if keys else np.empty(0, np.int64)
        es = EdgeSet.from_edges(*_unkey(intra), np.ones(len(intra), np.int32))
        inter = _fresh_pairs(self._inter_sampler, n_inter, es, rng)
        k = np.concatenate([intra, inter])
        u, v = _unkey(np.sort(k))
        return u, v, np.ones(len(u), np.int32)

    def _intra_sampler(self, rng, k):
        b = rng.integers(0, self.blocks, size=k)
        sz = self.bstart[b + 1] - self.bstart[b]
        i = (rng.random(k) * sz).astype(np.int64)
        j = (rng.random(k) * (sz - 1)).astype(np.int64)
        j = j + (j >= i)
        return self.order[self.bstart[b] + i], self.order[self.bstart[b] + j]

    def _inter_sampler(self, rng, k):
        u = rng.integers(0, self.n, size=k).astype(np.int32)
        v = rng.integers(0, self.n, size=k).astype(np.int32)
        ok = self.block_of[u] != self.block_of[v]
        return u[ok], v[ok]

    def batches(self, steps=4, n_ins=500, intra_frac=0.7, n_del=200, weight=None, graph=None):
        """Per step: ``n_ins`` insertions of non-edges (``intra_frac`` inside
        a block) and ``n_del`` deletions uniform over the current edges.
        ``graph``: the result of ``graph()`` when already drawn."""
        u, v, w = self.graph() if graph is None else graph
        es = EdgeSet.from_edges(u, v, w)
        out = []
        for t in range(steps):
            rng = _rng(self.seed, 3, t)
            du, dv = _pick_deletions(es, n_del, rng)
            n_intra = int(round(n_ins * intra_frac))
            ki = _fresh_pairs(self._intra_sampler, n_intra, es, rng)
            tmp = EdgeSet(np.sort(np.concatenate([es.keys, ki])), np.zeros(len(es) + len(ki), np.int32))
            ko = _fresh_pairs(self._inter_sampler, n_ins - n_intra, tmp, rng)
            k = np.concatenate([ki, ko])
            au, av = _unkey(k)
            aw = np.ones(len(k), np.int32) if weight is None else rng.integers(1, weight + 1, len(k)).astype(np.int32)
            b = Batch(au, av, aw, du, dv)
            es.apply(b)
            out.append(b)
        return (u, v, w), out


# ---------------------------------------------------------------------------
# Degree-corrected SBM with power-law propensities and Zipf block sizes.


def _powerlaw_int(rng, n, gamma, lo, hi):
    d = np.arange(lo, hi + 1, dtype=np.float64)
    p = d ** (-gamma)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    return (lo + np.searchsorted(cdf, rng.random(n), side="right")).astype(np.float64)


def _zipf_sizes(n, blocks, s):
    """Block sizes proportional to rank^(-s), each at least 1, summing to n."""
    r = np.arange(1, blocks + 1, dtype=np.float64) ** (-s)
    raw = r / r.sum() * n
    sz = np.maximum(np.floor(raw).astype(np.int64), 1)
    diff = n - int(sz.sum())
    if diff > 0:
        frac = raw - np.floor(raw)
        sz[np.argsort(-frac, kind="stable")[:diff]] += 1
    elif diff < 0:
        sz[0] += diff  # the largest block absorbs the excess of the minimum-1 rule
    return sz


@dataclass
class DCSBM:
    n: int = 1_000_000
    m: int = 20_000_000
    blocks: int = 1000
    zipf_s: float = 1.1
    gamma: float = 2.3
    dmin: int = 4
    dmax: int = 5000
    mixing: float = 0.2
    wmax: int = 8
    seed: int = 0

    def __post_init__(self):
        rng = _rng(self.seed, 11)
        self.theta = _powerlaw_int(rng, self.n, self.gamma, self.dmin, self.dmax)
        sizes = _zipf_sizes(self.n, self.blocks, self.zipf_s)
        perm = rng.permutation(self.n)
        self.block_of = np.empty(self.n, np.int32)
        self.block_of[perm] = np.repeat(np.arange(self.blocks, dtype=np.int32), sizes)
        self._index()

    def _index(self):
        order = np.argsort(self.block_of, kind="stable").astype(np.int32)
        self.order = order
        th = self.theta[order]
        self.cum_sorted = np.cumsum(th)
        counts = np.bincount(self.block_of, minlength=self.blocks)
        self.bstart = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        csum = np.concatenate([[0.0], self.cum_sorted])
        self.bmass_lo = csum[self.bstart[:-1]]
        self.bmass_hi = csum[self.bstart[1:]]
        self.cum_all = np.cumsum(self.theta)

    def _draw_global(self, rng, k):
        x = rng.random(k) * self.cum_all[-1]
        return np.minimum(_searchsorted(self.cum_all, x, side="right"), self.n - 1).astype(np.int32)

    def _draw_in_block(self, rng, b):
        lo, hi = self.bmass_lo[b], self.bmass_hi[b]
        x = lo + rng.random(len(b)) * (hi - lo)
        pos = _searchsorted(self.cum_sorted, x, side="right")
        pos = np.clip(pos, self.bstart[b], self.bstart[b + 1] - 1)
        return self.order[pos]

    def _sampler(self, rng, k):
        u = self._draw_global(rng, k)
        inside = rng.random(k) >= self.mixing
        v = np.empty(k, np.int32)
        v[inside] = self._draw_in_block(rng, self.block_of[u[inside]])
        out_idx = np.flatnonzero(~inside)
        vo = self._draw_global(rng, len(out_idx))
        same = self.block_of[vo] == self.block_of[u[out_idx]]
        for _ in range(64):
            if not same.any():
                break
            vo[same] = self._draw_global(rng, int(same.sum()))
            same = self.block_of[vo] == self.block_of[u[out_idx]]
        v[out_idx] = vo
        keep = np.ones(k, bool)
        keep[out_idx[same]] = False  # a pair still inside one block is dropped
        return u[keep], v[keep]

    def graph(self):
        rng = _rng(self.seed, 12)
        empty = EdgeSet(np.empty(0, np.int64), np.empty(0, np.int32))
        k = np.sort(_fresh_pairs(self._sampler, self.m, empty, rng))
        u, v = _unkey(k)
        w = rng.integers(1, self.wmax + 1, len(k)).astype(np.int32) if self.wmax > 1 else np.ones(len(k), np.int32)
        return u, v, w

    def next_batch(self, es: EdgeSet, t: int, frac=0.01, ins_frac=0.6):
        rng = _rng(self.seed, 13, t)
        total = int(round(len(es) * frac))
        n_ins = int(round(total * ins_frac))
        n_del = total - n_ins
        du, dv = _pick_deletions(es, n_del, rng)
        k = _fresh_pairs(self._sampler, n_ins, es, rng)
        au, av = _unkey(k)
        aw = rng.integers(1, self.wmax + 1, len(k)).astype(np.int32) if self.wmax > 1 else np.ones(len(k), np.int32)
        return Batch(au, av, aw, du, dv)

    def stream(self, steps, frac=0.01, ins_frac=0.6):
        """Initial graph plus ``steps`` batches; yields batches lazily."""
        u, v, w = self.graph()
        es = EdgeSet.from_edges(u, v, w)

        def gen():
            for t in range(steps):
                b = self.next_batch(es, t, frac, ins_frac)
                es.apply(b)
                yield b

        return (u, v, w), gen()

    def drift(self, t, frac):
        """Reassign ``frac`` of the vertices to blocks drawn by size."""
        rng = _rng(self.seed, 14, t)
        k = int(round(self.n * frac))
        who = rng.choice(self.n, size=k, replace=False)
        counts = np.bincount(self.block_of, minlength=self.blocks).astype(np.float64)
        cdf = np.cumsum(counts)
        cdf /= cdf[-1]
        nb = np.minimum(np.searchsorted(cdf, rng.random(k), side="right"), self.blocks - 1)
        self.block_of[who] = nb.astype(np.int32)
        self._index()


def temporal_stream(n=8_000_000, events=63_000_000, steps=12, ins_frac=0.85,
                    blocks=8000, gamma=2.1, dmin=2, dmax=100_000, mixing=0.2,
                    drift=0.02, seed=0):
    """Temporal interaction stream with ``events`` unit-weight edge events in
    ``steps`` equal steps.  Step 1 holds insertions only (the initial graph);
    later steps hold ``ins_frac`` insertions and deletions of edges alive
    before the step, and ``drift`` of the vertices change block first."""
    g = DCSBM(n=n, m=0, blocks=blocks, gamma=gamma, dmin=dmin, dmax=dmax,
              mixing=mixing, wmax=1, seed=seed)
    per = events // steps
    rng = _rng(seed, 21)
    empty = EdgeSet(np.empty(0, np.int64), np.empty(0, np.int32))
    k = np.sort(_fresh_pairs(g._sampler, per, empty, rng))
    u, v = _unkey(k)
    w = np.ones(len(k), np.int32)
    es = EdgeSet(k, w.copy())

    def gen():
        for t in range(1, steps):
            g.drift(t, drift)
            r = _rng(seed, 22, t)
            n_ins = int(round(per * ins_frac))
            n_del = per - n_ins
            du, dv = _pick_deletions(es, n_del, r)
            kk = _fresh_pairs(g._sampler, n_ins, es, r)
            au, av = _unkey(kk)
            b = Batch(au, av, np.ones(len(kk), np.int32), du, dv)
            es.apply(b)
            yield b

    return (u, v, w), gen()


@dataclass
class EventStream:
    """Time-ordered unit-weight edge events: event e inserts (op[e] = 1) or
    deletes (op[e] = -1) the pair (u[e], v[e]).  The events of one pair
    alternate, starting with an insertion."""
    n: int
    u: np.ndarray
    v: np.ndarray
    op: np.ndarray

    def __len__(self):
        return len(self.u)


def temporal_events(n=8_000_000, events=63_000_000, slices=12, seed=0, **kw) -> EventStream:
    """The stream of ``temporal_stream`` as one event sequence: the initial
    graph's insertions, then each later slice's insertions and deletions,
    every slice in a random order (a slice never holds two events of one
    pair)."""
    (u0, v0, _), it = temporal_stream(n=n, events=events, steps=slices, seed=seed, **kw)
    r = _rng(seed, 23)
    perm = r.permutation(len(u0))
    us, vs, ops = [u0[perm]], [v0[perm]], [np.ones(len(u0), np.int8)]
    for t, b in enumerate(it, start=1):
        r = _rng(seed, 23, t)
        u = np.concatenate([b.add_u, b.del_u])
        v = np.concatenate([b.add_v, b.del_v])
        op = np.concatenate([np.ones(len(b.add_u), np.int8), -np.ones(len(b.del_u), np.int8)])
        perm = r.permutation(len(u))
        us.append(u[perm])
        vs.append(v[perm])
        ops.append(op[perm])
    return EventStream(n, np.concatenate(us).astype(np.int32), np.concatenate(vs).astype(np.int32),
                       np.concatenate(ops))


def bin_bounds(count: int, steps: int):
    """Event index bounds of ``steps`` bins of equal count: bin j holds
    events [floor(j count / steps), floor((j + 1) count / steps)), so the
    bins of s steps nest in those of any multiple of s."""
    return [(j * count) // steps for j in range(steps + 1)]


def _net(stream: EventStream, a: int, b: int):
    """Pairs inserted and deleted on balance by events [a, b)."""
    if b <= a:
        e = np.empty(0, np.int64)
        return e, e
    k = _key(stream.u[a:b], stream.v[a:b])
    uk, inv = np.unique(k, return_inverse=True)
    s = np.bincount(inv, weights=stream.op[a:b].astype(np.float64), minlength=len(uk))
    if np.any(np.abs(s) > 1):
        raise ValueError("the events of a pair do not alternate")
    return uk[s > 0], uk[s < 0]


def rebin(stream: EventStream, steps: int):
    """The stream cut into ``steps`` time steps (``bin_bounds``).  Returns
    the initial graph (the first bin's pairs inserted on balance, unit
    weights) and an iterator over the later bins' batches: a pair with more
    insertions than deletions inside the bin is an insertion (it was absent
    before the bin), the reverse a deletion, equal counts no change."""
    bounds = bin_bounds(len(stream), steps)
    ins0, del0 = _net(stream, bounds[0], bounds[1])
    if len(del0):
        raise ValueError("the first bin deletes a pair it never inserted")
    u, v = _unkey(ins0)

    def gen():
        for j in range(1, steps):
            ins, dele = _net(stream, bounds[j], bounds[j + 1])
            au, av = _unkey(ins)
            du, dv = _unkey(dele)
            yield Batch(au, av, np.ones(len(au), np.int32), du, dv)

    return (u, v, np.ones(len(u), np.int32)), gen()


# ---------------------------------------------------------------------------
# Learned-screener and serving workloads.


def screener_graph(seed, n=None, n_lo=100_000, n_hi=1_000_000, steps=4, ins_frac=0.073,
                   del_frac=0.029, intra_frac=0.7):
    """A training or evaluation graph of the learned screener: planted
    partition with 100-vertex blocks (expected intra-community degree 4.95,
    inter-community degree 1.9), n log-uniform in [n_lo, n_hi] unless given,
    unit weights, and ``steps`` batches of ``ins_frac`` (70% intra-community)
    insertions and ``del_frac`` deletions of the initial edge count.
    Returns (n, (u, v, w), batches)."""
    if n is None:
        r = _rng(seed, 41)
        n = int(round(np.exp(r.uniform(np.log(n_lo), np.log(n_hi)))))
    n = max(200, (n // 100) * 100)
    pp = PlantedPartition(n=n, blocks=n // 100, p_in=0.05, p_out=1.9 / (n - 100), seed=seed)
    u, v, w = pp.graph()
    m = len(u)
    (u, v, w), batches = pp.batches(steps=steps, n_ins=int(round(ins_frac * m)),
                                    intra_frac=intra_frac, n_del=int(round(del_frac * m)),
                                    graph=(u, v, w))
    return n, (u, v, w), batches


def serving_graph(seed, batches, n=None, n_lo=10_000, n_hi=2_000_000, size_lo=100_000,
                  size_hi=200_000, ins_frac=0.6):
    """One graph of the serving workload: degree-corrected SBM shaped like
    the 1M/20M stream (20 edges per vertex, max(10, n/1000) blocks), n
    log-uniform in [n_lo, n_hi] unless given, and ``batches`` batches of
    U[size_lo, size_hi] changes (``ins_frac`` insertions) clipped to the
    current edge count, deletions to at most 40% of it.
    Returns (n, (u, v, w), [Batch])."""
    r = _rng(seed, 51)
    if n is None:
        n = int(round(np.exp(r.uniform(np.log(n_lo), np.log(n_hi)))))
    gen = DCSBM(n=n, m=20 * n, blocks=max(10, n // 1000), dmax=min(5000, n // 2), seed=seed)
    u, v, w = gen.graph()
    es = EdgeSet.from_edges(u, v, w)
    out = []
    for t in range(batches):
        size = min(int(r.integers(size_lo, size_hi + 1)), len(es))
        n_del = min(int(round(size * (1 - ins_frac))), int(0.4 * len(es)))
        b = gen.next_batch(es, t, frac=size / max(len(es), 1),
                           ins_frac=1.0 - n_del / max(size, 1))
        es.apply(b)
        out.append(b)
    return n, (u, v, w), out


def _distinct_pairs(sampler, count, rng):
    """``count`` distinct canonical pairs (no self-loops) from ``sampler``,
    in a seeded random order."""
    got = np.empty(0, np.int64)
    for _ in range(64):
        need = count - len(got)
        if need <= 0:
            break
        u, v = sampler(rng, int(need * 1.3) + 64)
        ok = u != v
        got = np.union1d(got, _key(u[ok], v[ok]))
    if len(got) < count:
        raise RuntimeError("could not draw enough distinct pairs")
    return got[rng.permutation(len(got))[:count]]


class ServingStream:
    """One graph of the serving workload at full scale, drawn in time
    proportional to each batch.  A universe of distinct pairs is drawn once
    from the degree-corrected SBM of the 1M/20M stream (20 edges per vertex,
    max(10, n/1000) blocks, weights in [1, 8]): the first 20 n pairs form G_1,
    the other ``reserve`` x 20 n are absent and form the pool new edges come
    from.  A batch of U[size_lo, size_hi] changes (``ins_frac`` insertions;
    deletions at most 40% of the current edges; insertions at most the pool)
    deletes present pairs and inserts absent ones, each chosen uniformly, so
    every insertion is a non-edge of the current graph and every deletion an
    edge of it; deleted pairs return to the pool."""

    def __init__(self, seed, n=None, n_lo=10_000, n_hi=2_000_000, reserve=0.5):
        r = _rng(seed, 61)
        if n is None:
            n = int(round(np.exp(r.uniform(np.log(n_lo), np.log(n_hi)))))
        self.n = int(n)
        gen = DCSBM(n=self.n, m=0, blocks=max(10, self.n // 1000), dmax=min(5000, self.n // 2),
                    seed=seed)
        m0 = 20 * self.n
        total = int(round(m0 * (1 + reserve)))
        keys = _distinct_pairs(gen._sampler, total, _rng(seed, 62))
        self.u, self.v = _unkey(keys)
        self.w = _rng(seed, 63).integers(1, 9, total).astype(np.int32)
        # present / absent pairs as index lists with room for every pair
        self.present = np.empty(total, np.int64)
        self.absent = np.empty(total, np.int64)
        self.present[:m0] = np.arange(m0)
        self.absent[: total - m0] = np.arange(m0, total)
        self.np_, self.na_ = m0, total - m0
        self.rng = _rng(seed, 64)

    def graph(self):
        idx = self.present[: self.np_]
        return self.u[idx], self.v[idx], self.w[idx]

    @staticmethod
    def _take(arr, length, k, rng):
        """k uniform distinct entries of arr[:length]; the hole they leave is
        filled from the tail.  Returns (taken, new length)."""
        if k <= 0:
            return np.empty(0, np.int64), length
        pos = np.sort(rng.choice(length, size=k, replace=False))
        taken = arr[pos].copy()
        new_len = length - k
        holes = pos[pos < new_len]
        tail = np.arange(new_len, length)
        movers = tail[~np.isin(tail, pos, assume_unique=True)]
        arr[holes] = arr[movers]
        return taken, new_len

    def next_batch(self, size_lo=100_000, size_hi=200_000, ins_frac=0.6):
        r = self.rng
        size = min(int(r.integers(size_lo, size_hi + 1)), self.np_)
        n_del = min(int(round(size * (1 - ins_frac))), int(0.4 * self.np_))
        n_ins = min(size - n_del, self.na_)
        di, self.np_ = self._take(self.present, self.np_, n_del, r)
        ai, self.na_ = self._take(self.absent, self.na_, n_ins, r)
        self.present[self.np_: self.np_ + len(ai)] = ai
        self.np_ += len(ai)
        self.absent[self.na_: self.na_ + len(di)] = di
        self.na_ += len(di)
        return Batch(self.u[ai], self.v[ai], self.w[ai], self.u[di], self.v[di])


def random_dynamic(n, m, steps, n_add, n_del, seed, wmax=3):
    """Uniform random graph and batches (used for tiny exhaustive tests)."""
    rng = _rng(seed, 31)
    full = n * (n - 1) // 2
    m = min(m, full)
    iu, ju = np.triu_indices(n, 1)
    pick = rng.choice(full, size=m, replace=False)
    u, v = iu[pick].astype(np.int32), ju[pick].astype(np.int32)
    w = rng.integers(1, wmax + 1, m).astype(np.int32)
    es = EdgeSet.from_edges(u, v, w)
    out = []
    for t in range(steps):
        r = _rng(seed, 32, t)
        du, dv = _pick_deletions(es, min(n_del, len(es)), r)
        present = set(es.keys.tolist())
        cand = [(a, b) for a, b in zip(iu.tolist(), ju.tolist()) if ((a << 32) | b) not in present]
        na = min(n_add, len(cand))
        sel = r.choice(len(cand), size=na, replace=False) if na else np.empty(0, np.int64)
        au = np.array([cand[s][0] for s in sel], np.int32)
        av = np.array([cand[s][1] for s in sel], np.int32)
        aw = r.integers(1, wmax + 1, na).astype(np.int32)
        b = Batch(au, av, aw, du, dv)
        es.apply(b)
        out.append(b)
    return (u, v, w), out
