"""Spec-literal mini implementation of the method in exact rationals.

A second, deliberately naive reading of arXiv 1904.08553, written without the
oracle's scaled-integer gain: every modularity gain here is obtained by
recomputing Eq. (1) (Sec. 3.1) on the partition with the vertex moved, every
set of Alg. 2 (Sec. 3.5) is a Python set, and coarsening (Alg. 1, Sec. 3.2)
accumulates a dict of dicts.  Only usable on tiny graphs; it exists to pin the
oracle's traces from a different derivation.
"""
from __future__ import annotations

from fractions import Fraction


def adjacency(n, u, v, w):
    adj = {i: {} for i in range(n)}
    for a, b, x in zip(u, v, w):
        a, b, x = int(a), int(b), int(x)
        adj[a][b] = adj[a].get(b, 0) + x
        adj[b][a] = adj[b].get(a, 0) + x
    return adj


def degree(adj, i):
    return sum(adj[i].values())


def two_m(adj):
    return sum(degree(adj, i) for i in adj)


def modularity(adj, C):
    """Eq. (1): Q = (1/2m) (sum_i e_{i->C(i)} - (1/2m) sum_C a_C^2).
    A vertex's self-loop entry (coarse graphs) is part of e_{i->C(i)}."""
    tm = two_m(adj)
    if tm == 0:
        return Fraction(0)
    intra = sum(x for i in adj for j, x in adj[i].items() if C[j] == C[i])
    a = {}
    for i in adj:
        a[C[i]] = a.get(C[i], 0) + degree(adj, i)
    return Fraction(intra, tm) - Fraction(sum(y * y for y in a.values()), tm * tm)


def gain(adj, C, i, D):
    """Delta Q of moving i to community D, by recomputing Eq. (1)."""
    if C[i] == D:
        return Fraction(0)
    C2 = dict(C)
    C2[i] = D
    return modularity(adj, C2) - modularity(adj, C)


def decide(adj, C, i, guard=True):
    """Louvain rule (Sec. 3.2): best neighbouring community by gain, smallest
    label on ties, strictly positive gain to move, minimum-label guard for two
    singletons.  Returns (label, best gain among other communities)."""
    c = C[i]
    cands = sorted({C[j] for j in adj[i] if j != i} - {c})
    if degree(adj, i) == 0 or not cands:
        return c, Fraction(0)
    best, bg = None, None
    for D in cands:
        g = gain(adj, C, i, D)
        if bg is None or g > bg:
            best, bg = D, g
    if bg <= 0:
        return c, bg
    if guard:
        size = {}
        for x in C.values():
            size[x] = size.get(x, 0) + 1
        if size[c] == 1 and size[best] == 1 and best > c:
            return c, bg
    return best, bg


def sweeps(adj, C, active, max_sweeps, T, guard, level, trace):
    tm = two_m(adj)
    total = Fraction(0)
    for s in range(max_sweeps):
        C2 = dict(C)
        moves = 0
        for i in sorted(active):
            d, _ = decide(adj, C, i, guard)
            if d != C[i]:
                C2[i] = d
                moves += 1
        dQ = modularity(adj, C2) - modularity(adj, C)
        dN = dQ * tm * tm
        assert dN.denominator == 1
        kept = moves > 0 and dN >= 0
        trace.append((level, s, len(adj), len(active), moves, int(dN), int(kept)))
        if moves == 0 or dN < 0:
            break
        C.clear()
        C.update(C2)
        total += dN
        if dN <= T:
            break
    return total


def coarsen(adj, C):
    labels = sorted(set(C.values()))
    rank = {x: r for r, x in enumerate(labels)}
    H = {r: {} for r in range(len(labels))}
    for i in adj:
        for j, x in adj[i].items():
            a, b = rank[C[i]], rank[C[j]]
            H[a][b] = H[a].get(b, 0) + x
    return H, rank


def run_levels(adj0, C0, active0, max_levels=32, max_sweeps=100, tau_den=10**6, guard=True):
    tm = two_m(adj0)
    T = (tm * tm) // tau_den if tau_den else 0
    adj = adj0
    C = dict(C0)
    member_of = {v: v for v in adj0}  # level-0 vertex -> current level vertex
    trace = []
    level = 0
    while True:
        act = active0 if level == 0 else set(adj)
        g = sweeps(adj, C, act, max_sweeps, T, guard, level, trace)
        if level + 1 >= max_levels or (level >= 1 and g <= T):
            break
        adj, rank = coarsen(adj, C)
        member_of = {v: rank[C[x]] for v, x in member_of.items()}
        C = {x: x for x in adj}
        level += 1
    final = {v: C[x] for v, x in member_of.items()}
    groups = {}
    for v in sorted(final):
        groups.setdefault(final[v], v)
    return {v: groups[final[v]] for v in final}, trace, level + 1


# ---------------------------------------------------------------------------
# Smart local moving (the paper's second host method, Sec. 3.4; steps of its
# reference [waltman2013smart]): local moving, refinement of every community
# from singletons on the subnetwork it induces, compaction by the refined
# communities, next level from the parent communities.


def weighted_modularity(sub, C, weight, tm):
    """Eq. (1) on a subnetwork whose vertex weights and total weight are those
    of the larger graph it is part of: intra-community weight of `sub` over
    tm, minus the squared community weights over tm^2."""
    if tm == 0:
        return Fraction(0)
    intra = sum(x for i in sub for j, x in sub[i].items() if C[j] == C[i])
    a = {}
    for i in sub:
        a[C[i]] = a.get(C[i], 0) + weight[i]
    return Fraction(intra, tm) - Fraction(sum(y * y for y in a.values()), tm * tm)


def refine(sub, weight, tm, max_sweeps, T, guard, level, trace):
    """Local moving on the subnetwork from singletons (every vertex active),
    the Louvain rule with gains from weighted_modularity; returns labels."""
    C = {i: i for i in sub}
    for s in range(max_sweeps):
        C2 = dict(C)
        moves = 0
        size = {}
        for x in C.values():
            size[x] = size.get(x, 0) + 1
        base = weighted_modularity(sub, C, weight, tm)
        for i in sorted(sub):
            c = C[i]
            cands = sorted({C[j] for j in sub[i] if j != i} - {c})
            if weight[i] == 0 or not cands:
                continue
            best, bg = None, None
            for D in cands:
                Ct = dict(C)
                Ct[i] = D
                g = weighted_modularity(sub, Ct, weight, tm) - base
                if bg is None or g > bg:
                    best, bg = D, g
            if bg <= 0:
                continue
            if guard and size[c] == 1 and size[best] == 1 and best > c:
                continue
            C2[i] = best
            moves += 1
        dN = (weighted_modularity(sub, C2, weight, tm) - base) * tm * tm
        assert dN.denominator == 1
        kept = moves > 0 and dN >= 0
        trace.append((level, s, len(sub), len(sub), moves, int(dN), int(kept), 1))
        if moves == 0 or dN < 0:
            break
        C = C2
        if dN <= T:
            break
    return C


def run_levels_slm(adj0, C0, active0, max_levels=32, max_sweeps=100, tau_den=10**6,
                   guard=True):
    tm = two_m(adj0)
    T = (tm * tm) // tau_den if tau_den else 0
    adj = adj0
    C = dict(C0)
    member_of = {v: v for v in adj0}  # level-0 vertex -> current level vertex
    trace = []
    level = 0
    while True:
        act = active0 if level == 0 else set(adj)
        sweeps(adj, C, act, max_sweeps, T, guard, level, trace)
        if len(set(C.values())) == len(adj) or level + 1 >= max_levels:
            break
        sub = {i: {j: x for j, x in adj[i].items() if C[j] == C[i]} for i in adj}
        weight = {i: degree(adj, i) for i in adj}
        Rf = refine(sub, weight, tm, max_sweeps, T, guard, level, trace)
        H, rank = coarsen(adj, Rf)
        if len(H) == len(adj):
            break
        parent_of = {rank[Rf[i]]: C[i] for i in adj}
        first = {}
        for x, p in parent_of.items():
            first[p] = min(first.get(p, x), x)
        member_of = {v: rank[Rf[x]] for v, x in member_of.items()}
        adj, C = H, {x: first[p] for x, p in parent_of.items()}
        level += 1
    final = {v: C[x] for v, x in member_of.items()}
    groups = {}
    for v in sorted(final):
        groups.setdefault(final[v], v)
    return {v: groups[final[v]] for v in final}, trace, level + 1


def screen(adj, C, add_pairs, del_pairs, del_rule="gain", cascade=None):
    """Alg. 2 on additions plus the deletion extension; returns R_t.
    cascade = (num, den): the cascade extension -- every neighbour v of an
    accepted source i with C(v) = C(i) whose best move to another
    neighbouring community has Delta Q >= -2 theta k_v / 2m (theta = num/den)
    adds v and its neighbours."""
    R = set()
    accepted = []
    sinks = {}
    for a, b in add_pairs:
        sinks.setdefault(a, set()).add(b)
        sinks.setdefault(b, set()).add(a)
    for i in sorted(sinks):
        best = None
        for j in sorted(sinks[i]):
            g = gain(adj, C, i, C[j])
            key = (-g, C[j], j)
            if best is None or key < best[0]:
                best = (key, j, g)
        _, js, g1 = best
        g2 = gain(adj, C, js, C[i])
        if g1 >= g2 and g1 > 0:
            accepted.append(i)
            R |= {i, js} | set(adj[i]) | {v for v in adj if C[v] == C[js]}
    if cascade is not None:
        theta = Fraction(cascade[0], cascade[1])
        tm = two_m(adj)
        cand = {v for i in accepted for v in adj[i] if v != i and C[v] == C[i]}
        for v in sorted(cand):
            others = {C[j] for j in adj[v] if j != v} - {C[v]}
            if not others:
                continue
            best = max(gain(adj, C, v, D) for D in others)
            if best >= -2 * theta * degree(adj, v) / tm:
                R |= {v} | set(adj[v])
    srcs = set()
    for a, b in del_pairs:
        if C[a] == C[b]:
            srcs |= {a, b}
    for i in sorted(srcs):
        if del_rule == "conservative":
            R |= {i} | set(adj[i])
            continue
        d, _ = decide(adj, C, i, guard=False)
        if d != C[i]:
            R |= {i} | set(adj[i]) | {v for v in adj if C[v] == d}
    return R


class Literal:
    """Dynamic driver mirroring the incremental procedure of Sec. 3.4."""

    def __init__(self, n, u, v, w, mode="delta", del_rule="gain", cascade=None,
                 algorithm="louvain", **lv):
        self.n = n
        self.adj = adjacency(n, u, v, w)
        self.mode, self.del_rule, self.lv = mode, del_rule, lv
        self.cascade = cascade
        self.levels_fn = run_levels_slm if algorithm == "slm" else run_levels
        C0 = {i: i for i in range(n)}
        self.C, self.trace, self.levels = self.levels_fn(self.adj, C0, set(range(n)), **lv)
        self.R = set(range(n))

    def apply_batch(self, au, av, aw, du, dv):
        for a, b in zip(du, dv):
            a, b = int(a), int(b)
            del self.adj[a][b]
            del self.adj[b][a]
        for a, b, x in zip(au, av, aw):
            a, b, x = int(a), int(b), int(x)
            self.adj[a][b] = self.adj[a].get(b, 0) + x
            self.adj[b][a] = self.adj[b].get(a, 0) + x
        if self.mode == "delta":
            R = screen(self.adj, self.C, list(zip(map(int, au), map(int, av))),
                       list(zip(map(int, du), map(int, dv))), self.del_rule,
                       self.cascade)
            C0 = dict(self.C)
        elif self.mode == "all":
            R, C0 = set(range(self.n)), dict(self.C)
        else:
            R, C0 = set(range(self.n)), {i: i for i in range(self.n)}
        self.R = R
        self.C, self.trace, self.levels = self.levels_fn(self.adj, C0, R, **self.lv)
        return self.C

    def modularity(self):
        return modularity(self.adj, self.C)
