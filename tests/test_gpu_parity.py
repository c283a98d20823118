"""GPU parity: the HIP path (through include/dc.h) against the CPU oracle,
element by element, bit-exact for labels, R_t and every exact integer."""
import numpy as np
import pytest

from gpu_common import compare, make_pair, step_pair
from oracle import oracle as O
from paper_1904_08553_amd import dc
from paper_1904_08553_amd import workloads as W

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def test_two_triangles():
    _log("case: two triangles")
    o, g = make_pair(6, [0, 0, 1, 3, 3, 4, 2], [1, 2, 2, 4, 5, 5, 3], [1] * 7)
    compare(o, g, "init")
    assert list(g.communities()) == [0, 0, 0, 3, 3, 3]


@pytest.mark.parametrize("guard", [1, 0])
def test_k2(guard):
    _log(f"case: K2 guard={guard}")
    o, g = make_pair(2, [0], [1], [1], max_levels=1, guard=guard)
    compare(o, g, "init")


def test_edgeless_and_single_vertex():
    _log("case: edgeless")
    o, g = make_pair(5, [], [], [])
    compare(o, g, "init")
    assert g.modularity()[2] == 0
    o, g = make_pair(1, [], [], [])
    compare(o, g, "init")
    # a batch that adds the first edges
    o, g = make_pair(4, [], [], [])
    o.apply_batch([0, 2], [1, 3], [2, 5])
    g.apply_batch([0, 2], [1, 3], [2, 5])
    compare(o, g, "first edges")


CASES = [
    dict(mode="delta"),
    dict(mode="delta", del_rule=1, max_levels=2),
    dict(mode="all"),
    dict(mode="static", max_levels=3),
    dict(mode="delta", max_levels=1, guard=0),
    dict(mode="delta", tau_den=0),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("seed", range(8))
def test_random_small_dynamic(case, seed):
    cfg = CASES[case]
    n = 9 + seed
    _log(f"case: random small n={n} seed={seed} cfg={cfg}")
    (u, v, w), batches = W.random_dynamic(n, 2 * n, 4, 5, 3, seed=3000 + seed)
    o, g = make_pair(n, u, v, w, **cfg)
    compare(o, g, "init")
    for t, b in enumerate(batches):
        step_pair(o, g, b)
        compare(o, g, f"step {t}")


@pytest.mark.parametrize("mode", ["delta", "all", "static"])
def test_planted_partition_2000(mode):
    """2,000 vertices in 20 equal blocks (p_in 0.05, p_out 0.001), 4 steps of
    500 insertions (70% intra) and 200 deletions, one coarsening level."""
    _log(f"case: planted partition mode={mode}")
    pp = W.PlantedPartition()
    (u, v, w), batches = pp.batches()
    o, g = make_pair(pp.n, u, v, w, mode=mode, max_levels=2)
    compare(o, g, "init")
    for t, b in enumerate(batches):
        step_pair(o, g, b)
        compare(o, g, f"step {t}")


@pytest.mark.parametrize("seed", [0, 2])
def test_dcsbm_with_hubs(seed):
    """Power-law degrees up to thousands: all row-length bins and
    multi-chunk coarsening are exercised; several steps of 1% batches.  The
    first sweep from singletons gives rows of 257-512 and 1025-4096 entries
    more distinct labels than their small LDS tables hold, so those rows are
    evaluated again with the full table."""
    _log(f"case: dcsbm hubs seed={seed}")
    gen = W.DCSBM(n=20000, m=200000, blocks=40, dmax=20000, seed=seed)
    (u, v, w), it = gen.stream(3, frac=0.01)
    deg = np.bincount(np.concatenate([u, v]), minlength=gen.n)
    assert deg.max() > 2048 and ((deg > 128) & (deg <= 2048)).any()
    assert ((deg > 256) & (deg <= 512)).any() and ((deg > 1024) & (deg <= 4096)).any()
    o, g = make_pair(gen.n, u, v, w)
    compare(o, g, "init")
    for t, b in enumerate(it):
        step_pair(o, g, b)
        compare(o, g, f"step {t}")


def test_contexts_on_reused_device_memory():
    """Device buffers of a destroyed context go back to the library's block
    cache and the next context takes them with the old contents in place:
    a graph run after another graph of the same size (and then after its own
    earlier run) still equals the oracle, so no kernel relies on memory that
    starts at zero unless it clears it; after dc_trim_device_cache the same
    graph runs on fresh blocks."""
    gen_a = W.DCSBM(n=20000, m=200000, blocks=40, dmax=20000, seed=7)
    gen_b = W.DCSBM(n=20000, m=200000, blocks=40, dmax=20000, seed=8)
    (ua, va, wa), it_a = gen_a.stream(2, frac=0.01)
    (ub, vb, wb), it_b = gen_b.stream(2, frac=0.01)
    batches_b = list(it_b)
    _log("case: reused memory, graph A fills the cache")
    ga = dc.DynamicCommunities(gen_a.n, ua, va, wa)
    for b in it_a:
        ga.apply_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)
    ga.close()
    for rep in range(3):
        if rep == 2:
            dc.trim_device_cache()  # the last run on freshly allocated memory
        _log(f"case: reused memory, graph B run {rep}")
        o, g = make_pair(gen_b.n, ub, vb, wb)
        compare(o, g, f"run {rep} init")
        for t, b in enumerate(batches_b):
            step_pair(o, g, b)
            compare(o, g, f"run {rep} step {t}")
        g.close()


def test_batch_errors_leave_state_unchanged():
    from paper_1904_08553_amd.dc import DCError
    _log("case: batch errors")
    pp = W.PlantedPartition(n=200, blocks=4, p_in=0.2, p_out=0.01)
    (u, v, w), _ = pp.batches(steps=0)
    o, g = make_pair(200, u, v, w)
    C0 = g.communities().copy()
    q0 = g.modularity()
    csr0 = g.csr()
    e0 = (int(u[0]), int(v[0]))
    missing = next((a, b) for a in range(200) for b in range(a + 1, 200)
                   if not ((u == a) & (v == b)).any())
    bad = [
        (dict(add_u=[0], add_v=[700], add_w=[1]), -2),
        (dict(del_u=[-1], del_v=[2]), -2),
        (dict(add_u=[3], add_v=[3], add_w=[1]), -3),
        (dict(add_u=[3], add_v=[4], add_w=[0]), -4),
        (dict(del_u=[e0[0], e0[1]], del_v=[e0[1], e0[0]]), -6),
        (dict(del_u=[missing[0]], del_v=[missing[1]]), -5),
        (dict(add_u=[3], add_v=[4], add_w=[2 ** 30]), -7),
    ]
    for kw, code in bad:
        with pytest.raises(DCError) as e:
            g.apply_batch(**kw)
        assert e.value.status == code
        assert np.array_equal(g.communities(), C0)
        assert g.modularity() == q0
        c1 = g.csr()
        assert all(np.array_equal(x, y) for x, y in zip(csr0, c1))
    # the context still works and agrees with the oracle afterwards
    o.apply_batch([missing[0]], [missing[1]], [3], [e0[0]], [e0[1]])
    g.apply_batch([missing[0]], [missing[1]], [3], [e0[0]], [e0[1]])
    compare(o, g, "after errors")


def test_replace_and_duplicate_insertions():
    _log("case: replace + duplicates")
    (u, v, w), _ = W.random_dynamic(30, 60, 0, 0, 0, seed=77)
    o, g = make_pair(30, u, v, w)
    a, b = int(u[0]), int(v[0])
    # delete and re-add one edge, add a new pair twice in both orientations
    new = next((x, y) for x in range(30) for y in range(x + 1, 30)
               if not ((u == x) & (v == y)).any())
    add_u = [a, new[0], new[1]]
    add_v = [b, new[1], new[0]]
    add_w = [7, 2, 3]
    o.apply_batch(add_u, add_v, add_w, [b], [a])
    g.apply_batch(add_u, add_v, add_w, [b], [a])
    compare(o, g, "replace")
    offo, colo, wo = o.csr()
    offg, colg, wg = g.csr()
    assert np.array_equal(offo, offg) and np.array_equal(colo, colg) and np.array_equal(wo, wg)


@pytest.mark.parametrize("graph", ["planted", "dcsbm", "random"])
def test_full_and_incremental_coarsening_agree(graph):
    """Level-0 compaction from all of G_t (full_coarsen=1) and from the
    previous graph of communities plus the batch and the movers (default)
    give the same run, and both equal the oracle, over several steps."""
    _log(f"case: full vs incremental compaction {graph}")
    if graph == "planted":
        pp = W.PlantedPartition()
        (u, v, w), batches = pp.batches()
        n = pp.n
    elif graph == "dcsbm":
        gen = W.DCSBM(n=20000, m=200000, blocks=40, dmax=20000, seed=5)
        (u, v, w), it = gen.stream(4, frac=0.02)
        batches, n = list(it), gen.n
    else:
        (u, v, w), batches = W.random_dynamic(40, 120, 6, 20, 12, seed=4242)
        n = 40
    o = O.Oracle(n, u, v, w)
    from paper_1904_08553_amd import dc
    gi = dc.DynamicCommunities(n, u, v, w)
    gf = dc.DynamicCommunities(n, u, v, w, full_coarsen=1)
    for t, b in enumerate(batches):
        o.apply_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)
        for g in (gi, gf):
            g.apply_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)
            compare(o, g, f"step {t}")
        assert gi.last_trace() == gf.last_trace()


def _merge_case(seed):
    """A batch with a hub row of 6000 entries (several merge tiles) taking
    more than 4096 changes (more than a tile stages in LDS), rows of 600,
    300 and 200 entries with tens of changes, replacements, and a sparse
    background with a few changes per row."""
    rng = np.random.default_rng(seed)
    n = 12000
    pairs = set()

    def star(c, lo, hi):
        for x in range(lo, hi):
            pairs.add((min(c, x), max(c, x)))

    star(0, 1, 6001)
    star(7000, 7001, 7601)
    star(8000, 8001, 8301)
    star(9000, 9001, 9201)
    while len(pairs) < 6000 + 600 + 300 + 200 + 30000:
        a, b = (int(x) for x in rng.integers(0, n, 2))
        if a != b:
            pairs.add((min(a, b), max(a, b)))
    edges = sorted(pairs)
    u = np.array([p[0] for p in edges], np.int32)
    v = np.array([p[1] for p in edges], np.int32)
    w = rng.integers(1, 9, len(edges)).astype(np.int32)
    add, dele, rep = [], [], []

    def fresh(a, cands):
        out = []
        for b in cands:
            p = (min(a, int(b)), max(a, int(b)))
            if a != int(b) and p not in pairs:
                pairs.add(p)
                out.append(p)
        return out

    add += fresh(0, range(6001, 10601))                              # 4600 insertions
    dele += [(0, int(x)) for x in rng.choice(np.arange(1, 6001), 200, replace=False)]
    rep += [(0, int(x)) for x in rng.choice(np.arange(1, 6001), 50, replace=False)
            if (0, int(x)) not in dele]
    add += fresh(7000, rng.choice(np.arange(10601, n), 20, replace=False))
    dele += [(7000, int(x)) for x in rng.choice(np.arange(7001, 7601), 10, replace=False)]
    add += fresh(8000, rng.choice(np.arange(10601, n), 50, replace=False))
    dele += [(8000, int(x)) for x in rng.choice(np.arange(8001, 8301), 30, replace=False)]
    add += fresh(9000, rng.choice(np.arange(10601, n), 25, replace=False))
    dele += [(9000, int(x)) for x in rng.choice(np.arange(9001, 9201), 15, replace=False)]
    rep += [(9000, 9199), (8000, 8299)]
    bg = [e for e in edges[6000 + 600 + 300 + 200:] if e[0] not in (0, 7000, 8000, 9000)]
    idx = rng.choice(len(bg), 300, replace=False)
    dele += [bg[i] for i in idx[:200]]
    rep += [bg[i] for i in idx[200:]]
    add += fresh(int(rng.integers(0, n)), rng.integers(0, n, 400))
    dset = set(dele)
    rep = [p for p in rep if p not in dset]
    add_u = [p[0] for p in add] + [p[1] for p in rep]
    add_v = [p[1] for p in add] + [p[0] for p in rep]
    add_w = list(rng.integers(1, 9, len(add))) + [9] * len(rep)
    del_u = [p[1] for p in dele] + [p[0] for p in rep]
    del_v = [p[0] for p in dele] + [p[1] for p in rep]
    return n, (u, v, w), (add_u, add_v, add_w, del_u, del_v)


@pytest.mark.parametrize("seed", [0, 1])
def test_merge_paths_csr_equal(seed):
    """G_t's CSR after a batch equals the oracle's entry for entry."""
    _log(f"case: merge paths seed={seed}")
    n, (u, v, w), b = _merge_case(seed)
    o, g = make_pair(n, u, v, w)
    compare(o, g, "init")
    o.apply_batch(*b)
    g.apply_batch(*b)
    offo, colo, wo = o.csr()
    offg, colg, wg = g.csr()
    assert np.array_equal(offo, offg), "row offsets differ"
    assert np.array_equal(colo, colg) and np.array_equal(wo, wg), "entries differ"
    compare(o, g, "after batch")


def test_merge_tile_edges():
    """Merge corner cases: insertions into rows that were empty, a row that
    loses every entry, a 2500-entry row spanning three merge tiles whose
    600 changes (more than a tile stages in LDS) include a new neighbour
    below all old ones, new ones above all, and deletions of its first and
    last entries; then a second batch on the merged graph."""
    _log("case: merge tile edges")
    rng = np.random.default_rng(7)
    n = 5000
    pairs = {(1, x) for x in range(2, 2502)}
    while len(pairs) < 2500 + 20000:
        a, b = (int(x) for x in rng.integers(2, 4990, 2))
        if a != b:
            pairs.add((min(a, b), max(a, b)))
    edges = sorted(pairs)
    u = np.array([p[0] for p in edges], np.int32)
    v = np.array([p[1] for p in edges], np.int32)
    w = rng.integers(1, 9, len(edges)).astype(np.int32)
    deg = np.bincount(np.concatenate([u, v]), minlength=n)
    assert (deg[4990:] == 0).all() and deg[0] == 0
    victim = next(x for x in range(2502, 4990) if 2 <= deg[x] <= 6)
    add = [(4990, 4991), (4990, 4992), (4993, 10), (4999, 0), (0, 1), (4998, 4999)]
    add += [(1, x) for x in range(4990, 4998)]
    dele = [(1, 2), (1, 2501)] + [p for p in edges if victim in p]
    dele += [(1, int(x)) for x in rng.choice(np.arange(3, 2501), 300, replace=False)]
    dset = set(dele)
    rep = [(1, int(x)) for x in rng.choice(np.arange(3, 2501), 400, replace=False)
           if (1, int(x)) not in dset][:280]
    add_u = [p[0] for p in add] + [p[1] for p in rep]
    add_v = [p[1] for p in add] + [p[0] for p in rep]
    add_w = [3] * len(add) + [7] * len(rep)
    del_u = [p[1] for p in dele] + [p[0] for p in rep]
    del_v = [p[0] for p in dele] + [p[1] for p in rep]
    o, g = make_pair(n, u, v, w)
    compare(o, g, "init")
    for t, b in enumerate([(add_u, add_v, add_w, del_u, del_v),
                           ([4990, 0], [4999, 4993], [2, 2], [4990, 1], [4991, 0])]):
        o.apply_batch(*b)
        g.apply_batch(*b)
        offo, colo, wo = o.csr()
        offg, colg, wg = g.csr()
        assert np.array_equal(offo, offg), f"batch {t}: row offsets differ"
        assert np.array_equal(colo, colg) and np.array_equal(wo, wg), f"batch {t}: entries differ"
        compare(o, g, f"after batch {t}")


@pytest.mark.parametrize("mode", ["delta", "all"])
def test_empty_batch_and_deleting_every_edge(mode):
    """Degenerate batches: nothing at all (no change list, nothing to
    merge), then every edge deleted (G_t left without entries), then edges
    added back to the empty graph."""
    _log(f"case: empty and delete-all batches mode={mode}")
    (u, v, w), _ = W.random_dynamic(40, 90, 1, 1, 1, seed=77)
    o, g = make_pair(40, u, v, w, mode=mode)
    compare(o, g, "init")
    step_batch = lambda *b: (o.apply_batch(*b), g.apply_batch(*b))
    step_batch([], [], [], [], [])
    compare(o, g, "empty batch")
    step_batch([], [], [], list(u), list(v))
    compare(o, g, "every edge deleted")
    offo, colo, _ = o.csr()
    offg, colg, _ = g.csr()
    assert offg[-1] == 0 and np.array_equal(offo, offg) and len(colg) == len(colo) == 0
    step_batch(list(u[:30]), list(v[:30]), list(w[:30]), [], [])
    compare(o, g, "edges added back")


@pytest.mark.parametrize("mode", ["delta", "all"])
def test_weights_near_the_2m_limit(mode):
    """Weights of 2^21..2^22 and one edge that brings 2m to 2^31 - 2, the
    largest total the int64 gains allow (products of 2m and e near 2^62);
    one more unit of weight is refused on both sides, state unchanged."""
    from paper_1904_08553_amd.dc import DCError
    _log(f"case: weights near the 2m limit mode={mode}")
    (u, v, w), batches = W.random_dynamic(60, 200, 3, 30, 20, seed=5, wmax=2 ** 22)
    w = np.maximum(w, 2 ** 21).astype(np.int32)
    o, g = make_pair(60, u, v, w, mode=mode)
    compare(o, g, "init")
    for t, b in enumerate(batches):
        b.add_w[:] = np.maximum(b.add_w, 2 ** 21)
        step_pair(o, g, b)
        compare(o, g, f"step {t}")
    two_m = o.modularity()[2]
    off, col, _ = o.csr()
    a, b = next((a, b) for a in range(60) for b in range(a + 1, 60)
                if b not in col[off[a]:off[a + 1]])
    heavy = (2 ** 31 - 2 - two_m) // 2
    assert 1 <= heavy < 2 ** 31
    step_pair(o, g, W.Batch(np.array([a], np.int32), np.array([b], np.int32),
                            np.array([heavy], np.int32), np.empty(0, np.int32),
                            np.empty(0, np.int32)))
    compare(o, g, "2m = 2^31 - 2")
    assert g.modularity()[2] == 2 ** 31 - 2
    C0, q0 = g.communities().copy(), g.modularity()
    c, d = next((c, d) for c in range(60) for d in range(c + 1, 60)
                if (c, d) != (a, b) and d not in col[off[c]:off[c + 1]])
    with pytest.raises(DCError) as e:
        g.apply_batch([c], [d], [1])
    assert e.value.status == -7
    with pytest.raises(O.OracleError) as eo:
        o.apply_batch([c], [d], [1])
    assert eo.value.status == -7
    assert np.array_equal(g.communities(), C0) and g.modularity() == q0
    assert np.array_equal(o.C, C0) and o.modularity()[1:] == q0[1:]


@pytest.mark.parametrize("seed", [3, 4])
def test_alg2_sinks_with_long_rows(seed):
    """Alg. 2 sources whose best sink j* is a hub (rows of thousands of
    entries): gain2 is the gain stored at the mirror record j* -> i, and the
    R_t, labels and traces equal the oracle's, which walks j*'s row."""
    _log(f"case: Alg. 2 with hub sinks, seed {seed}")
    gen = W.DCSBM(n=20000, m=200000, blocks=40, dmax=20000, seed=seed)
    (u, v, w), it = gen.stream(3, frac=0.02)
    o, g = make_pair(gen.n, u, v, w)
    compare(o, g, "init")
    for t, b in enumerate(it):
        step_pair(o, g, b)
        compare(o, g, f"step {t}")


@pytest.mark.parametrize("mode", ["delta", "learned_fallback"])
def test_screening_set_kinds(mode):
    """Batches whose screening set is empty or one-sided: only deletions
    between communities of C_{t-1} (no Alg. 2 source, no intra-community
    deletion: the screening set and R_t are empty while the graph changes),
    only deletions inside communities (deletion endpoints alone), only
    insertions (Alg. 2 sources alone), and weight increases of existing
    pairs (insertion records that change no row's length)."""
    _log(f"case: screening set kinds mode={mode}")
    pp = W.PlantedPartition(n=400, blocks=4, p_in=0.12, p_out=0.01, seed=21)
    (u, v, w), _ = pp.batches(steps=1, n_ins=1, n_del=1)
    u, v, w = np.asarray(u), np.asarray(v), np.asarray(w)
    o, g = make_pair(pp.n, u, v, w, mode="delta")
    if mode == "learned_fallback":  # LEARNED without a screener runs Alg. 2 itself
        g.close()
        g = dc.DynamicCommunities(pp.n, u, v, w, mode=dc.MODE_LEARNED)
    compare(o, g, "init")
    rng = np.random.default_rng(5)
    live = {(int(a), int(b)): int(c) for a, b, c in zip(u, v, w)}

    def step(au, av, aw, du, dv, where):
        o.apply_batch(au, av, aw, du, dv)
        g.apply_batch(au, av, aw, du, dv)
        for a, b in zip(du, dv):
            live.pop((a, b), None)
        for a, b, c in zip(au, av, aw):
            live[(a, b)] = live.get((a, b), 0) + c
        compare(o, g, where)

    C = o.C.copy()
    inter = [e for e in live if C[e[0]] != C[e[1]]]
    pick = [inter[i] for i in rng.choice(len(inter), size=min(6, len(inter)), replace=False)]
    step([], [], [], [e[0] for e in pick], [e[1] for e in pick], "inter-community deletions only")
    assert int(g.last_R().sum()) == int(o.R.sum())
    C = o.C.copy()
    intra = [e for e in live if C[e[0]] == C[e[1]]]
    pick = [intra[i] for i in rng.choice(len(intra), size=8, replace=False)]
    step([], [], [], [e[0] for e in pick], [e[1] for e in pick], "intra-community deletions only")
    new = []
    while len(new) < 10:
        a, b = sorted(int(x) for x in rng.choice(pp.n, size=2, replace=False))
        if (a, b) not in live and (a, b) not in new:
            new.append((a, b))
    step([e[0] for e in new], [e[1] for e in new], [2] * len(new), [], [], "insertions only")
    have = list(live)[:12]
    step([e[0] for e in have], [e[1] for e in have], [3] * len(have), [], [],
         "weight increases of existing pairs")
