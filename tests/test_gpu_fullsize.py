"""Full-size parity on the benchmark workload (1,000,000 vertices, 20,000,000
edges, batches of 1% of the edges), in the launch configuration bench.py
times: every step's C_t and R_t must hash to the oracle's, with equal exact
N, 2m and sweep traces.  The oracle's results are stored in
tests/golden/dcsbm_1M_20M_oracle.json by tests/golden/make_dcsbm_golden.py."""
import hashlib
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                    "dcsbm_1M_20M_oracle.json")


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def record(g):
    q, N, tm = g.modularity()
    R = g.last_R()
    return {"C": digest(g.communities()), "R": digest(R), "R_size": int(R.sum()), "N": N,
            "two_m": tm, "trace": [list(map(int, r)) for r in g.last_trace()]}


@pytest.fixture(scope="module")
def stream():
    from paper_1904_08553_amd import workloads as W
    gold = json.load(open(GOLD))
    steps = max(len(v) - 1 for v in gold["modes"].values())
    gen = W.DCSBM()
    (u, v, w), it = gen.stream(steps, frac=0.01, ins_frac=0.6)
    print("generated the full-size stream", flush=True)
    return gold, gen.n, (u, v, w), list(it)


@pytest.mark.parametrize("mode", ["delta", "all"])
def test_full_size_matches_oracle(stream, mode):
    import torch
    from paper_1904_08553_amd import dc
    gold, n, (u, v, w), batches = stream
    recs = gold["modes"][mode]
    g = dc.DynamicCommunities(n, u, v, w, mode=dc.MODE_DELTA if mode == "delta" else dc.MODE_ALL,
                              timing=1 if mode == "delta" else 0)
    assert record(g) == recs[0], "init differs"
    to_dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()
    for t, b in enumerate(batches[: len(recs) - 1]):
        print(f"{mode} step {t}", flush=True)
        g.apply_batch(to_dev(b.add_u), to_dev(b.add_v), to_dev(b.add_w), to_dev(b.del_u),
                      to_dev(b.del_v))
        got = record(g)
        want = recs[t + 1]
        for key in ("C", "R", "R_size", "N", "two_m"):
            assert got[key] == want[key], f"{mode} step {t}: {key} differs"
        assert got["trace"] == want["trace"], f"{mode} step {t}: sweep trace differs"
    g.close()
