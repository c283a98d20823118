"""Writes tests/golden/dcsbm_1M_20M_oracle.json: the CPU oracle's results on
the benchmark workload (DC-SBM, 1,000,000 vertices, 20,000,000 edges,
seed 0, batches of 1% of the edges, 60% insertions / 40% deletions).

Only the oracle and the seeded input generator are used.  Per step the file
holds the SHA-256 of C_t (int32 little endian) and of R_t (uint8), |R_t|, the
exact numerator N and 2m, and the sweep trace (level, sweep, n_level,
n_active, nnz_level, moves, dN, kept).  Takes a few minutes on one core.
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1904_08553_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "dcsbm_1M_20M_oracle.json")
STEPS = {"delta": 4, "all": 2}


def digest(a):
    return hashlib.sha256(a.tobytes()).hexdigest()


def record(o):
    q, N, tm = o.modularity()
    return {"C": digest(o.C), "R": digest(o.R), "R_size": int(o.R.sum()), "N": N, "two_m": tm,
            "trace": [list(map(int, r)) for r in o.trace]}


def main():
    res = {"workload": "DCSBM(n=1_000_000, m=20_000_000, blocks=1000, seed=0), "
                       "stream(frac=0.01, ins_frac=0.6)", "modes": {}}
    gen = W.DCSBM()
    (u, v, w), it = gen.stream(max(STEPS.values()), frac=0.01, ins_frac=0.6)
    batches = list(it)
    for mode, steps in STEPS.items():
        t0 = time.time()
        o = O.Oracle(gen.n, u, v, w, mode=O.MODE_DELTA if mode == "delta" else O.MODE_ALL)
        recs = [record(o)]
        print(mode, "init", time.time() - t0, flush=True)
        for b in batches[:steps]:
            o.apply_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)
            recs.append(record(o))
            print(mode, "step", time.time() - t0, flush=True)
        res["modes"][mode] = recs
        o.close()
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
