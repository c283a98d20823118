"""Writes tests/golden/temporal_8M_63M_oracle.json: the CPU oracle's results on
the paper-scale temporal stream (8,000,000 vertices, 63,000,000 unit-weight
events in 12 steps of 5,250,000; step 1 builds G_1, steps 2..12 are batches of
85% insertions and 15% deletions of earlier edges, 8,000 Zipf(1.1) blocks,
mixing 0.2, propensities from a power law 2.1 on [2, 10^5], 2% of the vertices
changing block before each step; seed 0).  This is the shape of the paper's
63M-event interaction stream of Sec. 4.1 (Table 1).

Only the oracle and the seeded input generator are used.  Per step the file
holds the SHA-256 of C_t (int32 little endian) and of R_t (uint8), |R_t|, the
exact numerator N and 2m, and the sweep trace (level, sweep, n_level,
n_active, nnz_level, moves, dN, kept): every step under Delta-screening, the
first steps under the full recompute (mode ALL).  Each mode runs in a process
of its own; the whole run takes tens of minutes of host time.

    python tests/golden/make_temporal_golden.py            # both modes
    python tests/golden/make_temporal_golden.py --mode all # one mode, merged in
"""
import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "temporal_8M_63M_oracle.json")
WORKLOAD = dict(n=8_000_000, events=63_000_000, steps=12, blocks=8000, seed=0)
STEPS = {"delta": 11, "all": 2}  # batches after G_1


def digest(a):
    return hashlib.sha256(a.tobytes()).hexdigest()


def record(o):
    q, N, tm = o.modularity()
    return {"C": digest(o.C), "R": digest(o.R), "R_size": int(o.R.sum()), "N": N, "two_m": tm,
            "trace": [list(map(int, r)) for r in o.trace]}


def run_mode(mode):
    from oracle import oracle as O
    from paper_1904_08553_amd import workloads as W
    t0 = time.time()
    (u, v, w), it = W.temporal_stream(**WORKLOAD)
    o = O.Oracle(WORKLOAD["n"], u, v, w, mode=O.MODE_DELTA if mode == "delta" else O.MODE_ALL)
    recs = [record(o)]
    print(f"{mode} init {time.time() - t0:.0f} s", flush=True)
    for t, b in enumerate(it):
        if t >= STEPS[mode]:
            break
        o.apply_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)
        recs.append(record(o))
        print(f"{mode} step {t + 2}: {time.time() - t0:.0f} s, |R| = {recs[-1]['R_size']}",
              flush=True)
    o.close()
    return mode, recs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mode", choices=sorted(STEPS), action="append")
    args = ap.parse_args()
    modes = args.mode or sorted(STEPS)
    res = {"workload": "temporal_stream(" + ", ".join(f"{k}={v}" for k, v in WORKLOAD.items())
                       + ")", "modes": {}}
    if os.path.exists(OUT):
        old = json.load(open(OUT))
        if old.get("workload") == res["workload"]:
            res["modes"].update(old["modes"])
    with mp.get_context("spawn").Pool(len(modes)) as pool:
        for mode, recs in pool.imap_unordered(run_mode, modes):
            res["modes"][mode] = recs
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
