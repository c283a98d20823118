"""Temporal-resolution study (Sec. 4.4): one temporal event stream cut into
different numbers of time steps, each cut run with Delta-screening and with
the baseline that re-evaluates every vertex at the first level, reporting
the average modularity over the steps and the share of the total time that
Delta-screening saves.

The cuts are ``workloads.rebin`` of a ``workloads.temporal_events`` stream:
bin j of K holds events [floor(j E / K), floor((j + 1) E / K)), the first
bin builds G_1 (``dc_init``), and each later bin is one batch of the pairs
inserted or deleted on balance inside it.  Everything here is plumbing
around libdc.so; batches are copied to device memory before the clock
starts and C_t is written to a device buffer.

    python -m paper_1904_08553_amd.resolution --n 1000000 --events 7875000
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import dc
from . import workloads as W

STEPS = (2, 4, 8, 12, 16, 20, 24, 28)


def log(msg):
    print(f"[resolution] {msg}", file=sys.stderr, flush=True)


def run_cut(stream, steps, mode):
    """One cut under one mode: per-step seconds (step 1 = the static run
    on G_1) and modularity after every step."""
    import torch
    (u, v, w), it = W.rebin(stream, steps)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()
    batches = [(d(b.add_u), d(b.add_v), d(b.add_w), d(b.del_u), d(b.del_v)) for b in it]
    c_out = torch.empty(stream.n, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t = time.perf_counter()
    g = dc.DynamicCommunities(stream.n, u, v, w, mode=mode)
    torch.cuda.synchronize()
    secs = [time.perf_counter() - t]
    q = [g.last_stats().q]
    changes = 0
    for b in batches:
        t = time.perf_counter()
        g.apply_batch(*b, out=c_out)
        secs.append(time.perf_counter() - t)
        q.append(g.stats.q)
        changes += g.stats.changes
    g.close()
    return {"seconds": secs, "q": q, "changes": changes}


def study(stream, steps_list=STEPS):
    """Both modes on every cut; one record per number of steps."""
    rows = []
    for k in steps_list:
        ds = run_cut(stream, k, dc.MODE_DELTA)
        al = run_cut(stream, k, dc.MODE_ALL)
        td, ta = sum(ds["seconds"]), sum(al["seconds"])
        id_, ia = sum(ds["seconds"][1:]), sum(al["seconds"][1:])
        rows.append({
            "steps": k,
            "avg_q_delta": float(np.mean(ds["q"])),
            "avg_q_all": float(np.mean(al["q"])),
            "total_s_delta": td,
            "total_s_all": ta,
            "savings_pct": 100.0 * (ta - td) / ta,
            "incremental_savings_pct": 100.0 * (ia - id_) / ia if ia > 0 else None,
            "batch_changes": ds["changes"],
        })
        log(f"{k} steps: avg Q {rows[-1]['avg_q_delta']:.5f} (all {rows[-1]['avg_q_all']:.5f}), "
            f"total {td:.3f} s vs {ta:.3f} s, savings {rows[-1]['savings_pct']:.1f}%")
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--n", type=int, default=8_000_000)
    ap.add_argument("--events", type=int, default=63_000_000)
    ap.add_argument("--slices", type=int, default=12)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--steps", type=int, nargs="*", default=list(STEPS))
    a = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    t = time.perf_counter()
    stream = W.temporal_events(n=a.n, events=a.events, slices=a.slices,
                               blocks=max(10, a.n // 1000), seed=a.seed)
    log(f"{len(stream)} events drawn in {time.perf_counter() - t:.0f} s")
    print(json.dumps({"n": a.n, "events": a.events, "rows": study(stream, a.steps)}))


if __name__ == "__main__":
    main()
