"""Throughput of Delta-screening incremental community detection on one MI355X.

Workload (default): degree-corrected SBM with 1,000,000 vertices and
20,000,000 undirected edges, power-law propensities (exponent 2.3 on
[4, 5000]), 1,000 Zipf(1.1)-sized blocks, mixing 0.2, int32 weights in
[1, 8]; every step is a batch of 1% of the current edges (60% insertions of
new edges, 40% deletions of existing ones).  All inputs are seeded synthetic
stand-ins for the paper's streaming SBM graphs.

A step is one dc_apply_batch (validate, merge, Alg. 2 screening, level-0
sweeps over R_t, coarsening, upper levels, canonical labels) with the batch
already in HBM.  The same batches are replayed in full-recompute mode (the
baseline of Sec. 3.4 with R_t = V_t) for the speedup and matched modularity.
Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "edge updates/sec at matched modularity (ΔS vs full); p50/p99 per-batch latency"
HBM_PEAK_GBS = 8000.0
TRAFFIC = os.path.join(ROOT, "profiles", "k_eval_groups_dcsbm_1M_20M_traffic.json")


ISSUE = os.path.join(ROOT, "profiles", "k_eval_groups_dcsbm_1M_20M_issue.json")


def measured_issue():
    """Share of the chip's vector-instruction issue capacity the timed kernel
    used, from the counter pass recorded in profiles/ (None once the kernel
    source has changed)."""
    import hashlib
    try:
        rec = json.load(open(ISSUE))
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, ValueError, KeyError):
        return None
    if hashlib.sha256(src).hexdigest() != rec.get("source_sha256"):
        return None
    return {"valu_issue_frac": rec["valu_issue_frac"], "summary": rec["summary"]}


def measured_traffic():
    """HBM bytes per launch of the timed kernel from the counter passes
    recorded in profiles/, or None once the kernel source has changed."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC))
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, ValueError, KeyError):
        return None
    if hashlib.sha256(src).hexdigest() != rec.get("source_sha256"):
        return None
    return rec["bytes_per_launch"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def percentile(xs, p):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=float), p)) if xs else None


def run_mode(mode, n, graph, batches_dev, warmup, steps, timing, **opt):
    import torch
    from paper_1904_08553_amd import dc
    u, v, w = graph
    t0 = time.perf_counter()
    g = dc.DynamicCommunities(n, u, v, w, mode=mode, timing=timing, **opt)
    torch.cuda.synchronize()
    init_ms = (time.perf_counter() - t0) * 1e3
    init_stats = g.last_stats()
    # C_t is written to a device buffer: the step stays in HBM end to end
    # (a host copy of C_t is a PCIe transfer, measured separately)
    c_out = torch.empty(n, dtype=torch.int32, device="cuda")
    for b in batches_dev[:warmup]:
        g.apply_batch(*b[:5], out=c_out)
    torch.cuda.synchronize()
    lat, qs, rs, evals, changes = [], [], [], 0, 0
    k_ms = k_bytes = k_launch = 0
    sweeps = 0
    ph_ms, ph_bytes = [0.0] * 4, [0] * 4
    t_start = time.perf_counter()
    for b in batches_dev[warmup:warmup + steps]:
        t = time.perf_counter()
        g.apply_batch(*b[:5], out=c_out)
        lat.append((time.perf_counter() - t) * 1e3)
        st = g.stats
        qs.append(st.q)
        rs.append(st.R_size / n)
        evals += st.vertex_evals
        changes += st.changes
        sweeps += st.sweeps
        k_ms += st.ms_sweep_kernel
        k_bytes += st.sweep_bytes
        k_launch += st.sweep_launches
        for k in range(4):
            ph_ms[k] += st.ms_phase[k]
            ph_bytes[k] += st.bytes_phase[k]
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t_start
    # the PCIe leg a host consumer of C_t adds per step (outside the timing)
    host = torch.empty(n, dtype=torch.int32)
    t = time.perf_counter()
    for _ in range(5):
        host.copy_(c_out)
    copy_ms = (time.perf_counter() - t) * 1e3 / 5
    out = dict(g=g, init_ms=init_ms, init_q=init_stats.q, lat=lat, q=qs, R_frac=rs,
               evals=evals, changes=changes, total_s=total_s, sweeps=sweeps,
               k_ms=k_ms, k_bytes=k_bytes, k_launch=k_launch, copy_ms=copy_ms,
               ph_ms=ph_ms, ph_bytes=ph_bytes)
    return out


PHASES = ("ingest and graph update", "screening (Alg. 2 and the deletion rule)",
          "level-0 sweeps (evaluate, apply, exact Delta N)",
          "compaction, levels >= 1, canonical labels")


def phase_table(r, steps):
    """Per phase of a step: device time (hipEvents), algorithmic bytes and
    the fraction of the 8 TB/s HBM peak they reach."""
    out = []
    for k, name in enumerate(PHASES):
        ms = r["ph_ms"][k] / steps
        b = r["ph_bytes"][k] / steps
        gbs = b / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        out.append({"phase": name, "ms_per_step": ms, "bytes_per_step": b,
                    "achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS})
    return out


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n, graph, batches, cpu_steps):
    """The oracle as it stands, single-threaded and pinned to one host core,
    on the first batches of the same stream, under Delta-screening and under
    the full recompute (each after its own static run, which is not timed)."""
    from oracle import oracle as O
    if not os.path.exists(O.LIB):
        O.build()
    u, v, w = graph
    prev = os.sched_getaffinity(0)
    core = min(prev)
    os.sched_setaffinity(0, {core})
    legs = {}
    try:
        for name, mode in (("delta", O.MODE_DELTA), ("all", O.MODE_ALL)):
            t0 = time.perf_counter()
            o = O.Oracle(n, u, v, w, mode=mode)
            init_s = time.perf_counter() - t0
            log(f"oracle {name}: static run {init_s:.1f} s")
            tot, ch = 0.0, 0
            for b in batches[:cpu_steps]:
                t = time.perf_counter()
                o.apply_batch(b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)
                tot += time.perf_counter() - t
                ch += b.size
                log(f"oracle {name}: step {time.perf_counter() - t:.1f} s")
            o.close()
            legs[name] = {"edge_updates_per_s": ch / tot, "seconds": tot, "changes": ch,
                          "static_run_s": init_s}
    finally:
        os.sched_setaffinity(0, prev)
    return {"value": legs["delta"]["edge_updates_per_s"], "unit": "edge updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"single-threaded oracle pinned to host core {core}, applying the first "
                      f"{cpu_steps} batches ({legs['delta']['changes']} changes) of the same "
                      f"stream after its own static run on G_1 (not counted); value = "
                      f"Delta-screening, full_recompute = mode ALL on the same batches",
            "full_recompute": legs["all"]["edge_updates_per_s"],
            "legs": legs, "cpu_model": _cpu_model(), "host_cores": os.cpu_count()}


def _serving_graph(args):
    """Worker: one serving graph's G_1 and its batches, written as .npy files
    into a shared-memory folder (the main process maps them)."""
    import numpy as np
    from paper_1904_08553_amd import workloads as W
    seed, batches, n_lo, n_hi, folder = args
    s = W.ServingStream(seed, n_lo=n_lo, n_hi=n_hi)
    u, v, w = s.graph()
    bs = [s.next_batch() for _ in range(batches)]
    cat = lambda f: np.concatenate([getattr(b, f) for b in bs]) if bs else np.empty(0, np.int32)
    parts = {"u": u, "v": v, "w": w, "au": cat("add_u"), "av": cat("add_v"), "aw": cat("add_w"),
             "du": cat("del_u"), "dv": cat("del_v"),
             "na": np.array([len(b.add_u) for b in bs], np.int64),
             "nd": np.array([len(b.del_u) for b in bs], np.int64)}
    for k, a in parts.items():
        np.save(os.path.join(folder, f"g{seed}_{k}.npy"), a)
    return seed, s.n


def _load_serving_graph(folder, seed, n):
    import numpy as np
    from paper_1904_08553_amd import workloads as W
    ld = lambda k: np.load(os.path.join(folder, f"g{seed}_{k}.npy"), mmap_mode="r")
    na, nd = ld("na"), ld("nd")
    ao = np.concatenate([[0], np.cumsum(na)])
    do = np.concatenate([[0], np.cumsum(nd)])
    au, av, aw, du, dv = ld("au"), ld("av"), ld("aw"), ld("du"), ld("dv")
    bs = [W.Batch(au[ao[j]:ao[j + 1]], av[ao[j]:ao[j + 1]], aw[ao[j]:ao[j + 1]],
                  du[do[j]:do[j + 1]], dv[do[j]:do[j + 1]]) for j in range(len(na))]
    return n, (ld("u"), ld("v"), ld("w")), bs


def serving_leg(graphs_k, arrivals, n_lo, n_hi, inflight, rate, warmup=None, budget_batches=600,
                seed=0, workers=16):
    """Many resident graphs behind one server (the serving workload: graphs_k
    DC-SBM graphs, n log-uniform in [n_lo, n_hi], 20 edges per vertex,
    batches of U[100K, 200K] changes, 60/40): closed-loop capacity one graph
    per round and merged, Poisson arrivals at `rate` per second for latency
    from arrival to C_t, and a run under a small memory budget (a quarter of
    the unlimited run's peak) for admission and eviction."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import shutil
    import tempfile
    import numpy as np
    from paper_1904_08553_amd import dc
    rng = np.random.default_rng(np.random.SeedSequence((seed, 77)))
    warmup = graphs_k if warmup is None else warmup
    total = warmup + arrivals
    # every graph gets one warm-up batch first (its buffers grow to their size),
    # then the timed arrivals pick a graph uniformly
    pick = np.concatenate([np.arange(graphs_k) % graphs_k if warmup == graphs_k
                           else rng.integers(0, graphs_k, size=warmup),
                           rng.integers(0, graphs_k, size=arrivals)])
    per = np.bincount(pick, minlength=graphs_k)
    t0 = time.perf_counter()
    folder = tempfile.mkdtemp(prefix="dc_serving_", dir="/dev/shm" if os.path.isdir("/dev/shm")
                              else None)
    try:
        jobs = [(1000 + g, int(per[g]), n_lo, n_hi, folder) for g in range(graphs_k)]
        with cf.ProcessPoolExecutor(max_workers=workers,
                                    mp_context=mp.get_context("spawn")) as ex:
            sizes = dict(ex.map(_serving_graph, jobs))
        graphs = [_load_serving_graph(folder, 1000 + g, sizes[1000 + g]) for g in range(graphs_k)]
        ns = np.array([g[0] for g in graphs])
        edges0 = int(sum(len(g[1][0]) for g in graphs))
        log(f"serving: {graphs_k} graphs ({ns.sum()} vertices, {edges0} edges), {total} batches "
            f"drawn in {time.perf_counter() - t0:.1f} s")
        order = []  # (graph, its batch index) in arrival order
        seen = [0] * graphs_k
        for g in pick:
            order.append((int(g), seen[g]))
            seen[g] += 1

        def run(max_inflight, gaps_ns, budget=0, count=None):
            srv = dc.Server(max_inflight=max_inflight, budget_bytes=budget)
            gids = [srv.add_graph(n, u, v, w) for n, (u, v, w), _ in graphs]
            events = order[:warmup + (arrivals if count is None else count)]
            # warm-up batches, then the timed ones
            for g, j in events[:warmup]:
                b = graphs[g][2][j]
                srv.poll(srv.submit(gids[g], b.add_u, b.add_v, b.add_w, b.del_u, b.del_v),
                         gids[g])
            st0 = srv.stats()
            base = time.monotonic_ns()
            tickets = []
            for (g, j), at in zip(events[warmup:], gaps_ns):
                due = base + int(at)
                while time.monotonic_ns() < due:
                    pass
                b = graphs[g][2][j]
                tickets.append((g, b.size, srv.submit(gids[g], b.add_u, b.add_v, b.add_w,
                                                      b.del_u, b.del_v, arrival_ns=due)))
            lat, changes, first, last = [], 0, None, 0
            for g, sz, tk in tickets:
                _, _, (arr, start, done) = srv.poll(tk, gids[g])
                lat.append((done - arr) / 1e6)
                changes += sz
                first = arr if first is None else min(first, arr)
                last = max(last, done)
            st = srv.stats()
            srv.close()
            span = (last - first) / 1e9
            rounds = st["rounds"] - st0["rounds"]
            return dict(batches=len(tickets), changes=changes,
                        edge_updates_per_s=changes / span, batches_per_s=len(tickets) / span,
                        latency_ms={"p50": percentile(lat, 50), "p99": percentile(lat, 99),
                                    "max": max(lat)},
                        seconds=span, rounds=rounds,
                        merged_rounds=st["merged_rounds"] - st0["merged_rounds"],
                        graphs_per_round=(st["merged_graphs"] - st0["merged_graphs"])
                        / max(rounds, 1),
                        evictions=st["evictions"], restores=st["restores"],
                        peak_resident_bytes=st["peak_resident_bytes"], budget_bytes=budget)

        zero = [0] * arrivals
        out = {"workload": f"{graphs_k} DC-SBM graphs, n log-uniform in [{n_lo}, {n_hi}] "
                           f"({int(ns.min())}..{int(ns.max())}, {int(ns.sum())} vertices, "
                           f"{edges0} edges), 20 edges per vertex; {arrivals} timed batches of "
                           f"U[100K, 200K] changes (60/40) after {warmup} warm-up batches, "
                           f"graph uniform per arrival",
               "closed_loop_sequential": run(1, zero),
               "closed_loop_merged": run(inflight, zero)}
        gaps = np.cumsum(rng.exponential(1e9 / rate, size=arrivals))
        poisson = run(inflight, gaps)
        poisson["arrival_rate_per_s"] = rate
        out["poisson"] = poisson
        budget = out["closed_loop_merged"]["peak_resident_bytes"] // 4
        out["small_budget"] = run(inflight, zero[:budget_batches], budget=budget,
                                  count=budget_batches)
        out["max_inflight"] = inflight
        out["merged_over_sequential"] = (out["closed_loop_merged"]["edge_updates_per_s"]
                                         / out["closed_loop_sequential"]["edge_updates_per_s"])
        return out
    finally:
        shutil.rmtree(folder, ignore_errors=True)


def temporal_leg(n, events, steps, blocks):
    """The paper-scale temporal stream: G_1 from step 1's events, then every
    later step as one batch, under Delta-screening and under full
    re-evaluation; whole-stream device-side time (generation excluded)."""
    import numpy as np
    import torch
    from paper_1904_08553_amd import dc, workloads as W
    t0 = time.perf_counter()
    (u, v, w), it = W.temporal_stream(n=n, events=events, steps=steps, blocks=blocks)
    batches = []
    for b in it:
        batches.append(b)
        log(f"temporal stream: batch {len(batches)} drawn ({time.perf_counter() - t0:.0f} s)")
    log(f"temporal stream: {len(u)} initial edges + {len(batches)} batches drawn in "
        f"{time.perf_counter() - t0:.0f} s")
    to_dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()
    out = {"workload": f"temporal stream: {n} vertices, {events} unit-weight events in {steps} "
                       f"steps (step 1 = G_1), 85% insertions / 15% deletions of earlier "
                       f"edges, 2% of the vertices change block per step, {blocks} blocks",
           "paper_context": "the paper reports 1056 s for its 63M-event stream over 12 steps on "
                            "its own hardware (not comparable hardware; context only)"}
    for name, mode in (("delta", dc.MODE_DELTA), ("all", dc.MODE_ALL)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        g = dc.DynamicCommunities(n, u, v, w, mode=mode)
        torch.cuda.synchronize()
        init_ms = (time.perf_counter() - t) * 1e3
        ms, q, R, ch = [], [], [], 0
        for b in batches:
            dev = [to_dev(x) for x in (b.add_u, b.add_v, b.add_w, b.del_u, b.del_v)]
            torch.cuda.synchronize()
            t = time.perf_counter()
            g.apply_batch(*dev)
            ms.append((time.perf_counter() - t) * 1e3)
            q.append(g.stats.q)
            R.append(g.stats.R_size / n)
            ch += b.size
        g.close()
        out[name] = {"init_ms": init_ms, "step_ms": ms, "stream_seconds": (init_ms + sum(ms)) / 1e3,
                     "edge_updates_per_s": ch / (sum(ms) / 1e3), "q": q, "R_frac": R}
        log(f"temporal {name}: {out[name]['stream_seconds']:.2f} s")
    out["speedup_delta_over_all"] = out["all"]["stream_seconds"] / out["delta"]["stream_seconds"]
    out["max_rel_q_diff"] = max(abs(a - b) / abs(b) for a, b in zip(out["delta"]["q"],
                                                                      out["all"]["q"]))
    return out


def learned_leg(seeds, workers=8):
    """Fresh graphs of the screener's workload under full re-evaluation,
    plain Delta-screening, Delta-screening with the cascade extension and the
    trained screener (committed weights)."""
    from paper_1904_08553_amd import screener as S
    w, theta, info = S.load()
    res = S.evaluate(seeds, w, theta, workers, modes=("all", "delta", "cascade", "learned"))
    out = S.summarize(res)
    out["workload"] = ("planted partition, 100-vertex blocks, n log-uniform in [100K, 1M], 4 "
                       "batches of 7.3% insertions / 2.9% deletions; fresh seeds "
                       f"{seeds[0]}..{seeds[-1]}")
    out["theta"] = theta
    out["training"] = {k: info.get(k) for k in ("train_graphs", "train_samples", "epochs",
                                                "val_recall", "val_selected_frac", "train_s")}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--m", type=int, default=20_000_000)
    ap.add_argument("--blocks", type=int, default=1000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-full", action="store_true", help="skip the full-recompute replay")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-screener leg")
    ap.add_argument("--learned-seeds", type=int, default=20)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-cascade", action="store_true",
                    help="skip the cascade-aware screening replay of the main batches")
    ap.add_argument("--no-slm", action="store_true",
                    help="skip the dSLM-DS / dSLM-base replay of the main batches")
    ap.add_argument("--serving-graphs", type=int, default=64)
    ap.add_argument("--serving-batches", type=int, default=5000)
    ap.add_argument("--serving-nmax", type=int, default=2_000_000)
    ap.add_argument("--serving-inflight", type=int, default=8)
    ap.add_argument("--serving-rate", type=float, default=500.0,
                    help="Poisson arrivals per second of the serving leg")
    ap.add_argument("--temporal", action="store_true",
                    help="also run the paper-scale temporal stream (minutes of host time)")
    ap.add_argument("--temporal-n", type=int, default=8_000_000)
    ap.add_argument("--temporal-events", type=int, default=63_000_000)
    ap.add_argument("--resolution", action="store_true",
                    help="also run the temporal-resolution study (cuts of the temporal "
                         "stream into 2..28 steps; minutes of host time)")
    ap.add_argument("--resolution-n", type=int, default=8_000_000)
    ap.add_argument("--resolution-events", type=int, default=63_000_000)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="also run three plain device-to-device copies of BYTES bytes (a "
                         "reference kernel of known traffic for hardware byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: runs on exactly one GPU (the method is measured on one MI355X; "
              "multi-GPU sharding is not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1904_08553_amd import dc, workloads as W

    torch.cuda.set_device(0)
    if args.calibrate_copy > 0:
        src = torch.empty(args.calibrate_copy, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration: 3 device copies of {args.calibrate_copy} bytes")
        del src, dst
    t0 = time.perf_counter()
    gen = W.DCSBM(n=args.n, m=args.m, blocks=args.blocks, seed=args.seed)
    graph, it = gen.stream(args.warmup + args.steps, frac=0.01, ins_frac=0.6)
    log(f"graph {len(graph[0])} edges in {time.perf_counter() - t0:.1f} s")
    batches = []
    for b in it:
        batches.append(b)
    log(f"{len(batches)} batches in {time.perf_counter() - t0:.1f} s")
    to_dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()
    batches_dev = [(to_dev(b.add_u), to_dev(b.add_v), to_dev(b.add_w), to_dev(b.del_u),
                    to_dev(b.del_v)) for b in batches]
    torch.cuda.synchronize()

    log("delta-screening run")
    d = run_mode(dc.MODE_DELTA, args.n, graph, batches_dev, args.warmup, args.steps, 1)
    res_full = None
    if not args.no_full:
        d["g"].close()
        log("full-recompute run")
        res_full = run_mode(dc.MODE_ALL, args.n, graph, batches_dev, args.warmup, args.steps, 1)
        res_full["g"].close()
    else:
        d["g"].close()

    res_casc = None
    if not args.no_cascade:
        log("cascade-aware screening run")
        res_casc = run_mode(dc.MODE_DELTA, args.n, graph, batches_dev, args.warmup, args.steps, 0,
                            cascade=(1, 20))
        res_casc["g"].close()

    res_slm = None
    if not args.no_slm:
        # dSLM-DS and dSLM-base (Sec. 3.4): the same batches with smart local
        # moving levels, from R_t and from every vertex
        log("dSLM runs")
        res_slm = {}
        for name, mode in (("delta", dc.MODE_DELTA), ("base", dc.MODE_ALL)):
            res_slm[name] = run_mode(mode, args.n, graph, batches_dev, args.warmup, args.steps,
                                     0, algorithm=dc.ALGO_SLM)
            res_slm[name]["g"].close()

    value = d["changes"] / d["total_s"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "edge updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": d["total_s"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {
            "workload": f"dcsbm_n{args.n}_m{args.m}_batch1pct_ins60_del40",
            "n": args.n, "edges": args.m, "blocks": args.blocks, "degree_law": "2.3 on [4,5000]",
            "weights": "int32 in [1,8]", "batch_frac": 0.01, "seed": args.seed,
            "parallelism": "single GPU",
        },
        "latency_ms": {"p50": percentile(d["lat"], 50), "p99": percentile(d["lat"], 99),
                       "max": max(d["lat"])},
        "vertex_gain_evals_per_s": d["evals"] / d["total_s"],
        "R_frac_mean": float(np.mean(d["R_frac"])),
        "sweeps_per_step": d["sweeps"] / args.steps,
        "init_ms": d["init_ms"],
        "pcie_inclusive": {"c_t_to_host_ms": d["copy_ms"],
                           "edge_updates_per_s": d["changes"] / (d["total_s"]
                                                                 + args.steps * d["copy_ms"] / 1e3)},
        "q_delta": d["q"],
    }
    if res_full is not None:
        f = res_full
        rel = [abs(a - b) / abs(b) for a, b in zip(d["q"], f["q"])]
        out["full_recompute"] = {
            "value": f["changes"] / f["total_s"],
            "ms_per_step": f["total_s"] * 1e3 / args.steps,
            "latency_ms": {"p50": percentile(f["lat"], 50), "p99": percentile(f["lat"], 99)},
            "q_full": f["q"],
            "speedup_delta_over_full": f["total_s"] / d["total_s"],
            "max_rel_q_diff": max(rel),
            "matched_modularity_within_0.1pct": bool(max(rel) <= 1e-3),
        }
    if res_casc is not None:
        cz = res_casc
        out["cascade"] = {
            "theta": [1, 20],
            "value": cz["changes"] / cz["total_s"],
            "ms_per_step": cz["total_s"] * 1e3 / args.steps,
            "R_frac_mean": float(np.mean(cz["R_frac"])),
            "q": cz["q"],
            "max_rel_q_diff_vs_delta": max(abs(a - b) / abs(b) for a, b in zip(cz["q"], d["q"])),
        }
    if res_slm is not None:
        sd, sb = res_slm["delta"], res_slm["base"]
        out["slm"] = {
            "delta": {"value": sd["changes"] / sd["total_s"],
                      "ms_per_step": sd["total_s"] * 1e3 / args.steps, "q": sd["q"],
                      "R_frac_mean": float(np.mean(sd["R_frac"])), "init_ms": sd["init_ms"],
                      "sweeps_per_step": sd["sweeps"] / args.steps},
            "base": {"value": sb["changes"] / sb["total_s"],
                     "ms_per_step": sb["total_s"] * 1e3 / args.steps, "q": sb["q"],
                     "init_ms": sb["init_ms"], "sweeps_per_step": sb["sweeps"] / args.steps},
            "speedup_delta_over_base": sb["total_s"] / sd["total_s"],
            "max_rel_q_diff": max(abs(a - b) / abs(b) for a, b in zip(sd["q"], sb["q"])),
            "mean_q_vs_louvain_delta": float(np.mean(sd["q"]) - np.mean(d["q"])),
        }
    if d["k_launch"] > 0 and d["k_ms"] > 0:
        ach = d["k_bytes"] / (d["k_ms"] * 1e-3) / 1e9
        out["roofline"] = {
            "kernel": "k_eval_groups<0> (level-0/1+ sweeps, rows of at most 64 entries: "
                      "the bins of 16, 32 and 64 lanes per vertex in one launch)",
            "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": measured_traffic(),
            "launches": d["k_launch"], "avg_launch_us": d["k_ms"] * 1e3 / d["k_launch"],
            "bytes_per_launch": d["k_bytes"] / d["k_launch"],
            "instruction_issue": measured_issue(),
            "phases_delta": phase_table(d, args.steps),
        }
        if res_full is not None:
            out["roofline"]["phases_full"] = phase_table(res_full, args.steps)
    if not args.no_learned:
        log("learned-screener leg")
        out["learned"] = learned_leg(list(range(10000, 10000 + args.learned_seeds)))
    if not args.no_serving:
        log("serving leg")
        out["serving"] = serving_leg(args.serving_graphs, args.serving_batches, 10_000,
                                     args.serving_nmax, args.serving_inflight, args.serving_rate)
    if args.temporal:
        log("temporal-stream leg")
        out["temporal"] = temporal_leg(args.temporal_n, args.temporal_events, 12,
                                       max(10, args.temporal_n // 1000))
    if args.resolution:
        log("temporal-resolution leg")
        from paper_1904_08553_amd import resolution as RS
        t0 = time.perf_counter()
        stream = W.temporal_events(n=args.resolution_n, events=args.resolution_events,
                                   blocks=max(10, args.resolution_n // 1000))
        log(f"resolution: {len(stream)} events drawn in {time.perf_counter() - t0:.0f} s")
        out["resolution"] = {
            "workload": f"temporal stream of {args.resolution_events} unit-weight events over "
                        f"{args.resolution_n} vertices, cut into K equal-count steps",
            "rows": RS.study(stream)}
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(args.n, graph, batches, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
