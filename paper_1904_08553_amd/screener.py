"""Training, calibration and evaluation of the learned screener.

The screener (an extension; the paper has no learned component) scores the
vertices a batch touches from eight exact-integer features and lets LEARNED
mode run level 0 over the touched vertices whose logit clears a threshold
theta instead of the Delta-screening set R_t.  Everything here is plumbing
around libdc.so: samples come from its collect mode (move labels from a full
re-evaluation of level 0, bit-exact with the CPU oracle's), and the network
is trained by its BF16 matrix-core forward/backward kernels and Adam
(dc.MLP).  torch serves as device memory (sample storage, shuffling by
index) only.

Workload: planted-partition graphs with 100-vertex blocks, n log-uniform in
[100K, 1M], four batches of 7.3% insertions (70% intra-community) and 2.9%
deletions (workloads.screener_graph); graphs of seeds 0..179 train, 180..199
calibrate theta (the largest threshold whose worst calibration batch stays
within 0.08% of the full recompute's modularity, from the thresholds keeping
0.99 ... 1 of the move labels), fresh seeds from 10000 evaluate.

    python -m paper_1904_08553_amd.screener train   # writes screener_weights.json
    python -m paper_1904_08553_amd.screener eval    # LEARNED vs plain Delta-screening
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

from . import dc
from . import workloads as W

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "screener_weights.json")
IN, HID, NPARAM = dc.MLP_INPUTS, dc.MLP_HIDDEN, dc.MLP_PARAMS


def log(msg):
    print(f"[screener] {msg}", file=sys.stderr, flush=True)


def init_weights(seed: int) -> np.ndarray:
    """He-uniform hidden layers, a small output layer, zero biases."""
    rng = np.random.default_rng(np.random.SeedSequence((seed, 0xA11CE)))
    w = np.zeros(NPARAM, np.float64)
    o1 = HID * IN
    o2 = o1 + HID
    o3 = o2 + HID * HID
    o4 = o3 + HID
    w[:o1] = rng.uniform(-1, 1, o1) * np.sqrt(6.0 / IN)
    w[o2:o3] = rng.uniform(-1, 1, HID * HID) * np.sqrt(6.0 / HID)
    w[o4:o4 + HID] = rng.uniform(-1, 1, HID) * np.sqrt(1.0 / HID)
    return w.astype(np.float32)


def _graph(seed, n=None):
    return W.screener_graph(seed, n=n)


def graphs(seeds, workers, n=None):
    """Yields (seed, n, graph, batches) in seed order; drawn by worker
    processes (numpy only, no GPU) ahead of the consumer.  n: fixed vertex
    count instead of the log-uniform draw."""
    if workers <= 1:
        for s in seeds:
            yield (s,) + W.screener_graph(s, n=n)
        return
    ctx = mp.get_context("spawn")
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        futs = [ex.submit(_graph, s, n) for s in seeds]
        for s, f in zip(seeds, futs):
            yield (s,) + f.result()


def _dev_batches(batches):
    import torch
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()
    return [(d(b.add_u), d(b.add_v), d(b.add_w), d(b.del_u), d(b.del_v)) for b in batches]


def collect(seeds, workers=8, n=None):
    """Samples of every batch of the given graphs (device tensors X int16
    [N, 8] of bfloat16 bits and y uint8 [N]) and per-graph counts."""
    import torch
    Xs, ys, meta = [], [], []
    t0 = time.perf_counter()
    for s, nv, (u, v, w), batches in graphs(seeds, workers, n):
        g = dc.DynamicCommunities(nv, u, v, w, mode=dc.MODE_DELTA, collect=1)
        cnt = pos = 0
        for b in _dev_batches(batches):
            g.apply_batch(*b)
            smp = g.samples(device=True)
            Xs.append(smp["X"].clone())
            ys.append(smp["y"].clone())
            cnt += smp["y"].numel()
            pos += int(smp["y"].sum().item())
        g.close()
        meta.append(dict(seed=s, n=nv, edges=len(u), samples=cnt, positives=pos))
        log(f"graph {s}: n={nv} samples={cnt} positives={pos} ({time.perf_counter() - t0:.0f} s)")
    return torch.cat(Xs), torch.cat(ys), meta


def train(X, y, epochs=3, batch=8192, lr=1e-3, pos_weight=None, seed=0):
    """Adam on the mean weighted BCE with the library's kernels; returns the
    network and the loss curve (one mean per epoch)."""
    import torch
    N = y.numel()
    npos = int(y.sum().item())
    if pos_weight is None:
        pos_weight = float(np.sqrt(max(N - npos, 1) / max(npos, 1)))
    net = dc.MLP(init_weights(seed))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    curve = []
    for ep in range(epochs):
        perm = torch.randperm(N, device="cuda", generator=gen)
        tot, cnt = 0.0, 0
        for i in range(0, N, batch):
            idx = perm[i:i + batch]
            want = (i // batch) % 64 == 0
            loss = net.train_step(X[idx].contiguous(), y[idx].contiguous(), pos_weight, lr,
                                  want_loss=want)
            if want:
                tot += loss
                cnt += 1
        curve.append(tot / max(cnt, 1))
        log(f"epoch {ep}: sampled loss {curve[-1]:.4f}")
    return net, curve, pos_weight


def logits(net, X, chunk=1 << 22):
    import torch
    return torch.cat([net.forward(X[i:i + chunk].contiguous()) for i in range(0, X.shape[0], chunk)])


def threshold_for_recall(z, y, recall):
    """Largest theta with {z >= theta} holding at least `recall` of the
    positives."""
    z = np.asarray(z, np.float64)
    pos = np.sort(z[np.asarray(y) != 0])
    if len(pos) == 0:
        return float("-inf")
    drop = int(np.floor((1.0 - recall) * len(pos) + 1e-9))
    return float(np.float32(pos[drop]))


def calibrate_theta(w, z, y, seeds, workers=8, bar=1e-3, margin=0.8,
                    recalls=(0.99, 0.995, 0.999, 0.9995, 0.9999, 1.0)):
    """theta for LEARNED mode on the calibration graphs: candidates are the
    thresholds keeping each recall of the move labels (logits z, labels y of
    the calibration samples), from the fewest vertices up; the first whose
    worst batch loses at most margin * bar of ALL's modularity (relative) is
    taken.  Returns theta and the curve (theta, recall, selected fraction,
    worst and mean relative modularity change against ALL)."""
    pregen = list(graphs(seeds, workers))
    qa = np.asarray(evaluate(seeds, w, 0.0, workers, modes=("all",), pregen=pregen)["all"]["q"])
    curve, chosen = [], None
    for r in recalls:
        th = threshold_for_recall(z, y, r) if r < 1.0 else float(np.min(z))
        ql = np.asarray(evaluate(seeds, w, th, workers, modes=("learned",),
                                 pregen=pregen)["learned"]["q"])
        rel = (ql - qa) / np.abs(qa)
        sel = z >= th
        row = dict(theta=th, recall=float((sel & (y != 0)).sum() / max(int((y != 0).sum()), 1)),
                   selected_frac=float(sel.mean()), worst_rel_q=float(rel.min()),
                   mean_rel_q=float(rel.mean()))
        curve.append(row)
        log(f"calibration: {row}")
        if chosen is None and row["worst_rel_q"] >= -margin * bar:
            chosen = th
    if chosen is None:
        chosen = curve[-1]["theta"]
    return chosen, curve


def save(w, theta, info, path=WEIGHTS):
    with open(path, "w") as f:
        json.dump(dict(theta=theta, weights=[float(x) for x in w], info=info), f)


def load(path=WEIGHTS):
    d = json.load(open(path))
    w = np.asarray(d["weights"], np.float32)
    if w.size != NPARAM:
        raise ValueError(f"{path}: expected {NPARAM} parameters")
    return w, float(d["theta"]), d.get("info", {})


CASCADE = (1, 20)  # theta of the cascade-aware screening compared here


def evaluate(seeds, w, theta, workers=8, modes=("all", "delta", "learned"), n=None,
             pregen=None):
    """Each graph's four batches under full re-evaluation (ALL), plain
    Delta-screening, Delta-screening with the cascade extension (mode
    "cascade", threshold CASCADE) and LEARNED; per mode the batch times (each
    call returns after C_t is written to a device buffer, inputs resident),
    changes, Q per batch, level-0 evaluations."""
    import torch
    code = {"all": dc.MODE_ALL, "delta": dc.MODE_DELTA, "cascade": dc.MODE_DELTA,
            "learned": dc.MODE_LEARNED}
    out = {m: dict(ms=[], bi=[], changes=0, q=[], level0=0, R=0, touched=0) for m in modes}
    src = pregen if pregen is not None else graphs(seeds, workers, n)
    for s, nn, (u, v, w_), batches in src:
        dev = _dev_batches(batches)
        out_C = torch.empty(nn, dtype=torch.int32, device="cuda")  # C_t stays in HBM
        for m in modes:
            extra = {"cascade": CASCADE} if m == "cascade" else {}
            g = dc.DynamicCommunities(nn, u, v, w_, mode=code[m], **extra)
            if m == "learned":
                g.set_screener(w, theta)
            torch.cuda.synchronize()
            for i, (b, hb) in enumerate(zip(dev, batches)):
                t = time.perf_counter()
                g.apply_batch(*b, out=out_C)
                out[m]["ms"].append((time.perf_counter() - t) * 1e3)
                out[m]["bi"].append(i)
                st = g.stats
                out[m]["changes"] += hb.size
                out[m]["q"].append(st.q)
                out[m]["level0"] += st.level0_active
                out[m]["R"] += st.R_size
                out[m]["touched"] += st.touched
            g.close()
        log(f"eval graph {s}: n={nn}")
    return out


def summarize(res):
    s = {}
    qa = np.asarray(res["all"]["q"]) if "all" in res else None
    for m, r in res.items():
        t = sum(r["ms"]) / 1e3
        ms = np.asarray(r["ms"])
        later = ms[np.asarray(r["bi"]) > 0]
        # each graph's first batch also sets up its new context (buffers
        # taken from the allocator); the later batches and the median show
        # the steady state without it or single slow batches
        d = dict(edge_updates_per_s=r["changes"] / t, ms_per_batch=float(ms.mean()),
                 ms_per_batch_median=float(np.median(ms)),
                 ms_per_later_batch=float(later.mean()) if later.size else None,
                 level0_evals=r["level0"], R_total=r["R"])
        if qa is not None:
            rel = (np.asarray(r["q"]) - qa) / np.abs(qa)
            d["rel_q_vs_all_mean"] = float(rel.mean())
            d["rel_q_vs_all_min"] = float(rel.min())
        s[m] = d
    if "delta" in s and "learned" in s:
        s["learned_speedup_over_delta"] = (s["learned"]["edge_updates_per_s"]
                                           / s["delta"]["edge_updates_per_s"])
        s["learned_speedup_over_delta_median"] = (s["delta"]["ms_per_batch_median"]
                                                  / s["learned"]["ms_per_batch_median"])
        if s["learned"]["ms_per_later_batch"]:
            s["learned_speedup_over_delta_later"] = (s["delta"]["ms_per_later_batch"]
                                                     / s["learned"]["ms_per_later_batch"])
    if "delta" in s and "cascade" in s:
        s["cascade_speedup_over_delta"] = (s["cascade"]["edge_updates_per_s"]
                                           / s["delta"]["edge_updates_per_s"])
        s["cascade_theta"] = list(CASCADE)
    return s


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("cmd", choices=["train", "eval"])
    ap.add_argument("--train-graphs", type=int, default=180)
    ap.add_argument("--val-graphs", type=int, default=20)
    ap.add_argument("--eval-seeds", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=3)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--recall", type=float, default=0.99)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--out", default=WEIGHTS)
    a = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    if a.cmd == "train":
        t0 = time.perf_counter()
        tr = list(range(a.train_graphs))
        va = list(range(a.train_graphs, a.train_graphs + a.val_graphs))
        X, y, meta = collect(tr, a.workers)
        t_col = time.perf_counter() - t0
        log(f"training samples {y.numel()} positives {int(y.sum().item())} in {t_col:.0f} s")
        t1 = time.perf_counter()
        net, curve, pw = train(X, y, a.epochs, a.batch, a.lr)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t1
        del X, y
        Xv, yv, vmeta = collect(va, a.workers)
        z = logits(net, Xv).cpu().numpy()
        yv_h = yv.cpu().numpy()
        theta, curve_theta = calibrate_theta(net.weights(), z, yv_h, va, a.workers)
        sel = z >= theta
        info = dict(train_graphs=a.train_graphs, val_graphs=a.val_graphs, epochs=a.epochs,
                    batch=a.batch, lr=a.lr, pos_weight=pw, recall_target=a.recall,
                    loss_curve=curve, collect_s=t_col, train_s=t_train,
                    train_samples=int(sum(m["samples"] for m in meta)),
                    val_samples=int(yv_h.size), val_positives=int(yv_h.sum()),
                    val_recall=float((sel & (yv_h != 0)).sum() / max(int(yv_h.sum()), 1)),
                    val_selected_frac=float(sel.mean()), theta_curve=curve_theta,
                    theta_rule="largest theta whose worst calibration batch loses at most "
                               "0.8e-3 of ALL's modularity")
        save(net.weights(), theta, info, a.out)
        log(json.dumps(info))
        print(json.dumps(dict(theta=theta, **info)))
    else:
        w, theta, _ = load(a.out)
        res = evaluate(list(range(10000, 10000 + a.eval_seeds)), w, theta, a.workers)
        print(json.dumps(summarize(res)))


if __name__ == "__main__":
    main()
