// api.hip -- the C ABI of dc.h: context, dc_init, dc_apply_batch and queries.
//
// dc_init runs Static(G_1) (Sec. 3.4 step 1).  dc_apply_batch runs one time
// step (Sec. 3.4 step 2): the batch is validated in full before anything is
// changed, merged into the CSR, R_t is chosen (Alg. 2 plus the deletion rule
// for DELTA, all vertices for ALL and STATIC), and the levels of Alg. 1 run
// with level 0 restricted to R_t.  All work goes to the caller's stream; the
// host waits only where a size or a convergence decision is needed.
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.h"

using namespace dc;

namespace dc_core {

thread_local std::string g_last_error;

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

dc_status map_device_error(const DeviceError& e) {
  g_last_error = e.what();
  return (e.code == hipErrorOutOfMemory || e.code == hipErrorMemoryAllocation) ? DC_E_OOM
                                                                              : DC_E_DEVICE;
}

bool options_ok(const dc_options* o) {
  if (!o) return false;
  if (o->mode < DC_MODE_DELTA || o->mode > DC_MODE_LEARNED) return false;
  if (o->collect != 0 && o->collect != 1) return false;
  if (o->full_coarsen != 0 && o->full_coarsen != 1) return false;
  if (o->max_levels < 1 || o->max_sweeps < 1) return false;
  if (o->del_rule != DC_DEL_GAIN && o->del_rule != DC_DEL_CONSERVATIVE) return false;
  if (o->tau_den < 0) return false;
  if (o->cascade_num < 0 || o->cascade_den < 0) return false;
  if (o->algorithm != DC_ALGO_LOUVAIN && o->algorithm != DC_ALGO_SLM) return false;
  if (o->reserved != 0) return false;
  return true;
}

// Copies an edge list to the device when it lives on the host.
void stage_edges(dc_ctx* c, const dc_edges* e, bool weights, DBuf& bu, DBuf& bv, DBuf& bw,
                 const int32_t** u, const int32_t** v, const int32_t** w) {
  *u = *v = *w = nullptr;
  if (!e || e->count <= 0) return;
  size_t bytes = size_t(e->count) * 4;
  if (e->on_device) {
    *u = e->u;
    *v = e->v;
    *w = weights ? e->w : nullptr;
    return;
  }
  bu.ensure(bytes);
  bv.ensure(bytes);
  DC_HIP(hipMemcpyAsync(bu.p, e->u, bytes, hipMemcpyHostToDevice, c->st));
  DC_HIP(hipMemcpyAsync(bv.p, e->v, bytes, hipMemcpyHostToDevice, c->st));
  *u = bu.as<int32_t>();
  *v = bv.as<int32_t>();
  if (weights) {
    bw.ensure(bytes);
    DC_HIP(hipMemcpyAsync(bw.p, e->w, bytes, hipMemcpyHostToDevice, c->st));
    *w = bw.as<int32_t>();
  }
}

void ensure_vertex_state(dc_ctx* c) {
  size_t n = size_t(c->n);
  for (DBuf* b : {&c->k0, &c->C, &c->a0, &c->sz0, &c->Cl, &c->Cn, &c->al, &c->szl, &c->lflag,
                  &c->tlist, &c->movers, &c->map0, &c->cnt[0], &c->cnt[1], &c->minv[0],
                  &c->minv[1], &c->lab, &c->cntf, &c->dflag, &c->dpos, &c->dlist, &c->rflag,
                  &c->rpos2, &c->Rlist, &c->seg_beg, &c->seg_end})
    b->ensure((n + 1) * 4);
  c->dpack.ensure((n + 1) * 8);
  c->R.ensure(n + 1);
  c->cflag.ensure(n + 1);
  c->stat.ensure(ST_COUNT * 8);
  DC_HIP(hipMemsetAsync(c->stat.p, 0, ST_COUNT * 8, c->st));  // counters and self-check flags
  c->done.ensure(DONE_WORDS * 4);
  DC_HIP(hipMemsetAsync(c->done.p, 0, DONE_WORDS * 4, c->st));
  fill_i64(c->dpack.as<int64_t>(), 0, int64_t(n) + 1, c->st);
  fill_i32(c->lflag.as<int32_t>(), 0, int64_t(n) + 1, c->st);
}

void ensure_sample_state(dc_ctx* c) {
  size_t n = size_t(c->n) + 1;
  for (DBuf* b : {&c->kprev, &c->tflag, &c->tpos, &c->Tlist, &c->f_own, &c->logits})
    b->ensure(n * 4);
  c->f_g1.ensure(n * 8);
  c->f_g2.ensure(n * 8);
  c->tmark.ensure(n);
  c->y.ensure(n);
  c->X.ensure(n * 16);
}

// Phase boundary k of a timed step (see dc_step_stats.ms_phase).
void mark_phase(dc_ctx* c, int k) {
  if (c->phase_timing) DC_HIP(hipEventRecord(c->evp[k], c->st));
}

// Raises when a kernel's self-check failed (the context is then poisoned).
void check_stat_errors(const long long* h) {
  if (h[ST_ERR] & 1) throw std::runtime_error("hub-row hash tables larger than their buffer");
}

void screening_counts(dc_ctx* c);

void read_stat(dc_ctx* c) {
  DC_HIP(hipMemcpyAsync(c->hstat, c->stat.p, ST_COUNT * 8, hipMemcpyDeviceToHost, c->st));
  DC_HIP(hipStreamSynchronize(c->st));
  check_stat_errors(c->hstat);
}

// Bookkeeping of one finished sweep whose status block is in c->hstat: the
// trace record and statistics (record), the level's gain, and whether the
// level stops (no move, a reverted sweep, a gain of at most T, or the sweep
// limit).  timed_ms >= 0: device time of the timed launch of this sweep.
bool sweep_account(dc_ctx* c, const LevelView& g, int level, int s, const Bins& bins,
                   long long T, bool record, float timed_ms, long long& level_gain,
                   int64_t n_active = -1, int32_t phase = 0) {
  const long long moves = c->hstat[ST_MOVES], dN = c->hstat[ST_DN];
  if (record) {
    dc_step_stats& S = c->stats;
    int64_t n_eval = 0;
    long long vol_eval = 0;
    for (int q = 0; q < NBINS; ++q) {
      n_eval += bins.n[q];
      vol_eval += bins.vol[q];
    }
    if (timed_ms >= 0.f) {
      S.ms_sweep_kernel += timed_ms;
      S.sweep_launches += 1;
      // algorithmic bytes of the timed launch: 12 B per adjacency entry
      // (8 B entry + 4 B neighbour label) and 32 B per evaluated vertex
      // (two offsets, label, degree, own total and size, best total, result)
      for (int q = 0; q < TIMED_BINS; ++q) S.sweep_bytes += 12 * bins.vol[q] + 32 * bins.n[q];
    }
    dc_sweep_rec r{};
    r.level = level;
    r.sweep = s;
    r.n_level = g.n;
    r.n_active = int32_t(n_active >= 0 ? n_active : n_eval);
    r.nnz_level = g.nnz;
    r.moves = moves;
    r.dN = dN;
    r.kept = int32_t(c->hstat[ST_KEEP]);
    r.phase = phase;
    c->trace.push_back(r);
    S.vertex_evals += n_eval;
    if (level == 0 && phase == 0) {
      S.level0_sweeps += 1;
      S.level0_active += n_eval;
      S.level0_volume += vol_eval;
    }
    if (moves > 0 && dN >= 0) S.moves += moves;
  }
  if (moves == 0 || dN < 0) return true;
  level_gain += dN;
  return dN <= T || s + 1 >= c->opt.max_sweeps;
}

// Synchronous sweeps of one level over the binned active set (Alg. 1 inner
// loop); returns the level's total exact gain.  record: trace records,
// statistics and timing of the call.  pre_done: the first sweep evaluates
// only the first parts of the bins (the active vertices whose first-sweep
// labels are already in Cn are binned last); later sweeps take whole bins.
long long run_sweeps(dc_ctx* c, const LevelView& g, const int32_t* act, int64_t nact,
                     const Bins& all_bins, int level, long long T, bool record,
                     bool pre_done = false, int32_t phase = 0) {
  hipStream_t st = c->st;
  long long level_gain = 0;
  Bins bins = pre_done ? first_part(all_bins) : all_bins;
  for (int s = 0; s < c->opt.max_sweeps; ++s) {
    if (s == 1) bins = all_bins;
    if (s == 0) sweep_reset(c->stat.as<long long>(), st);  // later: cleared by sweep_apply
    const bool timed = record && c->opt.timing && bins.n[0] + bins.n[1] + bins.n[2] > 0;
    sweep_eval(g, c->Cl.as<int32_t>(), c->Cn.as<int32_t>(), c->al.as<int32_t>(),
               c->szl.as<int32_t>(), c->two_m, c->opt.singleton_guard, bins,
               c->stat.as<long long>(), st, timed ? c->ev0 : nullptr,
               timed ? c->ev1 : nullptr);
    sweep_apply(g, act, nact, c->Cl.as<int32_t>(), c->Cn.as<int32_t>(), c->al.as<int32_t>(),
                c->szl.as<int32_t>(), c->two_m, c->movers.as<int32_t>(),
                c->dpack.as<long long>(), c->lflag.as<int32_t>(), c->tlist.as<int32_t>(),
                c->stat.as<long long>(), c->done.as<unsigned>(), c->hstat_dev, st);
    // the status block reaches c->hstat from the sweep's last kernel
    DC_HIP(hipStreamSynchronize(st));
    check_stat_errors(c->hstat);
    float ms = -1.f;
    if (timed) DC_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    if (sweep_account(c, g, level, s, bins, T, record, ms, level_gain, nact, phase)) break;
  }
  return level_gain;
}

// Alg. 1 in two parts around the level-0 sweeps, so that several graphs can
// run their level-0 sweeps together: levels_begin bins R_t for level 0
// (null = every vertex) over the level-0 partition (Cl, al, szl) the caller
// prepared; levels_finish coarsens, runs the upper levels and writes the
// canonical labels, the totals and N.

void levels_begin(dc_ctx* c, const int32_t* active, int64_t n_active, LevelRun& L,
                  const uint8_t* skip) {
  c->pre_count = 0;  // the screening's first-sweep labels serve run_levels only
  const long long two_m = c->two_m;
  L.T = c->opt.tau_den > 0 ? (two_m * two_m) / c->opt.tau_den : 0;
  L.g = LevelView{c->n, c->nnz, c->off[c->cur].as<int32_t>(), c->adj[c->cur].as<int2>(),
                  c->k0.as<int32_t>()};
  L.act = active;
  L.nact = n_active;
  c->trace.clear();
  if (active && c->R_dcount) {
    // R_t from the screening pass: binned by its device length, which comes
    // back with the binning's wait together with the screening counters
    make_bins(active, n_active, L.g.off, L.bins, c->bins, c->st, skip, c->R_dcount,
              c->stat.as<long long>(), c->hstat_dev, ST_COUNT);
    check_stat_errors(c->hstat);
    c->R_dcount = nullptr;
    c->R_count = L.bins.total;
    L.nact = L.bins.total;
    screening_counts(c);
    return;
  }
  make_bins(active, n_active, L.g.off, L.bins, c->bins, c->st, skip);
}

void levels_finish(dc_ctx* c, LevelRun& L, long long level0_gain) {
  hipStream_t st = c->st;
  const long long two_m = c->two_m;
  const long long T = L.T;
  LevelView g = L.g;
  int32_t* Cl = c->Cl.as<int32_t>();
  int32_t* Cn = c->Cn.as<int32_t>();
  int32_t* al = c->al.as<int32_t>();
  int32_t* szl = c->szl.as<int32_t>();
  dc_step_stats& S = c->stats;
  int level = 0;
  long long level_gain = level0_gain;
  while (true) {
    if (level > 0) {
      Bins bins;
      make_bins(nullptr, g.n, g.off, bins, c->bins, st, nullptr, nullptr, nullptr, nullptr, 0,
                true);
      inc_check(c->cs);
      level_gain = run_sweeps(c, g, nullptr, g.n, bins, level, T, true);
    }
    const bool stop = (level + 1 >= c->opt.max_levels) || (level >= 1 && level_gain <= T);
    if (stop && level >= 1) break;
    // coarsen (after level 0 always: it also yields the canonical labels)
    const int next = level % 2;
    const int32_t* cnt_in = level == 0 ? nullptr : c->cnt[(level - 1) % 2].as<int32_t>();
    const int32_t* minv_in = level == 0 ? nullptr : c->minv[(level - 1) % 2].as<int32_t>();
    const bool inc = level == 0 && c->inc.valid && c->inc_ready &&
                     c->opt.mode != DC_MODE_STATIC && !c->opt.full_coarsen;
    if (inc)
      coarsen_first_inc(g, Cl, c->C.as<int32_t>(), szl, al, c->ch_key.as<uint64_t>(),
                        c->ch_dk.as<int32_t>(), c->nch_last, c->map0.as<int32_t>(), c->cg[next],
                        c->cnt[next].as<int32_t>(), c->minv[next].as<int32_t>(), c->cs, c->inc,
                        st);
    else
      coarsen(g, Cl, szl, al, cnt_in, minv_in, level == 0, c->n, c->map0.as<int32_t>(),
              c->cg[next], c->cnt[next].as<int32_t>(), c->minv[next].as<int32_t>(), c->cs, st);
    if (level == 0 && !inc)
      save_level1(c->cg[next], c->cs, c->minv[next].as<int32_t>(), c->inc, st);
    g = c->cg[next].view();
    start_level(Cl, Cn, al, szl, g.k, g.n, st);
    level++;
    if (stop) break;  // max_levels == 1: final = the identity partition of level 1
  }
  S.levels = c->trace.empty() ? 1 : c->trace.back().level + 1;
  S.sweeps = int32_t(c->trace.size());
  const int32_t* cntL = c->cnt[(level - 1) % 2].as<int32_t>();
  const int32_t* minvL = c->minv[(level - 1) % 2].as<int32_t>();
  // (the labels' first launch also clears the numerator's two counters)
  long long* stat = c->stat.as<long long>();
  static_assert(ST_S == ST_I + 1, "the numerator's counters are adjacent");
  finalize_labels(g.n, Cl, al, szl, cntL, minvL, c->n, c->map0.as<int32_t>(),
                  c->lab.as<int32_t>(), c->cntf.as<int32_t>(), c->C.as<int32_t>(),
                  c->a0.as<int32_t>(), c->sz0.as<int32_t>(), st, stat + ST_I);
  inc_finish(c->inc, c->C.as<int32_t>(), c->n, c->cs, st);  // H(G_t, C_t) for the next step
  c->inc_ready = false;
  // exact numerator on the final level (coarsening preserves N); C_t goes
  // to the caller of dc_apply_batch before the same wait
  modularity_terms(g.off, g.adj, Cl, al, g.n, stat + ST_I, stat + ST_S, st);
  if (c->out_C) {
    DC_HIP(hipMemcpyAsync(c->out_C, c->C.p, size_t(c->n) * 4,
                          c->out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          st));
    c->out_C = nullptr;
  }
  read_stat(c);
  inc_check(c->cs);
  S.N = two_m * c->hstat[ST_I] - c->hstat[ST_S];
  S.two_m = two_m;
  S.q = two_m == 0 ? 0.0 : double(S.N) / (double(two_m) * double(two_m));
}

// Exact numerator of the final partition (Cl, al over the last level g;
// compaction preserves N) and the step's level and sweep counts.
void finish_stats(dc_ctx* c, const LevelView& g) {
  dc_step_stats& S = c->stats;
  S.levels = c->trace.empty() ? 1 : c->trace.back().level + 1;
  S.sweeps = int32_t(c->trace.size());
  long long* stat = c->stat.as<long long>();
  DC_HIP(hipMemsetAsync(stat + ST_I, 0, 16, c->st));
  modularity_terms(g.off, g.adj, c->Cl.as<int32_t>(), c->al.as<int32_t>(), g.n, stat + ST_I,
                   stat + ST_S, c->st);
  read_stat(c);
  S.N = c->two_m * c->hstat[ST_I] - c->hstat[ST_S];
  S.two_m = c->two_m;
  S.q = c->two_m == 0 ? 0.0 : double(S.N) / (double(c->two_m) * double(c->two_m));
}

// Levels of smart local moving (the SLM host method of Sec. 3.4, level
// structure of its reference [waltman2013smart]), level 0 over `active`
// (null = every vertex) from the level-0 partition (Cl, al, szl):
//   1. local moving of the level (the Louvain sweeps; level 0 over R_t);
//   2. stop when every vertex is alone or no level is left;
//   3. refinement: local moving from singletons on the subgraph inside the
//      communities (vertex weights k and 2m of the whole level graph, so the
//      gains and the exact Delta N are the whole graph's), phase 1 records;
//   4. compaction by the refined communities; stop when it does not reduce;
//   5. the next level starts from the parent communities (each coarse vertex
//      labelled by the smallest coarse id among its parent's refined
//      communities) and runs local moving over every vertex.
void run_levels_slm(dc_ctx* c, const int32_t* active, int64_t n_active) {
  hipStream_t st = c->st;
  const int64_t npre = active ? c->pre_count : 0;
  const uint8_t* skip = nullptr;
  if (npre > 0) {
    apply_pre(c->pre_list, npre, c->R.as<uint8_t>(), c->pre.as<int32_t>(), c->Cn.as<int32_t>(),
              st);
    skip = c->pre_skip;
  }
  LevelRun L;
  levels_begin(c, active, n_active, L, skip);
  const long long T = L.T;
  LevelView g = L.g;
  int32_t* Cl = c->Cl.as<int32_t>();
  int32_t* Cn = c->Cn.as<int32_t>();
  int32_t* al = c->al.as<int32_t>();
  int32_t* szl = c->szl.as<int32_t>();
  long long* stat = c->stat.as<long long>();
  const size_t n4 = size_t(c->n + 1) * 4;
  for (DBuf* b : {&c->sub_cnt, &c->sub_off, &c->par, &c->first}) b->ensure(n4);
  int32_t* par = c->par.as<int32_t>();
  int level = 0;
  (void)run_sweeps(c, g, L.act, L.nact, L.bins, 0, T, true, npre > 0);
  mark_phase(c, 3);
  while (true) {
    // 2. communities after the local moving
    DC_HIP(hipMemsetAsync(stat + ST_N0, 0, 8, st));
    nonempty_count(szl, g.n, stat + ST_N0, st);
    read_stat(c);
    if (c->hstat[ST_N0] == g.n || level + 1 >= c->opt.max_levels) break;
    // 3. refinement inside the communities, from singletons
    {
      int32_t* dst[1] = {par};
      const int32_t* src[1] = {Cl};
      copy_i32(dst, src, 1, g.n, st);
    }
    const int64_t nnz_s = induced_subgraph(g, par, c->sub_cnt.as<int32_t>(),
                                           c->sub_off.as<int32_t>(), c->sub_adj, c->hbuf, st);
    start_level(Cl, Cn, al, szl, g.k, g.n, st);
    const LevelView gs{g.n, nnz_s, c->sub_off.as<int32_t>(), c->sub_adj.as<int2>(), g.k};
    Bins rb;
    make_bins(nullptr, g.n, gs.off, rb, c->bins, st, nullptr, nullptr, nullptr, nullptr, 0,
              level > 0);
    (void)run_sweeps(c, gs, nullptr, g.n, rb, level, T, true, false, 1);
    // 4. compaction by the refined communities
    const int next = level % 2;
    const int32_t* cnt_in = level == 0 ? nullptr : c->cnt[(level - 1) % 2].as<int32_t>();
    const int32_t* minv_in = level == 0 ? nullptr : c->minv[(level - 1) % 2].as<int32_t>();
    coarsen(g, Cl, szl, al, cnt_in, minv_in, level == 0, c->n, c->map0.as<int32_t>(),
            c->cg[next], c->cnt[next].as<int32_t>(), c->minv[next].as<int32_t>(), c->cs, st);
    const LevelView h = c->cg[next].view();
    const bool reduced = h.n < g.n;
    // 5. start partition of the compacted graph: the parent communities (also
    // when nothing was reduced: then it is the final partition, over the
    // coarse ids, which may permute the level's ids)
    parent_start(par, Cl, c->cs.rank.as<int32_t>(), g.n, c->first.as<int32_t>(), Cn, st);
    g = h;
    level++;
    {
      int32_t* dst[1] = {Cl};
      const int32_t* src[1] = {Cn};
      copy_i32(dst, src, 1, g.n, st);
    }
    totals_sizes(g.k, Cl, g.n, al, szl, st);
    if (!reduced) break;
    Bins b;
    make_bins(nullptr, g.n, g.off, b, c->bins, st, nullptr, nullptr, nullptr, nullptr, 0, true);
    (void)run_sweeps(c, g, nullptr, g.n, b, level, T, true);
  }
  const int32_t *cntL, *minvL;
  if (level == 0) {  // the level-0 partition is final: identity maps
    fill_i32(c->cnt[1].as<int32_t>(), 1, c->n, st);
    iota_i32(c->first.as<int32_t>(), c->n, st);
    iota_i32(c->map0.as<int32_t>(), c->n, st);
    cntL = c->cnt[1].as<int32_t>();
    minvL = c->first.as<int32_t>();
  } else {
    cntL = c->cnt[(level - 1) % 2].as<int32_t>();
    minvL = c->minv[(level - 1) % 2].as<int32_t>();
  }
  finalize_labels(g.n, Cl, al, szl, cntL, minvL, c->n, c->map0.as<int32_t>(),
                  c->lab.as<int32_t>(), c->cntf.as<int32_t>(), c->C.as<int32_t>(),
                  c->a0.as<int32_t>(), c->sz0.as<int32_t>(), st);
  c->inc.valid = false;  // the first compaction follows the refinement, not H(G, C)
  c->inc_ready = false;
  finish_stats(c, g);
}

// Alg. 1 with level 0 visiting `active` (null = every vertex).  The level-0
// partition is (Cl, al, szl), prepared by the caller.
void run_levels(dc_ctx* c, const int32_t* active, int64_t n_active) {
  if (c->opt.algorithm == DC_ALGO_SLM) {
    run_levels_slm(c, active, n_active);
    return;
  }
  LevelRun L;
  // Screening evaluated its vertices on the state the first level-0 sweep
  // reads (labels C_{t-1}, totals and sizes on G_t): their decisions go
  // into Cn and the first sweep evaluates only the rest of R_t.
  const int64_t npre = active ? c->pre_count : 0;
  const uint8_t* skip = nullptr;
  if (npre > 0) {
    apply_pre(c->pre_list, npre, c->R.as<uint8_t>(), c->pre.as<int32_t>(), c->Cn.as<int32_t>(),
              c->st);
    skip = c->pre_skip;
  }
  levels_begin(c, active, n_active, L, skip);
  const long long gain0 = run_sweeps(c, L.g, L.act, L.nact, L.bins, 0, L.T, true, npre > 0);
  mark_phase(c, 3);
  levels_finish(c, L, gain0);
}

void load_level0_partition(dc_ctx* c);

// Move labels of the touched vertices: level 0 rerun from C_{t-1} with every
// vertex active (full re-evaluation), nothing recorded, state untouched.
void level0_labels(dc_ctx* c) {
  hipStream_t st = c->st;
  const long long two_m = c->two_m;
  const long long T = c->opt.tau_den > 0 ? (two_m * two_m) / c->opt.tau_den : 0;
  LevelView g{c->n, c->nnz, c->off[c->cur].as<int32_t>(), c->adj[c->cur].as<int2>(),
              c->k0.as<int32_t>()};
  load_level0_partition(c);
  Bins bins;
  make_bins(nullptr, c->n, g.off, bins, c->bins, st);
  (void)run_sweeps(c, g, nullptr, c->n, bins, 0, T, false);
  move_labels(c->Tlist.as<int32_t>(), c->T_count, c->Cl.as<int32_t>(), c->C.as<int32_t>(),
              c->y.as<uint8_t>(), st);
}

// The touched set T = R (screened) + S_Delta + Gamma_t(S_Delta) (tmark holds
// the last two), its features on (G_t, C_{t-1}), and, as asked, its move
// labels and its screener logits.
void touched_samples(dc_ctx* c, const LevelView& g0, bool labels, bool score) {
  hipStream_t st = c->st;
  const int32_t n = c->n;
  int32_t* tflag = c->tflag.as<int32_t>();
  int32_t* tpos = c->tpos.as<int32_t>();
  merge_flags(c->R.as<uint8_t>(), c->tmark.as<uint8_t>(), n, tflag, st);
  scan_excl_i32(tflag, tpos, n, tpos + n, st);
  compact_index(tflag, tpos, n, c->Tlist.as<int32_t>(), st);
  // binned by its device length, which comes back with the binning's wait
  Bins b;
  make_bins(c->Tlist.as<int32_t>(), n, g0.off, b, c->bins, st, nullptr, tpos + n);
  c->T_count = b.total;
  if (c->T_count == 0) return;
  // a scored batch keeps each touched vertex's first-sweep decision: the
  // features are taken on the state the first level-0 sweep reads, and R_t
  // is a subset of the touched set
  int32_t* pre = nullptr;
  if (score) {
    c->pre.ensure(size_t(n) * 4);
    pre = c->pre.as<int32_t>();
  }
  feat_eval(g0, c->C.as<int32_t>(), c->a0.as<int32_t>(), c->two_m, b, c->f_own.as<int32_t>(),
            c->f_g1.as<long long>(), c->f_g2.as<long long>(), c->stat.as<long long>(), st,
            c->sz0.as<int32_t>(), c->opt.singleton_guard, pre);
  if (score) {
    c->pre_count = c->T_count;
    c->pre_list = c->Tlist.as<int32_t>();
    c->pre_skip = c->R.as<uint8_t>();  // R_t, once the scores have chosen it
  }
  assemble_features(c->Tlist.as<int32_t>(), c->T_count, c->k0.as<int32_t>(),
                    c->kprev.as<int32_t>(), c->cptr.as<int32_t>(), c->f_own.as<int32_t>(),
                    c->f_g1.as<long long>(), c->f_g2.as<long long>(), c->a0.as<int32_t>(),
                    c->C.as<int32_t>(), c->R.as<uint8_t>(), c->two_m, c->X.as<uint16_t>(), st);
  c->stats.vertex_evals += c->T_count;
  if (labels) {
    level0_labels(c);
    c->have_y = true;
  }
  if (score) {
    mlp_forward(c->scr_wq.as<uint16_t>(), c->X.as<uint16_t>(), c->T_count,
                c->logits.as<float>(), st);
    c->have_logits = true;
  }
}

void start_from_singletons(dc_ctx* c) {
  iota_i32(c->C.as<int32_t>(), c->n, c->st);
  DC_HIP(hipMemcpyAsync(c->a0.p, c->k0.p, size_t(c->n) * 4, hipMemcpyDeviceToDevice, c->st));
  fill_i32(c->sz0.as<int32_t>(), 1, c->n, c->st);
}

// (Cl, Cn, al, szl) = (C, C, a0, sz0): the level-0 start partition.
void load_level0_partition(dc_ctx* c) {
  int32_t* dst[4] = {c->Cl.as<int32_t>(), c->Cn.as<int32_t>(), c->al.as<int32_t>(),
                     c->szl.as<int32_t>()};
  const int32_t* src[4] = {c->C.as<int32_t>(), c->C.as<int32_t>(), c->a0.as<int32_t>(),
                           c->sz0.as<int32_t>()};
  copy_i32(dst, src, 4, c->n, c->st);
}

dc_status status_from_flags(int32_t f) {
  if (f & F_RANGE) return DC_E_RANGE;
  if (f & F_SELF) return DC_E_SELF_LOOP;
  if (f & F_WEIGHT) return DC_E_WEIGHT;
  if (f & F_DUP) return DC_E_DUP;
  if (f & F_NO_EDGE) return DC_E_NO_EDGE;
  return DC_OK;
}

int sort_bits(int32_t n) { return ilog2_ceil(uint64_t(n) * uint64_t(n)); }

dc_status do_init(dc_ctx* c, const dc_edges* g1) {
  hipStream_t st = c->st;
  ensure_vertex_state(c);
  long long* stat = c->stat.as<long long>();
  DC_HIP(hipMemsetAsync(stat, 0, ST_COUNT * 8, st));
  const int32_t *u, *v, *w;
  stage_edges(c, g1, true, c->in_au, c->in_av, c->in_aw, &u, &v, &w);
  const int64_t m = g1 ? g1->count : 0;
  validate_edges(u, v, w, m, c->n, reinterpret_cast<int32_t*>(stat + ST_FLAGS),
                 stat + ST_WSUM_ADD, st);
  read_stat(c);
  int32_t f = int32_t(c->hstat[ST_FLAGS]);
  if (f) return status_from_flags(f);
  const long long wsum = slot_total(c->hstat, ST_WSUM_ADD);
  if (2 * wsum >= TWO_M_LIMIT) return DC_E_OVERFLOW;
  // directed entries, sorted, duplicates summed
  const int64_t md = 2 * m;
  c->akeys.ensure(size_t(md + 1) * 8);
  c->ak1.ensure(size_t(md + 1) * 8);
  c->avals.ensure(size_t(md + 1) * 4);
  c->av1.ensure(size_t(md + 1) * 4);
  c->aheads.ensure(size_t(md + 1) * 4);
  c->apos.ensure(size_t(md + 1) * 4);
  uint64_t* keys = c->akeys.as<uint64_t>();
  uint32_t* vals = c->avals.as<uint32_t>();
  make_directed(u, v, w, m, c->n, keys, vals, st);
  radix_sort_pairs(keys, vals, c->ak1.as<uint64_t>(), c->av1.as<uint32_t>(), md,
                   sort_bits(c->n), st);
  run_heads(keys, md, c->aheads.as<int32_t>(), st);
  int32_t* pos = c->apos.as<int32_t>();
  scan_excl_i32(c->aheads.as<int32_t>(), pos, md, pos + md, st);
  int32_t U = 0;
  if (md > 0) {
    DC_HIP(hipMemcpyAsync(c->hbuf, pos + md, 4, hipMemcpyDeviceToHost, st));
    DC_HIP(hipStreamSynchronize(st));
    U = *static_cast<int32_t*>(c->hbuf);
  }
  c->ukeys.ensure(size_t(U + 1) * 8);
  c->uw.ensure(size_t(U + 1) * 4);
  fill_i32(c->uw.as<int32_t>(), 0, U, st);
  reduce_runs(keys, vals, nullptr, pos, md, c->ukeys.as<uint64_t>(), c->uw.as<int32_t>(), st);
  c->cur = 0;
  c->off[0].ensure(size_t(c->n + 1) * 4);
  c->adj[0].ensure(size_t(U + 1) * 8);
  row_bounds(c->ukeys.as<uint64_t>(), U, c->n, c->off[0].as<int32_t>(), st);
  keys_to_adj(c->ukeys.as<uint64_t>(), c->uw.as<int32_t>(), U, c->n, c->adj[0].as<int2>(), st);
  row_weight_sums(c->off[0].as<int32_t>(), c->adj[0].as<int2>(), c->n, c->k0.as<int32_t>(), st);
  c->nnz = U;
  c->two_m = 2 * wsum;
  start_from_singletons(c);
  load_level0_partition(c);
  c->stats = dc_step_stats{};
  c->stats.R_size = c->n;
  c->inc_ready = false;
  run_levels(c, nullptr, c->n);
  c->have_R_all = true;
  // the initial edge list's sort buffers serve dc_init only (a batch sorts
  // its records in buffers of its own size)
  for (DBuf* b : {&c->akeys, &c->ak1, &c->avals, &c->av1, &c->aheads, &c->apos, &c->ukeys, &c->uw})
    b->release();
  return DC_OK;
}

// First part of a time step: validate, merge, choose R_t; on success the
// level-0 partition is loaded and *act / *nact give the level-0 active set
// (null = every vertex).
dc_status apply_front(dc_ctx* c, const dc_edges* add, const dc_edges* del, const int32_t** act,
                      int64_t* nact) {
  hipStream_t st = c->st;
  c->R_dcount = nullptr;
  const int32_t n = c->n;
  long long* stat = c->stat.as<long long>();
  long long* hs = c->hstat;
  mark_phase(c, 0);
  DC_HIP(hipMemsetAsync(stat, 0, ST_COUNT * 8, st));
  c->pre_count = 0;
  const int32_t *au, *av, *aw, *du, *dv, *dw;
  stage_edges(c, add, true, c->in_au, c->in_av, c->in_aw, &au, &av, &aw);
  stage_edges(c, del, false, c->in_du, c->in_dv, c->in_aw, &du, &dv, &dw);
  const int64_t na = add ? add->count : 0;
  const int64_t nd = del ? del->count : 0;
  int32_t* flags = reinterpret_cast<int32_t*>(stat + ST_FLAGS);
  validate_edges(du, dv, nullptr, nd, n, flags, nullptr, st);
  validate_edges(au, av, aw, na, n, flags, stat + ST_WSUM_ADD, st);
  const int bits = sort_bits(n);
  // every deletion and insertion as two directed records, sorted once; a
  // run of equal keys is one directed pair of the batch
  const int32_t* off_old = c->off[c->cur].as<int32_t>();
  const int2* adj_old = c->adj[c->cur].as<int2>();
  const int64_t nr = 2 * (nd + na);
  for (DBuf* b : {&c->rkeys, &c->rk1, &c->ch_key, &c->ukeys}) b->ensure(size_t(nr + 1) * 8);
  for (DBuf* b : {&c->rvals, &c->rv1, &c->rheads, &c->rpos, &c->ch_op, &c->ch_w, &c->ch_dk,
                  &c->dnet, &c->cnet, &c->ins_flag, &c->ins_pos,
                  &c->src_flag, &c->src_pos, &c->src_list, &c->uw, &c->dw_old})
    b->ensure(size_t(nr + 1) * 4);
  c->ins_keys.ensure(size_t(nr + 1) * 8);
  uint64_t* rkeys = c->rkeys.as<uint64_t>();
  uint32_t* rvals = c->rvals.as<uint32_t>();
  batch_records(du, dv, nd, au, av, na, n, rkeys, rvals, st);
  radix_sort_pairs(rkeys, rvals, c->rk1.as<uint64_t>(), c->rv1.as<uint32_t>(), nr, bits, st);
  int32_t* rheads = c->rheads.as<int32_t>();
  int32_t* rpos = c->rpos.as<int32_t>();
  run_heads(rkeys, nr, rheads, st);
  int32_t* nruns = reinterpret_cast<int32_t*>(stat + ST_N1);
  scan_excl_i32(rheads, rpos, nr, nruns, st);
  uint64_t* ch_key = c->ch_key.as<uint64_t>();
  int32_t* ch_op = c->ch_op.as<int32_t>();
  int32_t* ch_w = c->ch_w.as<int32_t>();
  int32_t* ch_dk = c->ch_dk.as<int32_t>();
  resolve_changes(rkeys, rvals, rpos, nr, nruns, aw, n, off_old, adj_old,
                  c->ukeys.as<uint64_t>(), c->uw.as<int32_t>(), c->dw_old.as<int32_t>(), ch_key,
                  ch_op, ch_w, ch_dk, c->dnet.as<int32_t>(), flags,
                  stat + ST_WSUM_DEL, st);
  read_stat(c);
  // checks in the documented order; nothing has been changed yet
  if (int32_t f = int32_t(hs[ST_FLAGS])) return status_from_flags(f);
  const long long two_m_new =
      c->two_m - 2 * slot_total(hs, ST_WSUM_DEL) + 2 * slot_total(hs, ST_WSUM_ADD);
  if (two_m_new >= TWO_M_LIMIT) return DC_E_OVERFLOW;

  // ---- from here on the state changes ----
  const int64_t nch = nr > 0 ? int32_t(hs[ST_N1]) : 0;
  c->nch_last = nch;
  int32_t* cnet = c->cnet.as<int32_t>();
  scan_excl_i32(c->dnet.as<int32_t>(), cnet, nch, cnet + nch, st);
  c->cptr.ensure(size_t(n + 1) * 4);
  c->new_deg.ensure(size_t(n + 1) * 4);
  int32_t* cptr = c->cptr.as<int32_t>();
  row_bounds(ch_key, nch, n, cptr, st);
  const int mode = c->opt.mode;
  const bool samples = mode == DC_MODE_LEARNED || c->opt.collect;
  c->T_count = 0;
  c->have_y = c->have_logits = false;
  if (samples) {
    ensure_sample_state(c);
    DC_HIP(hipMemcpyAsync(c->kprev.p, c->k0.p, size_t(n) * 4, hipMemcpyDeviceToDevice, st));
  }
  c->tile_row.ensure(size_t(ceil_div(c->nnz, MERGE_TILE) + 1) * 4);
  row_changes(cptr, ch_op, ch_dk, off_old, n, c->new_deg.as<int32_t>(), c->k0.as<int32_t>(),
              c->C.as<int32_t>(), c->a0.as<int32_t>(), c->tile_row.as<int32_t>(), st);
  const int nxt = c->cur ^ 1;
  c->off[nxt].ensure(size_t(n + 1) * 4);
  int32_t* off_new = c->off[nxt].as<int32_t>();
  // (the scans write the new entry count and the insertion count to host
  // memory as well: one wait, no copy)
  int32_t* hb = static_cast<int32_t*>(c->hbuf);
  scan_excl_i32(c->new_deg.as<int32_t>(), off_new, n, off_new + n, st, c->hbuf_dev);
  // insertion keys (sorted directed pairs) and their sources
  select_insertions(ch_op, nch, c->ins_flag.as<int32_t>(), st);
  hb[1] = 0;
  scan_excl_i32(c->ins_flag.as<int32_t>(), c->ins_pos.as<int32_t>(), nch,
                reinterpret_cast<int32_t*>(stat + ST_N2), st, c->hbuf_dev + 1);
  DC_HIP(hipStreamSynchronize(st));
  const int64_t nnz_new = hb[0];
  const int64_t n_ins = nch > 0 ? hb[1] : 0;
  c->n_ins_last = n_ins;
  c->adj[nxt].ensure(size_t(nnz_new + 1) * 8);
  merge_rows(off_old, adj_old, c->nnz, off_new, c->adj[nxt].as<int2>(), n, cptr,
             c->tile_row.as<int32_t>(), ch_key, ch_op, ch_w, cnet, nch, st);
  mark_phase(c, 1);
  c->cur = nxt;
  c->nnz = nnz_new;
  c->two_m = two_m_new;

  dc_step_stats& S = c->stats;
  S = dc_step_stats{};
  S.changes = na + nd;
  LevelView g0{n, c->nnz, c->off[c->cur].as<int32_t>(), c->adj[c->cur].as<int2>(),
               c->k0.as<int32_t>()};
  if (samples) {
    // endpoints of the changed pairs (the distinct sources of the change
    // list) and their neighbours in G_t
    int32_t* crow_flag = c->rheads.as<int32_t>();
    int32_t* crow_pos = c->rpos.as<int32_t>();
    c->chsrc.ensure(size_t(nr + 1) * 4);
    int32_t* crows = c->chsrc.as<int32_t>();
    source_heads(ch_key, nch, n, crow_flag, st);
    scan_excl_i32(crow_flag, crow_pos, nch, crow_pos + nch, st);
    gather_sources(ch_key, crow_flag, crow_pos, nch, n, crows, st);
    fill_u8(c->tmark.as<uint8_t>(), 0, n, st);
    mark_touched(crows, crow_pos + nch, nch, g0.off, g0.adj, c->tmark.as<uint8_t>(), st);
  }
  if (mode == DC_MODE_DELTA || samples) {
    const bool fused = c->opt.del_rule == DC_DEL_GAIN;
    const bool cascade = c->opt.cascade_den > 0;
    if (cascade) c->accflag.ensure(size_t(n) + 1);
    if (fused) {
      c->uflag.ensure(size_t(n) + 1);
      c->ulist.ensure(size_t(n + 1) * 4);
    }
    uint8_t* R = c->R.as<uint8_t>();
    uint8_t* cflag = c->cflag.as<uint8_t>();
    int32_t* dflag = c->dflag.as<int32_t>();
    uint8_t* accflag = cascade ? c->accflag.as<uint8_t>() : nullptr;
    {
      // R, the community flags, the deletion-source flags, the accepted
      // flags (cascade), the union flags (fused) and the count of R_t's
      // list start at zero
      void* zp[6] = {R, cflag, dflag, accflag, fused ? c->uflag.p : nullptr,
                     c->rpos2.as<int32_t>() + n};
      const int64_t zb[6] = {n, n, 4 * int64_t(n), cascade ? int64_t(n) : 0,
                             fused ? int64_t(n) : 0, 4};
      zero_buffers(zp, zb, 6, st);
    }
    uint64_t* ins_keys = c->ins_keys.as<uint64_t>();
    gather_u64(ch_key, c->ins_flag.as<int32_t>(), c->ins_pos.as<int32_t>(), nch, ins_keys, st);
    // Alg. 2 scratch: a gain per insertion record, the best sink per source
    const int64_t item_cap = ds_item_cap(std::min<int64_t>(n, n_ins), c->nnz);
    c->sink_g.ensure(size_t(n_ins + 1) * 8);
    c->best_j.ensure(size_t(n + 1) * 4);
    c->best_g.ensure(size_t(n + 1) * 8);
    c->ds_items.ensure(size_t(item_cap) * 8);
    const DsScratch dsx{c->sink_g.as<long long>(), c->best_j.as<int32_t>(),
                        c->best_g.as<long long>(), c->ds_items.as<int2>(), stat + ST_MARK,
                        item_cap};
    int32_t* src_flag = c->src_flag.as<int32_t>();
    int32_t* src_pos = c->src_pos.as<int32_t>();
    // without the cascade the fused pass needs no list of insertion sources:
    // its vertex set comes straight from the change list
    const bool direct = fused && !cascade;
    if (!direct) {
      source_heads(ins_keys, n_ins, n, src_flag, st);
      scan_excl_i32(src_flag, src_pos, n_ins, reinterpret_cast<int32_t*>(stat + ST_N3), st);
      gather_sources(ins_keys, src_flag, src_pos, n_ins, n, c->src_list.as<int32_t>(), st);
      source_segments(ins_keys, n_ins, n, c->seg_beg.as<int32_t>(), c->seg_end.as<int32_t>(),
                      st);
      // deletion sources (labels C_{t-1})
      deletion_sources(ch_key, ch_op, nch, n, c->C.as<int32_t>(), dflag, st);
    }
    int64_t n_src = 0, n_dsrc = 0;
    if (fused) {
      // one evaluation pass over the insertion sources and the deletion
      // endpoints together (Alg. 2 and the deletion rule read the same state)
      uint8_t* uflag = c->uflag.as<uint8_t>();
      int64_t n_u = 0;
      Bins b;
      bool binned = false;
      if (direct) {
        // uflag, sink segments and the heads of the flagged sources in one
        // pass over the sorted changes; the union list is the heads' sources,
        // binned by its device count (at most nch) with the counters copied
        // back before the binning's wait
        screen_union(ch_key, ch_op, c->ins_pos.as<int32_t>(), ins_keys, n_ins, nch, n,
                     c->C.as<int32_t>(), dflag, uflag, c->seg_beg.as<int32_t>(),
                     c->seg_end.as<int32_t>(), src_flag, stat + ST_NSRC, stat + ST_NDSRC, st);
        scan_excl_i32(src_flag, src_pos, nch, reinterpret_cast<int32_t*>(stat + ST_N0), st);
        gather_sources(ch_key, src_flag, src_pos, nch, n, c->ulist.as<int32_t>(), st);
        make_bins(c->ulist.as<int32_t>(), nch, g0.off, b, c->bins, st, nullptr,
                  reinterpret_cast<const int32_t*>(stat + ST_N0), stat, c->hstat_dev, ST_COUNT);
        check_stat_errors(hs);
        binned = true;
        n_src = slot_total(hs, ST_NSRC);
        n_dsrc = slot_total(hs, ST_NDSRC);
        n_u = b.total;
      } else {
        int32_t* f32 = c->rflag.as<int32_t>();
        int32_t* p32 = c->rpos2.as<int32_t>();
        union_flags(c->src_list.as<int32_t>(), reinterpret_cast<int32_t*>(stat + ST_N3), n_ins,
                    dflag, n, uflag, f32, stat + ST_DEL_SRC, st);
        scan_excl_i32(f32, p32, n, reinterpret_cast<int32_t*>(stat + ST_N0), st);
        compact_index(f32, p32, n, c->ulist.as<int32_t>(), st);
        read_stat(c);
        n_src = n_ins > 0 ? int32_t(hs[ST_N3]) : 0;
        n_dsrc = hs[ST_DEL_SRC];
        n_u = int32_t(hs[ST_N0]);
      }
      if (n_u > 0) {
        if (!binned) make_bins(c->ulist.as<int32_t>(), n_u, g0.off, b, c->bins, st);
        for (int q = 0; q < NBINS; ++q) S.screen_volume += b.vol[q];
        S.screen_vertices = n_u;
        int32_t* pre = nullptr;
        if (mode == DC_MODE_DELTA) {
          c->pre.ensure(size_t(n) * 4);
          pre = c->pre.as<int32_t>();
        }
        ds_both(g0, c->C.as<int32_t>(), c->a0.as<int32_t>(), c->sz0.as<int32_t>(),
                c->opt.singleton_guard, c->two_m, ins_keys, n_ins, c->seg_beg.as<int32_t>(),
                c->seg_end.as<int32_t>(), uflag, b, R, cflag, accflag, pre, dsx, stat, st);
        c->pre_count = pre ? n_u : 0;
        c->pre_list = c->ulist.as<int32_t>();
        c->pre_skip = uflag;
      }
    } else {
      int32_t* dpos = c->dpos.as<int32_t>();
      scan_excl_i32(dflag, dpos, n, dpos + n, st);
      compact_index(dflag, dpos, n, c->dlist.as<int32_t>(), st);
      DC_HIP(hipMemcpyAsync(c->hbuf, dpos + n, 4, hipMemcpyDeviceToHost, st));
      read_stat(c);
      n_src = n_ins > 0 ? int32_t(hs[ST_N3]) : 0;
      n_dsrc = *static_cast<int32_t*>(c->hbuf);
      if (n_src > 0) {
        Bins b;
        make_bins(c->src_list.as<int32_t>(), n_src, g0.off, b, c->bins, st);
        for (int q = 0; q < NBINS; ++q) S.screen_volume += b.vol[q];
        S.screen_vertices = n_src;
        ds_additions(g0, c->C.as<int32_t>(), c->a0.as<int32_t>(), c->two_m, ins_keys, n_ins,
                     c->seg_beg.as<int32_t>(), c->seg_end.as<int32_t>(), b, R, cflag, accflag,
                     dsx, stat, st);
      }
    }
    if (cascade && n_src > 0) {
      // same-community neighbours of the accepted sources, their best gains
      // to another community (EV_FEAT), and the neighbourhoods that join R
      c->cascand.ensure(size_t(n) + 1);
      c->clist.ensure(size_t(n + 1) * 4);
      uint8_t* cand = c->cascand.as<uint8_t>();
      fill_u8(cand, 0, n, st);
      cascade_candidates(c->src_list.as<int32_t>(), n_src, accflag, g0.off, g0.adj,
                         c->C.as<int32_t>(), cand, st);
      int32_t* f32 = c->rflag.as<int32_t>();
      int32_t* p32 = c->rpos2.as<int32_t>();
      merge_flags(cand, nullptr, n, f32, st);
      scan_excl_i32(f32, p32, n, reinterpret_cast<int32_t*>(stat + ST_CASC_CAND), st);
      compact_index(f32, p32, n, c->clist.as<int32_t>(), st);
      read_stat(c);
      const int64_t n_cand = int32_t(hs[ST_CASC_CAND]);
      S.cascade_candidates = n_cand;
      if (n_cand > 0) {
        ensure_sample_state(c);
        Bins b;
        make_bins(c->clist.as<int32_t>(), n_cand, g0.off, b, c->bins, st);
        feat_eval(g0, c->C.as<int32_t>(), c->a0.as<int32_t>(), c->two_m, b,
                  c->f_own.as<int32_t>(), c->f_g1.as<long long>(), c->f_g2.as<long long>(),
                  stat, st);
        cascade_mark(c->clist.as<int32_t>(), n_cand, c->f_g1.as<long long>(), g0.k, c->two_m,
                     c->opt.cascade_num, c->opt.cascade_den, g0.off, g0.adj, R,
                     stat + ST_CASC_EXP, st);
      }
    }
    if (n_dsrc > 0 && !fused)
      mark_neighbourhoods(c->dlist.as<int32_t>(), n_dsrc, g0.off, g0.adj, R, st);
    int32_t* rpos2 = c->rpos2.as<int32_t>();
    materialize_R(R, cflag, c->C.as<int32_t>(), n, c->Rlist.as<int32_t>(), rpos2 + n, st);
    S.ds_sources = n_src;
    S.del_sources = n_dsrc;
    S.vertex_evals += S.ds_sources + S.del_sources + S.cascade_candidates;
    if (mode == DC_MODE_DELTA && !samples) {
      // R_t goes to level 0 as is: its length and the screening counters
      // are read with the level-0 binning's wait (levels_begin)
      c->R_dcount = rpos2 + n;
      c->R_count = n;
    } else if (mode == DC_MODE_LEARNED && c->have_scr) {
      // the scores choose R_t below; the counters come back with its binning
    } else {
      DC_HIP(hipMemcpyAsync(c->hbuf, rpos2 + n, 4, hipMemcpyDeviceToHost, st));
      read_stat(c);
      c->R_count = *static_cast<int32_t*>(c->hbuf);
      screening_counts(c);
    }
  }
  if (samples) {
    const bool score = mode == DC_MODE_LEARNED && c->have_scr;
    touched_samples(c, g0, c->opt.collect != 0, score);
    S.touched = c->T_count;
    if (score) {
      // R_t = touched vertices scoring at least theta
      uint8_t* R = c->R.as<uint8_t>();
      int32_t* rpos2 = c->rpos2.as<int32_t>();
      void* zp[2] = {R, rpos2 + n};
      const int64_t zb[2] = {n, 4};
      zero_buffers(zp, zb, 2, st);
      select_by_score(c->Tlist.as<int32_t>(), c->T_count, c->logits.as<float>(), c->theta, R,
                      st);
      materialize_R(R, nullptr, nullptr, n, c->Rlist.as<int32_t>(), rpos2 + n, st);
      // its length is read with the level-0 binning's wait (levels_begin)
      c->R_dcount = rpos2 + n;
      c->R_count = n;
      S.screened = 1;
    }
  }
  c->inc_ready = true;
  mark_phase(c, 2);
  if (mode == DC_MODE_DELTA || mode == DC_MODE_LEARNED) {
    c->have_R_all = false;
    load_level0_partition(c);
    *act = c->Rlist.as<int32_t>();
    *nact = c->R_count;
  } else {
    if (mode == DC_MODE_STATIC) start_from_singletons(c);
    load_level0_partition(c);
    S.R_size = n;
    c->have_R_all = true;
    *act = nullptr;
    *nact = n;
  }
  return DC_OK;
}

// Statistics of the screening pass from the status block copy in hstat
// (R_count known).
void screening_counts(dc_ctx* c) {
  dc_step_stats& S = c->stats;
  const long long* hs = c->hstat;
  S.ds_accepted = hs[ST_DS_ACC];
  S.del_accepted = c->opt.del_rule == DC_DEL_CONSERVATIVE ? S.del_sources : hs[ST_DEL_ACC];
  S.R_size = c->R_count;
  S.cascade_expanded = hs[ST_CASC_EXP];
  S.accepted_volume = hs[ST_ACCVOL];
}

// Last part of a time step: C_t to the caller (device or host memory),
// unless levels_finish has already copied it with its last wait.
void apply_output(dc_ctx* c) {
  if (!c->out_C) return;
  DC_HIP(hipMemcpyAsync(c->out_C, c->C.p, size_t(c->n) * 4,
                        c->out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                        c->st));
  DC_HIP(hipStreamSynchronize(c->st));
  c->out_C = nullptr;
}

void apply_output(dc_ctx* c, int32_t* C_out, int32_t out_on_device) {
  c->out_C = C_out;
  c->out_on_device = out_on_device;
  apply_output(c);
}

// Device time and algorithmic bytes of a timed step's phases (the bytes of
// each phase as documented with dc_step_stats.ms_phase).
void phase_stats(dc_ctx* c) {
  dc_step_stats& S = c->stats;
  DC_HIP(hipEventSynchronize(c->evp[4]));
  for (int k = 0; k < 4; ++k) {
    float ms = 0.f;
    DC_HIP(hipEventElapsedTime(&ms, c->evp[k], c->evp[k + 1]));
    S.ms_phase[k] = ms;
  }
  S.bytes_phase[0] = 28 * S.changes;
  if (c->opt.mode == DC_MODE_DELTA) {
    S.bytes_phase[1] = 12 * S.screen_volume + 32 * S.screen_vertices + 20 * c->n_ins_last +
                       8 * S.accepted_volume + 5 * int64_t(c->n) + 4 * S.R_size;
  }
  S.bytes_phase[2] = 12 * S.level0_volume + 32 * S.level0_active;
  int64_t upper = 12 * int64_t(c->n);
  for (const dc_sweep_rec& r : c->trace)
    if (r.level > 0 || r.phase != 0) upper += 12 * r.nnz_level + 32 * int64_t(r.n_active);
  S.bytes_phase[3] = upper;
}

dc_status do_apply(dc_ctx* c, const dc_edges* add, const dc_edges* del, int32_t* C_out,
                   int32_t out_on_device) {
  const int32_t* act = nullptr;
  int64_t nact = 0;
  c->phase_timing = c->opt.timing != 0;
  const dc_status s = apply_front(c, add, del, &act, &nact);
  if (s != DC_OK) {
    c->phase_timing = false;
    return s;
  }
  c->out_C = C_out;
  c->out_on_device = out_on_device;
  struct ClearOut {  // no destination outlives the call (also on an error)
    dc_ctx* c;
    ~ClearOut() { c->out_C = nullptr; }
  } clear_out{c};
  run_levels(c, act, nact);
  apply_output(c);
  mark_phase(c, 4);
  if (c->phase_timing) phase_stats(c);
  c->phase_timing = false;
  return DC_OK;
}

template <class F>
dc_status guarded(dc_ctx* c, F&& f) {
  if (!c) return DC_E_ARG;
  if (c->poisoned) return DC_E_STATE;
  try {
    return f();
  } catch (const DeviceError& e) {
    dc_status s = map_device_error(e);
    if (s == DC_E_DEVICE) c->poisoned = true;
    return s;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return DC_E_OOM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    c->poisoned = true;
    return DC_E_DEVICE;
  } catch (...) {
    c->poisoned = true;
    return DC_E_DEVICE;
  }
}

void destroy_ctx(dc_ctx* c) {
  if (!c) return;
  if (c->st) (void)hipStreamSynchronize(c->st);
  if (c->hstat) (void)hipHostFree(c->hstat);
  if (c->hbuf) (void)hipHostFree(c->hbuf);
  if (c->bins.host) (void)hipHostFree(c->bins.host);
  if (c->cs.host) (void)hipHostFree(c->cs.host);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  for (hipEvent_t e : c->evp)
    if (e) (void)hipEventDestroy(e);
  if (c->bins.side) {
    (void)hipStreamSynchronize(c->bins.side);
    (void)hipStreamDestroy(c->bins.side);
  }
  if (c->bins.fork) (void)hipEventDestroy(c->bins.fork);
  if (c->bins.join) (void)hipEventDestroy(c->bins.join);
  delete c;
}


// Every device buffer of a context (the screener weights excepted: small,
// and kept across eviction).
template <class F>
void for_each_buf(dc_ctx* c, F&& f) {
  for (DBuf* b : {&c->off[0], &c->off[1], &c->adj[0], &c->adj[1], &c->k0, &c->C, &c->a0,
                  &c->sz0, &c->in_au, &c->in_av, &c->in_aw, &c->in_du, &c->in_dv, &c->dw_old, &c->akeys, &c->avals, &c->ak1,
                  &c->av1, &c->aheads, &c->apos, &c->ukeys, &c->uw, &c->rkeys, &c->rvals,
                  &c->rk1, &c->rv1, &c->rheads, &c->rpos, &c->ch_key, &c->ch_op, &c->ch_w,
                  &c->ch_dk, &c->dnet, &c->cnet, &c->cptr, &c->new_deg, &c->tile_row, &c->ins_flag, &c->ins_pos, &c->ins_keys, &c->src_flag,
                  &c->src_pos, &c->src_list, &c->dflag, &c->dpos, &c->dlist, &c->R, &c->cflag,
                  &c->rflag, &c->rpos2, &c->Rlist, &c->seg_beg, &c->seg_end, &c->chsrc,
                  &c->accflag, &c->cascand, &c->clist, &c->uflag, &c->ulist, &c->pre, &c->sink_g, &c->best_j,
                  &c->best_g, &c->ds_items, &c->sub_cnt, &c->sub_off, &c->sub_adj,
                  &c->par, &c->first,
                  &c->kprev, &c->tmark, &c->tflag, &c->tpos, &c->Tlist, &c->f_own,
                  &c->f_g1, &c->f_g2, &c->X, &c->y, &c->logits, &c->Cl, &c->Cn, &c->al,
                  &c->szl, &c->dpack, &c->lflag, &c->tlist, &c->movers, &c->map0, &c->cnt[0],
                  &c->cnt[1], &c->minv[0], &c->minv[1], &c->lab, &c->cntf, &c->stat, &c->done,
                  &c->cg[0].off, &c->cg[0].adj, &c->cg[0].k, &c->cg[1].off, &c->cg[1].adj,
                  &c->cg[1].k, &c->bins.lists, &c->bins.lists_rb, &c->bins.ovf,
                  &c->bins.bcnt, &c->bins.boff, &c->bins.counts,
                  &c->bins.tab_off, &c->bins.gkeys, &c->bins.gvals, &c->cs.flag, &c->cs.rank,
                  &c->cs.keys0, &c->cs.keys1, &c->cs.vals0, &c->cs.vals1, &c->cs.cntr,
                  &c->cs.mstart, &c->cs.labof, &c->cs.mdeg, &c->cs.mvol, &c->cs.chead,
                  &c->cs.cpos, &c->cs.chunks, &c->cs.mcnt, &c->cs.pk0, &c->cs.pk1, &c->cs.pv0,
                  &c->cs.pv1, &c->cs.ph, &c->cs.pp, &c->cs.pS, &c->cs.pcnt, &c->cs.hidx,
                  &c->cs.ukey, &c->cs.rc, &c->inc.lkey, &c->inc.lw,
                  &c->inc.lminv, &c->inc.ek0, &c->inc.ek1, &c->inc.ev0, &c->inc.ev1,
                  &c->inc.heads, &c->inc.hpos, &c->inc.v64, &c->inc.S, &c->inc.starts,
                  &c->inc.nz, &c->inc.npos, &c->inc.mflag, &c->inc.mvol, &c->inc.tkey,
                  &c->inc.tw})
    f(*b);
}

int64_t ctx_footprint(const dc_ctx* c) {
  int64_t t = int64_t(c->scr_wq.bytes);
  for_each_buf(const_cast<dc_ctx*>(c), [&](DBuf& b) { t += int64_t(b.bytes); });
  return t;
}

void ctx_evict(dc_ctx* c, SavedState& s) {
  hipStream_t st = c->st;
  const size_t n = size_t(c->n);
  s.nnz = c->nnz;
  s.two_m = c->two_m;
  s.off.resize(n + 1);
  s.adj.resize(size_t(c->nnz));
  s.k.resize(n);
  s.C.resize(n);
  s.a.resize(n);
  s.sz.resize(n);
  DC_HIP(hipMemcpyAsync(s.off.data(), c->off[c->cur].p, (n + 1) * 4, hipMemcpyDeviceToHost, st));
  if (c->nnz > 0)
    DC_HIP(hipMemcpyAsync(s.adj.data(), c->adj[c->cur].p, size_t(c->nnz) * 8,
                          hipMemcpyDeviceToHost, st));
  DC_HIP(hipMemcpyAsync(s.k.data(), c->k0.p, n * 4, hipMemcpyDeviceToHost, st));
  DC_HIP(hipMemcpyAsync(s.C.data(), c->C.p, n * 4, hipMemcpyDeviceToHost, st));
  DC_HIP(hipMemcpyAsync(s.a.data(), c->a0.p, n * 4, hipMemcpyDeviceToHost, st));
  DC_HIP(hipMemcpyAsync(s.sz.data(), c->sz0.p, n * 4, hipMemcpyDeviceToHost, st));
  DC_HIP(hipStreamSynchronize(st));
  for_each_buf(c, [](DBuf& b) { b.release(); });
  pool_trim();  // the evicted bytes leave the GPU, not just the context
  c->inc.valid = false;  // the first step after restore compacts from all of G_t
  c->inc.h = 0;
}

void ensure_vertex_state(dc_ctx* c);

void ctx_restore(dc_ctx* c, const SavedState& s) {
  hipStream_t st = c->st;
  const size_t n = size_t(c->n);
  ensure_vertex_state(c);
  c->cur = 0;
  c->nnz = s.nnz;
  c->two_m = s.two_m;
  c->off[0].ensure((n + 1) * 4);
  c->adj[0].ensure(size_t(s.nnz + 1) * 8);
  DC_HIP(hipMemcpyAsync(c->off[0].p, s.off.data(), (n + 1) * 4, hipMemcpyHostToDevice, st));
  if (s.nnz > 0)
    DC_HIP(hipMemcpyAsync(c->adj[0].p, s.adj.data(), size_t(s.nnz) * 8, hipMemcpyHostToDevice,
                          st));
  DC_HIP(hipMemcpyAsync(c->k0.p, s.k.data(), n * 4, hipMemcpyHostToDevice, st));
  DC_HIP(hipMemcpyAsync(c->C.p, s.C.data(), n * 4, hipMemcpyHostToDevice, st));
  DC_HIP(hipMemcpyAsync(c->a0.p, s.a.data(), n * 4, hipMemcpyHostToDevice, st));
  DC_HIP(hipMemcpyAsync(c->sz0.p, s.sz.data(), n * 4, hipMemcpyHostToDevice, st));
  DC_HIP(hipStreamSynchronize(st));
}

void level0_merged(dc_ctx* const* cs, LevelRun* Ls, long long* gains, int m, MergeScratch& X) {
  if (m <= 0) return;
  hipStream_t st = cs[0]->st;
  for (int j = 1; j < m; ++j)
    if (cs[j]->st != st) throw std::runtime_error("merged sweeps need one stream");
  if (m > X.cap) throw std::runtime_error("merge scratch too small");
  std::vector<const Bins*> bl(static_cast<size_t>(m)), bl0(static_cast<size_t>(m));
  std::vector<Bins> firsts(static_cast<size_t>(m));
  bool any_pre = false;
  for (int j = 0; j < m; ++j) {
    bl[size_t(j)] = &Ls[j].bins;
    firsts[size_t(j)] = Ls[j].pre_done ? first_part(Ls[j].bins) : Ls[j].bins;
    bl0[size_t(j)] = &firsts[size_t(j)];
    any_pre = any_pre || Ls[j].pre_done;
  }
  build_multi_bins(bl.data(), m, X.mb, X.hsegs, X.segs, st);
  // the first round evaluates only what the screening pass has not decided
  if (any_pre)
    build_multi_bins(bl0.data(), m, X.mb0, X.hsegs + size_t(NBINS) * size_t(X.cap), X.segs0, st);
  int max_sw = 1;
  int64_t max_nact = 1;
  for (int j = 0; j < m; ++j) {
    max_sw = std::max(max_sw, cs[j]->opt.max_sweeps);
    max_nact = std::max<int64_t>(max_nact, Ls[j].nact);
  }
  X.descs.ensure(size_t(m) * sizeof(EvalArgs));
  X.gdesc.ensure(size_t(m) * sizeof(MergedGraph));
  X.done.ensure(size_t(m) * 4);
  X.sweeps.ensure(size_t(m) * 4);
  X.rec.ensure(size_t(m) * size_t(max_sw) * 3 * 8);
  long long* rec = X.rec.as<long long>();
  for (int j = 0; j < m; ++j) {
    dc_ctx* c = cs[j];
    const LevelRun& L = Ls[j];
    X.hdescs[j] = sweep_args_bins(L.g, c->Cl.as<int32_t>(), c->Cn.as<int32_t>(),
                                  c->al.as<int32_t>(), c->szl.as<int32_t>(), c->two_m,
                                  c->opt.singleton_guard, c->stat.as<long long>(), L.bins);
    MergedGraph& G = X.hgdesc[j];
    G.off = L.g.off;
    G.adj = L.g.adj;
    G.k = L.g.k;
    G.C = c->Cl.as<int32_t>();
    G.Cn = c->Cn.as<int32_t>();
    G.a = c->al.as<int32_t>();
    G.sz = c->szl.as<int32_t>();
    G.act = L.act;
    G.nact = L.nact;
    G.dpack = c->dpack.as<long long>();
    G.tflag = c->lflag.as<int32_t>();
    G.tlist = c->tlist.as<int32_t>();
    G.movers = c->movers.as<int32_t>();
    G.stat = c->stat.as<long long>();
    G.two_m = c->two_m;
    G.T = L.T;
    G.max_sweeps = c->opt.max_sweeps;
    G.pad = 0;
    G.rec = rec + size_t(j) * size_t(max_sw) * 3;
    gains[j] = 0;
  }
  DC_HIP(hipMemcpyAsync(X.descs.p, X.hdescs, size_t(m) * sizeof(EvalArgs),
                        hipMemcpyHostToDevice, st));
  DC_HIP(hipMemcpyAsync(X.gdesc.p, X.hgdesc, size_t(m) * sizeof(MergedGraph),
                        hipMemcpyHostToDevice, st));
  int32_t* state = X.done.as<int32_t>();
  int32_t* sweeps = X.sweeps.as<int32_t>();
  const MergedGraph* G = X.gdesc.as<MergedGraph>();
  {
    void* zp[2] = {state, sweeps};
    const int64_t zb[2] = {4 * int64_t(m), 4 * int64_t(m)};
    zero_buffers(zp, zb, 2, st);
  }
  // Rounds run without host waits: convergence is decided on the device
  // (the state words); the host reads the states every `batch` rounds.
  int32_t* hstate = X.hdone;
  int32_t* hsweeps = X.hdone + m;
  int batch = 2, rounds = 0;
  while (true) {
    for (int r = 0; r < batch; ++r) {
      merged_reset(G, m, state, st);
      sweep_eval_multi(X.descs.as<EvalArgs>(), state, rounds + r == 0 && any_pre ? X.mb0 : X.mb,
                       st);
      merged_apply(G, m, max_nact, state, sweeps, st);
    }
    rounds += batch;
    DC_HIP(hipMemcpyAsync(hstate, state, size_t(m) * 4, hipMemcpyDeviceToHost, st));
    DC_HIP(hipStreamSynchronize(st));
    bool all = true;
    for (int j = 0; j < m; ++j) all = all && hstate[j] != 0;
    if (all || rounds >= max_sw) break;
    batch = std::min(2 * batch, max_sw - rounds);
  }
  // the sweep records and the status blocks (self-check bits), one wait
  DC_HIP(hipMemcpyAsync(hsweeps, sweeps, size_t(m) * 4, hipMemcpyDeviceToHost, st));
  std::vector<long long> hrec(size_t(m) * size_t(max_sw) * 3);
  DC_HIP(hipMemcpyAsync(hrec.data(), rec, hrec.size() * 8, hipMemcpyDeviceToHost, st));
  for (int j = 0; j < m; ++j)
    DC_HIP(hipMemcpyAsync(cs[j]->hstat, cs[j]->stat.p, ST_COUNT * 8, hipMemcpyDeviceToHost, st));
  DC_HIP(hipStreamSynchronize(st));
  for (int j = 0; j < m; ++j) {
    dc_ctx* c = cs[j];
    check_stat_errors(c->hstat);
    const long long* r = hrec.data() + size_t(j) * size_t(max_sw) * 3;
    for (int s = 0; s < hsweeps[j]; ++s) {
      c->hstat[ST_MOVES] = r[3 * s];
      c->hstat[ST_DN] = r[3 * s + 1];
      c->hstat[ST_KEEP] = r[3 * s + 2];
      (void)sweep_account(c, Ls[j].g, 0, s, s == 0 ? firsts[size_t(j)] : Ls[j].bins, Ls[j].T,
                          true, -1.f, gains[j], Ls[j].nact);
    }
  }
}

// A new context with its pinned host buffers, events and second stream;
// `build` fills its device state.  On failure everything is released.
template <class F>
dc_status create_ctx(dc_ctx** out, int32_t n, const dc_options* opt, F&& build) {
  *out = nullptr;
  dc_ctx* c = new (std::nothrow) dc_ctx();
  if (!c) return DC_E_OOM;
  c->n = n;
  c->opt = *opt;
  c->st = static_cast<hipStream_t>(opt->stream);
  dc_status s;
  try {
    DC_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->hstat), ST_COUNT * 8));
    DC_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&c->hstat_dev), c->hstat, 0));
    DC_HIP(hipHostMalloc(&c->hbuf, 64));
    DC_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&c->hbuf_dev), c->hbuf, 0));
    DC_HIP(hipHostMalloc(&c->bins.host, 256));
    std::memset(c->bins.host, 0, 256);
    DC_HIP(hipHostMalloc(&c->cs.host, 64));
    DC_HIP(hipEventCreate(&c->ev0));
    DC_HIP(hipEventCreate(&c->ev1));
    for (hipEvent_t& e : c->evp) DC_HIP(hipEventCreate(&e));
    DC_HIP(hipStreamCreateWithFlags(&c->bins.side, hipStreamNonBlocking));
    DC_HIP(hipEventCreateWithFlags(&c->bins.fork, hipEventDisableTiming));
    DC_HIP(hipEventCreateWithFlags(&c->bins.join, hipEventDisableTiming));
    double t0 = now_ms();
    s = build(c);
    c->stats.ms_total = now_ms() - t0;
  } catch (const DeviceError& e) {
    s = map_device_error(e);
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    s = DC_E_OOM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    s = DC_E_DEVICE;
  } catch (...) {
    s = DC_E_DEVICE;
  }
  if (s != DC_OK) {
    destroy_ctx(c);
    return s;
  }
  *out = c;
  return DC_OK;
}
}  // namespace dc_core

using namespace dc_core;

extern "C" {

void dc_default_options(dc_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->mode = DC_MODE_DELTA;
  opt->max_levels = 32;
  opt->max_sweeps = 100;
  opt->singleton_guard = 1;
  opt->del_rule = DC_DEL_GAIN;
  opt->timing = 0;
  opt->tau_den = 1000000;
  opt->stream = nullptr;
}

dc_status dc_init(dc_ctx** out, int32_t n, const dc_edges* g1, const dc_options* opt) {
  if (!out || n < 1 || !options_ok(opt)) return DC_E_ARG;
  if (g1 && g1->count < 0) return DC_E_ARG;
  if (g1 && g1->count > 0 && (!g1->u || !g1->v || !g1->w)) return DC_E_ARG;
  return create_ctx(out, n, opt, [&](dc_ctx* c) { return do_init(c, g1); });
}

dc_status dc_init_from_state(dc_ctx** out, int32_t n, const int64_t* off, const int32_t* col,
                             const int32_t* w, const int32_t* C, const dc_options* opt) {
  if (!out || n < 1 || !off || !C || !options_ok(opt)) return DC_E_ARG;
  *out = nullptr;
  const int64_t nnz = off[n];
  if (off[0] != 0 || nnz < 0 || nnz > (int64_t(1) << 31) || (nnz > 0 && (!col || !w)))
    return DC_E_ARG;
  SavedState st;
  try {
    st.off.resize(size_t(n) + 1);
    st.adj.resize(size_t(nnz));
    st.k.assign(size_t(n), 0);
    st.C.assign(C, C + n);
    st.a.assign(size_t(n), 0);
    st.sz.assign(size_t(n), 0);
  } catch (const std::bad_alloc&) {
    return DC_E_OOM;
  }
  // rows: monotone offsets, neighbours in range, sorted, no self-loop, w >= 1
  int64_t two_m = 0;
  for (int32_t u = 0; u < n; ++u) {
    if (off[u + 1] < off[u] || off[u + 1] > nnz) return DC_E_ARG;
    st.off[size_t(u)] = int32_t(off[u]);
    int64_t ku = 0;
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      const int32_t v = col[e];
      if (v < 0 || v >= n || v == u || w[e] < 1) return DC_E_ARG;
      if (e > off[u] && col[e - 1] >= v) return DC_E_ARG;
      st.adj[size_t(e)] = make_int2(v, w[e]);
      ku += w[e];
    }
    two_m += ku;
    if (two_m >= TWO_M_LIMIT) return DC_E_OVERFLOW;
    st.k[size_t(u)] = int32_t(ku);
  }
  st.off[size_t(n)] = int32_t(nnz);
  // symmetry: (u, v, w) needs (v, u, w)
  for (int32_t u = 0; u < n; ++u)
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      const int32_t v = col[e];
      const int32_t* b = col + off[v];
      const int32_t* f = std::lower_bound(b, col + off[v + 1], u);
      if (f == col + off[v + 1] || *f != u || w[off[v] + (f - b)] != w[e]) return DC_E_ARG;
    }
  // canonical labels: each community labelled by its smallest member
  for (int32_t v = 0; v < n; ++v) {
    const int32_t c = C[v];
    if (c < 0 || c > v || C[c] != c) return DC_E_ARG;
    st.a[size_t(c)] += st.k[size_t(v)];
    st.sz[size_t(c)] += 1;
  }
  st.nnz = nnz;
  st.two_m = two_m;
  return create_ctx(out, n, opt, [&](dc_ctx* c) {
    ctx_restore(c, st);
    c->stats = dc_step_stats{};
    c->stats.two_m = two_m;
    return DC_OK;
  });
}

dc_status dc_export_state(dc_ctx* ctx, int64_t* off, int32_t* col, int32_t* w, int32_t* C) {
  if (!C) return DC_E_ARG;
  dc_status s = dc_export_csr(ctx, off, col, w);
  if (s != DC_OK) return s;
  return dc_communities(ctx, C, 0);
}

dc_status dc_apply_batch(dc_ctx* ctx, const dc_edges* add, const dc_edges* del, int32_t* C_out,
                         int32_t out_on_device, dc_step_stats* stats) {
  if (add && (add->count < 0 || (add->count > 0 && (!add->u || !add->v || !add->w))))
    return DC_E_ARG;
  if (del && (del->count < 0 || (del->count > 0 && (!del->u || !del->v)))) return DC_E_ARG;
  return guarded(ctx, [&] {
    double t0 = now_ms();
    dc_status s = do_apply(ctx, add, del, C_out, out_on_device);
    if (s == DC_OK) {
      ctx->stats.ms_total = now_ms() - t0;
      if (stats) *stats = ctx->stats;
    }
    return s;
  });
}

dc_status dc_modularity(dc_ctx* ctx, double* q, int64_t* num, int64_t* two_m) {
  return guarded(ctx, [&] {
    hipStream_t st = ctx->st;
    long long* stat = ctx->stat.as<long long>();
    DC_HIP(hipMemsetAsync(stat + ST_I, 0, 16, st));
    int32_t* atmp = ctx->lab.as<int32_t>();
    fill_i32(atmp, 0, ctx->n, st);
    intra_weight(ctx->off[ctx->cur].as<int32_t>(), ctx->adj[ctx->cur].as<int2>(),
                 ctx->C.as<int32_t>(), ctx->n, stat + ST_I, st);
    label_totals(ctx->k0.as<int32_t>(), ctx->C.as<int32_t>(), ctx->n, atmp, st);
    sum_squares(atmp, ctx->n, stat + ST_S, st);
    read_stat(ctx);
    long long N = ctx->two_m * ctx->hstat[ST_I] - ctx->hstat[ST_S];
    if (num) *num = N;
    if (two_m) *two_m = ctx->two_m;
    if (q) *q = ctx->two_m == 0 ? 0.0 : double(N) / (double(ctx->two_m) * double(ctx->two_m));
    return DC_OK;
  });
}

dc_status dc_communities(dc_ctx* ctx, int32_t* out, int32_t on_device) {
  if (!out) return DC_E_ARG;
  return guarded(ctx, [&] {
    DC_HIP(hipMemcpyAsync(out, ctx->C.p, size_t(ctx->n) * 4,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, ctx->st));
    DC_HIP(hipStreamSynchronize(ctx->st));
    return DC_OK;
  });
}

dc_status dc_last_R(dc_ctx* ctx, uint8_t* out, int32_t on_device) {
  if (!out) return DC_E_ARG;
  return guarded(ctx, [&] {
    if (ctx->have_R_all) {
      if (on_device) {
        fill_u8(out, 1, ctx->n, ctx->st);
        DC_HIP(hipStreamSynchronize(ctx->st));
      } else {
        std::memset(out, 1, size_t(ctx->n));
      }
      return DC_OK;
    }
    DC_HIP(hipMemcpyAsync(out, ctx->R.p, size_t(ctx->n),
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, ctx->st));
    DC_HIP(hipStreamSynchronize(ctx->st));
    return DC_OK;
  });
}

dc_status dc_last_trace(dc_ctx* ctx, dc_sweep_rec* out, int32_t cap, int32_t* count) {
  if (cap < 0 || (cap > 0 && !out)) return DC_E_ARG;
  return guarded(ctx, [&] {
    int32_t total = int32_t(ctx->trace.size());
    for (int32_t i = 0; i < total && i < cap; ++i) out[i] = ctx->trace[size_t(i)];
    if (count) *count = total;
    return DC_OK;
  });
}

dc_status dc_last_stats(dc_ctx* ctx, dc_step_stats* out) {
  if (!out) return DC_E_ARG;
  return guarded(ctx, [&] {
    *out = ctx->stats;
    return DC_OK;
  });
}

dc_status dc_num_entries(dc_ctx* ctx, int64_t* nnz) {
  if (!nnz) return DC_E_ARG;
  return guarded(ctx, [&] {
    *nnz = ctx->nnz;
    return DC_OK;
  });
}

dc_status dc_export_csr(dc_ctx* ctx, int64_t* off, int32_t* col, int32_t* w) {
  if (!off || (!col && ctx && ctx->nnz > 0) || (!w && ctx && ctx->nnz > 0)) return DC_E_ARG;
  return guarded(ctx, [&] {
    std::vector<int32_t> o(size_t(ctx->n) + 1);
    std::vector<int2> e(size_t(ctx->nnz));
    DC_HIP(hipMemcpyAsync(o.data(), ctx->off[ctx->cur].p, o.size() * 4, hipMemcpyDeviceToHost,
                          ctx->st));
    if (ctx->nnz > 0)
      DC_HIP(hipMemcpyAsync(e.data(), ctx->adj[ctx->cur].p, e.size() * 8, hipMemcpyDeviceToHost,
                            ctx->st));
    DC_HIP(hipStreamSynchronize(ctx->st));
    for (size_t i = 0; i < o.size(); ++i) off[i] = o[i];
    for (size_t i = 0; i < e.size(); ++i) {
      col[i] = e[i].x;
      w[i] = e[i].y;
    }
    return DC_OK;
  });
}

void dc_destroy(dc_ctx* ctx) { destroy_ctx(ctx); }

void dc_trim_device_cache(void) { pool_trim(); }

dc_status dc_screener_set(dc_ctx* ctx, const float* w, float theta) {
  return guarded(ctx, [&] {
    if (!w) {
      ctx->have_scr = false;
      return DC_OK;
    }
    std::vector<uint16_t> q(MLP_P);
    for (int p = 0; p < MLP_P; ++p) q[size_t(p)] = bf16_bits(w[p]);
    ctx->scr_wq.ensure(MLP_P * 2);
    DC_HIP(hipMemcpyAsync(ctx->scr_wq.p, q.data(), MLP_P * 2, hipMemcpyHostToDevice, ctx->st));
    DC_HIP(hipStreamSynchronize(ctx->st));
    ctx->theta = theta;
    ctx->have_scr = true;
    ensure_sample_state(ctx);  // the scoring buffers, sized once here
    return DC_OK;
  });
}

dc_status dc_last_samples(dc_ctx* ctx, int64_t* count, int32_t* ids, uint16_t* X, uint8_t* y,
                          float* logits, int32_t on_device) {
  if (!count) return DC_E_ARG;
  return guarded(ctx, [&] {
    const int64_t cnt = ctx->T_count;
    *count = cnt;
    if (cnt == 0) return DC_OK;
    if ((y && !ctx->have_y) || (logits && !ctx->have_logits)) return DC_E_ARG;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (ids) DC_HIP(hipMemcpyAsync(ids, ctx->Tlist.p, size_t(cnt) * 4, kind, ctx->st));
    if (X) DC_HIP(hipMemcpyAsync(X, ctx->X.p, size_t(cnt) * 16, kind, ctx->st));
    if (y) DC_HIP(hipMemcpyAsync(y, ctx->y.p, size_t(cnt), kind, ctx->st));
    if (logits) DC_HIP(hipMemcpyAsync(logits, ctx->logits.p, size_t(cnt) * 4, kind, ctx->st));
    DC_HIP(hipStreamSynchronize(ctx->st));
    return DC_OK;
  });
}

const char* dc_last_error(void) { return g_last_error.c_str(); }

const char* dc_strerror(dc_status s) {
  switch (s) {
    case DC_OK: return "ok";
    case DC_E_ARG: return "invalid argument";
    case DC_E_RANGE: return "vertex id out of range";
    case DC_E_SELF_LOOP: return "self-loop";
    case DC_E_WEIGHT: return "edge weight below 1";
    case DC_E_NO_EDGE: return "deleted edge not present";
    case DC_E_DUP: return "pair deleted twice";
    case DC_E_OVERFLOW: return "total weight 2m would reach 2^31";
    case DC_E_OOM: return "device memory exhausted";
    case DC_E_DEVICE: return "device error";
    case DC_E_STATE: return "context poisoned by an earlier device error";
    default: return "unknown status";
  }
}

}  // extern "C"
