// server.hip -- serving many dynamic graphs from one GPU (an extension: the
// paper treats one graph).  dc_server_* of dc.h.
//
// A worker thread owns the GPU work.  Round after round it takes the
// oldest waiting batch of up to max_inflight distinct graphs (each graph's
// batches in submission order; batches arriving meanwhile join later
// rounds), admits the graphs under the device-memory budget (moving idle
// graphs' state to host memory, least recently used first), runs every
// batch's front part (validation, merge, R_t), the graphs' level-0 sweeps
// merged into shared launches, and every batch's remaining levels.  All
// graphs use the server's stream, so the merged launches see a consistent
// order; results equal those of each graph run alone (exact integer
// arithmetic on disjoint state).
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "ctx.h"

using namespace dc_core;

namespace {

int64_t mono_ns() {
  using namespace std::chrono;
  return duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
  int64_t ticket = 0;
  int32_t gid = 0;
  bool init = false;  // add_graph: build G_1 and run Static(G_1)
  int32_t n = 0;
  std::vector<int32_t> au, av, aw, du, dv;
  int64_t arrival_ns = 0, start_ns = 0, done_ns = 0;
  dc_status status = DC_PENDING;  // published under the server's lock
  dc_status result = DC_PENDING;  // the worker's result, published at round end
  double t0_ms = 0;
  std::vector<int32_t> C;
  dc_step_stats stats{};
};

struct Graph {
  dc_ctx* ctx = nullptr;
  int32_t n = 0;
  int64_t edges = 0;
  bool resident = false;
  bool busy = false;
  int64_t footprint = 0;  // device bytes while resident (last measured)
  int64_t last_used = 0;
  SavedState saved;
};

// Copies an edge list (host or device) into host vectors.
void copy_edges(const dc_edges* e, bool weights, std::vector<int32_t>& u,
                std::vector<int32_t>& v, std::vector<int32_t>& w) {
  const size_t m = e ? size_t(e->count) : 0;
  u.resize(m);
  v.resize(m);
  w.resize(weights ? m : 0);
  if (m == 0) return;
  const hipMemcpyKind kind = e->on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
  DC_HIP(hipMemcpy(u.data(), e->u, m * 4, kind));
  DC_HIP(hipMemcpy(v.data(), e->v, m * 4, kind));
  if (weights) DC_HIP(hipMemcpy(w.data(), e->w, m * 4, kind));
}

// Upper estimate of a context's device bytes (grow-only buffers, 25%
// headroom each) after a call that leaves `edges` undirected edges and sorted
// a batch of `changes` changes: per-vertex state, bins and labels (about 150
// B per vertex), the CSR double buffer and the coarsening and screening
// scratch sized by the entries (about 170 B per edge), the batch's records
// (about 240 B per change).  dc_init's own sort buffers are released before
// it returns.  Admission reserves these; after each round the reservations
// are replaced by the measured footprints.
int64_t est_step_bytes(int64_t n, int64_t edges, int64_t changes) {
  return 160 * n + 192 * edges + 256 * changes + (int64_t(1) << 18);
}
int64_t est_init_bytes(int64_t n, int64_t edges) { return est_step_bytes(n, edges, 0); }

bool edges_ok(const dc_edges* e, bool weights) {
  return !e || e->count == 0 ||
         (e->count > 0 && e->u && e->v && (!weights || e->w));
}

}  // namespace

struct dc_server {
  dc_options opt{};
  int64_t budget = 0;
  int32_t max_inflight = 1;
  int device = 0;
  hipStream_t st = nullptr;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  std::deque<Graph> graphs;  // stable addresses as graphs are added
  std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
  std::deque<int64_t> queue;  // waiting tickets in arrival order
  int64_t next_ticket = 1;
  int64_t round_no = 0;
  int64_t resident_bytes = 0;
  dc_server_stats stats{};
  MergeScratch X;

  void run();
  bool admit(Graph& g, int64_t need, const std::vector<Graph*>& all);
  void finish(Request* r, dc_status s);
};

// Makes room for `need` more bytes by moving idle resident graphs to host
// memory, least recently used first.  False if not enough can be freed.
bool dc_server::admit(Graph& g, int64_t need, const std::vector<Graph*>& all) {
  if (budget <= 0) return true;
  while (resident_bytes + need > budget) {
    Graph* victim = nullptr;
    for (Graph* h : all)
      if (h != &g && h->resident && !h->busy && h->ctx &&
          (!victim || h->last_used < victim->last_used))
        victim = h;
    if (!victim) return false;
    ctx_evict(victim->ctx, victim->saved);
    victim->resident = false;
    resident_bytes -= victim->footprint;
    stats.evictions++;
  }
  return true;
}

void dc_server::finish(Request* r, dc_status s) {
  r->result = s;
  r->done_ns = mono_ns();
}

void dc_server::run() {
  (void)hipSetDevice(device);
  for (;;) {
    std::vector<Request*> round;
    std::vector<Graph*> all;  // the graphs as of this round (the deque may grow meanwhile)
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || !queue.empty(); });
      if (queue.empty() && stop) return;
      for (Graph& g : graphs) all.push_back(&g);
      // the oldest waiting batch of each idle graph, up to max_inflight
      for (auto it = queue.begin(); it != queue.end() && int(round.size()) < max_inflight;) {
        Request* r = reqs[*it].get();
        Graph& g = graphs[size_t(r->gid)];
        bool taken = false;
        for (Request* q : round) taken = taken || q->gid == r->gid;
        if (g.busy || taken) {
          ++it;
          continue;
        }
        g.busy = true;
        round.push_back(r);
        it = queue.erase(it);
      }
    }
    if (round.empty()) {  // every waiting batch's graph is busy: cannot happen
      std::this_thread::sleep_for(std::chrono::microseconds(50));
      continue;
    }
    round_no++;
    std::vector<Request*> run_now, deferred;
    // admission in arrival order
    for (Request* r : round) {
      Graph& g = *all[size_t(r->gid)];
      try {
        // every admitted request reserves its estimated bytes, so several
        // requests of one round never share the same headroom
        if (r->init) {
          const int64_t need = est_init_bytes(r->n, g.edges);
          if (budget > 0 && need > budget) {
            finish(r, DC_E_OOM);
            continue;
          }
          if (!admit(g, need, all)) {
            deferred.push_back(r);
            continue;
          }
          resident_bytes += need;
        } else {
          const int64_t changes = int64_t(r->au.size() + r->du.size());
          int64_t want = est_step_bytes(r->n, g.edges + int64_t(r->au.size()), changes);
          if (want < g.footprint) want = g.footprint;
          if (budget > 0 && g.footprint > budget) {
            finish(r, DC_E_OOM);
            continue;
          }
          if (budget > 0 && want > budget) want = budget;  // runs with nothing else resident
          const int64_t need = g.resident ? want - g.footprint : want;
          if (!admit(g, need, all)) {
            deferred.push_back(r);
            continue;
          }
          resident_bytes += need;
          if (!g.resident) {
            ctx_restore(g.ctx, g.saved);
            g.saved = SavedState{};
            g.resident = true;
            stats.restores++;
          }
        }
        r->start_ns = mono_ns();
        run_now.push_back(r);
      } catch (const std::exception&) {
        finish(r, DC_E_DEVICE);
      }
    }
    // fronts (and whole init requests); then merged level-0 sweeps
    std::vector<dc_ctx*> cs;
    std::vector<LevelRun> Ls;
    std::vector<Request*> swept;
    cs.reserve(run_now.size());
    Ls.reserve(run_now.size());
    for (Request* r : run_now) {
      Graph& g = *all[size_t(r->gid)];
      if (r->init) {
        dc_edges e{int64_t(r->au.size()), r->au.data(), r->av.data(), r->aw.data(), 0, 0};
        dc_options o = opt;
        o.stream = st;
        dc_ctx* c = nullptr;
        const dc_status s = dc_init(&c, r->n, &e, &o);
        if (s == DC_OK) {
          g.ctx = c;
          g.resident = true;
          r->stats = c->stats;
        }
        finish(r, s);
        continue;
      }
      dc_ctx* c = g.ctx;
      if (c->poisoned) {
        finish(r, DC_E_STATE);
        continue;
      }
      try {
        r->t0_ms = std::chrono::duration<double, std::milli>(
                       std::chrono::steady_clock::now().time_since_epoch())
                       .count();
        dc_edges add{int64_t(r->au.size()), r->au.data(), r->av.data(), r->aw.data(), 0, 0};
        dc_edges del{int64_t(r->du.size()), r->du.data(), r->dv.data(), nullptr, 0, 0};
        const int32_t* act = nullptr;
        int64_t nact = 0;
        const dc_status s = apply_front(c, &add, &del, &act, &nact);
        if (s != DC_OK) {
          finish(r, s);
          continue;
        }
        if (c->opt.algorithm == DC_ALGO_SLM) {
          // SLM refines level 0 after its local moving: its levels run whole
          run_levels(c, act, nact);
          r->C.resize(size_t(c->n));
          apply_output(c, r->C.data(), 0);
          c->stats.ms_total = std::chrono::duration<double, std::milli>(
                                  std::chrono::steady_clock::now().time_since_epoch())
                                  .count() -
                              r->t0_ms;
          r->stats = c->stats;
          finish(r, DC_OK);
          continue;
        }
        // the screening pass's first-sweep decisions, as in run_levels
        const int64_t npre = act ? c->pre_count : 0;
        const uint8_t* skip = nullptr;
        if (npre > 0) {
          apply_pre(c->pre_list, npre, c->R.as<uint8_t>(), c->pre.as<int32_t>(),
                    c->Cn.as<int32_t>(), c->st);
          skip = c->pre_skip;
        }
        LevelRun L;
        levels_begin(c, act, nact, L, skip);
        L.pre_done = skip != nullptr;
        cs.push_back(c);
        Ls.push_back(L);
        swept.push_back(r);
      } catch (const DeviceError&) {
        c->poisoned = true;
        finish(r, DC_E_DEVICE);
      }
    }
    if (!swept.empty()) {
      std::vector<long long> gains(swept.size(), 0);
      bool ok = true;
      try {
        level0_merged(cs.data(), Ls.data(), gains.data(), int(swept.size()), X);
      } catch (const std::exception&) {
        ok = false;
      }
      for (size_t j = 0; j < swept.size(); ++j) {
        Request* r = swept[j];
        dc_ctx* c = cs[j];
        if (!ok) {
          c->poisoned = true;
          finish(r, DC_E_DEVICE);
          continue;
        }
        try {
          levels_finish(c, Ls[j], gains[j]);
          r->C.resize(size_t(c->n));
          apply_output(c, r->C.data(), 0);
          const double now = std::chrono::duration<double, std::milli>(
                                 std::chrono::steady_clock::now().time_since_epoch())
                                 .count();
          c->stats.ms_total = now - r->t0_ms;
          r->stats = c->stats;
          finish(r, DC_OK);
        } catch (const DeviceError&) {
          c->poisoned = true;
          finish(r, DC_E_DEVICE);
        }
      }
      for (size_t j = 0; j < swept.size(); ++j) all[size_t(swept[j]->gid)]->edges = cs[j]->nnz / 2;
      if (swept.size() > 1) stats.merged_rounds++;
      stats.merged_graphs += int64_t(swept.size());
    }
    // footprints after the round (buffers grow with the graphs)
    int64_t total = 0;
    for (Graph* g : all) {
      if (g->resident && g->ctx) g->footprint = ctx_footprint(g->ctx);
      if (g->resident) total += g->footprint;
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      resident_bytes = total;
      if (total > stats.peak_resident_bytes) stats.peak_resident_bytes = total;
      stats.rounds++;
      for (Request* r : round) {
        all[size_t(r->gid)]->busy = false;
        if (r->result != DC_PENDING) r->status = r->result;  // deferred ones stay pending
      }
      for (Request* r : run_now) {
        all[size_t(r->gid)]->last_used = round_no;
        if (r->status == DC_OK && !r->init) stats.batches++;
      }
      // a deferred batch goes back to the front, keeping arrival order
      for (auto it = deferred.rbegin(); it != deferred.rend(); ++it) {
        queue.push_front((*it)->ticket);
        stats.deferred++;
      }
    }
    cv_done.notify_all();
    if (!deferred.empty() && run_now.empty())  // nothing could run: wait briefly
      std::this_thread::sleep_for(std::chrono::microseconds(200));
  }
}

extern "C" {

dc_status dc_server_create(dc_server** out, const dc_options* opt, int64_t budget_bytes,
                           int32_t max_inflight) {
  if (!out || !opt || max_inflight < 1 || max_inflight > 1024) return DC_E_ARG;
  *out = nullptr;
  dc_server* s = new (std::nothrow) dc_server();
  if (!s) return DC_E_OOM;
  s->opt = *opt;
  s->budget = budget_bytes;
  s->max_inflight = max_inflight;
  try {
    DC_HIP(hipGetDevice(&s->device));
    DC_HIP(hipStreamCreate(&s->st));
    s->X.cap = max_inflight;
    DC_HIP(hipHostMalloc(reinterpret_cast<void**>(&s->X.hdescs),
                         size_t(max_inflight) * sizeof(EvalArgs)));
    DC_HIP(hipHostMalloc(reinterpret_cast<void**>(&s->X.hdone), size_t(max_inflight) * 8));
    DC_HIP(hipHostMalloc(reinterpret_cast<void**>(&s->X.hgdesc),
                         size_t(max_inflight) * sizeof(MergedGraph)));
    DC_HIP(hipHostMalloc(reinterpret_cast<void**>(&s->X.hsegs),
                         2 * size_t(NBINS) * size_t(max_inflight) * sizeof(MultiSeg)));
  } catch (const DeviceError&) {
    dc_server_destroy(s);
    return DC_E_DEVICE;
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return DC_OK;
}

dc_status dc_server_add_graph(dc_server* s, int32_t n, const dc_edges* g1, int32_t* gid) {
  if (!s || n < 1 || !gid || !edges_ok(g1, true)) return DC_E_ARG;
  auto r = std::make_unique<Request>();
  r->init = true;
  r->n = n;
  try {
    copy_edges(g1, true, r->au, r->av, r->aw);
  } catch (const DeviceError&) {
    return DC_E_DEVICE;
  } catch (const std::bad_alloc&) {
    return DC_E_OOM;
  }
  Request* rp = r.get();
  int64_t t;
  int32_t id;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->graphs.emplace_back();
    Graph& g = s->graphs.back();
    g.n = n;
    g.edges = int64_t(rp->au.size());
    rp->gid = id = int32_t(s->graphs.size() - 1);
    rp->ticket = t = s->next_ticket++;
    rp->arrival_ns = mono_ns();
    s->reqs.emplace(t, std::move(r));
    s->queue.push_back(t);
    s->stats.graphs++;
  }
  s->cv_work.notify_one();
  // the poll releases the request: only the local copy of its id is used
  const dc_status st = dc_server_poll(s, t, 1, nullptr, nullptr, nullptr);
  *gid = st == DC_OK ? id : -1;
  return st;
}

dc_status dc_server_submit(dc_server* s, int32_t gid, const dc_edges* add, const dc_edges* del,
                           int64_t arrival_ns, int64_t* ticket) {
  if (!s || !ticket || !edges_ok(add, true) || !edges_ok(del, false)) return DC_E_ARG;
  auto r = std::make_unique<Request>();
  r->gid = gid;
  r->arrival_ns = arrival_ns;
  try {
    std::vector<int32_t> unused;
    copy_edges(add, true, r->au, r->av, r->aw);
    copy_edges(del, false, r->du, r->dv, unused);
  } catch (const DeviceError&) {
    return DC_E_DEVICE;
  } catch (const std::bad_alloc&) {
    return DC_E_OOM;
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (gid < 0 || size_t(gid) >= s->graphs.size() || !s->graphs[size_t(gid)].ctx)
      return DC_E_ARG;
    r->ticket = *ticket = s->next_ticket++;
    r->n = s->graphs[size_t(gid)].n;
    s->queue.push_back(r->ticket);
    s->reqs.emplace(r->ticket, std::move(r));
  }
  s->cv_work.notify_one();
  return DC_OK;
}

dc_status dc_server_poll(dc_server* s, int64_t ticket, int32_t wait, int32_t* C_out,
                         dc_step_stats* stats, int64_t* times) {
  if (!s) return DC_E_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return DC_E_ARG;
  Request* r = it->second.get();
  if (r->status == DC_PENDING) {
    if (!wait) return DC_PENDING;
    s->cv_done.wait(lk, [&] { return r->status != DC_PENDING; });
  }
  const dc_status st = r->status;
  if (st == DC_OK) {
    if (C_out && !r->C.empty()) std::memcpy(C_out, r->C.data(), r->C.size() * 4);
    if (stats) *stats = r->stats;
  }
  if (times) {
    times[0] = r->arrival_ns;
    times[1] = r->start_ns;
    times[2] = r->done_ns;
  }
  s->reqs.erase(it);
  return st;
}

dc_status dc_server_stats_get(dc_server* s, dc_server_stats* out) {
  if (!s || !out) return DC_E_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->resident_bytes = s->resident_bytes;
  return DC_OK;
}

void dc_server_destroy(dc_server* s) {
  if (!s) return;
  if (s->worker.joinable()) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv_work.notify_all();
    s->worker.join();
  }
  for (Graph& g : s->graphs) dc_destroy(g.ctx);
  if (s->X.hdescs) (void)hipHostFree(s->X.hdescs);
  if (s->X.hdone) (void)hipHostFree(s->X.hdone);
  if (s->X.hsegs) (void)hipHostFree(s->X.hsegs);
  if (s->X.hgdesc) (void)hipHostFree(s->X.hgdesc);
  if (s->st) (void)hipStreamDestroy(s->st);
  delete s;
}

}  // extern "C"
