// ctx.h -- the context behind dc_ctx and the phases of a time step, shared
// by the C ABI (api.hip) and the serving loop (server.hip).
#pragma once

#include <string>
#include <vector>

#include "dc_louvain.h"
#include "learned.h"

using namespace dc;

struct dc_ctx {
  int32_t n = 0;
  dc_options opt{};
  hipStream_t st = nullptr;
  bool poisoned = false;
  int64_t two_m = 0;
  int64_t nnz = 0;
  int cur = 0;
  DBuf off[2], adj[2];
  DBuf k0, C, a0, sz0;
  // batch
  DBuf in_au, in_av, in_aw, in_du, in_dv;
  DBuf dw_old;
  DBuf akeys, avals, ak1, av1, aheads, apos, ukeys, uw;
  DBuf rkeys, rvals, rk1, rv1, rheads, rpos;
  DBuf ch_key, ch_op, ch_w, ch_dk, dnet, cnet, cptr, new_deg, tile_row;
  DBuf ins_flag, ins_pos, ins_keys, src_flag, src_pos, src_list, dflag, dpos, dlist;
  DBuf R, cflag, rflag, rpos2, Rlist, seg_beg, seg_end, chsrc;
  DBuf accflag, cascand, clist;  // cascade-aware screening
  DBuf uflag, ulist;             // union of insertion sources and deletion endpoints
  DBuf pre;                      // first-sweep labels taken by the screening pass
  DBuf sink_g, best_j, best_g, ds_items;  // Alg. 2: gains per record, best sinks, marked rows
  DBuf sub_cnt, sub_off, sub_adj, par, first;  // SLM: induced subgraph, parent labels
  int64_t pre_count = 0;         // entries of pre_list that hold them (0: none)
  const int32_t* pre_list = nullptr;  // the vertices evaluated on the first sweep's state
  const uint8_t* pre_skip = nullptr;  // their flags (binned after the others at level 0)
  // learned screener: touched set, features, labels, scores
  DBuf kprev, tmark, tflag, tpos, Tlist, f_own, f_g1, f_g2, X, y, logits, scr_wq;
  bool have_scr = false;
  float theta = 0.f;
  int64_t T_count = 0;
  bool have_y = false, have_logits = false;
  // levels
  DBuf Cl, Cn, al, szl, dpack, lflag, tlist, movers, map0, cnt[2], minv[2], lab, cntf;
  CoarseGraph cg[2];
  DBuf stat;
  long long* hstat = nullptr;  // pinned mirror of the status block
  long long* hstat_dev = nullptr;  // its address for the kernels that write it
  DBuf done;                   // finished-block counters (DONE_WORDS, zero between launches)
  void* hbuf = nullptr;        // pinned scratch for the kernels' host reads
  int32_t* hbuf_dev = nullptr; // its address for the kernels that write it
  BinScratch bins;
  CoarsenScratch cs;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t evp[5] = {};      // phase boundaries of a timed dc_apply_batch
  bool phase_timing = false;   // record them (dc_apply_batch with timing = 1)
  std::vector<dc_sweep_rec> trace;
  dc_step_stats stats{};
  int32_t* out_C = nullptr;   // C_t's destination of the running dc_apply_batch (copied
  int32_t out_on_device = 0;  // with the last wait of the step)
  int64_t R_count = 0;
  const int32_t* R_dcount = nullptr;  // |R_t| in device memory, not yet read back
  bool have_R_all = true;
  // graph of communities kept across steps (incremental level-0 compaction)
  IncCoarsen inc;
  int64_t nch_last = 0;     // change records of the current batch
  int64_t n_ins_last = 0;   // its directed insertion records
  bool inc_ready = false;   // they belong to the step being run
};

namespace dc_core {

// Level-0 run of one context between levels_begin and levels_finish.
struct LevelRun {
  LevelView g;
  const int32_t* act;
  int64_t nact;
  long long T;
  Bins bins;
  bool pre_done = false;  // the first sweep takes only the bins' first parts
};

// Host-side copy of a context's resident state (G_t, labels, totals).
struct SavedState {
  std::vector<int32_t> off;
  std::vector<int2> adj;
  std::vector<int32_t> k, C, a, sz;
  int64_t nnz = 0, two_m = 0;
  int cur = 0;
};

// Scratch of merged level-0 sweeps over several contexts.
struct MergeScratch {
  MultiBins mb, mb0;              // every round's lists; the first round's when some
                                  // graph's screened vertices have their decisions
  DBuf descs, done, segs, segs0, gdesc, sweeps, rec;
  EvalArgs* hdescs = nullptr;     // pinned, cap entries
  int32_t* hdone = nullptr;       // pinned, 2 * cap entries: states, then sweep counts
  MultiSeg* hsegs = nullptr;      // pinned, 2 * NBINS * cap entries (mb, then mb0)
  MergedGraph* hgdesc = nullptr;  // pinned, cap entries
  int cap = 0;
};

dc_status apply_front(dc_ctx* c, const dc_edges* add, const dc_edges* del, const int32_t** act,
                      int64_t* nact);
void levels_begin(dc_ctx* c, const int32_t* active, int64_t n_active, LevelRun& L,
                  const uint8_t* skip = nullptr);
void levels_finish(dc_ctx* c, LevelRun& L, long long level0_gain);
void apply_output(dc_ctx* c, int32_t* C_out, int32_t out_on_device);
// All levels of one step (Louvain or SLM per the options), level 0 over
// `active` (null = every vertex); for graphs that do not merge level 0.
void run_levels(dc_ctx* c, const int32_t* active, int64_t n_active);
// Level-0 sweeps of m contexts sharing one stream, merged per round: the
// evaluation of every unfinished context in one launch per row-length bin,
// then each context's apply, one wait per round; gains[j] receives context
// j's level-0 gain.  Results are those of running each context alone.
void level0_merged(dc_ctx* const* cs, LevelRun* Ls, long long* gains, int m, MergeScratch& X);
// Device bytes a context holds.
int64_t ctx_footprint(const dc_ctx* c);
// Moves the resident state to the host and frees every device buffer of the
// context; ctx_restore brings it back (the next call rebuilds the rest).
void ctx_evict(dc_ctx* c, SavedState& s);
void ctx_restore(dc_ctx* c, const SavedState& s);

}  // namespace dc_core
