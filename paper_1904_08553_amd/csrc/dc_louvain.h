// dc_louvain.h -- launchers of the level, screening and coarsening kernels.
#pragma once

#include "dc_kernels.h"

namespace dc {

// Slots of the int64 device status block shared by the kernels of one call.
enum StatSlot : int {
  ST_MOVES = 0,    // movers of the current sweep
  ST_TOUCHED = 1,  // labels touched by the current sweep
  ST_DI = 2,       // change of the intra-community weight I
  ST_DS = 3,       // change of sum a^2
  ST_DN = 4,       // exact change of N = 2m*I - sum a^2
  ST_KEEP = 5,     // 1: the sweep was applied
  ST_DS_SRC = 6,   // Alg. 2 sources examined
  ST_DS_ACC = 7,   // Alg. 2 sources accepted
  ST_DEL_SRC = 8,
  ST_DEL_ACC = 9,
  ST_I = 10,       // modularity: intra weight
  ST_S = 11,       // modularity: sum of squares
  ST_N0 = 12,      // scratch counters (sizes read by the host)
  ST_N1 = 13,
  ST_N2 = 14,
  ST_N3 = 15,
  ST_FLAGS = 16,   // batch validation flags (int32 in the low half)
  ST_CASC_CAND = 19,  // cascade candidates (int32 in the low half)
  ST_CASC_EXP = 20,   // cascade candidates whose neighbourhood joined R
  ST_ERR = 21,        // self-checks of the kernels (bit 0: a hub-row table past its buffer)
  ST_MARK = 22,       // Alg. 2: accepted row chunks listed for marking
  ST_ACCVOL = 23,     // Alg. 2: entries of the accepted sources' rows
  ST_WSUM_ADD = 24,   // inserted weight: SUM_SLOTS counters
  ST_WSUM_DEL = ST_WSUM_ADD + SUM_SLOTS,  // deleted weight: SUM_SLOTS counters
  ST_NSRC = ST_WSUM_DEL + SUM_SLOTS,      // screening set: Alg. 2 sources (SUM_SLOTS)
  ST_NDSRC = ST_NSRC + SUM_SLOTS,         // and deletion endpoints (SUM_SLOTS)
  ST_COUNT = ST_NDSRC + SUM_SLOTS
};

// The total of the SUM_SLOTS counters from `base` of a status block copy.
inline long long slot_total(const long long* h, int base) {
  long long t = 0;
  for (int i = 0; i < SUM_SLOTS; ++i) t += h[base + i];
  return t;
}

// EV_FEAT: e_{i->C(i)} and the gains to the best and second-best other
// neighbouring community, the integer inputs of the screener features.
// EV_DSBOTH: Alg. 2 and the deletion rule in one pass over the union of
// the insertion sources and the deletion endpoints (EvalArgs::uflag).
enum EvalMode : int { EV_SWEEP = 0, EV_DSADD = 1, EV_DSDEL = 2, EV_FEAT = 3, EV_DSBOTH = 4 };
constexpr long long NO_GAIN = (long long)0x8000000000000000ull;

// Row-length bins of the evaluation kernels (eval.hip): rows of at most 16,
// 32 and 64 entries (4, 2 and 1 vertices per wave, no table), then
constexpr int NBINS = 6;
constexpr int WTAB_MAX = 512;     // one wave, wave-private LDS table
constexpr int WTAB_SLOTS = 1024;  // (merged sweeps; single graphs use 512 slots
                                  // and a full-table retry on overflow)
constexpr int BTAB_MAX = 4096;    // one block, block LDS table
constexpr int BTAB_SLOTS = 8192;  // beyond: one block, global table
constexpr int TIMED_BINS = 3;     // the timing option brackets the launch of bins [0, 3)

struct LevelView {
  int32_t n;
  int64_t nnz;
  const int32_t* off;
  const int2* adj;
  const int32_t* k;
};

// Arguments of the evaluation kernels for one graph (one level).
struct EvalArgs {
  const int32_t* off;
  const int2* adj;
  const int32_t* k;
  const int32_t* C;   // labels read (snapshot)
  int32_t* Cn;        // next labels (EV_SWEEP)
  const int32_t* a;   // community totals by label
  const int32_t* sz;  // community sizes by label
  long long two_m;
  int32_t guard;
  const int32_t* list;   // vertices (or sources) of this bin
  const int32_t* list_rb;  // their row starts (set for bins built by make_bins)
  int64_t nnz;             // adjacency entries of the level graph
  const int32_t* count;  // device count of list
  int* gkeys;            // bin G tables: row idx owns slots [tab_off[idx], tab_off[idx + 1])
  int* gvals;
  const long long* tab_off;
  int64_t gslots;        // slots of gkeys / gvals
  int32_t* ovf_list;     // bins W and B: vertices whose labels overflowed the
  int32_t* ovf_count;    // small LDS table (device count)
  long long* stat;
  const uint64_t* ins_keys;  // Alg. 2: sorted directed insertions src*n0+dst
  const int32_t* seg_beg;    // per source vertex: its sinks are ins_keys[beg, end)
  const int32_t* seg_end;
  int64_t n_ins;
  int32_t n0;
  uint8_t* R;
  uint8_t* cflag;
  uint8_t* accflag;  // EV_DSADD: accepted sources flagged here (null: not kept)
  long long* sink_g;   // Alg. 2: per record q of ins_keys, G(src -> C(dst))
  int32_t* best_j;     // Alg. 2: per source, j* when its best gain is positive, else -1
  long long* best_g;   // Alg. 2: per such source, gain1
  const uint8_t* uflag;  // EV_DSBOTH: bit 0 insertion source, bit 1 deletion endpoint
  int32_t* pre;  // EV_DSBOTH (may be null): each evaluated vertex's first-sweep label
  int32_t* f_own;  // EV_FEAT outputs, indexed by vertex
  long long* f_g1;
  long long* f_g2;
};

struct BinScratch;

struct Bins {
  int64_t n[NBINS];
  const int32_t* list[NBINS];
  const int32_t* list_rb[NBINS];  // row start (off[v]) of each listed vertex
  long long vol[NBINS];       // adjacency entries of each bin
  int64_t total = 0;          // vertices binned (the sum of n)
  const int32_t* count_dev;   // NBINS device counts
  // each bin's list starts with the vertices that make_bins' skip flags
  // leave unset: their number, volume and device counts
  int64_t n_first[NBINS];
  long long vol_first[NBINS];
  const int32_t* count_first_dev;
  int* gkeys;
  int* gvals;
  const long long* tab_off;
  int64_t gslots;      // slots of gkeys / gvals
  int32_t* ovf_list;   // rows of bins W and B re-evaluated with the full table
  int32_t* ovf_count;  // their device count (cleared by the re-evaluation)
  int32_t* ovf_done;   // blocks of the re-evaluation that have finished
  hipStream_t side;    // the hub-row bin runs here, overlapping the other
  hipEvent_t fork;     // bins (null: on the caller's stream)
  hipEvent_t join;
};

// The bins restricted to their first parts (the vertices not skipped).
inline Bins first_part(const Bins& b) {
  Bins f = b;
  for (int q = 0; q < NBINS; ++q) {
    f.n[q] = b.n_first[q];
    f.vol[q] = b.vol_first[q];
  }
  f.count_dev = b.count_first_dev;
  return f;
}

struct BinScratch {
  DBuf lists, lists_rb, bcnt, boff, bvol, counts, tab_off, gkeys, gvals, ovf;
  void* host = nullptr;      // pinned, 256 bytes
  void* host_dev = nullptr;  // its address for the kernels that write it
  hipStream_t side = nullptr;  // second stream and fork / join events of the
  hipEvent_t fork = nullptr;   // evaluation launches (owned by the context)
  hipEvent_t join = nullptr;
};

// Splits a vertex list (null = all of [0, count)) into the row-length bins,
// keeping list order within a bin; synchronises to read the bin sizes.
// skip (may be null): vertices v with skip[v] != 0 go to the end of their
// bin, after the first part (first_part gives the bins without them).
// dcount (may be null): the list's length in device memory, count then
// being a bound of it; the length is known after the call as b.total, so
// the caller needs no wait of its own to read it.  copy_src (may be null):
// copy_n int64 slots copied to copy_dst (device-visible pinned host memory)
// before the same wait, e.g. a status block the caller reads with the bins.
// coarse: the graph of a level above 0, whose rows hold mostly distinct
// labels (rows past half of WTAB_MAX go to the block-table bin).
void make_bins(const int32_t* list, int64_t count, const int32_t* off, Bins& b, BinScratch& s,
               hipStream_t st, const uint8_t* skip = nullptr, const int32_t* dcount = nullptr,
               const long long* copy_src = nullptr, long long* copy_dst = nullptr,
               int copy_n = 0, bool coarse = false);

// Clears the per-sweep counters of the status block (before the first
// sweep of a level; each sweep_apply clears them again for the next one).
void sweep_reset(long long* stat, hipStream_t st);
// Writes the next label of every active vertex that moves.  ev0/ev1 (may be
// null) bracket the one launch of bins [0, TIMED_BINS) (rows of at most 64
// entries), the kernel that carries the most vertices.
void sweep_eval(const LevelView& g, const int32_t* C, int32_t* Cn, const int32_t* a,
                const int32_t* sz, long long two_m, int guard, const Bins& bins,
                long long* stat, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1);
// Collects movers from the active list (null = all of [0, n_active)),
// applies them, computes the exact Delta N and keeps or reverts the sweep.
// The sweep's status block (ST_COUNT slots, ST_DN and ST_KEEP filled in)
// is written to host_stat, a device-visible address of pinned host memory,
// by the last kernel: after a wait on the stream it is there, with no copy.
// done: DONE_WORDS zeroed words (finished-block counters).
void sweep_apply(const LevelView& g, const int32_t* active, int64_t n_active, int32_t* C,
                 int32_t* Cn, int32_t* a, int32_t* sz, long long two_m, int32_t* movers,
                 long long* dpack, int32_t* tflag, int32_t* tlist, long long* stat,
                 unsigned* done, long long* host_stat, hipStream_t st);

// Scratch of one Alg. 2 pass: per directed insertion record its gain
// (sink_g, n_ins entries), per vertex the best sink and gain1 (best_j,
// best_g, n entries), the accepted rows' chunks (items, item_cap entries from
// ds_item_cap) and their count (a zeroed device counter).
struct DsScratch {
  long long* sink_g;
  int32_t* best_j;
  long long* best_g;
  int2* items;
  long long* item_count;
  int64_t item_cap;
};
int64_t ds_item_cap(int64_t n_sources, int64_t nnz);

// seg_beg/seg_end: per source vertex, its sinks are ins_keys[beg, end).
void ds_additions(const LevelView& g, const int32_t* C, const int32_t* a, long long two_m,
                  const uint64_t* ins_keys, int64_t n_ins, const int32_t* seg_beg,
                  const int32_t* seg_end, const Bins& bins, uint8_t* R, uint8_t* cflag,
                  uint8_t* accflag, const DsScratch& X, long long* stat, hipStream_t st);

// Alg. 2 over the insertion sources and the deletion rule over the deletion
// endpoints in one evaluation pass: bins hold the union, uflag[v] bit 0
// marks an insertion source (its sinks in ins_keys[seg_beg[v], seg_end[v])),
// bit 1 a deletion endpoint (the deletion rule, extension: a move with a
// positive gain adds the endpoint, its neighbours and the members of its best
// community).  Same effect as running the two screenings one after the other.
// pre (may be null): every listed vertex's decision of the first level-0
// sweep from the same state (labels C, totals a, sizes sz, singleton guard
// as guard): the best community if it moves, else its own label.
void ds_both(const LevelView& g, const int32_t* C, const int32_t* a, const int32_t* sz,
             int32_t guard, long long two_m, const uint64_t* ins_keys, int64_t n_ins,
             const int32_t* seg_beg, const int32_t* seg_end, const uint8_t* uflag,
             const Bins& bins, uint8_t* R, uint8_t* cflag, uint8_t* accflag, int32_t* pre,
             const DsScratch& X, long long* stat, hipStream_t st);
// uflag[v] |= 1 for v in list[0, *count) (count on the device); then
// uflag[v] |= 2 where dflag[v] != 0, flag[v] = uflag[v] != 0, and
// *ndel += the number of such v.
void union_flags(const int32_t* list, const int32_t* count, int64_t max_count,
                 const int32_t* dflag, int32_t n, uint8_t* uflag, int32_t* flag, long long* ndel,
                 hipStream_t st);

// Cascade-aware screening (extension of Alg. 2; see dc_options.cascade_*):
// cand[v] = 1 for every neighbour v != i of a flagged accepted source i of
// list[0, cnt) with C[v] == C[i].
void cascade_candidates(const int32_t* list, int64_t cnt, const uint8_t* accflag,
                        const int32_t* off, const int2* adj, const int32_t* C, uint8_t* cand,
                        hipStream_t st);
// For v in list[0, cnt) with f_g1[v] != NO_GAIN and
// f_g1[v] * den >= -num * two_m * k[v] (exact, 128-bit): R[v] = 1 and R of
// its neighbours = 1; *expanded += the number of such v.
void cascade_mark(const int32_t* list, int64_t cnt, const long long* f_g1, const int32_t* k,
                  long long two_m, long long num, long long den, const int32_t* off,
                  const int2* adj, uint8_t* R, long long* expanded, hipStream_t st);


// ---- merged sweeps of several graphs (one launch per row-length bin) ----
// The bins of several graphs concatenated, each graph's part padded to whole
// waves (list entry -1), with the graph index of every item; for the
// hub-row bin also the item's index within its graph's bin (its hash-table
// slice).
struct MultiBins {
  DBuf list[NBINS], gid[NBINS], lidx;
  int64_t count[NBINS] = {};
};

// One graph's level-0 sweep state for the merged bookkeeping kernels
// (merged.hip): its level graph, labels, totals, active list, scratch of the
// moves, status block, threshold T, sweep limit and the device record of
// its sweeps (moves, Delta N, kept: three int64 per sweep).
struct MergedGraph {
  const int32_t* off;
  const int2* adj;
  const int32_t* k;
  int32_t* C;
  int32_t* Cn;
  int32_t* a;
  int32_t* sz;
  const int32_t* act;  // null: every vertex of [0, nact)
  int64_t nact;
  long long* dpack;
  int32_t* tflag;
  int32_t* tlist;
  int32_t* movers;
  long long* stat;
  long long two_m;
  long long T;
  int32_t max_sweeps;
  int32_t pad;
  long long* rec;
};
// state[j]: 0 running, 1 stopped in the current round, 2 stopped.
void merged_reset(const MergedGraph* G, int m, int32_t* state, hipStream_t st);
// Apply, exact Delta N, keep / revert / stop and commit of one sweep of every
// running graph (max_nact: the longest active list).
void merged_apply(const MergedGraph* G, int m, int64_t max_nact, int32_t* state,
                  int32_t* sweeps, hipStream_t st);
struct MultiSeg {  // one graph's bin, for build_multi_bins
  const int32_t* src;
  int64_t n, padded, dst;
  int32_t gid, bin;
};
// Sweep arguments of one graph's level (the `list`/`count` fields unused).
EvalArgs sweep_args(const LevelView& g, const int32_t* C, int32_t* Cn, const int32_t* a,
                    const int32_t* sz, long long two_m, int guard, long long* stat);
// Merges bins[0..ngraphs) (graph j's bins at position j); segs_host: pinned
// scratch of NBINS * ngraphs MultiSeg, segs_dev: device scratch.
void build_multi_bins(const Bins* const* bins, int ngraphs, MultiBins& mb, MultiSeg* segs_host,
                      DBuf& segs_dev, hipStream_t st);
// One sweep evaluation of every graph j with done[j] == 0 over the merged
// bins, the hub-row bin included (descs[j]: its sweep arguments with its
// hub-row tables, device memory).
void sweep_eval_multi(const EvalArgs* descs, const int32_t* done, const MultiBins& mb,
                      hipStream_t st);
// The sweep arguments of graph j's level with its hub-row tables.
EvalArgs sweep_args_bins(const LevelView& g, const int32_t* C, int32_t* Cn, const int32_t* a,
                         const int32_t* sz, long long two_m, int guard, long long* stat,
                         const Bins& bins);


// Per listed vertex i: f_own[i] = e_{i->C(i)}, f_g1[i] / f_g2[i] = scaled
// gains to the best / second-best other neighbouring community (score
// descending, label ascending), NO_GAIN when absent.  pre (may be null):
// also the label a sweep on the same state would give i (the singleton
// guard applied when guard is set, with the sizes sz).
void feat_eval(const LevelView& g, const int32_t* C, const int32_t* a, long long two_m,
               const Bins& bins, int32_t* f_own, long long* f_g1, long long* f_g2,
               long long* stat, hipStream_t st, const int32_t* sz = nullptr, int guard = 0,
               int32_t* pre = nullptr);

// ---- screen.hip ----
// out[pos[i]] = i for flag[i] != 0 (pos = exclusive scan of flag).
void compact_index(const int32_t* flag, const int32_t* pos, int64_t n, int32_t* out,
                   hipStream_t st);
// Insertion changes (op != DELETE) of the sorted change list, compacted.
void select_insertions(const int32_t* ch_op, int64_t nch, int32_t* flag, hipStream_t st);
void gather_u64(const uint64_t* in, const int32_t* flag, const int32_t* pos, int64_t n,
                uint64_t* out, hipStream_t st);
// flag[q] = 1 where the source of sorted directed keys changes; out ids.
void source_heads(const uint64_t* keys, int64_t m, int32_t n, int32_t* flag, hipStream_t st);
void gather_sources(const uint64_t* keys, const int32_t* flag, const int32_t* pos, int64_t m,
                    int32_t n, int32_t* out, hipStream_t st);
// seg_beg[src] / seg_end[src] = first / one-past-last index of src's keys.
void source_segments(const uint64_t* keys, int64_t m, int32_t n, int32_t* seg_beg,
                     int32_t* seg_end, hipStream_t st);
// dflag[src] = 1 for deleted pairs inside one community.
void deletion_sources(const uint64_t* ch_key, const int32_t* ch_op, int64_t nch, int32_t n,
                      const int32_t* C, int32_t* dflag, hipStream_t st);
// The fused screening set from the sorted change list (labels C = C_{t-1}):
// per source, uflag bit 0 (an insertion record: an Alg. 2 source, its sinks
// ins_keys[seg_beg, seg_end), ins_pos locating each record there) and bit
// 1 (an intra-community deletion); hflag[q] = 1 at the first change of
// each flagged source (nch entries); n_src / n_dsrc (SUM_SLOTS counters
// each) += the sources of each kind.  sbits (n ints) and uflag must be zero
// beforehand.
void screen_union(const uint64_t* ch_key, const int32_t* ch_op, const int32_t* ins_pos,
                  const uint64_t* ins_keys, int64_t n_ins, int64_t nch, int32_t n,
                  const int32_t* C, int32_t* sbits, uint8_t* uflag, int32_t* seg_beg,
                  int32_t* seg_end, int32_t* hflag, long long* n_src, long long* n_dsrc,
                  hipStream_t st);
// R[i] = 1 and R[Gamma(i)] = 1 for every listed vertex.
void mark_neighbourhoods(const int32_t* list, int64_t cnt, const int32_t* off, const int2* adj,
                         uint8_t* R, hipStream_t st);
// R[v] |= cflag[C[v]] (cflag null: R as it is), and the vertices with
// R[v] != 0 appended to list
// (*count, zero before the call, becomes their number; the order of the
// list is not fixed).
void materialize_R(uint8_t* R, const uint8_t* cflag, const int32_t* C, int32_t n,
                   int32_t* list, int32_t* count, hipStream_t st);
// Cn[v] = pre[v] for every listed v with R[v] != 0: the first sweep's
// decisions that the screening pass already took.
void apply_pre(const int32_t* list, int64_t cnt, const uint8_t* R, const int32_t* pre,
               int32_t* Cn, hipStream_t st);

// ---- slm.hip (smart local moving levels) ----
// The subgraph of the entries inside one community of C (diagonal included):
// cnt (n ints) scratch, off_s (n + 1 ints) its offsets, adj_s grown to fit;
// returns its entry count (one host read).
int64_t induced_subgraph(const LevelView& g, const int32_t* C, int32_t* cnt, int32_t* off_s,
                         DBuf& adj_s, void* host, hipStream_t st);
// Cnext[rank[R[u]]] = the smallest rank[R[v]] over v with P[v] == P[u]
// (first: n ints of scratch): the parents' partition over the coarse ids.
void parent_start(const int32_t* P, const int32_t* R, const int32_t* rank, int32_t n,
                  int32_t* first, int32_t* Cnext, hipStream_t st);
// a[X] = sum of k over members of label X, sz[X] = their number.
void totals_sizes(const int32_t* k, const int32_t* C, int32_t n, int32_t* a, int32_t* sz,
                  hipStream_t st);
// *count += the labels x < n with sz[x] > 0.
void nonempty_count(const int32_t* sz, int32_t n, long long* count, hipStream_t st);

// ---- coarsen.hip ----
struct CoarsenScratch {
  DBuf flag, rank, keys0, keys1, vals0, vals1, cntr, mstart, labof, mdeg, mvol, chead, cpos,
      chunks, mcnt, pk0, pk1, pv0, pv1, ph, pp, pS, pcnt, hidx, ukey, rc;
  void* host = nullptr;      // pinned, 64 bytes
  void* host_dev = nullptr;  // its address for the kernels that write it
  bool inc_check = false;    // coarsen_first_inc's self-check flag awaits a wait
};

struct CoarseGraph {
  DBuf off, adj, k;
  int32_t n = 0;
  int64_t nnz = 0;
  LevelView view() const {
    return LevelView{n, nnz, off.as<int32_t>(), adj.as<int2>(), k.as<int32_t>()};
  }
};

// Builds the next level from the partition C of g (Alg. 1 compaction): one
// coarse vertex per non-empty community, numbered by ascending label, with
// A'_{XY} = sum of the entries between the two communities (diagonal kept).
// Updates map0 (level-0 vertex -> vertex of the new level); cnt/minv of the
// new level from those of g (first_level: all ones / identity).
void coarsen(const LevelView& g, const int32_t* C, const int32_t* sz, const int32_t* a,
             const int32_t* cnt, const int32_t* minv, bool first_level, int32_t n0,
             int32_t* map0, CoarseGraph& out, int32_t* cnt_out, int32_t* minv_out,
             CoarsenScratch& s, hipStream_t st);

// ---- incremental first-level compaction (coarsen.hip) ----
// H(G, C): the graph of communities of the current graph and partition,
// keys X*n + Y over community labels, weights > 0, sorted and unique; plus
// the last level-1 graph (keys x*nc + y over coarse ids, weights) and the
// smallest level-0 member of each of its vertices, from which the next H
// is relabelled once the final labels are known.
struct IncCoarsen {
  int64_t h = 0;  // entries of H, at the front of ek0 / ev0
  bool valid = false;
  DBuf lkey, lw, lminv;
  int64_t lh = 0;
  int32_t lnc = 0;
  DBuf ek0, ek1, ev0, ev1, heads, hpos, v64, S, starts, nz, npos, mflag, mvol, tkey, tw;
};

// Level 0 -> 1 from H(G_{t-1}, C_{t-1}) instead of all of G_t: H plus the
// batch's directed changes mapped by Cold = C_{t-1} (ch_key / ch_dk, nch
// records) plus the rows of the level-0 movers (Cl != Cold) moved from their
// old labels to their new ones, summed by one sort; the result (entries of
// zero weight dropped) is the coarse graph of (G_t, Cl), numbered as
// coarsen() numbers it.  Outputs as coarsen(first_level = true).
void coarsen_first_inc(const LevelView& g, const int32_t* Cl, const int32_t* Cold,
                       const int32_t* sz, const int32_t* a, const uint64_t* ch_key,
                       const int32_t* ch_dk, int64_t nch, int32_t* map0, CoarseGraph& out,
                       int32_t* cnt_out, int32_t* minv_out, CoarsenScratch& s, IncCoarsen& H,
                       hipStream_t st);
// After the caller's next wait on the stream following coarsen_first_inc:
// raises its self-check (an entry of an empty community or of weight below
// 1 in the graph of communities), which the kernel reports in host memory.
void inc_check(CoarsenScratch& s);
// Keeps the level-1 graph just built (and its vertices' smallest members);
// coarsen_first_inc keeps its own as it builds it.
void save_level1(const CoarseGraph& out, const CoarsenScratch& s, const int32_t* minv,
                 IncCoarsen& H, hipStream_t st);
// H(G_t, C_t) from the saved level-1 graph and the final labels C_t: its
// entries relabelled, neither sorted nor merged (communities that merged
// above level 0 leave repeated keys); the next step's sort orders them and
// sums equal keys with the batch's and the movers' entries.
void inc_finish(IncCoarsen& H, const int32_t* Ct, int32_t n, CoarsenScratch& s,
                hipStream_t st);

// Canonical labels of the final partition (smallest level-0 id per
// community), the level-0 totals and sizes by label, and C_t.  zero2 (may
// be null): two int64 counters cleared on the way (the caller's next sums).
void finalize_labels(int32_t nL, const int32_t* CL, const int32_t* aL, const int32_t* szL,
                     const int32_t* cntL, const int32_t* minvL, int32_t n0, const int32_t* map0,
                     int32_t* lab, int32_t* cntf, int32_t* C0, int32_t* a0, int32_t* sz0,
                     hipStream_t st, long long* zero2 = nullptr);

}  // namespace dc
