// eval.hip -- per-vertex evaluation of a vertex against the communities of
// its neighbours, the inner operation of both Louvain local moving (Alg. 1,
// the move rule of Sec. 3.2) and Delta-screening (Alg. 2, Sec. 3.5).
//
// For vertex i with label c the kernels form e_{i->X} (sum of w(i,v) over
// neighbours v != i with C(v) = X) and compare, in exact int64,
//     score(X) = 2m * e_{i->X} - k_i * a_X^{(-i)}
// (the gain of Sec. 3.1 scaled by (2m)^2/2; a^{(-i)} takes i out of c).
//
// Grouping equal labels is the hot operation.  Most neighbours of a vertex
// share one or a few communities, so a hash insert per entry would pile
// atomics onto the same slot.  Instead a wave loads 64 entries, picks the
// label of the first unprocessed lane, finds all lanes holding it with one
// ballot and parks the label in the lane numbered by the iteration: one
// register-only iteration per distinct label.  Each lane then adds its
// weight into a per-wave LDS slot of its label's rank.  The community totals are then gathered (or the table
// inserts issued) by all pair-holding lanes at once, so no chain of
// dependent memory accesses remains.  Rows of up to 64 entries finish this
// way (bin S, one wave per vertex).  Longer rows collect per 64-entry chunk
// and add the chunk's pairs to a hash table: wave-private LDS for rows up
// to 512 entries (bin W), a block-shared LDS table up to 4096 (bin B),
// global memory beyond (bin G).  A sweep writes only the next label;
// movers are collected afterwards.
#include "dc_louvain.h"

namespace dc {

namespace {

constexpr int TPB = 256;
constexpr int NW = TPB / WAVE;



__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }


struct Cand {  // Alg. 2 candidate: larger gain, then smaller C(j), then smaller j
  long long g;
  int x;
  int j;
};

__device__ __forceinline__ bool cand_better(const Cand& p, const Cand& q) {
  return p.g > q.g || (p.g == q.g && (p.x < q.x || (p.x == q.x && p.j < q.j)));
}


// Alg. 2 (gain2 from the mirror record).  Every insertion (i, j) is a pair of
// directed records i -> j and j -> i, so the best sink j* of a source i is
// itself a source with i among its sinks.  The evaluation pass stores, per
// directed record j -> i, the scaled gain G(j -> C(i)) on (G_t, C_{t-1}),
// and, per source i with a positive best gain, j* and gain1 = G(i -> C(j*)).
// Since gain1 > 0 implies C(j*) != C(i), gain2 = G(j* -> C(i)) of Alg. 2 is
// exactly the gain stored at the record j* -> i: k_ds_resolve compares the
// two, and no row is walked a second time.

// --------------------------------------------------------------------------
// bins S16/S32/S64: rows of at most GS entries, no table.  A wave is split
// into 64/GS groups of GS lanes, each group evaluating its own vertex: wave
// instructions cost the same for 16 or 64 busy lanes, so packing four
// 16-entry rows into one wave divides the instruction count per vertex by
// four.  Ballots stay wave-wide, each group's leader label is read with a
// scalar readlane, and reductions run within the group on DPP row
// exchanges.

template <int GS, int S = 0>
__device__ __forceinline__ long long group_sum_ll(long long v) {
  if constexpr ((1 << S) >= GS) {
    return v;
  } else if constexpr (S == 5) {
    return readlane64(v, 0) + readlane64(v, 32);
  } else {
    return group_sum_ll<GS, S + 1>(v + xchg64<S>(v));
  }
}

template <int GS, int S = 0>
__device__ __forceinline__ Best group_best_w(Best b) {
  if constexpr ((1 << S) >= GS) {
    return b;
  } else if constexpr (S == 5) {
    const Best b0 = {readlane64(b.s, 0), __builtin_amdgcn_readlane(b.x, 0)};
    const Best b1 = {readlane64(b.s, 32), __builtin_amdgcn_readlane(b.x, 32)};
    return better(b1.s, b1.x, b0.s, b0.x) ? b1 : b0;
  } else {
    const Best y = {xchg64<S>(b.s), xchg<S>(b.x)};
    return group_best_w<GS, S + 1>(better(y.s, y.x, b.s, b.x) ? y : b);
  }
}

template <int GS, int S = 0>
__device__ __forceinline__ Cand group_cand_w(Cand c) {
  if constexpr ((1 << S) >= GS) {
    return c;
  } else if constexpr (S == 5) {
    const Cand c0 = {readlane64(c.g, 0), __builtin_amdgcn_readlane(c.x, 0),
                     __builtin_amdgcn_readlane(c.j, 0)};
    const Cand c1 = {readlane64(c.g, 32), __builtin_amdgcn_readlane(c.x, 32),
                     __builtin_amdgcn_readlane(c.j, 32)};
    return cand_better(c1, c0) ? c1 : c0;
  } else {
    const Cand y = {xchg64<S>(c.g), xchg<S>(c.x), xchg<S>(c.j)};
    return group_cand_w<GS, S + 1>(cand_better(y, c) ? y : c);
  }
}

// Value of lane r (uniform) of each lane's own group.
template <int GS>
__device__ __forceinline__ int group_bcast(int v, int r) {
  constexpr int GPW = WAVE / GS;
  int out = 0;
#pragma unroll
  for (int g = 0; g < GPW; ++g) {
    const int x = __builtin_amdgcn_readlane(v, g * GS + r);
    if (int(lane_id()) / GS == g) out = x;
  }
  return out;
}

// The value of the lane of each lane's own group whose flag is set (at most
// one per group), 0 when none is: one ballot and a readlane per group.
template <int GS>
__device__ __forceinline__ int group_pick(bool flag, int v) {
  constexpr int GPW = WAVE / GS;
  const uint64_t m = __ballot(flag);
  int out = 0;
#pragma unroll
  for (int g = 0; g < GPW; ++g) {
    uint64_t sub;
    if constexpr (GPW == 1)
      sub = m;
    else
      sub = (m >> (g * GS)) & ((uint64_t(1) << GS) - 1);
    const int x = sub ? __builtin_amdgcn_readlane(v, g * GS + __builtin_ctzll(sub)) : 0;
    if (int(lane_id()) / GS == g) out = x;
  }
  return out;
}

// Per group: lane r of the group (r < returned count) receives the r-th
// distinct label of the group's valid lanes (order of first appearance)
// and its weight sum.  Each iteration takes, for every group of the wave at
// once, the label of the lowest lane not yet matched (scalar readlanes) and
// matches it with one ballot; afterwards every valid lane adds its weight
// into the LDS slot of its label's rank.  lsum: the wave's 64 ints, zero on
// entry and on return.
// probe / prank (may be null): each lane's rank of label `probe` among its
// group's distinct labels, -1 when absent (found as the labels are taken).
template <int GS>
__device__ __forceinline__ int group_collect(bool valid, int key, int w, int* lsum, int& ck,
                                             int& cs, int* iters = nullptr, int probe = 0,
                                             int* prank = nullptr) {
  constexpr int GPW = WAVE / GS;
  const int lane = lane_id();
  const int gl = lane & (GS - 1);
  const int grp = lane / GS;
  uint64_t rem = __ballot(valid);
  int r = 0, myr = 0, it = 0, pr = -1;
  while (rem) {
    ++it;
    int kl = 0;
    bool act = false;
#pragma unroll
    for (int g = 0; g < GPW; ++g) {
      uint64_t sub;
      if constexpr (GPW == 1)
        sub = rem;
      else
        sub = (rem >> (g * GS)) & ((uint64_t(1) << GS) - 1);
      if (sub) {
        const int kg = __builtin_amdgcn_readlane(key, g * GS + __builtin_ctzll(sub));
        if (grp == g) {
          kl = kg;
          act = true;
        }
      }
    }
    const bool mine = act && valid && key == kl;
    rem &= ~__ballot(mine);
    if (mine) myr = r;
    if (act && gl == r) ck = kl;
    if (prank && act && probe == kl) pr = r;
    r += act ? 1 : 0;
  }
  if (prank) *prank = pr;
  if (valid) atomicAdd(&lsum[lane - gl + myr], w);
  wave_sync();
  cs = gl < r ? lsum[lane] : 0;
  lsum[lane] = 0;
  wave_sync();
  if (iters) *iters = it;  // wave-uniform: the largest count of any group
  return r;
}

// Best (score, label) of lanes [0, 2^steps) of each group, in the group's
// first lane (the other lanes hold partial results): candidates sit in the
// first nd lanes of a group, so ceil(log2(nd)) butterfly steps suffice.
template <int GS>
__device__ __forceinline__ Best group_best_first(Best b, int nd_max) {
  if (nd_max > 1) b = best_step<0>(b);
  if (nd_max > 2) b = best_step<1>(b);
  if (nd_max > 4) b = best_step<2>(b);
  if (GS > 8 && nd_max > 8) b = best_step<3>(b);
  if (GS > 16 && nd_max > 16) b = best_step<4>(b);
  if (GS > 32 && nd_max > 32) {
    const Best y = {readlane64(b.s, 32), __builtin_amdgcn_readlane(b.x, 32)};
    const Best z = {readlane64(b.s, 0), __builtin_amdgcn_readlane(b.x, 0)};
    b = better(y.s, y.x, z.s, z.x) ? y : z;
  }
  return b;
}

// Best Alg. 2 candidate of each group, in the group's first lane, as
// group_best_first: candidates sit in the first n lanes of a group (n, the
// group's candidate count, held by every lane of the group), so a step runs
// only when some group of the wave needs it.
template <int GS>
__device__ __forceinline__ Cand group_cand_first(Cand c, int n) {
  auto step = [](Cand v, auto s) {
    constexpr int S = decltype(s)::value;
    const Cand y = {xchg64<S>(v.g), xchg<S>(v.x), xchg<S>(v.j)};
    return cand_better(y, v) ? y : v;
  };
  if (__ballot(n > 1)) c = step(c, std::integral_constant<int, 0>{});
  if (__ballot(n > 2)) c = step(c, std::integral_constant<int, 1>{});
  if (__ballot(n > 4)) c = step(c, std::integral_constant<int, 2>{});
  if (GS > 8 && __ballot(n > 8)) c = step(c, std::integral_constant<int, 3>{});
  if (GS > 16 && __ballot(n > 16)) c = step(c, std::integral_constant<int, 4>{});
  if (GS > 32 && __ballot(n > 32)) {
    const Cand y = {readlane64(c.g, 32), __builtin_amdgcn_readlane(c.x, 32),
                    __builtin_amdgcn_readlane(c.j, 32)};
    const Cand z = {readlane64(c.g, 0), __builtin_amdgcn_readlane(c.x, 0),
                    __builtin_amdgcn_readlane(c.j, 0)};
    c = cand_better(y, z) ? y : z;
  }
  return c;
}

// Accepted screening tests, counted in one integer: insertion sources (Alg.
// 2, counted by k_ds_resolve) in the low 32 bits, deletion endpoints in the
// high 32 bits.
constexpr long long ACC_DEL = 1ll << 32;

__device__ __forceinline__ void add_accepted(long long* stat, long long acc) {
  const long long add = acc & 0xffffffffll, del = acc >> 32;
  if (add) atomicAdd((unsigned long long*)&stat[ST_DS_ACC], (unsigned long long)add);
  if (del) atomicAdd((unsigned long long*)&stat[ST_DEL_ACC], (unsigned long long)del);
}

// Sweep decision of vertex i: the group's first lane writes the next label
// unless the singleton guard (Sec. 3.2) holds the move back.
__device__ __forceinline__ void sweep_commit(const EvalArgs& A, int i, bool move, int c, int x,
                                             int gl) {
  if (move && gl == 0) {
    if (!(A.guard && A.sz[c] == 1 && A.sz[x] == 1 && x > c)) A.Cn[i] = x;
  }
}

// The same decision kept for the first level-0 sweep (EV_DSBOTH with pre):
// the label it would write, or the vertex's own label when it stays.
__device__ __forceinline__ void pre_commit(const EvalArgs& A, int i, bool move, int c, int x) {
  const bool held = move && A.guard && A.sz[c] == 1 && A.sz[x] == 1 && x > c;
  A.pre[i] = move && !held ? x : c;
}

// One item of a group kernel: group (lane / GS) of the wave evaluates vertex
// i (have = false: no vertex, the lanes still take part in the wave-wide
// steps).  EV_SWEEP: the sweep decision (the merged multi-graph sweep);
// EV_DSADD: Alg. 2 for an insertion source (its gain toward each sink's
// label, stored per record, and its best sink); EV_DSDEL: the deletion rule
// for a deletion endpoint (the conservative-rule path runs the two tests in
// separate passes).  Returns the deletion tests accepted (0 or ACC_DEL).
template <int MODE, int GS>
__device__ __forceinline__ long long group_item(const EvalArgs& A, int i, bool have, int lane,
                                                int gl, int gbase, int* lsum) {
  static_assert(MODE == EV_SWEEP || MODE == EV_DSADD || MODE == EV_DSDEL,
                "the paired kernels take the other modes");
  long long accepted = 0;
  const int32_t rb = have ? A.off[i] : 0;
  const int32_t re = have ? A.off[i + 1] : 0;
  const int c = have ? A.C[i] : 0;
  const long long ki = have ? A.k[i] : 0;
  const int2 e = rb + gl < re ? A.adj[rb + gl] : make_int2(-1, 0);
  const bool valid = e.x >= 0 && e.x != i;
  const int key = valid ? A.C[e.x] : EMPTY_KEY;
  int ck = EMPTY_KEY, cs = 0;
  const int nd = group_collect<GS>(valid, key, e.y, lsum, ck, cs);
  const bool pair = gl < nd;
  const long long e_own = group_pick<GS>(pair && ck == c, cs);
  const int tm = int(A.two_m);  // 2m < 2^31: 32x32->64 products
  const long long s_own = (long long)tm * e_own - ki * ((have ? A.a[c] : 0) - ki);
  if (MODE == EV_DSADD) {
    const int q0 = have ? A.seg_beg[i] : 0;
    const int nsk = have ? A.seg_end[i] - q0 : 0;  // sinks are neighbours: <= GS
    const bool has = gl < nsk;
    const int sj = has ? int(A.ins_keys[q0 + gl] - uint64_t(i) * uint64_t(A.n0)) : 0;
    const int Xj = has ? A.C[sj] : EMPTY_KEY;
    long long ej = 0;
    const int ndw = wave_max(nd);
    for (int r = 0; r < ndw; ++r) {
      const int kr = group_bcast<GS>(ck, r);
      const int sr = group_bcast<GS>(cs, r);
      if (r < nd && Xj == kr) ej = sr;
    }
    Cand cd = {NO_SCORE, NO_LABEL, NO_LABEL};
    if (has) {
      long long g = Xj == c ? 0 : (long long)tm * int(ej) - (long long)int(ki) * A.a[Xj] - s_own;
      cd = {g, Xj, sj};
      A.sink_g[q0 + gl] = g;
    }
    const Cand best = group_cand_w<GS>(cd);
    if (have && gl == 0) {
      const bool live = best.j != NO_LABEL && best.x != c && best.g > 0;
      A.best_j[i] = live ? best.j : -1;
      if (live) A.best_g[i] = best.g;
    }
    return accepted;
  }
  Best b = {NO_SCORE, NO_LABEL};
  if (pair && ck != c) b = {(long long)tm * cs - (long long)int(ki) * A.a[ck], ck};
  b = group_best_w<GS>(b);
  const bool move = have && b.x != NO_LABEL && b.s > s_own;
  if (MODE == EV_SWEEP) {
    sweep_commit(A, i, move, c, b.x, gl);
  } else if (move) {  // EV_DSDEL
    if (e.x >= 0) A.R[e.x] = 1;
    if (gl == 0) {
      A.R[i] = 1;
      A.cflag[b.x] = 1;
      accepted += ACC_DEL;
    }
  }
  return accepted;
}

// Two sweep items per group with their loads interleaved: every stage of
// the chain row bounds -> entries -> neighbour labels -> community totals
// issues both items' loads before it waits on either, so a wave keeps
// twice the gathers in flight.  The arithmetic is group_item<EV_SWEEP>'s.
// The row starts come with the bin list, so the entry loads are issued
// with the row-end loads: a lane past its row's end reads another row's
// entry (any index below nnz) and drops it once the row end is known.
// Loads use clamped indices (every index is valid memory; an absent item
// reads entry 0) so that no load needs a branch: the kernel is bound by
// vector-instruction issue, not by memory.
template <int GS>
__device__ __forceinline__ void sweep_pair(const EvalArgs& A, int i0, bool h0, int32_t rb0,
                                           int i1, bool h1, int32_t rb1, int gl, int* lsum) {
  const int32_t x0 = A.off[i0 + 1], x1 = A.off[i1 + 1];
  const int32_t re0 = h0 ? x0 : 0, re1 = h1 ? x1 : 0;
  const int c0 = A.C[i0], c1 = A.C[i1];
  const int k0 = A.k[i0], k1 = A.k[i1];
  const int64_t last = A.nnz > 0 ? A.nnz - 1 : 0;
  const int2 e0 = A.adj[rb0 + gl < last ? rb0 + gl : last];
  const int2 e1 = A.adj[rb1 + gl < last ? rb1 + gl : last];
  const int ao0 = A.a[c0], ao1 = A.a[c1];
  const bool v0 = rb0 + gl < re0 && e0.x != i0, v1 = rb1 + gl < re1 && e1.x != i1;
  const int y0 = A.C[v0 ? e0.x : 0], y1 = A.C[v1 ? e1.x : 0];  // e.x is only valid in-row
  const int key0 = v0 ? y0 : EMPTY_KEY;
  const int key1 = v1 ? y1 : EMPTY_KEY;
  int ck0 = EMPTY_KEY, cs0 = 0, ck1 = EMPTY_KEY, cs1 = 0, it0 = 0, it1 = 0;
  const int nd0 = group_collect<GS>(v0, key0, e0.y, lsum, ck0, cs0, &it0);
  const int nd1 = group_collect<GS>(v1, key1, e1.y, lsum, ck1, cs1, &it1);
  const bool p0 = gl < nd0 && ck0 != c0, p1 = gl < nd1 && ck1 != c1;
  const int ak0 = A.a[p0 ? ck0 : 0];
  const int ak1 = A.a[p1 ? ck1 : 0];
  // e_{i->C(i)}: the weight sum parked in the one lane holding label C(i)
  const int own0 = group_pick<GS>(gl < nd0 && ck0 == c0, cs0);
  const int own1 = group_pick<GS>(gl < nd1 && ck1 == c1, cs1);
  // 2m < 2^31, so every factor fits in 32 bits: one 32x32->64 product each
  const int tm = int(A.two_m);
  const long long s0 = (long long)tm * own0 - (long long)k0 * (ao0 - k0);
  const long long s1 = (long long)tm * own1 - (long long)k1 * (ao1 - k1);
  Best b0 = {NO_SCORE, NO_LABEL}, b1 = {NO_SCORE, NO_LABEL};
  if (p0) b0 = {(long long)tm * cs0 - (long long)k0 * ak0, ck0};
  if (p1) b1 = {(long long)tm * cs1 - (long long)k1 * ak1, ck1};
  b0 = group_best_first<GS>(b0, it0);
  b1 = group_best_first<GS>(b1, it1);
  sweep_commit(A, i0, h0 && b0.x != NO_LABEL && b0.s > s0, c0, b0.x, gl);
  sweep_commit(A, i1, h1 && b1.x != NO_LABEL && b1.s > s1, c1, b1.x, gl);
}

// Screener features (EV_FEAT) for two items per group, loads interleaved as
// in sweep_pair: f_own = e_{i->C(i)}, and f_g1 / f_g2 the scaled gains to
// the best and the second-best other neighbouring community (score
// descending, label ascending; NO_GAIN when absent), the best taken over
// the group's distinct labels, then again without it; with pre, also the
// first level-0 sweep's decision (the same state is read).
template <int GS>
__device__ __forceinline__ void feat_pair(const EvalArgs& A, int i0, bool h0, int32_t rb0, int i1,
                                          bool h1, int32_t rb1, int gl, int* lsum) {
  const int32_t x0 = A.off[i0 + 1], x1 = A.off[i1 + 1];
  const int32_t re0 = h0 ? x0 : 0, re1 = h1 ? x1 : 0;
  const int c0 = A.C[i0], c1 = A.C[i1];
  const int k0 = A.k[i0], k1 = A.k[i1];
  const int64_t last = A.nnz > 0 ? A.nnz - 1 : 0;
  const int2 e0 = A.adj[rb0 + gl < last ? rb0 + gl : last];
  const int2 e1 = A.adj[rb1 + gl < last ? rb1 + gl : last];
  const int ao0 = A.a[c0], ao1 = A.a[c1];
  const bool v0 = rb0 + gl < re0 && e0.x != i0, v1 = rb1 + gl < re1 && e1.x != i1;
  const int y0 = A.C[v0 ? e0.x : 0], y1 = A.C[v1 ? e1.x : 0];
  int ck0 = EMPTY_KEY, cs0 = 0, ck1 = EMPTY_KEY, cs1 = 0, it0 = 0, it1 = 0;
  const int nd0 = group_collect<GS>(v0, v0 ? y0 : EMPTY_KEY, e0.y, lsum, ck0, cs0, &it0);
  const int nd1 = group_collect<GS>(v1, v1 ? y1 : EMPTY_KEY, e1.y, lsum, ck1, cs1, &it1);
  const bool p0 = gl < nd0 && ck0 != c0, p1 = gl < nd1 && ck1 != c1;
  const int ak0 = A.a[p0 ? ck0 : 0], ak1 = A.a[p1 ? ck1 : 0];
  const int own0 = group_pick<GS>(gl < nd0 && ck0 == c0, cs0);
  const int own1 = group_pick<GS>(gl < nd1 && ck1 == c1, cs1);
  const int tm = int(A.two_m);  // 2m < 2^31: 32x32->64 products
  const long long s0 = (long long)tm * own0 - (long long)k0 * (ao0 - k0);
  const long long s1 = (long long)tm * own1 - (long long)k1 * (ao1 - k1);
  Best b0 = {NO_SCORE, NO_LABEL}, b1 = {NO_SCORE, NO_LABEL};
  if (p0) b0 = {(long long)tm * cs0 - (long long)k0 * ak0, ck0};
  if (p1) b1 = {(long long)tm * cs1 - (long long)k1 * ak1, ck1};
  const Best f0 = group_best_first<GS>(b0, it0), f1 = group_best_first<GS>(b1, it1);
  // second best: the same candidates without the best label
  const int x0b = group_bcast<GS>(f0.x, 0), x1b = group_bcast<GS>(f1.x, 0);
  const Best g0 = group_best_first<GS>(b0.x != x0b ? b0 : Best{NO_SCORE, NO_LABEL}, it0);
  const Best g1 = group_best_first<GS>(b1.x != x1b ? b1 : Best{NO_SCORE, NO_LABEL}, it1);
  if (gl == 0) {
    if (h0) {
      A.f_own[i0] = own0;
      A.f_g1[i0] = f0.x != NO_LABEL ? f0.s - s0 : NO_GAIN;
      A.f_g2[i0] = g0.x != NO_LABEL ? g0.s - s0 : NO_GAIN;
      if (A.pre) pre_commit(A, i0, f0.x != NO_LABEL && f0.s > s0, c0, f0.x);
    }
    if (h1) {
      A.f_own[i1] = own1;
      A.f_g1[i1] = f1.x != NO_LABEL ? f1.s - s1 : NO_GAIN;
      A.f_g2[i1] = g1.x != NO_LABEL ? g1.s - s1 : NO_GAIN;
      if (A.pre) pre_commit(A, i1, f1.x != NO_LABEL && f1.s > s1, c1, f1.x);
    }
  }
}

// The screening pass (EV_DSBOTH) for two items per group, loads interleaved
// as in sweep_pair: everything indexed by a vertex -- its row end, label,
// degree, flags and sink segment -- is loaded with its row's entries, and
// the sinks' labels with the entries' labels, before either item's labels
// are grouped.  Per vertex, by its flags (uflag): for an insertion source
// (bit 0) Alg. 2's gain toward each sink's label, stored per record
// (sink_g), and its best sink with gain1 (best_j, best_g); for a deletion
// endpoint (bit 1) the deletion rule (a move would mark the vertex, its row
// and the target community); for every vertex the first-sweep decision
// when asked (pre).  Returns the deletion tests accepted (in the groups'
// first lanes).
template <int GS>
__device__ __forceinline__ long long screen_pair(const EvalArgs& A, int i0, bool h0, int32_t rb0,
                                                 int i1, bool h1, int32_t rb1, int gl,
                                                 int* lsum) {
  const int32_t x0 = A.off[i0 + 1], x1 = A.off[i1 + 1];
  const int c0 = A.C[i0], c1 = A.C[i1];
  const int k0 = A.k[i0], k1 = A.k[i1];
  const int uf0 = h0 ? int(A.uflag[i0]) : 0, uf1 = h1 ? int(A.uflag[i1]) : 0;
  const int32_t sb0 = A.seg_beg[i0], se0 = A.seg_end[i0];
  const int32_t sb1 = A.seg_beg[i1], se1 = A.seg_end[i1];
  const int64_t last = A.nnz > 0 ? A.nnz - 1 : 0;
  const int2 e0 = A.adj[rb0 + gl < last ? rb0 + gl : last];
  const int2 e1 = A.adj[rb1 + gl < last ? rb1 + gl : last];
  const int32_t re0 = h0 ? x0 : 0, re1 = h1 ? x1 : 0;
  const bool in0 = rb0 + gl < re0, in1 = rb1 + gl < re1;
  const bool v0 = in0 && e0.x != i0, v1 = in1 && e1.x != i1;
  // an insertion source's sinks are row entries, so there are at most GS
  const int ns0 = (uf0 & 1) ? se0 - sb0 : 0, ns1 = (uf1 & 1) ? se1 - sb1 : 0;
  const bool s0 = gl < ns0, s1 = gl < ns1;
  const uint64_t kq0 = A.ins_keys[s0 ? sb0 + gl : 0];
  const uint64_t kq1 = A.ins_keys[s1 ? sb1 + gl : 0];
  const int ao0 = A.a[c0], ao1 = A.a[c1];
  const int y0 = A.C[v0 ? e0.x : 0], y1 = A.C[v1 ? e1.x : 0];
  const int j0 = s0 ? int(kq0 - uint64_t(i0) * uint64_t(A.n0)) : 0;
  const int j1 = s1 ? int(kq1 - uint64_t(i1) * uint64_t(A.n0)) : 0;
  const int X0 = A.C[j0], X1 = A.C[j1];
  // the labels are grouped as in the sweep; a sink lane also learns the rank
  // of its sink's label among them (a sink is an entry of the row, so its
  // label is there), and reads that label's weight from the lane holding it
  int ck0 = EMPTY_KEY, cs0 = 0, ck1 = EMPTY_KEY, cs1 = 0, it0 = 0, it1 = 0, xr0 = -1, xr1 = -1;
  const int nd0 = group_collect<GS>(v0, v0 ? y0 : EMPTY_KEY, e0.y, lsum, ck0, cs0, &it0,
                                    s0 ? X0 : EMPTY_KEY, &xr0);
  const int nd1 = group_collect<GS>(v1, v1 ? y1 : EMPTY_KEY, e1.y, lsum, ck1, cs1, &it1,
                                    s1 ? X1 : EMPTY_KEY, &xr1);
  const int gbase = lane_id() - gl;
  const int sx0 = __shfl(cs0, gbase + (xr0 < 0 ? 0 : xr0), WAVE);
  const int sx1 = __shfl(cs1, gbase + (xr1 < 0 ? 0 : xr1), WAVE);
  const int ej0 = xr0 < 0 ? 0 : sx0, ej1 = xr1 < 0 ? 0 : sx1;
  const bool p0 = gl < nd0 && ck0 != c0, p1 = gl < nd1 && ck1 != c1;
  const int ak0 = A.a[p0 ? ck0 : 0], ak1 = A.a[p1 ? ck1 : 0];
  const int ax0 = A.a[X0], ax1 = A.a[X1];
  const int own0 = group_pick<GS>(gl < nd0 && ck0 == c0, cs0);
  const int own1 = group_pick<GS>(gl < nd1 && ck1 == c1, cs1);
  const int tm = int(A.two_m);  // 2m < 2^31: 32x32->64 products
  const long long so0 = (long long)tm * own0 - (long long)k0 * (ao0 - k0);
  const long long so1 = (long long)tm * own1 - (long long)k1 * (ao1 - k1);
  // Alg. 2: each sink's gain, stored per record, and the best sink per source
  if (__ballot((uf0 | uf1) & 1)) {  // wave-uniform
    Cand d0 = {NO_SCORE, NO_LABEL, NO_LABEL}, d1 = {NO_SCORE, NO_LABEL, NO_LABEL};
    if (s0) {
      const long long g = X0 == c0 ? 0 : (long long)tm * ej0 - (long long)k0 * ax0 - so0;
      A.sink_g[sb0 + gl] = g;
      d0 = {g, X0, j0};
    }
    if (s1) {
      const long long g = X1 == c1 ? 0 : (long long)tm * ej1 - (long long)k1 * ax1 - so1;
      A.sink_g[sb1 + gl] = g;
      d1 = {g, X1, j1};
    }
    d0 = group_cand_first<GS>(d0, ns0);
    d1 = group_cand_first<GS>(d1, ns1);
    if ((uf0 & 1) && gl == 0) {
      const bool live = d0.j != NO_LABEL && d0.x != c0 && d0.g > 0;
      A.best_j[i0] = live ? d0.j : -1;
      if (live) A.best_g[i0] = d0.g;
    }
    if ((uf1 & 1) && gl == 0) {
      const bool live = d1.j != NO_LABEL && d1.x != c1 && d1.g > 0;
      A.best_j[i1] = live ? d1.j : -1;
      if (live) A.best_g[i1] = d1.g;
    }
  }
  // the best move: the first-sweep decision and the deletion rule
  Best b0 = {NO_SCORE, NO_LABEL}, b1 = {NO_SCORE, NO_LABEL};
  if (p0) b0 = {(long long)tm * cs0 - (long long)k0 * ak0, ck0};
  if (p1) b1 = {(long long)tm * cs1 - (long long)k1 * ak1, ck1};
  // (decided in each group's first lane)
  b0 = group_best_first<GS>(b0, it0);
  b1 = group_best_first<GS>(b1, it1);
  const bool m0 = h0 && b0.x != NO_LABEL && b0.s > so0;
  const bool m1 = h1 && b1.x != NO_LABEL && b1.s > so1;
  if (A.pre && h0 && gl == 0) pre_commit(A, i0, m0, c0, b0.x);
  if (A.pre && h1 && gl == 0) pre_commit(A, i1, m1, c1, b1.x);
  long long accepted = 0;
  const bool d0 = gl == 0 && m0 && (uf0 & 2), d1 = gl == 0 && m1 && (uf1 & 2);
  if (__ballot(d0 || d1)) {  // wave-uniform; a deletion endpoint that would move
    // its group's lanes mark the row (the leader's decision, broadcast)
    if (group_pick<GS>(d0, 1) && in0) A.R[e0.x] = 1;
    if (group_pick<GS>(d1, 1) && in1) A.R[e1.x] = 1;
    if (d0) {
      A.R[i0] = 1;
      A.cflag[b0.x] = 1;
      accepted += ACC_DEL;
    }
    if (d1) {
      A.R[i1] = 1;
      A.cflag[b1.x] = 1;
      accepted += ACC_DEL;
    }
  }
  return accepted;
}

// The items of one row-length bin of at most 64 entries, groups of GS
// lanes, as block bid of nblocks (ls: the wave's zeroed LDS row).
template <int MODE, int GS>
__device__ __forceinline__ void eval_group_body(const EvalArgs& A, int64_t bid, int64_t nblocks,
                                                int* ls) {
  constexpr int GPW = WAVE / GS;  // groups per wave
  const int lane = lane_id();
  const int gl = lane & (GS - 1);
  const int gbase = lane - gl;
  const int64_t cnt = *A.count;
  const int64_t ngroups = nblocks * NW * GPW;
  long long accepted = 0;
  const int64_t g0 = (bid * NW + threadIdx.x / WAVE) * GPW + lane / GS;
  // every group of a wave runs the same number of iterations (wave-uniform)
  const int64_t w0 = g0 - lane / GS;
  if constexpr (MODE == EV_SWEEP || MODE == EV_FEAT || MODE == EV_DSBOTH) {
    // two items per group and round (their loads interleaved)
    for (int64_t wb = w0; wb < cnt; wb += 2 * ngroups) {
      const int64_t idx0 = wb + lane / GS, idx1 = wb + ngroups + lane / GS;
      const bool h0 = idx0 < cnt, h1 = idx1 < cnt;
      const int64_t j0 = h0 ? idx0 : 0, j1 = h1 ? idx1 : 0;  // valid indices
      const int i0 = h0 ? A.list[j0] : 0;
      const int i1 = h1 ? A.list[j1] : 0;
      const int32_t rb0 = A.list_rb[j0], rb1 = A.list_rb[j1];
      if constexpr (MODE == EV_SWEEP)
        sweep_pair<GS>(A, i0, h0, rb0, i1, h1, rb1, gl, ls);
      else if constexpr (MODE == EV_FEAT)
        feat_pair<GS>(A, i0, h0, rb0, i1, h1, rb1, gl, ls);
      else
        accepted += screen_pair<GS>(A, i0, h0, rb0, i1, h1, rb1, gl, ls);
    }
  } else {
    for (int64_t wb = w0; wb < cnt; wb += ngroups) {
      const int64_t idx = wb + lane / GS;
      const bool have = idx < cnt;
      const int i = have ? A.list[idx] : 0;
      accepted += group_item<MODE, GS>(A, i, have, lane, gl, gbase, ls);
    }
  }
  if constexpr (MODE != EV_SWEEP && MODE != EV_FEAT) {
    accepted = group_sum_ll<WAVE>(accepted);
    if (lane == 0 && accepted) add_accepted(A.stat, accepted);
  }
}

template <int MODE, int GS>
__global__ void __launch_bounds__(TPB) k_eval_group(EvalArgs A) {
  __shared__ int lsum_all[NW][WAVE];
  int* ls = lsum_all[threadIdx.x / WAVE];
  ls[lane_id()] = 0;
  wave_sync();
  eval_group_body<MODE, GS>(A, blockIdx.x, gridDim.x, ls);
}

// The three short-row bins in one launch, block ranges [0, nb16), [nb16,
// nb16 + nb32) and the rest: three launches in a row each waited out the
// latency of one evaluation, which a bin too short to fill the chip (the
// screening set's, the sweeps' over part of the vertices) cannot hide.
template <int MODE>
__global__ void __launch_bounds__(TPB)
    k_eval_groups(EvalArgs A16, EvalArgs A32, EvalArgs A64, int nb16, int nb32) {
  __shared__ int lsum_all[NW][WAVE];
  int* ls = lsum_all[threadIdx.x / WAVE];
  ls[lane_id()] = 0;
  wave_sync();
  const int b = int(blockIdx.x);
  if (b < nb16)
    eval_group_body<MODE, 16>(A16, b, nb16, ls);
  else if (b < nb16 + nb32)
    eval_group_body<MODE, 32>(A32, b - nb16, nb32, ls);
  else
    eval_group_body<MODE, 64>(A64, b - nb16 - nb32, int64_t(gridDim.x) - nb16 - nb32, ls);
}

// --------------------------------------------------------------------------
// bins W, B, G: chunked distinct loop into a hash table, then a scan of it.

template <int G>
struct GroupLds {
  static constexpr int W = G / WAVE;  // waves of the group
  Best best[W];
  Cand cand[W];
  long long s0[W], s1[W];
  int own;
};

template <int G>
__device__ __forceinline__ void group_sync() {
  if (G == WAVE)
    wave_sync();
  else
    __syncthreads();
}

template <int G>
__device__ __forceinline__ Best group_best(Best b, GroupLds<G>& L) {
  b = wave_best(b);
  if (G == WAVE) return b;
  const int wid = threadIdx.x / WAVE;
  if (lane_id() == 0) L.best[wid] = b;
  __syncthreads();
  Best r = L.best[0];
#pragma unroll
  for (int w = 1; w < G / WAVE; ++w)
    if (better(L.best[w].s, L.best[w].x, r.s, r.x)) r = L.best[w];
  __syncthreads();
  return r;
}

template <int G>
__device__ __forceinline__ Cand group_cand(Cand c, GroupLds<G>& L) {
  c = group_cand_w<WAVE>(c);
  if (G == WAVE) return c;
  const int wid = threadIdx.x / WAVE;
  if (lane_id() == 0) L.cand[wid] = c;
  __syncthreads();
  Cand r = L.cand[0];
#pragma unroll
  for (int w = 1; w < G / WAVE; ++w)
    if (cand_better(L.cand[w], r)) r = L.cand[w];
  __syncthreads();
  return r;
}

template <int G>
__device__ __forceinline__ void group_sum2(long long& x, long long& y, GroupLds<G>& L) {
  x = wave_sum(x);
  y = wave_sum(y);
  if (G == WAVE) return;
  const int wid = threadIdx.x / WAVE;
  if (lane_id() == 0) {
    L.s0[wid] = x;
    L.s1[wid] = y;
  }
  __syncthreads();
  x = 0;
  y = 0;
#pragma unroll
  for (int w = 0; w < G / WAVE; ++w) {
    x += L.s0[w];
    y += L.s1[w];
  }
  __syncthreads();
}

// Power of two >= 2 * deg (at least 64), at most max_slots: the table is
// at most half full, and only that many slots are cleared and scanned.
__device__ __forceinline__ uint32_t table_cap(int deg, uint32_t max_slots) {
  uint32_t want = 2u * uint32_t(deg > 32 ? deg : 32);
  uint32_t cap = 1u << (32 - __clz(want - 1));
  return cap < max_slots ? cap : max_slots;
}

constexpr int GTPB = 1024;  // threads of a bin-G block (one hub row per block)
constexpr int GT_UI = 8;     // bin G: row chunks per load round
constexpr int WTAB_UI = WTAB_MAX / WAVE;   // bin W: the whole row in one load round
constexpr int WTAB_US = 8;                 // and its table in rounds of 8 slots

// This thread's best (score, label) over its slots of the table, skipping
// label `skip`; the community totals of US slots are gathered together.
template <int G, int US>
__device__ __forceinline__ Best table_best(const EvalArgs& A, const int* keys, const int* vals,
                                           uint32_t mask, long long ki, int skip, int t) {
  Best b = {NO_SCORE, NO_LABEL};
  for (uint32_t s0 = t; s0 <= mask; s0 += US * G) {
    int X[US], V[US], AX[US];
#pragma unroll
    for (int u = 0; u < US; ++u) {
      const uint32_t s = s0 + uint32_t(u * G);
      X[u] = s <= mask ? keys[s] : EMPTY_KEY;
      V[u] = s <= mask ? vals[s] : 0;
      if (X[u] == skip) X[u] = EMPTY_KEY;
    }
#pragma unroll
    for (int u = 0; u < US; ++u) AX[u] = X[u] != EMPTY_KEY ? A.a[X[u]] : 0;
#pragma unroll
    for (int u = 0; u < US; ++u) {
      if (X[u] == EMPTY_KEY) continue;
      // 2m < 2^31: 32x32->64 products
      const long long sc = (long long)int(A.two_m) * V[u] - (long long)int(ki) * AX[u];
      if (better(sc, X[u], b.s, b.x)) {
        b.s = sc;
        b.x = X[u];
      }
    }
  }
  return b;
}

// One group (a wave, or the whole block) evaluates vertex i with table
// (keys, vals, mask).  Returns the number of accepted screening tests (0/1)
// in thread 0 of the group.  BOUNDED: the table may be too small (at most
// (mask + 1) / 2 distinct labels fit); tstate holds two ints of group
// scratch, and if the row brings more labels the call returns TABLE_FULL
// to every thread before it has written anything outside the group.
constexpr long long TABLE_FULL = -1;
template <int MODE, int G, int UI, int US, bool BOUNDED = false>
__device__ long long eval_table(const EvalArgs& A, int i, int* keys, int* vals, uint32_t mask,
                                GroupLds<G>& L, int* own, int* tstate = nullptr) {
  const int t = (G == WAVE) ? lane_id() : int(threadIdx.x);
  const int lane = lane_id();
  const int32_t rb = A.off[i], re = A.off[i + 1];
  const int c = A.C[i];
  const long long ki = A.k[i];
  // loaded now, used after the table is built: the own community's total
  // and, for an insertion source, the sink segment and the labels and
  // totals of its first G sinks
  const int ac = A.a[c];
  // EV_DSBOTH: bit 0 an insertion source (Alg. 2), bit 1 a deletion endpoint
  const int uf = MODE == EV_DSBOTH ? int(A.uflag[i]) : (MODE == EV_DSADD ? 1 : 2);
  const bool dsadd = (MODE == EV_DSADD || MODE == EV_DSBOTH) && (uf & 1);
  const int64_t q0 = dsadd ? A.seg_beg[i] : 0, q1 = dsadd ? A.seg_end[i] : 0;
  const uint64_t base = uint64_t(i) * uint64_t(A.n0);
  const bool pf = q0 + t < q1;
  const int pj = pf ? int(A.ins_keys[q0 + t] - base) : 0;
  const int pX = pf ? A.C[pj] : 0;
  const int paX = pf ? A.a[pX] : 0;
  for (uint32_t s = t; s <= mask; s += G) {
    keys[s] = EMPTY_KEY;
    vals[s] = 0;
  }
  if (BOUNDED && t == 0) tstate[0] = tstate[1] = 0;
  group_sync<G>();
  // the own community (usually most of the row) is summed in registers;
  // every other entry goes straight into the table, one lane per entry
  // (UI chunks per round: their entry loads, then their label gathers, are
  // issued before any is waited on)
  long long own_part = 0;
  const int w0 = (G == WAVE) ? 0 : int(threadIdx.x) / WAVE;
  for (int32_t c0 = rb + w0 * WAVE; c0 < re; c0 += UI * G) {
    int2 e[UI];
    bool valid[UI];
    int key[UI];
#pragma unroll
    for (int u = 0; u < UI; ++u) {
      const int32_t q = c0 + u * G + lane;
      valid[u] = q < re;
      e[u] = valid[u] ? A.adj[q] : make_int2(0, 0);
    }
#pragma unroll
    for (int u = 0; u < UI; ++u) {
      if (e[u].x == i) valid[u] = false;
      key[u] = valid[u] ? A.C[e[u].x] : EMPTY_KEY;
    }
#pragma unroll
    for (int u = 0; u < UI; ++u) {
      if (key[u] == c)
        own_part += e[u].y;
      else if (valid[u]) {
        if (BOUNDED)
          table_add_bounded(keys, vals, mask, key[u], e[u].y, &tstate[0], &tstate[1],
                            int((mask + 1) / 2));
        else
          table_add(keys, vals, mask, key[u], e[u].y);
      }
    }
  }
  long long e_own = own_part, unused = 0;
  if constexpr (G == WAVE)
    e_own = wave_sum(int(own_part));  // at most k_i < 2m < 2^31: exact in 32 bits
  else
    group_sum2<G>(e_own, unused, L);
  group_sync<G>();
  if (BOUNDED && tstate[1]) return TABLE_FULL;  // group-uniform after the sync
  long long accepted = 0;
  // EV_DSBOTH: Alg. 2 for an insertion source (flag bit 0), then the
  // deletion rule for a deletion endpoint (bit 1), on the same table
  if (dsadd) {
    const long long s_own = A.two_m * e_own - ki * (ac - ki);
    Cand best = {NO_SCORE, NO_LABEL, NO_LABEL};
    for (int64_t q = q0 + t; q < q1; q += G) {
      const bool first = q == q0 + t;  // the prefetched sink
      const int j = first ? pj : int(A.ins_keys[q] - base);
      const int X = first ? pX : A.C[j];
      const int aX = first ? paX : A.a[X];
      long long g = 0;
      if (X != c) g = A.two_m * table_get(keys, vals, mask, X) - ki * aX - s_own;
      A.sink_g[q] = g;
      Cand cd = {g, X, j};
      if (cand_better(cd, best)) best = cd;
    }
    if constexpr (G == WAVE)  // the sinks sit in the first lanes (one vertex per wave)
      best = group_cand_first<WAVE>(best, int(q1 - q0 < WAVE ? q1 - q0 : WAVE));
    else
      best = group_cand<G>(best, L);
    if (t == 0) {
      const bool live = best.j != NO_LABEL && best.x != c && best.g > 0;
      A.best_j[i] = live ? best.j : -1;
      if (live) A.best_g[i] = best.g;
    }
    group_sync<G>();  // the table is reused (by the deletion rule or the next item)
  }
  if (MODE == EV_DSADD || (MODE == EV_DSBOTH && !(uf & 2) && !A.pre)) return accepted;
  Best b = table_best<G, US>(A, keys, vals, mask, ki, EMPTY_KEY, t);
  b = group_best<G>(b, L);
  group_sync<G>();
  const long long s_own = A.two_m * e_own - ki * (ac - ki);
  if (MODE == EV_FEAT) {
    // the table holds only foreign labels; a second scan skips the best
    Best b2 = table_best<G, US>(A, keys, vals, mask, ki, b.x, t);
    b2 = group_best<G>(b2, L);
    if (t == 0) {
      A.f_own[i] = int32_t(e_own);
      A.f_g1[i] = b.x != NO_LABEL ? b.s - s_own : NO_GAIN;
      A.f_g2[i] = b2.x != NO_LABEL ? b2.s - s_own : NO_GAIN;
      if (A.pre) pre_commit(A, i, b.x != NO_LABEL && b.s > s_own, c, b.x);
    }
    group_sync<G>();  // the table is reused by the next item of this group
    return 0;
  }
  bool move = b.x != NO_LABEL && b.s > s_own;
  if (MODE == EV_DSBOTH && A.pre && t == 0) pre_commit(A, i, move, c, b.x);
  if (MODE == EV_SWEEP) {
    if (move && A.guard && A.sz[c] == 1 && A.sz[b.x] == 1 && b.x > c) move = false;
    if (move && t == 0) A.Cn[i] = b.x;
  } else if (move && (MODE != EV_DSBOTH || (uf & 2))) {  // EV_DSDEL, EV_DSBOTH
    for (int32_t q = rb + t; q < re; q += G) A.R[A.adj[q].x] = 1;
    if (t == 0) {
      A.R[i] = 1;
      A.cflag[b.x] = 1;
      accepted += ACC_DEL;
    }
  }
  // the table is reused by the next item of this group
  group_sync<G>();
  return accepted;
}

// Bins W and B evaluate with small LDS tables (more blocks fit a CU): a row
// of at most a quarter as many entries as slots always fits; a longer row
// whose foreign labels overflow the table is listed for k_eval_ovf, which
// evaluates it again with the full table.  Overflow is detected before
// anything outside the group is written.
constexpr int WT_SLOTS = 512;   // bin W: per-wave table
constexpr int BT_SLOTS = 2048;  // bin B: per-block table

// bin W: one wave per vertex, wave-private LDS table
template <int MODE>
__global__ void __launch_bounds__(TPB, MODE == EV_SWEEP ? 8 : 7) k_eval_wtab(EvalArgs A) {
  __shared__ int keys[NW][WT_SLOTS];
  __shared__ int vals[NW][WT_SLOTS];
  __shared__ GroupLds<WAVE> L[NW];
  __shared__ int own[NW];
  __shared__ int tst[NW][2];
  const int wid = threadIdx.x / WAVE;
  const int64_t cnt = *A.count;
  const int64_t nwaves = int64_t(gridDim.x) * NW;
  long long accepted = 0;
  for (int64_t idx = int64_t(blockIdx.x) * NW + wid; idx < cnt; idx += nwaves) {
    const int i = uniform(A.list[idx]);
    const uint32_t cap = table_cap(A.off[i + 1] - A.off[i], WT_SLOTS);
    const long long acc = eval_table<MODE, WAVE, WTAB_UI, WTAB_US, true>(
        A, i, keys[wid], vals[wid], cap - 1, L[wid], &own[wid], tst[wid]);
    if (acc == TABLE_FULL) {
      if (lane_id() == 0) A.ovf_list[atomicAdd(A.ovf_count, 1)] = i;
    } else {
      accepted += acc;
    }
  }
  if (MODE != EV_SWEEP && lane_id() == 0 && accepted) add_accepted(A.stat, accepted);
}

// bin B: one block per vertex, block-shared LDS table
template <int MODE>
__global__ void __launch_bounds__(TPB) k_eval_btab(EvalArgs A) {
  __shared__ int keys[BT_SLOTS];
  __shared__ int vals[BT_SLOTS];
  __shared__ GroupLds<TPB> L;
  __shared__ int own;
  __shared__ int tst[2];
  const int64_t idx = blockIdx.x;
  if (idx >= *A.count) return;  // uniform over the block
  const int i = A.list[idx];
  const uint32_t cap = table_cap(A.off[i + 1] - A.off[i], BT_SLOTS);
  const long long acc =
      eval_table<MODE, TPB, 4, 8, true>(A, i, keys, vals, cap - 1, L, &own, tst);
  if (threadIdx.x != 0) return;
  if (acc == TABLE_FULL)
    A.ovf_list[atomicAdd(A.ovf_count, 1)] = i;
  else if (MODE != EV_SWEEP && acc)
    add_accepted(A.stat, acc);
}

// The rows of bins W and B that overflowed their small table, with the
// full one (rows of at most BTAB_MAX entries always fit).  A fixed grid
// loops over the list; the last block to finish clears the list for the
// next launch.
template <int MODE>
__global__ void __launch_bounds__(TPB) k_eval_ovf(EvalArgs A, int32_t* done) {
  __shared__ int keys[BTAB_SLOTS];
  __shared__ int vals[BTAB_SLOTS];
  __shared__ GroupLds<TPB> L;
  __shared__ int own;
  const int64_t cnt = *A.ovf_count;
  long long accepted = 0;
  for (int64_t idx = blockIdx.x; idx < cnt; idx += gridDim.x) {
    const int i = A.ovf_list[idx];
    const uint32_t cap = table_cap(A.off[i + 1] - A.off[i], BTAB_SLOTS);
    accepted += eval_table<MODE, TPB, 4, 8>(A, i, keys, vals, cap - 1, L, &own);
  }
  if (MODE != EV_SWEEP && threadIdx.x == 0 && accepted) add_accepted(A.stat, accepted);
  __syncthreads();  // every thread of the block has read the count
  if (threadIdx.x == 0 && atomicAdd(done, 1) == int(gridDim.x) - 1) {
    *A.ovf_count = 0;
    *done = 0;
  }
}

// bin G: one block per vertex.  The row's foreign labels usually fit the
// LDS table (a hub's neighbours mostly share a few communities), and the
// whole row is loaded in one round; a row with more labels than that
// table takes is evaluated again with its table in global memory (>= 2
// slots per entry).
template <int MODE>
__global__ void __launch_bounds__(GTPB) k_eval_gtab(EvalArgs A) {
  __shared__ int keys[BTAB_SLOTS];
  __shared__ int vals[BTAB_SLOTS];
  __shared__ GroupLds<GTPB> L;
  __shared__ int own;
  __shared__ int tstate[2];
  const int64_t idx = blockIdx.x;
  if (idx >= *A.count) return;
  const int i = A.list[idx];
  long long acc = eval_table<MODE, GTPB, GT_UI, 8, true>(A, i, keys, vals, BTAB_SLOTS - 1, L,
                                                         &own, tstate);
  if (acc == TABLE_FULL) {
    const long long o0 = A.tab_off[idx], o1 = A.tab_off[idx + 1];
    if (o1 > A.gslots) {
      // the table buffer is smaller than the rows' capacities: report, write nothing
      if (threadIdx.x == 0) atomicOr((unsigned long long*)&A.stat[ST_ERR], 1ull);
      return;
    }
    acc = eval_table<MODE, GTPB, 4, 8>(A, i, A.gkeys + o0, A.gvals + o0, uint32_t(o1 - o0) - 1,
                                       L, &own);
  }
  if (MODE != EV_SWEEP && threadIdx.x == 0 && acc) add_accepted(A.stat, acc);
}

// --------------------------------------------------------------------------
// merged sweeps: the items of several graphs in one launch per bin.  Lists
// are padded per graph to whole waves, so each wave (or block) works for one
// graph and loads that graph's arguments as uniform values.

struct MultiArgs {
  const EvalArgs* descs;
  const int32_t* list;
  const int32_t* gid;
  const int32_t* done;
  int64_t count;
};

template <int GS>
__global__ void __launch_bounds__(TPB) k_sweep_group_multi(MultiArgs M) {
  constexpr int GPW = WAVE / GS;
  const int lane = lane_id();
  const int gl = lane & (GS - 1);
  const int gbase = lane - gl;
  __shared__ int lsum_all[NW][WAVE];
  int* ls = lsum_all[threadIdx.x / WAVE];
  ls[lane] = 0;
  wave_sync();
  const int64_t ngroups = int64_t(gridDim.x) * NW * GPW;
  const int64_t w0 = (int64_t(blockIdx.x) * NW + threadIdx.x / WAVE) * GPW;
  for (int64_t wb = w0; wb < M.count; wb += ngroups) {
    const int g = uniform(M.gid[wb]);
    if (M.done[g]) continue;  // uniform: this graph's level has converged
    const EvalArgs A = M.descs[g];
    const int i = M.list[wb + lane / GS];
    (void)group_item<EV_SWEEP, GS>(A, i < 0 ? 0 : i, i >= 0, lane, gl, gbase, ls);
  }
}

__global__ void __launch_bounds__(TPB) k_sweep_wtab_multi(MultiArgs M) {
  __shared__ int keys[NW][WTAB_SLOTS];
  __shared__ int vals[NW][WTAB_SLOTS];
  __shared__ GroupLds<WAVE> L[NW];
  __shared__ int own[NW];
  const int wid = threadIdx.x / WAVE;
  const int64_t nwaves = int64_t(gridDim.x) * NW;
  for (int64_t idx = int64_t(blockIdx.x) * NW + wid; idx < M.count; idx += nwaves) {
    const int g = uniform(M.gid[idx]);
    if (M.done[g]) continue;
    const EvalArgs A = M.descs[g];
    const int i = uniform(M.list[idx]);
    const uint32_t cap = table_cap(A.off[i + 1] - A.off[i], WTAB_SLOTS);
    (void)eval_table<EV_SWEEP, WAVE, WTAB_UI, WTAB_US>(A, i, keys[wid], vals[wid], cap - 1,
                                                       L[wid], &own[wid]);
  }
}

__global__ void __launch_bounds__(TPB) k_sweep_btab_multi(MultiArgs M) {
  __shared__ int keys[BTAB_SLOTS];
  __shared__ int vals[BTAB_SLOTS];
  __shared__ GroupLds<TPB> L;
  __shared__ int own;
  for (int64_t idx = blockIdx.x; idx < M.count; idx += gridDim.x) {
    const int g = M.gid[idx];  // uniform over the block
    if (M.done[g]) continue;
    const EvalArgs A = M.descs[g];
    const int i = M.list[idx];
    const uint32_t cap = table_cap(A.off[i + 1] - A.off[i], BTAB_SLOTS);
    (void)eval_table<EV_SWEEP, TPB, 4, 8>(A, i, keys, vals, cap - 1, L, &own);
  }
}

// bin G: one 1024-thread block per hub row of any graph (k_eval_gtab's
// evaluation; the row's global-table slice from its graph's own tables)
__global__ void __launch_bounds__(GTPB)
    k_sweep_gtab_multi(MultiArgs M, const int32_t* __restrict__ lidx) {
  __shared__ int keys[BTAB_SLOTS];
  __shared__ int vals[BTAB_SLOTS];
  __shared__ GroupLds<GTPB> L;
  __shared__ int own;
  __shared__ int tstate[2];
  const int64_t idx = blockIdx.x;
  if (idx >= M.count) return;
  const int g = M.gid[idx];  // uniform over the block
  if (M.done[g]) return;
  const EvalArgs A = M.descs[g];
  const int i = M.list[idx];
  const int64_t q = lidx[idx];
  const long long acc = eval_table<EV_SWEEP, GTPB, GT_UI, 8, true>(A, i, keys, vals,
                                                                    BTAB_SLOTS - 1, L, &own, tstate);
  if (acc == TABLE_FULL) {
    const long long o0 = A.tab_off[q], o1 = A.tab_off[q + 1];
    if (o1 > A.gslots) {
      if (threadIdx.x == 0) atomicOr((unsigned long long*)&A.stat[ST_ERR], 1ull);
      return;
    }
    (void)eval_table<EV_SWEEP, GTPB, 4, 8>(A, i, A.gkeys + o0, A.gvals + o0,
                                           uint32_t(o1 - o0) - 1, L, &own);
  }
}

struct MultiDst {
  int32_t* list[NBINS];
  int32_t* gid[NBINS];
  int32_t* lidx;  // bin G: position in the graph's own bin
};

// block per segment: copy a graph's bin list into its merged slot, padding
// with -1, and tag every item with the graph index
__global__ void k_build_multi(const MultiSeg* __restrict__ segs, int nsegs, MultiDst D) {
  for (int sidx = blockIdx.x; sidx < nsegs; sidx += gridDim.x) {
    const MultiSeg sg = segs[sidx];
    int32_t* lst = D.list[sg.bin] + sg.dst;
    int32_t* gd = D.gid[sg.bin] + sg.dst;
    for (int64_t i = threadIdx.x; i < sg.padded; i += blockDim.x) {
      lst[i] = i < sg.n ? sg.src[i] : -1;
      gd[i] = sg.gid;
      if (sg.bin == NBINS - 1) D.lidx[sg.dst + i] = int32_t(i);
    }
  }
}

// --------------------------------------------------------------------------
// binning by row length: per-block counts, one scan, stable scatter.

constexpr int BIN_ITEMS = 4;
constexpr int BIN_TILE = TPB * BIN_ITEMS;

// wmax: the longest row of bin W (WTAB_MAX, or half of it on coarse levels,
// whose rows hold mostly distinct labels and would overflow the wave table)
__device__ __forceinline__ int bin_of(int d, int wmax) {
  return d <= 16 ? 0 : d <= 32 ? 1 : d <= 64 ? 2 : d <= wmax ? 3 : d <= BTAB_MAX ? 4 : 5;
}

// Rows of the binning: bin q of a vertex v is split into row 2q (evaluated
// by every sweep) and row 2q + 1 (skip[v] != 0: left out of the first
// sweep), so that each bin's list holds its first-sweep vertices first.
constexpr int NROWS = 2 * NBINS;

__global__ void __launch_bounds__(TPB)
    k_bin_count(const int32_t* __restrict__ list, int64_t cnt, const int32_t* __restrict__ dcnt,
                const int32_t* __restrict__ off, const uint8_t* __restrict__ skip, int32_t* bcnt,
                long long* bvol, int64_t nblocks, int wmax) {
  if (dcnt) cnt = *dcnt;  // the list's length on the device (cnt: its bound)
  __shared__ int c[NROWS];
  __shared__ long long v[NROWS];
  if (threadIdx.x < NROWS) {
    c[threadIdx.x] = 0;
    v[threadIdx.x] = 0;
  }
  __syncthreads();
  int lc[NROWS];
  long long lv[NROWS];
#pragma unroll
  for (int q = 0; q < NROWS; ++q) {
    lc[q] = 0;
    lv[q] = 0;
  }
  if (cnt > 0) {  // block-uniform
    // the BIN_ITEMS vertices, then their bounds and flags: clamped indexes,
    // so each round of loads is in flight together
    int u[BIN_ITEMS], d[BIN_ITEMS], sk[BIN_ITEMS];
#pragma unroll
    for (int r = 0; r < BIN_ITEMS; ++r) {
      const int64_t p = int64_t(blockIdx.x) * BIN_TILE + int64_t(r) * TPB + threadIdx.x;
      const int64_t pc = p < cnt ? p : cnt - 1;
      u[r] = list ? list[pc] : int(pc);
    }
#pragma unroll
    for (int r = 0; r < BIN_ITEMS; ++r) d[r] = off[u[r] + 1] - off[u[r]];
    if (skip) {
#pragma unroll
      for (int r = 0; r < BIN_ITEMS; ++r) sk[r] = skip[u[r]];
    } else {
#pragma unroll
      for (int r = 0; r < BIN_ITEMS; ++r) sk[r] = 0;
    }
#pragma unroll
    for (int r = 0; r < BIN_ITEMS; ++r) {
      const int64_t p = int64_t(blockIdx.x) * BIN_TILE + int64_t(r) * TPB + threadIdx.x;
      const int row = p < cnt ? 2 * bin_of(d[r], wmax) + (sk[r] ? 1 : 0) : -1;
#pragma unroll
      for (int q = 0; q < NROWS; ++q) {
        if (row == q) {
          lc[q]++;
          lv[q] += d[r];
        }
      }
    }
  }
#pragma unroll
  for (int b = 0; b < NROWS; ++b) {
    int x = wave_sum(lc[b]);
    long long y = wave_sum(lv[b]);
    if (lane_id() == 0) {
      if (x) atomicAdd(&c[b], x);
      if (y) atomicAdd((unsigned long long*)&v[b], (unsigned long long)y);
    }
  }
  __syncthreads();
  if (threadIdx.x < NROWS) {
    bcnt[int64_t(threadIdx.x) * nblocks + blockIdx.x] = c[threadIdx.x];
    bvol[int64_t(threadIdx.x) * nblocks + blockIdx.x] = v[threadIdx.x];
  }
}

// out[boff[row][block] + rank] = vertex: rows are contiguous segments of
// out, in list order within each row
__global__ void __launch_bounds__(TPB)
    k_bin_scatter(const int32_t* __restrict__ list, int64_t cnt,
                  const int32_t* __restrict__ dcnt, const int32_t* __restrict__ off,
                  const uint8_t* __restrict__ skip, const int32_t* __restrict__ boff,
                  int64_t nblocks, int32_t* out, int32_t* out_rb, int wmax) {
  if (dcnt) cnt = *dcnt;
  __shared__ int base[NROWS];
  __shared__ int wc[NW][NROWS];
  const int wid = threadIdx.x / WAVE, lane = lane_id();
  if (threadIdx.x < NROWS) base[threadIdx.x] = boff[int64_t(threadIdx.x) * nblocks + blockIdx.x];
  __syncthreads();
  const uint64_t lt = (uint64_t(1) << lane) - 1;
  // every item's vertex, row start and row first (clamped indexes: the
  // loads of a round are in flight together), then the ranking rounds
  int uu[BIN_ITEMS], rrow[BIN_ITEMS], rrb[BIN_ITEMS];
  if (cnt > 0) {  // block-uniform
#pragma unroll
    for (int r = 0; r < BIN_ITEMS; ++r) {
      const int64_t p = int64_t(blockIdx.x) * BIN_TILE + int64_t(r) * TPB + threadIdx.x;
      const int64_t pc = p < cnt ? p : cnt - 1;
      uu[r] = list ? list[pc] : int(pc);
    }
    int b1[BIN_ITEMS], sk[BIN_ITEMS];
#pragma unroll
    for (int r = 0; r < BIN_ITEMS; ++r) {
      rrb[r] = off[uu[r]];
      b1[r] = off[uu[r] + 1];
    }
    if (skip) {
#pragma unroll
      for (int r = 0; r < BIN_ITEMS; ++r) sk[r] = skip[uu[r]];
    } else {
#pragma unroll
      for (int r = 0; r < BIN_ITEMS; ++r) sk[r] = 0;
    }
#pragma unroll
    for (int r = 0; r < BIN_ITEMS; ++r) {
      const int64_t p = int64_t(blockIdx.x) * BIN_TILE + int64_t(r) * TPB + threadIdx.x;
      rrow[r] = p < cnt ? 2 * bin_of(b1[r] - rrb[r], wmax) + (sk[r] ? 1 : 0) : -1;
    }
  } else {
#pragma unroll
    for (int r = 0; r < BIN_ITEMS; ++r) {
      uu[r] = 0;
      rrb[r] = 0;
      rrow[r] = -1;
    }
  }
#pragma unroll
  for (int r = 0; r < BIN_ITEMS; ++r) {
    const bool valid = rrow[r] >= 0;
    const int u = uu[r], row = rrow[r], rb = rrb[r];
    int rank = 0;
#pragma unroll
    for (int q = 0; q < NROWS; ++q) {
      uint64_t m = __ballot(row == q);
      if (lane == 0) wc[wid][q] = __popcll(m);
      if (row == q) rank = __popcll(m & lt);
    }
    __syncthreads();
    if (valid) {
      int pos = base[row] + rank;
      for (int w = 0; w < wid; ++w) pos += wc[w][row];
      out[pos] = u;
      out_rb[pos] = rb;
    }
    __syncthreads();
    if (threadIdx.x < NROWS) {
      int add = 0;
      for (int w = 0; w < NW; ++w) add += wc[w][threadIdx.x];
      base[threadIdx.x] += add;
    }
    __syncthreads();
  }
}

// Metadata of a binning (int32 slots): [0, NBINS) bin sizes, [NBINS,
// 2 NBINS) first-part sizes (row 2q), [2 NBINS, 3 NBINS) bin starts, then
// the total, the overflow count and the overflow pass's finished blocks
// (both zero); from slot 32 on the NROWS row volumes (int64).
constexpr int M_START = 2 * NBINS, M_TOTAL = 3 * NBINS, M_OVF = 3 * NBINS + 1;
constexpr int META_WORDS = 32 + 2 * NROWS;
static_assert(M_OVF + 2 <= 32, "bin metadata slots overlap the volumes");
static_assert(META_WORDS * 4 <= 256, "bin metadata must fit the pinned host buffer");

constexpr int META_TPB = 1024;
constexpr int META_PER = 32;                    // counts per thread in the scan
constexpr int META_SCAN_MAX = META_TPB * META_PER;

// Inclusive prefix sum over a wave (shuffles: 6 steps).
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int y = __shfl_up(v, o, WAVE);
    if (lane >= o) v += y;
  }
  return v;
}

// One block after k_bin_count: with scan, the exclusive scan of the per-block
// row counts bcnt (row-major, NROWS * nblocks of them, at most META_SCAN_MAX)
// into boff; without, boff and its total (counts[M_TOTAL]) are given.  Then
// the metadata, written to counts and to host (device-visible pinned host
// memory), and copy_n slots of copy_src copied to copy_dst (host memory too)
// so that the caller's one wait brings back both.
__global__ void __launch_bounds__(META_TPB)
    k_bin_meta(const int32_t* __restrict__ bcnt, int32_t* boff,
               const long long* __restrict__ bvol, int64_t nblocks, int scan, int32_t* counts,
               int32_t* host, const long long* __restrict__ copy_src, long long* copy_dst,
               int copy_n) {
  __shared__ int wtot[META_TPB / WAVE];
  __shared__ long long vpart[META_TPB / WAVE][NROWS];
  __shared__ int meta[META_WORDS];
  const int t = threadIdx.x, lane = lane_id(), wid = t / WAVE;
  const int64_t M = int64_t(NROWS) * nblocks;
  if (t < META_WORDS) meta[t] = 0;
  __syncthreads();
  // row volumes: row by row, the threads stride over the blocks' partials
  // (all loads independent), then one wave sum per row and wave
#pragma unroll 1
  for (int r = 0; r < NROWS; ++r) {
    long long acc = 0;
    for (int64_t b = t; b < nblocks; b += META_TPB) acc += bvol[int64_t(r) * nblocks + b];
    acc = wave_sum(acc);
    if (lane == 0) vpart[wid][r] = acc;
  }
  if (scan) {
    // thread t scans the contiguous chunk [t * per, (t + 1) * per), its
    // counts held in registers (per <= META_PER)
    const int per = int(ceil_div(M, META_TPB));
    const int64_t b0 = int64_t(t) * per;
    int v[META_PER];
    int sum = 0;
#pragma unroll
    for (int i = 0; i < META_PER; ++i) {
      v[i] = (i < per && b0 + i < M) ? bcnt[b0 + i] : 0;
      sum += v[i];
    }
    const int incl = wave_incl_scan(sum);
    if (lane == WAVE - 1) wtot[wid] = incl;
    __syncthreads();
    if (t == 0) {
      int run = 0;
      for (int w = 0; w < META_TPB / WAVE; ++w) {
        const int x = wtot[w];
        wtot[w] = run;
        run += x;
      }
      meta[M_TOTAL] = run;
    }
    __syncthreads();
    int run = wtot[wid] + incl - sum;
#pragma unroll
    for (int i = 0; i < META_PER; ++i) {
      if (i < per && b0 + i < M) boff[b0 + i] = run;
      run += v[i];
    }
  } else if (t == 0) {
    meta[M_TOTAL] = counts[M_TOTAL];
  }
  __syncthreads();  // boff (global, this block's writes) and the total
  if (t < NBINS && M > 0) {
    // boff is row-major: row r starts at boff[r * nblocks]
    const int q = t;
    const int s0 = boff[int64_t(2 * q) * nblocks];
    const int s1 = boff[int64_t(2 * q + 1) * nblocks];
    const int e = (q + 1 < NBINS) ? boff[int64_t(2 * q + 2) * nblocks] : meta[M_TOTAL];
    meta[M_START + q] = s0;
    meta[q] = e - s0;
    meta[NBINS + q] = s1 - s0;
  }
  if (t < NROWS) {
    long long v = 0;
    for (int w = 0; w < META_TPB / WAVE; ++w) v += vpart[w][t];
    meta[32 + 2 * t] = int(uint32_t(uint64_t(v)));
    meta[32 + 2 * t + 1] = int(uint32_t(uint64_t(v) >> 32));
  }
  __syncthreads();
  if (t < META_WORDS) {
    counts[t] = meta[t];
    host_store(&host[t], meta[t]);
  }
  for (int i = t; i < copy_n; i += META_TPB) host_store(&copy_dst[i], copy_src[i]);
}

__global__ void k_table_caps(const int32_t* __restrict__ list, const int32_t* __restrict__ off,
                             int64_t cnt, long long* caps) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < cnt;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int v = list[i];
    const long long d = off[v + 1] - off[v];
    long long c = 2;
    while (c < 2 * d) c <<= 1;
    caps[i] = c;
  }
}

inline int grid_for(int64_t n, int cap = 4096) {
  int64_t g = ceil_div(n, TPB);
  if (g > cap) g = cap;
  return int(g < 1 ? 1 : g);
}

inline int wave_grid(int64_t items) {
  // one wave per item, at most 16384 blocks; waves loop over the rest
  int64_t g = ceil_div(items, NW);
  if (g > 16384) g = 16384;
  return int(g < 1 ? 1 : g);
}

// Alg. 2 acceptance, one thread per directed insertion record j -> i: the
// record decides source i when j is i's best sink j*; then gain1 (stored
// with i) is compared with gain2 = the gain stored at this record.  An
// accepted source sets R[i], R[j*], the flag of C(j*) and (cascade) its
// accepted flag, and lists its row in chunks of MARK_CHUNK entries for
// k_mark_rows (R gets Gamma_t(i)); chunk positions come from a block scan
// and one atomic per block.
constexpr int MARK_CHUNK = 256;

__global__ void __launch_bounds__(TPB)
    k_ds_resolve(EvalArgs A, int2* __restrict__ items, long long* __restrict__ item_count) {
  __shared__ int wsum[NW];
  __shared__ long long bbase;
  const int lane = lane_id(), wid = threadIdx.x / WAVE;
  const uint64_t n0 = uint64_t(A.n0);
  long long accepted = 0, accvol = 0;
  for (int64_t base = int64_t(blockIdx.x) * TPB; base < A.n_ins;
       base += int64_t(gridDim.x) * TPB) {  // block-uniform
    const int64_t q = base + threadIdx.x;
    int32_t rb = 0, re = 0;
    int nit = 0;
    if (q < A.n_ins) {
      const uint64_t key = A.ins_keys[q];
      const int j = int(key / n0);
      const int i = int(key - uint64_t(j) * n0);
      if (A.best_j[i] == j && A.best_g[i] >= A.sink_g[q]) {
        A.R[i] = 1;
        A.R[j] = 1;
        A.cflag[A.C[j]] = 1;
        if (A.accflag) A.accflag[i] = 1;
        accepted += 1;
        rb = A.off[i];
        re = A.off[i + 1];
        accvol += re - rb;
        nit = int(ceil_div(re - rb, MARK_CHUNK));
      }
    }
    // exclusive block scan of the chunk counts
    int incl = nit;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      const int y = __shfl_up(incl, o, WAVE);
      if (lane >= o) incl += y;
    }
    if (lane == WAVE - 1) wsum[wid] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int w = 0; w < NW; ++w) tot += wsum[w];
      bbase = tot ? (long long)atomicAdd((unsigned long long*)item_count, (unsigned long long)tot)
                  : 0;
    }
    __syncthreads();
    long long pos = bbase + incl - nit;
    for (int w = 0; w < wid; ++w) pos += wsum[w];
    for (int r = 0; r < nit; ++r) {
      const int32_t cb = rb + r * MARK_CHUNK;
      items[pos + r] = make_int2(cb, re - cb < MARK_CHUNK ? re : cb + MARK_CHUNK);
    }
    __syncthreads();  // wsum and bbase are rewritten by the next tile
  }
  block_add(accepted, &A.stat[ST_DS_ACC]);
  block_add(accvol, &A.stat[ST_ACCVOL]);
}

// R of every entry of the listed row chunks [x, y): one wave per chunk.
__global__ void __launch_bounds__(TPB)
    k_mark_rows(const int2* __restrict__ items, const long long* __restrict__ item_count,
                const int2* __restrict__ adj, uint8_t* R) {
  const int64_t cnt = *item_count;
  const int64_t nwaves = int64_t(gridDim.x) * NW;
  for (int64_t it = int64_t(blockIdx.x) * NW + threadIdx.x / WAVE; it < cnt; it += nwaves) {
    const int2 ch = items[it];
    int2 e[MARK_CHUNK / WAVE];
#pragma unroll
    for (int u = 0; u < MARK_CHUNK / WAVE; ++u) {
      const int32_t q = ch.x + u * WAVE + lane_id();
      e[u] = q < ch.y ? adj[q] : make_int2(-1, 0);
    }
#pragma unroll
    for (int u = 0; u < MARK_CHUNK / WAVE; ++u)
      if (e[u].x >= 0) R[e[u].x] = 1;
  }
}

constexpr int64_t OVF_GRID = 128;  // blocks of k_eval_ovf

template <int MODE>
void launch_eval(const EvalArgs& base, const Bins& bins, hipStream_t st, hipEvent_t ev0,
                 hipEvent_t ev1) {
  EvalArgs A = base;
  A.ovf_list = bins.ovf_list;
  A.ovf_count = bins.ovf_count;
  auto setbin = [&](int q) {
    A.list = bins.list[q];
    A.list_rb = bins.list_rb[q];
    A.count = bins.count_dev + q;
  };
  // items a group takes per loop round: two in the sweep, the screening pass
  // and the feature pass (their loads interleaved); a wave holds 64 / GS
  // groups
  constexpr int PAIR = (MODE == EV_SWEEP || MODE == EV_DSBOTH || MODE == EV_FEAT) ? 2 : 1;
  // the sweeps and the screening and feature passes take their three
  // short-row bins in one launch (k_eval_groups), which ev0 / ev1 bracket
  constexpr bool JOINT = MODE == EV_SWEEP || MODE == EV_DSBOTH || MODE == EV_FEAT;
  if constexpr (JOINT) {
    if (bins.n[0] + bins.n[1] + bins.n[2] > 0) {
      const int nb[3] = {bins.n[0] > 0 ? wave_grid(ceil_div(bins.n[0], 4 * PAIR)) : 0,
                         bins.n[1] > 0 ? wave_grid(ceil_div(bins.n[1], 2 * PAIR)) : 0,
                         bins.n[2] > 0 ? wave_grid(ceil_div(bins.n[2], PAIR)) : 0};
      EvalArgs Aq[3];
      for (int q = 0; q < 3; ++q) {
        setbin(q);
        Aq[q] = A;
      }
      if (ev0) DC_HIP(hipEventRecord(ev0, st));
      k_eval_groups<MODE><<<nb[0] + nb[1] + nb[2], TPB, 0, st>>>(Aq[0], Aq[1], Aq[2], nb[0],
                                                                  nb[1]);
      DC_LAUNCH_CHECK();
      if (ev1) DC_HIP(hipEventRecord(ev1, st));
    }
  }
  if (!JOINT && bins.n[0] > 0) {
    setbin(0);
    k_eval_group<MODE, 16><<<wave_grid(ceil_div(bins.n[0], 4 * PAIR)), TPB, 0, st>>>(A);
    DC_LAUNCH_CHECK();
  }
  if (!JOINT && bins.n[1] > 0) {
    setbin(1);
    k_eval_group<MODE, 32><<<wave_grid(ceil_div(bins.n[1], 2 * PAIR)), TPB, 0, st>>>(A);
    DC_LAUNCH_CHECK();
  }
  // hub rows: few long blocks, so they run on the second stream beside the
  // other bins (all read one snapshot and write disjoint labels; shared
  // flags and counters are written as idempotent stores or atomics)
  const bool fork = bins.n[5] > 0 && bins.side;
  if (fork) {
    EvalArgs G = A;
    G.list = bins.list[5];
    G.list_rb = bins.list_rb[5];
    G.count = bins.count_dev + 5;
    G.gkeys = bins.gkeys;
    G.gvals = bins.gvals;
    G.tab_off = bins.tab_off;
    G.gslots = bins.gslots;
    DC_HIP(hipEventRecord(bins.fork, st));
    DC_HIP(hipStreamWaitEvent(bins.side, bins.fork, 0));
    k_eval_gtab<MODE><<<bins.n[5], GTPB, 0, bins.side>>>(G);
    DC_LAUNCH_CHECK();
    DC_HIP(hipEventRecord(bins.join, bins.side));
  }
  if (!JOINT && bins.n[2] > 0) {
    setbin(2);
    k_eval_group<MODE, 64><<<wave_grid(ceil_div(bins.n[2], PAIR)), TPB, 0, st>>>(A);
    DC_LAUNCH_CHECK();
  }
  if (bins.n[3] > 0) {
    setbin(3);
    k_eval_wtab<MODE><<<wave_grid(bins.n[3]), TPB, 0, st>>>(A);
    DC_LAUNCH_CHECK();
  }
  if (bins.n[4] > 0) {
    setbin(4);
    k_eval_btab<MODE><<<bins.n[4], TPB, 0, st>>>(A);
    DC_LAUNCH_CHECK();
  }
  if (bins.n[3] + bins.n[4] > 0) {
    const int64_t g = bins.n[3] + bins.n[4] < OVF_GRID ? bins.n[3] + bins.n[4] : OVF_GRID;
    k_eval_ovf<MODE><<<int(g), TPB, 0, st>>>(A, bins.ovf_done);
    DC_LAUNCH_CHECK();
  }
  if (fork) {
    DC_HIP(hipStreamWaitEvent(st, bins.join, 0));
  } else if (bins.n[5] > 0) {
    setbin(5);
    A.gkeys = bins.gkeys;
    A.gvals = bins.gvals;
    A.tab_off = bins.tab_off;
    A.gslots = bins.gslots;
    k_eval_gtab<MODE><<<bins.n[5], GTPB, 0, st>>>(A);
    DC_LAUNCH_CHECK();
  }
}

}  // namespace

void make_bins(const int32_t* list, int64_t count, const int32_t* off, Bins& b, BinScratch& s,
               hipStream_t st, const uint8_t* skip, const int32_t* dcount,
               const long long* copy_src, long long* copy_dst, int copy_n, bool coarse) {
  const int wmax = coarse ? WTAB_MAX / 2 : WTAB_MAX;
  const int64_t nb = count > 0 ? ceil_div(count, BIN_TILE) : 1;
  const int64_t cap = count > 0 ? count : 1;
  s.lists.ensure(size_t(cap) * sizeof(int32_t));
  s.lists_rb.ensure(size_t(cap) * sizeof(int32_t));
  s.bcnt.ensure(size_t(NROWS * nb + 1) * sizeof(int32_t));
  s.boff.ensure(size_t(NROWS * nb + 1) * sizeof(int32_t));
  s.bvol.ensure(size_t(NROWS * nb) * sizeof(long long));
  s.counts.ensure(META_WORDS * sizeof(int32_t));
  int32_t* counts = s.counts.as<int32_t>();
  int32_t* bcnt = s.bcnt.as<int32_t>();
  int32_t* boff = s.boff.as<int32_t>();
  long long* bvol = s.bvol.as<long long>();
  if (!s.host_dev) DC_HIP(hipHostGetDevicePointer(&s.host_dev, s.host, 0));
  // count, then the scan and the metadata in one block (the scan of many
  // blocks' counts takes the two-launch scan first), then one wait
  const int64_t M = count > 0 ? int64_t(NROWS) * nb : 0;
  if (count > 0) {
    k_bin_count<<<nb, TPB, 0, st>>>(list, count, dcount, off, skip, bcnt, bvol, nb, wmax);
    DC_LAUNCH_CHECK();
  }
  const bool one_block = M <= META_SCAN_MAX;
  if (!one_block) scan_excl_i32(bcnt, boff, M, counts + M_TOTAL, st);
  k_bin_meta<<<1, META_TPB, 0, st>>>(bcnt, boff, bvol, count > 0 ? nb : 0, one_block ? 1 : 0,
                                      counts, static_cast<int32_t*>(s.host_dev), copy_src,
                                      copy_dst, copy_src ? copy_n : 0);
  DC_LAUNCH_CHECK();
  DC_HIP(hipStreamSynchronize(st));
  const int32_t* hc = static_cast<const int32_t*>(s.host);
  const long long* hv = reinterpret_cast<const long long*>(hc + 32);
  int32_t* lists = s.lists.as<int32_t>();
  int32_t* lists_rb = s.lists_rb.as<int32_t>();
  b.total = 0;
  for (int q = 0; q < NBINS; ++q) {
    b.n[q] = hc[q];
    b.total += hc[q];
    b.n_first[q] = hc[NBINS + q];
    b.list[q] = lists + hc[M_START + q];
    b.list_rb[q] = lists_rb + hc[M_START + q];
    b.vol[q] = hv[2 * q] + hv[2 * q + 1];
    b.vol_first[q] = hv[2 * q];
  }
  b.count_dev = counts;
  b.count_first_dev = counts + NBINS;
  // overflow list of bins W and B; its count and finished-block counter sit
  // in the zeroed metadata and are cleared again by each k_eval_ovf
  s.ovf.ensure(size_t(cap) * sizeof(int32_t));
  b.ovf_list = s.ovf.as<int32_t>();
  b.ovf_count = counts + M_OVF;
  b.ovf_done = counts + M_OVF + 1;
  b.side = s.side;
  b.fork = s.fork;
  b.join = s.join;
  b.gkeys = nullptr;
  b.gvals = nullptr;
  b.tab_off = nullptr;
  b.gslots = 0;
  if (count > 0) {
    k_bin_scatter<<<nb, TPB, 0, st>>>(list, count, dcount, off, skip, boff, nb, lists,
                                      lists_rb, wmax);
    DC_LAUNCH_CHECK();
  }
  constexpr int G = NBINS - 1;
  if (b.n[G] > 0) {
    s.tab_off.ensure(size_t(b.n[G] + 1) * sizeof(long long));
    long long* caps = s.tab_off.as<long long>();
    k_table_caps<<<grid_for(b.n[G]), TPB, 0, st>>>(b.list[G], off, b.n[G], caps);
    DC_LAUNCH_CHECK();
    scan_excl_i64(reinterpret_cast<int64_t*>(caps), reinterpret_cast<int64_t*>(caps), b.n[G],
                  reinterpret_cast<int64_t*>(caps + b.n[G]), st);
    // row v takes the power of two >= 2 deg(v) (< 4 deg(v) for deg(v) >= 1),
    // so the bin's volume bounds the sum; the kernel checks tab_off against
    // gslots before it writes
    const size_t slots = size_t(4 * b.vol[G] + 2 * b.n[G] + 16);
    s.gkeys.ensure(slots * sizeof(int));
    s.gvals.ensure(slots * sizeof(int));
    b.gkeys = s.gkeys.as<int>();
    b.gvals = s.gvals.as<int>();
    b.tab_off = caps;
    b.gslots = int64_t(slots);
  }
}

void sweep_eval(const LevelView& g, const int32_t* C, int32_t* Cn, const int32_t* a,
                const int32_t* sz, long long two_m, int guard, const Bins& bins,
                long long* stat, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  EvalArgs A{};
  A.off = g.off;
  A.nnz = g.nnz;
  A.adj = g.adj;
  A.k = g.k;
  A.C = C;
  A.Cn = Cn;
  A.a = a;
  A.sz = sz;
  A.two_m = two_m;
  A.guard = guard;
  A.stat = stat;
  A.n0 = g.n;
  launch_eval<EV_SWEEP>(A, bins, st, ev0, ev1);
}

// Alg. 2 acceptance after an evaluation pass (every source's best sink and
// every record's gain stored): resolve, then mark the accepted rows.
void ds_resolve(const EvalArgs& A, const DsScratch& X, hipStream_t st) {
  if (A.n_ins <= 0) return;
  // (each block adds its counts with one atomic per counter: few blocks)
  k_ds_resolve<<<grid_for(A.n_ins, 512), TPB, 0, st>>>(A, X.items, X.item_count);
  DC_LAUNCH_CHECK();
  // chunks: at most one per source plus one per MARK_CHUNK entries of G_t
  const int64_t cap = X.item_cap;
  k_mark_rows<<<wave_grid(cap < 65536 ? cap : 65536), TPB, 0, st>>>(X.items, X.item_count,
                                                                    A.adj, A.R);
  DC_LAUNCH_CHECK();
}

int64_t ds_item_cap(int64_t n_sources, int64_t nnz) {
  return n_sources + nnz / MARK_CHUNK + 1;
}

void ds_additions(const LevelView& g, const int32_t* C, const int32_t* a, long long two_m,
                  const uint64_t* ins_keys, int64_t n_ins, const int32_t* seg_beg,
                  const int32_t* seg_end, const Bins& bins, uint8_t* R, uint8_t* cflag,
                  uint8_t* accflag, const DsScratch& X, long long* stat, hipStream_t st) {
  EvalArgs A{};
  A.off = g.off;
  A.nnz = g.nnz;
  A.adj = g.adj;
  A.k = g.k;
  A.C = C;
  A.a = a;
  A.two_m = two_m;
  A.stat = stat;
  A.ins_keys = ins_keys;
  A.seg_beg = seg_beg;
  A.seg_end = seg_end;
  A.n_ins = n_ins;
  A.n0 = g.n;
  A.R = R;
  A.cflag = cflag;
  A.accflag = accflag;
  A.sink_g = X.sink_g;
  A.best_j = X.best_j;
  A.best_g = X.best_g;
  launch_eval<EV_DSADD>(A, bins, st, nullptr, nullptr);
  ds_resolve(A, X, st);
}

void ds_both(const LevelView& g, const int32_t* C, const int32_t* a, const int32_t* sz,
             int32_t guard, long long two_m, const uint64_t* ins_keys, int64_t n_ins,
             const int32_t* seg_beg, const int32_t* seg_end, const uint8_t* uflag,
             const Bins& bins, uint8_t* R, uint8_t* cflag, uint8_t* accflag, int32_t* pre,
             const DsScratch& X, long long* stat, hipStream_t st) {
  EvalArgs A{};
  A.sz = sz;
  A.guard = guard;
  A.pre = pre;
  A.off = g.off;
  A.nnz = g.nnz;
  A.adj = g.adj;
  A.k = g.k;
  A.C = C;
  A.a = a;
  A.two_m = two_m;
  A.stat = stat;
  A.ins_keys = ins_keys;
  A.seg_beg = seg_beg;
  A.seg_end = seg_end;
  A.n_ins = n_ins;
  A.n0 = g.n;
  A.R = R;
  A.cflag = cflag;
  A.accflag = accflag;
  A.uflag = uflag;
  A.sink_g = X.sink_g;
  A.best_j = X.best_j;
  A.best_g = X.best_g;
  launch_eval<EV_DSBOTH>(A, bins, st, nullptr, nullptr);
  ds_resolve(A, X, st);
}

void feat_eval(const LevelView& g, const int32_t* C, const int32_t* a, long long two_m,
               const Bins& bins, int32_t* f_own, long long* f_g1, long long* f_g2,
               long long* stat, hipStream_t st, const int32_t* sz, int guard, int32_t* pre) {
  EvalArgs A{};
  A.stat = stat;
  A.sz = sz;
  A.guard = guard;
  A.pre = pre;
  A.off = g.off;
  A.nnz = g.nnz;
  A.adj = g.adj;
  A.k = g.k;
  A.C = C;
  A.a = a;
  A.two_m = two_m;
  A.n0 = g.n;
  A.f_own = f_own;
  A.f_g1 = f_g1;
  A.f_g2 = f_g2;
  launch_eval<EV_FEAT>(A, bins, st, nullptr, nullptr);
}

EvalArgs sweep_args(const LevelView& g, const int32_t* C, int32_t* Cn, const int32_t* a,
                    const int32_t* sz, long long two_m, int guard, long long* stat) {
  EvalArgs A{};
  A.stat = stat;
  A.off = g.off;
  A.nnz = g.nnz;
  A.adj = g.adj;
  A.k = g.k;
  A.C = C;
  A.Cn = Cn;
  A.a = a;
  A.sz = sz;
  A.two_m = two_m;
  A.guard = guard;
  A.n0 = g.n;
  return A;
}

void build_multi_bins(const Bins* const* bins, int ngraphs, MultiBins& mb, MultiSeg* segs_host,
                      DBuf& segs_dev, hipStream_t st) {
  constexpr int PAD[NBINS] = {WAVE / 16, WAVE / 32, 1, 1, 1, 1};
  int nsegs = 0;
  for (int q = 0; q < NBINS; ++q) {
    int64_t off = 0;
    for (int j = 0; j < ngraphs; ++j) {
      const int64_t n = bins[j]->n[q];
      if (n == 0) continue;
      const int64_t padded = ceil_div(n, PAD[q]) * PAD[q];
      segs_host[nsegs++] = MultiSeg{bins[j]->list[q], n, padded, off, j, q};
      off += padded;
    }
    mb.count[q] = off;
    mb.list[q].ensure(size_t(off + 1) * 4);
    mb.gid[q].ensure(size_t(off + 1) * 4);
  }
  mb.lidx.ensure(size_t(mb.count[NBINS - 1] + 1) * 4);
  if (nsegs == 0) return;
  segs_dev.ensure(size_t(nsegs) * sizeof(MultiSeg));
  DC_HIP(hipMemcpyAsync(segs_dev.p, segs_host, size_t(nsegs) * sizeof(MultiSeg),
                        hipMemcpyHostToDevice, st));
  MultiDst D;
  for (int q = 0; q < NBINS; ++q) {
    D.list[q] = mb.list[q].as<int32_t>();
    D.gid[q] = mb.gid[q].as<int32_t>();
  }
  D.lidx = mb.lidx.as<int32_t>();
  k_build_multi<<<nsegs, TPB, 0, st>>>(segs_dev.as<MultiSeg>(), nsegs, D);
  DC_LAUNCH_CHECK();
}

void sweep_eval_multi(const EvalArgs* descs, const int32_t* done, const MultiBins& mb,
                      hipStream_t st) {
  auto args = [&](int q) {
    return MultiArgs{descs, mb.list[q].as<int32_t>(), mb.gid[q].as<int32_t>(), done,
                     mb.count[q]};
  };
  if (mb.count[0] > 0) {
    k_sweep_group_multi<16><<<wave_grid(ceil_div(mb.count[0], 4)), TPB, 0, st>>>(args(0));
    DC_LAUNCH_CHECK();
  }
  if (mb.count[1] > 0) {
    k_sweep_group_multi<32><<<wave_grid(ceil_div(mb.count[1], 2)), TPB, 0, st>>>(args(1));
    DC_LAUNCH_CHECK();
  }
  if (mb.count[2] > 0) {
    k_sweep_group_multi<64><<<wave_grid(mb.count[2]), TPB, 0, st>>>(args(2));
    DC_LAUNCH_CHECK();
  }
  if (mb.count[3] > 0) {
    k_sweep_wtab_multi<<<wave_grid(mb.count[3]), TPB, 0, st>>>(args(3));
    DC_LAUNCH_CHECK();
  }
  if (mb.count[4] > 0) {
    const int64_t nb = mb.count[4] < 16384 ? mb.count[4] : 16384;
    k_sweep_btab_multi<<<int(nb), TPB, 0, st>>>(args(4));
    DC_LAUNCH_CHECK();
  }
  if (mb.count[5] > 0) {
    k_sweep_gtab_multi<<<int(mb.count[5]), GTPB, 0, st>>>(args(5), mb.lidx.as<int32_t>());
    DC_LAUNCH_CHECK();
  }
}

EvalArgs sweep_args_bins(const LevelView& g, const int32_t* C, int32_t* Cn, const int32_t* a,
                         const int32_t* sz, long long two_m, int guard, long long* stat,
                         const Bins& bins) {
  EvalArgs A = sweep_args(g, C, Cn, a, sz, two_m, guard, stat);
  A.gkeys = bins.gkeys;
  A.gvals = bins.gvals;
  A.tab_off = bins.tab_off;
  A.gslots = bins.gslots;
  return A;
}

}  // namespace dc
