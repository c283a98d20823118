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
// ballot, sums their weights with a wave reduction, and parks the pair in
// the lane numbered by the iteration: one register-only iteration per
// distinct label.  The community totals are then gathered (or the table
// inserts issued) by all pair-holding lanes at once, so no chain of
// dependent memory accesses remains.  Rows of up to 64 entries finish this
// way (bin S, one wave per vertex).  Longer rows collect per 64-entry chunk
// and add the chunk's pairs to a hash table: wave-private LDS for rows up
// to 256 entries (bin W), a block-shared LDS table up to 4096 (bin B),
// global memory beyond (bin G).  A sweep writes only the next label;
// movers are collected afterwards.
#include "dc_louvain.h"

namespace dc {

namespace {

constexpr int TPB = 256;
constexpr int NW = TPB / WAVE;

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
  const int32_t* count;  // device count of list
  int* gkeys;            // bin G tables
  int* gvals;
  const long long* tab_off;
  long long* stat;
  const uint64_t* ins_keys;  // Alg. 2: sorted directed insertions src*n0+dst
  int64_t n_ins;
  int32_t n0;
  uint8_t* R;
  uint8_t* cflag;
};

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Orders LDS traffic among the lanes of one wave (no cross-wave barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Groups the valid lanes by label: lane r (r < return value) receives the
// r-th distinct label (order of first appearance) and its weight sum.  One
// iteration per distinct label, register-only, no memory traffic, so the
// gathers and inserts that follow run in parallel across lanes.
__device__ __forceinline__ int wave_collect(bool valid, int key, int w, int& ck, int& cs) {
  const int lane = lane_id();
  uint64_t rem = __ballot(valid);
  int r = 0;
  while (rem) {
    const int leader = __ffsll((unsigned long long)rem) - 1;
    const int kl = __builtin_amdgcn_readlane(key, leader);
    const bool mine = valid && key == kl;
    rem &= ~__ballot(mine);
    const int s = wave_sum(mine ? w : 0);
    if (lane == r) {
      ck = kl;
      cs = s;
    }
    ++r;
  }
  return r;
}

// Weight sum of label X among the collected pairs (0 if absent).
__device__ __forceinline__ int collected_sum(int nd, int ck, int cs, int X) {
  const uint64_t m = __ballot(lane_id() < nd && ck == X);
  return m ? __builtin_amdgcn_readlane(cs, __ffsll((unsigned long long)m) - 1) : 0;
}

struct Cand {  // Alg. 2 candidate: larger gain, then smaller C(j), then smaller j
  long long g;
  int x;
  int j;
};

__device__ __forceinline__ bool cand_better(const Cand& p, const Cand& q) {
  return p.g > q.g || (p.g == q.g && (p.x < q.x || (p.x == q.x && p.j < q.j)));
}

__device__ __forceinline__ Cand wave_cand(Cand c) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    Cand y;
    y.g = __shfl_xor(c.g, o, WAVE);
    y.x = __shfl_xor(c.x, o, WAVE);
    y.j = __shfl_xor(c.j, o, WAVE);
    if (cand_better(y, c)) c = y;
  }
  return c;
}

// Sources of i among the sorted directed insertion keys: [q0, q1).
__device__ __forceinline__ void sink_range(const EvalArgs& A, int i, int64_t& q0,
                                           int64_t& q1) {
  const uint64_t base = uint64_t(i) * uint64_t(A.n0);
  int64_t lo = 0, hi = A.n_ins;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (A.ins_keys[mid] < base) lo = mid + 1; else hi = mid;
  }
  q0 = lo;
  hi = A.n_ins;
  const uint64_t end = base + uint64_t(A.n0);
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (A.ins_keys[mid] < end) lo = mid + 1; else hi = mid;
  }
  q1 = lo;
}

// gain2 of Alg. 2: G(j* -> c), streamed over the row of j* by one wave.
__device__ __forceinline__ long long reverse_gain(const EvalArgs& A, int js, int cj, int c) {
  long long e_to = 0, e_self = 0;
  for (int32_t q = A.off[js] + lane_id(); q < A.off[js + 1]; q += WAVE) {
    int2 e = A.adj[q];
    if (e.x == js) continue;
    int X = A.C[e.x];
    if (X == c) e_to += e.y;
    if (X == cj) e_self += e.y;
  }
  e_to = wave_sum(e_to);
  e_self = wave_sum(e_self);
  const long long kj = A.k[js];
  return (A.two_m * e_to - kj * A.a[c]) - (A.two_m * e_self - kj * (A.a[cj] - kj));
}

// --------------------------------------------------------------------------
// bin S: rows of at most 64 entries, one wave per vertex, no table.

template <int MODE>
__global__ void __launch_bounds__(TPB) k_eval_small(EvalArgs A) {
  const int lane = lane_id();
  const int64_t cnt = *A.count;
  const int64_t nwaves = int64_t(gridDim.x) * NW;
  long long accepted = 0;
  for (int64_t idx = int64_t(blockIdx.x) * NW + threadIdx.x / WAVE; idx < cnt; idx += nwaves) {
    const int i = uniform(A.list[idx]);
    const int32_t rb = A.off[i], re = A.off[i + 1];
    const int c = A.C[i];
    const long long ki = A.k[i];
    bool valid = rb + lane < re;
    int2 e = valid ? A.adj[rb + lane] : make_int2(0, 0);
    if (e.x == i) valid = false;
    const int key = valid ? A.C[e.x] : EMPTY_KEY;
    int ck = EMPTY_KEY, cs = 0;
    const int nd = wave_collect(valid, key, e.y, ck, cs);
    const long long e_own = collected_sum(nd, ck, cs, c);
    const long long s_own = A.two_m * e_own - ki * (A.a[c] - ki);
    if (MODE == EV_DSADD) {
      int64_t q0, q1;
      sink_range(A, i, q0, q1);
      const int nsk = int(q1 - q0);  // sinks are neighbours, so nsk <= 64
      const bool has = lane < nsk;
      const int j = has ? int(A.ins_keys[q0 + lane] - uint64_t(i) * uint64_t(A.n0)) : 0;
      const int Xj = has ? A.C[j] : EMPTY_KEY;
      // e_{i->C(j)} for every sink lane: scan the nd collected pairs
      long long ej = 0;
      for (int r = 0; r < nd; ++r) {
        const int kr = __builtin_amdgcn_readlane(ck, r);
        const int sr = __builtin_amdgcn_readlane(cs, r);
        if (Xj == kr) ej = sr;
      }
      Cand cd = {NO_SCORE, NO_LABEL, NO_LABEL};
      if (has) {
        long long g = Xj == c ? 0 : A.two_m * ej - ki * A.a[Xj] - s_own;
        cd = {g, Xj, j};
      }
      const Cand best = wave_cand(cd);
      if (best.j != NO_LABEL && best.x != c && best.g > 0) {
        const long long g2 = reverse_gain(A, best.j, best.x, c);
        if (best.g >= g2) {
          if (valid) A.R[e.x] = 1;
          if (lane == 0) {
            A.R[i] = 1;
            A.R[best.j] = 1;
            A.cflag[best.x] = 1;
            accepted++;
          }
        }
      }
      continue;
    }
    Best b = {NO_SCORE, NO_LABEL};
    if (lane < nd && ck != c) b = {A.two_m * cs - ki * A.a[ck], ck};
    b = wave_best(b);
    bool move = b.x != NO_LABEL && b.s > s_own;
    if (MODE == EV_SWEEP) {
      if (move && A.guard && A.sz[c] == 1 && A.sz[b.x] == 1 && b.x > c) move = false;
      if (move && lane == 0) A.Cn[i] = b.x;
    } else if (move) {  // EV_DSDEL
      if (valid) A.R[e.x] = 1;
      if (lane == 0) {
        A.R[i] = 1;
        A.cflag[b.x] = 1;
        accepted++;
      }
    }
  }
  if (MODE != EV_SWEEP && lane == 0 && accepted)
    atomicAdd((unsigned long long*)&A.stat[MODE == EV_DSADD ? ST_DS_ACC : ST_DEL_ACC],
              (unsigned long long)accepted);
}

// --------------------------------------------------------------------------
// bins W, B, G: chunked distinct loop into a hash table, then a scan of it.

template <int G>
struct GroupLds {
  Best best[NW];
  Cand cand[NW];
  long long s0[NW], s1[NW];
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
  for (int w = 1; w < NW; ++w)
    if (better(L.best[w].s, L.best[w].x, r.s, r.x)) r = L.best[w];
  __syncthreads();
  return r;
}

template <int G>
__device__ __forceinline__ Cand group_cand(Cand c, GroupLds<G>& L) {
  c = wave_cand(c);
  if (G == WAVE) return c;
  const int wid = threadIdx.x / WAVE;
  if (lane_id() == 0) L.cand[wid] = c;
  __syncthreads();
  Cand r = L.cand[0];
#pragma unroll
  for (int w = 1; w < NW; ++w)
    if (cand_better(L.cand[w], r)) r = L.cand[w];
  __syncthreads();
  return r;
}

template <int G>
__device__ __forceinline__ long long group_reverse_gain(const EvalArgs& A, int js, int cj, int c,
                                                        GroupLds<G>& L) {
  if (G == WAVE) return reverse_gain(A, js, cj, c);
  long long e_to = 0, e_self = 0;
  for (int32_t q = A.off[js] + threadIdx.x; q < A.off[js + 1]; q += G) {
    int2 e = A.adj[q];
    if (e.x == js) continue;
    int X = A.C[e.x];
    if (X == c) e_to += e.y;
    if (X == cj) e_self += e.y;
  }
  e_to = wave_sum(e_to);
  e_self = wave_sum(e_self);
  const int wid = threadIdx.x / WAVE;
  if (lane_id() == 0) {
    L.s0[wid] = e_to;
    L.s1[wid] = e_self;
  }
  __syncthreads();
  e_to = 0;
  e_self = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    e_to += L.s0[w];
    e_self += L.s1[w];
  }
  __syncthreads();
  const long long kj = A.k[js];
  return (A.two_m * e_to - kj * A.a[c]) - (A.two_m * e_self - kj * (A.a[cj] - kj));
}

// Power of two >= 2 * deg (at least 64), at most max_slots: the table is
// at most half full, and only that many slots are cleared and scanned.
__device__ __forceinline__ uint32_t table_cap(int deg, uint32_t max_slots) {
  uint32_t want = 2u * uint32_t(deg > 32 ? deg : 32);
  uint32_t cap = 1u << (32 - __clz(want - 1));
  return cap < max_slots ? cap : max_slots;
}

// One group (a wave, or the whole block) evaluates vertex i with table
// (keys, vals, mask).  Returns the number of accepted screening tests (0/1)
// in thread 0 of the group.
template <int MODE, int G>
__device__ int eval_table(const EvalArgs& A, int i, int* keys, int* vals, uint32_t mask,
                          GroupLds<G>& L, int* own) {
  const int t = (G == WAVE) ? lane_id() : int(threadIdx.x);
  const int lane = lane_id();
  const int32_t rb = A.off[i], re = A.off[i + 1];
  const int c = A.C[i];
  const long long ki = A.k[i];
  for (uint32_t s = t; s <= mask; s += G) {
    keys[s] = EMPTY_KEY;
    vals[s] = 0;
  }
  if (t == 0) *own = 0;
  group_sync<G>();
  const int w0 = (G == WAVE) ? 0 : int(threadIdx.x) / WAVE;
  for (int32_t c0 = rb + w0 * WAVE; c0 < re; c0 += G) {
    bool valid = c0 + lane < re;
    int2 e = valid ? A.adj[c0 + lane] : make_int2(0, 0);
    if (e.x == i) valid = false;
    const int key = valid ? A.C[e.x] : EMPTY_KEY;
    int ck = EMPTY_KEY, cs = 0;
    const int nd = wave_collect(valid, key, e.y, ck, cs);
    if (lane < nd) table_add(keys, vals, mask, ck, cs);
  }
  group_sync<G>();
  int accepted = 0;
  if (MODE == EV_DSADD) {
    const int e_own = table_get(keys, vals, mask, c);
    const long long s_own = A.two_m * e_own - ki * (A.a[c] - ki);
    int64_t q0, q1;
    sink_range(A, i, q0, q1);
    const uint64_t base = uint64_t(i) * uint64_t(A.n0);
    Cand best = {NO_SCORE, NO_LABEL, NO_LABEL};
    for (int64_t q = q0 + t; q < q1; q += G) {
      const int j = int(A.ins_keys[q] - base);
      const int X = A.C[j];
      long long g = 0;
      if (X != c) g = A.two_m * table_get(keys, vals, mask, X) - ki * A.a[X] - s_own;
      Cand cd = {g, X, j};
      if (cand_better(cd, best)) best = cd;
    }
    best = group_cand<G>(best, L);
    if (best.j != NO_LABEL && best.x != c && best.g > 0) {
      const long long g2 = group_reverse_gain<G>(A, best.j, best.x, c, L);
      if (best.g >= g2) {
        for (int32_t q = rb + t; q < re; q += G) A.R[A.adj[q].x] = 1;
        if (t == 0) {
          A.R[i] = 1;
          A.R[best.j] = 1;
          A.cflag[best.x] = 1;
          accepted = 1;
        }
      }
    }
    group_sync<G>();  // the table is reused by the next item of this group
    return accepted;
  }
  Best b = {NO_SCORE, NO_LABEL};
  for (uint32_t s = t; s <= mask; s += G) {
    const int X = keys[s];
    if (X == EMPTY_KEY) continue;
    const int e = vals[s];
    if (X == c) {
      *own = e;
      continue;
    }
    const long long sc = A.two_m * e - ki * A.a[X];
    if (better(sc, X, b.s, b.x)) {
      b.s = sc;
      b.x = X;
    }
  }
  b = group_best<G>(b, L);
  group_sync<G>();
  const long long s_own = A.two_m * (long long)(*own) - ki * (A.a[c] - ki);
  bool move = b.x != NO_LABEL && b.s > s_own;
  if (MODE == EV_SWEEP) {
    if (move && A.guard && A.sz[c] == 1 && A.sz[b.x] == 1 && b.x > c) move = false;
    if (move && t == 0) A.Cn[i] = b.x;
  } else if (move) {  // EV_DSDEL
    for (int32_t q = rb + t; q < re; q += G) A.R[A.adj[q].x] = 1;
    if (t == 0) {
      A.R[i] = 1;
      A.cflag[b.x] = 1;
      accepted = 1;
    }
  }
  // the table is reused by the next item of this group
  group_sync<G>();
  return accepted;
}

// bin W: one wave per vertex, wave-private LDS table
template <int MODE>
__global__ void __launch_bounds__(TPB) k_eval_wtab(EvalArgs A) {
  __shared__ int keys[NW][WTAB_SLOTS];
  __shared__ int vals[NW][WTAB_SLOTS];
  __shared__ GroupLds<WAVE> L[NW];
  __shared__ int own[NW];
  const int wid = threadIdx.x / WAVE;
  const int64_t cnt = *A.count;
  const int64_t nwaves = int64_t(gridDim.x) * NW;
  long long accepted = 0;
  for (int64_t idx = int64_t(blockIdx.x) * NW + wid; idx < cnt; idx += nwaves) {
    const int i = uniform(A.list[idx]);
    const uint32_t cap = table_cap(A.off[i + 1] - A.off[i], WTAB_SLOTS);
    accepted += eval_table<MODE, WAVE>(A, i, keys[wid], vals[wid], cap - 1, L[wid], &own[wid]);
  }
  if (MODE != EV_SWEEP && lane_id() == 0 && accepted)
    atomicAdd((unsigned long long*)&A.stat[MODE == EV_DSADD ? ST_DS_ACC : ST_DEL_ACC],
              (unsigned long long)accepted);
}

// bin B: one block per vertex, block-shared LDS table
template <int MODE>
__global__ void __launch_bounds__(TPB) k_eval_btab(EvalArgs A) {
  __shared__ int keys[BTAB_SLOTS];
  __shared__ int vals[BTAB_SLOTS];
  __shared__ GroupLds<TPB> L;
  __shared__ int own;
  const int64_t idx = blockIdx.x;
  if (idx >= *A.count) return;  // uniform over the block
  const int i = A.list[idx];
  const uint32_t cap = table_cap(A.off[i + 1] - A.off[i], BTAB_SLOTS);
  int acc = eval_table<MODE, TPB>(A, i, keys, vals, cap - 1, L, &own);
  if (MODE != EV_SWEEP && threadIdx.x == 0 && acc)
    atomicAdd((unsigned long long*)&A.stat[MODE == EV_DSADD ? ST_DS_ACC : ST_DEL_ACC], 1ull);
}

// bin G: one block per vertex, table in global memory (>= 2 slots per entry)
template <int MODE>
__global__ void __launch_bounds__(TPB) k_eval_gtab(EvalArgs A) {
  __shared__ GroupLds<TPB> L;
  __shared__ int own;
  const int64_t idx = blockIdx.x;
  if (idx >= *A.count) return;
  const int i = A.list[idx];
  const long long o0 = A.tab_off[idx], o1 = A.tab_off[idx + 1];
  int acc = eval_table<MODE, TPB>(A, i, A.gkeys + o0, A.gvals + o0, uint32_t(o1 - o0) - 1, L,
                                  &own);
  if (MODE != EV_SWEEP && threadIdx.x == 0 && acc)
    atomicAdd((unsigned long long*)&A.stat[MODE == EV_DSADD ? ST_DS_ACC : ST_DEL_ACC], 1ull);
}

// --------------------------------------------------------------------------
// binning by row length: per-block counts, one scan, stable scatter.

constexpr int BIN_ITEMS = 4;
constexpr int BIN_TILE = TPB * BIN_ITEMS;

__device__ __forceinline__ int bin_of(int d) {
  return d <= SMALL_MAX ? 0 : (d <= WTAB_MAX ? 1 : (d <= BTAB_MAX ? 2 : 3));
}

__global__ void __launch_bounds__(TPB)
    k_bin_count(const int32_t* __restrict__ list, int64_t cnt, const int32_t* __restrict__ off,
                int32_t* bcnt, long long* vol, int64_t nblocks) {
  __shared__ int c[NBINS];
  __shared__ long long v[NBINS];
  if (threadIdx.x < NBINS) {
    c[threadIdx.x] = 0;
    v[threadIdx.x] = 0;
  }
  __syncthreads();
  int lc[NBINS] = {0, 0, 0, 0};
  long long lv[NBINS] = {0, 0, 0, 0};
  for (int r = 0; r < BIN_ITEMS; ++r) {
    int64_t p = int64_t(blockIdx.x) * BIN_TILE + int64_t(r) * TPB + threadIdx.x;
    if (p < cnt) {
      int u = list ? list[p] : int(p);
      int d = off[u + 1] - off[u];
      int b = bin_of(d);
#pragma unroll
      for (int q = 0; q < NBINS; ++q) {
        if (b == q) {
          lc[q]++;
          lv[q] += d;
        }
      }
    }
  }
#pragma unroll
  for (int b = 0; b < NBINS; ++b) {
    int x = wave_sum(lc[b]);
    long long y = wave_sum(lv[b]);
    if (lane_id() == 0) {
      if (x) atomicAdd(&c[b], x);
      if (y) atomicAdd((unsigned long long*)&v[b], (unsigned long long)y);
    }
  }
  __syncthreads();
  if (threadIdx.x < NBINS) {
    bcnt[int64_t(threadIdx.x) * nblocks + blockIdx.x] = c[threadIdx.x];
    if (v[threadIdx.x])
      atomicAdd((unsigned long long*)&vol[threadIdx.x], (unsigned long long)v[threadIdx.x]);
  }
}

// out[boff[b][block] + rank] = vertex: bins are contiguous segments of out,
// in list order within each bin
__global__ void __launch_bounds__(TPB)
    k_bin_scatter(const int32_t* __restrict__ list, int64_t cnt,
                  const int32_t* __restrict__ off, const int32_t* __restrict__ boff,
                  int64_t nblocks, int32_t* out) {
  __shared__ int base[NBINS];
  __shared__ int wc[NW][NBINS];
  const int wid = threadIdx.x / WAVE, lane = lane_id();
  if (threadIdx.x < NBINS) base[threadIdx.x] = boff[int64_t(threadIdx.x) * nblocks + blockIdx.x];
  __syncthreads();
  const uint64_t lt = (uint64_t(1) << lane) - 1;
  for (int r = 0; r < BIN_ITEMS; ++r) {
    int64_t p = int64_t(blockIdx.x) * BIN_TILE + int64_t(r) * TPB + threadIdx.x;
    const bool valid = p < cnt;
    int u = 0, b = -1;
    if (valid) {
      u = list ? list[p] : int(p);
      b = bin_of(off[u + 1] - off[u]);
    }
    int rank = 0;
#pragma unroll
    for (int q = 0; q < NBINS; ++q) {
      uint64_t m = __ballot(b == q);
      if (lane == 0) wc[wid][q] = __popcll(m);
      if (b == q) rank = __popcll(m & lt);
    }
    __syncthreads();
    if (valid) {
      int pos = base[b] + rank;
      for (int w = 0; w < wid; ++w) pos += wc[w][b];
      out[pos] = u;
    }
    __syncthreads();
    if (threadIdx.x < NBINS) {
      int add = 0;
      for (int w = 0; w < NW; ++w) add += wc[w][threadIdx.x];
      base[threadIdx.x] += add;
    }
    __syncthreads();
  }
}

__global__ void k_bin_starts(const int32_t* boff, int64_t nblocks, int64_t total_entries,
                             const int32_t* total, int32_t* bin_start, int32_t* counts) {
  // boff is the exclusive scan of bcnt laid out bin-major: bin b starts at
  // boff[b * nblocks]
  if (threadIdx.x < NBINS) {
    int b = threadIdx.x;
    int s = boff[int64_t(b) * nblocks];
    int e = (b + 1 < NBINS) ? boff[int64_t(b + 1) * nblocks] : *total;
    bin_start[b] = s;
    counts[b] = e - s;
  }
  (void)total_entries;
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

template <int MODE>
void launch_eval(const EvalArgs& base, const Bins& bins, hipStream_t st, hipEvent_t ev0,
                 hipEvent_t ev1) {
  EvalArgs A = base;
  if (bins.n[0] > 0) {
    A.list = bins.list[0];
    A.count = bins.count_dev + 0;
    if (ev0) DC_HIP(hipEventRecord(ev0, st));
    k_eval_small<MODE><<<wave_grid(bins.n[0]), TPB, 0, st>>>(A);
    DC_LAUNCH_CHECK();
    if (ev1) DC_HIP(hipEventRecord(ev1, st));
  }
  if (bins.n[1] > 0) {
    A.list = bins.list[1];
    A.count = bins.count_dev + 1;
    k_eval_wtab<MODE><<<wave_grid(bins.n[1]), TPB, 0, st>>>(A);
    DC_LAUNCH_CHECK();
  }
  if (bins.n[2] > 0) {
    A.list = bins.list[2];
    A.count = bins.count_dev + 2;
    k_eval_btab<MODE><<<bins.n[2], TPB, 0, st>>>(A);
    DC_LAUNCH_CHECK();
  }
  if (bins.n[3] > 0) {
    A.list = bins.list[3];
    A.count = bins.count_dev + 3;
    A.gkeys = bins.gkeys;
    A.gvals = bins.gvals;
    A.tab_off = bins.tab_off;
    k_eval_gtab<MODE><<<bins.n[3], TPB, 0, st>>>(A);
    DC_LAUNCH_CHECK();
  }
}

}  // namespace

void make_bins(const int32_t* list, int64_t count, const int32_t* off, Bins& b, BinScratch& s,
               hipStream_t st) {
  const int64_t nb = count > 0 ? ceil_div(count, BIN_TILE) : 1;
  const int64_t cap = count > 0 ? count : 1;
  s.lists.ensure(size_t(cap) * sizeof(int32_t));
  s.bcnt.ensure(size_t(NBINS * nb + 1) * sizeof(int32_t));
  s.boff.ensure(size_t(NBINS * nb + 1) * sizeof(int32_t));
  constexpr size_t META = 16 * sizeof(int32_t) + NBINS * sizeof(long long);
  s.counts.ensure(META);
  int32_t* counts = s.counts.as<int32_t>();      // [0..3] counts, [4..7] starts, [8] total
  long long* vol = reinterpret_cast<long long*>(counts + 16);
  int32_t* bcnt = s.bcnt.as<int32_t>();
  int32_t* boff = s.boff.as<int32_t>();
  DC_HIP(hipMemsetAsync(counts, 0, META, st));
  if (count > 0) {
    k_bin_count<<<nb, TPB, 0, st>>>(list, count, off, bcnt, vol, nb);
    DC_LAUNCH_CHECK();
    scan_excl_i32(bcnt, boff, NBINS * nb, counts + 8, st);
    k_bin_starts<<<1, 64, 0, st>>>(boff, nb, NBINS * nb, counts + 8, counts + 4, counts);
    DC_LAUNCH_CHECK();
  }
  DC_HIP(hipMemcpyAsync(s.host, counts, META, hipMemcpyDeviceToHost, st));
  DC_HIP(hipStreamSynchronize(st));
  const int32_t* hc = static_cast<const int32_t*>(s.host);
  const long long* hv = reinterpret_cast<const long long*>(hc + 16);
  int32_t* lists = s.lists.as<int32_t>();
  for (int q = 0; q < NBINS; ++q) {
    b.n[q] = hc[q];
    b.list[q] = lists + hc[4 + q];
    b.vol[q] = hv[q];
  }
  b.count_dev = counts;
  b.gkeys = nullptr;
  b.gvals = nullptr;
  b.tab_off = nullptr;
  if (count > 0) {
    k_bin_scatter<<<nb, TPB, 0, st>>>(list, count, off, boff, nb, lists);
    DC_LAUNCH_CHECK();
  }
  if (b.n[3] > 0) {
    s.tab_off.ensure(size_t(b.n[3] + 1) * sizeof(long long));
    long long* caps = s.tab_off.as<long long>();
    k_table_caps<<<grid_for(b.n[3]), TPB, 0, st>>>(b.list[3], off, b.n[3], caps);
    DC_LAUNCH_CHECK();
    scan_excl_i64(reinterpret_cast<int64_t*>(caps), reinterpret_cast<int64_t*>(caps), b.n[3],
                  reinterpret_cast<int64_t*>(caps + b.n[3]), st);
    const size_t slots = size_t(4 * hv[3] + 2 * b.n[3] + 16);
    s.gkeys.ensure(slots * sizeof(int));
    s.gvals.ensure(slots * sizeof(int));
    b.gkeys = s.gkeys.as<int>();
    b.gvals = s.gvals.as<int>();
    b.tab_off = caps;
  }
}

void sweep_eval(const LevelView& g, const int32_t* C, int32_t* Cn, const int32_t* a,
                const int32_t* sz, long long two_m, int guard, const Bins& bins,
                long long* stat, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  EvalArgs A{};
  A.off = g.off;
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

void ds_additions(const LevelView& g, const int32_t* C, const int32_t* a, long long two_m,
                  const uint64_t* ins_keys, int64_t n_ins, const Bins& bins, uint8_t* R,
                  uint8_t* cflag, long long* stat, hipStream_t st) {
  EvalArgs A{};
  A.off = g.off;
  A.adj = g.adj;
  A.k = g.k;
  A.C = C;
  A.a = a;
  A.two_m = two_m;
  A.stat = stat;
  A.ins_keys = ins_keys;
  A.n_ins = n_ins;
  A.n0 = g.n;
  A.R = R;
  A.cflag = cflag;
  launch_eval<EV_DSADD>(A, bins, st, nullptr, nullptr);
}

void ds_deletions(const LevelView& g, const int32_t* C, const int32_t* a, const int32_t* sz,
                  long long two_m, const Bins& bins, uint8_t* R, uint8_t* cflag,
                  long long* stat, hipStream_t st) {
  EvalArgs A{};
  A.off = g.off;
  A.adj = g.adj;
  A.k = g.k;
  A.C = C;
  A.a = a;
  A.sz = sz;
  A.two_m = two_m;
  A.stat = stat;
  A.n0 = g.n;
  A.R = R;
  A.cflag = cflag;
  launch_eval<EV_DSDEL>(A, bins, st, nullptr, nullptr);
}

}  // namespace dc
