// louvain.hip -- per-vertex evaluation kernels and sweep bookkeeping.
//
// One templated body evaluates a vertex i against the communities of its
// neighbours: it aggregates e_{i->X} = sum of w(i,v) over neighbours v != i
// with C(v) = X into a hash table (LDS for rows up to 2048 entries, global
// memory beyond), then scores
//     score(X) = 2m * e_{i->X} - k_i * a_X^{(-i)}
// in exact int64 (the modularity gain of Sec. 3.1 scaled by (2m)^2/2) and
// reduces with wave shuffles.  Three consumers share it:
//   EV_SWEEP  -- the Louvain move rule of Alg. 1 (best neighbouring community,
//                smallest label on ties, strict improvement, minimum-label
//                guard for two singletons), synchronous over the active set;
//   EV_DSADD  -- Alg. 2: the best sink community of a source of new edges,
//                the conflict test gain1 >= gain2 against the reverse move of
//                j*, and the R_t update {i, j*} + Gamma(i) + C_{t-1}(j*);
//   EV_DSDEL  -- the deletion rule: best move of a source of an
//                intra-community deletion.
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
  const int32_t* list;  // vertices (or sources) of this bin
  const int32_t* count; // device count of list
  // global tables (bin 2)
  int* gkeys;
  int* gvals;
  const long long* tab_off;
  // movers
  int32_t* movers;
  long long* stat;
  // Alg. 2 inputs
  const uint64_t* ins_keys;  // sorted directed insertion keys src*n0+dst
  int64_t n_ins;
  int32_t n0;                // vertices of the level-0 graph
  uint8_t* R;
  uint8_t* cflag;
};

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

// Group = one wave (G = 64) or the whole block (G = 256).
template <int G>
struct GroupLds {
  Best best[NW];
  Cand cand[NW];
  long long s0[NW];
  long long s1[NW];
  int own;
};

template <int G>
__device__ __forceinline__ void group_sync() {
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
__device__ __forceinline__ void group_sum2(long long& x, long long& y,
                                          GroupLds<G>& L) {
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
  for (int w = 0; w < NW; ++w) {
    x += L.s0[w];
    y += L.s1[w];
  }
  __syncthreads();
}

// Evaluation of one item by one group.  S = LDS slots per group (0: global).
template <int MODE, int G, int S>
__device__ void eval_item(const EvalArgs& A, int64_t idx, bool valid,
                          int* keys, int* vals, uint32_t mask,
                          GroupLds<G>& L, int* own_slot) {
  const int t = (G == WAVE) ? lane_id() : int(threadIdx.x);
  const int i = valid ? A.list[idx] : 0;
  const int32_t rb = valid ? A.off[i] : 0;
  const int32_t re = valid ? A.off[i + 1] : 0;
  const int c = valid ? A.C[i] : 0;
  const long long ki = valid ? A.k[i] : 0;

  // phase 0: clear the table (a group without an item leaves it alone)
  if (valid) {
    for (uint32_t s = t; s <= mask; s += G) {
      keys[s] = EMPTY_KEY;
      vals[s] = 0;
    }
  }
  if (t == 0) *own_slot = 0;
  group_sync<G>();
  // phase 1: e_{i->X} over the row, the diagonal entry excluded
  for (int32_t j = rb + t; j < re; j += G) {
    int2 e = A.adj[j];
    if (e.x == i) continue;
    table_add(keys, vals, mask, A.C[e.x], e.y);
  }
  group_sync<G>();
  if (MODE == EV_DSADD) {
    // gains toward the communities of the new sinks of source i
    Cand best = {NO_SCORE, NO_LABEL, NO_LABEL};
    long long s_own = 0;
    if (valid) {
      int e_own = table_get(keys, vals, mask, c);
      s_own = A.two_m * e_own - ki * (A.a[c] - ki);
      const uint64_t base = uint64_t(i) * uint64_t(A.n0);
      // the sinks of i: the run of keys in [i*n0, (i+1)*n0)
      int64_t q0 = 0, q1 = A.n_ins;
      while (q0 < q1) {
        int64_t mid = (q0 + q1) >> 1;
        if (A.ins_keys[mid] < base)
          q0 = mid + 1;
        else
          q1 = mid;
      }
      for (int64_t q = q0 + t; q < A.n_ins && A.ins_keys[q] < base + uint64_t(A.n0); q += G) {
        int j = int(A.ins_keys[q] - base);
        int X = A.C[j];
        long long g = 0;
        if (X != c) g = A.two_m * table_get(keys, vals, mask, X) - ki * A.a[X] - s_own;
        Cand cd = {g, X, j};
        if (cand_better(cd, best)) best = cd;
      }
    }
    best = group_cand<G>(best, L);
    // gain2 = G(j* -> C(i)) from the row of j*
    long long e_to = 0, e_self = 0;
    const int js = best.j;
    const int cj = best.x;
    bool live = valid && best.j != NO_LABEL && cj != c;
    if (live) {
      for (int32_t q = A.off[js] + t; q < A.off[js + 1]; q += G) {
        int2 e = A.adj[q];
        if (e.x == js) continue;
        int X = A.C[e.x];
        if (X == c) e_to += e.y;
        if (X == cj) e_self += e.y;
      }
    }
    group_sum2<G>(e_to, e_self, L);
    if (live) {
      long long kj = A.k[js];
      long long g2 = (A.two_m * e_to - kj * A.a[c]) - (A.two_m * e_self - kj * (A.a[cj] - kj));
      bool accept = best.g >= g2 && best.g > 0;
      if (accept) {
        for (int32_t q = rb + t; q < re; q += G) A.R[A.adj[q].x] = 1;
        if (t == 0) {
          A.R[i] = 1;
          A.R[js] = 1;
          A.cflag[cj] = 1;
          atomicAdd((unsigned long long*)&A.stat[ST_DS_ACC], 1ull);
        }
      }
    }
    if (valid && t == 0) atomicAdd((unsigned long long*)&A.stat[ST_DS_SRC], 1ull);
    return;
  }
  // phase 2 (sweep, deletion rule): best other community and e_{i->C(i)}
  Best b = {NO_SCORE, NO_LABEL};
  for (uint32_t s = t; valid && s <= mask; s += G) {
    int X = keys[s];
    if (X == EMPTY_KEY) continue;
    int e = vals[s];
    if (X == c) {
      *own_slot = e;
      continue;
    }
    long long sc = A.two_m * e - ki * A.a[X];
    if (better(sc, X, b.s, b.x)) {
      b.s = sc;
      b.x = X;
    }
  }
  b = group_best<G>(b, L);
  group_sync<G>();
  if (!valid) return;
  const long long s_own = A.two_m * (long long)(*own_slot) - ki * (A.a[c] - ki);
  bool move = b.x != NO_LABEL && b.s > s_own;
  if (MODE == EV_SWEEP) {
    if (move && A.guard && A.sz[c] == 1 && A.sz[b.x] == 1 && b.x > c) move = false;
    if (move && t == 0) {
      A.Cn[i] = b.x;
      unsigned long long p = atomicAdd((unsigned long long*)&A.stat[ST_MOVES], 1ull);
      A.movers[p] = i;
    }
  } else {  // EV_DSDEL
    if (move) {
      for (int32_t q = rb + t; q < re; q += G) A.R[A.adj[q].x] = 1;
      if (t == 0) {
        A.R[i] = 1;
        A.cflag[b.x] = 1;
        atomicAdd((unsigned long long*)&A.stat[ST_DEL_ACC], 1ull);
      }
    }
    if (t == 0) atomicAdd((unsigned long long*)&A.stat[ST_DEL_SRC], 1ull);
  }
}

// Bin 0: one wave per item, LDS table of WAVE_SLOTS per wave.
template <int MODE>
__global__ void __launch_bounds__(TPB) k_eval_wave(EvalArgs A) {
  __shared__ int keys[NW][WAVE_SLOTS];
  __shared__ int vals[NW][WAVE_SLOTS];
  __shared__ GroupLds<WAVE> L[NW];
  __shared__ int own[NW];
  const int wid = threadIdx.x / WAVE;
  const int64_t idx = int64_t(blockIdx.x) * NW + wid;
  const bool valid = idx < *A.count;
  eval_item<MODE, WAVE, WAVE_SLOTS>(A, idx, valid, keys[wid], vals[wid],
                                    WAVE_SLOTS - 1, L[wid], &own[wid]);
}

// Bin 1: one block per item, LDS table of BLOCK_SLOTS.
template <int MODE>
__global__ void __launch_bounds__(TPB) k_eval_block(EvalArgs A) {
  __shared__ int keys[BLOCK_SLOTS];
  __shared__ int vals[BLOCK_SLOTS];
  __shared__ GroupLds<TPB> L;
  __shared__ int own;
  const int64_t idx = blockIdx.x;
  const bool valid = idx < *A.count;
  eval_item<MODE, TPB, BLOCK_SLOTS>(A, idx, valid, keys, vals, BLOCK_SLOTS - 1, L, &own);
}

// Bin 2: one block per item, table in global memory sized 2 * pow2 >= 2 deg.
template <int MODE>
__global__ void __launch_bounds__(TPB) k_eval_global(EvalArgs A) {
  __shared__ GroupLds<TPB> L;
  __shared__ int own;
  const int64_t idx = blockIdx.x;
  const bool valid = idx < *A.count;
  long long o0 = valid ? A.tab_off[idx] : 0;
  long long o1 = valid ? A.tab_off[idx + 1] : 1;
  uint32_t mask = uint32_t(o1 - o0) - 1;
  eval_item<MODE, TPB, 0>(A, idx, valid, A.gkeys + o0, A.gvals + o0, mask, L, &own);
}

// ---------------------------------------------------------------------------

__global__ void k_bin(const int32_t* __restrict__ list, const int32_t* count_dev,
                      int64_t count_host, const int32_t* __restrict__ off,
                      int32_t lim0, int32_t lim1, int32_t* out0, int32_t* out1,
                      int32_t* out2, int32_t* counts, long long* vol) {
  const int64_t cnt = count_dev ? *count_dev : count_host;
  const uint64_t lt = (uint64_t(1) << lane_id()) - 1;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t base = int64_t(blockIdx.x) * blockDim.x; base < cnt; base += stride) {
    int64_t i = base + threadIdx.x;
    bool valid = i < cnt;
    int v = valid ? (list ? list[i] : int(i)) : 0;
    int d = valid ? off[v + 1] - off[v] : 0;
    int bin = !valid ? -1 : (d <= lim0 ? 0 : (d <= lim1 ? 1 : 2));
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      uint64_t m = __ballot(bin == b);
      if (m == 0) continue;
      int leader = __ffsll((unsigned long long)m) - 1;
      int basepos = 0;
      if (lane_id() == leader) basepos = atomicAdd(&counts[b], __popcll(m));
      basepos = __shfl(basepos, leader, WAVE);
      int32_t* out = b == 0 ? out0 : (b == 1 ? out1 : out2);
      if (bin == b) out[basepos + __popcll(m & lt)] = v;
      long long dv = bin == b ? d : 0;
      dv = wave_sum(dv);
      if (lane_id() == 0 && dv) atomicAdd((unsigned long long*)&vol[b], (unsigned long long)dv);
    }
  }
}

__global__ void k_table_caps(const int32_t* __restrict__ list,
                             const int32_t* __restrict__ off, int64_t cnt,
                             long long* caps) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < cnt;
       i += int64_t(gridDim.x) * blockDim.x) {
    int v = list[i];
    long long d = off[v + 1] - off[v];
    long long c = 2;
    while (c < 2 * d) c <<= 1;
    caps[i] = c;
  }
}

// Moves of a sweep: community totals and sizes change by (-k, -1) on the old
// label and (+k, +1) on the new one; packed as size*2^32 + total so one
// 64-bit atomic carries both, pre-combined per block.
__device__ __forceinline__ long long pack2(int da, int dsz) {
  return (long long)dsz * 4294967296LL + (long long)da;
}

__global__ void __launch_bounds__(TPB)
    k_apply_moves(const int32_t* __restrict__ movers, const long long* stat,
                  const int32_t* __restrict__ C, const int32_t* __restrict__ Cn,
                  const int32_t* __restrict__ k, long long* dpack,
                  int32_t* tflag, int32_t* tlist, long long* stat_w) {
  __shared__ AggLds agg;
  const int64_t cnt = stat[ST_MOVES];
  const int64_t stride = int64_t(gridDim.x) * TPB;
  for (int64_t base = int64_t(blockIdx.x) * TPB; base < cnt; base += stride) {
    agg_init(agg);
    __syncthreads();
    int64_t p = base + threadIdx.x;
    if (p < cnt) {
      int u = movers[p];
      int ku = k[u];
      agg_put(agg, C[u], pack2(-ku, -1));
      agg_put(agg, Cn[u], pack2(ku, 1));
    }
    __syncthreads();
    for (int s = threadIdx.x; s < AGG_SLOTS; s += TPB) {
      int X = agg.keys[s];
      if (X == EMPTY_KEY) continue;
      long long v = agg.vals[s];
      if (v == 0) continue;
      atomicAdd((unsigned long long*)&dpack[X], (unsigned long long)v);
      if (atomicExch(&tflag[X], 1) == 0) {
        unsigned long long q = atomicAdd((unsigned long long*)&stat_w[ST_TOUCHED], 1ull);
        tlist[q] = X;
      }
    }
    __syncthreads();
  }
}

// Exact change of I = sum of intra-community entry weights over the movers'
// rows: an entry to a non-mover stands for both orientations.
__global__ void __launch_bounds__(TPB)
    k_delta_intra(const int32_t* __restrict__ movers, const long long* stat,
                  const int32_t* __restrict__ off, const int2* __restrict__ adj,
                  const int32_t* __restrict__ C, const int32_t* __restrict__ Cn,
                  long long* stat_w) {
  const int64_t cnt = stat[ST_MOVES];
  const int64_t nwaves = int64_t(gridDim.x) * NW;
  const int lane = lane_id();
  long long s = 0;
  for (int64_t p = int64_t(blockIdx.x) * NW + threadIdx.x / WAVE; p < cnt; p += nwaves) {
    int u = movers[p];
    int cu = C[u], nu = Cn[u];
    for (int32_t j = off[u] + lane; j < off[u + 1]; j += WAVE) {
      int2 e = adj[j];
      if (e.x == u) continue;
      int cy = C[e.x], ny = Cn[e.x];
      int d = int(nu == ny) - int(cu == cy);
      if (d) s += (long long)e.y * d * (cy != ny ? 1 : 2);
    }
  }
  s = wave_sum(s);
  if (lane == 0 && s) atomicAdd((unsigned long long*)&stat_w[ST_DI], (unsigned long long)s);
}

__device__ __forceinline__ int unpack_lo(long long d) { return int(uint32_t(uint64_t(d))); }
__device__ __forceinline__ int unpack_hi(long long d) {
  return int((d - (long long)unpack_lo(d)) >> 32);
}

__global__ void k_delta_squares(const int32_t* __restrict__ tlist,
                                long long* stat, const long long* __restrict__ dpack,
                                const int32_t* __restrict__ a) {
  const int64_t cnt = stat[ST_TOUCHED];
  long long s = 0;
  for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < cnt;
       p += int64_t(gridDim.x) * blockDim.x) {
    int X = tlist[p];
    long long ao = a[X];
    long long an = ao + unpack_lo(dpack[X]);
    s += an * an - ao * ao;
  }
  s = wave_sum(s);
  if (lane_id() == 0 && s) atomicAdd((unsigned long long*)&stat[ST_DS], (unsigned long long)s);
}

__global__ void k_finalize(long long* stat, long long two_m) {
  long long dN = two_m * stat[ST_DI] - stat[ST_DS];
  stat[ST_DN] = dN;
  stat[ST_KEEP] = (stat[ST_MOVES] > 0 && dN >= 0) ? 1 : 0;
}

__global__ void k_commit(const int32_t* __restrict__ movers,
                         const int32_t* __restrict__ tlist, const long long* stat,
                         int32_t* C, int32_t* Cn, long long* dpack, int32_t* tflag,
                         int32_t* a, int32_t* sz) {
  const int64_t nm = stat[ST_MOVES], nt = stat[ST_TOUCHED];
  const bool keep = stat[ST_KEEP] != 0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < nm; p += stride) {
    int u = movers[p];
    if (keep)
      C[u] = Cn[u];
    else
      Cn[u] = C[u];
  }
  for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < nt; p += stride) {
    int X = tlist[p];
    long long d = dpack[X];
    if (keep) {
      a[X] += unpack_lo(d);
      sz[X] += unpack_hi(d);
    }
    dpack[X] = 0;
    tflag[X] = 0;
  }
}

__global__ void k_reset_sweep(long long* stat) {
  int t = threadIdx.x;
  if (t == ST_MOVES || t == ST_TOUCHED || t == ST_DI || t == ST_DS || t == ST_DN ||
      t == ST_KEEP)
    stat[t] = 0;
}

template <int MODE>
void launch_eval(const EvalArgs& base, const Bins& bins, hipStream_t st,
                 hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
  EvalArgs A = base;
  if (bins.n[0] > 0) {
    A.list = bins.list[0];
    A.count = bins.count_dev + 0;
    if (ev0) DC_HIP(hipEventRecord(ev0, st));
    k_eval_wave<MODE><<<ceil_div(bins.n[0], NW), TPB, 0, st>>>(A);
    DC_LAUNCH_CHECK();
    if (ev1) DC_HIP(hipEventRecord(ev1, st));
  }
  if (bins.n[1] > 0) {
    A.list = bins.list[1];
    A.count = bins.count_dev + 1;
    k_eval_block<MODE><<<bins.n[1], TPB, 0, st>>>(A);
    DC_LAUNCH_CHECK();
  }
  if (bins.n[2] > 0) {
    A.list = bins.list[2];
    A.count = bins.count_dev + 2;
    A.gkeys = bins.gkeys;
    A.gvals = bins.gvals;
    A.tab_off = bins.tab_off;
    k_eval_global<MODE><<<bins.n[2], TPB, 0, st>>>(A);
    DC_LAUNCH_CHECK();
  }
}

inline int grid_for(int64_t n, int cap = 4096) {
  int64_t g = ceil_div(n, TPB);
  if (g > cap) g = cap;
  return int(g < 1 ? 1 : g);
}

}  // namespace

void make_bins(const int32_t* list, const int32_t* count_dev, int64_t count_host,
               const int32_t* off, Bins& b, BinScratch& s, hipStream_t st) {
  // count_host is an upper bound of the list length
  int64_t cap = count_host > 0 ? count_host : 1;
  for (int i = 0; i < 3; ++i) s.lists[i].ensure(size_t(cap) * sizeof(int32_t));
  constexpr size_t META = 4 * sizeof(int32_t) + 3 * sizeof(long long);
  s.counts.ensure(META);
  int32_t* counts = s.counts.as<int32_t>();
  long long* vol = reinterpret_cast<long long*>(counts + 4);
  DC_HIP(hipMemsetAsync(counts, 0, META, st));
  if (count_host > 0) {
    k_bin<<<grid_for(count_host), TPB, 0, st>>>(list, count_dev, count_host, off,
                                                WAVE_SLOTS / 2, BLOCK_SLOTS / 2,
                                                s.lists[0].as<int32_t>(), s.lists[1].as<int32_t>(),
                                                s.lists[2].as<int32_t>(), counts, vol);
    DC_LAUNCH_CHECK();
  }
  // host needs the counts for the grids
  DC_HIP(hipMemcpyAsync(s.host, counts, META, hipMemcpyDeviceToHost, st));
  DC_HIP(hipStreamSynchronize(st));
  const int32_t* hc = reinterpret_cast<const int32_t*>(s.host);
  const long long* hv = reinterpret_cast<const long long*>(hc + 4);
  for (int i = 0; i < 3; ++i) {
    b.n[i] = hc[i];
    b.list[i] = s.lists[i].as<int32_t>();
    b.vol[i] = hv[i];
  }
  b.count_dev = counts;
  b.gkeys = nullptr;
  b.gvals = nullptr;
  b.tab_off = nullptr;
  if (b.n[2] > 0) {
    s.tab_off.ensure(size_t(b.n[2] + 1) * sizeof(long long));
    long long* caps = s.tab_off.as<long long>();
    k_table_caps<<<grid_for(b.n[2]), TPB, 0, st>>>(b.list[2], off, b.n[2], caps);
    DC_LAUNCH_CHECK();
    scan_excl_i64(reinterpret_cast<int64_t*>(caps), reinterpret_cast<int64_t*>(caps), b.n[2],
                  reinterpret_cast<int64_t*>(caps + b.n[2]), st);
    size_t slots = size_t(4 * hv[2] + 2 * b.n[2] + 16);
    s.gkeys.ensure(slots * sizeof(int));
    s.gvals.ensure(slots * sizeof(int));
    b.gkeys = s.gkeys.as<int>();
    b.gvals = s.gvals.as<int>();
    b.tab_off = caps;
  }
}

void sweep_eval(const LevelView& g, const int32_t* C, int32_t* Cn, const int32_t* a,
                const int32_t* sz, long long two_m, int guard, const Bins& bins,
                int32_t* movers, long long* stat, hipStream_t st, hipEvent_t ev0,
                hipEvent_t ev1) {
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
  A.movers = movers;
  A.stat = stat;
  A.n0 = g.n;
  launch_eval<EV_SWEEP>(A, bins, st, ev0, ev1);
}

void sweep_reset(long long* stat, hipStream_t st) {
  k_reset_sweep<<<1, 64, 0, st>>>(stat);
  DC_LAUNCH_CHECK();
}

void sweep_apply(const LevelView& g, int32_t* C, int32_t* Cn, int32_t* a, int32_t* sz,
                 long long two_m, int64_t max_movers, int32_t* movers, long long* dpack,
                 int32_t* tflag, int32_t* tlist, long long* stat, hipStream_t st) {
  int grid = grid_for(max_movers, 2048);
  k_apply_moves<<<grid, TPB, 0, st>>>(movers, stat, C, Cn, g.k, dpack, tflag, tlist, stat);
  DC_LAUNCH_CHECK();
  k_delta_intra<<<grid_for(max_movers * WAVE, 4096), TPB, 0, st>>>(movers, stat, g.off, g.adj,
                                                                   C, Cn, stat);
  DC_LAUNCH_CHECK();
  k_delta_squares<<<grid_for(2 * max_movers, 2048), TPB, 0, st>>>(tlist, stat, dpack, a);
  DC_LAUNCH_CHECK();
  k_finalize<<<1, 1, 0, st>>>(stat, two_m);
  DC_LAUNCH_CHECK();
  k_commit<<<grid_for(2 * max_movers, 2048), TPB, 0, st>>>(movers, tlist, stat, C, Cn, dpack,
                                                           tflag, a, sz);
  DC_LAUNCH_CHECK();
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
  launch_eval<EV_DSADD>(A, bins, st);
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
  launch_eval<EV_DSDEL>(A, bins, st);
}

}  // namespace dc
