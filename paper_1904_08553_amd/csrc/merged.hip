// merged.hip -- the bookkeeping half of the level-0 sweeps of several graphs
// at once (serving: every in-flight graph's sweep in the same launches).
//
// Per round, every graph whose level is still running has its vertices
// evaluated (eval.hip, *_multi kernels, one launch per row-length bin for all
// graphs), then these kernels apply the moves, take the exact Delta N,
// decide keep / revert / stop on the device and commit -- one launch each
// for all graphs, a 2-D grid with the graph in blockIdx.y.  The per-graph
// state word carries convergence: 0 running, 1 stopped in this round (its
// commit still runs), 2 stopped.  The host reads the states only every few
// rounds; a stopped graph's blocks exit at once.  Every graph's arithmetic
// is the single-graph sweep's (louvain.hip), so results are the same.
#include "dc_louvain.h"

namespace dc {

namespace {

constexpr int TPB = 256;
constexpr int NW = TPB / WAVE;

__device__ __forceinline__ long long pack2(int da, int dsz) {
  return (long long)dsz * 4294967296LL + (long long)da;
}
__device__ __forceinline__ int unpack_lo(long long d) { return int(uint32_t(uint64_t(d))); }
__device__ __forceinline__ int unpack_hi(long long d) {
  return int((d - (long long)unpack_lo(d)) >> 32);
}

__device__ __forceinline__ void touch_label(int X, long long v, long long* dpack, int32_t* tflag,
                                            int32_t* tlist, long long* stat) {
  atomicAdd((unsigned long long*)&dpack[X], (unsigned long long)v);
  if (atomicExch(&tflag[X], 1) == 0) {
    const unsigned long long q = atomicAdd((unsigned long long*)&stat[ST_TOUCHED], 1ull);
    tlist[q] = X;
  }
}

// Round start: a graph stopped in the previous round becomes stopped for
// good; a running graph's per-sweep counters are cleared.
__global__ void k_mg_reset(const MergedGraph* __restrict__ G, int m, int32_t* state) {
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    if (state[j] == 1) state[j] = 2;
    if (state[j] != 0) continue;
    long long* st = G[j].stat;
    st[ST_MOVES] = 0;
    st[ST_TOUCHED] = 0;
    st[ST_DI] = 0;
    st[ST_DS] = 0;
    st[ST_DN] = 0;
    st[ST_KEEP] = 0;
  }
}

// Movers of graph blockIdx.y's active list and their label-total changes
// (pre-combined per block in LDS), as k_apply_moves.
__global__ void __launch_bounds__(TPB)
    k_mg_apply(const MergedGraph* __restrict__ G, const int32_t* __restrict__ state) {
  const int j = blockIdx.y;
  if (state[j] != 0) return;  // uniform over the block
  const MergedGraph g = G[j];
  __shared__ AggLds agg;
  __shared__ int wcount[NW];
  __shared__ int btotal;
  __shared__ long long bbase;
  const int wid = threadIdx.x / WAVE, lane = lane_id();
  const uint64_t lt = (uint64_t(1) << lane) - 1;
  const int64_t stride = int64_t(gridDim.x) * TPB;
  agg_init(agg);
  for (int64_t base = int64_t(blockIdx.x) * TPB; base < g.nact; base += stride) {
    const int64_t p = base + threadIdx.x;
    int u = 0;
    bool mover = false;
    if (p < g.nact) {
      u = g.act ? g.act[p] : int(p);
      mover = g.Cn[u] != g.C[u];
    }
    const uint64_t mk = __ballot(mover);
    if (lane == 0) wcount[wid] = __popcll(mk);
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int w = 0; w < NW; ++w) tot += wcount[w];
      btotal = tot;
      bbase = tot ? (long long)atomicAdd((unsigned long long*)&g.stat[ST_MOVES],
                                         (unsigned long long)tot)
                  : 0;
    }
    __syncthreads();
    if (btotal == 0) continue;  // uniform
    if (mover) {
      long long pos = bbase + __popcll(mk & lt);
      for (int w = 0; w < wid; ++w) pos += wcount[w];
      g.movers[pos] = u;
      const int ku = g.k[u];
      const int from = g.C[u], to = g.Cn[u];
      if (!agg_try(agg, from, pack2(-ku, -1)))
        touch_label(from, pack2(-ku, -1), g.dpack, g.tflag, g.tlist, g.stat);
      if (!agg_try(agg, to, pack2(ku, 1)))
        touch_label(to, pack2(ku, 1), g.dpack, g.tflag, g.tlist, g.stat);
    }
    __syncthreads();
  }
  __syncthreads();
  for (int s = threadIdx.x; s < AGG_SLOTS; s += TPB) {
    const int X = agg.keys[s];
    if (X == EMPTY_KEY) continue;
    const long long v = agg.vals[s];
    if (v != 0) touch_label(X, v, g.dpack, g.tflag, g.tlist, g.stat);
  }
}

// Change of the intra-community weight over the movers' rows, one wave per
// mover (k_delta_intra).
__global__ void __launch_bounds__(TPB)
    k_mg_intra(const MergedGraph* __restrict__ G, const int32_t* __restrict__ state) {
  const int j = blockIdx.y;
  if (state[j] != 0) return;
  const MergedGraph g = G[j];
  const int64_t cnt = g.stat[ST_MOVES];
  const int64_t nwaves = int64_t(gridDim.x) * NW;
  const int lane = lane_id();
  long long s = 0;
  for (int64_t p = int64_t(blockIdx.x) * NW + threadIdx.x / WAVE; p < cnt; p += nwaves) {
    const int u = g.movers[p];
    const int cu = g.C[u], nu = g.Cn[u];
    for (int32_t q = g.off[u] + lane; q < g.off[u + 1]; q += WAVE) {
      const int2 e = g.adj[q];
      if (e.x == u) continue;
      const int cy = g.C[e.x], ny = g.Cn[e.x];
      const int d = int(nu == ny) - int(cu == cy);
      if (d) s += (long long)e.y * d * (cy != ny ? 1 : 2);
    }
  }
  block_add(s, &g.stat[ST_DI]);
}

// Change of sum a^2 over the touched labels (k_delta_squares).
__global__ void __launch_bounds__(TPB)
    k_mg_squares(const MergedGraph* __restrict__ G, const int32_t* __restrict__ state) {
  const int j = blockIdx.y;
  if (state[j] != 0) return;
  const MergedGraph g = G[j];
  const int64_t cnt = g.stat[ST_TOUCHED];
  long long s = 0;
  for (int64_t p = int64_t(blockIdx.x) * TPB + threadIdx.x; p < cnt;
       p += int64_t(gridDim.x) * TPB) {
    const int X = g.tlist[p];
    const long long ao = g.a[X];
    const long long an = ao + unpack_lo(g.dpack[X]);
    s += an * an - ao * ao;
  }
  block_add(s, &g.stat[ST_DS]);
}

// Exact Delta N, keep or revert, the sweep's record, and the stop decision
// of the level (no move, a reverted sweep, a gain of at most T, or the
// sweep limit), per running graph.
__global__ void k_mg_finalize(const MergedGraph* __restrict__ G, int m, int32_t* state,
                              int32_t* sweeps) {
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    if (state[j] != 0) continue;
    const MergedGraph& g = G[j];
    long long* st = g.stat;
    const long long moves = st[ST_MOVES];
    const long long dN = g.two_m * st[ST_DI] - st[ST_DS];
    const int keep = (moves > 0 && dN >= 0) ? 1 : 0;
    st[ST_DN] = dN;
    st[ST_KEEP] = keep;
    const int s = sweeps[j];
    g.rec[3 * s + 0] = moves;
    g.rec[3 * s + 1] = dN;
    g.rec[3 * s + 2] = keep;
    sweeps[j] = s + 1;
    const bool stop = moves == 0 || dN < 0 || dN <= g.T || s + 1 >= g.max_sweeps;
    if (stop) state[j] = 1;
  }
}

// Commit or revert the movers and the touched labels' totals (k_commit), for
// every graph that swept in this round.
__global__ void __launch_bounds__(TPB)
    k_mg_commit(const MergedGraph* __restrict__ G, const int32_t* __restrict__ state) {
  const int j = blockIdx.y;
  if (state[j] == 2) return;
  const MergedGraph g = G[j];
  const long long* st = g.stat;
  const int64_t nm = st[ST_MOVES], nt = st[ST_TOUCHED];
  const bool keep = st[ST_KEEP] != 0;
  const int64_t stride = int64_t(gridDim.x) * TPB;
  for (int64_t p = int64_t(blockIdx.x) * TPB + threadIdx.x; p < nm; p += stride) {
    const int u = g.movers[p];
    if (keep)
      g.C[u] = g.Cn[u];
    else
      g.Cn[u] = g.C[u];
  }
  for (int64_t p = int64_t(blockIdx.x) * TPB + threadIdx.x; p < nt; p += stride) {
    const int X = g.tlist[p];
    const long long d = g.dpack[X];
    if (keep) {
      g.a[X] += unpack_lo(d);
      g.sz[X] += unpack_hi(d);
    }
    g.dpack[X] = 0;
    g.tflag[X] = 0;
  }
}

}  // namespace

void merged_reset(const MergedGraph* G, int m, int32_t* state, hipStream_t st) {
  k_mg_reset<<<1, 256, 0, st>>>(G, m, state);
  DC_LAUNCH_CHECK();
}

void merged_apply(const MergedGraph* G, int m, int64_t max_nact, int32_t* state,
                  int32_t* sweeps, hipStream_t st) {
  // grid x: enough blocks for the largest active list (capped); blocks of a
  // graph with a shorter list, or of a stopped graph, exit at once
  int64_t gx = ceil_div(max_nact > 0 ? max_nact : 1, TPB);
  if (gx > 512) gx = 512;
  const dim3 grid{unsigned(gx), unsigned(m), 1u};
  k_mg_apply<<<grid, TPB, 0, st>>>(G, state);
  DC_LAUNCH_CHECK();
  const dim3 grid2{unsigned(gx < 256 ? gx : 256), unsigned(m), 1u};
  k_mg_intra<<<grid2, TPB, 0, st>>>(G, state);
  DC_LAUNCH_CHECK();
  k_mg_squares<<<grid2, TPB, 0, st>>>(G, state);
  DC_LAUNCH_CHECK();
  k_mg_finalize<<<1, 256, 0, st>>>(G, m, state, sweeps);
  DC_LAUNCH_CHECK();
  k_mg_commit<<<grid2, TPB, 0, st>>>(G, state);
  DC_LAUNCH_CHECK();
}

}  // namespace dc
