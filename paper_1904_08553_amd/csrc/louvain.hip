// louvain.hip -- bookkeeping of a synchronous sweep (Alg. 1 inner loop):
// collect the movers, apply their moves to the community totals a and sizes,
// compute the exact change of N = 2m*I - sum a^2, and keep or revert the
// sweep.  The evaluation kernels live in eval.hip.
#include "dc_louvain.h"

namespace dc {

namespace {

constexpr int TPB = 256;
constexpr int NW = TPB / WAVE;

// Moves of a sweep: community totals and sizes change by (-k, -1) on the old
// label and (+k, +1) on the new one; packed as size*2^32 + total so one
// 64-bit atomic carries both, pre-combined per block.  Movers (next label
// differs) are compacted from the active list, one atomic per block.
__device__ __forceinline__ long long pack2(int da, int dsz) {
  return (long long)dsz * 4294967296LL + (long long)da;
}

// dpack[X] += v and, on the label's first change of the sweep, X joins the
// touched-label list.
__device__ __forceinline__ void touch_label(int X, long long v, long long* dpack, int32_t* tflag,
                                            int32_t* tlist, long long* stat) {
  atomicAdd((unsigned long long*)&dpack[X], (unsigned long long)v);
  if (atomicExch(&tflag[X], 1) == 0) {
    const unsigned long long q = atomicAdd((unsigned long long*)&stat[ST_TOUCHED], 1ull);
    tlist[q] = X;
  }
}

// Block b takes AM_ROUNDS tiles of the active list; all its entries and
// their labels are loaded first, the block reserves its movers' places in
// the mover list with one atomic (a counter that every tile added to
// serialised thousands of same-address atomics when the movers were few and
// spread out), then lists them and applies their label changes.
constexpr int AM_ROUNDS = 8;
__global__ void __launch_bounds__(TPB)
    k_apply_moves(const int32_t* __restrict__ list, int64_t cnt,
                  const int32_t* __restrict__ C, const int32_t* __restrict__ Cn,
                  const int32_t* __restrict__ k, long long* dpack, int32_t* tflag,
                  int32_t* tlist, int32_t* movers, long long* stat) {
  __shared__ AggLds agg;
  __shared__ int wc[AM_ROUNDS][NW];
  __shared__ long long bbase;
  __shared__ int btotal;
  const int wid = threadIdx.x / WAVE, lane = lane_id();
  const uint64_t lt = (uint64_t(1) << lane) - 1;
  const int64_t v0 = int64_t(blockIdx.x) * (AM_ROUNDS * TPB) + threadIdx.x;
  int u[AM_ROUNDS], from[AM_ROUNDS], to[AM_ROUNDS];
  uint64_t fm[AM_ROUNDS];
#pragma unroll
  for (int r = 0; r < AM_ROUNDS; ++r) {
    const int64_t p = v0 + int64_t(r) * TPB;
    u[r] = p < cnt ? (list ? list[p] : int(p)) : -1;
  }
#pragma unroll
  for (int r = 0; r < AM_ROUNDS; ++r) {
    from[r] = u[r] >= 0 ? C[u[r]] : 0;
    to[r] = u[r] >= 0 ? Cn[u[r]] : 0;
  }
#pragma unroll
  for (int r = 0; r < AM_ROUNDS; ++r) {
    fm[r] = __ballot(from[r] != to[r]);
    if (lane == 0) wc[r][wid] = __popcll(fm[r]);
  }
  // the block's label changes are summed in LDS, so a large community gets
  // one update per block (see agg_try)
  agg_init(agg);
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int r = 0; r < AM_ROUNDS; ++r)
      for (int w = 0; w < NW; ++w) tot += wc[r][w];
    btotal = tot;
    bbase = tot ? (long long)atomicAdd((unsigned long long*)&stat[ST_MOVES],
                                       (unsigned long long)tot)
                : 0;
  }
  __syncthreads();
  if (btotal == 0) return;  // uniform: nothing moved in this block's tiles
  long long run = bbase;
#pragma unroll
  for (int r = 0; r < AM_ROUNDS; ++r) {
    if (from[r] != to[r]) {
      long long pos = run + __popcll(fm[r] & lt);
      for (int w = 0; w < wid; ++w) pos += wc[r][w];
      movers[pos] = u[r];
      const int ku = k[u[r]];
      if (!agg_try(agg, from[r], pack2(-ku, -1)))
        touch_label(from[r], pack2(-ku, -1), dpack, tflag, tlist, stat);
      if (!agg_try(agg, to[r], pack2(ku, 1)))
        touch_label(to[r], pack2(ku, 1), dpack, tflag, tlist, stat);
    }
    for (int w = 0; w < NW; ++w) run += wc[r][w];
  }
  // every label left in the table gets one global update; the labels that
  // this sweep touches first are appended to tlist with one counter update
  // for the block
  constexpr int FR = AGG_SLOTS / TPB;
  __shared__ int fcount[FR][NW];
  __shared__ long long fbase;
  __syncthreads();
  int fx[FR];
  uint64_t gm[FR];
#pragma unroll
  for (int r = 0; r < FR; ++r) {
    const int X = agg.keys[r * TPB + threadIdx.x];
    bool first = false;
    if (X != EMPTY_KEY) {
      const long long v = agg.vals[r * TPB + threadIdx.x];
      if (v != 0) {
        atomicAdd((unsigned long long*)&dpack[X], (unsigned long long)v);
        first = atomicExch(&tflag[X], 1) == 0;
      }
    }
    fx[r] = first ? X : -1;
    gm[r] = __ballot(first);
    if (lane == 0) fcount[r][wid] = __popcll(gm[r]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int r = 0; r < FR; ++r)
      for (int w = 0; w < NW; ++w) tot += fcount[r][w];
    fbase = tot ? (long long)atomicAdd((unsigned long long*)&stat[ST_TOUCHED],
                                       (unsigned long long)tot)
                : 0;
  }
  __syncthreads();
  long long pos = fbase;
#pragma unroll
  for (int r = 0; r < FR; ++r) {
    if (fx[r] >= 0) {
      long long q = pos + __popcll(gm[r] & lt);
      for (int w = 0; w < wid; ++w) q += fcount[r][w];
      tlist[q] = fx[r];
    }
    for (int w = 0; w < NW; ++w) pos += fcount[r][w];
  }
}


__device__ __forceinline__ int unpack_lo(long long d) { return int(uint32_t(uint64_t(d))); }
__device__ __forceinline__ int unpack_hi(long long d) {
  return int((d - (long long)unpack_lo(d)) >> 32);
}

// The two terms of the exact Delta N in one launch: blocks [0, nb_intra)
// sum the change of the intra-community weight over the movers' rows (GS
// lanes per mover: 16 on graphs of short rows, a wave otherwise), the other
// blocks the change of sum a^2 over the touched labels.
template <int GS>
__global__ void __launch_bounds__(TPB)
    k_delta_terms(const int32_t* __restrict__ movers, const int32_t* __restrict__ tlist,
                  const int32_t* __restrict__ off, const int2* __restrict__ adj,
                  const int32_t* __restrict__ C, const int32_t* __restrict__ Cn,
                  const long long* __restrict__ dpack, const int32_t* __restrict__ a,
                  int nb_intra, long long* stat) {
  long long s = 0;
  if (int(blockIdx.x) < nb_intra) {
    const int64_t cnt = stat[ST_MOVES];
    const int lane = lane_id(), gl = lane % GS;
    const int64_t nwaves = int64_t(nb_intra) * NW;
    // a wave takes WAVE / GS movers per round; a row longer than a wave is
    // left to the whole wave afterwards, so hubs keep wave speed
    for (int64_t wb = (int64_t(blockIdx.x) * NW + threadIdx.x / WAVE) * (WAVE / GS);
         wb < cnt; wb += nwaves * (WAVE / GS)) {
      const int64_t p = wb + lane / GS;
      const bool have = p < cnt;
      const int u = have ? movers[p] : 0;
      const int32_t rb = have ? off[u] : 0, re = have ? off[u + 1] : 0;
      const int cu = have ? C[u] : 0, nu = have ? Cn[u] : 0;
      const bool wide = GS < WAVE && re - rb > WAVE;
      if (!wide) {
        for (int32_t j = rb + gl; j < re; j += GS) {
          const int2 e = adj[j];
          if (e.x == u) continue;
          const int cy = C[e.x], ny = Cn[e.x];
          const int d = int(nu == ny) - int(cu == cy);
          if (d) s += (long long)e.y * d * (cy != ny ? 1 : 2);
        }
      }
      for (uint64_t wm = __ballot(wide && gl == 0); wm; wm &= wm - 1) {
        const int l = __ffsll((unsigned long long)wm) - 1;
        const int wu = __builtin_amdgcn_readlane(u, l);
        const int wcu = __builtin_amdgcn_readlane(cu, l), wnu = __builtin_amdgcn_readlane(nu, l);
        const int32_t wre = __builtin_amdgcn_readlane(re, l);
        for (int32_t j = __builtin_amdgcn_readlane(rb, l) + lane; j < wre; j += WAVE) {
          const int2 e = adj[j];
          if (e.x == wu) continue;
          const int cy = C[e.x], ny = Cn[e.x];
          const int d = int(wnu == ny) - int(wcu == cy);
          if (d) s += (long long)e.y * d * (cy != ny ? 1 : 2);
        }
      }
    }
    block_add(s, &stat[ST_DI]);
  } else {
    const int64_t cnt = stat[ST_TOUCHED];
    const int64_t nbs = int64_t(gridDim.x) - nb_intra;
    for (int64_t p = (int64_t(blockIdx.x) - nb_intra) * TPB + threadIdx.x; p < cnt;
         p += nbs * TPB) {
      const int X = tlist[p];
      const long long ao = a[X];
      const long long an = ao + unpack_lo(dpack[X]);
      s += an * an - ao * ao;
    }
    block_add(s, &stat[ST_DS]);
  }
}

// Keep (Delta N >= 0 and something moved) or revert the sweep: movers take
// or drop their next labels, the touched labels' totals and sizes take
// their changes, and the change buffers are cleared.  The last block to
// finish writes the sweep's status block (Delta N and the decision
// included) to host memory and clears the per-sweep counters, so the next
// sweep needs no reset launch and the host no copy.
__global__ void __launch_bounds__(TPB)
    k_commit(const int32_t* __restrict__ movers, const int32_t* __restrict__ tlist,
             long long* stat, long long two_m, int32_t* C, int32_t* Cn, long long* dpack,
             int32_t* tflag, int32_t* a, int32_t* sz, unsigned* done, long long* host_stat) {
  const int64_t nm = stat[ST_MOVES], nt = stat[ST_TOUCHED];
  const long long dN = two_m * stat[ST_DI] - stat[ST_DS];
  const bool keep = nm > 0 && dN >= 0;
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
  if (!last_block(done)) return;
  for (int i = threadIdx.x; i < ST_COUNT; i += blockDim.x)
    host_store(&host_stat[i], i == ST_DN ? dN : i == ST_KEEP ? (keep ? 1ll : 0ll) : stat[i]);
  __syncthreads();  // every slot is read before the counters are cleared
  if (threadIdx.x == 0) {
    stat[ST_MOVES] = 0;
    stat[ST_TOUCHED] = 0;
    stat[ST_DI] = 0;
    stat[ST_DS] = 0;
    stat[ST_DN] = dN;
    stat[ST_KEEP] = keep ? 1 : 0;
  }
}

__global__ void k_reset_sweep(long long* stat) {
  int t = threadIdx.x;
  if (t == ST_MOVES || t == ST_TOUCHED || t == ST_DI || t == ST_DS || t == ST_DN ||
      t == ST_KEEP)
    stat[t] = 0;
}

inline int grid_for(int64_t n, int cap = 4096) {
  int64_t g = ceil_div(n, TPB);
  if (g > cap) g = cap;
  return int(g < 1 ? 1 : g);
}

}  // namespace

void sweep_reset(long long* stat, hipStream_t st) {
  k_reset_sweep<<<1, 64, 0, st>>>(stat);
  DC_LAUNCH_CHECK();
}

void sweep_apply(const LevelView& g, const int32_t* active, int64_t n_active, int32_t* C,
                 int32_t* Cn, int32_t* a, int32_t* sz, long long two_m, int32_t* movers,
                 long long* dpack, int32_t* tflag, int32_t* tlist, long long* stat,
                 unsigned* done, long long* host_stat, hipStream_t st) {
  const int64_t cnt = n_active > 0 ? n_active : 1;
  k_apply_moves<<<int(ceil_div(cnt, AM_ROUNDS * TPB)), TPB, 0, st>>>(
      active, n_active, C, Cn, g.k, dpack, tflag, tlist, movers, stat);
  DC_LAUNCH_CHECK();
  // grids sized for the active list (the movers are known on the device
  // only); the loops stride, so most sweeps' few movers leave blocks idle
  const int nb_sq = grid_for(2 * cnt, 256);
  if (g.nnz <= 16 * int64_t(g.n)) {  // short rows: four movers per wave
    const int nb_intra = grid_for(ceil_div(cnt, 4) * WAVE, 4096);
    k_delta_terms<16><<<nb_intra + nb_sq, TPB, 0, st>>>(movers, tlist, g.off, g.adj, C, Cn,
                                                        dpack, a, nb_intra, stat);
  } else {
    const int nb_intra = grid_for(cnt * WAVE, 4096);
    k_delta_terms<WAVE><<<nb_intra + nb_sq, TPB, 0, st>>>(movers, tlist, g.off, g.adj, C, Cn,
                                                          dpack, a, nb_intra, stat);
  }
  DC_LAUNCH_CHECK();
  k_commit<<<grid_for(2 * cnt, 512), TPB, 0, st>>>(movers, tlist, stat, two_m, C, Cn, dpack,
                                                   tflag, a, sz, done, host_stat);
  DC_LAUNCH_CHECK();
}

}  // namespace dc
