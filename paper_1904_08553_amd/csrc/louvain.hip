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

__global__ void __launch_bounds__(TPB)
    k_apply_moves(const int32_t* __restrict__ list, int64_t cnt,
                  const int32_t* __restrict__ C, const int32_t* __restrict__ Cn,
                  const int32_t* __restrict__ k, long long* dpack, int32_t* tflag,
                  int32_t* tlist, int32_t* movers, long long* stat) {
  __shared__ AggLds agg;
  __shared__ int wcount[NW];
  __shared__ int btotal;
  __shared__ long long bbase;
  const int wid = threadIdx.x / WAVE, lane = lane_id();
  const uint64_t lt = (uint64_t(1) << lane) - 1;
  const int64_t stride = int64_t(gridDim.x) * TPB;
  // the block's label changes are summed in LDS over all its tiles, so a
  // large community gets one update per block (see agg_try)
  agg_init(agg);
  for (int64_t base = int64_t(blockIdx.x) * TPB; base < cnt; base += stride) {
    const int64_t p = base + threadIdx.x;
    int u = 0;
    bool mover = false;
    if (p < cnt) {
      u = list ? list[p] : int(p);
      mover = Cn[u] != C[u];
    }
    const uint64_t m = __ballot(mover);
    if (lane == 0) wcount[wid] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int w = 0; w < NW; ++w) tot += wcount[w];
      btotal = tot;
      bbase = tot ? (long long)atomicAdd((unsigned long long*)&stat[ST_MOVES],
                                         (unsigned long long)tot)
                  : 0;
    }
    __syncthreads();
    if (btotal == 0) continue;  // uniform: nothing moved in this tile
    if (mover) {
      long long pos = bbase + __popcll(m & lt);
      for (int w = 0; w < wid; ++w) pos += wcount[w];
      movers[pos] = u;
      const int ku = k[u];
      const int from = C[u], to = Cn[u];
      if (!agg_try(agg, from, pack2(-ku, -1))) touch_label(from, pack2(-ku, -1), dpack, tflag, tlist, stat);
      if (!agg_try(agg, to, pack2(ku, 1))) touch_label(to, pack2(ku, 1), dpack, tflag, tlist, stat);
    }
    __syncthreads();  // wcount and btotal are rewritten by the next tile
  }
  __syncthreads();
  for (int s = threadIdx.x; s < AGG_SLOTS; s += TPB) {
    const int X = agg.keys[s];
    if (X == EMPTY_KEY) continue;
    const long long v = agg.vals[s];
    if (v != 0) touch_label(X, v, dpack, tflag, tlist, stat);
  }
}

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
  block_add(s, &stat_w[ST_DI]);
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
  block_add(s, &stat[ST_DS]);
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
                 hipStream_t st) {
  const int64_t cnt = n_active > 0 ? n_active : 1;
  k_apply_moves<<<grid_for(cnt, 512), TPB, 0, st>>>(active, n_active, C, Cn, g.k, dpack, tflag,
                                                     tlist, movers, stat);
  DC_LAUNCH_CHECK();
  k_delta_intra<<<grid_for(cnt * WAVE, 4096), TPB, 0, st>>>(movers, stat, g.off, g.adj, C, Cn,
                                                            stat);
  DC_LAUNCH_CHECK();
  k_delta_squares<<<grid_for(2 * cnt, 2048), TPB, 0, st>>>(tlist, stat, dpack, a);
  DC_LAUNCH_CHECK();
  k_finalize<<<1, 1, 0, st>>>(stat, two_m);
  DC_LAUNCH_CHECK();
  k_commit<<<grid_for(2 * cnt, 2048), TPB, 0, st>>>(movers, tlist, stat, C, Cn, dpack, tflag, a,
                                                    sz);
  DC_LAUNCH_CHECK();
}

}  // namespace dc
