// slm.hip -- the pieces of the smart local moving levels (dSLM: the paper's
// second host method for Delta-screening, Sec. 3.4; the level structure of
// its reference [waltman2013smart]) that Louvain's levels do not have:
//   * the subgraph every community induces (refinement runs local moving on
//     it from singletons, with the whole level graph's vertex weights);
//   * the next level's start partition: each coarse vertex (a refined
//     community) joins its parent community, labelled by the smallest coarse
//     id among the parent's refined communities;
//   * community totals and sizes of a given partition.
// The sweeps, compaction and final labels are the Louvain kernels.
#include "dc_louvain.h"

namespace dc {

namespace {

constexpr int TPB = 256;
constexpr int NW = TPB / WAVE;

inline int grid_for(int64_t n, int64_t cap = 16384) {
  int64_t g = ceil_div(n, TPB);
  if (g > cap) g = cap;
  return int(g < 1 ? 1 : g);
}

inline int wave_grid(int64_t rows, int64_t cap = 16384) {
  int64_t g = ceil_div(rows, NW);
  if (g > cap) g = cap;
  return int(g < 1 ? 1 : g);
}

// cnt[u] = entries (u, v) of u's row with C[v] == C[u] (diagonal included):
// one wave per row.
__global__ void __launch_bounds__(TPB)
    k_intra_counts(const int32_t* __restrict__ off, const int2* __restrict__ adj,
                   const int32_t* __restrict__ C, int32_t n, int32_t* __restrict__ cnt) {
  const int lane = lane_id();
  const int64_t nwaves = int64_t(gridDim.x) * NW;
  for (int64_t u = int64_t(blockIdx.x) * NW + threadIdx.x / WAVE; u < n; u += nwaves) {
    const int32_t rb = off[u], re = off[u + 1];
    const int cu = C[u];
    int c = 0;
    for (int32_t q = rb + lane; q < re; q += WAVE) c += C[adj[q].x] == cu ? 1 : 0;
    c = wave_sum(c);
    if (lane == 0) cnt[u] = c;
  }
}

// The kept entries of each row, in row order, at the row's new offset.
__global__ void __launch_bounds__(TPB)
    k_intra_fill(const int32_t* __restrict__ off, const int2* __restrict__ adj,
                 const int32_t* __restrict__ C, int32_t n, const int32_t* __restrict__ off_s,
                 int2* __restrict__ adj_s) {
  const int lane = lane_id();
  const uint64_t lt = (uint64_t(1) << lane) - 1;
  const int64_t nwaves = int64_t(gridDim.x) * NW;
  for (int64_t u = int64_t(blockIdx.x) * NW + threadIdx.x / WAVE; u < n; u += nwaves) {
    const int32_t rb = off[u], re = off[u + 1];
    const int cu = C[u];
    int32_t pos = off_s[u];
    for (int32_t q0 = rb; q0 < re; q0 += WAVE) {
      const int32_t q = q0 + lane;
      const int2 e = q < re ? adj[q] : make_int2(0, 0);
      const bool keep = q < re && C[e.x] == cu;
      const uint64_t m = __ballot(keep);
      if (keep) adj_s[pos + __popcll(m & lt)] = e;
      pos += __popcll(m);
    }
  }
}

// first[P[u]] = min over u of rank[R[u]] (first: filled with INT32_MAX).
__global__ void k_parent_first(const int32_t* __restrict__ P, const int32_t* __restrict__ R,
                               const int32_t* __restrict__ rank, int32_t n,
                               int32_t* __restrict__ first) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t u = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; u < n; u += stride)
    atomicMin(&first[P[u]], rank[R[u]]);
}

// Cnext[rank[R[u]]] = first[P[u]]: every member of a refined community
// writes the same value.
__global__ void k_parent_start(const int32_t* __restrict__ P, const int32_t* __restrict__ R,
                               const int32_t* __restrict__ rank,
                               const int32_t* __restrict__ first, int32_t n,
                               int32_t* __restrict__ Cnext) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t u = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; u < n; u += stride)
    Cnext[rank[R[u]]] = first[P[u]];
}

// a[C[x]] += k[x], sz[C[x]] += 1 (a, sz zeroed), pre-combined per block.
__global__ void __launch_bounds__(TPB)
    k_totals_sizes(const int32_t* __restrict__ k, const int32_t* __restrict__ C, int32_t n,
                   int32_t* __restrict__ a, int32_t* __restrict__ sz) {
  __shared__ AggLds agg;
  agg_init(agg);
  __syncthreads();
  const int64_t stride = int64_t(gridDim.x) * TPB;
  for (int64_t x = int64_t(blockIdx.x) * TPB + threadIdx.x; x < n; x += stride) {
    // size in the high half, total in the low half of one 64-bit sum
    const long long v = (1ll << 32) + (long long)k[x];
    if (!agg_try(agg, C[x], v)) {
      atomicAdd(&a[C[x]], k[x]);
      atomicAdd(&sz[C[x]], 1);
    }
  }
  __syncthreads();
  for (int s = threadIdx.x; s < AGG_SLOTS; s += TPB) {
    const int X = agg.keys[s];
    if (X == EMPTY_KEY) continue;
    const long long v = agg.vals[s];
    atomicAdd(&a[X], int(v & 0xffffffffll));
    atomicAdd(&sz[X], int(v >> 32));
  }
}

// *count += number of x < n with sz[x] > 0.
__global__ void __launch_bounds__(TPB)
    k_nonempty_count(const int32_t* __restrict__ sz, int32_t n, long long* count) {
  long long c = 0;
  const int64_t stride = int64_t(gridDim.x) * TPB;
  for (int64_t x = int64_t(blockIdx.x) * TPB + threadIdx.x; x < n; x += stride)
    c += sz[x] > 0 ? 1 : 0;
  block_add(c, count);
}

}  // namespace

int64_t induced_subgraph(const LevelView& g, const int32_t* C, int32_t* cnt, int32_t* off_s,
                         DBuf& adj_s, void* host, hipStream_t st) {
  const int32_t n = g.n;
  k_intra_counts<<<wave_grid(n), TPB, 0, st>>>(g.off, g.adj, C, n, cnt);
  DC_LAUNCH_CHECK();
  scan_excl_i32(cnt, off_s, n, off_s + n, st);
  DC_HIP(hipMemcpyAsync(host, off_s + n, 4, hipMemcpyDeviceToHost, st));
  DC_HIP(hipStreamSynchronize(st));
  const int64_t nnz = *static_cast<int32_t*>(host);
  adj_s.ensure(size_t(nnz + 1) * 8);
  k_intra_fill<<<wave_grid(n), TPB, 0, st>>>(g.off, g.adj, C, n, off_s, adj_s.as<int2>());
  DC_LAUNCH_CHECK();
  return nnz;
}

void parent_start(const int32_t* P, const int32_t* R, const int32_t* rank, int32_t n,
                  int32_t* first, int32_t* Cnext, hipStream_t st) {
  if (n <= 0) return;
  fill_i32(first, 0x7fffffff, n, st);
  k_parent_first<<<grid_for(n), TPB, 0, st>>>(P, R, rank, n, first);
  DC_LAUNCH_CHECK();
  k_parent_start<<<grid_for(n), TPB, 0, st>>>(P, R, rank, first, n, Cnext);
  DC_LAUNCH_CHECK();
}

void totals_sizes(const int32_t* k, const int32_t* C, int32_t n, int32_t* a, int32_t* sz,
                  hipStream_t st) {
  if (n <= 0) return;
  fill_i32(a, 0, n, st);
  fill_i32(sz, 0, n, st);
  k_totals_sizes<<<grid_for(n, 2048), TPB, 0, st>>>(k, C, n, a, sz);
  DC_LAUNCH_CHECK();
}

void nonempty_count(const int32_t* sz, int32_t n, long long* count, hipStream_t st) {
  if (n <= 0) return;
  k_nonempty_count<<<grid_for(n, 1024), TPB, 0, st>>>(sz, n, count);
  DC_LAUNCH_CHECK();
}

}  // namespace dc
