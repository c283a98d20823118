// screen.hip -- list plumbing of Delta-screening (Alg. 2, Sec. 3.5): the
// sorted directed insertions and their sources, the sources of
// intra-community deletions, and R_t = (marked vertices) union (members of
// flagged communities C_{t-1}(j*)), compacted in ascending vertex order.
#include "dc_louvain.h"

namespace dc {

namespace {

constexpr int TPB = 256;

inline int grid_for(int64_t n, int64_t cap = 16384) {
  int64_t g = ceil_div(n, TPB);
  if (g > cap) g = cap;
  return int(g < 1 ? 1 : g);
}

#define GRID_STRIDE(i, n)                                              \
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;     \
       i < (n); i += int64_t(gridDim.x) * blockDim.x)

__global__ void k_compact_index(const int32_t* __restrict__ flag,
                                const int32_t* __restrict__ pos, int64_t n,
                                int32_t* out) {
  GRID_STRIDE(i, n) {
    if (flag[i]) out[pos[i]] = int32_t(i);
  }
}

__global__ void k_select_insertions(const int32_t* __restrict__ op, int64_t n,
                                    int32_t* flag) {
  GRID_STRIDE(i, n) { flag[i] = op[i] != OP_DELETE ? 1 : 0; }
}

__global__ void k_gather_u64(const uint64_t* __restrict__ in,
                             const int32_t* __restrict__ flag,
                             const int32_t* __restrict__ pos, int64_t n,
                             uint64_t* out) {
  GRID_STRIDE(i, n) {
    if (flag[i]) out[pos[i]] = in[i];
  }
}

__global__ void k_source_heads(const uint64_t* __restrict__ keys, int64_t m,
                               int32_t n, int32_t* flag) {
  GRID_STRIDE(i, m) {
    flag[i] = (i == 0 || keys[i] / uint64_t(n) != keys[i - 1] / uint64_t(n)) ? 1 : 0;
  }
}

__global__ void k_gather_sources(const uint64_t* __restrict__ keys,
                                 const int32_t* __restrict__ flag,
                                 const int32_t* __restrict__ pos, int64_t m,
                                 int32_t n, int32_t* out) {
  GRID_STRIDE(i, m) {
    if (flag[i]) out[pos[i]] = int32_t(keys[i] / uint64_t(n));
  }
}

__global__ void k_source_segments(const uint64_t* __restrict__ keys, int64_t m, int32_t n,
                                  int32_t* seg_beg, int32_t* seg_end) {
  GRID_STRIDE(i, m) {
    const uint64_t src = keys[i] / uint64_t(n);
    if (i == 0 || keys[i - 1] / uint64_t(n) != src) seg_beg[src] = int32_t(i);
    if (i == m - 1 || keys[i + 1] / uint64_t(n) != src) seg_end[src] = int32_t(i + 1);
  }
}

__global__ void k_deletion_sources(const uint64_t* __restrict__ key,
                                   const int32_t* __restrict__ op, int64_t nch,
                                   int32_t n, const int32_t* __restrict__ C,
                                   int32_t* dflag) {
  GRID_STRIDE(i, nch) {
    int32_t o = op[i];
    if (o != OP_DELETE && o != OP_REPLACE) continue;
    int32_t s = int32_t(key[i] / uint64_t(n)), d = int32_t(key[i] % uint64_t(n));
    if (C[s] == C[d]) dflag[s] = 1;
  }
}

// one wave per listed vertex
__global__ void k_mark_neighbourhoods(const int32_t* __restrict__ list,
                                      int64_t cnt, const int32_t* __restrict__ off,
                                      const int2* __restrict__ adj, uint8_t* R) {
  const int64_t nwaves = int64_t(gridDim.x) * (TPB / WAVE);
  for (int64_t p = int64_t(blockIdx.x) * (TPB / WAVE) + threadIdx.x / WAVE; p < cnt;
       p += nwaves) {
    int i = list[p];
    if (lane_id() == 0) R[i] = 1;
    for (int32_t j = off[i] + lane_id(); j < off[i + 1]; j += WAVE) R[adj[j].x] = 1;
  }
}

__global__ void k_materialize_R(uint8_t* R, const uint8_t* __restrict__ cflag,
                                const int32_t* __restrict__ C, int32_t n,
                                int32_t* rflag) {
  GRID_STRIDE(v, n) {
    uint8_t r = R[v] | cflag[C[v]];
    R[v] = r;
    rflag[v] = r;
  }
}

}  // namespace

void compact_index(const int32_t* flag, const int32_t* pos, int64_t n, int32_t* out,
                   hipStream_t st) {
  if (n <= 0) return;
  k_compact_index<<<grid_for(n), TPB, 0, st>>>(flag, pos, n, out);
  DC_LAUNCH_CHECK();
}

void select_insertions(const int32_t* ch_op, int64_t nch, int32_t* flag, hipStream_t st) {
  if (nch <= 0) return;
  k_select_insertions<<<grid_for(nch), TPB, 0, st>>>(ch_op, nch, flag);
  DC_LAUNCH_CHECK();
}

void gather_u64(const uint64_t* in, const int32_t* flag, const int32_t* pos, int64_t n,
                uint64_t* out, hipStream_t st) {
  if (n <= 0) return;
  k_gather_u64<<<grid_for(n), TPB, 0, st>>>(in, flag, pos, n, out);
  DC_LAUNCH_CHECK();
}

void source_heads(const uint64_t* keys, int64_t m, int32_t n, int32_t* flag, hipStream_t st) {
  if (m <= 0) return;
  k_source_heads<<<grid_for(m), TPB, 0, st>>>(keys, m, n, flag);
  DC_LAUNCH_CHECK();
}

void gather_sources(const uint64_t* keys, const int32_t* flag, const int32_t* pos, int64_t m,
                    int32_t n, int32_t* out, hipStream_t st) {
  if (m <= 0) return;
  k_gather_sources<<<grid_for(m), TPB, 0, st>>>(keys, flag, pos, m, n, out);
  DC_LAUNCH_CHECK();
}

void source_segments(const uint64_t* keys, int64_t m, int32_t n, int32_t* seg_beg,
                     int32_t* seg_end, hipStream_t st) {
  if (m <= 0) return;
  k_source_segments<<<grid_for(m), TPB, 0, st>>>(keys, m, n, seg_beg, seg_end);
  DC_LAUNCH_CHECK();
}

void deletion_sources(const uint64_t* ch_key, const int32_t* ch_op, int64_t nch, int32_t n,
                      const int32_t* C, int32_t* dflag, hipStream_t st) {
  if (nch <= 0) return;
  k_deletion_sources<<<grid_for(nch), TPB, 0, st>>>(ch_key, ch_op, nch, n, C, dflag);
  DC_LAUNCH_CHECK();
}

void mark_neighbourhoods(const int32_t* list, int64_t cnt, const int32_t* off, const int2* adj,
                         uint8_t* R, hipStream_t st) {
  if (cnt <= 0) return;
  k_mark_neighbourhoods<<<grid_for(cnt * WAVE, 4096), TPB, 0, st>>>(list, cnt, off, adj, R);
  DC_LAUNCH_CHECK();
}

void materialize_R(uint8_t* R, const uint8_t* cflag, const int32_t* C, int32_t n,
                   int32_t* rflag, hipStream_t st) {
  if (n <= 0) return;
  k_materialize_R<<<grid_for(n), TPB, 0, st>>>(R, cflag, C, n, rflag);
  DC_LAUNCH_CHECK();
}

}  // namespace dc
