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

// The screening set of the fused pass straight from the sorted change list,
// one thread per change.  First pass: the change's kind goes into its
// source's word sbits (bit 0: an insertion record, op != OP_DELETE, so the
// source is an Alg. 2 source; bit 1: the deletion or replacement of a pair
// inside one community C_{t-1}), and an insertion record at either end of
// its source's run of insertion keys sets that end of the sink segment
// [seg_beg, seg_end).  Second pass: the head of each source's run of
// changes copies the word into uflag, marks itself in hflag when it is
// non-zero (the union list, ascending, is the heads' compaction) and
// counts the two kinds of sources (block b adds to counter b % SUM_SLOTS:
// with a single counter the blocks' atomics would serialise).
__global__ void k_screen_kinds(const uint64_t* __restrict__ key, const int32_t* __restrict__ op,
                               const int32_t* __restrict__ ins_pos,
                               const uint64_t* __restrict__ ins_keys, int64_t n_ins,
                               int64_t nch, int32_t n, const int32_t* __restrict__ C,
                               int32_t* sbits, int32_t* seg_beg, int32_t* seg_end) {
  GRID_STRIDE(q, nch) {
    const uint64_t kq = key[q];
    const int32_t s = int32_t(kq / uint64_t(n));
    const int32_t o = op[q];
    int b = 0;
    if (o != OP_DELETE) {
      b |= 1;
      const int64_t p = ins_pos[q];
      if (p == 0 || int32_t(ins_keys[p - 1] / uint64_t(n)) != s) seg_beg[s] = int32_t(p);
      if (p == n_ins - 1 || int32_t(ins_keys[p + 1] / uint64_t(n)) != s)
        seg_end[s] = int32_t(p + 1);
    }
    if ((o == OP_DELETE || o == OP_REPLACE) && C[int32_t(kq % uint64_t(n))] == C[s]) b |= 2;
    if (b) atomicOr(&sbits[s], b);
  }
}

__global__ void __launch_bounds__(TPB)
    k_screen_heads(const uint64_t* __restrict__ key, int64_t nch, int32_t n,
                   const int32_t* __restrict__ sbits, uint8_t* uflag, int32_t* hflag,
                   long long* n_src, long long* n_dsrc) {
  long long ns = 0, nd = 0;
  GRID_STRIDE(q, nch) {
    const int32_t s = int32_t(key[q] / uint64_t(n));
    int32_t head = 0;
    if (q == 0 || int32_t(key[q - 1] / uint64_t(n)) != s) {
      const int bits = sbits[s];
      if (bits) {
        uflag[s] = uint8_t(bits);
        head = 1;
        ns += bits & 1;
        nd += bits >> 1;
      }
    }
    hflag[q] = head;
  }
  block_add(ns, n_src + blockIdx.x % SUM_SLOTS);
  block_add(nd, n_dsrc + blockIdx.x % SUM_SLOTS);
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

// R[v] |= cflag[C[v]] (cflag may be null), and the vertices of R appended
// to list: a block
// takes RL_ROUNDS tiles of TPB vertices and reserves its places with one
// atomic on *count (ascending within the block, blocks in any order).
constexpr int RL_ROUNDS = 8;
__global__ void __launch_bounds__(TPB)
    k_materialize_R(uint8_t* R, const uint8_t* __restrict__ cflag,
                    const int32_t* __restrict__ C, int32_t n, int32_t* list, int32_t* count) {
  __shared__ int wc[RL_ROUNDS][TPB / WAVE];
  __shared__ int base;
  const int lane = lane_id(), wid = threadIdx.x / WAVE;
  const uint64_t lt = (uint64_t(1) << lane) - 1;
  const int64_t v0 = int64_t(blockIdx.x) * (RL_ROUNDS * TPB) + threadIdx.x;
  uint64_t fm[RL_ROUNDS];
  bool f[RL_ROUNDS];
  // the rounds' flags (and labels, then community flags) are loaded round
  // after round at clamped indexes (n >= 1), so each kind is in flight
  // together; lanes past n use none of it
  uint8_t x[RL_ROUNDS];
#pragma unroll
  for (int r = 0; r < RL_ROUNDS; ++r) {
    const int64_t v = v0 + int64_t(r) * TPB;
    x[r] = R[v < n ? v : n - 1];
  }
  if (cflag) {
    int32_t c[RL_ROUNDS];
#pragma unroll
    for (int r = 0; r < RL_ROUNDS; ++r) {
      const int64_t v = v0 + int64_t(r) * TPB;
      c[r] = C[v < n ? v : n - 1];
    }
#pragma unroll
    for (int r = 0; r < RL_ROUNDS; ++r) x[r] |= cflag[c[r]];
#pragma unroll
    for (int r = 0; r < RL_ROUNDS; ++r) {
      const int64_t v = v0 + int64_t(r) * TPB;
      if (v < n) R[v] = x[r];
    }
  }
#pragma unroll
  for (int r = 0; r < RL_ROUNDS; ++r) {
    const int64_t v = v0 + int64_t(r) * TPB;
    f[r] = v < n && x[r] != 0;
    fm[r] = __ballot(f[r]);
    if (lane == 0) wc[r][wid] = __popcll(fm[r]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int r = 0; r < RL_ROUNDS; ++r)
      for (int w = 0; w < TPB / WAVE; ++w) tot += wc[r][w];
    base = tot ? atomicAdd(count, tot) : 0;
  }
  __syncthreads();
  int pos = base;
#pragma unroll
  for (int r = 0; r < RL_ROUNDS; ++r) {
    if (f[r]) {
      int q = pos + __popcll(fm[r] & lt);
      for (int w = 0; w < wid; ++w) q += wc[r][w];
      list[q] = int32_t(v0 + int64_t(r) * TPB);
    }
    for (int w = 0; w < TPB / WAVE; ++w) pos += wc[r][w];
  }
}

__global__ void k_apply_pre(const int32_t* __restrict__ list, int64_t cnt,
                            const uint8_t* __restrict__ R, const int32_t* __restrict__ pre,
                            int32_t* __restrict__ Cn) {
  GRID_STRIDE(p, cnt) {
    const int32_t v = list[p];
    if (R[v]) Cn[v] = pre[v];
  }
}

}  // namespace

// Cascade-aware screening (an extension for the indirect effect noted after
// the proof of Lemma 3.2).  One wave per source of the list: the neighbours
// of an accepted source in its own community C_{t-1}(i) become candidates.
__global__ void __launch_bounds__(TPB)
    k_cascade_candidates(const int32_t* __restrict__ list, int64_t cnt,
                         const uint8_t* __restrict__ accflag, const int32_t* __restrict__ off,
                         const int2* __restrict__ adj, const int32_t* __restrict__ C,
                         uint8_t* cand) {
  const int64_t nwaves = int64_t(gridDim.x) * (TPB / WAVE);
  const int lane = lane_id();
  for (int64_t p = (int64_t(blockIdx.x) * TPB + threadIdx.x) / WAVE; p < cnt; p += nwaves) {
    const int i = list[p];
    if (!accflag[i]) continue;  // uniform: one source per wave
    const int ci = C[i];
    for (int32_t q = off[i] + lane; q < off[i + 1]; q += WAVE) {
      const int v = adj[q].x;
      if (v != i && C[v] == ci) cand[v] = 1;
    }
  }
}

// One wave per candidate v: with G1(v) the scaled gain of v's best move to
// another neighbouring community (f_g1, NO_GAIN when there is none), v and
// its neighbours join R when G1(v) * den >= -num * 2m * k_v, compared in
// 128-bit integers.
__global__ void __launch_bounds__(TPB)
    k_cascade_mark(const int32_t* __restrict__ list, int64_t cnt,
                   const long long* __restrict__ f_g1, const int32_t* __restrict__ k,
                   long long two_m, long long num, long long den,
                   const int32_t* __restrict__ off, const int2* __restrict__ adj, uint8_t* R,
                   long long* expanded) {
  const int64_t nwaves = int64_t(gridDim.x) * (TPB / WAVE);
  const int lane = lane_id();
  long long cntx = 0;
  for (int64_t p = (int64_t(blockIdx.x) * TPB + threadIdx.x) / WAVE; p < cnt; p += nwaves) {
    const int v = list[p];
    const long long g1 = f_g1[v];
    if (g1 == NO_GAIN) continue;  // uniform
    const __int128 lhs = (__int128)g1 * den;
    const __int128 rhs = -(__int128)num * two_m * k[v];
    if (lhs < rhs) continue;
    if (lane == 0) {
      R[v] = 1;
      cntx++;
    }
    for (int32_t q = off[v] + lane; q < off[v + 1]; q += WAVE) R[adj[q].x] = 1;
  }
  block_add(cntx, expanded);
}

__global__ void k_src_bits(const int32_t* __restrict__ list, const int32_t* __restrict__ count,
                           uint8_t* uflag) {
  const int64_t cnt = *count;
  GRID_STRIDE(p, cnt) { uflag[list[p]] = 1; }
}

__global__ void __launch_bounds__(TPB)
    k_union_flags(const int32_t* __restrict__ dflag, int32_t n, uint8_t* uflag, int32_t* flag,
                  long long* ndel) {
  long long c = 0;
  GRID_STRIDE(v, n) {
    const bool d = dflag[v] != 0;
    const uint8_t f = uint8_t(uflag[v] | (d ? 2 : 0));
    uflag[v] = f;
    flag[v] = f != 0 ? 1 : 0;
    c += d ? 1 : 0;
  }
  block_add(c, ndel);
}

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

void screen_union(const uint64_t* ch_key, const int32_t* ch_op, const int32_t* ins_pos,
                  const uint64_t* ins_keys, int64_t n_ins, int64_t nch, int32_t n,
                  const int32_t* C, int32_t* sbits, uint8_t* uflag, int32_t* seg_beg,
                  int32_t* seg_end, int32_t* hflag, long long* n_src, long long* n_dsrc,
                  hipStream_t st) {
  if (nch <= 0) return;
  k_screen_kinds<<<grid_for(nch), TPB, 0, st>>>(ch_key, ch_op, ins_pos, ins_keys, n_ins, nch, n,
                                                C, sbits, seg_beg, seg_end);
  DC_LAUNCH_CHECK();
  k_screen_heads<<<grid_for(nch), TPB, 0, st>>>(ch_key, nch, n, sbits, uflag, hflag,
                                                      n_src, n_dsrc);
  DC_LAUNCH_CHECK();
}

void mark_neighbourhoods(const int32_t* list, int64_t cnt, const int32_t* off, const int2* adj,
                         uint8_t* R, hipStream_t st) {
  if (cnt <= 0) return;
  k_mark_neighbourhoods<<<grid_for(cnt * WAVE, 4096), TPB, 0, st>>>(list, cnt, off, adj, R);
  DC_LAUNCH_CHECK();
}

void materialize_R(uint8_t* R, const uint8_t* cflag, const int32_t* C, int32_t n,
                   int32_t* list, int32_t* count, hipStream_t st) {
  if (n <= 0) return;
  k_materialize_R<<<int(ceil_div(n, RL_ROUNDS * TPB)), TPB, 0, st>>>(R, cflag, C, n, list,
                                                                      count);
  DC_LAUNCH_CHECK();
}

void apply_pre(const int32_t* list, int64_t cnt, const uint8_t* R, const int32_t* pre,
               int32_t* Cn, hipStream_t st) {
  if (cnt <= 0) return;
  k_apply_pre<<<grid_for(cnt), TPB, 0, st>>>(list, cnt, R, pre, Cn);
  DC_LAUNCH_CHECK();
}

void cascade_candidates(const int32_t* list, int64_t cnt, const uint8_t* accflag,
                        const int32_t* off, const int2* adj, const int32_t* C, uint8_t* cand,
                        hipStream_t st) {
  if (cnt <= 0) return;
  k_cascade_candidates<<<grid_for(cnt * WAVE), TPB, 0, st>>>(list, cnt, accflag, off,
                                                                       adj, C, cand);
  DC_LAUNCH_CHECK();
}

void cascade_mark(const int32_t* list, int64_t cnt, const long long* f_g1, const int32_t* k,
                  long long two_m, long long num, long long den, const int32_t* off,
                  const int2* adj, uint8_t* R, long long* expanded, hipStream_t st) {
  if (cnt <= 0) return;
  k_cascade_mark<<<grid_for(cnt * WAVE), TPB, 0, st>>>(list, cnt, f_g1, k, two_m, num,
                                                                 den, off, adj, R, expanded);
  DC_LAUNCH_CHECK();
}

void union_flags(const int32_t* list, const int32_t* count, int64_t max_count,
                 const int32_t* dflag, int32_t n, uint8_t* uflag, int32_t* flag, long long* ndel,
                 hipStream_t st) {
  if (n <= 0) return;
  if (max_count > 0) {
    k_src_bits<<<grid_for(max_count), TPB, 0, st>>>(list, count, uflag);
    DC_LAUNCH_CHECK();
  }
  k_union_flags<<<grid_for(n, 512), TPB, 0, st>>>(dflag, n, uflag, flag, ndel);
  DC_LAUNCH_CHECK();
}

}  // namespace dc
