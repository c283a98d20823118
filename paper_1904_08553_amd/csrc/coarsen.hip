// coarsen.hip -- graph compaction between levels (Alg. 1) and the final
// projection to canonical labels.
//
// Coarse vertices are the non-empty communities numbered by ascending label.
// Members are grouped by a stable radix sort of (coarse id, vertex), so each
// community's members are contiguous and ascending.  The member list is cut
// into chunks of bounded adjacency volume; one block sums a chunk's entries
// by coarse neighbour in an LDS hash table and writes the distinct sums as
// (coarse row, coarse column, weight) partials.  Sorting the partials by
// (row, column) and taking segment sums from a prefix scan gives the coarse
// CSR with sorted rows -- no global atomics on hot rows (a hub community's
// diagonal gets one partial per chunk).
#include <cstring>
#include <stdexcept>
#include <utility>

#include "dc_louvain.h"

namespace dc {

namespace {

constexpr int TPB = 256;
constexpr int VCH = 1024;            // target adjacency volume of a chunk
constexpr int CHUNK_SLOTS = 4096;    // LDS table; a slice holds <= 2*VCH entries
constexpr int SLICE = 2 * VCH;       // entries aggregated per table fill
constexpr int MAXM = 512;            // members per chunk (rows may be empty)

inline int grid_for(int64_t n, int64_t cap = 16384) {
  int64_t g = ceil_div(n, TPB);
  if (g > cap) g = cap;
  return int(g < 1 ? 1 : g);
}

#define GRID_STRIDE(i, n)                                              \
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;     \
       i < (n); i += int64_t(gridDim.x) * blockDim.x)

__global__ void k_nonempty(const int32_t* __restrict__ sz, int32_t n, int32_t* flag) {
  GRID_STRIDE(x, n) { flag[x] = sz[x] > 0 ? 1 : 0; }
}

__global__ void k_member_pairs(const int32_t* __restrict__ C,
                               const int32_t* __restrict__ rank, int32_t n,
                               uint64_t* keys, uint32_t* vals, int32_t* rc) {
  GRID_STRIDE(x, n) {
    const int32_t r = rank[C[x]];
    keys[x] = uint64_t(uint32_t(r));
    vals[x] = uint32_t(x);
    rc[x] = r;
  }
}

__global__ void k_comm_info(const int32_t* __restrict__ flag,
                            const int32_t* __restrict__ rank,
                            const int32_t* __restrict__ sz, int32_t n,
                            int32_t* cntr, int32_t* labof) {
  GRID_STRIDE(x, n) {
    if (!flag[x]) continue;
    int32_t r = rank[x];
    cntr[r] = sz[x];
    labof[r] = int32_t(x);
  }
}

__global__ void k_member_deg(const uint32_t* __restrict__ members,
                             const int32_t* __restrict__ off, int32_t n,
                             int32_t* mdeg) {
  GRID_STRIDE(p, n) {
    uint32_t x = members[p];
    mdeg[p] = off[x + 1] - off[x];
  }
}

__global__ void k_chunk_heads(const uint64_t* __restrict__ rkey,
                              const int32_t* __restrict__ mstart,
                              const int32_t* __restrict__ mvol,
                              const int32_t* __restrict__ mdeg, int32_t n,
                              int32_t* head) {
  GRID_STRIDE(p, n) {
    int32_t r = int32_t(rkey[p]);
    int32_t ms = mstart[r];
    int32_t h;
    if (p == ms || mdeg[p] > VCH || mdeg[p - 1] > VCH || (p - ms) % MAXM == 0) {
      h = 1;
    } else {
      int32_t vin = mvol[p] - mvol[ms];
      int32_t vprev = mvol[p - 1] - mvol[ms];
      h = (vin / VCH) != (vprev / VCH) ? 1 : 0;
    }
    head[p] = h;
  }
}

// One block per chunk of members of one community r.  Entries whose far end
// is also in r (the diagonal of the coarse row, usually most of the volume)
// are summed in registers; the rest go into an LDS hash table sized to the
// chunk's volume.  A chunk is either one member whose row exceeds VCH
// entries (walked in slices of SLICE entries) or up to MAXM members with
// fewer than 2*VCH entries in total (one table fill; every thread takes
// independent entries, finding its member in LDS-staged row starts).
// The diagonal sum and the occupied slots are appended as partials.
__device__ __forceinline__ void emit_partials(const int* keys, const int* vals, uint32_t cap,
                                              uint64_t row, int32_t nc, long long diag,
                                              uint64_t* pkey, uint32_t* pval, int32_t* pcount,
                                              int* wc, int* bbase) {
  const int wid = threadIdx.x / WAVE, lane = lane_id();
  const uint64_t lt = (uint64_t(1) << lane) - 1;
  int n_mine = 0;
  for (uint32_t s = threadIdx.x; s < cap; s += TPB) n_mine += keys[s] != EMPTY_KEY ? 1 : 0;
  const int wsum = wave_sum(n_mine);
  if (lane == 0) wc[wid] = wsum;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = diag != 0 ? 1 : 0;
    for (int w = 0; w < TPB / WAVE; ++w) tot += wc[w];
    const int b = atomicAdd(pcount, tot);
    *bbase = b;
    if (diag != 0) {
      pkey[b] = row * uint64_t(nc) + row;
      pval[b] = uint32_t(diag);
    }
  }
  __syncthreads();
  int pos = *bbase + (diag != 0 ? 1 : 0);
  for (int w = 0; w < wid; ++w) pos += wc[w];
  for (uint32_t s0 = 0; s0 < cap; s0 += TPB) {
    const uint32_t s = s0 + threadIdx.x;
    const bool occ = s < cap && keys[s] != EMPTY_KEY;
    const uint64_t m = __ballot(occ);
    if (occ) {
      const int at = pos + __popcll(m & lt);
      pkey[at] = row * uint64_t(nc) + uint64_t(keys[s]);
      pval[at] = uint32_t(vals[s]);
    }
    pos += __popcll(m);
  }
  __syncthreads();
}

__device__ __forceinline__ long long block_sum(long long v, long long* red) {
  v = wave_sum(v);
  const int wid = threadIdx.x / WAVE;
  if (lane_id() == 0) red[wid] = v;
  __syncthreads();
  long long t = 0;
  for (int w = 0; w < TPB / WAVE; ++w) t += red[w];
  __syncthreads();
  return t;
}

__global__ void __launch_bounds__(TPB)
    k_coarse_partials(const int32_t* __restrict__ chunks, const uint64_t* __restrict__ rkey,
                      const uint32_t* __restrict__ members, const int32_t* __restrict__ mvol,
                      const int32_t* __restrict__ off, const int2* __restrict__ adj,
                      const int32_t* __restrict__ rc, int32_t nc, uint64_t* pkey,
                      uint32_t* pval, int32_t* pcount) {
  __shared__ int keys[CHUNK_SLOTS];
  __shared__ int vals[CHUNK_SLOTS];
  __shared__ int wc[TPB / WAVE];
  __shared__ int bbase;
  __shared__ long long red[TPB / WAVE];
  __shared__ int lvol[MAXM + 1];
  __shared__ int lrow[MAXM];
  const int32_t p0 = chunks[blockIdx.x], p1 = chunks[blockIdx.x + 1];
  const int32_t r = int32_t(rkey[p0]);
  const int32_t v0 = mvol[p0], v1 = mvol[p1];
  if (p1 - p0 == 1 && v1 - v0 > VCH) {
    // one long row, in slices
    const uint32_t x = members[p0];
    const int32_t rb = off[x];
    for (int32_t s0 = 0; s0 < v1 - v0; s0 += SLICE) {
      const int32_t s1 = s0 + SLICE < v1 - v0 ? s0 + SLICE : v1 - v0;
      for (int s = threadIdx.x; s < CHUNK_SLOTS; s += TPB) {
        keys[s] = EMPTY_KEY;
        vals[s] = 0;
      }
      __syncthreads();
      long long diag = 0;
      for (int32_t q = s0 + threadIdx.x; q < s1; q += TPB) {
        const int2 e = adj[rb + q];
        const int Y = rc[e.x];
        if (Y == r)
          diag += e.y;
        else
          table_add(keys, vals, CHUNK_SLOTS - 1, Y, e.y);
      }
      diag = block_sum(diag, red);
      emit_partials(keys, vals, CHUNK_SLOTS, uint64_t(r), nc, diag, pkey, pval, pcount, wc,
                    &bbase);
    }
    return;
  }
  // table sized to the chunk: at least twice its volume
  const uint32_t want = 2u * uint32_t(v1 - v0 > 32 ? v1 - v0 : 32);
  uint32_t cap = 1u << (32 - __clz(want - 1));
  if (cap > CHUNK_SLOTS) cap = CHUNK_SLOTS;
  for (uint32_t s = threadIdx.x; s < cap; s += TPB) {
    keys[s] = EMPTY_KEY;
    vals[s] = 0;
  }
  // member volumes and row starts staged in LDS: entry q of the chunk
  // belongs to the last member m with lvol[m] <= q
  const int nm = p1 - p0;
  for (int m = threadIdx.x; m <= nm; m += TPB) lvol[m] = mvol[p0 + m] - v0;
  for (int m = threadIdx.x; m < nm; m += TPB) lrow[m] = off[members[p0 + m]];
  __syncthreads();
  long long diag = 0;
  for (int32_t q = threadIdx.x; q < v1 - v0; q += TPB) {
    int lo = 0, hi = nm - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (lvol[mid] <= q)
        lo = mid;
      else
        hi = mid - 1;
    }
    const int2 e = adj[lrow[lo] + (q - lvol[lo])];
    const int Y = rc[e.x];
    if (Y == r)
      diag += e.y;
    else
      table_add(keys, vals, cap - 1, Y, e.y);
  }
  diag = block_sum(diag, red);
  emit_partials(keys, vals, cap, uint64_t(r), nc, diag, pkey, pval, pcount, wc, &bbase);
}

// Segment sums of sorted partials: the u-th distinct key spans positions
// [hidx[u], hidx[u+1]); its sum is S[hidx[u+1]] - S[hidx[u]] with S the
// exclusive prefix of the weights.
__global__ void k_segment_sums(const uint64_t* __restrict__ pkey,
                               const int32_t* __restrict__ hidx, int64_t U,
                               const int32_t* __restrict__ S, int32_t nc, int2* cadj,
                               uint64_t* ukey) {
  for (int64_t u = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; u < U;
       u += int64_t(gridDim.x) * blockDim.x) {
    const int32_t i = hidx[u], j = hidx[u + 1];
    const uint64_t k = pkey[i];
    cadj[u] = make_int2(int32_t(k % uint64_t(nc)), S[j] - S[i]);
    ukey[u] = k;
  }
}

__global__ void k_u32_to_i32(const uint32_t* __restrict__ in, int64_t n, int32_t* out) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    out[i] = int32_t(in[i]);
}

__global__ void k_coarse_k(const int32_t* __restrict__ labof, const int32_t* __restrict__ a,
                           int32_t nc, int32_t* k) {
  GRID_STRIDE(r, nc) { k[r] = a[labof[r]]; }
}

__global__ void k_first_level_meta(const int32_t* __restrict__ labof,
                                   const int32_t* __restrict__ sz,
                                   const int32_t* __restrict__ mstart,
                                   const uint32_t* __restrict__ members, int32_t nc,
                                   int32_t* cnt_out, int32_t* minv_out, int32_t* minv_keep) {
  GRID_STRIDE(r, nc) {
    cnt_out[r] = sz[labof[r]];
    const int32_t v = int32_t(members[mstart[r]]);
    minv_out[r] = v;
    if (minv_keep) minv_keep[r] = v;
  }
}

__global__ void k_member_cnt(const uint32_t* __restrict__ members,
                             const int32_t* __restrict__ cnt, int32_t n, int32_t* mcnt) {
  GRID_STRIDE(p, n) { mcnt[p] = cnt[members[p]]; }
}

__global__ void k_seg_diff(const int32_t* __restrict__ mstart, const int32_t* __restrict__ S,
                           int32_t nc, int32_t* out) {
  GRID_STRIDE(r, nc) { out[r] = S[mstart[r + 1]] - S[mstart[r]]; }
}

__global__ void k_minv_upper(const int32_t* __restrict__ C, const int32_t* __restrict__ rank,
                             const int32_t* __restrict__ minv, int32_t n, int32_t* minv_out) {
  GRID_STRIDE(x, n) { atomicMin(&minv_out[rank[C[x]]], minv[x]); }
}

__global__ void k_project(const int32_t* __restrict__ C, const int32_t* __restrict__ rank,
                          int32_t n0, bool first, int32_t* map0) {
  GRID_STRIDE(v, n0) {
    int32_t x = first ? int32_t(v) : map0[v];
    map0[v] = rank[C[x]];
  }
}

__global__ void k_final_min(const int32_t* __restrict__ CL, const int32_t* __restrict__ cntL,
                            const int32_t* __restrict__ minvL, int32_t nL, int32_t* lab,
                            int32_t* cntf) {
  GRID_STRIDE(x, nL) {
    int32_t Y = CL[x];
    atomicMin(&lab[Y], minvL[x]);
    atomicAdd(&cntf[Y], cntL[x]);
  }
}

__global__ void k_final_scatter(const int32_t* __restrict__ lab,
                                const int32_t* __restrict__ cntf,
                                const int32_t* __restrict__ aL,
                                const int32_t* __restrict__ szL, int32_t nL, int32_t* a0,
                                int32_t* sz0) {
  GRID_STRIDE(Y, nL) {
    if (szL[Y] <= 0) continue;
    int32_t l = lab[Y];
    a0[l] = aL[Y];
    sz0[l] = cntf[Y];
  }
}

__global__ void k_final_project(const int32_t* __restrict__ lab,
                                const int32_t* __restrict__ CL,
                                const int32_t* __restrict__ map0, int32_t n0, int32_t* C0) {
  GRID_STRIDE(v, n0) { C0[v] = lab[CL[map0[v]]]; }
}

// ---- incremental first-level compaction ----------------------------------

// Entry q of mover u's row (u -> v, weight w) owns four slots from
// 4 * (mpos[u] + q): w leaves (Cold u, Cold v) and joins (Cl u, Cl v); when v
// did not move, the mirror entry (v -> u) moves the same way (a moving v's
// own row carries it, so its mirror slots get weight 0).  A wave checks 64
// consecutive vertices with one load and emits the movers' rows one after
// the other, all lanes on each row.
__global__ void __launch_bounds__(TPB)
    k_emit_movers(const int32_t* __restrict__ Cl, const int32_t* __restrict__ Cold,
                  const int32_t* __restrict__ off, const int2* __restrict__ adj,
                  const int32_t* __restrict__ mpos, int32_t n, uint64_t* keys, uint32_t* vals) {
  const int64_t nbatch = ceil_div(n, WAVE);
  const int64_t nwaves = int64_t(gridDim.x) * (TPB / WAVE);
  const uint64_t N = uint64_t(n);
  const int lane = lane_id();
  for (int64_t bt = int64_t(blockIdx.x) * (TPB / WAVE) + threadIdx.x / WAVE; bt < nbatch;
       bt += nwaves) {
    const int64_t u = bt * WAVE + lane;
    const int co = u < n ? Cold[u] : 0, cn = u < n ? Cl[u] : 0;
    const bool mover = u < n && co != cn;
    const int32_t rb = mover ? off[u] : 0, re = mover ? off[u + 1] : 0;
    const int32_t mp = mover ? mpos[u] : 0;
    for (uint64_t m = __ballot(mover); m; m &= m - 1) {
      const int l = __ffsll((unsigned long long)m) - 1;
      const int cu_old = __builtin_amdgcn_readlane(co, l);
      const int cu_new = __builtin_amdgcn_readlane(cn, l);
      const int32_t b = __builtin_amdgcn_readlane(rb, l), e = __builtin_amdgcn_readlane(re, l);
      const int64_t base = 4 * int64_t(__builtin_amdgcn_readlane(mp, l));
      for (int32_t q = b + lane; q < e; q += WAVE) {
        const int2 en = adj[q];
        const int vo = Cold[en.x], vn = Cl[en.x];
        const bool still = vo == vn;
        const int64_t at = base + 4 * int64_t(q - b);
        keys[at] = uint64_t(cu_old) * N + uint64_t(vo);
        vals[at] = uint32_t(-en.y);
        keys[at + 1] = uint64_t(cu_new) * N + uint64_t(vn);
        vals[at + 1] = uint32_t(en.y);
        keys[at + 2] = uint64_t(vo) * N + uint64_t(cu_old);
        vals[at + 2] = still ? uint32_t(-en.y) : 0u;
        keys[at + 3] = uint64_t(vn) * N + uint64_t(cu_new);
        vals[at + 3] = still ? uint32_t(en.y) : 0u;
      }
    }
  }
}

// The batch's directed changes between the old communities.
__global__ void k_emit_changes(const uint64_t* __restrict__ ch_key,
                               const int32_t* __restrict__ ch_dk, int64_t nch, int32_t n,
                               const int32_t* __restrict__ Cold, uint64_t* keys, uint32_t* vals) {
  GRID_STRIDE(i, nch) {
    const uint64_t k = ch_key[i];
    const int32_t u = int32_t(k / uint64_t(n)), v = int32_t(k % uint64_t(n));
    keys[i] = uint64_t(Cold[u]) * uint64_t(n) + uint64_t(Cold[v]);
    vals[i] = uint32_t(ch_dk[i]);
  }
}

__global__ void k_signed_to_i64(const uint32_t* __restrict__ in, int64_t m, long long* out) {
  GRID_STRIDE(i, m) { out[i] = (long long)int32_t(in[i]); }
}

__global__ void k_set_at(int32_t* arr, const int32_t* __restrict__ idx, int32_t v) {
  arr[*idx] = v;
}

// Run of equal keys starting at head i: sum = S[end] - S[i] (S the exclusive
// prefix sums); flags the runs whose sum is not zero.
__global__ void k_run_sums(const int32_t* __restrict__ heads, const int32_t* __restrict__ hpos,
                           const int32_t* __restrict__ starts, const long long* __restrict__ S,
                           int64_t m, int32_t* nz, long long* rsum) {
  GRID_STRIDE(i, m) {
    int32_t f = 0;
    long long w = 0;
    if (heads[i]) {
      w = S[starts[hpos[i] + 1]] - S[i];
      f = w != 0 ? 1 : 0;
    }
    nz[i] = f;
    rsum[i] = w;
  }
}

__global__ void k_compact_runs(const uint64_t* __restrict__ keys, const int32_t* __restrict__ nz,
                               const int32_t* __restrict__ npos, const long long* __restrict__ rsum,
                               int64_t m, uint64_t* okey, int32_t* ow) {
  GRID_STRIDE(i, m) {
    if (nz[i]) {
      okey[npos[i]] = keys[i];
      ow[npos[i]] = int32_t(rsum[i]);
    }
  }
}

// The two flag arrays of the incremental compaction: non-empty labels and
// the row volumes of the level-0 movers.
__global__ void k_inc_flags(const int32_t* __restrict__ sz, const int32_t* __restrict__ Cl,
                            const int32_t* __restrict__ Cold, const int32_t* __restrict__ off,
                            int32_t n, int32_t* flag, int32_t* mvol) {
  GRID_STRIDE(v, n) {
    flag[v] = sz[v] > 0 ? 1 : 0;
    mvol[v] = Cl[v] != Cold[v] ? off[v + 1] - off[v] : 0;
  }
}

// Community-label entries to coarse ids; bad |= 1 for an entry that touches
// an empty community or has a weight below 1 (cannot happen when H is the
// graph of communities it claims to be).
// The coarse CSR entries of the summed community pairs, and the level-1
// graph kept for the next step (keys x*nc + y, weights).  An entry of an
// empty community or of weight below 1 sets the flag in host memory.
__global__ void k_inc_csr(const uint64_t* __restrict__ keys, const int32_t* __restrict__ w,
                          int64_t cnt, const int32_t* __restrict__ rank,
                          const int32_t* __restrict__ sz, int32_t n, int32_t nc, int2* adj,
                          uint64_t* ukey, int32_t* uw, int32_t* bad_host) {
  GRID_STRIDE(i, cnt) {
    const int32_t X = int32_t(keys[i] / uint64_t(n)), Y = int32_t(keys[i] % uint64_t(n));
    if (sz[X] <= 0 || sz[Y] <= 0 || w[i] < 1) {
      host_store(bad_host, 1);
      adj[i] = make_int2(0, 0);
      ukey[i] = 0;
      uw[i] = 0;
      continue;
    }
    const int32_t x = rank[X], y = rank[Y];
    adj[i] = make_int2(y, w[i]);
    ukey[i] = uint64_t(x) * uint64_t(nc) + uint64_t(y);
    uw[i] = w[i];
  }
}

__global__ void k_adj_weights(const int2* __restrict__ adj, int64_t m, int32_t* w) {
  GRID_STRIDE(i, m) { w[i] = adj[i].y; }
}

// Level-1 entries relabelled by the final labels of their vertices (the
// final label of a level-0 community is that of any of its members).
__global__ void k_relabel(const uint64_t* __restrict__ lkey, const int32_t* __restrict__ lw,
                          int64_t m, int32_t nc, const int32_t* __restrict__ lminv,
                          const int32_t* __restrict__ Ct, int32_t n, uint64_t* okey,
                          uint32_t* ow) {
  GRID_STRIDE(i, m) {
    const uint64_t k = lkey[i];
    okey[i] = uint64_t(Ct[lminv[int32_t(k / uint64_t(nc))]]) * uint64_t(n) +
              uint64_t(Ct[lminv[int32_t(k % uint64_t(nc))]]);
    ow[i] = uint32_t(lw[i]);
  }
}

// Starting values of finalize_labels: the smallest-member labels at +inf,
// the member counts and the level-0 totals and sizes at zero, and the two
// counters zero2 (may be null) at zero.
__global__ void k_final_init(int32_t* lab, int32_t* cntf, int32_t nL, int32_t* a0, int32_t* sz0,
                             int32_t n0, long long* zero2) {
  const int64_t n = nL > n0 ? nL : n0;
  GRID_STRIDE(i, n) {
    if (i < nL) {
      lab[i] = 0x7fffffff;
      cntf[i] = 0;
    }
    if (i < n0) {
      a0[i] = 0;
      sz0[i] = 0;
    }
  }
  if (zero2 && blockIdx.x == 0 && threadIdx.x < 2) zero2[threadIdx.x] = 0;
}

}  // namespace

void coarsen(const LevelView& g, const int32_t* C, const int32_t* sz, const int32_t* a,
             const int32_t* cnt, const int32_t* minv, bool first_level, int32_t n0,
             int32_t* map0, CoarseGraph& out, int32_t* cnt_out, int32_t* minv_out,
             CoarsenScratch& s, hipStream_t st) {
  const int32_t nl = g.n;
  int32_t* host = static_cast<int32_t*>(s.host);
  // ranks of the non-empty labels
  s.flag.ensure(size_t(nl + 1) * 4);
  s.rank.ensure(size_t(nl + 1) * 4);
  int32_t* flag = s.flag.as<int32_t>();
  int32_t* rank = s.rank.as<int32_t>();
  k_nonempty<<<grid_for(nl), TPB, 0, st>>>(sz, nl, flag);
  DC_LAUNCH_CHECK();
  scan_excl_i32(flag, rank, nl, rank + nl, st);
  DC_HIP(hipMemcpyAsync(host, rank + nl, 4, hipMemcpyDeviceToHost, st));
  DC_HIP(hipStreamSynchronize(st));
  const int32_t nc = host[0];

  // members grouped by coarse id, ascending vertex within a group
  s.keys0.ensure(size_t(nl) * 8);
  s.keys1.ensure(size_t(nl) * 8);
  s.vals0.ensure(size_t(nl) * 4);
  s.vals1.ensure(size_t(nl) * 4);
  uint64_t* rkey = s.keys0.as<uint64_t>();
  uint32_t* members = s.vals0.as<uint32_t>();
  s.rc.ensure(size_t(nl + 1) * 4);
  int32_t* rc = s.rc.as<int32_t>();
  k_member_pairs<<<grid_for(nl), TPB, 0, st>>>(C, rank, nl, rkey, members, rc);
  DC_LAUNCH_CHECK();
  radix_sort_pairs(rkey, members, s.keys1.as<uint64_t>(), s.vals1.as<uint32_t>(), nl,
                   ilog2_ceil(uint64_t(nc)), st);

  s.cntr.ensure(size_t(nc + 1) * 4);
  s.mstart.ensure(size_t(nc + 1) * 4);
  s.labof.ensure(size_t(nc + 1) * 4);
  int32_t* cntr = s.cntr.as<int32_t>();
  int32_t* mstart = s.mstart.as<int32_t>();
  int32_t* labof = s.labof.as<int32_t>();
  k_comm_info<<<grid_for(nl), TPB, 0, st>>>(flag, rank, sz, nl, cntr, labof);
  DC_LAUNCH_CHECK();
  scan_excl_i32(cntr, mstart, nc, mstart + nc, st);

  s.mdeg.ensure(size_t(nl + 1) * 4);
  s.mvol.ensure(size_t(nl + 1) * 4);
  int32_t* mdeg = s.mdeg.as<int32_t>();
  int32_t* mvol = s.mvol.as<int32_t>();
  k_member_deg<<<grid_for(nl), TPB, 0, st>>>(members, g.off, nl, mdeg);
  DC_LAUNCH_CHECK();
  scan_excl_i32(mdeg, mvol, nl, mvol + nl, st);

  // chunks of bounded volume
  s.chead.ensure(size_t(nl + 1) * 4);
  s.cpos.ensure(size_t(nl + 1) * 4);
  s.chunks.ensure(size_t(nl + 1) * 4);
  int32_t* chead = s.chead.as<int32_t>();
  int32_t* cpos = s.cpos.as<int32_t>();
  int32_t* chunks = s.chunks.as<int32_t>();
  k_chunk_heads<<<grid_for(nl), TPB, 0, st>>>(rkey, mstart, mvol, mdeg, nl, chead);
  DC_LAUNCH_CHECK();
  scan_excl_i32(chead, cpos, nl, cpos + nl, st);
  compact_index(chead, cpos, nl, chunks, st);
  DC_HIP(hipMemcpyAsync(host, cpos + nl, 4, hipMemcpyDeviceToHost, st));
  DC_HIP(hipStreamSynchronize(st));
  const int32_t nchunks = host[0];
  fill_i32(chunks + nchunks, nl, 1, st);

  // partial sums per chunk, at most one per entry
  const int64_t pcap = g.nnz + 1;
  s.pk0.ensure(size_t(pcap) * 8);
  s.pk1.ensure(size_t(pcap) * 8);
  s.pv0.ensure(size_t(pcap) * 4);
  s.pv1.ensure(size_t(pcap) * 4);
  s.ph.ensure(size_t(pcap + 1) * 4);
  s.pp.ensure(size_t(pcap + 1) * 4);
  s.pS.ensure(size_t(pcap + 1) * 4);
  uint64_t* pkey = s.pk0.as<uint64_t>();
  uint32_t* pval = s.pv0.as<uint32_t>();
  s.pcnt.ensure(8);
  int32_t* pcnt_dev = s.pcnt.as<int32_t>();
  fill_i32(pcnt_dev, 0, 1, st);
  if (nchunks > 0) {
    k_coarse_partials<<<nchunks, TPB, 0, st>>>(chunks, rkey, members, mvol, g.off, g.adj, rc, nc,
                                               pkey, pval, pcnt_dev);
    DC_LAUNCH_CHECK();
  }
  DC_HIP(hipMemcpyAsync(host, pcnt_dev, 4, hipMemcpyDeviceToHost, st));
  DC_HIP(hipStreamSynchronize(st));
  const int64_t P = host[0];
  radix_sort_pairs(pkey, pval, s.pk1.as<uint64_t>(), s.pv1.as<uint32_t>(), P,
                   ilog2_ceil(uint64_t(nc) * uint64_t(nc)), st);
  int32_t* ph = s.ph.as<int32_t>();
  int32_t* pp = s.pp.as<int32_t>();
  int32_t* pS = s.pS.as<int32_t>();
  run_heads(pkey, P, ph, st);
  scan_excl_i32(ph, pp, P, pp + P, st);
  k_u32_to_i32<<<grid_for(P), TPB, 0, st>>>(pval, P, pS);
  DC_LAUNCH_CHECK();
  scan_excl_i32(pS, pS, P, pS + P, st);
  DC_HIP(hipMemcpyAsync(host, pp + P, 4, hipMemcpyDeviceToHost, st));
  DC_HIP(hipStreamSynchronize(st));
  const int32_t cnnz = P > 0 ? host[0] : 0;
  s.hidx.ensure(size_t(cnnz + 1) * 4);
  int32_t* hidx = s.hidx.as<int32_t>();
  compact_index(ph, pp, P, hidx, st);
  fill_i32(hidx + cnnz, int32_t(P), 1, st);

  // coarse CSR: rows sorted by coarse neighbour
  out.off.ensure(size_t(nc + 1) * 4);
  out.adj.ensure(size_t(cnnz + 1) * 8);
  out.k.ensure(size_t(nc + 1) * 4);
  s.ukey.ensure(size_t(cnnz + 1) * 8);
  int32_t* coff = out.off.as<int32_t>();
  if (P > 0) {
    k_segment_sums<<<grid_for(cnnz), TPB, 0, st>>>(pkey, hidx, cnnz, pS, nc,
                                                   out.adj.as<int2>(), s.ukey.as<uint64_t>());
    DC_LAUNCH_CHECK();
  }
  row_bounds(s.ukey.as<uint64_t>(), cnnz, nc, coff, st);
  k_coarse_k<<<grid_for(nc), TPB, 0, st>>>(labof, a, nc, out.k.as<int32_t>());
  DC_LAUNCH_CHECK();
  out.n = nc;
  out.nnz = cnnz;

  // level-0 vertex counts and smallest level-0 ids of the coarse vertices
  if (first_level) {
    k_first_level_meta<<<grid_for(nc), TPB, 0, st>>>(labof, sz, mstart, members, nc, cnt_out,
                                                     minv_out, nullptr);
    DC_LAUNCH_CHECK();
  } else {
    s.mcnt.ensure(size_t(nl + 1) * 4);
    int32_t* mcnt = s.mcnt.as<int32_t>();
    k_member_cnt<<<grid_for(nl), TPB, 0, st>>>(members, cnt, nl, mcnt);
    DC_LAUNCH_CHECK();
    scan_excl_i32(mcnt, mcnt, nl, mcnt + nl, st);
    k_seg_diff<<<grid_for(nc), TPB, 0, st>>>(mstart, mcnt, nc, cnt_out);
    DC_LAUNCH_CHECK();
    fill_i32(minv_out, 0x7fffffff, nc, st);
    k_minv_upper<<<grid_for(nl), TPB, 0, st>>>(C, rank, minv, nl, minv_out);
    DC_LAUNCH_CHECK();
  }
  k_project<<<grid_for(n0), TPB, 0, st>>>(C, rank, n0, first_level, map0);
  DC_LAUNCH_CHECK();
}

namespace {

void swap_buf(DBuf& x, DBuf& y) {
  std::swap(x.p, y.p);
  std::swap(x.bytes, y.bytes);
}

// ensure(bytes) that keeps the first `keep` bytes when the buffer grows
void grow_keep(DBuf& b, size_t bytes, size_t keep, hipStream_t st) {
  if (b.p && bytes <= b.bytes) return;
  DBuf nb;
  nb.ensure(bytes);
  if (keep > 0 && b.p) DC_HIP(hipMemcpyAsync(nb.p, b.p, keep, hipMemcpyDeviceToDevice, st));
  swap_buf(b, nb);  // the old buffer is freed (after the copy) with nb
}

int32_t* host_alias(CoarsenScratch& s) {
  if (!s.host_dev) DC_HIP(hipHostGetDevicePointer(&s.host_dev, s.host, 0));
  return static_cast<int32_t*>(s.host_dev);
}

// Sums runs of equal keys of a sorted list (values: int32 bit patterns) into
// (okey, ow), dropping runs that sum to zero; returns the number kept.
int64_t reduce_sorted(const uint64_t* keys, const uint32_t* vals, int64_t m, uint64_t* okey,
                      int32_t* ow, IncCoarsen& H, int32_t* host, int32_t* host_dev,
                      hipStream_t st) {
  if (m <= 0) return 0;
  const size_t mm = size_t(m) + 1;
  H.heads.ensure(mm * 4);
  H.hpos.ensure(mm * 4);
  H.starts.ensure(mm * 4);
  H.nz.ensure(mm * 4);
  H.npos.ensure(mm * 4);
  H.v64.ensure(mm * 8);
  H.S.ensure(mm * 8);
  int32_t* heads = H.heads.as<int32_t>();
  int32_t* hpos = H.hpos.as<int32_t>();
  int32_t* starts = H.starts.as<int32_t>();
  int32_t* nz = H.nz.as<int32_t>();
  int32_t* npos = H.npos.as<int32_t>();
  long long* v64 = H.v64.as<long long>();
  long long* S = H.S.as<long long>();
  run_heads(keys, m, heads, st);
  scan_excl_i32(heads, hpos, m, hpos + m, st);
  compact_index(heads, hpos, m, starts, st);
  k_set_at<<<1, 1, 0, st>>>(starts, hpos + m, int32_t(m));
  DC_LAUNCH_CHECK();
  k_signed_to_i64<<<grid_for(m), TPB, 0, st>>>(vals, m, v64);
  DC_LAUNCH_CHECK();
  scan_excl_i64(reinterpret_cast<int64_t*>(v64), reinterpret_cast<int64_t*>(S), m,
                reinterpret_cast<int64_t*>(S + m), st);
  k_run_sums<<<grid_for(m), TPB, 0, st>>>(heads, hpos, starts, S, m, nz, v64);
  DC_LAUNCH_CHECK();
  scan_excl_i32(nz, npos, m, npos + m, st, host_dev);
  k_compact_runs<<<grid_for(m), TPB, 0, st>>>(keys, nz, npos, v64, m, okey, ow);
  DC_LAUNCH_CHECK();
  DC_HIP(hipStreamSynchronize(st));
  return host[0];
}

}  // namespace

void coarsen_first_inc(const LevelView& g, const int32_t* Cl, const int32_t* Cold,
                       const int32_t* sz, const int32_t* a, const uint64_t* ch_key,
                       const int32_t* ch_dk, int64_t nch, int32_t* map0, CoarseGraph& out,
                       int32_t* cnt_out, int32_t* minv_out, CoarsenScratch& s, IncCoarsen& H,
                       hipStream_t st) {
  const int32_t nl = g.n;
  int32_t* host = static_cast<int32_t*>(s.host);
  int32_t* hdev = host_alias(s);  // the kernels write the sizes the host reads here
  // ranks of the non-empty labels (as coarsen)
  s.flag.ensure(size_t(nl + 1) * 4);
  s.rank.ensure(size_t(nl + 1) * 4);
  int32_t* flag = s.flag.as<int32_t>();
  int32_t* rank = s.rank.as<int32_t>();
  // and the movers' row volumes
  H.mvol.ensure(size_t(nl + 1) * 4);
  H.mflag.ensure(size_t(nl + 1) * 4);
  int32_t* mvol = H.mvol.as<int32_t>();
  int32_t* mpos = H.mflag.as<int32_t>();
  k_inc_flags<<<grid_for(nl), TPB, 0, st>>>(sz, Cl, Cold, g.off, nl, flag, mvol);
  DC_LAUNCH_CHECK();
  scan_excl_i32(flag, rank, nl, rank + nl, st, hdev);
  scan_excl_i32(mvol, mpos, nl, mpos + nl, st, hdev + 1);
  DC_HIP(hipStreamSynchronize(st));
  const int32_t nc = host[0];
  const int64_t vol = host[1];

  // members grouped by coarse id: counts and smallest members (as coarsen)
  s.keys0.ensure(size_t(nl) * 8);
  s.keys1.ensure(size_t(nl) * 8);
  s.vals0.ensure(size_t(nl) * 4);
  s.vals1.ensure(size_t(nl) * 4);
  uint64_t* rkey = s.keys0.as<uint64_t>();
  uint32_t* members = s.vals0.as<uint32_t>();
  s.rc.ensure(size_t(nl + 1) * 4);
  k_member_pairs<<<grid_for(nl), TPB, 0, st>>>(Cl, rank, nl, rkey, members, s.rc.as<int32_t>());
  DC_LAUNCH_CHECK();
  if (radix_sort_pairs_swap(rkey, members, s.keys1.as<uint64_t>(), s.vals1.as<uint32_t>(), nl,
                            ilog2_ceil(uint64_t(nc)), st)) {
    swap_buf(s.keys0, s.keys1);  // the sorted pairs are in the second buffers
    swap_buf(s.vals0, s.vals1);
    rkey = s.keys0.as<uint64_t>();
    members = s.vals0.as<uint32_t>();
  }
  s.cntr.ensure(size_t(nc + 1) * 4);
  s.mstart.ensure(size_t(nc + 1) * 4);
  s.labof.ensure(size_t(nc + 1) * 4);
  int32_t* cntr = s.cntr.as<int32_t>();
  int32_t* mstart = s.mstart.as<int32_t>();
  int32_t* labof = s.labof.as<int32_t>();
  k_comm_info<<<grid_for(nl), TPB, 0, st>>>(flag, rank, sz, nl, cntr, labof);
  DC_LAUNCH_CHECK();
  scan_excl_i32(cntr, mstart, nc, mstart + nc, st);

  // H(G_{t-1}, C_{t-1}) + the batch's changes + the movers' rows, one sort;
  // H's h entries already lead the sort's input buffers (inc_finish)
  const int64_t h = H.h, m = h + nch + 4 * vol;
  grow_keep(H.ek0, size_t(m + 1) * 8, size_t(h) * 8, st);
  grow_keep(H.ev0, size_t(m + 1) * 4, size_t(h) * 4, st);
  H.ek1.ensure(size_t(m + 1) * 8);
  H.ev1.ensure(size_t(m + 1) * 4);
  uint64_t* ek = H.ek0.as<uint64_t>();
  uint32_t* ev = H.ev0.as<uint32_t>();
  if (nch > 0) {
    k_emit_changes<<<grid_for(nch), TPB, 0, st>>>(ch_key, ch_dk, nch, nl, Cold, ek + h, ev + h);
    DC_LAUNCH_CHECK();
  }
  if (vol > 0) {
    k_emit_movers<<<grid_for(ceil_div(nl, WAVE) * WAVE), TPB, 0, st>>>(Cl, Cold, g.off, g.adj, mpos, nl,
                                                              ek + h + nch, ev + h + nch);
    DC_LAUNCH_CHECK();
  }
  radix_sort_pairs(ek, ev, H.ek1.as<uint64_t>(), H.ev1.as<uint32_t>(), m,
                   ilog2_ceil(uint64_t(nl) * uint64_t(nl)), st);
  H.tkey.ensure(size_t(m + 1) * 8);
  H.tw.ensure(size_t(m + 1) * 4);
  const int64_t cnnz = reduce_sorted(ek, ev, m, H.tkey.as<uint64_t>(), H.tw.as<int32_t>(), H,
                                     host, hdev, st);

  // coarse CSR over coarse ids (rows come out sorted: ranks keep label order)
  // its entries go to the coarse CSR and, as the level-1 graph kept for the
  // next step, to H.lkey / H.lw
  out.off.ensure(size_t(nc + 1) * 4);
  out.adj.ensure(size_t(cnnz + 1) * 8);
  out.k.ensure(size_t(nc + 1) * 4);
  H.lkey.ensure(size_t(cnnz + 1) * 8);
  H.lw.ensure(size_t(cnnz + 1) * 4);
  H.lminv.ensure(size_t(nc + 1) * 4);
  host[2] = 0;  // the self-check flag, set by the kernel in host memory
  if (cnnz > 0) {
    k_inc_csr<<<grid_for(cnnz), TPB, 0, st>>>(H.tkey.as<uint64_t>(), H.tw.as<int32_t>(), cnnz,
                                              rank, sz, nl, nc, out.adj.as<int2>(),
                                              H.lkey.as<uint64_t>(), H.lw.as<int32_t>(),
                                              hdev + 2);
    DC_LAUNCH_CHECK();
  }
  s.inc_check = true;  // read after the caller's next wait (inc_check)
  row_bounds(H.lkey.as<uint64_t>(), cnnz, nc, out.off.as<int32_t>(), st);
  k_coarse_k<<<grid_for(nc), TPB, 0, st>>>(labof, a, nc, out.k.as<int32_t>());
  DC_LAUNCH_CHECK();
  out.n = nc;
  out.nnz = cnnz;
  k_first_level_meta<<<grid_for(nc), TPB, 0, st>>>(labof, sz, mstart, members, nc, cnt_out,
                                                   minv_out, H.lminv.as<int32_t>());
  DC_LAUNCH_CHECK();
  k_project<<<grid_for(nl), TPB, 0, st>>>(Cl, rank, nl, true, map0);
  DC_LAUNCH_CHECK();
  H.lh = cnnz;
  H.lnc = nc;
}

void inc_check(CoarsenScratch& s) {
  if (!s.inc_check) return;
  s.inc_check = false;
  if (static_cast<const int32_t*>(s.host)[2])
    throw std::runtime_error("incremental coarsening: inconsistent community graph");
}

void save_level1(const CoarseGraph& out, const CoarsenScratch& s, const int32_t* minv,
                 IncCoarsen& H, hipStream_t st) {
  H.lkey.ensure(size_t(out.nnz + 1) * 8);
  H.lw.ensure(size_t(out.nnz + 1) * 4);
  H.lminv.ensure(size_t(out.n + 1) * 4);
  if (out.nnz > 0) {
    DC_HIP(hipMemcpyAsync(H.lkey.p, s.ukey.p, size_t(out.nnz) * 8, hipMemcpyDeviceToDevice, st));
    k_adj_weights<<<grid_for(out.nnz), TPB, 0, st>>>(out.adj.as<int2>(), out.nnz,
                                                      H.lw.as<int32_t>());
    DC_LAUNCH_CHECK();
  }
  if (out.n > 0)
    DC_HIP(hipMemcpyAsync(H.lminv.p, minv, size_t(out.n) * 4, hipMemcpyDeviceToDevice, st));
  H.lh = out.nnz;
  H.lnc = out.n;
}

void inc_finish(IncCoarsen& H, const int32_t* Ct, int32_t n, CoarsenScratch& s,
                hipStream_t st) {
  (void)s;
  const int64_t m = H.lh;
  // written where the next step's sort reads its input (coarsen_first_inc)
  H.ek0.ensure(size_t(m + 1) * 8);
  H.ev0.ensure(size_t(m + 1) * 4);
  if (m > 0) {
    k_relabel<<<grid_for(m), TPB, 0, st>>>(H.lkey.as<uint64_t>(), H.lw.as<int32_t>(), m, H.lnc,
                                           H.lminv.as<int32_t>(), Ct, n, H.ek0.as<uint64_t>(),
                                           H.ev0.as<uint32_t>());
    DC_LAUNCH_CHECK();
  }
  H.h = m;
  H.valid = true;
}

void finalize_labels(int32_t nL, const int32_t* CL, const int32_t* aL, const int32_t* szL,
                     const int32_t* cntL, const int32_t* minvL, int32_t n0, const int32_t* map0,
                     int32_t* lab, int32_t* cntf, int32_t* C0, int32_t* a0, int32_t* sz0,
                     hipStream_t st, long long* zero2) {
  k_final_init<<<grid_for(nL > n0 ? nL : n0), TPB, 0, st>>>(lab, cntf, nL, a0, sz0, n0, zero2);
  DC_LAUNCH_CHECK();
  k_final_min<<<grid_for(nL), TPB, 0, st>>>(CL, cntL, minvL, nL, lab, cntf);
  DC_LAUNCH_CHECK();
  k_final_scatter<<<grid_for(nL), TPB, 0, st>>>(lab, cntf, aL, szL, nL, a0, sz0);
  DC_LAUNCH_CHECK();
  k_final_project<<<grid_for(n0), TPB, 0, st>>>(lab, CL, map0, n0, C0);
  DC_LAUNCH_CHECK();
}

}  // namespace dc
