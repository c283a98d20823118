// coarsen.hip -- graph compaction between levels (Alg. 1) and the final
// projection to canonical labels.
//
// Coarse vertices are the non-empty communities numbered by ascending label.
// Members are grouped by a stable radix sort of (coarse id, vertex), so each
// community's members are contiguous and ascending.  The member list is cut
// into chunks of bounded adjacency volume; one block aggregates a chunk's
// entries by coarse neighbour in an LDS hash table and flushes the partial
// sums into the community's global table, so a hub community's diagonal costs
// one atomic per chunk instead of one per entry.  A pass per community then
// packs its table into the coarse CSR row.
#include <cstring>

#include "dc_louvain.h"

namespace dc {

namespace {

constexpr int TPB = 256;
constexpr int VCH = 1024;            // target adjacency volume of a chunk
constexpr int CHUNK_SLOTS = 4096;    // LDS table; a chunk holds < 2*VCH entries

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
                               uint64_t* keys, uint32_t* vals) {
  GRID_STRIDE(x, n) {
    keys[x] = uint64_t(uint32_t(rank[C[x]]));
    vals[x] = uint32_t(x);
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

__global__ void k_comm_caps(const int32_t* __restrict__ mstart,
                            const int32_t* __restrict__ mvol, int32_t nc,
                            long long* caps) {
  GRID_STRIDE(r, nc) {
    int64_t U = mvol[mstart[r + 1]] - mvol[mstart[r]];
    int64_t lim = U < nc ? U : nc;
    long long c = 2;
    while (c < 2 * lim) c <<= 1;
    caps[r] = c;
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
    if (p == ms || mdeg[p] > VCH || mdeg[p - 1] > VCH) {
      h = 1;
    } else {
      int32_t vin = mvol[p] - mvol[ms];
      int32_t vprev = mvol[p - 1] - mvol[ms];
      h = (vin / VCH) != (vprev / VCH) ? 1 : 0;
    }
    head[p] = h;
  }
}

// one block per chunk of members of one community
__global__ void __launch_bounds__(TPB)
    k_coarse_agg(const int32_t* __restrict__ chunks, const uint64_t* __restrict__ rkey,
                 const uint32_t* __restrict__ members, const int32_t* __restrict__ mvol,
                 const int32_t* __restrict__ mdeg, const int32_t* __restrict__ off,
                 const int2* __restrict__ adj, const int32_t* __restrict__ C,
                 const int32_t* __restrict__ rank, const long long* __restrict__ tab_off,
                 int* tkeys, int* tvals) {
  __shared__ int keys[CHUNK_SLOTS];
  __shared__ int vals[CHUNK_SLOTS];
  const int32_t p0 = chunks[blockIdx.x], p1 = chunks[blockIdx.x + 1];
  const int32_t r = int32_t(rkey[p0]);
  const long long t0 = tab_off[r];
  int* gk = tkeys + t0;
  int* gv = tvals + t0;
  const uint32_t gmask = uint32_t(tab_off[r + 1] - t0) - 1;
  if (p1 - p0 == 1 && mdeg[p0] > VCH) {
    const uint32_t x = members[p0];
    for (int32_t j = off[x] + threadIdx.x; j < off[x + 1]; j += TPB) {
      int2 e = adj[j];
      table_add(gk, gv, gmask, rank[C[e.x]], e.y);
    }
    return;
  }
  for (int s = threadIdx.x; s < CHUNK_SLOTS; s += TPB) {
    keys[s] = EMPTY_KEY;
    vals[s] = 0;
  }
  __syncthreads();
  const int32_t v0 = mvol[p0], v1 = mvol[p1];
  for (int32_t q = v0 + threadIdx.x; q < v1; q += TPB) {
    // member p with mvol[p] <= q < mvol[p+1]
    int32_t lo = p0, hi = p1 - 1;
    while (lo < hi) {
      int32_t mid = (lo + hi + 1) >> 1;
      if (mvol[mid] <= q)
        lo = mid;
      else
        hi = mid - 1;
    }
    const uint32_t x = members[lo];
    int2 e = adj[off[x] + (q - mvol[lo])];
    table_add(keys, vals, CHUNK_SLOTS - 1, rank[C[e.x]], e.y);
  }
  __syncthreads();
  for (int s = threadIdx.x; s < CHUNK_SLOTS; s += TPB) {
    int key = keys[s];
    if (key != EMPTY_KEY) table_add(gk, gv, gmask, key, vals[s]);
  }
}

// one wave per community: number of occupied slots
__global__ void k_comm_count(const long long* __restrict__ tab_off,
                             const int* __restrict__ tkeys, int32_t nc, int32_t* cdeg) {
  const int64_t nwaves = int64_t(gridDim.x) * (TPB / WAVE);
  for (int64_t r = int64_t(blockIdx.x) * (TPB / WAVE) + threadIdx.x / WAVE; r < nc;
       r += nwaves) {
    int32_t c = 0;
    for (long long s = tab_off[r] + lane_id(); s < tab_off[r + 1]; s += WAVE)
      c += tkeys[s] != EMPTY_KEY ? 1 : 0;
    c = wave_sum(c);
    if (lane_id() == 0) cdeg[r] = c;
  }
}

__global__ void k_comm_fill(const long long* __restrict__ tab_off,
                            const int* __restrict__ tkeys, const int* __restrict__ tvals,
                            int32_t nc, const int32_t* __restrict__ coff, int2* cadj) {
  const int64_t nwaves = int64_t(gridDim.x) * (TPB / WAVE);
  const uint64_t lt = (uint64_t(1) << lane_id()) - 1;
  for (int64_t r = int64_t(blockIdx.x) * (TPB / WAVE) + threadIdx.x / WAVE; r < nc;
       r += nwaves) {
    int32_t w = coff[r];
    for (long long s0 = tab_off[r]; s0 < tab_off[r + 1]; s0 += WAVE) {
      long long s = s0 + lane_id();
      bool occ = s < tab_off[r + 1] && tkeys[s] != EMPTY_KEY;
      uint64_t m = __ballot(occ);
      if (occ) cadj[w + __popcll(m & lt)] = make_int2(tkeys[s], tvals[s]);
      w += __popcll(m);
    }
  }
}

__global__ void k_coarse_k(const int32_t* __restrict__ labof, const int32_t* __restrict__ a,
                           int32_t nc, int32_t* k) {
  GRID_STRIDE(r, nc) { k[r] = a[labof[r]]; }
}

__global__ void k_first_level_meta(const int32_t* __restrict__ labof,
                                   const int32_t* __restrict__ sz,
                                   const int32_t* __restrict__ mstart,
                                   const uint32_t* __restrict__ members, int32_t nc,
                                   int32_t* cnt_out, int32_t* minv_out) {
  GRID_STRIDE(r, nc) {
    cnt_out[r] = sz[labof[r]];
    minv_out[r] = int32_t(members[mstart[r]]);
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
  k_member_pairs<<<grid_for(nl), TPB, 0, st>>>(C, rank, nl, rkey, members);
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

  // per-community global tables
  s.caps.ensure(size_t(nc + 1) * 8);
  long long* caps = s.caps.as<long long>();
  k_comm_caps<<<grid_for(nc), TPB, 0, st>>>(mstart, mvol, nc, caps);
  DC_LAUNCH_CHECK();
  scan_excl_i64(reinterpret_cast<int64_t*>(caps), reinterpret_cast<int64_t*>(caps), nc,
                reinterpret_cast<int64_t*>(caps + nc), st);

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
  DC_HIP(hipMemcpyAsync(host + 2, caps + nc, 8, hipMemcpyDeviceToHost, st));
  DC_HIP(hipStreamSynchronize(st));
  const int32_t nchunks = host[0];
  long long tslots;
  memcpy(&tslots, host + 2, 8);
  fill_i32(chunks + nchunks, nl, 1, st);

  s.tkeys.ensure(size_t(tslots) * 4);
  s.tvals.ensure(size_t(tslots) * 4);
  int* tkeys = s.tkeys.as<int>();
  int* tvals = s.tvals.as<int>();
  fill_i32(tkeys, EMPTY_KEY, tslots, st);
  fill_i32(tvals, 0, tslots, st);
  if (nchunks > 0) {
    k_coarse_agg<<<nchunks, TPB, 0, st>>>(chunks, rkey, members, mvol, mdeg, g.off, g.adj, C,
                                           rank, caps, tkeys, tvals);
    DC_LAUNCH_CHECK();
  }

  // coarse CSR
  s.cdeg.ensure(size_t(nc + 1) * 4);
  int32_t* cdeg = s.cdeg.as<int32_t>();
  k_comm_count<<<grid_for(int64_t(nc) * WAVE, 4096), TPB, 0, st>>>(caps, tkeys, nc, cdeg);
  DC_LAUNCH_CHECK();
  out.off.ensure(size_t(nc + 1) * 4);
  int32_t* coff = out.off.as<int32_t>();
  scan_excl_i32(cdeg, coff, nc, coff + nc, st);
  DC_HIP(hipMemcpyAsync(host, coff + nc, 4, hipMemcpyDeviceToHost, st));
  DC_HIP(hipStreamSynchronize(st));
  const int32_t cnnz = host[0];
  out.adj.ensure(size_t(cnnz) * 8);
  out.k.ensure(size_t(nc) * 4);
  k_comm_fill<<<grid_for(int64_t(nc) * WAVE, 4096), TPB, 0, st>>>(caps, tkeys, tvals, nc, coff,
                                                                  out.adj.as<int2>());
  DC_LAUNCH_CHECK();
  k_coarse_k<<<grid_for(nc), TPB, 0, st>>>(labof, a, nc, out.k.as<int32_t>());
  DC_LAUNCH_CHECK();
  out.n = nc;
  out.nnz = cnnz;

  // level-0 vertex counts and smallest level-0 ids of the coarse vertices
  if (first_level) {
    k_first_level_meta<<<grid_for(nc), TPB, 0, st>>>(labof, sz, mstart, members, nc, cnt_out,
                                                     minv_out);
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

void finalize_labels(int32_t nL, const int32_t* CL, const int32_t* aL, const int32_t* szL,
                     const int32_t* cntL, const int32_t* minvL, int32_t n0, const int32_t* map0,
                     int32_t* lab, int32_t* cntf, int32_t* C0, int32_t* a0, int32_t* sz0,
                     hipStream_t st) {
  fill_i32(lab, 0x7fffffff, nL, st);
  fill_i32(cntf, 0, nL, st);
  k_final_min<<<grid_for(nL), TPB, 0, st>>>(CL, cntL, minvL, nL, lab, cntf);
  DC_LAUNCH_CHECK();
  fill_i32(a0, 0, n0, st);
  fill_i32(sz0, 0, n0, st);
  k_final_scatter<<<grid_for(nL), TPB, 0, st>>>(lab, cntf, aL, szL, nL, a0, sz0);
  DC_LAUNCH_CHECK();
  k_final_project<<<grid_for(n0), TPB, 0, st>>>(lab, CL, map0, n0, C0);
  DC_LAUNCH_CHECK();
}

}  // namespace dc
