// graph.hip -- the dynamic graph G_t (Sec. 3.1): CSR construction, batch
// validation, and the sorted merge of a batch of additions and deletions into
// the next CSR (a streaming pass over tiles of old entries).
#include "dc_kernels.h"

namespace dc {

namespace {

constexpr int TPB = 256;

inline int grid_for(int64_t n, int threads = TPB, int64_t cap = 16384) {
  int64_t g = ceil_div(n, threads);
  if (g > cap) g = cap;
  return int(g < 1 ? 1 : g);
}

#define GRID_STRIDE(i, n)                                              \
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;     \
       i < (n); i += int64_t(gridDim.x) * blockDim.x)

__global__ void k_validate(const int32_t* __restrict__ u,
                           const int32_t* __restrict__ v,
                           const int32_t* __restrict__ w, int64_t m, int32_t n,
                           int32_t* flags, long long* wsum) {
  int32_t f = 0;
  long long s = 0;
  GRID_STRIDE(e, m) {
    int32_t a = u[e], b = v[e];
    if (a < 0 || a >= n || b < 0 || b >= n) f |= F_RANGE;
    if (a == b) f |= F_SELF;
    if (w) {
      int32_t x = w[e];
      if (x < 1) f |= F_WEIGHT;
      s += x;
    }
  }
  block_or(f, flags);
  if (w) block_add(s, wsum + blockIdx.x % SUM_SLOTS);
}

__global__ void k_make_directed(const int32_t* __restrict__ u,
                                const int32_t* __restrict__ v,
                                const int32_t* __restrict__ w, int64_t m,
                                int32_t n, uint64_t* keys, uint32_t* vals) {
  GRID_STRIDE(e, m) {
    uint64_t a = uint32_t(u[e]), b = uint32_t(v[e]);
    keys[2 * e] = a * uint64_t(n) + b;
    keys[2 * e + 1] = b * uint64_t(n) + a;
    vals[2 * e] = uint32_t(w[e]);
    vals[2 * e + 1] = uint32_t(w[e]);
  }
}

__global__ void k_run_heads(const uint64_t* __restrict__ keys, int64_t m,
                            int32_t* flag) {
  GRID_STRIDE(i, m) { flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0; }
}

__global__ void k_reduce_runs(const uint64_t* __restrict__ keys,
                              const uint32_t* __restrict__ vals,
                              const int32_t* __restrict__ wsrc,
                              const int32_t* __restrict__ pos, int64_t m,
                              uint64_t* out_key, int32_t* out_w) {
  GRID_STRIDE(i, m) {
    // pos is the exclusive scan of the head flags: a head at i has index
    // pos[i]; a non-head belongs to the run of the head before it.
    bool head = (i == 0 || keys[i] != keys[i - 1]);
    int32_t r = head ? pos[i] : pos[i] - 1;
    int32_t x = wsrc ? wsrc[vals[i]] : int32_t(vals[i]);
    if (head) out_key[r] = keys[i];
    atomicAdd(&out_w[r], x);
  }
}

// row_ptr[r] = index of the first key of row r or a later row (row = key /
// n, keys sorted), row_ptr[n] = m.  Thread per key, plus one past the end:
// the first key of a row writes the bounds of the rows from the previous
// key's row (exclusive) to its own; a long run of empty rows is written by
// the whole wave.
__global__ void __launch_bounds__(TPB)
    k_row_bounds(const uint64_t* __restrict__ keys, int64_t m, int32_t n, int32_t* row_ptr) {
  const int lane = lane_id();
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  // the loop runs while the wave's first thread is in range (whole waves)
  for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q - lane <= m; q += stride) {
    const bool h = q <= m;
    const long long r1 = !h ? 0 : (q < m ? (long long)(keys[q] / uint64_t(n)) : (long long)n);
    const long long r0 = !h ? 0 : (q > 0 ? (long long)(keys[q - 1] / uint64_t(n)) : -1);
    const bool wide = h && r1 - r0 > WAVE;
    if (h && !wide)
      for (long long r = r0 + 1; r <= r1; ++r) row_ptr[r] = int32_t(q);
    for (uint64_t wm = __ballot(wide); wm; wm &= wm - 1) {
      const int l = __ffsll((unsigned long long)wm) - 1;
      const long long a = readlane64(r0, l) + 1, b = readlane64(r1, l);
      const int32_t qv = __builtin_amdgcn_readlane(int32_t(q), l);
      for (long long r = a + lane; r <= b; r += WAVE) row_ptr[r] = qv;
    }
  }
}

__global__ void k_keys_to_adj(const uint64_t* __restrict__ keys,
                              const int32_t* __restrict__ w, int64_t m,
                              int32_t n, int2* adj) {
  GRID_STRIDE(i, m) { adj[i] = make_int2(int32_t(keys[i] % uint64_t(n)), w[i]); }
}

// one wave per row
__global__ void k_row_weight_sums(const int32_t* __restrict__ off,
                                  const int2* __restrict__ adj, int32_t n,
                                  int32_t* k) {
  int64_t row = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / WAVE;
  int lane = lane_id();
  if (row >= n) return;
  int32_t b = off[row], e = off[row + 1];
  int32_t s = 0;
  for (int32_t j = b + lane; j < e; j += WAVE) s += adj[j].y;
  s = wave_sum(s);
  if (lane == 0) k[row] = s;
}

__device__ __forceinline__ int32_t find_in_row(const int2* adj, int32_t b,
                                               int32_t e, int32_t c) {
  // first position p in [b, e) with adj[p].x >= c
  while (b < e) {
    int32_t mid = (b + e) >> 1;
    if (adj[mid].x < c)
      b = mid + 1;
    else
      e = mid;
  }
  return b;
}

// Directed change records straight from the batch: deletion e gives keys
// u*n+v and v*n+u with value 2e, insertion e the same keys with value 2e+1.
__global__ void k_batch_records(const int32_t* __restrict__ du, const int32_t* __restrict__ dv,
                                int64_t nd, const int32_t* __restrict__ au,
                                const int32_t* __restrict__ av, int64_t na, int32_t n,
                                uint64_t* keys, uint32_t* vals) {
  GRID_STRIDE(i, nd + na) {
    const bool del = i < nd;
    const int64_t j = del ? i : i - nd;
    const uint64_t a = uint32_t(del ? du[j] : au[j]), b = uint32_t(del ? dv[j] : av[j]);
    const uint32_t val = (uint32_t(j) << 1) | (del ? 0u : 1u);
    keys[2 * i] = a * uint64_t(n) + b;
    keys[2 * i + 1] = b * uint64_t(n) + a;
    vals[2 * i] = val;
    vals[2 * i + 1] = val;
  }
}

// Per sorted record: its run (pos = exclusive scan of the run heads) gets
// the record's insertion weight, or one more deletion.  run_w and run_ndel
// must be zeroed.
__global__ void k_run_accumulate(const uint64_t* __restrict__ keys,
                                 const uint32_t* __restrict__ vals,
                                 const int32_t* __restrict__ pos, int64_t m,
                                 const int32_t* __restrict__ ins_w, uint64_t* run_key,
                                 int32_t* run_w, int32_t* run_ndel) {
  GRID_STRIDE(i, m) {
    const bool head = i == 0 || keys[i] != keys[i - 1];
    const int32_t r = head ? pos[i] : pos[i] - 1;
    if (head) run_key[r] = keys[i];
    const uint32_t v = vals[i];
    if (v & 1u)
      atomicAdd(&run_w[r], ins_w[v >> 1]);
    else
      atomicAdd(&run_ndel[r], 1);
  }
}

// One change per directed pair (run r < *nruns): two deletions of one pair
// flag F_DUP, a deletion of a pair absent from G_{t-1} flags F_NO_EDGE;
// *wsum += the old weights of the deleted pairs (counted once, at src < dst).
// A deletion with insertions is a REPLACE (new weight = their sum), a
// deletion alone a DELETE, insertions alone an ADD to an existing pair or a
// NEW one.  Ids out of range are skipped (their batch fails on F_RANGE).
__global__ void k_resolve_runs(const uint64_t* __restrict__ run_key,
                               const int32_t* __restrict__ run_w,
                               const int32_t* __restrict__ run_ndel,
                               const int32_t* __restrict__ nruns, int32_t n,
                               const int32_t* __restrict__ off, const int2* __restrict__ adj,
                               uint64_t* ch_key, int32_t* ch_op, int32_t* ch_w, int32_t* ch_dk,
                               int32_t* dnet, int32_t* flags, long long* wsum) {
  const int64_t cnt = *nruns;
  int32_t f = 0;
  long long s = 0;
  GRID_STRIDE(r, cnt) {
    const uint64_t key = run_key[r];
    const uint64_t src = key / uint64_t(n), dst = key % uint64_t(n);
    const int32_t nd = run_ndel[r], wi = run_w[r];
    int32_t wo = 0;
    bool exists = false;
    if (src < uint64_t(n) && dst < uint64_t(n)) {
      // G is symmetric: search the shorter of the two rows (a hub's
      // neighbours find their pair in their own short row)
      const int32_t bs = off[src], es = off[src + 1], bd = off[dst], ed = off[dst + 1];
      const bool own = es - bs <= ed - bd;
      const int32_t b = own ? bs : bd, e = own ? es : ed;
      const int32_t x = own ? int32_t(dst) : int32_t(src);
      const int32_t p = find_in_row(adj, b, e, x);
      exists = p < e && adj[p].x == x;
      wo = exists ? adj[p].y : 0;
    }
    if (nd > 1) f |= F_DUP;
    if (nd > 0 && !exists) f |= F_NO_EDGE;
    if (nd > 0 && src < dst) s += wo;
    int32_t op, w, dk;
    if (nd > 0 && wi > 0) {
      op = OP_REPLACE;
      w = wi;
      dk = wi - wo;
    } else if (nd > 0) {
      op = OP_DELETE;
      w = 0;
      dk = -wo;
    } else {
      op = exists ? OP_ADD : OP_NEW;
      w = wi;
      dk = wi;
    }
    ch_key[r] = key;
    ch_op[r] = op;
    ch_w[r] = w;
    ch_dk[r] = dk;
    dnet[r] = op == OP_NEW ? 1 : (op == OP_DELETE ? -1 : 0);
  }
  block_or(f, flags);
  block_add(s, wsum + blockIdx.x % SUM_SLOTS);
}


// Thread per row: new degree, k += the row's weight change, the label
// totals a[C(u)] += the same change, and the rows that begin the merge's
// tiles.  A block walks many rows and sums the
// label changes in its LDS table first, so a large community receives one
// update per block instead of one per row (same-address atomics serialise).
constexpr int RC_U = 4;        // rows a thread takes per iteration
constexpr int RC_MANY = 8;     // rows with more changes are summed by a wave
constexpr int RC_TPB = 1024;   // one large block per CU: fewer flushes per label
constexpr int RC_BLOCKS = 256;
__global__ void __launch_bounds__(RC_TPB)
    k_row_changes(const int32_t* __restrict__ cptr,
                  const int32_t* __restrict__ ch_op,
                  const int32_t* __restrict__ ch_dk,
                  const int32_t* __restrict__ off, int32_t n, int32_t* new_deg,
                  int32_t* k, const int32_t* __restrict__ C, int32_t* a,
                  int32_t* tile_row) {
  __shared__ AggLds agg;
  agg_init(agg);
  __syncthreads();
  const int32_t nnz = off[n];
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  // RC_U rows per iteration, their loads issued before any is used; the
  // loop runs while the wave's first row is in range, so whole waves take
  // part in the wave sums below
  for (int64_t u0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; u0 - lane_id() < n;
       u0 += RC_U * stride) {
    int32_t b[RC_U], e[RC_U], ob[RC_U], oe[RC_U], cu[RC_U];
#pragma unroll
    for (int r = 0; r < RC_U; ++r) {
      // clamped index (n >= 1): unconditional loads, all in flight together
      const int64_t u = u0 + r * stride;
      const bool h = u < n;
      const int64_t uc = h ? u : n - 1;
      const int32_t x0 = cptr[uc], x1 = cptr[uc + 1], y0 = off[uc], y1 = off[uc + 1], c = C[uc];
      b[r] = h ? x0 : 0;
      e[r] = h ? x1 : 0;
      ob[r] = h ? y0 : 0;
      oe[r] = h ? y1 : 0;
      cu[r] = h ? c : 0;
    }
#pragma unroll
    for (int r = 0; r < RC_U; ++r) {
      const int64_t u = u0 + r * stride;
      int32_t dd = 0, dk = 0;
      // a row with many changes (a hub) is summed by the whole wave, one
      // such row after the other; the others by their own thread
      uint64_t many = __ballot(e[r] - b[r] > RC_MANY);
      while (many) {
        const int l = __ffsll((unsigned long long)many) - 1;
        many &= many - 1;
        const int32_t qb = __builtin_amdgcn_readlane(b[r], l);
        const int32_t qe = __builtin_amdgcn_readlane(e[r], l);
        int32_t sd = 0, sk = 0;
        for (int32_t q = qb + lane_id(); q < qe; q += WAVE) {
          const int32_t op = ch_op[q];
          sd += op == OP_NEW ? 1 : (op == OP_DELETE ? -1 : 0);
          sk += ch_dk[q];
        }
        sd = wave_sum(sd);
        sk = wave_sum(sk);
        if (lane_id() == l) {
          dd = sd;
          dk = sk;
        }
      }
      if (e[r] > b[r] && e[r] - b[r] <= RC_MANY) {
        // all RC_MANY slots loaded at once (indexes clamped to the row's
        // last change), then the ones inside the row summed
        int32_t ops[RC_MANY], dks[RC_MANY];
#pragma unroll
        for (int j = 0; j < RC_MANY; ++j) {
          const int32_t q = b[r] + j < e[r] ? b[r] + j : e[r] - 1;
          ops[j] = ch_op[q];
          dks[j] = ch_dk[q];
        }
#pragma unroll
        for (int j = 0; j < RC_MANY; ++j) {
          if (b[r] + j < e[r]) {
            dd += ops[j] == OP_NEW ? 1 : (ops[j] == OP_DELETE ? -1 : 0);
            dk += dks[j];
          }
        }
      }
      if (u >= n) continue;
      new_deg[u] = oe[r] - ob[r] + dd;
      // merge tiles: the row holding each tile's first entry, and after
      // the last tile the row holding the last entry
      if (oe[r] > ob[r]) {
        for (int64_t t = ceil_div(ob[r], MERGE_TILE); t * MERGE_TILE < oe[r]; ++t)
          tile_row[t] = int32_t(u);
        if (oe[r] == nnz) tile_row[ceil_div(nnz, MERGE_TILE)] = int32_t(u);
      }
      if (dk != 0) {
        k[u] += dk;
        if (!agg_try(agg, cu[r], dk)) atomicAdd(&a[cu[r]], dk);
      }
    }
  }
  __syncthreads();
  for (int s = threadIdx.x; s < AGG_SLOTS; s += blockDim.x) {
    const int key = agg.keys[s];
    if (key != EMPTY_KEY && agg.vals[s] != 0) atomicAdd(&a[key], int32_t(agg.vals[s]));
  }
}

constexpr int MT_PER = MERGE_TILE / TPB;    // old entries per thread
constexpr int MT_SEGS = MERGE_TILE / WAVE;  // wave-wide segments of a tile
constexpr int MT_CH = 512;                  // changes of a tile staged in LDS
constexpr int MT_ST = MT_CH / TPB + 1;      // staging loads per thread (covers MT_CH + 1)
static_assert(MT_ST * TPB > MT_CH, "the staging loads cover the slice and its end");

// first k in [a, b) with keys[k] >= key
__device__ __forceinline__ int change_rank(const uint64_t* keys, int a, int b, uint64_t key) {
  while (a < b) {
    const int mid = (a + b) >> 1;
    if (keys[mid] < key)
      a = mid + 1;
    else
      b = mid;
  }
  return a;
}

// first k in [a, b) with nbr[k] >= v (the changes of one row, by neighbour)
__device__ __forceinline__ int nbr_rank(const int32_t* nbr, int a, int b, int32_t v) {
  while (a < b) {
    const int mid = (a + b) >> 1;
    if (nbr[mid] < v)
      a = mid + 1;
    else
      b = mid;
  }
  return a;
}

// G_{t-1} -> G_t in one launch over the old entries, cut into tiles of
// MERGE_TILE consecutive entries regardless of where rows begin, so every
// block streams the same amount of contiguous memory.
//
// Old entry j of row r lands at off_new[r] + (j - off_old[r]) + the
// insertions minus the deletions among r's changes with a smaller neighbour
// id: cnet (the exclusive prefix sum of +1 per NEW, -1 per DELETE over the
// change list, which is sorted by (row, neighbour)) at the entry's rank
// among the row's changes, minus cnet at the row's first change.  A DELETE
// of the entry drops it, ADD / REPLACE change its weight.
//
// A tile block first puts, at each row's first entry inside the tile, that
// row's id, offset shift and change range into LDS, together with the
// tile's slice of the change list (the rows of a tile own one contiguous
// slice): per change its neighbour id, its weight, and its op packed with
// cnet relative to the slice's start.  An entry finds its row's slot by a
// ballot over the row-start marks of its 64-entry segment (the nearest mark
// at or before the lane), or from the slot recorded for the segment's first
// entry.  The global loads before the first barrier take clamped indexes
// instead of per-lane bounds branches, so a wave issues them together
// rather than one round trip after another.
//
// The first `nib` blocks instead place the insertions: NEW change q of row
// r goes after the old entries of r with a smaller neighbour (binary search
// in the old row), shifted by cnet[q] - cnet[cptr[r]].  The two kinds of
// block write disjoint slots.
__global__ void __launch_bounds__(TPB)
    k_merge_tiles(const int32_t* __restrict__ off_old, const int2* __restrict__ adj_old,
                  int64_t nnz_old, const int32_t* __restrict__ off_new, int2* adj_new,
                  int32_t n, const int32_t* __restrict__ cptr,
                  const int32_t* __restrict__ tile_row, const uint64_t* __restrict__ ch_key,
                  const int32_t* __restrict__ ch_op, const int32_t* __restrict__ ch_w,
                  const int32_t* __restrict__ cnet, int64_t nch, int nib) {
  __shared__ int32_t s_row[MERGE_TILE];  // at a row's first entry in the tile: the row
  __shared__ int32_t s_sh[MERGE_TILE];   // ... off_new[r] - off_old[r]
  __shared__ int32_t s_cb[MERGE_TILE];   // ... cptr[r]
  __shared__ int32_t s_ce[MERGE_TILE];   // ... cptr[r + 1]
  __shared__ int32_t s_seg[MT_SEGS];     // slot of the row holding entry q * WAVE
  __shared__ int32_t s_nbr[MT_CH];       // neighbour id of change c0 + k
  __shared__ int32_t s_w[MT_CH];         // its weight
  __shared__ int32_t s_nop[MT_CH + 1];   // (cnet[c0 + k] - cnet[c0]) * 8 + its op

  if (int(blockIdx.x) < nib) {
    for (int64_t q = int64_t(blockIdx.x) * TPB + threadIdx.x; q < nch; q += int64_t(nib) * TPB) {
      if (ch_op[q] != OP_NEW) continue;
      const uint64_t key = ch_key[q];
      const int32_t src = int32_t(key / uint64_t(n));
      const int32_t dst = int32_t(key - uint64_t(src) * uint64_t(n));
      const int32_t ob = off_old[src], oe = off_old[src + 1];
      const int32_t less = find_in_row(adj_old, ob, oe, dst) - ob;
      adj_new[off_new[src] + less + cnet[q] - cnet[cptr[src]]] = make_int2(dst, ch_w[q]);
    }
    return;  // block-uniform
  }

  const int64_t tile = int64_t(blockIdx.x) - nib;
  const int64_t t0 = tile * MERGE_TILE;
  const int64_t t1 = t0 + MERGE_TILE < nnz_old ? t0 + MERGE_TILE : nnz_old;
  const int len = int(t1 - t0);  // >= 1: the grid holds ceil(nnz_old / MERGE_TILE) tiles
  const int lane = lane_id();
  const int wbase = int(threadIdx.x / WAVE) * (WAVE * MT_PER);
  int2 e[MT_PER];
#pragma unroll
  for (int q = 0; q < MT_PER; ++q) {
    const int i = wbase + q * WAVE + lane;
    e[q] = adj_old[t0 + (i < len ? i : len - 1)];  // lanes past the end store nothing
  }
  const int32_t r0 = tile_row[tile], r1 = tile_row[tile + 1];  // rows, r1 <= n - 1
  // the bounds of this thread's first row (clamped to r1 where the tile has
  // fewer rows than threads; only rows <= r1 are put)
  const int32_t rf = r0 + int32_t(threadIdx.x);
  const bool hf = rf <= r1;
  const int32_t rc = hf ? rf : r1;
  const int32_t fb = off_old[rc], fen = off_old[rc + 1];
  const int32_t fnb = off_new[rc], fcb = cptr[rc], fce = cptr[rc + 1];
  const int32_t c0 = cptr[r0], nloc = cptr[r1 + 1] - c0;
  const bool staged = nloc <= MT_CH;  // block-uniform
  if (staged && nloc > 0) {           // block-uniform; then c0 + nloc - 1 < nch
    int32_t sn[MT_ST];
    uint64_t sk[MT_ST];
    int32_t so[MT_ST], sw[MT_ST];
#pragma unroll
    for (int u = 0; u < MT_ST; ++u) {
      const int k = u * TPB + int(threadIdx.x);
      const int kn = k < nloc ? k : nloc;      // cnet has nch + 1 entries
      const int kc = k < nloc ? k : nloc - 1;  // the change arrays nch
      sn[u] = cnet[c0 + kn];
      sk[u] = ch_key[c0 + kc];
      so[u] = ch_op[c0 + kc];
      sw[u] = ch_w[c0 + kc];
    }
    const int32_t base = cnet[c0];
#pragma unroll
    for (int u = 0; u < MT_ST; ++u) {
      const int k = u * TPB + int(threadIdx.x);
      if (k < nloc) {
        const uint64_t row = sk[u] / uint64_t(n);
        s_nbr[k] = int32_t(sk[u] - row * uint64_t(n));
        s_w[k] = sw[u];
        s_nop[k] = (sn[u] - base) * 8 + so[u];
      } else if (k == nloc) {
        s_nop[k] = (sn[u] - base) * 8;
      }
    }
  }
  for (int i = threadIdx.x; i < MERGE_TILE; i += TPB) s_row[i] = -1;
  __syncthreads();
  auto put = [&](int32_t r, int32_t b, int32_t en, int32_t sh, int32_t cb, int32_t ce) {
    const int64_t lo = b > t0 ? int64_t(b) : t0, hi = en < t1 ? int64_t(en) : t1;
    if (lo < hi) {
      const int p = int(lo - t0);
      s_row[p] = r;
      s_sh[p] = sh;
      s_cb[p] = cb;
      s_ce[p] = ce;
      for (int s = int(ceil_div(p, WAVE)) * WAVE; s < int(hi - t0); s += WAVE) s_seg[s / WAVE] = p;
    }
  };
  if (hf) put(rf, fb, fen, fnb - fb, fcb, fce);
  for (int32_t r = rf + TPB; r <= r1; r += TPB) {
    const int32_t b = off_old[r];
    put(r, b, off_old[r + 1], off_new[r] - b, cptr[r], cptr[r + 1]);
  }
  __syncthreads();
  const uint64_t upto = (uint64_t(2) << lane) - 1;  // lanes <= this one
#pragma unroll
  for (int q = 0; q < MT_PER; ++q) {
    const int i = wbase + q * WAVE + lane;
    const uint64_t marks = __ballot(s_row[i] >= 0) & upto;
    if (i >= len) continue;
    const int p = marks ? i - lane + 63 - __clzll((long long)marks) : s_seg[i / WAVE];
    const int32_t r = s_row[p], cb = s_cb[p], ce = s_ce[p];
    int32_t shift = s_sh[p];
    int2 v = e[q];
    if (cb != ce) {
      int32_t op = 0, w = 0;
      if (staged) {
        const int k = nbr_rank(s_nbr, cb - c0, ce - c0, v.x);
        const int32_t pk = s_nop[k];
        shift += (pk >> 3) - (s_nop[cb - c0] >> 3);
        if (k < ce - c0 && s_nbr[k] == v.x) {
          op = pk & 7;
          w = s_w[k];
        }
      } else {
        const uint64_t key = uint64_t(r) * uint64_t(n) + uint64_t(uint32_t(v.x));
        const int k = change_rank(ch_key, cb, ce, key);
        shift += cnet[k] - cnet[cb];
        if (k < ce && ch_key[k] == key) {
          op = ch_op[k];
          w = ch_w[k];
        }
      }
      if (op == OP_DELETE) continue;
      if (op == OP_ADD) v.y += w;
      if (op == OP_REPLACE) v.y = w;
    }
    adj_new[t0 + i + shift] = v;
  }
}

// one wave per row: sum of w over entries whose endpoints share a label
__global__ void k_intra_weight(const int32_t* __restrict__ off,
                               const int2* __restrict__ adj,
                               const int32_t* __restrict__ C, int32_t n,
                               long long* I) {
  int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / WAVE;
  int64_t nwaves = int64_t(gridDim.x) * blockDim.x / WAVE;
  const int lane = lane_id();
  long long s = 0;
  for (int64_t row = wave; row < n; row += nwaves) {
    int32_t c = C[row];
    for (int32_t j = off[row] + lane; j < off[row + 1]; j += WAVE) {
      int2 e = adj[j];
      if (C[e.x] == c) s += e.y;
    }
  }
  block_add(s, I);
}

__global__ void __launch_bounds__(TPB)
    k_label_totals(const int32_t* __restrict__ k, const int32_t* __restrict__ C,
                   int32_t n, int32_t* a) {
  __shared__ AggLds agg;
  agg_init(agg);
  __syncthreads();
  // two rows per thread keep the 1024-slot table at most half full
  int64_t base = int64_t(blockIdx.x) * TPB * 2;
  for (int r = 0; r < 2; ++r) {
    int64_t u = base + int64_t(r) * TPB + threadIdx.x;
    if (u < n && k[u] != 0) agg_put(agg, C[u], k[u]);
  }
  __syncthreads();
  for (int s = threadIdx.x; s < AGG_SLOTS; s += blockDim.x) {
    int key = agg.keys[s];
    if (key != EMPTY_KEY && agg.vals[s] != 0) atomicAdd(&a[key], int32_t(agg.vals[s]));
  }
}

__global__ void k_sum_squares(const int32_t* __restrict__ a, int32_t n,
                              long long* S) {
  long long s = 0;
  GRID_STRIDE(i, n) {
    long long x = a[i];
    s += x * x;
  }
  block_add(s, S);
}

// Blocks [0, nb_intra) add the intra-community weight (one wave per row),
// the others the squares of the label totals.
__global__ void __launch_bounds__(TPB)
    k_modularity_terms(const int32_t* __restrict__ off, const int2* __restrict__ adj,
                       const int32_t* __restrict__ C, const int32_t* __restrict__ a, int32_t n,
                       int nb_intra, long long* I, long long* S) {
  long long s = 0;
  if (int(blockIdx.x) < nb_intra) {
    const int64_t nwaves = int64_t(nb_intra) * (TPB / WAVE);
    const int lane = lane_id();
    for (int64_t row = int64_t(blockIdx.x) * (TPB / WAVE) + threadIdx.x / WAVE; row < n;
         row += nwaves) {
      const int32_t c = C[row];
      for (int32_t j = off[row] + lane; j < off[row + 1]; j += WAVE) {
        const int2 e = adj[j];
        if (C[e.x] == c) s += e.y;
      }
    }
    block_add(s, I);
  } else {
    const int64_t nbs = int64_t(gridDim.x) - nb_intra;
    for (int64_t i = (int64_t(blockIdx.x) - nb_intra) * TPB + threadIdx.x; i < n; i += nbs * TPB) {
      const long long x = a[i];
      s += x * x;
    }
    block_add(s, S);
  }
}

}  // namespace

void modularity_terms(const int32_t* off, const int2* adj, const int32_t* C, const int32_t* a,
                      int32_t n, long long* I, long long* S, hipStream_t st) {
  if (n <= 0) return;
  const int nb_intra = grid_for(int64_t(n) * WAVE, TPB, 4096);
  const int nb_sq = grid_for(n, TPB, 2048);
  k_modularity_terms<<<nb_intra + nb_sq, TPB, 0, st>>>(off, adj, C, a, n, nb_intra, I, S);
  DC_LAUNCH_CHECK();
}

void validate_edges(const int32_t* u, const int32_t* v, const int32_t* w,
                    int64_t m, int32_t n, int32_t* flags, long long* wsum,
                    hipStream_t st) {
  if (m <= 0) return;
  k_validate<<<grid_for(m), TPB, 0, st>>>(u, v, w, m, n, flags, wsum);
  DC_LAUNCH_CHECK();
}

void make_directed(const int32_t* u, const int32_t* v, const int32_t* w,
                   int64_t m, int32_t n, uint64_t* keys, uint32_t* vals,
                   hipStream_t st) {
  if (m <= 0) return;
  k_make_directed<<<grid_for(m), TPB, 0, st>>>(u, v, w, m, n, keys, vals);
  DC_LAUNCH_CHECK();
}

void run_heads(const uint64_t* keys, int64_t m, int32_t* flag, hipStream_t st) {
  if (m <= 0) return;
  k_run_heads<<<grid_for(m), TPB, 0, st>>>(keys, m, flag);
  DC_LAUNCH_CHECK();
}

void reduce_runs(const uint64_t* keys, const uint32_t* vals,
                 const int32_t* wsrc, const int32_t* pos, int64_t m,
                 uint64_t* out_key, int32_t* out_w, hipStream_t st) {
  if (m <= 0) return;
  k_reduce_runs<<<grid_for(m), TPB, 0, st>>>(keys, vals, wsrc, pos, m, out_key, out_w);
  DC_LAUNCH_CHECK();
}

void row_bounds(const uint64_t* keys, int64_t m, int32_t n, int32_t* row_ptr,
                hipStream_t st) {
  k_row_bounds<<<grid_for(m + 1), TPB, 0, st>>>(keys, m, n, row_ptr);
  DC_LAUNCH_CHECK();
}

void keys_to_adj(const uint64_t* keys, const int32_t* w, int64_t m, int32_t n,
                 int2* adj, hipStream_t st) {
  if (m <= 0) return;
  k_keys_to_adj<<<grid_for(m), TPB, 0, st>>>(keys, w, m, n, adj);
  DC_LAUNCH_CHECK();
}

void row_weight_sums(const int32_t* off, const int2* adj, int32_t n, int32_t* k,
                     hipStream_t st) {
  if (n <= 0) return;
  k_row_weight_sums<<<ceil_div(int64_t(n) * WAVE, TPB), TPB, 0, st>>>(off, adj, n, k);
  DC_LAUNCH_CHECK();
}

void batch_records(const int32_t* du, const int32_t* dv, int64_t nd, const int32_t* au,
                   const int32_t* av, int64_t na, int32_t n, uint64_t* keys, uint32_t* vals,
                   hipStream_t st) {
  if (nd + na <= 0) return;
  k_batch_records<<<grid_for(nd + na), TPB, 0, st>>>(du, dv, nd, au, av, na, n, keys, vals);
  DC_LAUNCH_CHECK();
}

void resolve_changes(const uint64_t* keys, const uint32_t* vals, const int32_t* pos, int64_t m,
                     const int32_t* nruns, const int32_t* ins_w, int32_t n, const int32_t* off,
                     const int2* adj, uint64_t* run_key, int32_t* run_w, int32_t* run_ndel,
                     uint64_t* ch_key, int32_t* ch_op, int32_t* ch_w, int32_t* ch_dk,
                     int32_t* dnet, int32_t* flags, long long* wsum, hipStream_t st) {
  if (m <= 0) return;
  void* zp[2] = {run_w, run_ndel};
  const int64_t zb[2] = {4 * m, 4 * m};
  zero_buffers(zp, zb, 2, st);
  k_run_accumulate<<<grid_for(m), TPB, 0, st>>>(keys, vals, pos, m, ins_w, run_key, run_w,
                                                run_ndel);
  DC_LAUNCH_CHECK();
  k_resolve_runs<<<grid_for(m), TPB, 0, st>>>(run_key, run_w, run_ndel, nruns, n, off, adj,
                                              ch_key, ch_op, ch_w, ch_dk, dnet, flags, wsum);
  DC_LAUNCH_CHECK();
}

void row_changes(const int32_t* cptr, const int32_t* ch_op, const int32_t* ch_dk,
                 const int32_t* off, int32_t n, int32_t* new_deg, int32_t* k,
                 const int32_t* C, int32_t* a, int32_t* tile_row, hipStream_t st) {
  if (n <= 0) return;
  k_row_changes<<<grid_for(n, RC_TPB, RC_BLOCKS), RC_TPB, 0, st>>>(cptr, ch_op, ch_dk, off, n, new_deg, k,
                                                       C, a, tile_row);
  DC_LAUNCH_CHECK();
}

void merge_rows(const int32_t* off_old, const int2* adj_old, int64_t nnz_old,
                const int32_t* off_new, int2* adj_new, int32_t n, const int32_t* cptr,
                const int32_t* tile_row, const uint64_t* ch_key, const int32_t* ch_op,
                const int32_t* ch_w, const int32_t* cnet, int64_t nch, hipStream_t st) {
  if (n <= 0) return;
  const int64_t ntiles = ceil_div(nnz_old, MERGE_TILE);
  const int nib = nch > 0 ? grid_for(nch, TPB, 1024) : 0;
  if (ntiles + nib == 0) return;
  k_merge_tiles<<<int(ntiles + nib), TPB, 0, st>>>(off_old, adj_old, nnz_old, off_new, adj_new,
                                                   n, cptr, tile_row, ch_key, ch_op, ch_w, cnet,
                                                   nch, nib);
  DC_LAUNCH_CHECK();
}

void intra_weight(const int32_t* off, const int2* adj, const int32_t* C,
                  int32_t n, long long* I, hipStream_t st) {
  if (n <= 0) return;
  k_intra_weight<<<grid_for(int64_t(n) * WAVE, TPB, 4096), TPB, 0, st>>>(off, adj, C, n, I);
  DC_LAUNCH_CHECK();
}

void label_totals(const int32_t* k, const int32_t* C, int32_t n, int32_t* a,
                  hipStream_t st) {
  if (n <= 0) return;
  k_label_totals<<<ceil_div(n, TPB * 2), TPB, 0, st>>>(k, C, n, a);
  DC_LAUNCH_CHECK();
}

void sum_squares(const int32_t* a, int32_t n, long long* S, hipStream_t st) {
  if (n <= 0) return;
  k_sum_squares<<<grid_for(n), TPB, 0, st>>>(a, n, S);
  DC_LAUNCH_CHECK();
}

}  // namespace dc
