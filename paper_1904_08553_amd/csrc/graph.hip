// graph.hip -- the dynamic graph G_t (Sec. 3.1): CSR construction, batch
// validation, and the sorted merge of a batch of additions and deletions into
// the next CSR (a streaming pass, one wave per row).
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
  if (w) block_add(s, wsum);
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

__global__ void k_row_bounds(const uint64_t* __restrict__ keys, int64_t m,
                             int32_t n, int32_t* row_ptr) {
  GRID_STRIDE(uu, int64_t(n) + 1) {
    uint64_t target = uint64_t(uu) * uint64_t(n);
    int64_t lo = 0, hi = m;
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if (keys[mid] < target)
        lo = mid + 1;
      else
        hi = mid;
    }
    row_ptr[uu] = int32_t(lo);
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
                               int32_t* is_del, int32_t* is_new, int32_t* flags,
                               long long* wsum) {
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
    is_del[r] = op == OP_DELETE ? 1 : 0;
    is_new[r] = op == OP_NEW ? 1 : 0;
  }
  block_or(f, flags);
  block_add(s, wsum);
}


// Thread per row: new degree, k += the row's weight change, and the label
// totals a[C(u)] += the same change.  A block walks many rows and sums the
// label changes in its LDS table first, so a large community receives one
// update per block instead of one per row (same-address atomics serialise).
__global__ void __launch_bounds__(TPB)
    k_row_changes(const int32_t* __restrict__ cptr,
                  const int32_t* __restrict__ ch_op,
                  const int32_t* __restrict__ ch_dk,
                  const int32_t* __restrict__ off, int32_t n, int32_t* new_deg,
                  int32_t* k, const int32_t* __restrict__ C, int32_t* a) {
  __shared__ AggLds agg;
  agg_init(agg);
  __syncthreads();
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t u = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; u < n; u += stride) {
    const int32_t b = cptr[u], e = cptr[u + 1];
    int32_t dd = 0, dk = 0;
    for (int32_t q = b; q < e; ++q) {
      const int32_t op = ch_op[q];
      dd += op == OP_NEW ? 1 : (op == OP_DELETE ? -1 : 0);
      dk += ch_dk[q];
    }
    new_deg[u] = off[u + 1] - off[u] + dd;
    if (dk != 0) {
      k[u] += dk;
      const int c = C[u];
      if (!agg_try(agg, c, dk)) atomicAdd(&a[c], dk);
    }
  }
  __syncthreads();
  for (int s = threadIdx.x; s < AGG_SLOTS; s += blockDim.x) {
    const int key = agg.keys[s];
    if (key != EMPTY_KEY && agg.vals[s] != 0) atomicAdd(&a[key], int32_t(agg.vals[s]));
  }
}

constexpr int MC_ROWS = 4;  // unchanged rows a wave copies per round

// Untouched rows move as a block: entry e of row r goes to
// e + off_new[r] - off_old[r].  A wave takes 64 consecutive rows: one
// coalesced load brings each row's bounds, shift and changed-flag into a
// lane, then the wave copies the unchanged rows MC_ROWS at a time with
// contiguous reads and writes.
__global__ void __launch_bounds__(TPB)
    k_merge_copy(const int32_t* __restrict__ off_old, const int2* __restrict__ adj_old,
                 const int32_t* __restrict__ off_new, int2* adj_new, int32_t n,
                 const int32_t* __restrict__ cptr) {
  const int64_t nbatch = ceil_div(n, WAVE);
  const int64_t nwaves = int64_t(gridDim.x) * (TPB / WAVE);
  const int lane = lane_id();
  for (int64_t bt = int64_t(blockIdx.x) * (TPB / WAVE) + threadIdx.x / WAVE; bt < nbatch;
       bt += nwaves) {
    const int64_t r = bt * WAVE + lane;
    int beg = 0, end = 0, shift = 0, skip = 1;
    if (r < n) {
      beg = off_old[r];
      end = off_old[r + 1];
      shift = off_new[r] - beg;
      skip = cptr[r] != cptr[r + 1];
    }
    // rows to copy, in lane order, MC_ROWS per round: the rounds' loads are
    // issued before their stores
    uint64_t todo = __ballot(!skip && end > beg);
    while (todo) {
      int b[MC_ROWS], e[MC_ROWS], sh[MC_ROWS];
      int longest = 0;
#pragma unroll
      for (int k = 0; k < MC_ROWS; ++k) {
        b[k] = e[k] = sh[k] = 0;
        if (todo) {
          const int l = __ffsll((unsigned long long)todo) - 1;
          todo &= todo - 1;
          b[k] = __builtin_amdgcn_readlane(beg, l);
          e[k] = __builtin_amdgcn_readlane(end, l);
          sh[k] = __builtin_amdgcn_readlane(shift, l);
          longest = e[k] - b[k] > longest ? e[k] - b[k] : longest;
        }
      }
      for (int o = 0; o < longest; o += WAVE) {
        int2 v[MC_ROWS];
#pragma unroll
        for (int k = 0; k < MC_ROWS; ++k) {
          const int q = b[k] + o + lane;
          v[k] = q < e[k] ? adj_old[q] : make_int2(0, 0);
        }
#pragma unroll
        for (int k = 0; k < MC_ROWS; ++k) {
          const int q = b[k] + o + lane;
          if (q < e[k]) adj_new[q + sh[k]] = v[k];
        }
      }
    }
  }
}

// Rows with changes: one wave per row.  For a row with few changes relative
// to its length the changes (sorted by neighbour) sit one per lane, and the
// number of deletions and insertions before a neighbour id comes from a
// register loop instead of searches in memory; other rows use searches.
// Long rows with many changes: every old entry and every insertion finds
// its place by binary search (changes with a smaller neighbour id, counted
// through the prefix sums of the DELETE / NEW flags).
__device__ void merge_row_search(int32_t row, int32_t n, const int2* __restrict__ adj_old,
                                 int32_t ob, int32_t oe, int32_t nb, int32_t cb, int32_t ce,
                                 int2* adj_new, const uint64_t* __restrict__ ch_key,
                                 const int32_t* __restrict__ ch_op,
                                 const int32_t* __restrict__ ch_w,
                                 const int32_t* __restrict__ cum_del,
                                 const int32_t* __restrict__ cum_new) {
  const int lane = lane_id();
  const uint64_t base = uint64_t(row) * uint64_t(n);
  const int32_t del0 = cum_del[cb], new0 = cum_new[cb];
  for (int32_t j = lane; j < oe - ob; j += WAVE) {
    int2 e = adj_old[ob + j];
    int32_t lo = cb, hi = ce;
    while (lo < hi) {
      const int32_t mid = (lo + hi) >> 1;
      if (int32_t(ch_key[mid] - base) < e.x)
        lo = mid + 1;
      else
        hi = mid;
    }
    const int32_t shift = (cum_new[lo] - new0) - (cum_del[lo] - del0);
    if (lo < ce && int32_t(ch_key[lo] - base) == e.x) {
      const int32_t op = ch_op[lo];
      if (op == OP_DELETE) continue;
      if (op == OP_ADD) e.y += ch_w[lo];
      if (op == OP_REPLACE) e.y = ch_w[lo];
    }
    adj_new[nb + j + shift] = e;
  }
  for (int32_t q = cb + lane; q < ce; q += WAVE) {
    if (ch_op[q] != OP_NEW) continue;
    const int32_t c = int32_t(ch_key[q] - base);
    const int32_t pos = find_in_row(adj_old, ob, oe, c) - ob;
    const int32_t shift = (cum_new[q] - new0) - (cum_del[q] - del0);
    adj_new[nb + pos + shift] = make_int2(c, ch_w[q]);
  }
}

constexpr int WROW_CH = 4;                 // row chunks a wave holds in registers
constexpr int BIG_ROW = 1024;              // longer rows are merged by a block
constexpr int MERGE_ROWS = 2;              // rows a wave merges per iteration
constexpr int BIG_CHANGES = 4096;          // changes staged in LDS per big row
constexpr int BIG_SEG = BIG_CHANGES / TPB; // histogram bins per thread in the scan
constexpr int BIG_U = 4;                   // row chunks per load round of a block

// Long changed rows (more than BIG_ROW entries or more than WAVE changes):
// one block per row.  The row's change neighbours and the shift before each
// change (insertions minus deletions before it) are staged in LDS; each old
// entry finds its rank lo among the changes by a binary search on chip and
// counts itself in bin lo of an LDS histogram.  An insertion at change k
// lands after the old entries with a smaller neighbour, which are exactly
// those of rank <= k: the histogram's prefix sum at k.
__global__ void __launch_bounds__(TPB)
    k_merge_big(const int32_t* __restrict__ big,
                const int32_t* __restrict__ off_old, const int2* __restrict__ adj_old,
                const int32_t* __restrict__ off_new, int2* adj_new, int32_t n,
                const int32_t* __restrict__ cptr, const uint64_t* __restrict__ ch_key,
                const int32_t* __restrict__ ch_op, const int32_t* __restrict__ ch_w,
                const int32_t* __restrict__ cum_del, const int32_t* __restrict__ cum_new) {
  __shared__ int ldst[BIG_CHANGES];
  __shared__ int lsh[BIG_CHANGES + 1];
  __shared__ int hcnt[BIG_CHANGES + 1];
  __shared__ int part[TPB];
  const int64_t nrows = big[0];  // rows listed from big[1]
  for (int64_t p = blockIdx.x; p < nrows; p += gridDim.x) {
    const int32_t row = big[1 + p];
    const int32_t ob = off_old[row], oe = off_old[row + 1];
    const int32_t nb = off_new[row], cb = cptr[row], ce = cptr[row + 1];
    const int32_t nchg = ce - cb;
    if (nchg > BIG_CHANGES) {
      if (threadIdx.x < WAVE)
        merge_row_search(row, n, adj_old, ob, oe, nb, cb, ce, adj_new, ch_key, ch_op, ch_w,
                         cum_del, cum_new);
      __syncthreads();
      continue;
    }
    const uint64_t base = uint64_t(row) * uint64_t(n);
    const int32_t del0 = cum_del[cb], new0 = cum_new[cb];
    for (int k = threadIdx.x; k <= nchg; k += TPB) {
      if (k < nchg) ldst[k] = int32_t(ch_key[cb + k] - base);
      lsh[k] = (cum_new[cb + k] - new0) - (cum_del[cb + k] - del0);
      hcnt[k] = 0;
    }
    __syncthreads();
    const int32_t deg = oe - ob;
    for (int32_t j0 = threadIdx.x; j0 < deg; j0 += BIG_U * TPB) {
      int2 e[BIG_U];
#pragma unroll
      for (int u = 0; u < BIG_U; ++u) {
        const int32_t j = j0 + u * TPB;
        e[u] = j < deg ? adj_old[ob + j] : make_int2(0, 0);
      }
#pragma unroll
      for (int u = 0; u < BIG_U; ++u) {
        const int32_t j = j0 + u * TPB;
        if (j >= deg) continue;
        int lo = 0, hi = nchg;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (ldst[mid] < e[u].x)
            lo = mid + 1;
          else
            hi = mid;
        }
        atomicAdd(&hcnt[lo], 1);
        if (lo < nchg && ldst[lo] == e[u].x) {
          const int32_t op = ch_op[cb + lo];
          if (op == OP_DELETE) continue;
          if (op == OP_ADD) e[u].y += ch_w[cb + lo];
          if (op == OP_REPLACE) e[u].y = ch_w[cb + lo];
        }
        adj_new[nb + j + lsh[lo]] = e[u];
      }
    }
    __syncthreads();
    // inclusive prefix sums of hcnt: per-thread segments of BIG_SEG bins,
    // then a scan of the TPB segment totals
    const int sb = int(threadIdx.x) * BIG_SEG;
    int tot = 0;
    for (int q = 0; q < BIG_SEG; ++q)
      if (sb + q <= nchg) tot += hcnt[sb + q];
    part[threadIdx.x] = tot;
    __syncthreads();
    for (int o = 1; o < TPB; o <<= 1) {
      const int add = int(threadIdx.x) >= o ? part[threadIdx.x - o] : 0;
      __syncthreads();
      part[threadIdx.x] += add;
      __syncthreads();
    }
    for (int k = threadIdx.x; k < nchg; k += TPB) {
      if (ch_op[cb + k] != OP_NEW) continue;
      const int seg = k / BIG_SEG;
      int less = seg > 0 ? part[seg - 1] : 0;
      for (int q = seg * BIG_SEG; q <= k; ++q) less += hcnt[q];
      adj_new[nb + less + lsh[k]] = make_int2(ldst[k], ch_w[cb + k]);
    }
    __syncthreads();
  }
}

// Changed rows of at most BIG_ROW entries and at most WAVE changes: one
// wave per row, everything in registers.  The row's entries sit in windows
// of WROW_CH chunks of one per lane and its changes (sorted by neighbour) one
// per lane; a loop over the changes, each broadcast by readlane, gives every
// old entry its shift (insertions minus deletions before it) and its fate,
// and every change the number of old entries with a smaller neighbour (one
// ballot per chunk), which places the insertions.  A wave takes
// MERGE_ROWS rows per iteration and issues all their loads before it waits
// on any.
// Other rows are listed for k_merge_big.
struct MergeRow {
  int32_t ob, deg, nb, nchg;
  bool live;
  int dst, op, cw;
  int2 e[WROW_CH];
};

__device__ __forceinline__ void merge_head(MergeRow& r, int32_t row, bool have,
                                           const int32_t* __restrict__ off_old,
                                           const int32_t* __restrict__ off_new,
                                           const int32_t* __restrict__ cptr, int32_t* cb_out) {
  r.live = false;
  r.ob = r.deg = r.nb = r.nchg = 0;
  *cb_out = 0;
  if (!have) return;
  const int32_t ob = off_old[row], oe = off_old[row + 1], nb = off_new[row];
  const int32_t cb = cptr[row], ce = cptr[row + 1];
  r.ob = ob;
  r.deg = oe - ob;
  r.nb = nb;
  r.nchg = ce - cb;
  r.live = true;
  *cb_out = cb;
}

__device__ __forceinline__ void merge_load(MergeRow& r, int32_t row, int32_t cb, int32_t n,
                                           const int2* __restrict__ adj_old,
                                           const uint64_t* __restrict__ ch_key,
                                           const int32_t* __restrict__ ch_op,
                                           const int32_t* __restrict__ ch_w, int lane) {
  const bool hq = r.live && lane < r.nchg;
  const uint64_t base = uint64_t(row) * uint64_t(n);
  r.dst = hq ? int32_t(ch_key[cb + lane] - base) : 0x7fffffff;
  r.op = hq ? ch_op[cb + lane] : 0;
  r.cw = hq ? ch_w[cb + lane] : 0;
#pragma unroll
  for (int u = 0; u < WROW_CH; ++u) {
    const int32_t j = u * WAVE + lane;
    r.e[u] = r.live && j < r.deg ? adj_old[r.ob + j] : make_int2(0x7fffffff, 0);
  }
}

// The row is walked in windows of WROW_CH chunks: window 0 was loaded by
// merge_load, later windows are loaded here.
__device__ __forceinline__ void merge_finish(MergeRow& r, const int2* __restrict__ adj_old,
                                             int2* adj_new, int lane, uint64_t lt) {
  if (!r.live) return;  // uniform
  const int nck = (r.deg + WAVE - 1) / WAVE;
  int less = 0;
  for (int w0 = 0; w0 == 0 || w0 < nck; w0 += WROW_CH) {
    if (w0 > 0) {
#pragma unroll
      for (int u = 0; u < WROW_CH; ++u) {
        const int32_t j = (w0 + u) * WAVE + lane;
        r.e[u] = j < r.deg ? adj_old[r.ob + j] : make_int2(0x7fffffff, 0);
      }
    }
    int shift[WROW_CH];
    bool drop[WROW_CH];
#pragma unroll
    for (int u = 0; u < WROW_CH; ++u) {
      shift[u] = 0;
      drop[u] = false;
    }
    for (int k = 0; k < r.nchg; ++k) {
      const int dk = __builtin_amdgcn_readlane(r.dst, k);
      const int ok = __builtin_amdgcn_readlane(r.op, k);
      const int wk = __builtin_amdgcn_readlane(r.cw, k);
      const int dsh = ok == OP_NEW ? 1 : (ok == OP_DELETE ? -1 : 0);
      int cnt = 0;
#pragma unroll
      for (int u = 0; u < WROW_CH; ++u) {
        if (w0 + u >= nck) break;
        if (dk < r.e[u].x) {
          shift[u] += dsh;
        } else if (dk == r.e[u].x) {
          if (ok == OP_DELETE) drop[u] = true;
          if (ok == OP_ADD) r.e[u].y += wk;
          if (ok == OP_REPLACE) r.e[u].y = wk;
        }
        cnt += __popcll(__ballot(r.e[u].x < dk));
      }
      if (lane == k) less += cnt;
    }
#pragma unroll
    for (int u = 0; u < WROW_CH; ++u) {
      const int32_t j = (w0 + u) * WAVE + lane;
      if (w0 + u < nck && j < r.deg && !drop[u]) adj_new[r.nb + j + shift[u]] = r.e[u];
    }
  }
  // insertion k: after `less` old entries, minus the deletions and plus
  // the insertions among the changes before it
  const bool hq = lane < r.nchg;
  const bool isnew = hq && r.op == OP_NEW;
  const uint64_t mnew = __ballot(isnew), mdel = __ballot(hq && r.op == OP_DELETE);
  if (isnew)
    adj_new[r.nb + less + __popcll(mnew & lt) - __popcll(mdel & lt)] = make_int2(r.dst, r.cw);
}

__global__ void __launch_bounds__(TPB)
    k_merge_changed(const int32_t* __restrict__ rows, const int32_t* nrows_dev,
                    const int32_t* __restrict__ off_old, const int2* __restrict__ adj_old,
                    const int32_t* __restrict__ off_new, int2* adj_new, int32_t n,
                    const int32_t* __restrict__ cptr, const uint64_t* __restrict__ ch_key,
                    const int32_t* __restrict__ ch_op, const int32_t* __restrict__ ch_w,
                    int32_t* big) {
  const int64_t nrows = *nrows_dev;
  const int64_t nwaves = int64_t(gridDim.x) * (blockDim.x / WAVE);
  const int lane = lane_id();
  const uint64_t lt = (uint64_t(1) << lane) - 1;
  for (int64_t p = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / WAVE; p < nrows;
       p += MERGE_ROWS * nwaves) {
    MergeRow M[MERGE_ROWS];
    int32_t row[MERGE_ROWS], cb[MERGE_ROWS];
#pragma unroll
    for (int r = 0; r < MERGE_ROWS; ++r) {
      const bool h = p + r * nwaves < nrows;
      row[r] = h ? rows[p + r * nwaves] : 0;
      merge_head(M[r], row[r], h, off_old, off_new, cptr, &cb[r]);
    }
#pragma unroll
    for (int r = 0; r < MERGE_ROWS; ++r) {
      if (M[r].live && (M[r].deg > BIG_ROW || M[r].nchg > WAVE)) {
        if (lane == 0) big[1 + atomicAdd(&big[0], 1)] = row[r];
        M[r].live = false;
      }
    }
#pragma unroll
    for (int r = 0; r < MERGE_ROWS; ++r)
      merge_load(M[r], row[r], cb[r], n, adj_old, ch_key, ch_op, ch_w, lane);
#pragma unroll
    for (int r = 0; r < MERGE_ROWS; ++r) merge_finish(M[r], adj_old, adj_new, lane, lt);
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

}  // namespace

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
  k_row_bounds<<<grid_for(int64_t(n) + 1), TPB, 0, st>>>(keys, m, n, row_ptr);
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
                     int32_t* is_del, int32_t* is_new, int32_t* flags, long long* wsum,
                     hipStream_t st) {
  if (m <= 0) return;
  fill_i32(run_w, 0, m, st);
  fill_i32(run_ndel, 0, m, st);
  k_run_accumulate<<<grid_for(m), TPB, 0, st>>>(keys, vals, pos, m, ins_w, run_key, run_w,
                                                run_ndel);
  DC_LAUNCH_CHECK();
  k_resolve_runs<<<grid_for(m), TPB, 0, st>>>(run_key, run_w, run_ndel, nruns, n, off, adj,
                                              ch_key, ch_op, ch_w, ch_dk, is_del, is_new, flags,
                                              wsum);
  DC_LAUNCH_CHECK();
}

void row_changes(const int32_t* cptr, const int32_t* ch_op, const int32_t* ch_dk,
                 const int32_t* off, int32_t n, int32_t* new_deg, int32_t* k,
                 const int32_t* C, int32_t* a, hipStream_t st) {
  if (n <= 0) return;
  k_row_changes<<<grid_for(n, TPB, 512), TPB, 0, st>>>(cptr, ch_op, ch_dk, off, n, new_deg, k,
                                                       C, a);
  DC_LAUNCH_CHECK();
}

void merge_rows(const int32_t* off_old, const int2* adj_old, int64_t nnz_old,
                const int32_t* off_new, int2* adj_new, int32_t n, const int32_t* cptr,
                const int32_t* rows, const int32_t* nrows_dev, int64_t nrows_max,
                const uint64_t* ch_key, const int32_t* ch_op, const int32_t* ch_w,
                const int32_t* cum_del, const int32_t* cum_new, int32_t* big,
                hipStream_t st) {
  if (n <= 0) return;
  if (nnz_old > 0) {
    k_merge_copy<<<grid_for(ceil_div(n, WAVE) * WAVE, TPB, 16384), TPB, 0, st>>>(
        off_old, adj_old, off_new, adj_new, n, cptr);
    DC_LAUNCH_CHECK();
  }
  if (nrows_max > 0) {
    fill_i32(big, 0, 1, st);
    k_merge_changed<<<grid_for(nrows_max * WAVE, TPB, 16384), TPB, 0, st>>>(
        rows, nrows_dev, off_old, adj_old, off_new, adj_new, n, cptr, ch_key, ch_op, ch_w, big);
    DC_LAUNCH_CHECK();
    const int nbig = int(nrows_max < 2048 ? nrows_max : 2048);
    k_merge_big<<<nbig, TPB, 0, st>>>(big, off_old, adj_old, off_new, adj_new, n, cptr, ch_key,
                                      ch_op, ch_w, cum_del, cum_new);
    DC_LAUNCH_CHECK();
  }
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
