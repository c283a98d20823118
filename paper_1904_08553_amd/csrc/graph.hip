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
  // combine per wave, one atomic per wave
  for (int o = WAVE / 2; o > 0; o >>= 1) f |= __shfl_xor(f, o, WAVE);
  s = wave_sum(s);
  if (lane_id() == 0) {
    if (f) atomicOr(flags, f);
    if (w && s) atomicAdd((unsigned long long*)wsum, (unsigned long long)s);
  }
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

__global__ void k_make_canonical(const int32_t* __restrict__ u,
                                 const int32_t* __restrict__ v, int64_t m,
                                 int32_t n, uint64_t* keys, uint32_t* vals) {
  GRID_STRIDE(e, m) {
    uint32_t a = uint32_t(u[e]), b = uint32_t(v[e]);
    uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
    keys[e] = lo * uint64_t(n) + hi;
    vals[e] = uint32_t(e);
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

__global__ void k_detect_dups(const uint64_t* __restrict__ keys, int64_t m,
                              int32_t* flags) {
  int32_t f = 0;
  GRID_STRIDE(i, m) {
    if (i > 0 && keys[i] == keys[i - 1]) f = F_DUP;
  }
  for (int o = WAVE / 2; o > 0; o >>= 1) f |= __shfl_xor(f, o, WAVE);
  if (lane_id() == 0 && f) atomicOr(flags, f);
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

__global__ void k_lookup_deleted(const uint64_t* __restrict__ keys, int64_t m,
                                 int32_t n, const int32_t* __restrict__ off,
                                 const int2* __restrict__ adj, int32_t* w_old,
                                 int32_t* flags, long long* wsum) {
  int32_t f = 0;
  long long s = 0;
  GRID_STRIDE(i, m) {
    uint64_t key = keys[i];
    uint64_t lo = key / uint64_t(n), hi = key % uint64_t(n);
    int32_t wo = 0;
    if (lo < uint64_t(n) && hi < uint64_t(n)) {
      int32_t b = off[lo], e = off[lo + 1];
      int32_t p = find_in_row(adj, b, e, int32_t(hi));
      if (p < e && adj[p].x == int32_t(hi)) wo = adj[p].y;
    }
    if (wo == 0) f |= F_NO_EDGE;
    w_old[i] = wo;
    s += wo;
  }
  for (int o = WAVE / 2; o > 0; o >>= 1) f |= __shfl_xor(f, o, WAVE);
  s = wave_sum(s);
  if (lane_id() == 0) {
    if (f) atomicOr(flags, f);
    if (s) atomicAdd((unsigned long long*)wsum, (unsigned long long)s);
  }
}

__global__ void k_make_change_records(const uint64_t* __restrict__ del_keys,
                                      int64_t nd,
                                      const uint64_t* __restrict__ ins_keys,
                                      int64_t na, int32_t n, uint64_t* rkeys,
                                      uint32_t* rvals) {
  GRID_STRIDE(i, nd + na) {
    bool is_del = i < nd;
    int64_t j = is_del ? i : i - nd;
    uint64_t key = is_del ? del_keys[j] : ins_keys[j];
    uint64_t lo = key / uint64_t(n), hi = key % uint64_t(n);
    uint32_t val = (uint32_t(j) << 1) | (is_del ? 0u : 1u);
    rkeys[2 * i] = lo * uint64_t(n) + hi;
    rkeys[2 * i + 1] = hi * uint64_t(n) + lo;
    rvals[2 * i] = val;
    rvals[2 * i + 1] = val;
  }
}

__global__ void k_combine_changes(
    const uint64_t* __restrict__ rkeys, const uint32_t* __restrict__ rvals,
    int64_t nr, const int32_t* __restrict__ heads,
    const int32_t* __restrict__ pos, int32_t n,
    const int32_t* __restrict__ del_w_old, const int32_t* __restrict__ ins_w,
    const int32_t* __restrict__ off, const int2* __restrict__ adj,
    uint64_t* ch_key, int32_t* ch_op, int32_t* ch_w, int32_t* ch_dk,
    int32_t* is_del, int32_t* is_new) {
  GRID_STRIDE(i, nr) {
    if (!heads[i]) continue;
    uint64_t key = rkeys[i];
    int32_t w_del = -1, w_ins = -1;
    for (int64_t j = i; j < nr && j < i + 2 && rkeys[j] == key; ++j) {
      uint32_t v = rvals[j];
      if (v & 1u)
        w_ins = ins_w[v >> 1];
      else
        w_del = del_w_old[v >> 1];
    }
    int32_t op, w, dk;
    if (w_del >= 0 && w_ins >= 0) {
      op = OP_REPLACE;
      w = w_ins;
      dk = w_ins - w_del;
    } else if (w_del >= 0) {
      op = OP_DELETE;
      w = 0;
      dk = -w_del;
    } else {
      uint64_t src = key / uint64_t(n), dst = key % uint64_t(n);
      int32_t b = off[src], e = off[src + 1];
      int32_t p = find_in_row(adj, b, e, int32_t(dst));
      bool exists = p < e && adj[p].x == int32_t(dst);
      op = exists ? OP_ADD : OP_NEW;
      w = w_ins;
      dk = w_ins;
    }
    int32_t r = pos[i];
    ch_key[r] = key;
    ch_op[r] = op;
    ch_w[r] = w;
    ch_dk[r] = dk;
    is_del[r] = op == OP_DELETE ? 1 : 0;
    is_new[r] = op == OP_NEW ? 1 : 0;
  }
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

// Untouched rows move as a block: entry e of row r goes to
// e + off_new[r] - off_old[r].  A wave takes 64 consecutive rows: one
// coalesced load brings each row's bounds, shift and changed-flag into a
// lane, then the wave copies the rows one after another with contiguous
// reads and writes.
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
    // rows to copy, in lane order
    for (uint64_t todo = __ballot(!skip && end > beg); todo; todo &= todo - 1) {
      const int l = __ffsll((unsigned long long)todo) - 1;
      const int b = __builtin_amdgcn_readlane(beg, l);
      const int e = __builtin_amdgcn_readlane(end, l);
      const int sh = __builtin_amdgcn_readlane(shift, l);
      for (int q = b + lane; q < e; q += WAVE) adj_new[q + sh] = adj_old[q];
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

constexpr int BIG_ROW = 1024;       // rows longer than this are merged by a block
constexpr int BIG_CHANGES = 4096;   // changes staged in LDS per big row

// Long changed rows: one block per row.  The row's change neighbours and the
// cumulative shift before each change are staged in LDS, so every old entry
// finds its place by a binary search on chip.
__global__ void __launch_bounds__(TPB)
    k_merge_big(const int32_t* __restrict__ big,
                const int32_t* __restrict__ off_old, const int2* __restrict__ adj_old,
                const int32_t* __restrict__ off_new, int2* adj_new, int32_t n,
                const int32_t* __restrict__ cptr, const uint64_t* __restrict__ ch_key,
                const int32_t* __restrict__ ch_op, const int32_t* __restrict__ ch_w,
                const int32_t* __restrict__ cum_del, const int32_t* __restrict__ cum_new) {
  __shared__ int ldst[BIG_CHANGES];
  __shared__ int lsh[BIG_CHANGES + 1];
  const int64_t nrows = big[0];  // rows longer than BIG_ROW, listed from big[1]
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
    }
    __syncthreads();
    for (int32_t j = threadIdx.x; j < oe - ob; j += TPB) {
      int2 e = adj_old[ob + j];
      int lo = 0, hi = nchg;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ldst[mid] < e.x)
          lo = mid + 1;
        else
          hi = mid;
      }
      if (lo < nchg && ldst[lo] == e.x) {
        const int32_t op = ch_op[cb + lo];
        if (op == OP_DELETE) continue;
        if (op == OP_ADD) e.y += ch_w[cb + lo];
        if (op == OP_REPLACE) e.y = ch_w[cb + lo];
      }
      adj_new[nb + j + lsh[lo]] = e;
    }
    for (int k = threadIdx.x; k < nchg; k += TPB) {
      if (ch_op[cb + k] != OP_NEW) continue;
      const int32_t pos = find_in_row(adj_old, ob, oe, ldst[k]) - ob;
      adj_new[nb + pos + lsh[k]] = make_int2(ldst[k], ch_w[cb + k]);
    }
    __syncthreads();
  }
}

__global__ void k_merge_changed(const int32_t* __restrict__ rows, const int32_t* nrows_dev,
                                const int32_t* __restrict__ off_old,
                                const int2* __restrict__ adj_old,
                                const int32_t* __restrict__ off_new, int2* adj_new, int32_t n,
                                const int32_t* __restrict__ cptr,
                                const uint64_t* __restrict__ ch_key,
                                const int32_t* __restrict__ ch_op,
                                const int32_t* __restrict__ ch_w,
                                const int32_t* __restrict__ cum_del,
                                const int32_t* __restrict__ cum_new, int32_t* big) {
  const int64_t nrows = *nrows_dev;
  const int64_t nwaves = int64_t(gridDim.x) * (blockDim.x / WAVE);
  const int lane = lane_id();
  for (int64_t p = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / WAVE; p < nrows;
       p += nwaves) {
    const int32_t row = rows[p];
    const int32_t ob = off_old[row], oe = off_old[row + 1], nb = off_new[row];
    const int32_t cb = cptr[row], ce = cptr[row + 1];
    if (oe - ob > BIG_ROW) {  // merged by k_merge_big
      if (lane == 0) big[1 + atomicAdd(&big[0], 1)] = row;
      continue;
    }
    if (int64_t(ce - cb) * ceil_div(oe - ob + 1, WAVE) > WAVE) {
      merge_row_search(row, n, adj_old, ob, oe, nb, cb, ce, adj_new, ch_key, ch_op, ch_w,
                       cum_del, cum_new);
      continue;
    }
    const uint64_t base = uint64_t(row) * uint64_t(n);
    // old entries: final position = nb + j - (#DELETE with dst < col) + (#NEW with dst < col)
    for (int32_t j0 = 0; j0 < oe - ob; j0 += WAVE) {
      const int32_t j = j0 + lane;
      const bool live = j < oe - ob;
      int2 e = live ? adj_old[ob + j] : make_int2(0x7fffffff, 0);
      int shift = 0;
      bool drop = false;
      for (int32_t w0 = cb; w0 < ce; w0 += WAVE) {
        const int32_t q = w0 + lane;
        const bool hq = q < ce;
        const int dst = hq ? int32_t(ch_key[q] - base) : 0x7fffffff;
        const int op = hq ? ch_op[q] : 0;
        const int cw = hq ? ch_w[q] : 0;
        const int nw = ce - w0 < WAVE ? ce - w0 : WAVE;
        for (int k = 0; k < nw; ++k) {
          const int dk = __builtin_amdgcn_readlane(dst, k);
          const int ok = __builtin_amdgcn_readlane(op, k);
          if (dk < e.x) {
            shift += ok == OP_NEW ? 1 : (ok == OP_DELETE ? -1 : 0);
          } else if (dk == e.x) {
            const int wk = __builtin_amdgcn_readlane(cw, k);
            if (ok == OP_DELETE) drop = true;
            if (ok == OP_ADD) e.y += wk;
            if (ok == OP_REPLACE) e.y = wk;
          }
        }
      }
      if (live && !drop) adj_new[nb + j + shift] = e;
    }
    // new entries: position = nb + (#old with col < dst) - (#DELETE before) + (#NEW before)
    for (int32_t w0 = cb; w0 < ce; w0 += WAVE) {
      const int32_t q = w0 + lane;
      const bool hq = q < ce && ch_op[q] == OP_NEW;
      const int dst = q < ce ? int32_t(ch_key[q] - base) : 0x7fffffff;
      const int nw0 = ce - w0 < WAVE ? ce - w0 : WAVE;
      int pos = 0;
      for (int32_t j0 = 0; j0 < oe - ob; j0 += WAVE) {
        const int col = j0 + lane < oe - ob ? adj_old[ob + j0 + lane].x : 0x7fffffff;
        for (int k = 0; k < nw0; ++k) {
          const int c = __popcll(__ballot(col < __builtin_amdgcn_readlane(dst, k)));
          if (lane == k) pos += c;
        }
      }
      for (int32_t v0 = cb; v0 < ce; v0 += WAVE) {
        const int32_t qq = v0 + lane;
        const int d2 = qq < ce ? int32_t(ch_key[qq] - base) : 0x7fffffff;
        const int o2 = qq < ce ? ch_op[qq] : 0;
        const int nw = ce - v0 < WAVE ? ce - v0 : WAVE;
        for (int k = 0; k < nw; ++k) {
          const int dk = __builtin_amdgcn_readlane(d2, k);
          const int ok = __builtin_amdgcn_readlane(o2, k);
          if (dk < dst) pos += ok == OP_NEW ? 1 : (ok == OP_DELETE ? -1 : 0);
        }
      }
      if (hq) adj_new[nb + pos] = make_int2(dst, ch_w[q]);
    }
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
  s = wave_sum(s);
  if (lane == 0 && s) atomicAdd((unsigned long long*)I, (unsigned long long)s);
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
  s = wave_sum(s);
  if (lane_id() == 0 && s) atomicAdd((unsigned long long*)S, (unsigned long long)s);
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

void make_canonical(const int32_t* u, const int32_t* v, int64_t m, int32_t n,
                    uint64_t* keys, uint32_t* vals, hipStream_t st) {
  if (m <= 0) return;
  k_make_canonical<<<grid_for(m), TPB, 0, st>>>(u, v, m, n, keys, vals);
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

void detect_dups(const uint64_t* keys, int64_t m, int32_t* flags,
                 hipStream_t st) {
  if (m <= 1) return;
  k_detect_dups<<<grid_for(m), TPB, 0, st>>>(keys, m, flags);
  DC_LAUNCH_CHECK();
}

void lookup_deleted(const uint64_t* keys, int64_t m, int32_t n,
                    const int32_t* off, const int2* adj, int32_t* w_old,
                    int32_t* flags, long long* wsum, hipStream_t st) {
  if (m <= 0) return;
  k_lookup_deleted<<<grid_for(m), TPB, 0, st>>>(keys, m, n, off, adj, w_old, flags, wsum);
  DC_LAUNCH_CHECK();
}

void make_change_records(const uint64_t* del_keys, int64_t nd,
                         const uint64_t* ins_keys, int64_t na, int32_t n,
                         uint64_t* rkeys, uint32_t* rvals, hipStream_t st) {
  if (nd + na <= 0) return;
  k_make_change_records<<<grid_for(nd + na), TPB, 0, st>>>(del_keys, nd, ins_keys, na, n,
                                                           rkeys, rvals);
  DC_LAUNCH_CHECK();
}

void combine_changes(const uint64_t* rkeys, const uint32_t* rvals, int64_t nr,
                     const int32_t* heads, const int32_t* pos, int32_t n,
                     const int32_t* del_w_old, const int32_t* ins_w,
                     const int32_t* off, const int2* adj, uint64_t* ch_key,
                     int32_t* ch_op, int32_t* ch_w, int32_t* ch_dk,
                     int32_t* is_del, int32_t* is_new, hipStream_t st) {
  if (nr <= 0) return;
  k_combine_changes<<<grid_for(nr), TPB, 0, st>>>(rkeys, rvals, nr, heads, pos, n, del_w_old,
                                                  ins_w, off, adj, ch_key, ch_op, ch_w, ch_dk,
                                                  is_del, is_new);
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
        rows, nrows_dev, off_old, adj_old, off_new, adj_new, n, cptr, ch_key, ch_op, ch_w,
        cum_del, cum_new, big);
    DC_LAUNCH_CHECK();
    k_merge_big<<<256, TPB, 0, st>>>(big, off_old, adj_old, off_new, adj_new, n, cptr, ch_key,
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
