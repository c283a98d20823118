// dc_kernels.h -- host launchers of the gfx950 kernels (plain pointers, one
// stream).  The orchestration in api.hip composes them into dc_init and
// dc_apply_batch.
#pragma once

#include "dc_common.h"

namespace dc {

// ---- per-block aggregated scatter-add (hot community labels) ------------
// Pre-combines (key, value) pairs of a 256-thread block in an LDS table so a
// label shared by many vertices of the block costs one global atomic.
constexpr int AGG_SLOTS = 1024;

struct AggLds {
  int keys[AGG_SLOTS];
  long long vals[AGG_SLOTS];
};

__device__ __forceinline__ void agg_init(AggLds& s) {
  for (int i = threadIdx.x; i < AGG_SLOTS; i += blockDim.x) {
    s.keys[i] = EMPTY_KEY;
    s.vals[i] = 0;
  }
}

__device__ __forceinline__ void agg_put(AggLds& s, int key, long long v) {
  uint32_t h = hash_slot(key, AGG_SLOTS - 1);
  while (true) {
    int prev = atomicCAS(&s.keys[h], EMPTY_KEY, key);
    if (prev == EMPTY_KEY || prev == key) {
      atomicAdd((unsigned long long*)&s.vals[h], (unsigned long long)v);
      return;
    }
    h = (h + 1) & (AGG_SLOTS - 1);
  }
}

// Bounded insert-or-add: false when AGG_PROBES slots are taken by other
// keys (the caller then updates global memory directly).  Lets one block's
// table absorb many rows: updates of a large community, which would
// serialise as same-address atomics from every block, arrive as one sum.
constexpr int AGG_PROBES = 16;
__device__ __forceinline__ bool agg_try(AggLds& s, int key, long long v) {
  uint32_t h = hash_slot(key, AGG_SLOTS - 1);
  for (int p = 0; p < AGG_PROBES; ++p) {
    const int prev = atomicCAS(&s.keys[h], EMPTY_KEY, key);
    if (prev == EMPTY_KEY || prev == key) {
      atomicAdd((unsigned long long*)&s.vals[h], (unsigned long long)v);
      return true;
    }
    h = (h + 1) & (AGG_SLOTS - 1);
  }
  return false;
}

// ---- graph.hip -----------------------------------------------------------
enum EdgeFlag : int32_t { F_RANGE = 1, F_SELF = 2, F_WEIGHT = 4, F_DUP = 8, F_NO_EDGE = 16 };

// Weight sums that thousands of blocks add to are spread over SUM_SLOTS
// counters (block b adds to slot b % SUM_SLOTS; the reader adds them up):
// same-address atomics serialise.
constexpr int SUM_SLOTS = 64;

// flags |= F_RANGE / F_SELF / F_WEIGHT (w may be null); wsum (SUM_SLOTS
// counters) += sum of w.
void validate_edges(const int32_t* u, const int32_t* v, const int32_t* w,
                    int64_t m, int32_t n, int32_t* flags, long long* wsum,
                    hipStream_t st);

// Directed entries of an edge list for the initial CSR: keys u*n+v and v*n+u
// with the weight as value.
void make_directed(const int32_t* u, const int32_t* v, const int32_t* w,
                   int64_t m, int32_t n, uint64_t* keys, uint32_t* vals,
                   hipStream_t st);

// flag[i] = 1 if keys[i] starts a run of equal keys.
void run_heads(const uint64_t* keys, int64_t m, int32_t* flag, hipStream_t st);

// Sums runs of equal sorted keys: out_key[pos[i]] = keys[i] at heads and
// out_w[pos[i]] += w_of(vals[i]) where w_of is wsrc[vals[i]] (wsrc != null)
// or vals[i] itself.  out_w must be zeroed.
void reduce_runs(const uint64_t* keys, const uint32_t* vals,
                 const int32_t* wsrc, const int32_t* pos, int64_t m,
                 uint64_t* out_key, int32_t* out_w, hipStream_t st);

// row_ptr[u] = first index i with keys[i] >= u*n (u in [0, n]).
void row_bounds(const uint64_t* keys, int64_t m, int32_t n, int32_t* row_ptr,
                hipStream_t st);

// CSR entries from sorted unique directed keys.
void keys_to_adj(const uint64_t* keys, const int32_t* w, int64_t m, int32_t n,
                 int2* adj, hipStream_t st);

// k[u] = sum of row weights.
void row_weight_sums(const int32_t* off, const int2* adj, int32_t n,
                     int32_t* k, hipStream_t st);

// Change records of a batch, sorted by directed key src*n+dst.
enum ChangeOp : int32_t { OP_DELETE = 1, OP_ADD = 2, OP_NEW = 3, OP_REPLACE = 4 };

// Directed records of a batch: deletion e gives keys u*n+v and v*n+u with
// value (e<<1)|0, insertion e the same keys with value (e<<1)|1.
void batch_records(const int32_t* du, const int32_t* dv, int64_t nd, const int32_t* au,
                   const int32_t* av, int64_t na, int32_t n, uint64_t* keys, uint32_t* vals,
                   hipStream_t st);

// One change per run of equal sorted record keys (pos: exclusive scan of the
// run heads, *nruns on the device): ch_key, ch_op, ch_w (new weight for NEW
// and REPLACE, added weight for ADD), ch_dk (change of the row's weighted
// degree), dnet (+1 for NEW, -1 for DELETE, else 0); flags |= F_DUP (a pair
// deleted twice) and F_NO_EDGE (a deletion of a pair absent from off/adj);
// wsum (SUM_SLOTS counters) += the old weights of the deleted edges.
// run_key/run_w/run_ndel: scratch of m.
void resolve_changes(const uint64_t* keys, const uint32_t* vals, const int32_t* pos, int64_t m,
                     const int32_t* nruns, const int32_t* ins_w, int32_t n, const int32_t* off,
                     const int2* adj, uint64_t* run_key, int32_t* run_w, int32_t* run_ndel,
                     uint64_t* ch_key, int32_t* ch_op, int32_t* ch_w, int32_t* ch_dk,
                     int32_t* dnet, int32_t* flags, long long* wsum, hipStream_t st);

// Old CSR entries per block of the merge.
constexpr int MERGE_TILE = 1024;

// Per row: new degree and degree-weight change; k += dk; a[C[u]] += dk.
// tile_row (ceil(off[n] / MERGE_TILE) + 1 ints): the row holding entry
// t * MERGE_TILE for each tile t, then the row holding the last entry.
void row_changes(const int32_t* cptr, const int32_t* ch_op, const int32_t* ch_dk,
                 const int32_t* off, int32_t n, int32_t* new_deg, int32_t* k,
                 const int32_t* C, int32_t* a, int32_t* tile_row, hipStream_t st);

// Merge G_{t-1} with the sorted change list (ch_*, nch entries, row bounds
// cptr) into G_t: one launch, tiles of MERGE_TILE old entries (tile_row from
// row_changes) plus blocks that place the NEW pairs.  cnet: exclusive prefix
// sum of dnet over the change list (nch + 1 ints).  off_new must already
// hold G_t's offsets.
void merge_rows(const int32_t* off_old, const int2* adj_old, int64_t nnz_old,
                const int32_t* off_new, int2* adj_new, int32_t n, const int32_t* cptr,
                const int32_t* tile_row, const uint64_t* ch_key, const int32_t* ch_op,
                const int32_t* ch_w, const int32_t* cnet, int64_t nch, hipStream_t st);

// Exact numerator pieces of Eq. (1) over a CSR with labels C:
// *I += sum of intra-community entry weights; a_tmp (zeroed, n) receives
// sum of k by label; *S += sum a^2 (second launcher).
void intra_weight(const int32_t* off, const int2* adj, const int32_t* C,
                  int32_t n, long long* I, hipStream_t st);
void label_totals(const int32_t* k, const int32_t* C, int32_t n, int32_t* a,
                  hipStream_t st);
void sum_squares(const int32_t* a, int32_t n, long long* S, hipStream_t st);
// Both pieces in one launch over a partition whose label totals a are given:
// *I += intra-community weight, *S += sum over labels of a^2.
void modularity_terms(const int32_t* off, const int2* adj, const int32_t* C, const int32_t* a,
                      int32_t n, long long* I, long long* S, hipStream_t st);

}  // namespace dc
