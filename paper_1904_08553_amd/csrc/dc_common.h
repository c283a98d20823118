// dc_common.h -- internal declarations of the gfx950 library behind dc.h.
//
// Layout in HBM (one GPU, everything resident):
//   level-0 graph G_t   : CSR, int32 row offsets (n+1) and packed int2
//                         entries {neighbour, weight} (8 B, one 64-bit load
//                         per entry); double-buffered so a batch merge
//                         streams old -> new.  2m < 2^31 keeps every count,
//                         offset, degree and community total in int32.
//   k, C, a, size       : int32 per vertex / per label.
//   coarse levels       : the same CSR form, built per step.
// Exact integer arithmetic everywhere (scores in int64), so every reduction
// order gives the same bits and results do not depend on scheduling.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "dc.h"

namespace dc {

constexpr int WAVE = 64;
constexpr int64_t TWO_M_LIMIT = int64_t(1) << 31;

struct DeviceError : std::runtime_error {
  hipError_t code;
  DeviceError(hipError_t c, const std::string& what)
      : std::runtime_error(what), code(c) {}
};

#define DC_HIP(x)                                                        \
  do {                                                                   \
    hipError_t e_ = (x);                                                 \
    if (e_ != hipSuccess)                                                \
      throw ::dc::DeviceError(e_, std::string(#x) + " -> " +             \
                                      hipGetErrorString(e_) + " at " +   \
                                      __FILE__ + ":" +                   \
                                      std::to_string(__LINE__));         \
  } while (0)

// After every launch: the launch status, and with DC_SYNC_CHECK=1 in the
// environment also the kernel's completion (localises a failing kernel).
bool sync_check_enabled();
#define DC_LAUNCH_CHECK()                                                  \
  do {                                                                     \
    DC_HIP(hipGetLastError());                                             \
    if (::dc::sync_check_enabled()) DC_HIP(hipDeviceSynchronize());        \
  } while (0)

// Device memory of the library's buffers (alloc.hip).  Blocks come in size
// classes (four per doubling, so at most 25% over the request) and go back
// to a process-wide cache when released; pool_alloc hands out a cached block
// of the class before it calls hipMalloc, so a new context (a graph added
// to a server, a restored one, one graph per test) does not pay a hipMalloc
// per buffer in its first batch.  Released blocks become reusable after one
// device-wide wait on each device that released one (taken by the next
// pool_alloc), which is what hipFree costs anyway.  When hipMalloc runs out of memory, the cache
// is freed and the allocation tried once more.  pool_trim frees the cache
// (eviction to host memory calls it, so the evicted bytes leave the GPU).
void* pool_alloc(size_t bytes, size_t* got);
void pool_free(void* p, size_t bytes) noexcept;
void pool_trim() noexcept;

// Grow-only device buffer; contents are not preserved on growth.  Growth
// takes 25% headroom so sizes that creep up step by step (the edge count of
// a growing graph) do not pay a release and a new block (a device-wide wait)
// on every call.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) pool_free(p, bytes);
    p = nullptr;
    bytes = 0;
  }
  void ensure(size_t b) {
    if (b <= bytes && p) return;
    release();
    const size_t want = b < 256 ? 256 : b + b / 4;
    p = pool_alloc(want, &bytes);
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline int ilog2_ceil(uint64_t x) {
  int b = 0;
  while ((uint64_t(1) << b) < x) ++b;
  return b;
}

// ---------------------------------------------------------------------------
// device helpers

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

// Orders LDS traffic among the lanes of one wave (no cross-wave barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Butterfly step S of a cross-lane reduction.  Steps 0-3 exchange inside a
// 16-lane row with DPP (quad xor 1, quad xor 2, half-row mirror, row
// mirror), step 4 swaps the 16-lane halves of each 32 lanes (ds_swizzle):
// after steps 0..log2(G)-1 every lane of an aligned group of G <= 32 lanes
// has combined all G values.  The two 32-lane halves of a wave are then
// joined with two readlanes.  No step goes through ds_bpermute.
template <int S>
__device__ __forceinline__ int xchg(int v) {
  if constexpr (S == 0) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);
  else if constexpr (S == 1) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);
  else if constexpr (S == 2) return __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);
  else if constexpr (S == 3) return __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);
  else return __builtin_amdgcn_ds_swizzle(v, 0x401F);
}

template <int S>
__device__ __forceinline__ long long xchg64(long long v) {
  const int lo = xchg<S>(int(uint32_t(uint64_t(v))));
  const int hi = xchg<S>(int(uint32_t(uint64_t(v) >> 32)));
  return (long long)((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo));
}

__device__ __forceinline__ long long readlane64(long long v, int l) {
  const uint32_t lo = __builtin_amdgcn_readlane(int(uint32_t(uint64_t(v))), l);
  const uint32_t hi = __builtin_amdgcn_readlane(int(uint32_t(uint64_t(v) >> 32)), l);
  return (long long)((uint64_t(hi) << 32) | lo);
}

// Integer wave sums and maxima (exact, so the combining order is free).
__device__ __forceinline__ int wave_sum(int v) {
  v += xchg<0>(v);
  v += xchg<1>(v);
  v += xchg<2>(v);
  v += xchg<3>(v);
  v += xchg<4>(v);
  return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 32);
}

__device__ __forceinline__ long long wave_sum(long long v) {
  v += xchg64<0>(v);
  v += xchg64<1>(v);
  v += xchg64<2>(v);
  v += xchg64<3>(v);
  v += xchg64<4>(v);
  return readlane64(v, 0) + readlane64(v, 32);
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
  return (unsigned long long)wave_sum((long long)v);
}

__device__ __forceinline__ int wave_max(int v) {
  int y;
  y = xchg<0>(v); v = y > v ? y : v;
  y = xchg<1>(v); v = y > v ? y : v;
  y = xchg<2>(v); v = y > v ? y : v;
  y = xchg<3>(v); v = y > v ? y : v;
  y = xchg<4>(v); v = y > v ? y : v;
  const int a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 32);
  return a > b ? a : b;
}

__device__ __forceinline__ int wave_or(int v) {
  v |= xchg<0>(v);
  v |= xchg<1>(v);
  v |= xchg<2>(v);
  v |= xchg<3>(v);
  v |= xchg<4>(v);
  return __builtin_amdgcn_readlane(v, 0) | __builtin_amdgcn_readlane(v, 32);
}

// One global update per block instead of one per wave: same-address
// atomics serialise in L2, so a kernel of thousands of waves that each add
// to one counter queues thousands of them.  The waves reduce with DPP, their
// results meet in LDS, and thread 0 issues the atomic.  Every thread of the
// block must call these (no early exit before them).
__device__ __forceinline__ void block_add(long long v, long long* dst) {
  __shared__ long long part[16];
  v = wave_sum(v);
  if ((threadIdx.x & (WAVE - 1)) == 0) part[threadIdx.x / WAVE] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
    for (unsigned w = 0; w < blockDim.x / WAVE; ++w) t += part[w];
    if (t) atomicAdd((unsigned long long*)dst, (unsigned long long)t);
  }
  __syncthreads();
}

__device__ __forceinline__ void block_or(int v, int* dst) {
  __shared__ int part[16];
  v = wave_or(v);
  if ((threadIdx.x & (WAVE - 1)) == 0) part[threadIdx.x / WAVE] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (unsigned w = 0; w < blockDim.x / WAVE; ++w) t |= part[w];
    if (t) atomicOr(dst, t);
  }
  __syncthreads();
}

// A store to pinned host memory that the host reads after its next wait on
// the stream: a system-scope store, written through the caches.  (A
// system-scope fence instead would write back the whole L2.)
template <class T>
__device__ __forceinline__ void host_store(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Finished blocks of a launch: true in exactly one block, the last to get
// here, once every block has passed the call, so the others' reads before
// it are done (the barrier waits for them).  Their stores are not made
// visible to it: that would take a device-scope release per block, which
// on this chip writes back the L2 of the block's die.  The blocks count
// first in DONE_GROUPS counters (block b in counter b % DONE_GROUPS) and the
// last of each group in one more: a single word that thousands of blocks
// add to would queue them all behind each other.  ctr: DONE_WORDS words,
// zero before the launch and zero again after it.  Every thread of every
// block must call it (no early exit).
constexpr int DONE_GROUPS = 16;
constexpr int DONE_STRIDE = 32;  // words between two counters (128 B)
constexpr int DONE_WORDS = (DONE_GROUPS + 1) * DONE_STRIDE;

__device__ __forceinline__ bool last_block(unsigned* ctr) {
  __shared__ int last;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned nb = gridDim.x, g = blockIdx.x % DONE_GROUPS;
    const unsigned gsize = (nb - g + DONE_GROUPS - 1) / DONE_GROUPS;  // blocks of group g
    const unsigned ngroups = nb < unsigned(DONE_GROUPS) ? nb : unsigned(DONE_GROUPS);
    int l = 0;
    unsigned* gc = ctr + (1 + g) * DONE_STRIDE;
    if (atomicAdd(gc, 1u) == gsize - 1u) {
      atomicExch(gc, 0u);
      if (atomicAdd(ctr, 1u) == ngroups - 1u) {
        atomicExch(ctr, 0u);
        l = 1;
      }
    }
    last = l;
  }
  __syncthreads();
  return last != 0;
}

// Other types (floating point): a fixed butterfly order through shuffles.
template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// Best candidate order: larger score first, then smaller label.
struct Best {
  long long s;
  int x;
};

__device__ __forceinline__ bool better(long long s, int x, long long bs,
                                       int bx) {
  return s > bs || (s == bs && x < bx);
}

template <int S>
__device__ __forceinline__ Best best_step(Best b) {
  const Best y = {xchg64<S>(b.s), xchg<S>(b.x)};
  return better(y.s, y.x, b.s, b.x) ? y : b;
}

__device__ __forceinline__ Best wave_best(Best b) {
  b = best_step<4>(best_step<3>(best_step<2>(best_step<1>(best_step<0>(b)))));
  const Best b0 = {readlane64(b.s, 0), __builtin_amdgcn_readlane(b.x, 0)};
  const Best b1 = {readlane64(b.s, 32), __builtin_amdgcn_readlane(b.x, 32)};
  return better(b1.s, b1.x, b0.s, b0.x) ? b1 : b0;
}

constexpr int EMPTY_KEY = -1;
constexpr long long NO_SCORE = (long long)0x8000000000000000ull;
constexpr int NO_LABEL = 0x7fffffff;

__device__ __forceinline__ uint32_t hash_slot(int key, uint32_t mask) {
  return (uint32_t(key) * 2654435761u) & mask;
}

// Open-addressing insert-or-add into a table of int32 keys and int32 sums;
// the table never fills (capacity >= 2 * distinct keys).
__device__ __forceinline__ void table_add(int* keys, int* vals, uint32_t mask,
                                          int key, int w) {
  uint32_t h = hash_slot(key, mask);
  while (true) {
    int prev = atomicCAS(&keys[h], EMPTY_KEY, key);
    if (prev == EMPTY_KEY || prev == key) {
      atomicAdd(&vals[h], w);
      return;
    }
    h = (h + 1) & mask;
  }
}

// table_add for a table that may hold too few slots: a new key first
// reserves one of `limit` claims (*claimed counts them; a claim whose CAS
// then loses the slot to another key is simply spent), so at most `limit`
// slots are ever taken and every probe sequence ends.  Past the limit the
// key is dropped and *ovf is set: the table is incomplete.
__device__ __forceinline__ void table_add_bounded(int* keys, int* vals, uint32_t mask, int key,
                                                  int w, int* claimed, int* ovf, int limit) {
  uint32_t h = hash_slot(key, mask);
  while (true) {
    const int k = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (k == key) {
      atomicAdd(&vals[h], w);
      return;
    }
    if (k == EMPTY_KEY) {
      if (atomicAdd(claimed, 1) >= limit) {
        *ovf = 1;
        return;
      }
      const int prev = atomicCAS(&keys[h], EMPTY_KEY, key);
      if (prev == EMPTY_KEY || prev == key) {
        atomicAdd(&vals[h], w);
        return;
      }
    }
    h = (h + 1) & mask;
  }
}

__device__ __forceinline__ int table_get(const int* keys, const int* vals,
                                         uint32_t mask, int key) {
  uint32_t h = hash_slot(key, mask);
  while (true) {
    int k = keys[h];
    if (k == key) return vals[h];
    if (k == EMPTY_KEY) return 0;
    h = (h + 1) & mask;
  }
}

// ---------------------------------------------------------------------------
// primitives (prims.hip)

// out[i] = sum_{j<i} in[j]; *total (device, may be null) = sum of all.
// host_total (may be null): a device-visible address of pinned host memory
// that the last kernel also writes the sum to, for the host to read after
// its next wait on the stream (no copy).
void scan_excl_i32(const int32_t* in, int32_t* out, int64_t n,
                   int32_t* total, hipStream_t st, int32_t* host_total = nullptr);
void scan_excl_i64(const int64_t* in, int64_t* out, int64_t n,
                   int64_t* total, hipStream_t st, int64_t* host_total = nullptr);

// Stable LSD radix sort of (key, value) pairs on key bits [0, bits).
// Sorted data ends in (k0, v0); (k1, v1) are scratch of the same size.
void radix_sort_pairs(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1,
                      int64_t n, int bits, hipStream_t st);
// The same without the copy back: true when the sorted data ends in
// (k1, v1) (an odd number of passes), false when in (k0, v0).
bool radix_sort_pairs_swap(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1,
                           int64_t n, int bits, hipStream_t st);

void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st);
void fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t st);
void fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t st);
// Sets count (<= 6) device buffers of bytes[j] bytes each to zero in one
// launch; a buffer of 16 bytes or more starts 16-byte aligned.
void zero_buffers(void* const* p, const int64_t* bytes, int count, hipStream_t st);
void iota_i32(int32_t* p, int64_t n, hipStream_t st);
// dst[j][i] = src[j][i] for j < count (<= 4) in one launch.
void copy_i32(int32_t* const* dst, const int32_t* const* src, int count, int64_t n,
              hipStream_t st);
// A level's start partition: C[i] = Cn[i] = i, a[i] = k[i], size[i] = 1.
void start_level(int32_t* C, int32_t* Cn, int32_t* a, int32_t* sz, const int32_t* k, int64_t n,
                 hipStream_t st);

// Scratch for the primitives (owned by the context).
struct PrimScratch {
  DBuf scan_tmp;
  DBuf sort_hist;
};
PrimScratch& prim_scratch();

}  // namespace dc
