// prims.hip -- scan, stable LSD radix sort, fills.  Hand-written for gfx950:
// 256-thread blocks of four 64-wide waves, wave prefix sums by shuffles,
// radix ranking by one 64-bit ballot per digit bit, running digit counts per wave.
#include <cstdlib>

#include "dc_common.h"

namespace dc {

bool sync_check_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("DC_SYNC_CHECK");
    return e && e[0] == '1';
  }();
  return on;
}

PrimScratch& prim_scratch() {
  static thread_local PrimScratch s;
  return s;
}

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;  // 2048
constexpr int64_t SCAN_RAW_MAX = 1024;  // tiles whose offsets are summed in-kernel
static_assert(SCAN_RAW_MAX % SCAN_THREADS == 0, "raw partials per thread");

template <class T, int NT = SCAN_THREADS>
__device__ T block_excl_scan(T v, T* lds, T* total) {
  const int lane = lane_id(), wid = threadIdx.x / WAVE;
  T x = v;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    T y = __shfl_up(x, o, WAVE);
    if (lane >= o) x += y;
  }
  if (lane == WAVE - 1) lds[wid] = x;
  __syncthreads();
  T pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NT / WAVE; ++w) {
    T t = lds[w];
    pre += (w < wid) ? t : T(0);
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return pre + x - v;
}

template <class T>
__global__ void __launch_bounds__(SCAN_THREADS)
    k_tile_reduce(const T* __restrict__ in, int64_t n, T* __restrict__ part) {
  __shared__ T lds[SCAN_THREADS / WAVE];
  int64_t base = int64_t(blockIdx.x) * SCAN_TILE;
  T s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    // clamped (n >= 1 in a launched tile): one unconditional load per item,
    // so the eight loads are in flight together
    const int64_t idx = base + int64_t(i) * SCAN_THREADS + threadIdx.x;
    const T x = in[idx < n ? idx : n - 1];
    s += idx < n ? x : T(0);
  }
  T tot;
  (void)block_excl_scan<T>(s, lds, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Each thread owns SCAN_ITEMS consecutive elements (blocked layout).  The
// tile's offset is part[blockIdx.x] when part holds exclusive prefixes
// (raw = 0), or the sum of part[0, blockIdx.x) when it holds the raw tile
// totals (raw = 1, used for at most SCAN_RAW_MAX tiles).
template <class T>
__global__ void __launch_bounds__(SCAN_THREADS)
    k_tile_scan(const T* in, T* out, int64_t n, const T* __restrict__ part, int raw,
                T* total, int64_t nblocks, T* htotal) {
  __shared__ T lds[SCAN_THREADS / WAVE];
  // the tile's items and the partials before it are loaded first, at
  // clamped indexes (n >= 1, nblocks >= 1), so they are in flight together
  const int64_t base = int64_t(blockIdx.x) * SCAN_TILE + int64_t(threadIdx.x) * SCAN_ITEMS;
  T v[SCAN_ITEMS];
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    const int64_t idx = base + i;
    const T x = in[idx < n ? idx : n - 1];
    v[i] = idx < n ? x : T(0);
  }
  T off = 0;
  if (part && raw) {  // nblocks <= SCAN_RAW_MAX
    T pv[SCAN_RAW_MAX / SCAN_THREADS];
#pragma unroll
    for (int j = 0; j < SCAN_RAW_MAX / SCAN_THREADS; ++j) {
      const int64_t b = int64_t(threadIdx.x) + int64_t(j) * SCAN_THREADS;
      const T x = part[b < nblocks ? b : nblocks - 1];
      pv[j] = b < int64_t(blockIdx.x) ? x : T(0);
    }
    T acc = 0;
#pragma unroll
    for (int j = 0; j < SCAN_RAW_MAX / SCAN_THREADS; ++j) acc += pv[j];
    (void)block_excl_scan<T>(acc, lds, &off);
  } else if (part) {
    off = part[blockIdx.x];
  }
  T s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) s += v[i];
  T tot;
  T pre = block_excl_scan<T>(s, lds, &tot);
  T run = off + pre;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    int64_t idx = base + i;
    if (idx < n) out[idx] = run;
    run += v[i];
  }
  if (blockIdx.x == nblocks - 1 && threadIdx.x == 0) {
    if (total) *total = off + tot;
    if (htotal) host_store(htotal, off + tot);
  }
}

template <class T>
__global__ void k_set_scalar(T* p, T v, T* hp) {
  if (p) *p = v;
  if (hp) host_store(hp, v);
}

template <class T>
void scan_excl_impl(const T* in, T* out, int64_t n, T* total, hipStream_t st,
                    T* tmp, size_t tmp_elems, T* htotal) {
  if (n <= 0) {
    if (total || htotal) {
      k_set_scalar<T><<<1, 1, 0, st>>>(total, T(0), htotal);
      DC_LAUNCH_CHECK();
    }
    return;
  }
  int64_t nb = ceil_div(n, SCAN_TILE);
  if (nb == 1) {
    k_tile_scan<T><<<1, SCAN_THREADS, 0, st>>>(in, out, n, nullptr, 0, total, 1, htotal);
    DC_LAUNCH_CHECK();
    return;
  }
  if (size_t(nb) > tmp_elems) throw std::runtime_error("scan scratch too small");
  T* part = tmp;
  k_tile_reduce<T><<<nb, SCAN_THREADS, 0, st>>>(in, n, part);
  DC_LAUNCH_CHECK();
  if (nb <= SCAN_RAW_MAX) {
    // each tile sums the totals before it (at most SCAN_RAW_MAX reads)
    k_tile_scan<T><<<nb, SCAN_THREADS, 0, st>>>(in, out, n, part, 1, total, nb, htotal);
    DC_LAUNCH_CHECK();
    return;
  }
  // exclusive scan of the block partials in place (recursion on the tail)
  scan_excl_impl<T>(part, part, nb, nullptr, st, tmp + nb, tmp_elems - size_t(nb), nullptr);
  k_tile_scan<T><<<nb, SCAN_THREADS, 0, st>>>(in, out, n, part, 0, total, nb, htotal);
  DC_LAUNCH_CHECK();
}

template <class T>
void scan_excl(const T* in, T* out, int64_t n, T* total, hipStream_t st, T* htotal) {
  // partial sums need ~ n/2048 + n/2048^2 + ... elements
  size_t need = size_t(ceil_div(n, SCAN_TILE)) + 64;
  need += need / SCAN_TILE + 64;
  DBuf& b = prim_scratch().scan_tmp;
  b.ensure(need * sizeof(T));
  scan_excl_impl<T>(in, out, n, total, st, b.as<T>(), b.bytes / sizeof(T), htotal);
}

// ---------------------------------------------------------------------------
// radix sort

// A tile of RS_TILE keys per block of the histogram and the scatter, 1024
// threads each: a batch of a few hundred thousand keys makes fewer tiles
// than the chip has CUs, so each block's chain of dependent steps is kept
// short by giving it many waves (two keys per thread) instead of long
// per-thread loops.
constexpr int RS_THREADS = 1024;
constexpr int RS_ROUNDS = 2;
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;  // 2048 keys per block
constexpr int RS_MAX_DIGIT = 10;  // 40-bit keys in 4 passes
constexpr int RS_BINS = 1 << RS_MAX_DIGIT;       // bins of the widest digit
constexpr int RS_WAVES = RS_THREADS / WAVE;

// Per-block digit histogram, written digit-major (hist[d * nblocks + block]):
// a scan of each digit's column plus the totals of the smaller digits give
// every (digit, block) its output offset.
__global__ void __launch_bounds__(RS_THREADS)
    k_radix_hist(const uint64_t* __restrict__ keys, int64_t n, int shift, int bins,
                 int32_t* __restrict__ hist, int64_t nblocks) {
  __shared__ int32_t h[RS_BINS];
  for (int b = threadIdx.x; b < bins; b += RS_THREADS) h[b] = 0;
  __syncthreads();
  const uint64_t mask = uint64_t(bins - 1);
  const int64_t base = int64_t(blockIdx.x) * RS_TILE;
  uint64_t k[RS_ROUNDS];
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t idx = base + int64_t(r) * RS_THREADS + threadIdx.x;
    k[r] = idx < n ? keys[idx] : 0;
  }
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t idx = base + int64_t(r) * RS_THREADS + threadIdx.x;
    if (idx < n) atomicAdd(&h[(k[r] >> shift) & mask], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < bins; b += RS_THREADS)
    hist[int64_t(b) * nblocks + blockIdx.x] = h[b];
}

// Column scan of the digit-major histogram, one block per digit: the
// tiles' counts of digit d become their exclusive prefix in place, and the
// digit's total goes to dtot[d] (the digit bases are summed by the scatter).
__global__ void __launch_bounds__(SCAN_THREADS)
    k_radix_colscan(int32_t* hist, int64_t nblocks, int32_t* dtot) {
  __shared__ int32_t lds[SCAN_THREADS / WAVE];
  int32_t* col = hist + int64_t(blockIdx.x) * nblocks;
  int32_t carry = 0;
  for (int64_t b0 = 0; b0 < nblocks; b0 += SCAN_THREADS * 4) {
    const int64_t base = b0 + int64_t(threadIdx.x) * 4;
    int32_t v[4], s = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      // clamped index (nblocks >= 1): the four loads in flight together
      const int32_t x = col[base + i < nblocks ? base + i : nblocks - 1];
      v[i] = base + i < nblocks ? x : 0;
      s += v[i];
    }
    int32_t tot;
    int32_t run = carry + block_excl_scan<int32_t>(s, lds, &tot);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (base + i < nblocks) col[base + i] = run;
      run += v[i];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) dtot[blockIdx.x] = carry;
}

// Stable scatter: wave w ranks the tile's elements [w * RS_WCHUNK,
// (w + 1) * RS_WCHUNK) in index order, RS_ROUNDS rounds of WAVE consecutive
// elements.  Within a round the rank among equal digits comes from a ballot
// match (one ballot per digit bit); across rounds the wave keeps running
// digit counts in its own LDS row (the group's first lane adds the group's
// size and hands the old count to the group), so ranking needs no block
// barrier.  A scan of each digit's per-wave counts then gives every wave its
// digit offsets.
constexpr int RS_WCHUNK = RS_ROUNDS * WAVE;
static_assert(RS_WCHUNK * RS_WAVES == RS_TILE, "waves cover the tile");
__global__ void __launch_bounds__(RS_THREADS)
    k_radix_scatter(const uint64_t* __restrict__ kin,
                    const uint32_t* __restrict__ vin, uint64_t* __restrict__ kout,
                    uint32_t* __restrict__ vout, int64_t n, int shift, int dbits,
                    const int32_t* __restrict__ colscan, const int32_t* __restrict__ dtot,
                    int64_t nblocks) {
  __shared__ int32_t base_d[RS_BINS];
  __shared__ int32_t wcnt[RS_WAVES][RS_BINS];  // 64 KB
  __shared__ int32_t lds[RS_WAVES];
  const int t = threadIdx.x, lane = lane_id(), wid = t / WAVE;
  const int bins = 1 << dbits;
  const int64_t wbase = int64_t(blockIdx.x) * RS_TILE + int64_t(wid) * RS_WCHUNK;
  // every global load of the block first, at clamped indexes (bins >= 2,
  // n >= 2), so the digit totals, this tile's digit offsets and the wave's
  // keys and values are in flight together: the wave's keys and values (all
  // rounds, loaded before the first is ranked), then per digit its total
  // and its count in the tiles before this one
  uint64_t kr[RS_ROUNDS];
  uint32_t vr[RS_ROUNDS];
  int32_t rk[RS_ROUNDS];
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t idx = wbase + int64_t(r) * WAVE + lane;
    const int64_t ic = idx < n ? idx : n - 1;
    kr[r] = kin[ic];
    vr[r] = vin[ic];
  }
  constexpr int DPT = RS_BINS / RS_THREADS;
  int32_t dv[DPT], cs[DPT];
#pragma unroll
  for (int i = 0; i < DPT; ++i) {
    const int d = t * DPT + i;
    const int dc = d < bins ? d : bins - 1;
    const int32_t x = dtot[dc], y = colscan[int64_t(dc) * nblocks + blockIdx.x];
    dv[i] = d < bins ? x : 0;
    cs[i] = y;
  }
  // output base of each digit in this tile: the totals of the smaller
  // digits (a block scan, RS_BINS / RS_THREADS digits per thread) plus the
  // digit's count in the tiles before this one
  {
    int32_t s = 0;
#pragma unroll
    for (int i = 0; i < DPT; ++i) s += dv[i];
    int32_t tot;
    int32_t run = block_excl_scan<int32_t, RS_THREADS>(s, lds, &tot);
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
      const int d = t * DPT + i;
      if (d < bins) base_d[d] = run + cs[i];
      run += dv[i];
    }
  }
  for (int b = t; b < bins; b += RS_THREADS) {
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w) wcnt[w][b] = 0;
  }
  __syncthreads();
  const uint64_t lt = (uint64_t(1) << lane) - 1;
  const uint64_t mask = uint64_t(bins - 1);
  int32_t* own = wcnt[wid];
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const bool valid = wbase + int64_t(r) * WAVE + lane < n;
    const int d = int((kr[r] >> shift) & mask);
    uint64_t m = __ballot(valid);
    for (int b = 0; b < dbits; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t bb = __ballot(valid && bit);
      m &= bit ? bb : ~bb;
    }
    // m holds this lane's digit group when valid (it is then nonzero)
    const int first = valid ? __ffsll((unsigned long long)m) - 1 : lane;
    int32_t old = 0;
    if (valid && first == lane) old = atomicAdd(&own[d], __popcll(m));
    old = __shfl(old, first);
    rk[r] = old + __popcll(m & lt);
  }
  __syncthreads();
  // per digit: the waves' counts become their exclusive prefix on top of
  // the digit's base in this tile
  for (int b = t; b < bins; b += RS_THREADS) {
    int32_t run = base_d[b];
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w) {
      const int32_t c = wcnt[w][b];
      wcnt[w][b] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    if (wbase + int64_t(r) * WAVE + lane < n) {
      const int d = int((kr[r] >> shift) & mask);
      const int32_t pos = own[d] + rk[r];
      kout[pos] = kr[r];
      vout[pos] = vr[r];
    }
  }
}

template <class T>
__global__ void k_fill(T* p, T v, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void k_iota(int32_t* p, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (; i < n; i += stride) p[i] = int32_t(i);
}

struct Copy4 {
  int32_t* dst[4];
  const int32_t* src[4];
};

__global__ void k_copy_i32(Copy4 c, int count, int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    for (int j = 0; j < count; ++j) c.dst[j][i] = c.src[j][i];
}

__global__ void k_start_level(int32_t* C, int32_t* Cn, int32_t* a, int32_t* sz,
                              const int32_t* __restrict__ k, int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    C[i] = int32_t(i);
    Cn[i] = int32_t(i);
    a[i] = k[i];
    sz[i] = 1;
  }
}

inline int grid_for(int64_t n, int threads = 256) {
  int64_t g = ceil_div(n, threads);
  if (g > 8192) g = 8192;
  return int(g < 1 ? 1 : g);
}

}  // namespace

void scan_excl_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* total,
                   hipStream_t st, int32_t* host_total) {
  scan_excl<int32_t>(in, out, n, total, st, host_total);
}

void scan_excl_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* total,
                   hipStream_t st, int64_t* host_total) {
  scan_excl<int64_t>(in, out, n, total, st, host_total);
}

void radix_sort_pairs(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1,
                      int64_t n, int bits, hipStream_t st) {
  if (radix_sort_pairs_swap(k0, v0, k1, v1, n, bits, st)) {
    DC_HIP(hipMemcpyAsync(k0, k1, size_t(n) * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
    DC_HIP(hipMemcpyAsync(v0, v1, size_t(n) * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
  }
}

bool radix_sort_pairs_swap(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1,
                           int64_t n, int bits, hipStream_t st) {
  if (n <= 1 || bits <= 0) return false;
  // fewest passes with digits of at most RS_MAX_DIGIT bits, equal widths
  const int passes = (bits + RS_MAX_DIGIT - 1) / RS_MAX_DIGIT;
  const int dbits = (bits + passes - 1) / passes;
  const int bins = 1 << dbits;
  const int64_t nb = ceil_div(n, RS_TILE);
  DBuf& hb = prim_scratch().sort_hist;
  hb.ensure((size_t(nb) + 1) * size_t(bins) * sizeof(int32_t));
  int32_t* hist = hb.as<int32_t>();
  int32_t* dtot = hist + size_t(nb) * size_t(bins);  // digit totals
  uint64_t *ka = k0, *kb = k1;
  uint32_t *va = v0, *vb = v1;
  for (int p = 0; p < passes; ++p) {
    const int shift = dbits * p;
    k_radix_hist<<<nb, RS_THREADS, 0, st>>>(ka, n, shift, bins, hist, nb);
    DC_LAUNCH_CHECK();
    k_radix_colscan<<<bins, SCAN_THREADS, 0, st>>>(hist, nb, dtot);
    DC_LAUNCH_CHECK();
    k_radix_scatter<<<nb, RS_THREADS, 0, st>>>(ka, va, kb, vb, n, shift, dbits, hist, dtot, nb);
    DC_LAUNCH_CHECK();
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  return ka != k0;
}

void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  k_fill<int32_t><<<grid_for(n), 256, 0, st>>>(p, v, n);
  DC_LAUNCH_CHECK();
}

void fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  k_fill<int64_t><<<grid_for(n), 256, 0, st>>>(p, v, n);
  DC_LAUNCH_CHECK();
}

void fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  k_fill<uint8_t><<<grid_for(n), 256, 0, st>>>(p, v, n);
  DC_LAUNCH_CHECK();
}

constexpr int ZERO_MAX = 6;
struct ZeroSet {
  uint8_t* p[ZERO_MAX];
  int64_t bytes[ZERO_MAX];
  int count;
};

__global__ void k_zero_buffers(ZeroSet z) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  for (int j = 0; j < z.count; ++j) {
    const int64_t nv = z.bytes[j] / 16;
    uint4* q = reinterpret_cast<uint4*>(z.p[j]);
    for (int64_t i = t; i < nv; i += stride) q[i] = make_uint4(0, 0, 0, 0);
    for (int64_t i = nv * 16 + t; i < z.bytes[j]; i += stride) z.p[j][i] = 0;
  }
}

void zero_buffers(void* const* p, const int64_t* bytes, int count, hipStream_t st) {
  ZeroSet z{};
  int64_t most = 0;
  for (int j = 0; j < count && j < ZERO_MAX; ++j) {
    if (bytes[j] <= 0) continue;
    z.p[z.count] = static_cast<uint8_t*>(p[j]);
    z.bytes[z.count] = bytes[j];
    ++z.count;
    most = bytes[j] / 16 > most ? bytes[j] / 16 : most;
  }
  if (z.count == 0) return;
  k_zero_buffers<<<grid_for(most + 1), 256, 0, st>>>(z);
  DC_LAUNCH_CHECK();
}

void copy_i32(int32_t* const* dst, const int32_t* const* src, int count, int64_t n,
              hipStream_t st) {
  if (n <= 0 || count <= 0) return;
  Copy4 c{};
  for (int j = 0; j < count && j < 4; ++j) {
    c.dst[j] = dst[j];
    c.src[j] = src[j];
  }
  k_copy_i32<<<grid_for(n), 256, 0, st>>>(c, count < 4 ? count : 4, n);
  DC_LAUNCH_CHECK();
}

void start_level(int32_t* C, int32_t* Cn, int32_t* a, int32_t* sz, const int32_t* k, int64_t n,
                 hipStream_t st) {
  if (n <= 0) return;
  k_start_level<<<grid_for(n), 256, 0, st>>>(C, Cn, a, sz, k, n);
  DC_LAUNCH_CHECK();
}

void iota_i32(int32_t* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  k_iota<<<grid_for(n), 256, 0, st>>>(p, n);
  DC_LAUNCH_CHECK();
}

}  // namespace dc
