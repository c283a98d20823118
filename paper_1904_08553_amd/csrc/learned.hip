// learned.hip -- the learned screener (an extension; the paper has no
// learned component): feature assembly for the touched vertices, the
// 8 -> 64 -> 64 -> 1 network forward and backward on the matrix cores, Adam,
// and the dc_mlp entry points of dc.h.
//
// Matrix-core layout (v_mfma_f32_16x16x16_bf16 and, on gfx950,
// v_mfma_f32_16x16x32_bf16).  Lane l = 16q + r (q = l/16, r = l%16) holds
//   A[m = r][k = Kq + j], B[k = Kq + j][n = r]   (K = 4 or 8 values per lane)
//   D[m = 4q + i][n = r], i = 0..3.
// The network runs transposed, one wave per tile of 16 samples: Z^T = W X^T,
// so a sample is a column n = r and hidden unit 16mb + 4q + i of sample r
// sits in lane (q, r).  The next layer's B operand takes its K slots from
// exactly the units a lane already holds (slot (q, j) of K block kb is unit
// 32kb + 16(j/4) + 4q + j%4), and the weight operand is loaded with the same
// permutation, so no transpose is needed between layers.  The weight
// gradients contract over samples and go through a 2 KB LDS transpose per
// operand.
#include <mutex>
#include <string>

#include "learned.h"

#include <cmath>
#include <cstring>
#include <string>

namespace dc {

namespace {

constexpr int TPB = 256;
constexpr int NW = TPB / WAVE;

typedef short s4v __attribute__((ext_vector_type(4)));
typedef __bf16 b8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef unsigned int u2v __attribute__((ext_vector_type(2)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf16_val(uint32_t b) { return __uint_as_float(b << 16); }
__device__ __forceinline__ uint32_t pack2(uint32_t lo, uint32_t hi) { return lo | (hi << 16); }

__device__ __forceinline__ f4v mma16(u2v a, u2v b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4v, a),
                                                    __builtin_bit_cast(s4v, b), c, 0, 0, 0);
}

__device__ __forceinline__ f4v mma32(u4v a, u4v b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8v, a),
                                                  __builtin_bit_cast(b8v, b), c, 0, 0, 0);
}

// Orders LDS traffic among the lanes of one wave.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// K slot (q, j) of block kb of a layer-2 contraction: the hidden unit that
// lane (q, *) holds in position (mb = 2kb + j/4, i = j%4).
__device__ __forceinline__ int slot_unit(int kb, int q, int j) {
  return 32 * kb + 16 * (j >> 2) + 4 * q + (j & 3);
}

struct Net {
  u2v w1[4];     // layer 1 A operand per output block: W1[16mb + r][4q .. 4q+3]
  u4v w2[4][2];  // layer 2 A operand per (output block, K block)
  float b1[4][4], b2[4][4], w3[4][4];  // of unit 16mb + 4q + i
  float b3;
};

__device__ __forceinline__ void load_net(const uint16_t* __restrict__ wq, Net& N, int q, int r) {
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    const int row = 16 * mb + r;
    N.w1[mb] = q < 2 ? *reinterpret_cast<const u2v*>(wq + OFF_W1 + row * MLP_IN + 4 * q)
                     : u2v{0u, 0u};
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      const uint16_t* p = wq + OFF_W2 + row * MLP_HID + slot_unit(kb, q, 0);
      const u2v lo = *reinterpret_cast<const u2v*>(p);
      const u2v hi = *reinterpret_cast<const u2v*>(p + 16);
      N.w2[mb][kb] = u4v{lo.x, lo.y, hi.x, hi.y};
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int u = 16 * mb + 4 * q + i;
      N.b1[mb][i] = bf16_val(wq[OFF_B1 + u]);
      N.b2[mb][i] = bf16_val(wq[OFF_B2 + u]);
      N.w3[mb][i] = bf16_val(wq[OFF_W3 + u]);
    }
  }
  N.b3 = bf16_val(wq[OFF_B3]);
}

struct Fwd {
  u2v xb;           // X[s][4q .. 4q+3] (q < 2), the layer-1 B operand
  f4v z1[4];        // pre-activations of unit 16mb + 4q + i, sample r
  uint32_t h1[4][4];
  u4v hb[2];        // layer-2 B operand (bf16 h1 in K-slot order)
  f4v z2[4];
  float h2[4][4];
  float z3;         // logit of sample r (every q)
};

__device__ __forceinline__ void forward_tile(const Net& N, const uint16_t* __restrict__ X,
                                             int64_t n, int64_t s0, int q, int r, Fwd& F) {
  const int64_t s = s0 + r;
  F.xb = (q < 2 && s < n) ? *reinterpret_cast<const u2v*>(X + s * MLP_IN + 4 * q) : u2v{0u, 0u};
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    f4v acc = {N.b1[mb][0], N.b1[mb][1], N.b1[mb][2], N.b1[mb][3]};
    F.z1[mb] = mma16(N.w1[mb], F.xb, acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) F.h1[mb][i] = bf16_bits(fmaxf(F.z1[mb][i], 0.f));
  }
#pragma unroll
  for (int kb = 0; kb < 2; ++kb)
    F.hb[kb] = u4v{pack2(F.h1[2 * kb][0], F.h1[2 * kb][1]), pack2(F.h1[2 * kb][2], F.h1[2 * kb][3]),
                   pack2(F.h1[2 * kb + 1][0], F.h1[2 * kb + 1][1]),
                   pack2(F.h1[2 * kb + 1][2], F.h1[2 * kb + 1][3])};
  float part = 0.f;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    f4v acc = {N.b2[mb][0], N.b2[mb][1], N.b2[mb][2], N.b2[mb][3]};
    acc = mma32(N.w2[mb][0], F.hb[0], acc);
    acc = mma32(N.w2[mb][1], F.hb[1], acc);
    F.z2[mb] = acc;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      F.h2[mb][i] = bf16_val(bf16_bits(fmaxf(acc[i], 0.f)));
      part += N.w3[mb][i] * F.h2[mb][i];
    }
  }
  part += __shfl_xor(part, 16, WAVE);
  part += __shfl_xor(part, 32, WAVE);
  F.z3 = part + N.b3;
}

__global__ void __launch_bounds__(TPB)
    k_mlp_forward(const uint16_t* __restrict__ wq, const uint16_t* __restrict__ X, int64_t n,
                  float* __restrict__ logits) {
  const int lane = lane_id(), q = lane >> 4, r = lane & 15;
  const int wid = threadIdx.x / WAVE;
  Net N;
  load_net(wq, N, q, r);
  const int64_t tiles = ceil_div(n, 16);
  for (int64_t t = int64_t(blockIdx.x) * NW + wid; t < tiles; t += int64_t(gridDim.x) * NW) {
    Fwd F;
    forward_tile(N, X, n, t * 16, q, r, F);
    if (q == 0 && t * 16 + r < n) logits[t * 16 + r] = F.z3;
  }
}

__device__ __forceinline__ float softplus(float x) {
  return fmaxf(x, 0.f) + log1pf(expf(-fabsf(x)));
}

__device__ __forceinline__ float sum16(float v) {
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// One block: its waves take tiles of 16 samples; each block writes the sum of
// its samples' gradient (and loss) to partial[blockIdx][GRAD_SLOTS], adding
// the waves in a fixed order.
__global__ void __launch_bounds__(TPB)
    k_mlp_grad(const uint16_t* __restrict__ wq, const uint16_t* __restrict__ X,
               const uint8_t* __restrict__ y, int64_t n, float pw, float inv_n,
               float* __restrict__ partial) {
  __shared__ float acc[GRAD_SLOTS];
  __shared__ __align__(16) uint16_t lt[NW][4][MLP_HID * 16];
  const int wid = threadIdx.x / WAVE, lane = lane_id(), q = lane >> 4, r = lane & 15;
  for (int p = threadIdx.x; p < GRAD_SLOTS; p += TPB) acc[p] = 0.f;
  Net N;
  load_net(wq, N, q, r);
  // A operand of dh1^T = W2^T dz2^T: row = hidden unit 16mj + r, K slots as
  // in the forward pass
  u4v w2t[4][2];
#pragma unroll
  for (int mj = 0; mj < 4; ++mj)
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      uint32_t e[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) e[j] = wq[OFF_W2 + slot_unit(kb, q, j) * MLP_HID + 16 * mj + r];
      w2t[mj][kb] = u4v{pack2(e[0], e[1]), pack2(e[2], e[3]), pack2(e[4], e[5]),
                        pack2(e[6], e[7])};
    }
  f4v gW2[4][4], gW1[4];
  float gw3[4][4], gb2[4][4], gb1[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    gW1[a] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      gW2[a][b] = f4v{0.f, 0.f, 0.f, 0.f};
      gw3[a][b] = gb2[a][b] = gb1[a][b] = 0.f;
    }
  }
  float gb3 = 0.f, gloss = 0.f;
  uint16_t* Ldz2 = lt[wid][0];  // [unit][sample]
  uint16_t* Lh1 = lt[wid][1];
  uint16_t* Ldz1 = lt[wid][2];
  uint16_t* LX = lt[wid][3];    // [feature (16 rows, 8..15 zero)][sample]
  const int64_t tiles = ceil_div(n, 16);
  for (int64_t t = int64_t(blockIdx.x) * NW + wid; t < tiles; t += int64_t(gridDim.x) * NW) {
    const int64_t s = t * 16 + r;
    Fwd F;
    forward_tile(N, X, n, t * 16, q, r, F);
    const bool valid = s < n;
    const float yv = valid ? float(y[s]) : 0.f;
    const float z = F.z3;
    const float p = 1.f / (1.f + expf(-z));
    const float dz3 = valid ? ((pw * yv + 1.f - yv) * p - pw * yv) * inv_n : 0.f;
    if (q == 0 && valid) {
      gloss += pw * yv * softplus(-z) + (1.f - yv) * softplus(z);
      gb3 += dz3;
    }
    uint32_t d2[4][4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        gw3[mb][i] += dz3 * F.h2[mb][i];
        d2[mb][i] = bf16_bits(F.z2[mb][i] > 0.f ? dz3 * N.w3[mb][i] : 0.f);
        gb2[mb][i] += bf16_val(d2[mb][i]);
        const int u = 16 * mb + 4 * q + i;
        Ldz2[u * 16 + r] = uint16_t(d2[mb][i]);
        Lh1[u * 16 + r] = uint16_t(F.h1[mb][i]);
      }
    {
      const uint32_t xs[4] = {F.xb.x & 0xffffu, F.xb.x >> 16, F.xb.y & 0xffffu, F.xb.y >> 16};
#pragma unroll
      for (int i = 0; i < 4; ++i) LX[(4 * q + i) * 16 + r] = uint16_t(xs[i]);
    }
    wave_sync();
    // dW2[o][j] += sum_s dz2[s][o] h1[s][j]
#pragma unroll
    for (int mo = 0; mo < 4; ++mo) {
      const u2v a = *reinterpret_cast<const u2v*>(Ldz2 + (16 * mo + r) * 16 + 4 * q);
#pragma unroll
      for (int mj = 0; mj < 4; ++mj) {
        const u2v b = *reinterpret_cast<const u2v*>(Lh1 + (16 * mj + r) * 16 + 4 * q);
        gW2[mo][mj] = mma16(a, b, gW2[mo][mj]);
      }
    }
    // dh1^T = W2^T dz2^T, then dz1 = bf16(dh1 * [z1 > 0])
    u4v db[2];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
      db[kb] = u4v{pack2(d2[2 * kb][0], d2[2 * kb][1]), pack2(d2[2 * kb][2], d2[2 * kb][3]),
                   pack2(d2[2 * kb + 1][0], d2[2 * kb + 1][1]),
                   pack2(d2[2 * kb + 1][2], d2[2 * kb + 1][3])};
#pragma unroll
    for (int mj = 0; mj < 4; ++mj) {
      f4v h = {0.f, 0.f, 0.f, 0.f};
      h = mma32(w2t[mj][0], db[0], h);
      h = mma32(w2t[mj][1], db[1], h);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t b = bf16_bits(F.z1[mj][i] > 0.f ? h[i] : 0.f);
        gb1[mj][i] += bf16_val(b);
        Ldz1[(16 * mj + 4 * q + i) * 16 + r] = uint16_t(b);
      }
    }
    wave_sync();
    // dW1[o][f] += sum_s dz1[s][o] X[s][f]
    const u2v xT = *reinterpret_cast<const u2v*>(LX + r * 16 + 4 * q);
#pragma unroll
    for (int mo = 0; mo < 4; ++mo) {
      const u2v a = *reinterpret_cast<const u2v*>(Ldz1 + (16 * mo + r) * 16 + 4 * q);
      gW1[mo] = mma16(a, xT, gW1[mo]);
    }
    wave_sync();  // the tile buffers are rewritten by the next tile
  }
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      gw3[mb][i] = sum16(gw3[mb][i]);
      gb2[mb][i] = sum16(gb2[mb][i]);
      gb1[mb][i] = sum16(gb1[mb][i]);
    }
  gb3 = wave_sum(gb3);
  gloss = wave_sum(gloss);
  __syncthreads();  // acc cleared
  for (int w = 0; w < NW; ++w) {
    if (wid == w) {
#pragma unroll
      for (int mo = 0; mo < 4; ++mo)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int o = 16 * mo + 4 * q + i;
#pragma unroll
          for (int mj = 0; mj < 4; ++mj) acc[OFF_W2 + o * MLP_HID + 16 * mj + r] += gW2[mo][mj][i];
          if (r < MLP_IN) acc[OFF_W1 + o * MLP_IN + r] += gW1[mo][i];
          if (r == 0) {
            acc[OFF_W3 + o] += gw3[mo][i];
            acc[OFF_B2 + o] += gb2[mo][i];
            acc[OFF_B1 + o] += gb1[mo][i];
          }
        }
      if (lane == 0) {
        acc[OFF_B3] += gb3;
        acc[MLP_P] += gloss;
      }
    }
    __syncthreads();
  }
  for (int p = threadIdx.x; p < GRAD_SLOTS; p += TPB)
    partial[int64_t(blockIdx.x) * GRAD_SLOTS + p] = acc[p];
}

__global__ void k_grad_reduce(const float* __restrict__ partial, int nblocks, float* grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= GRAD_SLOTS) return;
  float s = 0.f;
  for (int b = 0; b < nblocks; ++b) s += partial[int64_t(b) * GRAD_SLOTS + p];
  grad[p] = s;
}

__global__ void k_adam(float* w, float* m, float* v, const float* __restrict__ g, float lr,
                       float c1, float c2, uint16_t* wq) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= MLP_P) return;
  const float gg = g[p];
  const float mm = 0.9f * m[p] + 0.1f * gg;
  const float vv = 0.999f * v[p] + 0.001f * gg * gg;
  m[p] = mm;
  v[p] = vv;
  const float ww = w[p] - lr * (mm * c1) / (sqrtf(vv * c2) + 1e-8f);
  w[p] = ww;
  wq[p] = bf16_bits(ww);
}

__global__ void k_to_bf16(const float* __restrict__ w, int n, uint16_t* wq) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) wq[p] = bf16_bits(w[p]);
}

// ---- batch side ----

__global__ void k_assemble(const int32_t* __restrict__ T, int64_t cnt,
                           const int32_t* __restrict__ k, const int32_t* __restrict__ kprev,
                           const int32_t* __restrict__ cptr, const int32_t* __restrict__ f_own,
                           const long long* __restrict__ f_g1, const long long* __restrict__ f_g2,
                           const int32_t* __restrict__ a, const int32_t* __restrict__ C,
                           const uint8_t* __restrict__ Rds, long long two_m,
                           uint16_t* __restrict__ X) {
  for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < cnt;
       idx += int64_t(gridDim.x) * blockDim.x) {
    const int i = T[idx];
    const long long ki = k[i], kp = kprev[i], t = cptr[i + 1] - cptr[i];
    const long long mx = ki > kp ? ki : kp;
    const long long g1 = f_g1[i], g2 = f_g2[i];
    double x[MLP_IN];
    x[0] = double(ki) / (double(ki) + 16.0);
    x[1] = mx > 0 ? double(ki - kp) / double(mx) : 0.0;
    x[2] = double(t) / (double(t) + 4.0);
    x[3] = ki > 0 ? double(f_own[i]) / double(ki) : 0.0;
    x[4] = (ki > 0 && g1 != NO_GAIN) ? double(g1) / double(two_m * ki) : -3.0;
    x[5] = (ki > 0 && g2 != NO_GAIN) ? double(g2) / double(two_m * ki) : -3.0;
    x[6] = Rds[i] ? 1.0 : 0.0;
    x[7] = two_m > 0 ? double(a[C[i]]) / double(two_m) : 0.0;
    uint32_t b[MLP_IN];
#pragma unroll
    for (int j = 0; j < MLP_IN; ++j) b[j] = bf16_bits(float(x[j]));
    reinterpret_cast<u4v*>(X)[idx] =
        u4v{pack2(b[0], b[1]), pack2(b[2], b[3]), pack2(b[4], b[5]), pack2(b[6], b[7])};
  }
}

__global__ void k_move_labels(const int32_t* __restrict__ T, int64_t cnt,
                              const int32_t* __restrict__ Cl, const int32_t* __restrict__ C,
                              uint8_t* y) {
  for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < cnt;
       idx += int64_t(gridDim.x) * blockDim.x) {
    const int i = T[idx];
    y[idx] = Cl[i] != C[i] ? 1 : 0;
  }
}

__global__ void k_select(const int32_t* __restrict__ T, int64_t cnt,
                         const float* __restrict__ logits, float theta, uint8_t* R) {
  for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < cnt;
       idx += int64_t(gridDim.x) * blockDim.x)
    if (logits[idx] >= theta) R[T[idx]] = 1;
}

__global__ void k_flags(const uint8_t* __restrict__ a, const uint8_t* __restrict__ b, int32_t n,
                        int32_t* flag) {
  for (int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
       v += int64_t(gridDim.x) * blockDim.x)
    flag[v] = (a[v] | (b ? b[v] : 0)) ? 1 : 0;
}

// 16 lanes per listed vertex (four vertices per wave: the rows are short)
constexpr int MT_GS = 16;
__global__ void k_mark_touched(const int32_t* __restrict__ list, const int32_t* __restrict__ count,
                               const int32_t* __restrict__ off, const int2* __restrict__ adj,
                               uint8_t* out) {
  const int64_t cnt = *count;
  const int gl = lane_id() % MT_GS;
  const int64_t ngroups = int64_t(gridDim.x) * (TPB / MT_GS);
  for (int64_t p = (int64_t(blockIdx.x) * TPB + threadIdx.x) / MT_GS; p < cnt; p += ngroups) {
    const int i = list[p];
    if (gl == 0) out[i] = 1;
    for (int32_t j = off[i] + gl; j < off[i + 1]; j += MT_GS) out[adj[j].x] = 1;
  }
}

inline int grid_for(int64_t n, int64_t cap = 16384) {
  int64_t g = ceil_div(n, TPB);
  if (g > cap) g = cap;
  return int(g < 1 ? 1 : g);
}

constexpr int GRAD_BLOCKS_MAX = 128;

inline int grad_blocks(int64_t n) {
  // a fixed function of n, so the summation order (and the result) is too
  int64_t b = ceil_div(ceil_div(n, 16), NW);
  if (b > GRAD_BLOCKS_MAX) b = GRAD_BLOCKS_MAX;
  return int(b < 1 ? 1 : b);
}

}  // namespace

void assemble_features(const int32_t* T, int64_t cnt, const int32_t* k, const int32_t* kprev,
                       const int32_t* cptr, const int32_t* f_own, const long long* f_g1,
                       const long long* f_g2, const int32_t* a, const int32_t* C,
                       const uint8_t* Rds, long long two_m, uint16_t* X, hipStream_t st) {
  if (cnt <= 0) return;
  k_assemble<<<grid_for(cnt), TPB, 0, st>>>(T, cnt, k, kprev, cptr, f_own, f_g1, f_g2, a, C, Rds,
                                            two_m, X);
  DC_LAUNCH_CHECK();
}

void move_labels(const int32_t* T, int64_t cnt, const int32_t* Cl, const int32_t* C, uint8_t* y,
                 hipStream_t st) {
  if (cnt <= 0) return;
  k_move_labels<<<grid_for(cnt), TPB, 0, st>>>(T, cnt, Cl, C, y);
  DC_LAUNCH_CHECK();
}

void select_by_score(const int32_t* T, int64_t cnt, const float* logits, float theta, uint8_t* R,
                     hipStream_t st) {
  if (cnt <= 0) return;
  k_select<<<grid_for(cnt), TPB, 0, st>>>(T, cnt, logits, theta, R);
  DC_LAUNCH_CHECK();
}

void merge_flags(const uint8_t* a, const uint8_t* b, int32_t n, int32_t* flag, hipStream_t st) {
  if (n <= 0) return;
  k_flags<<<grid_for(n), TPB, 0, st>>>(a, b, n, flag);
  DC_LAUNCH_CHECK();
}

void mark_touched(const int32_t* list, const int32_t* count, int64_t max_count,
                  const int32_t* off, const int2* adj, uint8_t* out, hipStream_t st) {
  if (max_count <= 0) return;
  k_mark_touched<<<grid_for(max_count * MT_GS, 4096), TPB, 0, st>>>(list, count, off, adj, out);
  DC_LAUNCH_CHECK();
}

void mlp_forward(const uint16_t* wq, const uint16_t* X, int64_t n, float* logits, hipStream_t st) {
  if (n <= 0) return;
  // each wave loads the whole network into registers once, so the grid
  // stays at a few blocks per CU and the waves loop over many tiles
  int64_t b = ceil_div(ceil_div(n, 16), NW);
  if (b > 1024) b = 1024;
  k_mlp_forward<<<int(b), TPB, 0, st>>>(wq, X, n, logits);
  DC_LAUNCH_CHECK();
}

int64_t mlp_partial_floats(int64_t n) { return int64_t(grad_blocks(n)) * GRAD_SLOTS; }

void mlp_grad(const uint16_t* wq, const uint16_t* X, const uint8_t* y, int64_t n,
              float pos_weight, float* partial, float* grad, hipStream_t st) {
  const int nb = grad_blocks(n);
  k_mlp_grad<<<nb, TPB, 0, st>>>(wq, X, y, n, pos_weight, n > 0 ? 1.f / float(n) : 0.f, partial);
  DC_LAUNCH_CHECK();
  k_grad_reduce<<<int(ceil_div(GRAD_SLOTS, TPB)), TPB, 0, st>>>(partial, nb, grad);
  DC_LAUNCH_CHECK();
}

void mlp_adam(float* w, float* m, float* v, const float* grad, int step, float lr, uint16_t* wq,
              hipStream_t st) {
  const double c1 = 1.0 / (1.0 - std::pow(0.9, step));
  const double c2 = 1.0 / (1.0 - std::pow(0.999, step));
  k_adam<<<int(ceil_div(MLP_P, TPB)), TPB, 0, st>>>(w, m, v, grad, lr, float(c1), float(c2), wq);
  DC_LAUNCH_CHECK();
}

}  // namespace dc

// ---------------------------------------------------------------------------
// dc_mlp entry points

using namespace dc;

namespace {

// Scratch of dc_mlp_grad_noalloc, a file-scope device array: the per-block
// partial sums (at most GRAD_BLOCKS_MAX blocks of GRAD_SLOTS floats, the most
// the gradient kernel launches for any n) followed by the reduced gradient.
// Every device that runs the library holds its own copy until the process
// ends.  Host code never passes the array's name to a kernel: it stands for
// a host-side symbol there; the device address comes from
// hipGetSymbolAddress, once per device, and is kept in g_scratch_dev.
constexpr size_t NOALLOC_PARTIAL = size_t(GRAD_BLOCKS_MAX) * GRAD_SLOTS;
constexpr size_t NOALLOC_FLOATS = NOALLOC_PARTIAL + GRAD_SLOTS;
static __device__ __align__(256) float scratch[NOALLOC_FLOATS];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[MAX_DEVICES] = {};

// The current device's address of `scratch` (looked up on the first call
// on that device, with that device current).
float* scratch_on_current_device() {
  int dev = 0;
  DC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) throw std::runtime_error("device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    DC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_dev[dev] = static_cast<float*>(p);
  }
  return g_scratch_dev[dev];
}

}  // namespace

struct dc_mlp {
  hipStream_t st = nullptr;
  DBuf w, m, v, wq, grad, partial;
  float* hgrad = nullptr;  // pinned, GRAD_SLOTS floats
  int step = 0;
};

namespace dc_core {
extern thread_local std::string g_last_error;  // text of dc_last_error (api.hip)
}  // namespace dc_core

namespace {

template <class F>
dc_status mlp_guarded(dc_mlp* m, F&& f) {
  if (!m) return DC_E_ARG;
  try {
    return f();
  } catch (const DeviceError& e) {
    dc_core::g_last_error = e.what();
    return (e.code == hipErrorOutOfMemory || e.code == hipErrorMemoryAllocation) ? DC_E_OOM
                                                                                : DC_E_DEVICE;
  } catch (const std::bad_alloc&) {
    return DC_E_OOM;
  } catch (...) {
    return DC_E_DEVICE;
  }
}

void upload_weights(dc_mlp* m, const float* w) {
  m->w.ensure(MLP_P * 4);
  m->m.ensure(MLP_P * 4);
  m->v.ensure(MLP_P * 4);
  m->wq.ensure(MLP_P * 2);
  DC_HIP(hipMemcpyAsync(m->w.p, w, MLP_P * 4, hipMemcpyHostToDevice, m->st));
  DC_HIP(hipMemsetAsync(m->m.p, 0, MLP_P * 4, m->st));
  DC_HIP(hipMemsetAsync(m->v.p, 0, MLP_P * 4, m->st));
  k_to_bf16<<<int(ceil_div(MLP_P, TPB)), TPB, 0, m->st>>>(m->w.as<float>(), MLP_P,
                                                          m->wq.as<uint16_t>());
  DC_LAUNCH_CHECK();
  DC_HIP(hipStreamSynchronize(m->st));
  m->step = 0;
}

void run_grad(dc_mlp* m, const uint16_t* X, const uint8_t* y, int64_t n, float pw) {
  m->partial.ensure(size_t(mlp_partial_floats(n)) * 4);
  m->grad.ensure(GRAD_SLOTS * 4);
  mlp_grad(m->wq.as<uint16_t>(), X, y, n, pw, m->partial.as<float>(), m->grad.as<float>(), m->st);
}

}  // namespace

extern "C" {

dc_status dc_mlp_create(dc_mlp** out, const float* w, void* stream) {
  if (!out || !w) return DC_E_ARG;
  *out = nullptr;
  dc_mlp* m = new (std::nothrow) dc_mlp();
  if (!m) return DC_E_OOM;
  m->st = static_cast<hipStream_t>(stream);
  dc_status s = mlp_guarded(m, [&] {
    DC_HIP(hipHostMalloc(reinterpret_cast<void**>(&m->hgrad), GRAD_SLOTS * 4));
    (void)scratch_on_current_device();  // set-up of dc_mlp_grad_noalloc's scratch
    upload_weights(m, w);
    return DC_OK;
  });
  if (s != DC_OK) {
    dc_mlp_destroy(m);
    return s;
  }
  *out = m;
  return DC_OK;
}

dc_status dc_mlp_set_weights(dc_mlp* m, const float* w) {
  if (!w) return DC_E_ARG;
  return mlp_guarded(m, [&] {
    upload_weights(m, w);
    return DC_OK;
  });
}

dc_status dc_mlp_get_weights(dc_mlp* m, float* w) {
  if (!w) return DC_E_ARG;
  return mlp_guarded(m, [&] {
    DC_HIP(hipMemcpyAsync(w, m->w.p, MLP_P * 4, hipMemcpyDeviceToHost, m->st));
    DC_HIP(hipStreamSynchronize(m->st));
    return DC_OK;
  });
}

dc_status dc_mlp_forward(dc_mlp* m, const uint16_t* X, int64_t n, float* logits) {
  if (n < 0 || (n > 0 && (!X || !logits))) return DC_E_ARG;
  return mlp_guarded(m, [&] {
    mlp_forward(m->wq.as<uint16_t>(), X, n, logits, m->st);
    DC_HIP(hipStreamSynchronize(m->st));
    return DC_OK;
  });
}

dc_status dc_mlp_grad(dc_mlp* m, const uint16_t* X, const uint8_t* y, int64_t n,
                      float pos_weight, float* grad, double* loss) {
  if (n < 1 || !X || !y || !(pos_weight > 0.f)) return DC_E_ARG;
  return mlp_guarded(m, [&] {
    run_grad(m, X, y, n, pos_weight);
    DC_HIP(hipMemcpyAsync(m->hgrad, m->grad.p, GRAD_SLOTS * 4, hipMemcpyDeviceToHost, m->st));
    DC_HIP(hipStreamSynchronize(m->st));
    if (grad) std::memcpy(grad, m->hgrad, MLP_P * 4);
    if (loss) *loss = double(m->hgrad[MLP_P]) / double(n);
    return DC_OK;
  });
}

dc_status dc_mlp_grad_noalloc(dc_mlp* m, const uint16_t* X, const uint8_t* y, int64_t n,
                              float pos_weight, float* grad, double* loss) {
  if (n < 1 || !X || !y || !(pos_weight > 0.f)) return DC_E_ARG;
  return mlp_guarded(m, [&] {
    const int64_t partial = mlp_partial_floats(n);
    if (partial > int64_t(NOALLOC_PARTIAL)) {
      dc_core::g_last_error = "dc_mlp_grad_noalloc: " + std::to_string(partial) +
                    " partial sums exceed the fixed scratch of " +
                    std::to_string(NOALLOC_PARTIAL);
      return DC_E_ARG;
    }
    float* base = scratch_on_current_device();
    float* g = base + NOALLOC_PARTIAL;
    mlp_grad(m->wq.as<uint16_t>(), X, y, n, pos_weight, base, g, m->st);
    DC_HIP(hipMemcpyAsync(m->hgrad, g, GRAD_SLOTS * 4, hipMemcpyDeviceToHost, m->st));
    DC_HIP(hipStreamSynchronize(m->st));
    if (grad) std::memcpy(grad, m->hgrad, MLP_P * 4);
    if (loss) *loss = double(m->hgrad[MLP_P]) / double(n);
    return DC_OK;
  });
}

dc_status dc_mlp_train_step(dc_mlp* m, const uint16_t* X, const uint8_t* y, int64_t n,
                            float pos_weight, float lr, double* loss) {
  if (n < 1 || !X || !y || !(pos_weight > 0.f) || !(lr > 0.f)) return DC_E_ARG;
  return mlp_guarded(m, [&] {
    run_grad(m, X, y, n, pos_weight);
    m->step += 1;
    mlp_adam(m->w.as<float>(), m->m.as<float>(), m->v.as<float>(), m->grad.as<float>(), m->step,
             lr, m->wq.as<uint16_t>(), m->st);
    if (loss)
      DC_HIP(hipMemcpyAsync(m->hgrad + MLP_P, m->grad.as<float>() + MLP_P, 4,
                            hipMemcpyDeviceToHost, m->st));
    DC_HIP(hipStreamSynchronize(m->st));
    if (loss) *loss = double(m->hgrad[MLP_P]) / double(n);
    return DC_OK;
  });
}

void dc_mlp_destroy(dc_mlp* m) {
  if (!m) return;
  if (m->st) (void)hipStreamSynchronize(m->st);
  if (m->hgrad) (void)hipHostFree(m->hgrad);
  delete m;
}

}  // extern "C"
