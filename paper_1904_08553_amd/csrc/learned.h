// learned.h -- the learned screener: feature assembly, the 8-64-64-1
// network on the matrix cores, training kernels.  An extension of the
// method (the paper has no learned component).
#pragma once

#include "dc_louvain.h"

namespace dc {

constexpr int MLP_IN = DC_MLP_INPUTS;
constexpr int MLP_HID = DC_MLP_HIDDEN;
constexpr int MLP_P = DC_MLP_PARAMS;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + MLP_HID * MLP_IN;
constexpr int OFF_W2 = OFF_B1 + MLP_HID;
constexpr int OFF_B2 = OFF_W2 + MLP_HID * MLP_HID;
constexpr int OFF_W3 = OFF_B2 + MLP_HID;
constexpr int OFF_B3 = OFF_W3 + MLP_HID;
constexpr int GRAD_SLOTS = MLP_P + 1;  // gradient, then the loss sum
static_assert(OFF_B3 + 1 == MLP_P, "parameter layout");

// bfloat16 bit pattern of an fp32 value, round to nearest even (finite input).
__host__ __device__ inline uint16_t bf16_bits(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  return uint16_t((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// Features of the touched vertices T[0..cnt): X[idx][8] as bfloat16 bits,
// each feature one correctly rounded fp64 division of exact integers,
// then fp64 -> fp32 -> bfloat16 (nearest even at both steps).
void assemble_features(const int32_t* T, int64_t cnt, const int32_t* k, const int32_t* kprev,
                       const int32_t* cptr, const int32_t* f_own, const long long* f_g1,
                       const long long* f_g2, const int32_t* a, const int32_t* C,
                       const uint8_t* Rds, long long two_m, uint16_t* X, hipStream_t st);

// y[idx] = 1 when Cl[T[idx]] != C[T[idx]].
void move_labels(const int32_t* T, int64_t cnt, const int32_t* Cl, const int32_t* C, uint8_t* y,
                 hipStream_t st);

// R[T[idx]] = 1 for logit[idx] >= theta (R cleared beforehand by the caller).
void select_by_score(const int32_t* T, int64_t cnt, const float* logits, float theta, uint8_t* R,
                     hipStream_t st);

// flag[v] = a[v] | b[v] (int32, b may be null) for a compaction scan.
void merge_flags(const uint8_t* a, const uint8_t* b, int32_t n, int32_t* flag, hipStream_t st);

// out[v] |= 1 for v in list[0..*count) and their neighbours (count on device,
// at most max_count).
void mark_touched(const int32_t* list, const int32_t* count, int64_t max_count,
                  const int32_t* off, const int2* adj, uint8_t* out, hipStream_t st);

// logits[n] of X[n][8] with the bfloat16 parameters wq[MLP_P].
void mlp_forward(const uint16_t* wq, const uint16_t* X, int64_t n, float* logits, hipStream_t st);

// Mean weighted BCE gradient (and loss) into grad[GRAD_SLOTS] (device),
// deterministic for a given n.  partial: scratch of mlp_partial_floats(n).
int64_t mlp_partial_floats(int64_t n);
void mlp_grad(const uint16_t* wq, const uint16_t* X, const uint8_t* y, int64_t n,
              float pos_weight, float* partial, float* grad, hipStream_t st);

// One Adam step on the fp32 master w (moments m, v), refreshing wq.
void mlp_adam(float* w, float* m, float* v, const float* grad, int step, float lr, uint16_t* wq,
              hipStream_t st);

}  // namespace dc
