// Device-side pieces of the splitter-scoring network shared by the training
// kernels and the refinement kernel: parameter layout, bf16 rounding, LDS
// staging and the one-wave-per-row forward pass.
#pragma once

#include <stdint.h>

#include "internal.h"

namespace bisim {

constexpr int kMlpH = 64;     // hidden width (= wave size: lane j is unit j)
constexpr int kMlpMaxF = 32;  // largest supported input width
constexpr int kPolicyF = 19;  // block features used by the learned splitter

// flat parameter layout: W1 [H][F], b1 [H], W2 [H][H], b2 [H], w3 [H], b3 [1]
struct MlpOffsets {
  int64_t W1, b1, W2, b2, w3, b3, total;
};
__host__ __device__ inline MlpOffsets mlp_offsets(int F) {
  MlpOffsets o;
  o.W1 = 0;
  o.b1 = o.W1 + (int64_t)kMlpH * F;
  o.W2 = o.b1 + kMlpH;
  o.b2 = o.W2 + (int64_t)kMlpH * kMlpH;
  o.w3 = o.b2 + kMlpH;
  o.b3 = o.w3 + kMlpH;
  o.total = o.b3 + 1;
  return o;
}

// round to nearest even into bf16 (NaN inputs are not produced here)
__device__ __forceinline__ uint16_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ float bf16_rne(float f) { return bf16_to_f(bf16_bits(f)); }

// LDS copy of the bf16 parameters as fp32; W1 and W2 also transposed so that
// lane j reading unit j's weights touches consecutive words.
struct MlpLds {
  float* W1T;  // [F][H]
  float* b1;   // [H]
  float* W2T;  // [H][H]: W2T[i*H + j] = W2[j][i]
  float* W2;   // [H][H]: row-major W2[j][i]
  float* b2;
  float* w3;
  float* b3;   // [1] (+3 pad)
  float* end;
};
__host__ __device__ inline int64_t mlp_lds_floats(int F) {
  return (int64_t)F * kMlpH + kMlpH + 2 * kMlpH * kMlpH + 2 * kMlpH + 4;
}
__device__ __forceinline__ MlpLds mlp_lds_layout(float* base, int F) {
  MlpLds L;
  L.W1T = base;
  L.b1 = L.W1T + F * kMlpH;
  L.W2T = L.b1 + kMlpH;
  L.W2 = L.W2T + kMlpH * kMlpH;
  L.b2 = L.W2 + kMlpH * kMlpH;
  L.w3 = L.b2 + kMlpH;
  L.b3 = L.w3 + kMlpH;
  L.end = L.b3 + 4;
  return L;
}
// whole workgroup cooperates; caller synchronises afterwards
__device__ __forceinline__ void mlp_stage(const MlpLds& L, const uint16_t* __restrict__ w, int F) {
  const MlpOffsets o = mlp_offsets(F);
  for (int i = threadIdx.x; i < kMlpH * F; i += blockDim.x) {
    const int j = i / F, f = i % F;
    L.W1T[f * kMlpH + j] = bf16_to_f(w[o.W1 + i]);
  }
  for (int i = threadIdx.x; i < kMlpH * kMlpH; i += blockDim.x) {
    const int j = i / kMlpH, q = i % kMlpH;
    const float v = bf16_to_f(w[o.W2 + i]);
    L.W2[i] = v;
    L.W2T[q * kMlpH + j] = v;
  }
  for (int i = threadIdx.x; i < kMlpH; i += blockDim.x) {
    L.b1[i] = bf16_to_f(w[o.b1 + i]);
    L.b2[i] = bf16_to_f(w[o.b2 + i]);
    L.w3[i] = bf16_to_f(w[o.w3 + i]);
  }
  if (threadIdx.x == 0) L.b3[0] = bf16_to_f(w[o.b3]);
}

// Forward pass of one row by one wave; input feature f is held by lane f
// (xlane).  Returns the output on every lane; z1/z2 are lane j's
// pre-activations.
__device__ __forceinline__ float mlp_forward_lanes(const MlpLds& L, int F, float xlane, float* z1o,
                                                   float* z2o) {
  const int j = (int)lane();
  const float xr = bf16_rne(xlane);
  float z1 = L.b1[j];
  for (int f = 0; f < F; ++f) z1 = fmaf(L.W1T[f * kMlpH + j], __shfl(xr, f, kWave), z1);
  const float h1 = fmaxf(z1, 0.f);
  float z2 = L.b2[j];
#pragma unroll 16
  for (int i = 0; i < kMlpH; ++i) z2 = fmaf(L.W2T[i * kMlpH + j], __shfl(h1, i, kWave), z2);
  const float h2 = fmaxf(z2, 0.f);
  float y = L.w3[j] * h2;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) y += __shfl_xor(y, d, kWave);
  *z1o = z1;
  *z2o = z2;
  return y + L.b3[0];
}

// Same, input row read from memory.
__device__ __forceinline__ float mlp_row_forward(const MlpLds& L, int F, const float* xr,
                                                 float* z1o, float* z2o) {
  const int j = (int)lane();
  const float xl = j < F ? xr[j] : 0.f;
  return mlp_forward_lanes(L, F, xl, z1o, z2o);
}

// Priority level of a predicted log(1 + blocks split): 16 levels of width 1/3.
// The learned policy takes the smallest label of the highest non-empty level.
constexpr int kLevels = 16;
__device__ __forceinline__ uint32_t score_level(float y) {
  const float q = floorf(y * 3.0f);
  if (!(q > 0.f)) return 0u;  // also NaN
  return q >= (float)(kLevels - 1) ? (uint32_t)(kLevels - 1) : (uint32_t)q;
}

}  // namespace bisim
