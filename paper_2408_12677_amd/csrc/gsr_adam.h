// Adam over the Gaussian parameters: the per-element update shared by the standalone
// optimiser kernel and the backward projection kernels that apply it in place.
//
// The parameters are stored activated; the optimised variables are the means, the
// logarithms of the scales, the quaternions, the logits of the opacities and the SH
// coefficients.  Per element (Kingma and Ba, Algorithm 1):
//   m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
//   x <- x - lr (m / bc1) / (sqrt(v / bc2) + eps),  bc1 = 1 - b1^t, bc2 = 1 - b2^t,
// with g taken through the activation (scale: s dL/ds, opacity: o (1 - o) dL/do).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gsr {

enum AdamGroup { G_MEANS = 0, G_SCALES, G_QUATS, G_OPAC, G_SH, G_COUNT };

constexpr float kOpacityMin = 5.9604645e-08f;  // 2^-24
constexpr float kOpacityMax = 0.99999994f;     // 1 - 2^-24

struct AdamDev {
  float* p[G_COUNT];   // parameters, updated in place
  float* m[G_COUNT];   // first moments, parameter layouts
  float* v[G_COUNT];   // second moments
  const float* bc;     // device [bc1, bc2] of the current step (written by the step counter)
  float lr[G_COUNT + 1];  // means, log-scales, quaternions, opacity logits, SH DC, SH rest
  float b1, b2, eps;
  int on;
  const uint32_t* skip;  // device word or null: the fused update leaves everything unchanged when it is set
};

// Step counter words (device, caller-owned): [0] steps taken (u32), [1] bc1, [2] bc2.
constexpr int kAdamStateWords = 4;

__device__ inline float adam_move(float x, float g, float& m, float& v, float lr, const AdamDev& a, float bc1,
                                  float bc2) {
#pragma clang fp contract(off)  // one rounding per operation: every code path gives the same bits
  m = a.b1 * m + (1.f - a.b1) * g;
  v = a.b2 * v + (1.f - a.b2) * (g * g);
  return x - lr * (m / bc1) / (__builtin_sqrtf(v / bc2) + a.eps);
}

// The new stored value of one element of group GRP (x stored, g = dL/dx stored), with
// its moments m, v updated in place.
template <int GRP>
__device__ inline float adam_value(float x, float g, float& m, float& v, float lr, const AdamDev& a, float bc1,
                                   float bc2) {
#pragma clang fp contract(off)
  if (GRP == G_SCALES) return expf(adam_move(logf(x), g * x, m, v, lr, a, bc1, bc2));
  if (GRP == G_OPAC) {
    const float w = adam_move(logf(x / (1.f - x)), g * x * (1.f - x), m, v, lr, a, bc1, bc2);
    return fminf(fmaxf(1.f / (1.f + expf(-w)), kOpacityMin), kOpacityMax);
  }
  return adam_move(x, g, m, v, lr, a, bc1, bc2);
}

// Element i of group GRP whose stored value x was already loaded.
template <int GRP>
__device__ inline void adam_apply(const AdamDev& a, int64_t i, float x, float g, float lr, float bc1, float bc2) {
  float m = a.m[GRP][i], v = a.v[GRP][i];
  const float out = adam_value<GRP>(x, g, m, v, lr, a, bc1, bc2);
  a.m[GRP][i] = m;
  a.v[GRP][i] = v;
  a.p[GRP][i] = out;
}

}  // namespace gsr
