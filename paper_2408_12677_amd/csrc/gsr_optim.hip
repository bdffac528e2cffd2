// Optimiser step over the Gaussian parameters (Sec. III-B-3: the parameters are optimised
// directly by gradient descent; Adam, Kingma and Ba Algorithm 1, is the optimiser taken).
//
// k_adam_tick advances the caller's step counter and writes the two bias corrections of
// the new step; k_adam then updates every element of every parameter group in place.
// The update is elementwise and HBM bound: per element it reads the stored value, its
// gradient and both moments and writes the value and the moments back (28 bytes).  The
// groups are separate arrays, so the grid is cut into per-group block ranges and each
// thread moves four consecutive elements with 16-byte loads where the arrays allow it.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gsr_adam.h"
#include "gsr_internal.h"

namespace gsr {
namespace {

constexpr int kAdamThreads = 256;
constexpr int kAdamPer = 4;  // elements per thread
constexpr int kAdamBlock = kAdamThreads * kAdamPer;

__global__ __launch_bounds__(64) void k_adam_tick(uint32_t* state, float b1, float b2, const uint32_t* skip) {
  const int lane = threadIdx.x;
  if (lane != 0) return;
  if (skip && *skip) return;  // a step that overflowed its capacities updates nothing
  const uint32_t t = state[lane] + 1u;
  state[lane] = t;
  float* bc = reinterpret_cast<float*>(state + 1);
  bc[lane] = float(1.0 - ::pow(double(b1), double(t)));
  bc[lane + 1] = float(1.0 - ::pow(double(b2), double(t)));
}

struct AdamSeg {
  const float* g;        // gradient of the group
  int64_t n;             // elements
  uint32_t first_block;  // first block of the group's range
  int32_t kk;            // SH group: coefficients per Gaussian (K * 3); the first 3 are DC
  int32_t grp;
  int32_t vec;           // all four arrays 16-byte aligned
};

struct AdamPlan {
  AdamSeg seg[G_COUNT];
  int32_t nseg;
};

// Learning rate of an element at position j of its row (the SH rows start with the
// three DC coefficients).
template <int GRP>
__device__ inline float rate(const AdamDev& a, int j) {
  if (GRP != G_SH) return a.lr[GRP];
  return j < 3 ? a.lr[G_SH] : a.lr[G_SH + 1];
}

template <int GRP>
__device__ void adam_range(const AdamDev& a, const AdamSeg& sg, uint32_t local_block) {
  const int64_t e0 = (int64_t(local_block) * kAdamThreads + threadIdx.x) * kAdamPer;
  if (e0 >= sg.n) return;
  const float bc1 = a.bc[0], bc2 = a.bc[1];
  int j[kAdamPer];  // row positions of the thread's elements
  j[0] = GRP == G_SH ? int(e0 % sg.kk) : 0;
#pragma unroll
  for (int k = 1; k < kAdamPer; ++k) j[k] = (GRP == G_SH && j[k - 1] + 1 == sg.kk) ? 0 : j[k - 1] + 1;
  if (sg.vec && e0 + kAdamPer <= sg.n) {
    float4 x = *reinterpret_cast<const float4*>(a.p[GRP] + e0);
    const float4 g = *reinterpret_cast<const float4*>(sg.g + e0);
    float4 m = *reinterpret_cast<const float4*>(a.m[GRP] + e0);
    float4 v = *reinterpret_cast<const float4*>(a.v[GRP] + e0);
    x.x = adam_value<GRP>(x.x, g.x, m.x, v.x, rate<GRP>(a, j[0]), a, bc1, bc2);
    x.y = adam_value<GRP>(x.y, g.y, m.y, v.y, rate<GRP>(a, j[1]), a, bc1, bc2);
    x.z = adam_value<GRP>(x.z, g.z, m.z, v.z, rate<GRP>(a, j[2]), a, bc1, bc2);
    x.w = adam_value<GRP>(x.w, g.w, m.w, v.w, rate<GRP>(a, j[3]), a, bc1, bc2);
    *reinterpret_cast<float4*>(a.p[GRP] + e0) = x;
    *reinterpret_cast<float4*>(a.m[GRP] + e0) = m;
    *reinterpret_cast<float4*>(a.v[GRP] + e0) = v;
    return;
  }
#pragma unroll
  for (int k = 0; k < kAdamPer; ++k) {
    const int64_t e = e0 + k;
    if (e < sg.n) adam_apply<GRP>(a, e, a.p[GRP][e], sg.g[e], rate<GRP>(a, j[k]), bc1, bc2);
  }
}

__global__ __launch_bounds__(kAdamThreads) void k_adam(AdamDev a, AdamPlan plan) {
  // the group whose block range holds this block (uniform selects, no indexed copy)
  AdamSeg sg = plan.seg[0];
#pragma unroll
  for (int i = 1; i < G_COUNT; ++i)
    if (i < plan.nseg && blockIdx.x >= plan.seg[i].first_block) sg = plan.seg[i];
  const uint32_t lb = blockIdx.x - sg.first_block;
  switch (sg.grp) {
    case G_MEANS: adam_range<G_MEANS>(a, sg, lb); break;
    case G_SCALES: adam_range<G_SCALES>(a, sg, lb); break;
    case G_QUATS: adam_range<G_QUATS>(a, sg, lb); break;
    case G_OPAC: adam_range<G_OPAC>(a, sg, lb); break;
    default: adam_range<G_SH>(a, sg, lb); break;
  }
}

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

hipError_t launch_adam_tick(uint32_t* state, float b1, float b2, const uint32_t* skip, hipStream_t s) {
  k_adam_tick<<<1, 64, 0, s>>>(state, b1, b2, skip);
  return hipGetLastError();
}

hipError_t launch_adam(const AdamDev& a, const float* const grads[G_COUNT], int64_t n, int deg, hipStream_t s) {
  const int64_t per[G_COUNT] = {3, 3, 4, 1, int64_t(deg + 1) * (deg + 1) * 3};
  AdamPlan plan{};
  int64_t blocks = 0;
  for (int g = 0; g < G_COUNT; ++g) {
    const int64_t cnt = n * per[g];
    if (cnt == 0) continue;
    AdamSeg& sg = plan.seg[plan.nseg++];
    sg.g = grads[g];
    sg.n = cnt;
    sg.first_block = uint32_t(blocks);
    sg.kk = int32_t(per[G_SH]);
    sg.grp = g;
    sg.vec = aligned16(a.p[g]) && aligned16(a.m[g]) && aligned16(a.v[g]) && aligned16(grads[g]);
    blocks += (cnt + kAdamBlock - 1) / kAdamBlock;
  }
  if (blocks == 0) return hipSuccess;
  if (blocks > int64_t(0x7fffffff)) return hipErrorInvalidValue;
  k_adam<<<unsigned(blocks), kAdamThreads, 0, s>>>(a, plan);
  return hipGetLastError();
}

}  // namespace gsr
