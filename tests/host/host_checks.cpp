// Host-only units of the library (argument validation, keyframe schedule) driven with
// seeded random and edge-case arguments, for a build under the address and
// undefined-behaviour sanitizers.  Pointers handed to the validators are never
// dereferenced by them, so fake non-null addresses stand in for device buffers.
// Exit status 0 and "host checks ok" on success; the first failed expectation aborts.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <random>
#include <string>
#include <vector>

#include "gsr.h"
#include "gsr_validate.h"

using namespace gsr;

#define EXPECT(cond)                                                          \
  do {                                                                        \
    if (!(cond)) {                                                            \
      std::fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
      std::abort();                                                           \
    }                                                                         \
  } while (0)

namespace {

std::mt19937_64 rng(12345);

float pick(std::initializer_list<float> v) {
  std::uniform_int_distribution<size_t> d(0, v.size() - 1);
  return *(v.begin() + d(rng));
}

const float kNaN = std::numeric_limits<float>::quiet_NaN();
const float kInf = std::numeric_limits<float>::infinity();

float* fake(uintptr_t a) { return reinterpret_cast<float*>(a); }

gsr_settings good_settings() {
  gsr_settings s{};
  s.tile = 16;
  s.batch = 256;
  s.extent_k = 3.33f;
  s.lowpass = 0.3f;
  s.alpha_min = 1.f / 255.f;
  s.alpha_max = 0.99f;
  s.T_min = 1e-4f;
  s.guard = 0.15f;
  return s;
}

gsr_camera good_camera() {
  gsr_camera c{};
  c.width = 640;
  c.height = 480;
  c.fx = c.fy = 320.f;
  c.cx = 320.f;
  c.cy = 240.f;
  c.R[0] = c.R[4] = c.R[8] = 1.f;
  c.znear = 0.01f;
  return c;
}

void settings_cases() {
  std::string err;
  gsr_settings s = good_settings();
  EXPECT(check::settings(&s, err) == GSR_OK);
  EXPECT(check::settings(nullptr, err) == GSR_EINVAL && !err.empty());
  for (int i = 0; i < 20000; ++i) {
    gsr_settings t = good_settings();
    t.tile = int32_t(pick({8, 16, 32, 0, -16, 12, 64}));
    t.batch = int32_t(pick({128, 256, 0, 64, 512}));
    t.extent_k = pick({3.33f, 3.f, 0.f, -1.f, kNaN, kInf});
    t.lowpass = pick({0.3f, 0.f, -0.1f, kNaN});
    t.alpha_min = pick({1.f / 255.f, 0.f, -1e-3f, kNaN});
    t.alpha_max = pick({0.99f, 1.f, 0.f, 0.5f, kNaN});
    t.T_min = pick({1e-4f, 0.f, 1.f, -1.f, kNaN});
    t.guard = pick({0.15f, 0.f, -0.5f, kInf});
    t.flags = uint32_t(pick({0.f, 1.f, 2.f, 4.f, 7.f, 8.f, 1024.f}));
    const bool ok = (t.tile == 8 || t.tile == 16 || t.tile == 32) && (t.batch == 128 || t.batch == 256) &&
                    t.extent_k > 0.f && std::isfinite(t.extent_k) && t.lowpass >= 0.f && t.alpha_min >= 0.f &&
                    t.alpha_max > 0.f && t.alpha_max < 1.f && t.T_min >= 0.f && t.T_min < 1.f && t.guard >= 0.f &&
                    std::isfinite(t.guard) && (t.flags & ~7u) == 0u;
    err.clear();
    const gsr_status st = check::settings(&t, err);
    EXPECT((st == GSR_OK) == ok);
    EXPECT(st == GSR_OK || !err.empty());
  }
}

void gaussian_and_camera_cases() {
  std::string err;
  for (int i = 0; i < 20000; ++i) {
    gsr_gaussians g{};
    const int64_t ns[] = {0, 1, 500000, -1, (int64_t(1) << 32) - 1, int64_t(1) << 32, int64_t(1) << 40};
    g.n = ns[rng() % 7];
    g.sh_degree = int32_t(rng() % 6) - 1;
    g.means = rng() % 8 ? fake(0x1000) : nullptr;
    g.scales = rng() % 8 ? fake(0x2000) : nullptr;
    g.quats = rng() % 8 ? fake(rng() % 4 ? 0x3000 : 0x3004) : nullptr;
    g.opacities = rng() % 8 ? fake(0x4000) : nullptr;
    g.sh = rng() % 8 ? fake(0x5000) : nullptr;
    const int views = int(rng() % 20);
    const bool ptrs = g.means && g.scales && g.quats && g.opacities && g.sh;
    const bool ok = g.n >= 0 && g.sh_degree >= 0 && g.sh_degree <= 3 &&
                    (g.n == 0 || (ptrs && (reinterpret_cast<uintptr_t>(g.quats) & 15u) == 0)) &&
                    g.n < (int64_t(1) << 32) && int64_t(views) * g.n < (int64_t(1) << 32);
    err.clear();
    EXPECT((check::gaussians(&g, views, err) == GSR_OK) == ok);
  }
  for (int i = 0; i < 20000; ++i) {
    gsr_camera c = good_camera();
    c.width = int32_t(pick({640.f, 1.f, 0.f, -5.f, 8192.f, 8193.f}));
    c.height = int32_t(pick({480.f, 1.f, 0.f, 9000.f}));
    c.fx = pick({320.f, 0.f, -1.f, kNaN, kInf});
    c.cy = pick({240.f, -3.f, kNaN, kInf});
    c.znear = pick({0.01f, 0.f, -1.f, kNaN});
    c.R[rng() % 9] = pick({1.f, 0.f, kNaN});
    c.t[rng() % 3] = pick({0.f, 2.f, kInf});
    bool finite = true;
    for (float x : c.R) finite = finite && std::isfinite(x);
    for (float x : c.t) finite = finite && std::isfinite(x);
    const bool ok = c.width >= 1 && c.width <= 8192 && c.height >= 1 && c.height <= 8192 && c.fx > 0.f &&
                    std::isfinite(c.fx) && std::isfinite(c.cy) && c.znear > 0.f && finite;
    err.clear();
    EXPECT((check::camera(c, i % 16, err) == GSR_OK) == ok);
  }
  // forward_args: view count, NULL arrays, a NULL colour output in the last view
  gsr_gaussians g{};
  g.n = 10;
  g.means = g.scales = g.opacities = g.sh = fake(0x1000);
  g.quats = fake(0x2000);
  gsr_settings s = good_settings();
  std::vector<gsr_camera> cams(GSR_MAX_VIEWS + 1, good_camera());
  std::vector<gsr_view_out> outs(GSR_MAX_VIEWS + 1, gsr_view_out{fake(0x9000), nullptr, nullptr});
  for (int V = -1; V <= GSR_MAX_VIEWS + 1; ++V) {
    err.clear();
    EXPECT((check::forward_args(&g, cams.data(), V, &s, outs.data(), err) == GSR_OK) == (V >= 1 && V <= GSR_MAX_VIEWS));
  }
  EXPECT(check::forward_args(&g, nullptr, 1, &s, outs.data(), err) == GSR_EINVAL);
  EXPECT(check::forward_args(&g, cams.data(), 1, &s, nullptr, err) == GSR_EINVAL);
  outs[3].color = nullptr;
  EXPECT(check::forward_args(&g, cams.data(), 4, &s, outs.data(), err) == GSR_EINVAL);
  EXPECT(check::forward_args(&g, cams.data(), 3, &s, outs.data(), err) == GSR_OK);
}

void optimiser_seed_tsdf_cases() {
  std::string err;
  for (int i = 0; i < 20000; ++i) {
    gsr_adam a{};
    float* arrs[10];
    for (float*& p : arrs) p = rng() % 16 ? fake(0x1000) : nullptr;
    a.m = gsr_gaussian_grads{arrs[0], arrs[1], arrs[2], arrs[3], arrs[4]};
    a.v = gsr_gaussian_grads{arrs[5], arrs[6], arrs[7], arrs[8], arrs[9]};
    a.state = rng() % 16 ? reinterpret_cast<uint32_t*>(0x8000) : nullptr;
    a.lr_means = pick({1.6e-4f, 0.f, -1e-3f, kNaN, kInf});
    a.lr_sh_rest = pick({1.25e-4f, kInf});
    a.beta1 = pick({0.9f, 0.f, 1.f, -0.1f, kNaN});
    a.beta2 = pick({0.999f, 1.f});
    a.eps = pick({1e-15f, 0.f, -1.f, kInf});
    bool ptrs = a.state != nullptr;
    for (float* p : arrs) ptrs = ptrs && p;
    const bool ok = ptrs && a.lr_means >= 0.f && std::isfinite(a.lr_means) && std::isfinite(a.lr_sh_rest) &&
                    a.beta1 >= 0.f && a.beta1 < 1.f && a.beta2 < 1.f && a.eps >= 0.f && std::isfinite(a.eps);
    err.clear();
    EXPECT((check::adam(&a, err) == GSR_OK) == ok);
  }
  EXPECT(check::adam(nullptr, err) == GSR_EINVAL);
  for (int i = 0; i < 20000; ++i) {
    gsr_seed_settings s{};
    s.measure = int32_t(rng() % 4) - 1;
    s.threshold = pick({0.1f, 0.f, -0.1f, kNaN});
    s.min_side = int32_t(pick({1.f, 2.f, 3.f, 4.f, 64.f, 128.f, 0.f}));
    s.opacity = pick({0.5f, 0.f, 1.f, 1.5f, kNaN});
    s.sh_degree = int32_t(rng() % 6) - 1;
    const int64_t capacity = int64_t(rng() % 3) - 1;
    gsr_seed_out out{};
    if (rng() % 4) out = gsr_seed_out{fake(0x10), fake(0x20), fake(0x30), fake(0x40), fake(0x50), nullptr};
    const bool ms = s.min_side == 1 || s.min_side == 2 || s.min_side == 4 || s.min_side == 64;
    const bool ok = (s.measure == 0 || s.measure == 1) && ms && s.threshold >= 0.f && s.opacity >= 0.f &&
                    s.opacity <= 1.f && s.sh_degree >= 0 && s.sh_degree <= 3 && capacity >= 0 &&
                    (capacity == 0 || out.means);
    err.clear();
    EXPECT((check::seed_settings(&s, capacity, &out, err) == GSR_OK) == ok);
  }
  for (int i = 0; i < 20000; ++i) {
    gsr_tsdf_settings s{0.01f, 0.08f, 100.f, 0.01f, GSR_TSDF_EQ9};
    s.voxel = pick({0.01f, 0.f, -1.f, kNaN, kInf});
    s.w_max = pick({100.f, 1.f, 0.5f, kInf});
    s.weighting = int32_t(rng() % 3);
    const int64_t mbs[] = {1, 40000, 0, -3, int64_t(1) << 28, (int64_t(1) << 28) + 1};
    const int64_t mb = mbs[rng() % 6];
    int64_t slots = -1;
    const bool ok = s.voxel > 0.f && std::isfinite(s.voxel) && s.w_max >= 1.f && std::isfinite(s.w_max) &&
                    s.weighting <= 1 && mb >= 1 && mb <= (int64_t(1) << 28);
    err.clear();
    const gsr_status st = check::tsdf_settings(&s, mb, &slots, err);
    EXPECT((st == GSR_OK) == ok);
    if (ok) EXPECT(slots >= 1024 && slots >= 2 * mb && (slots & (slots - 1)) == 0);
  }
}

void schedule_cases() {
  for (int trial = 0; trial < 300; ++trial) {
    gsr_schedule_settings s{};
    s.n = int32_t(rng() % 12) - 1;
    s.m = s.n + int32_t(rng() % 12) - 2;
    s.threshold = int64_t(rng() % 200) - 20;
    s.store_all = int32_t(rng() % 2);
    s.seed = rng();
    gsr_schedule* h = nullptr;
    const gsr_status st = gsr_schedule_create(&s, &h);
    if (s.n < 0 || s.m < s.n) {
      EXPECT(st == GSR_EINVAL && h == nullptr);
      continue;
    }
    EXPECT(st == GSR_OK && h);
    std::vector<int64_t> iters(size_t(s.m) + 1, -7);
    int64_t keyframes = 0;
    for (int64_t frame = 0; frame < 200; ++frame) {
      const int64_t added = int64_t(rng() % 400);
      int32_t count = -1, kf = -1;
      EXPECT(gsr_schedule_step(h, frame, added, iters.data(), s.m - 1, &count, &kf) == GSR_EINVAL);  // m must fit
      EXPECT(gsr_schedule_step(h, frame, added, iters.data(), s.m, &count, &kf) == GSR_OK);
      EXPECT(count >= 0 && count <= s.m);
      EXPECT(kf == (added > s.threshold ? 1 : 0));
      if (kf) {
        EXPECT(count == s.m);
        ++keyframes;
      }
      for (int32_t i = 0; i < count; ++i) EXPECT(iters[size_t(i)] >= 0 && iters[size_t(i)] <= frame);
      if (!kf || s.store_all) keyframes += (!kf && s.store_all) ? 1 : 0;
    }
    int64_t L = -1;
    EXPECT(gsr_schedule_keyframes(h, nullptr, 0, &L) == GSR_OK && L == keyframes);
    std::vector<int64_t> list(size_t(L) + 1);
    if (L > 0) EXPECT(gsr_schedule_keyframes(h, list.data(), L - 1, &L) == GSR_EINVAL);
    EXPECT(gsr_schedule_keyframes(h, list.data(), L, &L) == GSR_OK);
    for (int64_t i = 1; i < L; ++i) EXPECT(list[size_t(i)] > list[size_t(i - 1)]);
    EXPECT(gsr_schedule_step(h, -1, 1, iters.data(), s.m, nullptr, nullptr) == GSR_EINVAL);
    EXPECT(gsr_schedule_free(h) == GSR_OK);
  }
  EXPECT(gsr_schedule_free(nullptr) == GSR_EINVAL);
  EXPECT(gsr_schedule_create(nullptr, nullptr) == GSR_EINVAL);
}

}  // namespace

int main() {
  settings_cases();
  gaussian_and_camera_cases();
  optimiser_seed_tsdf_cases();
  schedule_cases();
  std::printf("host checks ok\n");
  return 0;
}
