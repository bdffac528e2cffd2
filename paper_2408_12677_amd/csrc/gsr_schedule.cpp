// Keyframe-list optimisation schedule (Sec. III-B-3; settings of Sec. IV-A).  Host code
// only: it decides which views the optimisation iterations of a time step render.
//
// The number of Gaussians the seeding of a frame adds measures the frame's information
// gain.  A frame whose count exceeds the threshold is a keyframe: it joins the list and
// gets m iterations.  Any other frame gets n iterations, and the remaining m - n go to
// keyframes drawn at random from the list (the first m - n after a shuffle), one each.
// The shuffle orders the list by counter-based SplitMix64 keys (Steele, Lea and Flood,
// 2014), so the draw is reproducible from (seed, frame) alone.
#include <algorithm>
#include <cstdint>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "gsr.h"

struct gsr_schedule {
  gsr_schedule_settings s{};
  std::vector<int64_t> keyframes;
  std::string err;
};

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;  // SplitMix64's increment

// SplitMix64's output function (Stafford's Mix13).
uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// The k-th output (k >= 1) of SplitMix64 seeded with `seed`.
uint64_t splitmix64(uint64_t seed, uint64_t k) { return mix64(seed + k * kGolden); }

}  // namespace

extern "C" {

gsr_status gsr_schedule_create(const gsr_schedule_settings* s, gsr_schedule** out) {
  if (!s || !out) return GSR_EINVAL;
  *out = nullptr;
  if (s->n < 0 || s->m < s->n || s->m > 1000000) return GSR_EINVAL;
  gsr_schedule* h = new (std::nothrow) gsr_schedule;
  if (!h) return GSR_ENOMEM;
  h->s = *s;
  *out = h;
  return GSR_OK;
}

gsr_status gsr_schedule_free(gsr_schedule* h) {
  if (!h) return GSR_EINVAL;
  delete h;
  return GSR_OK;
}

gsr_status gsr_schedule_step(gsr_schedule* h, int64_t frame, int64_t new_gaussians, int64_t* iters, int32_t cap,
                             int32_t* count, int32_t* is_keyframe) {
  if (!h || !iters || !count || frame < 0 || new_gaussians < 0) return GSR_EINVAL;
  const gsr_schedule_settings& s = h->s;
  if (cap < s.m) return GSR_EINVAL;  // m iterations always fit
  const bool kf = new_gaussians > s.threshold;
  int32_t c = 0;
  if (kf) {
    try {
      h->keyframes.push_back(frame);
    } catch (...) {
      return GSR_ENOMEM;
    }
    for (int32_t i = 0; i < s.m; ++i) iters[c++] = frame;
  } else {
    for (int32_t i = 0; i < s.n; ++i) iters[c++] = frame;
    const size_t L = h->keyframes.size();
    const size_t draw = std::min<size_t>(size_t(s.m - s.n), L);
    if (draw > 0) {
      // key of list entry i: the (i+1)-th output of the stream seeded by the (frame+1)-th
      // output of the schedule's seed; order by (key, i)
      const uint64_t stream = splitmix64(s.seed, uint64_t(frame) + 1);
      std::vector<std::pair<uint64_t, uint64_t>> keyed;
      try {
        keyed.resize(L);
      } catch (...) {
        return GSR_ENOMEM;
      }
      for (size_t i = 0; i < L; ++i) keyed[i] = {splitmix64(stream, uint64_t(i) + 1), uint64_t(i)};
      std::partial_sort(keyed.begin(), keyed.begin() + std::ptrdiff_t(draw), keyed.end());
      for (size_t i = 0; i < draw; ++i) iters[c++] = h->keyframes[keyed[i].second];
    }
    if (s.store_all) {
      try {
        h->keyframes.push_back(frame);
      } catch (...) {
        return GSR_ENOMEM;
      }
    }
  }
  *count = c;
  if (is_keyframe) *is_keyframe = kf ? 1 : 0;
  return GSR_OK;
}

gsr_status gsr_schedule_keyframes(const gsr_schedule* h, int64_t* out, int64_t cap, int64_t* count) {
  if (!h || !count) return GSR_EINVAL;
  const int64_t L = int64_t(h->keyframes.size());
  *count = L;
  if (out) {
    if (cap < L) return GSR_EINVAL;
    std::copy(h->keyframes.begin(), h->keyframes.end(), out);
  }
  return GSR_OK;
}

}  // extern "C"
