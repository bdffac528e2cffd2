// gfx950 kernels of quadtree seeding and Gaussian initialisation (GSFusion Sec. III-B-2,
// Eq. 10).
//
//   k_seed<PASS>  one block of 256 threads per 64-pixel root cell.  Thread t owns the 4x4
//                 pixel block at Morton index t of the root, so the children of every
//                 cell are consecutive and the cell statistics of the whole quadtree
//                 (sides 64, 32, 16, 8, 4) form a Morton-ordered pyramid in LDS; sides 2
//                 and 1 stay in the thread.  A cell splits while its measure passes the
//                 threshold and its side exceeds the minimum; every thread walks its
//                 block's ancestors from the root to find the leaf that covers it, and
//                 the thread at a leaf's first Morton index (or the owner of a sub-block
//                 leaf) emits it, in depth-first order.  A leaf whose centre pixel has no
//                 valid depth yields no Gaussian.
//     PASS 0:     count the Gaussians of each root
//     PASS 1:     write them at the root's scanned offset: mean = T_WC pi^-1(u, D[u]),
//                 scale d (centre to top-left pixel at the centre's depth), identity
//                 rotation, opacity, and the DC SH coefficients from the pixel colour
//
// The statistics are binary64: the contrast measure (range of the mean of the three
// channels) selects values exactly, and the depth variance is the one-pass form.
#include "gsr_internal.h"

namespace gsr {
namespace {

constexpr int kSeedRoot = 64;
constexpr double kY00 = 0.28209479177387814347;  // 1 / (2 sqrt(pi))

struct CellStat {
  int n;     // samples: pixels (contrast) or valid depths (variance)
  double a;  // min grey (contrast) or sum of depths (variance)
  double b;  // max grey (contrast) or sum of squared depths (variance)
};

__device__ __forceinline__ CellStat stat_empty(int measure) {
  return measure == GSR_SEED_CONTRAST ? CellStat{0, 1e300, -1e300} : CellStat{0, 0.0, 0.0};
}

__device__ __forceinline__ void stat_add(CellStat& s, const CellStat& o, int measure) {
  s.n += o.n;
  if (measure == GSR_SEED_CONTRAST) {
    s.a = fmin(s.a, o.a);
    s.b = fmax(s.b, o.b);
  } else {
    s.a += o.a;
    s.b += o.b;
  }
}

// one pixel's sample (an empty stat outside the image or without a valid depth)
__device__ __forceinline__ CellStat pixel_stat(const SeedImage& im, int x, int y, int measure) {
  CellStat s = stat_empty(measure);
  if (x >= im.W || y >= im.H) return s;
  const int64_t i = int64_t(y) * im.W + x;
  if (measure == GSR_SEED_CONTRAST) {
    const int64_t P = int64_t(im.W) * im.H;
    const double g = ((double(im.rgb[i]) + double(im.rgb[P + i])) + double(im.rgb[2 * P + i])) / 3.0;
    s = CellStat{1, g, g};
  } else {
    const double d = double(im.depth[i]);
    if (d > 0.0) s = CellStat{1, d, d * d};
  }
  return s;
}

__device__ __forceinline__ bool stat_splits(const CellStat& s, int side, const SeedRules& r) {
  if (s.n == 0 || side <= r.min_side) return false;
  if (r.measure == GSR_SEED_CONTRAST) return s.b - s.a >= double(r.threshold);
  const double inv = 1.0 / double(s.n);
  const double mean = s.a * inv;
  return s.b * inv - mean * mean > double(r.threshold);
}

__device__ __forceinline__ int morton_x(int t) {
  return (t & 1) | ((t >> 1) & 2) | ((t >> 2) & 4) | ((t >> 3) & 8);
}
__device__ __forceinline__ int morton_y(int t) { return morton_x(t >> 1); }

// Mean of the leaf's Gaussian: T_WC pi^-1(centre, D[centre]), i.e. R^T (p_c - t) for the
// world-to-camera (R, t), in binary64 and rounded once to binary32.
__device__ __forceinline__ void leaf_mean(const SeedImage& im, int xc, int yc, double d, float mean[3]) {
  const double pc[3] = {(double(xc) - im.cx) / im.fx * d, (double(yc) - im.cy) / im.fy * d, d};
  const double q0 = pc[0] - im.t[0], q1 = pc[1] - im.t[1], q2 = pc[2] - im.t[2];
#pragma unroll
  for (int c = 0; c < 3; ++c) mean[c] = float(double(im.R[c]) * q0 + double(im.R[3 + c]) * q1 + double(im.R[6 + c]) * q2);
}

// Whether the leaf (x0, y0, w, h) gets a Gaussian: its centre depth is valid and, with the
// map check on, the voxel nearest its mean was first observed by the latest fused frame
// (weight exactly 1; Sec. III-B-2).
__device__ __forceinline__ bool leaf_valid(const SeedImage& im, const SeedRules& r, int x0, int y0, int w, int h) {
  const int xc = x0 + w / 2, yc = y0 + h / 2;
  const float d = im.depth[int64_t(yc) * im.W + xc];
  if (!(d > 0.f)) return false;
  if (!r.check) return true;
  float mean[3];
  leaf_mean(im, xc, yc, double(d), mean);
  return voxel_weight_at(r.map, mean[0], mean[1], mean[2]) == 1.f;
}

__device__ void write_gaussian(const SeedImage& im, const SeedRules& r, const SeedOut& out, int64_t k, int x0,
                               int y0, int w, int h) {
  const int xc = x0 + w / 2, yc = y0 + h / 2;
  const int64_t i = int64_t(yc) * im.W + xc, P = int64_t(im.W) * im.H;
  const double d = double(im.depth[i]);
  const double ox = (double(xc - x0)) / im.fx * d, oy = (double(yc - y0)) / im.fy * d;
  const double scale = sqrt(ox * ox + oy * oy);
  float mean[3];
  leaf_mean(im, xc, yc, d, mean);
#pragma unroll
  for (int c = 0; c < 3; ++c) out.means[k * 3 + c] = mean[c];
#pragma unroll
  for (int c = 0; c < 3; ++c) out.scales[k * 3 + c] = float(scale);
  out.quats[k * 4] = 1.f;
  out.quats[k * 4 + 1] = 0.f;
  out.quats[k * 4 + 2] = 0.f;
  out.quats[k * 4 + 3] = 0.f;
  out.opac[k] = r.opacity;
  const int KK = (r.sh_degree + 1) * (r.sh_degree + 1) * 3;
  float* sh = out.sh + k * KK;
#pragma unroll
  for (int c = 0; c < 3; ++c) sh[c] = float((double(im.rgb[c * P + i]) - 0.5) / kY00);
  for (int j = 3; j < KK; ++j) sh[j] = 0.f;
  if (out.leaves) {
    out.leaves[k * 4] = x0;
    out.leaves[k * 4 + 1] = y0;
    out.leaves[k * 4 + 2] = w;
    out.leaves[k * 4 + 3] = h;
  }
}

__device__ __forceinline__ uint32_t seed_block_sum(uint32_t v, uint32_t* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const uint32_t tot = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return tot;
}

__device__ __forceinline__ uint32_t seed_block_excl_scan(uint32_t v, uint32_t* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t incl = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t u = __shfl_up(incl, off);
    if (lane >= off) incl += u;
  }
  if (lane == 63) red[w] = incl;
  __syncthreads();
  uint32_t pre = 0;
  for (int i = 0; i < w; ++i) pre += red[i];
  return pre + incl - v;
}

template <int PASS>
__global__ __launch_bounds__(256) void k_seed(SeedImage im, SeedRules r, uint32_t* root_counts, SeedOut out) {
  __shared__ CellStat s4[256], s8[64], s16[16], s32[4], s64[1];
  __shared__ uint32_t red[4];
  const int t = threadIdx.x;
  const int roots_x = (im.W + kSeedRoot - 1) / kSeedRoot;
  const int rx0 = (blockIdx.x % roots_x) * kSeedRoot, ry0 = (blockIdx.x / roots_x) * kSeedRoot;
  const int bx0 = rx0 + 4 * morton_x(t), by0 = ry0 + 4 * morton_y(t);
  // this thread's 4x4 block: its four 2x2 cells (Morton order) and the block
  CellStat p2[4];
  CellStat blk = stat_empty(r.measure);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    p2[u] = stat_empty(r.measure);
#pragma unroll
    for (int v = 0; v < 4; ++v)
      stat_add(p2[u], pixel_stat(im, bx0 + 2 * (u & 1) + (v & 1), by0 + 2 * (u >> 1) + (v >> 1), r.measure),
               r.measure);
    stat_add(blk, p2[u], r.measure);
  }
  s4[t] = blk;
  __syncthreads();
  if (t < 64) {
    CellStat c = s4[4 * t];
    for (int k = 1; k < 4; ++k) stat_add(c, s4[4 * t + k], r.measure);
    s8[t] = c;
  }
  __syncthreads();
  if (t < 16) {
    CellStat c = s8[4 * t];
    for (int k = 1; k < 4; ++k) stat_add(c, s8[4 * t + k], r.measure);
    s16[t] = c;
  }
  __syncthreads();
  if (t < 4) {
    CellStat c = s16[4 * t];
    for (int k = 1; k < 4; ++k) stat_add(c, s16[4 * t + k], r.measure);
    s32[t] = c;
  }
  __syncthreads();
  if (t == 0) {
    CellStat c = s32[0];
    for (int k = 1; k < 4; ++k) stat_add(c, s32[k], r.measure);
    s64[0] = c;
  }
  __syncthreads();
  // the leaf covering this block: walk down from the root while cells split
  int leaf_side = 0, shift = 8;
  bool dropped = false;
  {
    int side = kSeedRoot;
    for (int l = 0; l < 5; ++l, side >>= 1, shift -= 2) {
      const CellStat c = l == 0 ? s64[0] : l == 1 ? s32[t >> 6] : l == 2 ? s16[t >> 4] : l == 3 ? s8[t >> 2] : s4[t];
      if (!stat_splits(c, side, r)) {
        leaf_side = side;
        dropped = c.n == 0;
        break;
      }
    }
  }
  const bool rep = leaf_side >= 4 && !dropped && (t & ((1 << shift) - 1)) == 0;
  // this thread's leaves in depth-first order, each passed to f(x0, y0, side)
  auto for_each_leaf = [&](auto&& f) {
    if (leaf_side >= 4) {
      if (rep) f(bx0, by0, leaf_side);
      return;
    }
    // the 4x4 block split (minimum side below 4): its 2x2 cells, then their pixels
    for (int u = 0; u < 4; ++u) {
      const int x2 = bx0 + 2 * (u & 1), y2 = by0 + 2 * (u >> 1);
      if (!stat_splits(p2[u], 2, r)) {
        if (p2[u].n > 0) f(x2, y2, 2);
        continue;
      }
      for (int v = 0; v < 4; ++v) {
        const int x = x2 + (v & 1), y = y2 + (v >> 1);
        if (pixel_stat(im, x, y, r.measure).n > 0) f(x, y, 1);
      }
    }
  };
  // clipped to the image, keeping the leaves whose centre depth is valid
  uint32_t cnt = 0;
  for_each_leaf([&](int x0, int y0, int side) {
    if (leaf_valid(im, r, x0, y0, min(side, im.W - x0), min(side, im.H - y0))) ++cnt;
  });
  if (PASS == 0) {
    const uint32_t total = seed_block_sum(cnt, red);
    if (t == 0) root_counts[blockIdx.x] = total;
    return;
  }
  int64_t k = int64_t(root_counts[blockIdx.x]) + seed_block_excl_scan(cnt, red);
  for_each_leaf([&](int x0, int y0, int side) {
    const int w = min(side, im.W - x0), h = min(side, im.H - y0);
    if (!leaf_valid(im, r, x0, y0, w, h)) return;
    if (k < out.capacity) write_gaussian(im, r, out, k, x0, y0, w, h);
    ++k;
  });
}

}  // namespace

int seed_roots(int W, int H) { return ((W + kSeedRoot - 1) / kSeedRoot) * ((H + kSeedRoot - 1) / kSeedRoot); }

hipError_t launch_seed_count(const SeedImage& im, const SeedRules& r, uint32_t* root_counts, hipStream_t s) {
  k_seed<0><<<seed_roots(im.W, im.H), 256, 0, s>>>(im, r, root_counts, SeedOut{});
  return hipGetLastError();
}

hipError_t launch_seed_emit(const SeedImage& im, const SeedRules& r, const uint32_t* root_offsets,
                            const SeedOut& out, hipStream_t s) {
  k_seed<1><<<seed_roots(im.W, im.H), 256, 0, s>>>(im, r, const_cast<uint32_t*>(root_offsets), out);
  return hipGetLastError();
}

}  // namespace gsr
