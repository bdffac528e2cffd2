// TSDF fusion of one depth frame into the voxel-block map (Sec. III-B-1, Eq. 6-9).
//
//   k_tsdf_alloc      one thread per pixel: march the viewing ray through the band
//                     [d - eps, d + eps] and insert every block a sample falls in (a key is
//                     read before any compare-and-swap, so the common case of a block
//                     already present costs one load); stamp the block's slot with the frame
//   k_tsdf_assign     one thread per table slot: give new keys a pool index (one counter
//                     atomic per wavefront with new keys, no thread waits on another)
//   k_tsdf_integrate  a 512-thread block per 512 table slots, one thread per voxel of
//                     each map block stamped with this frame: project the voxel centre, read
//                     the nearest pixel's depth, and apply Eq. 6-9 to the voxel's distance
//                     and weight (coalesced, HBM bound)
//   k_tsdf_weights    the weight of the voxel holding each query point (seeding check)
//
// The block of a sample and the pixel of a voxel are integer decisions taken from
// binary32 values; contraction is off so each operation rounds once, in the order of the
// comments, and the same inputs give the same blocks and pixels as any other
// implementation of that sequence.
#include <hip/hip_runtime.h>

#include "gsr_internal.h"
#include "gsr_tsdf.h"

namespace gsr {
namespace {

constexpr int kAllocThreads = 256;

// Inserts `key` (or finds it) and stamps its slot with the frame.
__device__ inline void insert_block(const TsdfDev& m, unsigned long long key, uint32_t frame) {
  uint32_t h = slot_of(key, m.slot_mask);
  for (uint32_t probe = 0; probe <= m.slot_mask; ++probe) {
    unsigned long long k = m.keys[h];
    if (k == kEmptyKey) k = atomicCAS(&m.keys[h], kEmptyKey, key);
    if (k == kEmptyKey || k == key) {  // inserted here, or already present
      if (m.stamp[h] != frame) m.stamp[h] = frame;  // most samples find it stamped already
      return;
    }
    h = (h + 1) & m.slot_mask;
  }
  atomicOr(&m.ctrl[TSDF_FLAGS], TSDF_TABLE_FULL);
}

__global__ __launch_bounds__(kAllocThreads) void k_tsdf_alloc(const float* depth, TsdfCam cam, TsdfDev m,
                                                              TsdfRules ru, uint32_t frame) {
#pragma clang fp contract(off)
  const int64_t p = int64_t(blockIdx.x) * kAllocThreads + threadIdx.x;
  if (p >= int64_t(cam.W) * cam.H) return;
  const float d = depth[p];
  if (!(d > 0.f)) return;
  const int u = int(p % cam.W), v = int(p / cam.W);
  const float xn = (float(u) - cam.cx) / cam.fx;
  const float yn = (float(v) - cam.cy) / cam.fy;
  const float a = d - ru.eps;
  const float bsize = 8.f * m.voxel;
  unsigned long long last = kEmptyKey;
  for (int i = 0; i < ru.n_samples; ++i) {
    const float z = a + float(i) * ru.step;
    if (!(z > 0.f)) continue;
    const float dx = xn * z - cam.t[0], dy = yn * z - cam.t[1], dz = z - cam.t[2];
    // world point R^T (camera point - t), one row of R^T (a column of R) per axis
    const float wx = (cam.R[0] * dx + cam.R[3] * dy) + cam.R[6] * dz;
    const float wy = (cam.R[1] * dx + cam.R[4] * dy) + cam.R[7] * dz;
    const float wz = (cam.R[2] * dx + cam.R[5] * dy) + cam.R[8] * dz;
    const float fx = floorf(wx / bsize), fy = floorf(wy / bsize), fz = floorf(wz / bsize);
    unsigned long long key;
    if (!(fabsf(fx) < 1.0e6f && fabsf(fy) < 1.0e6f && fabsf(fz) < 1.0e6f) ||
        !pack_block(int(fx), int(fy), int(fz), &key)) {
      atomicOr(&m.ctrl[TSDF_FLAGS], TSDF_OUT_OF_RANGE);
      continue;
    }
    if (key == last) continue;  // consecutive samples in one block
    last = key;
    insert_block(m, key, frame);
  }
}

// Reserves `count` consecutive entries of a counter for the lanes in `mask` with one atomic
// per wavefront; returns this lane's entry (rank among the mask's lanes below it).
__device__ inline uint32_t wave_reserve(uint32_t* counter, uint64_t mask, bool mine) {
  const int lane = threadIdx.x & 63;
  uint32_t base = 0;
  if (mask) {
    const int leader = __ffsll(static_cast<long long>(mask)) - 1;
    if (lane == leader) base = atomicAdd(counter, uint32_t(__popcll(mask)));
    base = __shfl(base, leader);
  }
  return mine ? base + uint32_t(__popcll(mask & ((1ull << lane) - 1ull))) : 0u;
}

__global__ __launch_bounds__(256) void k_tsdf_assign(TsdfDev m) {
  const uint32_t h = blockIdx.x * 256u + threadIdx.x;  // the grid covers the slots exactly
  const unsigned long long key = h <= m.slot_mask ? m.keys[h] : kEmptyKey;
  const bool fresh = key != kEmptyKey && m.vals[h] == kUnassigned;
  const uint32_t nb = wave_reserve(&m.ctrl[TSDF_ALLOCATED], __ballot(fresh), fresh);
  if (!fresh) return;
  if (nb < m.cap_blocks) {
    m.vals[h] = nb;
    m.coords[nb] = unpack_block(key);
  } else {
    atomicOr(&m.ctrl[TSDF_FLAGS], TSDF_POOL_FULL);
  }
}

// One 512-thread block per 512 table slots: every thread reads its slot's stamp
// and pool index, the block gathers the slots stamped with this frame into LDS (ballot
// ranks and a prefix over the eight wavefronts) with their coordinates, then every thread
// updates its voxel of
// each gathered block.  The number of met blocks is added once per block.
constexpr int kSlotsPerBlock = 512;

__global__ __launch_bounds__(kBlockVoxels) void k_tsdf_integrate(const float* depth, TsdfCam cam, TsdfDev m,
                                                                 TsdfRules ru, uint32_t frame) {
#pragma clang fp contract(off)
  __shared__ uint32_t s_blk[kSlotsPerBlock];
  __shared__ int4 s_crd[kSlotsPerBlock];
  __shared__ uint32_t s_cnt[kSlotsPerBlock / 64];
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const uint32_t h = blockIdx.x * uint32_t(kSlotsPerBlock) + uint32_t(t);
  bool met = false;
  uint32_t b = kUnassigned;
  if (t < kSlotsPerBlock && h <= m.slot_mask && m.stamp[h] == frame) {
    b = m.vals[h];
    met = b < m.cap_blocks;  // a block without a pool index (pool full) is skipped
  }
  const uint64_t mask = __ballot(met);
  if (t < kSlotsPerBlock && lane == 0) s_cnt[wv] = uint32_t(__popcll(mask));
  __syncthreads();
  uint32_t before = 0, total = 0;
#pragma unroll
  for (int i = 0; i < kSlotsPerBlock / 64; ++i) {
    before += i < wv ? s_cnt[i] : 0u;
    total += s_cnt[i];
  }
  if (met) {
    const uint32_t at = before + uint32_t(__popcll(mask & ((1ull << lane) - 1ull)));
    s_blk[at] = b;
    s_crd[at] = m.coords[b];
  }
  __syncthreads();
  const int lx = t & 7, ly = (t >> 3) & 7, lz = t >> 6;
  for (uint32_t i = 0; i < total; ++i) {
    const uint32_t blk = s_blk[i];
    const int4 c = s_crd[i];
    const size_t idx = size_t(blk) * kBlockVoxels + t;
    const float w = m.weight[idx], tv = m.tsdf[idx];  // in flight with the depth read below
    // voxel centre ((g + 0.5) voxel), then the camera point R p + t (sums left to right)
    const float px = (float(c.x * kBlockSide + lx) + 0.5f) * m.voxel;
    const float py = (float(c.y * kBlockSide + ly) + 0.5f) * m.voxel;
    const float pz = (float(c.z * kBlockSide + lz) + 0.5f) * m.voxel;
    const float x = ((cam.R[0] * px + cam.R[1] * py) + cam.R[2] * pz) + cam.t[0];
    const float y = ((cam.R[3] * px + cam.R[4] * py) + cam.R[5] * pz) + cam.t[1];
    const float z = ((cam.R[6] * px + cam.R[7] * py) + cam.R[8] * pz) + cam.t[2];
    if (!(z > 0.f)) continue;
    const float uh = (cam.fx * (x / z) + cam.cx) + 0.5f;  // nearest pixel: floor(u + 0.5)
    const float vh = (cam.fy * (y / z) + cam.cy) + 0.5f;
    if (!(uh >= 0.f && uh < float(cam.W) && vh >= 0.f && vh < float(cam.H))) continue;
    const float D = depth[int64_t(floorf(vh)) * cam.W + int64_t(floorf(uh))];
    if (!(D > 0.f)) continue;
    const float sdf = D - z;                                                    // Eq. 6
    const float q = sdf / ru.eps;
    const float tsdf = sdf > 0.f ? fminf(1.f, q) : fmaxf(-1.f, q);               // Eq. 7
    const float wn = fminf(ru.w_max, w + 1.f);                                  // Eq. 8
    m.tsdf[idx] = ru.unit_weight ? (tv * w + tsdf) / (w + 1.f)                   // running average
                                 : (tv * w + tsdf * wn) / (w + wn);               // Eq. 9
    m.weight[idx] = wn;
  }
  if (t == 0 && total) atomicAdd(&m.ctrl[TSDF_MET], total);
}

__global__ __launch_bounds__(256) void k_tsdf_weights(TsdfDev m, const float* pts, int64_t n, float* out) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  out[i] = voxel_weight_at(m, pts[i * 3], pts[i * 3 + 1], pts[i * 3 + 2]);
}

}  // namespace

int tsdf_band_samples(float eps, float step) {
#pragma clang fp contract(off)
  const float two_eps = 2.f * eps;
  return int(floorf(two_eps / step)) + 1;
}

hipError_t launch_tsdf_alloc(const float* depth, const TsdfCam& cam, const TsdfDev& m, const TsdfRules& ru,
                             uint32_t frame, hipStream_t s) {
  // the met-block count starts at zero (a fill kernel, so the sequence may be captured)
  hipError_t e = launch_fill_u32(m.ctrl + TSDF_MET, 0u, 1, s);
  if (e != hipSuccess) return e;
  const int64_t P = int64_t(cam.W) * cam.H;
  if (P > 0) k_tsdf_alloc<<<unsigned((P + kAllocThreads - 1) / kAllocThreads), kAllocThreads, 0, s>>>(depth, cam, m,
                                                                                                    ru, frame);
  k_tsdf_assign<<<unsigned((uint64_t(m.slot_mask) + 256) / 256), 256, 0, s>>>(m);
  return hipGetLastError();
}

hipError_t launch_tsdf_fuse(const float* depth, const TsdfCam& cam, const TsdfDev& m, const TsdfRules& ru,
                            uint32_t frame, hipStream_t s) {
  k_tsdf_integrate<<<unsigned((uint64_t(m.slot_mask) + kSlotsPerBlock) / kSlotsPerBlock), kBlockVoxels, 0, s>>>(
      depth, cam, m, ru, frame);
  return hipGetLastError();
}

hipError_t launch_tsdf_weights(const TsdfDev& m, const float* pts, int64_t n, float* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_tsdf_weights<<<unsigned((n + 255) / 256), 256, 0, s>>>(m, pts, n, out);
  return hipGetLastError();
}

}  // namespace gsr
