// Voxel-block TSDF map on the device (Sec. III-B-1): the view the kernels take of it, and
// the lookup shared by the fusion kernels and the seeding check.
//
// Blocks of 8 x 8 x 8 voxels are found through an open-addressing hash table of packed
// block coordinates (linear probing, at most one probe per slot, so every search ends);
// each key's slot holds the block's index in the pool, assigned after insertion.  The pool
// keeps per voxel a truncated signed distance and a weight, x fastest within a block.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gsr {

constexpr int kBlockSide = 8;
constexpr int kBlockVoxels = kBlockSide * kBlockSide * kBlockSide;
constexpr unsigned long long kEmptyKey = ~0ull;
constexpr uint32_t kUnassigned = 0xFFFFFFFFu;
constexpr int kCoordBits = 21;                    // per axis, offset by 2^20
constexpr int32_t kCoordMax = (1 << (kCoordBits - 1)) - 1;
enum { TSDF_ALLOCATED = 0, TSDF_MET = 1, TSDF_FLAGS = 2, TSDF_CTRL_WORDS = 4 };
enum { TSDF_TABLE_FULL = 1u, TSDF_POOL_FULL = 2u, TSDF_OUT_OF_RANGE = 4u };

// A depth camera as the fusion kernels take it (world -> camera R row-major, t).
struct TsdfCam {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t W, H;
};

struct TsdfRules {
  float eps;         // truncation band
  float step;        // ray-march step in camera depth
  float w_max;       // weight cap (Eq. 8)
  int32_t n_samples; // band samples per pixel: floor(2 eps / step) + 1
  int32_t unit_weight;  // 0: Eq. 9 as printed; 1: running average with unit measurement weight
};

struct TsdfDev {
  unsigned long long* keys;  // [slots] packed block coordinates or kEmptyKey
  uint32_t* vals;            // [slots] pool index or kUnassigned
  uint32_t* stamp;           // [slots] last frame whose band met the block
  float* tsdf;               // [cap_blocks * 512]
  float* weight;             // [cap_blocks * 512]
  int4* coords;              // [cap_blocks] block coordinates
  uint32_t* ctrl;            // TSDF_* words
  uint32_t slot_mask;        // slots - 1 (a power of two)
  uint32_t cap_blocks;
  float voxel;
};

__host__ __device__ inline bool pack_block(int x, int y, int z, unsigned long long* key) {
  if (x < -kCoordMax - 1 || x > kCoordMax || y < -kCoordMax - 1 || y > kCoordMax || z < -kCoordMax - 1 ||
      z > kCoordMax)
    return false;
  const unsigned long long off = 1ull << (kCoordBits - 1);
  *key = (static_cast<unsigned long long>(x + int64_t(off))) |
         (static_cast<unsigned long long>(y + int64_t(off)) << kCoordBits) |
         (static_cast<unsigned long long>(z + int64_t(off)) << (2 * kCoordBits));
  return true;
}

__host__ __device__ inline int4 unpack_block(unsigned long long key) {
  const int off = 1 << (kCoordBits - 1);
  const unsigned long long m = (1ull << kCoordBits) - 1;
  return make_int4(int(key & m) - off, int((key >> kCoordBits) & m) - off, int((key >> (2 * kCoordBits)) & m) - off, 0);
}

__device__ inline uint32_t slot_of(unsigned long long key, uint32_t mask) {
  return uint32_t((key * 0x9E3779B97F4A7C15ull) >> 32) & mask;
}

// Pool index of the block with this key, or kUnassigned (absent or not yet assigned).
__device__ inline uint32_t find_block(const TsdfDev& m, unsigned long long key) {
  uint32_t h = slot_of(key, m.slot_mask);
  for (uint32_t probe = 0; probe <= m.slot_mask; ++probe) {
    const unsigned long long k = m.keys[h];
    if (k == key) return m.vals[h];
    if (k == kEmptyKey) return kUnassigned;
    h = (h + 1) & m.slot_mask;
  }
  return kUnassigned;
}

// Weight of the voxel that contains point p (binary32 coordinates divided by the binary32
// voxel side, floored); 0 where no block is allocated.
__device__ inline float voxel_weight_at(const TsdfDev& m, float px, float py, float pz) {
#pragma clang fp contract(off)
  const float gx = floorf(px / m.voxel), gy = floorf(py / m.voxel), gz = floorf(pz / m.voxel);
  if (!(fabsf(gx) < 8.0e6f && fabsf(gy) < 8.0e6f && fabsf(gz) < 8.0e6f)) return 0.f;
  const int ix = int(gx), iy = int(gy), iz = int(gz);
  const int bx = ix >> 3, by = iy >> 3, bz = iz >> 3;  // arithmetic shifts: floor division by 8
  unsigned long long key;
  if (!pack_block(bx, by, bz, &key)) return 0.f;
  const uint32_t b = find_block(m, key);
  if (b == kUnassigned || b >= m.cap_blocks) return 0.f;
  const int lx = ix & 7, ly = iy & 7, lz = iz & 7;
  return m.weight[size_t(b) * kBlockVoxels + (lz * kBlockSide + ly) * kBlockSide + lx];
}

}  // namespace gsr
