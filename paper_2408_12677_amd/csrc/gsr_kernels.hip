// gfx950 kernels of the differentiable tile-based Gaussian-splatting rasterizer.
//
//   K1 k_project        per Gaussian, loop over views: Eq. 2, 4, 5 (+ low-pass), conic of
//                       the 2D splat (Eq. 3), SH colour, frustum cull, tile rectangle, tile count,
//                       block sums of the tile counts and of the visible records
//   K2 k_scan_pairs     exclusive scans of those block sums (one block)
//   K3/K4               the stable sort of the (tile id << 32 | depth bits) keys, without
//                       materialising them: k_compact + k_radix_* sort the visible records by
//                       depth bits (stable LSD, 8-bit digits: histogram / row scan /
//                       ballot-multisplit scatter); k_bin_* then bin that depth order stably,
//                       first into tile rows, then into the tiles of each row, so every
//                       tile receives its records in ascending (depth, record) order
//   K5                  the tile ranges come from the binning's scan (k_bin_ranges);
//                       k_tile_order queues the tiles heaviest first
//   K6 k_blend_fwd      per tile: front-to-back compositing, Eq. 11 with clamp/skip/stop
//   K7 k_loss_l1        Eq. 12 (mean L1 colour) + weighted mean L1 depth, its gradient
//   K8 k_blend_bwd2     per (tile, stride) item, back to front: transmittance recovered by
//      (k_blend_bwd)    division, per-(pixel, splat) partials of two pixels per lane
//                       (one for tiles of 8) reduced across the wavefront with DPP, summed
//                       per splat in LDS and added with float atomics, splat-major
//   K9 k_project_bwd    per Gaussian, loop over views: chain rule to means, scales,
//                       rotations, opacities and SH coefficients
//
// Nothing here is a dense contraction, so no MFMA: the per-Gaussian kernels are HBM
// bound, the blend kernels VALU/transcendental bound.
#include "gsr_internal.h"

namespace gsr {
namespace {

// ------------------------------------------------------------------------------------
// wavefront / block helpers (wave64)
// ------------------------------------------------------------------------------------
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_move(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK,
                                                               0xF, false));
}

// gfx950 lane-half / row swaps: (a, b) -> a's upper 32 lanes exchanged with b's lower 32
// (permlane32), or a's odd 16-lane rows exchanged with b's even rows (permlane16).
__device__ __forceinline__ void swap_halves(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(int, a), __builtin_bit_cast(int, b), false, false);
  a = __builtin_bit_cast(float, int(r[0]));
  b = __builtin_bit_cast(float, int(r[1]));
}
__device__ __forceinline__ void swap_rows(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(int, a), __builtin_bit_cast(int, b), false, false);
  a = __builtin_bit_cast(float, int(r[0]));
  b = __builtin_bit_cast(float, int(r[1]));
}

// Sums of ten per-lane values over the wavefront in 28 instructions: lane halves are folded
// pairwise (5 swaps + 5 adds), then 16-lane rows (3 swaps + 3 adds), then each row is
// reduced with 4 fused DPP adds.  Every lane of a row ends with its row's total:
//   w0 rows 0..3 = sums of v0, v2, v1, v3;  w1 rows = v4, v6, v5, v7;  w2 rows = v8, v8, v9, v9.
// Needs every lane active.
__device__ __forceinline__ void wave_sum10(const float (&v)[10], float& w0, float& w1, float& w2) {
  float u[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    float a = v[2 * i], b = v[2 * i + 1];
    swap_halves(a, b);
    u[i] = a + b;
  }
  float a = u[0], b = u[1];
  swap_rows(a, b);
  w0 = a + b;
  a = u[2];
  b = u[3];
  swap_rows(a, b);
  w1 = a + b;
  a = u[4];
  b = u[4];
  swap_rows(a, b);
  w2 = a + b;
  w0 += dpp_move<0xB1, 0xF>(w0);
  w1 += dpp_move<0xB1, 0xF>(w1);
  w2 += dpp_move<0xB1, 0xF>(w2);
  w0 += dpp_move<0x4E, 0xF>(w0);
  w1 += dpp_move<0x4E, 0xF>(w1);
  w2 += dpp_move<0x4E, 0xF>(w2);
  w0 += dpp_move<0x141, 0xF>(w0);
  w1 += dpp_move<0x141, 0xF>(w1);
  w2 += dpp_move<0x141, 0xF>(w2);
  w0 += dpp_move<0x140, 0xF>(w0);
  w1 += dpp_move<0x140, 0xF>(w1);
  w2 += dpp_move<0x140, 0xF>(w2);
  // the sums exist in every lane here, so the last adds stay with their DPP moves (fused)
  // rather than sinking into the callers' one-lane-per-row stores
  asm volatile("" : "+v"(w0), "+v"(w1), "+v"(w2));
}

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), CTRL, 0xF, 0xF, false));
}

// Minimum over the wavefront, returned as a wavefront-uniform value: each 16-lane row is
// reduced with DPP (quad swaps, half-row and row mirrors), then the four row results are
// read from lanes 0, 16, 32 and 48.  Needs every lane active.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  v = min(v, dpp_u32<0xB1>(v));
  v = min(v, dpp_u32<0x4E>(v));
  v = min(v, dpp_u32<0x141>(v));
  v = min(v, dpp_u32<0x140>(v));
  const uint32_t a = uint32_t(__builtin_amdgcn_readlane(int(v), 0));
  const uint32_t b = uint32_t(__builtin_amdgcn_readlane(int(v), 16));
  const uint32_t c = uint32_t(__builtin_amdgcn_readlane(int(v), 32));
  const uint32_t d = uint32_t(__builtin_amdgcn_readlane(int(v), 48));
  return min(min(a, b), min(c, d));
}

// A VALU copy of v.  Registers read by readlane inside a loop that also stores to
// global memory are copied once after their load, so the loop does not wait for its own
// stores (memory counter) before each readlane.
__device__ __forceinline__ uint32_t valu_copy(uint32_t v) {
  uint32_t r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(v));
  return r;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, uint32_t(__shfl_xor(v, off)));
  return v;
}

// Maximum over the wavefront as a wavefront-uniform value, by the DPP steps of
// wave_min_u32.  Needs every lane active.
__device__ __forceinline__ uint32_t wave_max_uniform_u32(uint32_t v) {
  v = max(v, dpp_u32<0xB1>(v));
  v = max(v, dpp_u32<0x4E>(v));
  v = max(v, dpp_u32<0x141>(v));
  v = max(v, dpp_u32<0x140>(v));
  const uint32_t a = uint32_t(__builtin_amdgcn_readlane(int(v), 0));
  const uint32_t b = uint32_t(__builtin_amdgcn_readlane(int(v), 16));
  const uint32_t c = uint32_t(__builtin_amdgcn_readlane(int(v), 32));
  const uint32_t d = uint32_t(__builtin_amdgcn_readlane(int(v), 48));
  return uint32_t(__builtin_amdgcn_readfirstlane(int(max(max(a, b), max(c, d)))));
}

// base + the number of lanes below this one set in m (v_mbcnt)
__device__ __forceinline__ uint32_t rank_below(uint64_t m, uint32_t base) {
  return __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), base));
}

__device__ __forceinline__ uint32_t block_sum_u32(uint32_t v, uint32_t* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  uint32_t tot = 0;
  for (int i = 0; i < nw; ++i) tot += red[i];
  __syncthreads();
  return tot;
}

__device__ __forceinline__ uint32_t block_exclusive_scan_u32(uint32_t v, uint32_t* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t incl = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(incl, off);
    if (lane >= off) incl += t;
  }
  if (lane == 63) red[w] = incl;
  __syncthreads();
  uint32_t pre = 0;
  for (int i = 0; i < w; ++i) pre += red[i];
  return pre + incl - v;
}

// ------------------------------------------------------------------------------------
// Discrete stage.  A fixed sequence of correctly rounded binary32 operations (no fused
// multiply-add: the pragma turns contraction off, divide and square root are built
// correctly rounded) so that culling, splat centre, depth bits and tile rectangle are
// reproducible bit for bit.
// ------------------------------------------------------------------------------------
struct Proj {
  float tx, ty, tz;
  float qw, qx, qy, qz, nq;
  float r[9];  // rotation of the normalised quaternion
  float m[9];  // R diag(s)
  float T[6];  // J W
  float U[6];  // T M
  float a, b, c;  // projected covariance + low-pass
  float txj, tyj;  // the offsets J uses: tx, ty, or +-limit * tz where clamped
  bool clx, cly;   // clamped
  float mux, muy;
  int x0, x1, y0, y1;  // inclusive pixel rectangle
  bool vis;
};

__device__ __forceinline__ void discrete_stage(const float p[3], const float s[3], const float q[4],
                                               const ViewDev& cam, float k, float lowpass, float guard,
                                               float jclamp, Proj& o) {
#pragma clang fp contract(off)
  const float* W = cam.R;
  o.vis = false;
  float tx = W[0] * p[0];
  tx = tx + W[1] * p[1];
  tx = tx + W[2] * p[2];
  tx = tx + cam.t[0];
  float ty = W[3] * p[0];
  ty = ty + W[4] * p[1];
  ty = ty + W[5] * p[2];
  ty = ty + cam.t[1];
  float tz = W[6] * p[0];
  tz = tz + W[7] * p[1];
  tz = tz + W[8] * p[2];
  tz = tz + cam.t[2];
  o.tx = tx;
  o.ty = ty;
  o.tz = tz;
  if (!(tz > cam.znear)) return;
  float nq = q[0] * q[0];
  nq = nq + q[1] * q[1];
  nq = nq + q[2] * q[2];
  nq = nq + q[3] * q[3];
  nq = __builtin_sqrtf(nq);
  o.nq = nq;
  if (!(nq > 0.f)) return;
  const float w = q[0] / nq, x = q[1] / nq, y = q[2] / nq, z = q[3] / nq;
  o.qw = w;
  o.qx = x;
  o.qy = y;
  o.qz = z;
  float* r = o.r;
  r[0] = 1.f - 2.f * (y * y + z * z);
  r[1] = 2.f * (x * y - w * z);
  r[2] = 2.f * (x * z + w * y);
  r[3] = 2.f * (x * y + w * z);
  r[4] = 1.f - 2.f * (x * x + z * z);
  r[5] = 2.f * (y * z - w * x);
  r[6] = 2.f * (x * z - w * y);
  r[7] = 2.f * (y * z + w * x);
  r[8] = 1.f - 2.f * (x * x + y * y);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) o.m[i * 3 + j] = r[i * 3 + j] * s[j];
  const float tz2 = tz * tz;
  const float j00 = cam.fx / tz;
  const float j11 = cam.fy / tz;
  // guard-band clamp: an offset beyond jclamp half fields of view enters J as limit * tz
  float txj = tx, tyj = ty;
  o.clx = o.cly = false;
  if (jclamp > 0.f) {
    const float limx = jclamp * ((0.5f * float(cam.W)) / cam.fx);
    const float limy = jclamp * ((0.5f * float(cam.H)) / cam.fy);
    const float ux = tx / tz, uy = ty / tz;
    if (ux < -limx) {
      txj = -limx * tz;
      o.clx = true;
    } else if (ux > limx) {
      txj = limx * tz;
      o.clx = true;
    }
    if (uy < -limy) {
      tyj = -limy * tz;
      o.cly = true;
    } else if (uy > limy) {
      tyj = limy * tz;
      o.cly = true;
    }
  }
  o.txj = txj;
  o.tyj = tyj;
  const float j02 = -(cam.fx * txj) / tz2;
  const float j12 = -(cam.fy * tyj) / tz2;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    o.T[c] = j00 * W[c] + j02 * W[6 + c];
    o.T[3 + c] = j11 * W[3 + c] + j12 * W[6 + c];
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float acc = o.T[i * 3 + 0] * o.m[0 * 3 + c];
      acc = acc + o.T[i * 3 + 1] * o.m[1 * 3 + c];
      acc = acc + o.T[i * 3 + 2] * o.m[2 * 3 + c];
      o.U[i * 3 + c] = acc;
    }
  const float* U = o.U;
  float a = U[0] * U[0];
  a = a + U[1] * U[1];
  a = a + U[2] * U[2];
  a = a + lowpass;
  float b = U[0] * U[3];
  b = b + U[1] * U[4];
  b = b + U[2] * U[5];
  float c = U[3] * U[3];
  c = c + U[4] * U[4];
  c = c + U[5] * U[5];
  c = c + lowpass;
  o.a = a;
  o.b = b;
  o.c = c;
  const float det = a * c - b * b;
  if (!(det > 0.f)) return;
  const float mux = cam.fx * (tx / tz) + cam.cx;
  const float muy = cam.fy * (ty / tz) + cam.cy;
  o.mux = mux;
  o.muy = muy;
  // view frustum: the centre must project inside the image widened by the guard band
  const float gx = guard * float(cam.W), gy = guard * float(cam.H);
  if (!(mux >= -gx && mux <= float(cam.W) + gx && muy >= -gy && muy <= float(cam.H) + gy)) return;
  const float rx = k * __builtin_sqrtf(a);
  const float ry = k * __builtin_sqrtf(c);
  float fx0 = __builtin_ceilf(mux - rx), fx1 = __builtin_floorf(mux + rx);
  float fy0 = __builtin_ceilf(muy - ry), fy1 = __builtin_floorf(muy + ry);
  const float wmax = float(cam.W - 1), hmax = float(cam.H - 1);
  fx0 = (fx0 < 0.f) ? 0.f : fx0;
  fy0 = (fy0 < 0.f) ? 0.f : fy0;
  fx1 = (fx1 > wmax) ? wmax : fx1;
  fy1 = (fy1 > hmax) ? hmax : fy1;
  if (!(fx0 <= fx1 && fy0 <= fy1)) return;
  o.x0 = int(fx0);
  o.x1 = int(fx1);
  o.y0 = int(fy0);
  o.y1 = int(fy1);
  o.vis = true;
}

// Conic (inverse projected covariance); shared by the forward and backward kernels so
// both see identical bits.
__device__ __forceinline__ void conic_of(float a, float b, float c, float& A, float& B, float& C) {
#pragma clang fp contract(off)
  const float det = a * c - b * b;
  const float inv = 1.f / det;
  A = c * inv;
  B = -b * inv;
  C = a * inv;
}

// Exact tile culling: the tile columns [lo, hi] of tile row ty (local) that the ellipse
// d^T Q d <= k^2 of a splat can reach within the row's pixel band, Q = (A, B; B, C) its
// binary32 conic.  Over the band's offsets [u0, u1] from the centre, the boundary's
// rightmost point lies at dy = clamp(-B k / sqrt(C det_Q), u0, u1) and the leftmost at
// dy = clamp(B k / sqrt(C det_Q), u0, u1), with x offsets (+-sqrt(max(0, A k^2 - det_Q
// dy^2)) - B dy) / A; the pixels between ceil and floor of the two edges, kept inside the
// rectangle's columns, name the tiles.  One correctly rounded operation per line (the
// kernels compile with contraction off here), so the lists are reproducible bit for bit;
// a degenerate conic or a NaN keeps the rectangle's columns.  False when the row keeps
// no tile.
// The row-independent part of row_run: det_Q, the boundary's extreme offset B k / sqrt(C
// det_Q) and A k^2; `whole` when the conic is degenerate (or a NaN): keep the rectangle.
struct RowCut {
  float dq, q, ak;
  bool whole;
};

__device__ __forceinline__ RowCut row_cut(float A, float B, float C, float k) {
#pragma clang fp contract(off)
  RowCut r{};
  r.dq = A * C - B * B;
  r.whole = true;
  if (!(r.dq > 0.f)) return r;
  const float sq = __builtin_sqrtf(C * r.dq);
  if (!(sq > 0.f)) return r;
  r.q = (B * k) / sq;
  r.ak = A * (k * k);
  r.whole = false;
  return r;
}

// row_run for tile row ty given the record's row_cut; ts = 1 << tshift
__device__ __forceinline__ bool row_run_at(const RowCut& rc, float mux, float muy, float A, float B, int ts,
                                           int tshift, int ty, int W, int H, int tx0, int tx1, int& lo, int& hi) {
#pragma clang fp contract(off)
  lo = tx0;
  hi = tx1;
  if (rc.whole) return true;
  const float dyr = -rc.q, dyl = rc.q;
  const int ylast = min(ty * ts + ts - 1, H - 1);
  const float u0 = float(ty * ts) - muy;
  const float u1 = float(ylast) - muy;
  const float ur = fminf(fmaxf(dyr, u0), u1);
  const float ul = fminf(fmaxf(dyl, u0), u1);
  const float sr = __builtin_sqrtf(fmaxf(rc.ak - rc.dq * (ur * ur), 0.f));
  const float xr = (sr - B * ur) / A;
  const float sl = __builtin_sqrtf(fmaxf(rc.ak - rc.dq * (ul * ul), 0.f));
  const float xl = ((-sl) - B * ul) / A;
  float pl = ceilf(mux + xl);
  float pr = floorf(mux + xr);
  const float xa = float(tx0 * ts);
  const float xb = float(min(tx1 * ts + ts - 1, W - 1));
  if (!(pl >= xa)) pl = xa;  // also a NaN
  if (!(pr <= xb)) pr = xb;
  if (!(pl <= pr)) return false;
  lo = int(pl) >> tshift;  // pl, pr >= 0 here
  hi = int(pr) >> tshift;
  return true;
}

__device__ __forceinline__ bool row_run(float mux, float muy, float A, float B, float C, float k, int ts, int ty,
                                        int W, int H, int tx0, int tx1, int& lo, int& hi) {
  return row_run_at(row_cut(A, B, C, k), mux, muy, A, B, ts, __builtin_ctz(unsigned(ts)), ty, W, H, tx0, tx1, lo,
                    hi);
}

// Splat value a = o * exp(-q/2), q = A dx^2 + 2 B dx dy + C dy^2.  The compositing kernels
// stage each record with its conic scaled by -log2(e)/2, (a', b', c') = (A, 2B, C) * k,
// so that exp(-q/2) = exp2(q') with q' = (a' dx + b' dy) dx + c' dy^2: five operations and
// one exp2.  One fixed instruction sequence, so the forward skip decision and its
// recomputation in the backward agree bitwise.
constexpr float kNegHalfLog2e = -0.72134752044448170368f;  // -log2(e) / 2

__device__ __forceinline__ float splat_alpha(float dx, float dy, float ap, float bp, float cp, float o, float& G) {
#pragma clang fp contract(off)
  const float q = __builtin_fmaf(__builtin_fmaf(ap, dx, bp * dy), dx, (cp * dy) * dy);
  G = __builtin_amdgcn_exp2f(q);
  return o * G;
}

// LDS copy of record id for the compositing kernels: r0 = (mu_x, mu_y, a', b'),
// r1 = (c', opacity, depth, 2 a'), rgb = (r, g, b, 2 c') with (a', b', c') as above.
__device__ __forceinline__ void stage_record(const Records& rec, uint32_t id, float4& r0, float4& r1, float4& rgb) {
  const float4 g0 = rec.r0[id], g1 = rec.r1[id];
  const float ap = kNegHalfLog2e * g0.z, cp = kNegHalfLog2e * g1.x;
  r0 = make_float4(g0.x, g0.y, ap, (2.f * kNegHalfLog2e) * g0.w);
  r1 = make_float4(cp, g1.y, g1.z, ap + ap);
  const float4 c = rec.rgb[id];
  rgb = make_float4(c.x, c.y, c.z, cp + cp);
}

// ------------------------------------------------------------------------------------
// Real spherical harmonics, orthonormal with Condon-Shortley phase, as Cartesian
// polynomials of the unit direction (x, y, z).  Constants are N_l^m (and sqrt 2 for
// m != 0) times the Legendre factors:
//   l=0: 1/(2 sqrt(pi))
//   l=1: sqrt(3/(4 pi))                          -> -y, z, -x
//   l=2: sqrt(15/(4 pi)) xy, -..yz, sqrt(5/(16 pi))(3z^2-1), -..xz, sqrt(15/(16 pi))(x^2-y^2)
//   l=3: sqrt(35/(32 pi)), sqrt(105/(4 pi)), sqrt(21/(32 pi)), sqrt(7/(16 pi)), sqrt(105/(16 pi))
// Gradients are those of these polynomials; the chain rule through the normalisation
// of the direction removes their radial part.
// ------------------------------------------------------------------------------------
constexpr float kY00 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
constexpr float kY1 = 0.4886025119029199f;     // sqrt(3/(4 pi))
constexpr float kY2a = 1.0925484305920792f;    // sqrt(15/(4 pi))
constexpr float kY2b = 0.31539156525252005f;   // sqrt(5/(16 pi))
constexpr float kY2c = 0.5462742152960396f;    // sqrt(15/(16 pi))
constexpr float kY3a = 0.5900435899266435f;    // sqrt(35/(32 pi))
constexpr float kY3b = 2.890611442640554f;     // sqrt(105/(4 pi))
constexpr float kY3c = 0.4570457994644658f;    // sqrt(21/(32 pi))
constexpr float kY3d = 0.3731763325901154f;    // sqrt(7/(16 pi))
constexpr float kY3e = 1.445305721320277f;     // sqrt(105/(16 pi))

template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
  Y[0] = kY00;
  if (DEG >= 1) {
    Y[1] = -kY1 * y;
    Y[2] = kY1 * z;
    Y[3] = -kY1 * x;
  }
  if (DEG >= 2) {
    Y[4] = kY2a * x * y;
    Y[5] = -kY2a * y * z;
    Y[6] = kY2b * (3.f * z * z - 1.f);
    Y[7] = -kY2a * x * z;
    Y[8] = kY2c * (x * x - y * y);
  }
  if (DEG >= 3) {
    Y[9] = -kY3a * y * (3.f * x * x - y * y);
    Y[10] = kY3b * x * y * z;
    Y[11] = -kY3c * y * (5.f * z * z - 1.f);
    Y[12] = kY3d * z * (5.f * z * z - 3.f);
    Y[13] = -kY3c * x * (5.f * z * z - 1.f);
    Y[14] = kY3e * z * (x * x - y * y);
    Y[15] = -kY3a * x * (x * x - 3.f * y * y);
  }
}

// d/d(x,y,z) of the basis polynomials, contracted with weights w[k]: out = sum_k w_k grad Y_k.
template <int DEG>
__device__ __forceinline__ void sh_grad_dot(float x, float y, float z, const float* w, float out[3]) {
  float gx = 0.f, gy = 0.f, gz = 0.f;
  if (DEG >= 1) {
    gy += -kY1 * w[1];
    gz += kY1 * w[2];
    gx += -kY1 * w[3];
  }
  if (DEG >= 2) {
    gx += kY2a * y * w[4];
    gy += kY2a * x * w[4];
    gy += -kY2a * z * w[5];
    gz += -kY2a * y * w[5];
    gz += 6.f * kY2b * z * w[6];
    gx += -kY2a * z * w[7];
    gz += -kY2a * x * w[7];
    gx += 2.f * kY2c * x * w[8];
    gy += -2.f * kY2c * y * w[8];
  }
  if (DEG >= 3) {
    gx += -6.f * kY3a * x * y * w[9];
    gy += -kY3a * (3.f * x * x - 3.f * y * y) * w[9];
    gx += kY3b * y * z * w[10];
    gy += kY3b * x * z * w[10];
    gz += kY3b * x * y * w[10];
    gy += -kY3c * (5.f * z * z - 1.f) * w[11];
    gz += -10.f * kY3c * y * z * w[11];
    gz += kY3d * (15.f * z * z - 3.f) * w[12];
    gx += -kY3c * (5.f * z * z - 1.f) * w[13];
    gz += -10.f * kY3c * x * z * w[13];
    gx += 2.f * kY3e * x * z * w[14];
    gy += -2.f * kY3e * y * z * w[14];
    gz += kY3e * (x * x - y * y) * w[14];
    gx += -kY3a * (3.f * x * x - 3.f * y * y) * w[15];
    gy += 6.f * kY3a * x * y * w[15];
  }
  out[0] = gx;
  out[1] = gy;
  out[2] = gz;
}

// ------------------------------------------------------------------------------------
// K1: projection.  Per view, the block also sums its tile counts and visible records.
// ------------------------------------------------------------------------------------
template <int DEG>
__global__ __launch_bounds__(kProjThreads) void k_project(GaussDev g, ViewTable vt, Rules ru, int tile,
                                                          Records rec, uint2* blocksums, int nblk,
                                                          float* zero_rows, uint32_t* ctrl, int clear_words,
                                                          float exact_k) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  __shared__ uint32_t red[kProjThreads / 64];
  // the step's control words start at zero (no kernel before the projection reads them)
  if (blockIdx.x == 0 && int(threadIdx.x) < clear_words) ctrl[threadIdx.x] = 0u;
  const int64_t gi = int64_t(blockIdx.x) * kProjThreads + threadIdx.x;
  const bool valid = gi < g.n;
  float p[3] = {0.f, 0.f, 0.f}, s[3] = {1.f, 1.f, 1.f}, q[4] = {1.f, 0.f, 0.f, 0.f}, op = 0.f;
  float sh[K * 3];
  if (valid) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      p[i] = g.means[gi * 3 + i];
      s[i] = g.scales[gi * 3 + i];
    }
    const float4 q4 = reinterpret_cast<const float4*>(g.quats)[gi];
    q[0] = q4.x;
    q[1] = q4.y;
    q[2] = q4.z;
    q[3] = q4.w;
    op = g.opac[gi];
  }
  // the colour coefficients are read at the first view that sees the Gaussian (none for
  // a Gaussian outside every view)
  bool have_sh = false;
#pragma unroll
  for (int i = 0; i < K * 3; ++i) sh[i] = 0.f;
  for (int v = 0; v < vt.nviews; ++v) {
    const ViewDev& cam = vt.v[v];
    uint32_t cnt = 0;
    if (valid) {
      Proj pr;
      discrete_stage(p, s, q, cam, ru.k, ru.lowpass, ru.guard, ru.jclamp, pr);
      const int64_t rid = int64_t(v) * g.n + gi;
      if (pr.vis) {
        if (!have_sh) {
          const float* src = g.sh + gi * (K * 3);
#pragma unroll
          for (int i = 0; i < K * 3; ++i) sh[i] = src[i];
          have_sh = true;
        }
        const int tx0 = pr.x0 / tile, tx1 = pr.x1 / tile, ty0 = pr.y0 / tile, ty1 = pr.y1 / tile;
        cnt = uint32_t((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
        float A, B, C;
        conic_of(pr.a, pr.b, pr.c, A, B, C);
        float d0 = p[0] - cam.cam_pos[0], d1 = p[1] - cam.cam_pos[1], d2 = p[2] - cam.cam_pos[2];
        const float inv = 1.f / __builtin_sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
        float Y[K];
        sh_basis<DEG>(d0 * inv, d1 * inv, d2 * inv, Y);
        float col[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          float acc = 0.5f;
#pragma unroll
          for (int kk = 0; kk < K; ++kk) acc += sh[kk * 3 + ch] * Y[kk];
          col[ch] = acc > 0.f ? acc : 0.f;
        }
        rec.r0[rid] = make_float4(pr.mux, pr.muy, A, B);
        rec.r1[rid] = make_float4(C, op, pr.tz, 0.f);
        rec.rgb[rid] = make_float4(col[0], col[1], col[2], 0.f);
        rec.rect[rid] = make_uint2(uint32_t(tx0) | (uint32_t(tx1) << 16), uint32_t(ty0) | (uint32_t(ty1) << 16));
        if (rec.runs) {  // exact tiles: the column runs of the first kRowRuns tile rows, once per record
          const RowCut rc = row_cut(A, B, C, exact_k);
          const int tshift = __builtin_ctz(unsigned(tile));
          uint32_t rr[kRowRuns];
#pragma unroll
          for (int k = 0; k < kRowRuns; ++k) {
            rr[k] = kRunEmpty;
            if (k <= ty1 - ty0) {
              int lo, hi;
              if (row_run_at(rc, pr.mux, pr.muy, A, B, tile, tshift, ty0 + k, cam.W, cam.H, tx0, tx1, lo, hi))
                rr[k] = uint32_t(lo) | (uint32_t(hi) << 16);
            }
          }
          uint4* dst = reinterpret_cast<uint4*>(rec.runs + rid * kRowRuns);
#pragma unroll
          for (int k = 0; k < kRowRuns / 4; ++k) dst[k] = make_uint4(rr[4 * k], rr[4 * k + 1], rr[4 * k + 2], rr[4 * k + 3]);
        }
        if (zero_rows) {  // the backward's 2D-gradient row of this record starts at zero
          float4* z = reinterpret_cast<float4*>(zero_rows + rid * kGrad2D);
          z[0] = make_float4(0.f, 0.f, 0.f, 0.f);
          z[1] = make_float4(0.f, 0.f, 0.f, 0.f);
          z[2] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
      }
      rec.counts[rid] = cnt;
    }
    const uint32_t bs = block_sum_u32(cnt, red);
    const uint32_t bv = block_sum_u32(cnt ? 1u : 0u, red);
    if (threadIdx.x == 0) blocksums[int64_t(v) * nblk + blockIdx.x] = make_uint2(bs, bv);
  }
}

// ------------------------------------------------------------------------------------
// K2: exclusive scans of per-block sums (one block of 1024 threads).  Totals are written
// as 64-bit values; consumers clamp them to their buffer capacity.
// ------------------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ unsigned long long block_inclusive_scan_u64(unsigned long long v, unsigned long long* part) {
  const int t = threadIdx.x;
  part[t] = v;
  __syncthreads();
  for (int off = 1; off < NT; off <<= 1) {
    const unsigned long long add = t >= off ? part[t - off] : 0ull;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  return part[t];
}

__global__ __launch_bounds__(1024) void k_scan_pairs(uint2* a, int count, unsigned long long* totals) {
  __shared__ unsigned long long part[1024];
  const int t = threadIdx.x;
  const int per = (count + 1023) / 1024;
  const int beg = min(count, t * per), end = min(count, beg + per);
  unsigned long long sx = 0, sy = 0;
  for (int i = beg; i < end; ++i) {
    const uint2 x = a[i];
    sx += x.x;
    sy += x.y;
  }
  const unsigned long long ix = block_inclusive_scan_u64<1024>(sx, part);
  __syncthreads();
  const unsigned long long iy = block_inclusive_scan_u64<1024>(sy, part);
  unsigned long long rx = ix - sx, ry = iy - sy;
  for (int i = beg; i < end; ++i) {
    const uint2 x = a[i];
    a[i] = make_uint2(uint32_t(rx), uint32_t(ry));
    rx += x.x;
    ry += x.y;
  }
  if (t == 1023) {
    totals[0] = ix;
    totals[1] = iy;
  }
}

__global__ __launch_bounds__(1024) void k_scan_u32(uint32_t* a, int count, unsigned long long* total) {
  __shared__ unsigned long long part[1024];
  const int t = threadIdx.x;
  const int per = (count + 1023) / 1024;
  const int beg = min(count, t * per), end = min(count, beg + per);
  unsigned long long sum = 0;
  for (int i = beg; i < end; ++i) sum += a[i];
  const unsigned long long incl = block_inclusive_scan_u64<1024>(sum, part);
  unsigned long long run = incl - sum;
  for (int i = beg; i < end; ++i) {
    const uint32_t x = a[i];
    a[i] = uint32_t(run);
    run += x;
  }
  if (t == 1023) *total = incl;
}

// Flags a capacity overflow: the step's word and the sticky copy next to it.
__device__ __forceinline__ void raise_overflow(uint32_t* overflow) {
  atomicOr(overflow, 1u);
  atomicOr(overflow + (kOverflowSticky - kOverflow), 1u);
}

// A device-side count clamped to the capacity the grid and buffers were sized for; zero
// once a capacity overflow has been flagged, so that nothing downstream of an overflow
// reads partially written buffers.
__device__ __forceinline__ uint32_t clamp_count(const unsigned long long* count, int64_t cap,
                                                const uint32_t* overflow) {
  if (*overflow) return 0u;
  const unsigned long long c = *count;
  return uint32_t(c < (unsigned long long)cap ? c : (unsigned long long)cap);
}

// ------------------------------------------------------------------------------------
// K3a: compaction of the visible records into (depth bits, record id) pairs, record order
// ------------------------------------------------------------------------------------
// raw: the block sums are the projection's, not scanned (at most kCompactRawMax of them):
// each block adds the visible records of the blocks in front of it itself, and the last
// block writes the totals (pairs, visible records) to totals[0..1].  Otherwise they were
// scanned (k_scan_pairs, which wrote the totals).
__global__ __launch_bounds__(kProjThreads) void k_compact(int64_t n, Records rec, const uint2* blocksums, int nblk,
                                                          unsigned long long* totals, int64_t cap_M,
                                                          uint32_t* dkeys, uint32_t* dvals, int64_t cap,
                                                          uint32_t* overflow, int raw) {
  __shared__ uint32_t red[kProjThreads / 64];
  __shared__ unsigned long long red64[kProjThreads / 64];
  const int v = blockIdx.y;
  const int64_t me = int64_t(v) * nblk + blockIdx.x;  // this block's sums
  const int64_t nb = int64_t(gridDim.y) * nblk;
  const int64_t gi = int64_t(blockIdx.x) * kProjThreads + threadIdx.x;
  const int64_t rid = int64_t(v) * n + gi;
  const uint32_t vis = (gi < n && rec.counts[rid] != 0u) ? 1u : 0u;
  uint32_t base;
  if (raw) {
    uint32_t before = 0;
    for (int64_t i = threadIdx.x; i < me; i += kProjThreads) before += blocksums[i].y;
    base = block_sum_u32(before, red);
    if (me == nb - 1) {  // block-uniform: the last block writes the totals
      unsigned long long px = 0;
      for (int64_t i = threadIdx.x; i < nb; i += kProjThreads) px += blocksums[i].x;
      for (int off = 32; off > 0; off >>= 1) px += __shfl_xor(px, off);
      if ((threadIdx.x & 63) == 0) red64[threadIdx.x >> 6] = px;
      const uint32_t mine = block_sum_u32(vis, red);  // (its barrier also publishes red64)
      if (threadIdx.x == 0) {
        unsigned long long pairs = 0;
        for (int i = 0; i < kProjThreads / 64; ++i) pairs += red64[i];
        totals[0] = pairs;
        totals[1] = (unsigned long long)base + mine;
        if (pairs > (unsigned long long)cap_M) raise_overflow(overflow);
      }
    }
  } else {
    base = blocksums[me].y;
    // more (tile, record) pairs than the binning buffers hold: flag it before anything
    // reads the flag (every later kernel then sees zero records)
    if (me == 0 && threadIdx.x == 0 && totals[0] > (unsigned long long)cap_M) raise_overflow(overflow);
  }
  const uint32_t excl = block_exclusive_scan_u32(vis, red);
  if (!vis) return;
  const uint32_t off = base + excl;
  if (int64_t(off) >= cap) {
    raise_overflow(overflow);
    return;
  }
  dkeys[off] = __float_as_uint(rec.r1[rid].z);
  dvals[off] = uint32_t(rid);
}

// ------------------------------------------------------------------------------------
// K4: stable LSD radix sort of (u32 key, u32 value) by digits of BITS bits, count read
// from the device (clamped to the capacity the grid was sized for).  Per pass:
//   hist:    per-block digit histograms, stored digit-major [2^BITS][nblk]
//   rowscan: one block per digit scans its row -> start of each block in that digit,
//            and the digit total
//   scatter: each block ranks its keys stably (wavefront multisplit by ballots, then
//            across the four wavefronts through LDS) and writes them to their slots
// ------------------------------------------------------------------------------------
// 8-bit digits: wider ones (11 bits, three passes for a depth key) ran slower on MI355X,
// their digit-major histograms being written and read across many more cache lines
constexpr int kSortBits = 8;

// Block b of a grid of G blocks (G a multiple of 8) as index (b mod 8) * (G / 8) + b / 8:
// the hardware hands consecutive blocks to the eight XCDs in turn, so with this index
// consecutive key tiles and record chunks run on one XCD, and the strided count words
// they share meet in that XCD's L2.  (Only for even work: the row-list segments stay
// round-robin, as a contiguous range of rows would load some XCDs far more than others.)
__device__ __forceinline__ int xcd_block(int b, int G) { return (b & 7) * (G >> 3) + (b >> 3); }
static int xcd_grid(int64_t blocks) { return int((blocks + 7) / 8 * 8); }


template <int BITS>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t* keys, const unsigned long long* count,
                                                             int64_t cap, const uint32_t* overflow, int shift,
                                                             uint32_t* hist, int nblk) {
  constexpr int D = 1 << BITS;
  constexpr uint32_t MASK = D - 1;
  __shared__ uint32_t h[D];
  const int tb = xcd_block(blockIdx.x, gridDim.x);  // this block's tile of keys
  if (tb >= nblk) return;                            // block-uniform
  for (int d = threadIdx.x; d < D; d += kSortThreads) h[d] = 0;
  __syncthreads();
  const int64_t M = clamp_count(count, cap, overflow);
  const int64_t base = int64_t(tb) * kSortTile;
#pragma unroll 4
  for (int i = 0; i < kSortItems; ++i) {
    const int64_t idx = base + i * kSortThreads + threadIdx.x;
    if (idx < M) atomicAdd(&h[(keys[idx] >> shift) & MASK], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < D; d += kSortThreads) hist[int64_t(d) * nblk + tb] = h[d];
}

__global__ __launch_bounds__(kSortThreads) void k_radix_rowscan(uint32_t* hist, int nblk, uint32_t* digit_tot) {
  __shared__ uint32_t red[kSortThreads / 64];
  __shared__ uint32_t carry;
  uint32_t* row = hist + int64_t(blockIdx.x) * nblk;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int start = 0; start < nblk; start += kSortThreads) {
    const int i = start + threadIdx.x;
    const uint32_t v = i < nblk ? row[i] : 0u;
    const uint32_t ex = block_exclusive_scan_u32(v, red);
    const uint32_t c = carry;
    if (i < nblk) row[i] = c + ex;
    __syncthreads();
    if (threadIdx.x == kSortThreads - 1) carry = c + ex + v;
    __syncthreads();
  }
  if (threadIdx.x == 0) digit_tot[blockIdx.x] = carry;
}

template <int BITS>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint32_t* kin, const uint32_t* vin,
                                                                uint32_t* kout, uint32_t* vout,
                                                                const unsigned long long* count, int64_t cap,
                                                                const uint32_t* overflow, int shift,
                                                                const uint32_t* hist, const uint32_t* digit_tot,
                                                                int nblk) {
  constexpr int D = 1 << BITS;
  constexpr int DPT = D / kSortThreads;  // digits per thread
  constexpr int NW = kSortThreads / 64;
  constexpr uint32_t MASK = D - 1;
  static_assert(D % kSortThreads == 0, "whole digits per thread");
  // bases and per-wavefront counters are double buffered so each round needs two barriers;
  // a round's counts and offsets are below kSortThreads, so 16 bits hold them
  __shared__ uint32_t base[2][D];
  __shared__ uint16_t wcnt[2][NW][D];
  __shared__ uint32_t red[NW];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int tb = xcd_block(blockIdx.x, gridDim.x);  // this block's tile of keys
  if (tb >= nblk) return;                            // block-uniform
  const int64_t M = clamp_count(count, cap, overflow);
  // first slot of each digit: thread t scans digits t * DPT .. t * DPT + DPT - 1
  {
    uint32_t tot[DPT], sum = 0;
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      tot[j] = digit_tot[t * DPT + j];
      sum += tot[j];
    }
    uint32_t run = block_exclusive_scan_u32(sum, red);
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      const int d = t * DPT + j;
      base[0][d] = run + hist[int64_t(d) * nblk + tb];
      run += tot[j];
    }
  }
  // the per-round work below takes digits t + kSortThreads j (consecutive lanes, banks)
#pragma unroll
  for (int j = 0; j < DPT; ++j)
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      wcnt[0][i][t + kSortThreads * j] = 0;
      wcnt[1][i][t + kSortThreads * j] = 0;
    }
  __syncthreads();
  const int64_t b0 = int64_t(tb) * kSortTile;
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  // every round's key and value loaded up front (one memory latency per block, not one
  // per round)
  uint32_t kk[kSortItems], vv[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t idx = b0 + r * kSortThreads + t;
    kk[r] = idx < M ? kin[idx] : 0u;
    vv[r] = idx < M ? vin[idx] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int b = r & 1;
    const int64_t idx = b0 + r * kSortThreads + t;
    const bool valid = idx < M;
    const uint32_t key = kk[r], val = vv[r];
    const uint32_t d = valid ? (key >> shift) & MASK : 0u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < BITS; ++bit) {
      const bool on = (d >> bit) & 1u;
      const uint64_t m = __ballot(on);
      peers &= on ? m : ~m;
    }
    const uint32_t rank = __popcll(peers & lt_mask);
    if (valid && rank == 0) wcnt[b][w][d] = uint16_t(__popcll(peers));
    __syncthreads();
    // per digit: offsets of the four wavefronts, next round's base, clear next round's counters
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      const int dd = t + kSortThreads * j;
      uint32_t run = 0;
#pragma unroll
      for (int i = 0; i < NW; ++i) {
        const uint32_t c = wcnt[b][i][dd];
        wcnt[b][i][dd] = uint16_t(run);
        run += c;
        wcnt[b ^ 1][i][dd] = 0;
      }
      base[b ^ 1][dd] = base[b][dd] + run;
    }
    __syncthreads();
    if (valid) {
      const uint32_t dst = base[b][d] + wcnt[b][w][d] + rank;
      kout[dst] = key;
      vout[dst] = val;
    }
  }
}

// ------------------------------------------------------------------------------------
// Device-wide exclusive scan of u32 counts, in place, in two launches: per-block sums,
// then each block adds up the sums of the blocks before it (a few hundred words at most
// for the counts of a step, read once per block) and scans its kScanTile elements from
// there; the block holding the last element writes the total.  The element count is read
// from the device (clamped to the capacity the grid was sized for) when `count` is given;
// blocks past it leave at once.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ int64_t scan_len(int64_t cap, const unsigned long long* count) {
  if (!count) return cap;
  const unsigned long long c = *count;
  return c < (unsigned long long)cap ? int64_t(c) : cap;
}

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t* a, int64_t cap, const unsigned long long* count,
                                                     uint32_t* part) {
  __shared__ uint32_t red[4];
  const int64_t n = scan_len(cap, count);
  const int64_t base = int64_t(blockIdx.x) * kScanTile;
  uint32_t sum = 0;
#pragma unroll 4
  for (int i = 0; i < kScanTile / 256; ++i) {
    const int64_t idx = base + i * 256 + threadIdx.x;
    if (idx < n) sum += a[idx];
  }
  const uint32_t tot = block_sum_u32(sum, red);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_scan_down(uint32_t* a, int64_t cap, const unsigned long long* count,
                                                   const uint32_t* part, unsigned long long* total) {
  __shared__ uint32_t red[4];
  const int64_t n = scan_len(cap, count);
  const int64_t b0 = int64_t(blockIdx.x) * kScanTile;
  if (b0 >= n) {  // block-uniform
    if (blockIdx.x == 0 && threadIdx.x == 0) *total = 0ull;
    return;
  }
  uint32_t before = 0;  // the sums of the blocks in front
  for (int i = int(threadIdx.x); i < int(blockIdx.x); i += 256) before += part[i];
  before = block_sum_u32(before, red);
  const int64_t base = b0 + int64_t(threadIdx.x) * 16;
  uint32_t x[16];
  if (base + 16 <= n) {
    const uint4* src = reinterpret_cast<const uint4*>(a + base);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint4 q = src[j];
      x[4 * j] = q.x;
      x[4 * j + 1] = q.y;
      x[4 * j + 2] = q.z;
      x[4 * j + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 16; ++j) x[j] = base + j < n ? a[base + j] : 0u;
  }
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < 16; ++j) sum += x[j];
  const uint32_t ex = block_exclusive_scan_u32(sum, red);
  if (threadIdx.x == 255 && b0 + kScanTile >= n) *total = (unsigned long long)before + ex + sum;
  uint32_t run = before + ex;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const uint32_t v = x[j];
    x[j] = run;
    run += v;
  }
  if (base + 16 <= n) {
    uint4* dst = reinterpret_cast<uint4*>(a + base);
#pragma unroll
    for (int j = 0; j < 4; ++j) dst[j] = make_uint4(x[4 * j], x[4 * j + 1], x[4 * j + 2], x[4 * j + 3]);
  } else {
#pragma unroll
    for (int j = 0; j < 16; ++j)
      if (base + j < n) a[base + j] = x[j];
  }
}

// ------------------------------------------------------------------------------------
// K3/K4 binning (see BinPlan).  Both stages place items that cover a contiguous run of
// bins [lo, hi] (tile rows of a record, tile columns of a row entry) stably: chunk by
// chunk from scanned per-(bin, chunk) counts, and inside a chunk by one wavefront that
// walks its 64 items' bins in ascending order; for each bin the covering lanes take
// consecutive slots in lane order from the bin's next free slot, kept in LDS (loaded from
// the scanned counts when the chunk starts).
// ------------------------------------------------------------------------------------
__device__ __forceinline__ int view_of_tile(const ViewTable& vt, int tile) {
  int v = 0;
  for (int i = 1; i < vt.nviews; ++i)
    if (tile >= vt.v[i].tile_off) v = i;
  return v;
}

__device__ __forceinline__ int view_of_row(const ViewTable& vt, uint32_t row) {
  int v = 0;
  for (int i = 1; i < vt.nviews; ++i)
    if (int(row) >= vt.v[i].row_off) v = i;
  return v;
}

__device__ __forceinline__ uint32_t view_of_record(const ViewTable& vt, uint32_t rid, int64_t n) {
  return vt.nviews == 1 ? 0u : rid / uint32_t(n);
}

// The column run of a row entry: for (record, rect columns) `entry` in its k-th tile row,
// with exact tiles the run the projection kept (rr, loaded by load_row_runs before the
// row walk) for k < kRowRuns and past those rows the rectangle's columns marked kRunUncut,
// so that stage 2 cuts them; without exact tiles the rectangle's columns.
__device__ __forceinline__ uint32_t row_entry_run(const Records& rec, uint2 entry, const uint32_t (&rr)[kRowRuns],
                                                  uint32_t k) {
  if (!rec.runs) return entry.y;
  uint32_t r = entry.y | kRunUncut;
#pragma unroll
  for (int j = 0; j < kRowRuns; ++j)
    if (k == uint32_t(j)) r = rr[j];
  return r;
}

__device__ __forceinline__ void load_row_runs(const Records& rec, uint2 entry, bool valid, uint32_t (&rr)[kRowRuns]) {
#pragma unroll
  for (int j = 0; j < kRowRuns; ++j) rr[j] = 0u;
  if (!rec.runs || !valid) return;
  const uint4* src = reinterpret_cast<const uint4*>(rec.runs + int64_t(entry.x) * kRowRuns);
#pragma unroll
  for (int j = 0; j < kRowRuns / 4; ++j) {
    const uint4 q = src[j];
    rr[4 * j] = q.x;
    rr[4 * j + 1] = q.y;
    rr[4 * j + 2] = q.z;
    rr[4 * j + 3] = q.w;
  }
}

// stage 1 counts: tile-row histogram of one chunk of depth-sorted records
__global__ __launch_bounds__(256) void k_bin_rows_count(ViewTable vt, int64_t n, Records rec, const uint32_t* dvals,
                                                        const unsigned long long* nvis, int64_t cap_vis,
                                                        const uint32_t* overflow, BinPlan plan) {
  extern __shared__ uint32_t hist[];
  const int R = plan.rows;
  const int chunk = xcd_block(blockIdx.x, gridDim.x);
  if (chunk >= plan.nch1) return;  // block-uniform
  for (int i = threadIdx.x; i < R; i += 256) hist[i] = 0;
  __syncthreads();
  const int64_t NV = clamp_count(nvis, cap_vis, overflow);
  const int64_t beg = int64_t(chunk) * 64 * plan.rounds1;
  const int64_t end = min(NV, beg + int64_t(64) * plan.rounds1);
  for (int64_t i = beg + threadIdx.x; i < end; i += 256) {
    const uint32_t rid = dvals[i];
    const uint2 rc = rec.rect[rid];
    const int ro = vt.v[view_of_record(vt, rid, n)].row_off;
    const int y0 = ro + int(rc.y & 0xFFFFu), y1 = min(ro + int(rc.y >> 16), R - 1);
    for (int y = y0; y <= y1; ++y) atomicAdd(&hist[y], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < R; i += 256) plan.cnt1[int64_t(i) * plan.nch1 + chunk] = hist[i];
}

// Per row: list start and length, its segments and its first flat (tile, segment) index;
// totals of segments and of the flat array.  Run by the whole of one block of NT threads
// (the last block of the row placement, before its own work: no launch of its own).
template <int NT>
__device__ void rows_meta(const ViewTable& vt, const BinPlan& plan, uint32_t* overflow, unsigned long long* part) {
  const int R = plan.rows, t = threadIdx.x;
  const int per = (R + NT - 1) / NT;
  const int beg = min(R, t * per), end = min(R, beg + per);
  const unsigned long long E1 = plan.words[0];
  const uint32_t S2 = 64u * uint32_t(plan.rounds2);
  auto row = [&](int r, uint32_t& start, uint32_t& len, uint32_t& nseg, uint32_t& w) {
    start = plan.cnt1[int64_t(r) * plan.nch1];
    const unsigned long long next = r + 1 < R ? plan.cnt1[int64_t(r + 1) * plan.nch1] : E1;
    len = uint32_t(next - start);
    nseg = (len + S2 - 1) / S2;
    w = nseg * uint32_t(vt.v[view_of_row(vt, uint32_t(r))].tiles_x);
  };
  unsigned long long sseg = 0, sw = 0;
  for (int r = beg; r < end; ++r) {
    uint32_t a, l, ns, w;
    row(r, a, l, ns, w);
    sseg += ns;
    sw += w;
  }
  const unsigned long long iseg = block_inclusive_scan_u64<NT>(sseg, part);
  __syncthreads();
  const unsigned long long iw = block_inclusive_scan_u64<NT>(sw, part);
  unsigned long long seg = iseg - sseg, flat = iw - sw;
  for (int r = beg; r < end; ++r) {
    uint32_t a, l, ns, w;
    row(r, a, l, ns, w);
    plan.rowinfo[r] = make_uint4(a, l, uint32_t(seg), uint32_t(flat));
    plan.seg_start[r] = uint32_t(seg);
    seg += ns;
    flat += w;
  }
  if (t == NT - 1) {
    const bool over = iseg > (unsigned long long)plan.cap_seg || iw > (unsigned long long)plan.cap_flat;
    if (over) raise_overflow(overflow);
    plan.seg_start[R] = uint32_t(over ? 0ull : iseg);
    plan.words[1] = over ? 0ull : iseg;
    plan.words[2] = over ? 0ull : iw;
  }
}

// stage 1 placement: one wavefront per chunk writes (record, column run) entries into the
// row lists
__global__ __launch_bounds__(64) void k_bin_rows_scatter(ViewTable vt, int64_t n, Records rec, const uint32_t* dvals,
                                                         const unsigned long long* nvis, int64_t cap_vis,
                                                         uint32_t* overflow, BinPlan plan) {
  extern __shared__ uint32_t next[];  // next free slot of each row for this chunk
  __shared__ unsigned long long s_part[64];
  if (blockIdx.x == gridDim.x - 1) rows_meta<64>(vt, plan, overflow, s_part);
  const int R = plan.rows;
  const int lane = threadIdx.x;
  const int64_t NV = clamp_count(nvis, cap_vis, overflow);
  const int64_t beg = int64_t(blockIdx.x) * 64 * plan.rounds1;
  if (beg >= NV) return;
  for (int i = lane; i < R; i += 64) next[i] = plan.cnt1[int64_t(i) * plan.nch1 + blockIdx.x];
  __syncthreads();
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  for (int r = 0; r < plan.rounds1; ++r) {
    const int64_t r0 = beg + int64_t(r) * 64;
    if (r0 >= NV) break;
    const int64_t i = r0 + lane;
    uint32_t cur = 0xFFFFFFFFu, hi = 0u;
    uint2 entry = make_uint2(0u, 0u);
    if (i < NV) {
      const uint32_t rid = dvals[i];
      const uint2 rc = rec.rect[rid];
      const int ro = vt.v[view_of_record(vt, rid, n)].row_off;
      cur = uint32_t(ro) + (rc.y & 0xFFFFu);
      hi = min(uint32_t(ro) + (rc.y >> 16), uint32_t(R - 1));
      entry = make_uint2(rid, rc.x);
    }
    const uint32_t first = cur;
    uint32_t rr[kRowRuns];
    load_row_runs(rec, entry, cur != 0xFFFFFFFFu, rr);
    for (uint32_t y = wave_min_u32(cur); y != 0xFFFFFFFFu; y = wave_min_u32(cur)) {
      const bool on = cur == y;
      const uint64_t m = __ballot(on);
      const uint32_t base = next[y];
      if (on) {
        const uint32_t dst = base + uint32_t(__popcll(m & lt_mask));
        if (int64_t(dst) < plan.cap_M) plan.rowlist[dst] = make_uint2(entry.x, row_entry_run(rec, entry, rr, y - first));
        cur = cur < hi ? cur + 1u : 0xFFFFFFFFu;
      }
      if (lane == 0) next[y] = base + uint32_t(__popcll(m));
    }
  }
}

// Next free slot of bin b when the slots of bins lane + 64 k sit in register k of that
// lane: readlanes and selects only, so the walks over bins carry no branches.
template <int NREG>
__device__ __forceinline__ uint32_t slot_of(const uint32_t (&nx)[NREG], uint32_t b) {
  const int src = int(b & 63u), kb = int(b >> 6);
  uint32_t base = uint32_t(__builtin_amdgcn_readlane(int(nx[0]), src));
#pragma unroll
  for (int k = 1; k < NREG; ++k) {
    const uint32_t v = uint32_t(__builtin_amdgcn_readlane(int(nx[k]), src));
    base = kb == k ? v : base;
  }
  return base;
}

// Advances every bin's next free slot (bin lane + 64 k in register k) by the number of
// this round's lanes whose run [lo, hi] covers it (lo = 0xFFFFFFFF: no run), from a
// difference histogram in the wavefront's LDS words diff[0 .. 64 NREG] (+1 at lo, -1
// past hi) and its inclusive scan over the bins.
template <int NREG>
__device__ __forceinline__ void advance_slots(uint32_t (&nx)[NREG], uint32_t* diff, uint32_t lo, uint32_t hi,
                                              int lane) {
#pragma unroll
  for (int k = 0; k < NREG; ++k) diff[lane + 64 * k] = 0u;
  if (lane == 0) diff[64 * NREG] = 0u;
  __builtin_amdgcn_wave_barrier();
  if (lo != 0xFFFFFFFFu) {
    atomicAdd(&diff[lo], 1u);
    atomicAdd(&diff[hi + 1u], 0xFFFFFFFFu);
  }
  __builtin_amdgcn_wave_barrier();
  uint32_t carry = 0;
#pragma unroll
  for (int k = 0; k < NREG; ++k) {
    uint32_t v = diff[lane + 64 * k];
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t t = uint32_t(__shfl_up(int(v), off));
      if (lane >= off) v += t;
    }
    v += carry;
    carry = uint32_t(__builtin_amdgcn_readlane(int(v), 63));
    nx[k] += v;
  }
  __builtin_amdgcn_wave_barrier();
}

// The same placement with the rows' next free slots in registers (row lane + 64 k in
// register k of that lane, read with readlane) for at most 64 * NREG rows: each round
// walks the rows from the wavefront's lowest to its highest with one ballot per row.
// Four wavefronts per block, each with its own chunk (blocks of one wavefront were held
// back by the per-CU workgroup limit).
template <int NREG>
__global__ __launch_bounds__(256) void k_bin_rows_scatter_r(ViewTable vt, int64_t n, Records rec,
                                                            const uint32_t* dvals, const unsigned long long* nvis,
                                                            int64_t cap_vis, uint32_t* overflow, BinPlan plan) {
  __shared__ unsigned long long s_part[256];
  __shared__ uint32_t s_rr[4][kRowRuns + 1][64];  // per wavefront: the round's row runs
  __shared__ uint32_t s_diff[4][64 * NREG + 1];     // per wavefront: rows covered (difference form)
  if (blockIdx.x == gridDim.x - 1) rows_meta<256>(vt, plan, overflow, s_part);
  const int R = plan.rows;
  const int lane = threadIdx.x & 63, wv = int(threadIdx.x >> 6);
  const int chunk = int(blockIdx.x) * 4 + int(threadIdx.x >> 6);  // one chunk per wavefront
  const int64_t NV = clamp_count(nvis, cap_vis, overflow);
  const int64_t beg = int64_t(chunk) * 64 * plan.rounds1;
  if (chunk >= plan.nch1 || beg >= NV) return;
  const uint32_t cap = uint32_t(min<int64_t>(plan.cap_M, int64_t(0xFFFFFFFFu)));
  uint32_t nx[NREG];
#pragma unroll
  for (int k = 0; k < NREG; ++k) {
    const int y = lane + 64 * k;
    nx[k] = valu_copy(y < R ? plan.cnt1[int64_t(y) * plan.nch1 + chunk] : 0u);
  }
  for (int r = 0; r < plan.rounds1; ++r) {
    const int64_t r0 = beg + int64_t(r) * 64;
    if (r0 >= NV) break;
    const int64_t i = r0 + lane;
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    uint2 entry = make_uint2(0u, 0u);
    if (i < NV) {
      const uint32_t rid = dvals[i];
      const uint2 rc = rec.rect[rid];
      const int ro = vt.v[view_of_record(vt, rid, n)].row_off;
      lo = uint32_t(ro) + (rc.y & 0xFFFFu);
      hi = min(uint32_t(ro) + (rc.y >> 16), uint32_t(R - 1));
      if (lo > hi) lo = 0xFFFFFFFFu;
      entry = make_uint2(rid, rc.x);
    }
    const uint32_t first = lo;
    // this lane's runs, row k of the splat at s_rr[wv][k][lane] (k = kRowRuns: the later
    // rows); each lane reads back only its own column
    if (rec.runs) {
      uint32_t rr[kRowRuns];
      load_row_runs(rec, entry, lo != 0xFFFFFFFFu, rr);
#pragma unroll
      for (int k = 0; k < kRowRuns; ++k) s_rr[wv][k][lane] = rr[k];
      s_rr[wv][kRowRuns][lane] = entry.y | kRunUncut;
    }
    const uint32_t y0 = wave_min_u32(lo);
    if (y0 == 0xFFFFFFFFu) continue;
    const uint32_t y1 = wave_max_uniform_u32(lo != 0xFFFFFFFFu ? hi : 0u);
    for (uint32_t y = y0; y <= y1; ++y) {  // branch-free but for the store
      const bool on = lo <= y && y <= hi;
      // (two ballots of plain compares: the compiler keeps them in scalar registers)
      const uint64_t m = __builtin_amdgcn_ballot_w64(lo <= y) & __builtin_amdgcn_ballot_w64(y <= hi);
      const uint32_t base = slot_of(nx, y);
      const uint32_t dst = rank_below(m, base);
      if (on && dst < cap) {
        const uint32_t run = rec.runs ? s_rr[wv][min(y - first, uint32_t(kRowRuns))][lane] : entry.y;
        plan.rowlist[dst] = make_uint2(entry.x, run);
      }
    }
    advance_slots(nx, s_diff[wv], lo, hi, lane);
  }
}

// the row whose segments contain segment s: the last r with seg_start[r] <= s
__device__ __forceinline__ int row_of_segment(const uint32_t* seg_start, int R, uint32_t s) {
  int lo = 0, hi = R - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (seg_start[mid] <= s)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

struct Segment {
  uint32_t beg, end;   // entries of the row list
  uint32_t flat;       // flat index of (column 0, this segment)
  uint32_t nseg;       // segments of the row (stride between columns)
  int tiles_x;
  int row;             // global tile row
};

__device__ __forceinline__ Segment segment_of(const ViewTable& vt, const BinPlan& plan, uint32_t s) {
  const int r = row_of_segment(plan.seg_start, plan.rows, s);
  const uint4 info = plan.rowinfo[r];
  const uint32_t S2 = 64u * uint32_t(plan.rounds2);
  Segment g;
  const uint32_t sidx = s - info.z;
  g.nseg = (info.y + S2 - 1) / S2;
  g.beg = info.x + sidx * S2;
  g.end = min(info.x + info.y, g.beg + S2);
  g.flat = info.w + sidx;
  g.tiles_x = vt.v[view_of_row(vt, uint32_t(r))].tiles_x;
  g.row = r;
  return g;
}

// ------------------------------------------------------------------------------------
// Tile work queue.  Tiles are ordered by decreasing expected work (a counting sort on
// buckets of eight steps per octave, in one block: the order inside a bucket is
// arbitrary) and the compositing kernels run as persistent blocks that take the next tile
// from a device counter, so the heaviest tiles start first and light ones fill the tail.
// A tile's work is its longest per-pixel contributor count, which the list length does
// not predict (a pixel stops once its transmittance is spent); when a previous forward
// of the same tiles left those counts (`hint`), they are the key, else the list length.
// ------------------------------------------------------------------------------------
constexpr int kOrderBuckets = 257;

__device__ __forceinline__ uint32_t work_bucket(uint32_t w) {
  if (w == 0) return 0;
  const uint32_t e = 31u - uint32_t(__clz(w));
  const uint32_t m = e >= 3 ? (w >> (e - 3)) & 7u : (w << (3 - e)) & 7u;
  return 1u + 8u * e + m;
}

// The queue order of `total` tiles by one whole block of NT threads (LDS: cnt and start
// of kOrderBuckets words, red of NT / 64): bucket counts, their scan heaviest bucket first,
// then each tile's slot (the order inside a bucket is arbitrary).  With a hint the ranges
// are not read.
template <int NT>
__device__ void tile_order_block(const uint2* ranges, const uint32_t* hint, int total, uint32_t* order,
                                 uint32_t* cnt, uint32_t* start, uint32_t* red) {
  const int t = threadIdx.x;
  for (int b = t; b < kOrderBuckets; b += NT) cnt[b] = 0;
  __syncthreads();
  auto key = [&](int i) {
    if (hint) return work_bucket(hint[i]);
    const uint2 r = ranges[i];
    return work_bucket(r.y - r.x);
  };
  for (int i = t; i < total; i += NT) atomicAdd(&cnt[key(i)], 1u);
  __syncthreads();
  // heaviest bucket first: thread t takes positions t P .. t P + P - 1 of the descending order
  constexpr int P = (kOrderBuckets + NT - 1) / NT;
  uint32_t c[P], sum = 0;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int bk = kOrderBuckets - 1 - (t * P + j);
    c[j] = bk >= 0 ? cnt[bk] : 0u;
    sum += c[j];
  }
  uint32_t run = block_exclusive_scan_u32(sum, red);
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int bk = kOrderBuckets - 1 - (t * P + j);
    if (bk >= 0) start[bk] = run;
    run += c[j];
  }
  __syncthreads();
  for (int i = t; i < total; i += NT) order[atomicAdd(&start[key(i)], 1u)] = uint32_t(i);
}

__global__ __launch_bounds__(1024) void k_tile_order(const uint2* ranges, const uint32_t* hint, int total,
                                                    uint32_t* order) {
  __shared__ uint32_t cnt[kOrderBuckets], start[kOrderBuckets];
  __shared__ uint32_t red[16];
  tile_order_block<1024>(ranges, hint, total, order, cnt, start, red);
}

// stage 2 counts: tile-column histogram of one segment of a row list, one wavefront per
// segment (its own LDS words, hist_stride >= tiles + 1: each run adds +1 at its first
// column and -1 past its last, and a scan over the columns gives the counts).  With exact tiles the runs of a
// record's first kRowRuns rows arrive cut by the projection; a run marked kRunUncut (a
// later row of a tall splat) is cut here to the columns its ellipse reaches in this row
// (row_run) and written back, so the placement below sees the same run; a row the
// ellipse misses gets the empty run kRunEmpty (lo > hi).
__global__ __launch_bounds__(256) void k_bin_tiles_count(ViewTable vt, BinPlan plan, Records rec, float exact_k,
                                                         int tile, int hist_stride) {
  extern __shared__ uint32_t hist_all[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t* hist = hist_all + wv * hist_stride;
  const unsigned long long S = plan.words[1];
  for (uint32_t s = blockIdx.x * 4u + uint32_t(wv); s < S; s += gridDim.x * 4u) {
    const Segment g = segment_of(vt, plan, s);
    for (int i = lane; i <= g.tiles_x; i += 64) hist[i] = 0;
    __builtin_amdgcn_wave_barrier();
    // each entry is loaded one iteration ahead
    uint2 e_next = g.beg + uint32_t(lane) < g.end ? plan.rowlist[g.beg + lane] : make_uint2(0u, kRunEmpty);
    for (uint32_t i = g.beg + lane; i < g.end; i += 64) {
      const uint2 e = e_next;
      e_next = i + 64u < g.end ? plan.rowlist[i + 64u] : make_uint2(0u, kRunEmpty);
      uint32_t cx = e.y;
      if (cx & kRunUncut) {
        cx &= ~kRunUncut;
        const uint32_t rid = e.x;
        const ViewDev& cam = vt.v[view_of_row(vt, uint32_t(g.row))];
        const float4 sp = rec.r0[rid];  // centre and conic A, B
        const float cc = rec.r1[rid].x;
        int lo, hi;
        const bool any = row_run(sp.x, sp.y, sp.z, sp.w, cc, exact_k, tile, g.row - cam.row_off, cam.W, cam.H,
                                 int(cx & 0xFFFFu), int(cx >> 16), lo, hi);
        cx = any ? uint32_t(lo) | (uint32_t(hi) << 16) : kRunEmpty;
        plan.rowlist[i].y = cx;
      }
      const int x0 = int(cx & 0xFFFFu), x1 = min(int(cx >> 16), g.tiles_x - 1);
      if (x0 <= x1) {  // the run in difference form: +1 at its first column, -1 past its last
        atomicAdd(&hist[x0], 1u);
        atomicAdd(&hist[x1 + 1], 0xFFFFFFFFu);
      }
    }
    __builtin_amdgcn_wave_barrier();
    uint32_t carry = 0;  // inclusive scan over the columns, 64 at a time
    for (int x = lane; x < ((g.tiles_x + 63) & ~63); x += 64) {
      uint32_t v = x < g.tiles_x ? hist[x] : 0u;
      for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = uint32_t(__shfl_up(int(v), off));
        if (lane >= off) v += t;
      }
      v += carry;
      carry = uint32_t(__builtin_amdgcn_readlane(int(v), 63));
      if (x < g.tiles_x) plan.cntF[g.flat + uint32_t(x) * g.nseg] = v;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// [start, end) of tile t from the flat scan; empty tiles are [0, 0)
__device__ __forceinline__ uint2 tile_range(const ViewTable& vt, const BinPlan& plan, const uint32_t* overflow,
                                            int t) {
  if (*overflow) return make_uint2(0u, 0u);  // nothing was binned
  const ViewDev& cam = vt.v[view_of_tile(vt, t)];
  const int local = t - cam.tile_off;
  const int r = cam.row_off + local / cam.tiles_x, x = local % cam.tiles_x;
  const uint4 info = plan.rowinfo[r];
  const uint32_t S2 = 64u * uint32_t(plan.rounds2);
  const uint32_t nseg = (info.y + S2 - 1) / S2;
  uint2 out = make_uint2(0u, 0u);
  if (nseg) {
    const unsigned long long F = plan.words[2];
    const uint32_t idx = info.w + uint32_t(x) * nseg;
    const uint32_t a = plan.cntF[idx];
    const uint32_t b = (unsigned long long)(idx + nseg) < F ? plan.cntF[idx + nseg] : uint32_t(plan.words[3]);
    if (b > a) out = make_uint2(a, b);
  }
  return out;
}

// stage 2 placement: one wavefront per segment writes record ids into the tile lists; the
// blocks first write the tile ranges (grid-stride over the tiles)
__global__ __launch_bounds__(64) void k_bin_tiles_scatter(ViewTable vt, BinPlan plan, uint32_t* vals,
                                                          const uint32_t* overflow, uint2* ranges) {
  extern __shared__ uint32_t next[];  // next free slot of each tile for this segment
  const int lane = threadIdx.x;
  for (int t = int(blockIdx.x) * 64 + lane; t < vt.total_tiles; t += int(gridDim.x) * 64)
    ranges[t] = tile_range(vt, plan, overflow, t);
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  const unsigned long long S = plan.words[1];
  for (uint32_t s = blockIdx.x; s < S; s += gridDim.x) {
    const Segment g = segment_of(vt, plan, s);
    __syncthreads();
    for (int i = lane; i < g.tiles_x; i += 64) next[i] = plan.cntF[g.flat + uint32_t(i) * g.nseg];
    __syncthreads();
    for (uint32_t r0 = g.beg; r0 < g.end; r0 += 64) {
      const uint32_t i = r0 + uint32_t(lane);
      uint32_t cur = 0xFFFFFFFFu, hi = 0u, rid = 0u;
      if (i < g.end) {
        const uint2 e = plan.rowlist[i];
        rid = e.x;
        cur = e.y & 0xFFFFu;
        hi = min(e.y >> 16, uint32_t(g.tiles_x - 1));
        if (cur > hi) cur = 0xFFFFFFFFu;  // a row the ellipse does not reach
      }
      for (uint32_t x = wave_min_u32(cur); x != 0xFFFFFFFFu; x = wave_min_u32(cur)) {
        const bool on = cur == x;
        const uint64_t m = __ballot(on);
        const uint32_t base = next[x];
        if (on) {
          const uint32_t dst = base + uint32_t(__popcll(m & lt_mask));
          if (int64_t(dst) < plan.cap_M) vals[dst] = rid;
          cur = cur < hi ? cur + 1u : 0xFFFFFFFFu;
        }
        if (lane == 0) next[x] = base + uint32_t(__popcll(m));
      }
    }
  }
}

// The same placement with the tiles' next free slots in registers (column lane + 64 k
// in register k of that lane) for rows of at most 64 * NREG tiles; four wavefronts per
// block, each with its own segments.
template <int NREG>
__global__ __launch_bounds__(256) void k_bin_tiles_scatter_r(ViewTable vt, BinPlan plan, uint32_t* vals,
                                                             const uint32_t* overflow, uint2* ranges,
                                                             const uint32_t* hint, uint32_t* order) {
  __shared__ uint32_t s_cnt[kOrderBuckets], s_start[kOrderBuckets], s_red[4];
  __shared__ uint32_t s_diff[4][64 * NREG + 1];  // per wavefront: tiles covered (difference form)
  // with a work hint the tile queue's order does not need the ranges: the last block
  // orders it here (no launch of its own)
  if (hint && blockIdx.x == gridDim.x - 1) tile_order_block<256>(nullptr, hint, vt.total_tiles, order, s_cnt, s_start, s_red);
  const int lane = threadIdx.x & 63;
  for (int t = int(blockIdx.x) * 256 + int(threadIdx.x); t < vt.total_tiles; t += int(gridDim.x) * 256)
    ranges[t] = tile_range(vt, plan, overflow, t);
  const uint32_t cap = uint32_t(min<int64_t>(plan.cap_M, int64_t(0xFFFFFFFFu)));
  const unsigned long long S = plan.words[1];
  // a segment per wavefront
  for (uint32_t s = blockIdx.x * 4u + (threadIdx.x >> 6); s < S; s += gridDim.x * 4u) {
    const Segment g = segment_of(vt, plan, s);
    uint32_t nx[NREG];
#pragma unroll
    for (int k = 0; k < NREG; ++k) {
      const int x = lane + 64 * k;
      nx[k] = valu_copy(x < g.tiles_x ? plan.cntF[g.flat + uint32_t(x) * g.nseg] : 0u);
    }
    // each round's entry is loaded one round ahead (its latency under the walk before it)
    uint2 e_next = g.beg + uint32_t(lane) < g.end ? plan.rowlist[g.beg + lane] : make_uint2(0u, kRunEmpty);
    for (uint32_t r0 = g.beg; r0 < g.end; r0 += 64) {
      const uint32_t i = r0 + uint32_t(lane);
      const uint2 e = e_next;
      e_next = i + 64u < g.end ? plan.rowlist[i + 64u] : make_uint2(0u, kRunEmpty);
      uint32_t lo = 0xFFFFFFFFu, hi = 0u, rid = 0u;
      if (i < g.end) {
        rid = e.x;
        lo = e.y & 0xFFFFu;
        hi = min(e.y >> 16, uint32_t(g.tiles_x - 1));
        if (lo > hi) lo = 0xFFFFFFFFu;  // a row the ellipse does not reach
      }
      const uint32_t x0 = wave_min_u32(lo);
      if (x0 == 0xFFFFFFFFu) continue;
      const uint32_t x1 = wave_max_uniform_u32(lo != 0xFFFFFFFFu ? hi : 0u);
      for (uint32_t x = x0; x <= x1; ++x) {  // branch-free but for the store
        const bool on = lo <= x && x <= hi;
        // (two ballots of plain compares: the compiler keeps them in scalar registers)
        const uint64_t m = __builtin_amdgcn_ballot_w64(lo <= x) & __builtin_amdgcn_ballot_w64(x <= hi);
        const uint32_t base = slot_of(nx, x);
        const uint32_t dst = rank_below(m, base);
        if (on && dst < cap) vals[dst] = rid;
      }
      advance_slots(nx, s_diff[threadIdx.x >> 6], lo, hi, lane);
    }
  }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* p, uint32_t value, int64_t count) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < count) p[i] = value;
}

// The smallest Gaussian index with a NaN or infinite parameter (first[0] starts at
// UINT32_MAX; it stays there when every value is finite).  Grid-stride over the five
// arrays taken as one run of n * (14 + 3 (K - 1)) values.
__global__ __launch_bounds__(256) void k_first_nonfinite(GaussDev g, int K, uint32_t* first) {
  const int64_t n = g.n;
  const int64_t sizes[5] = {3 * n, 3 * n, 4 * n, n, int64_t(3) * K * n};
  const int per[5] = {3, 3, 4, 1, 3 * K};
  const float* arrs[5] = {g.means, g.scales, g.quats, g.opac, g.sh};
  const int64_t total = sizes[0] + sizes[1] + sizes[2] + sizes[3] + sizes[4];
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < total; i += int64_t(gridDim.x) * 256) {
    int64_t j = i;
    int a = 0;
    while (j >= sizes[a]) j -= sizes[a++];
    if (!isfinite(arrs[a][j])) atomicMin(first, uint32_t(j / per[a]));
  }
}

// Wave priority 0..3 (s_setprio takes an immediate).
__device__ __forceinline__ void set_wave_prio(int p) {
  if (p >= 3)
    __builtin_amdgcn_s_setprio(3);
  else if (p == 2)
    __builtin_amdgcn_s_setprio(2);
  else if (p == 1)
    __builtin_amdgcn_s_setprio(1);
  else
    __builtin_amdgcn_s_setprio(0);
}

// Priority of a queue position: the first sixteenth of the items (the heaviest) 3, the
// rest of the first eighth 2, of the first quarter 1, else 0.
__device__ __forceinline__ int queue_prio(int item, int total) {
  return item * 16 < total ? 3 : (item * 8 < total ? 2 : (item * 4 < total ? 1 : 0));
}

// Block-uniform: the next tile of the queue, or -1 when it is exhausted; *prio is the
// queue position's priority.
__device__ __forceinline__ int next_tile(const TileQueue& q, uint32_t* head, int total, int* s_item, int* prio) {
  __syncthreads();
  if (threadIdx.x == 0) *s_item = int(atomicAdd(head, 1u));
  __syncthreads();
  const int item = *s_item;
  *prio = item < total && q.by_work ? queue_prio(item, total) : 0;
  return item < total ? int(q.order[item]) : -1;
}

// ------------------------------------------------------------------------------------
// K6: forward compositing.  Persistent blocks take tiles from the queue; one thread per
// pixel; the tile's sorted list is staged through LDS BATCH records at a time; a tile is
// left once every pixel has reached T < T_min.
// ------------------------------------------------------------------------------------
// entries evaluated together by the forward compositing (eight ran 5% faster than four,
// sixteen another 5% faster than eight: the heaviest tiles' single-wavefront chains wait
// on one group's LDS reads and exponentials at a time)
constexpr int kFwdGroup = 16;
// list entries between two checkpoints of the forward, and so the length of a backward
// work item: 64 rather than half a batch gives the backward about twice as many items,
// so that fewer long items are left running at the end of its launch (32 was slower:
// each item has a fixed cost, its setup reads and staging, of some 10 us under load)
constexpr int kCkptStride = 64;
static_assert(128 % kFwdGroup == 0 && kCkptStride % kFwdGroup == 0 && 128 % kCkptStride == 0,
              "batches and checkpoint strides hold whole groups");

template <int TS, int BATCH>
__global__ __launch_bounds__(TS* TS) void k_blend_fwd(ViewTable vt, Rules ru, Records rec, const uint2* ranges,
                                                     const uint32_t* vals, float* T_final, uint32_t* n_contrib,
                                                     TileQueue q, Ckpt ck) {
  constexpr int NT = TS * TS;
  constexpr int CK = kCkptStride;
  __shared__ float4 s_r0[BATCH];
  __shared__ float4 s_r1[BATCH];
  __shared__ float4 s_rgb[BATCH];
  __shared__ int s_item;
  __shared__ uint32_t s_nmax;
  int tile_of_block = 0;
  // checkpoint k: the state in front of list entry k * CK
  auto checkpoint = [&](int k, float T, float C0, float C1, float C2, float D) {
    if (k > ck.kmax) return;
    float* st = ck.state + (int64_t(tile_of_block) * ck.kmax + (k - 1)) * (5 * NT) + threadIdx.x;
    st[0] = T;
    st[NT] = C0;
    st[2 * NT] = C1;
    st[3 * NT] = C2;
    st[4 * NT] = D;
  };
  for (;;) {
    int qprio;
    const int tile = next_tile(q, q.ctrl + kHeadFwd, vt.total_tiles, &s_item, &qprio);
    if (tile < 0) return;
    tile_of_block = tile;
    if (threadIdx.x == 0) s_nmax = 0;
    const ViewDev& cam = vt.v[view_of_tile(vt, tile)];
    const int lt = tile - cam.tile_off;
    const int ty = lt / cam.tiles_x, tx = lt - ty * cam.tiles_x;
    const int px = tx * TS + int(threadIdx.x % TS), py = ty * TS + int(threadIdx.x / TS);
    const bool inside = px < cam.W && py < cam.H;
    const uint2 rg = ranges[tile];
    const int n = int(rg.y - rg.x);
    const float fpx = float(px), fpy = float(py);
    float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
    uint32_t last = 0;
    bool done = !inside;
    // the heaviest tiles (first in the queue) bound the kernel's duration: their
    // wavefronts take issue priority from the start; any tile still running after
    // several batches is raised too
    set_wave_prio(qprio);
    for (int b0 = 0; b0 < n; b0 += BATCH) {
      if (__syncthreads_count(!done) == 0) break;
      if (b0 > 0 && b0 <= 3 * BATCH && b0 % BATCH == 0) set_wave_prio(max(qprio, b0 / BATCH));
      if (b0 > 0) checkpoint(b0 / CK, T, C0, C1, C2, D);
      const int cnt = min(BATCH, n - b0);
      for (int j = threadIdx.x; j < BATCH && b0 + j < n; j += NT)
        stage_record(rec, vals[rg.x + b0 + j], s_r0[j], s_r1[j], s_rgb[j]);
      // a partial batch is padded to a multiple of kFwdGroup with splats of opacity -1,
      // whose alpha (-1) is below any skip threshold (which is >= 0): no pixel takes them
      for (int j = cnt + int(threadIdx.x); j < ((cnt + kFwdGroup - 1) & ~(kFwdGroup - 1)); j += NT) {
        s_r0[j] = make_float4(0.f, 0.f, 0.f, 0.f);
        s_r1[j] = make_float4(0.f, -1.f, 0.f, 0.f);
        s_rgb[j] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
      __syncthreads();
      // kFwdGroup staged entries at a time: their splat values do not depend on the
      // running transmittance, so they are evaluated together (LDS reads and exponentials
      // overlap); compositing then runs in list order, straight-line: a lane that has
      // stopped, or for which the splat is below the skip threshold, adds exact zeros and
      // keeps T.  The wavefront leaves the batch once all its lanes have stopped.
      for (int j = 0; j < cnt; j += kFwdGroup) {
        if (__ballot(!done) == 0ull) break;
        if (j > 0 && j % CK == 0) checkpoint((b0 + j) / CK, T, C0, C1, C2, D);
        float a4[kFwdGroup], z4[kFwdGroup];
        float4 c4[kFwdGroup];
#pragma unroll
        for (int u = 0; u < kFwdGroup; ++u) {
          const float4 r0 = s_r0[j + u];
          const float4 r1 = s_r1[j + u];
          c4[u] = s_rgb[j + u];
          float G;
          a4[u] = splat_alpha(fpx - r0.x, fpy - r0.y, r0.z, r0.w, r1.x, r1.y, G);
          z4[u] = r1.z;
        }
        // The group in list order with a short dependency chain: Tk[u] is the
        // transmittance in front of entry u as if no stop came first (a plain chain of
        // products); since transmittance never rises, the pixel has stopped before
        // entry u exactly when it was stopped on entry or Tk[u] < T_min, and up to that
        // entry Tk[u] is the true transmittance.  So every entry's decision and weight
        // are those of the entry-by-entry recurrence (same products, same order), and
        // the transmittance after the group is Tk at the first stopped position.
        float Tk[kFwdGroup + 1], alv[kFwdGroup];
        Tk[0] = T;
#pragma unroll
        for (int u = 0; u < kFwdGroup; ++u) {
          alv[u] = !(a4[u] < ru.amin) ? fminf(a4[u], ru.amax) : 0.f;  // 0: skipped, keeps T
          Tk[u + 1] = Tk[u] * (1.f - alv[u]);
        }
        float Tn = Tk[kFwdGroup];
#pragma unroll
        for (int u = kFwdGroup - 1; u >= 0; --u) Tn = (done || Tk[u] < ru.Tmin) ? Tk[u] : Tn;
        uint32_t lg = 0;  // 1 + the group position of the group's last contributor, 0: none
#pragma unroll
        for (int u = 0; u < kFwdGroup; ++u) {
          const bool act = !(done || Tk[u] < ru.Tmin) && !(a4[u] < ru.amin);
          const float wgt = act ? alv[u] * Tk[u] : 0.f;
          C0 += c4[u].x * wgt;
          C1 += c4[u].y * wgt;
          C2 += c4[u].z * wgt;
          D += z4[u] * wgt;
          lg = act ? uint32_t(u + 1) : lg;
        }
        last = lg ? uint32_t(b0 + j) + lg : last;
        T = Tn;
        done = done || Tn < ru.Tmin;
      }
    }
    if (inside) {
      const int64_t P = int64_t(cam.W) * cam.H;
      const int64_t pix = int64_t(py) * cam.W + px;
      cam.color[pix] = C0 + T * ru.bg[0];
      cam.color[P + pix] = C1 + T * ru.bg[1];
      cam.color[2 * P + pix] = C2 + T * ru.bg[2];
      if (cam.depth) cam.depth[pix] = !ru.norm_depth ? D : (T < 1.f ? D / (1.f - T) : 0.f);
      if (cam.alpha) cam.alpha[pix] = 1.f - T;
      T_final[cam.pix_off + pix] = T;
      n_contrib[cam.pix_off + pix] = last;
      ck.acc[cam.pix_off + pix] = make_float4(C0, C1, C2, D);
    }
    const uint32_t wl = wave_max_u32(last);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) atomicMax(&s_nmax, wl);
    __syncthreads();
    if (threadIdx.x == 0) ck.tile_nmax[tile] = s_nmax;
  }
}

// Per pixel, the list entries in front of its last contributor that passed the skip rule
// (a statistic of the forward, for inspection): the forward's alpha of each entry
// (the same staged values and splat evaluation) compared with the threshold.
__global__ __launch_bounds__(256) void k_count_used(ViewTable vt, Rules ru, Records rec, const uint2* ranges,
                                                   const uint32_t* vals, const uint32_t* n_contrib, int tile,
                                                   int64_t total_pix, uint32_t* n_used) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= total_pix) return;
  int v = 0;
  for (int k = 1; k < vt.nviews; ++k)
    if (i >= vt.v[k].pix_off) v = k;
  const ViewDev& cam = vt.v[v];
  const int64_t pix = i - cam.pix_off;
  const int py = int(pix / cam.W), px = int(pix - int64_t(py) * cam.W);
  const uint2 rg = ranges[cam.tile_off + (py / tile) * cam.tiles_x + px / tile];
  const uint32_t nc = n_contrib[i];
  const float fpx = float(px), fpy = float(py);
  uint32_t used = 0;
  for (uint32_t j = 0; j < nc && rg.x + j < rg.y; ++j) {
    float4 r0, r1, rgb;
    stage_record(rec, vals[rg.x + j], r0, r1, rgb);
    float G;
    const float a = splat_alpha(fpx - r0.x, fpy - r0.y, r0.z, r0.w, r1.x, r1.y, G);
    used += !(a < ru.amin) ? 1u : 0u;
  }
  n_used[i] = used;
}

// ------------------------------------------------------------------------------------
// Backward work items, in the tile queue's longest-first order: (tile, k) for every
// checkpoint stride k that holds a contributor of some pixel of the tile, up to the
// tile's last checkpoint; one more item (tile, kmax) covers all later entries.  Listed by
// one whole block of NT threads (red: NT / 64 words, carry: one): k_bwd_items, or in a
// captured step the last block of the loss kernel.
template <int NT>
__device__ void list_bwd_items(const uint32_t* order, int total, int batch, const Ckpt& ck, uint32_t* ctrl,
                               uint32_t* red, uint32_t& carry) {
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int i0 = 0; i0 < total; i0 += NT) {
    const int i = i0 + threadIdx.x;
    uint32_t t = 0, ni = 0;
    if (i < total) {
      t = order[i];
      const uint32_t nb = (ck.tile_nmax[t] + uint32_t(batch) - 1u) / uint32_t(batch);
      ni = nb <= uint32_t(ck.kmax) ? nb : uint32_t(ck.kmax) + 1u;
    }
    const uint32_t base = carry + block_exclusive_scan_u32(ni, red);
    for (uint32_t k = 0; k < ni; ++k)
      if (int64_t(base) + k < ck.cap_items) ck.items[base + k] = make_uint2(t, k);
    __syncthreads();
    if (threadIdx.x == NT - 1) carry = base + ni;
    __syncthreads();
  }
  if (threadIdx.x == 0) ctrl[kItems] = uint32_t(min<int64_t>(carry, ck.cap_items));
}

__global__ __launch_bounds__(1024) void k_bwd_items(const uint32_t* order, int total, int batch, Ckpt ck,
                                                   uint32_t* ctrl) {
  __shared__ uint32_t red[16], carry;
  list_bwd_items<1024>(order, total, batch, ck, ctrl, red, carry);
}

// ------------------------------------------------------------------------------------
// K7: L1 loss and its gradient with respect to the rendered colour and depth
// ------------------------------------------------------------------------------------
// With order non-null (a captured step) the last block also lists the backward's work
// items (list_bwd_items) for the tiles the forward just composited.
__global__ __launch_bounds__(256) void k_loss_l1(ViewTable vt, float depth_w, float* partial, const uint32_t* order,
                                                int total_tiles, int stride, Ckpt ck, uint32_t* ctrl) {
  __shared__ float red[4];
  __shared__ uint32_t ired[4], icarry;
  const ViewDev& cam = vt.v[blockIdx.y];
  const int64_t P = int64_t(cam.W) * cam.H;
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  float part = 0.f;
  if (i < P) {
    const float inv3p = 1.f / float(3 * P), invp = 1.f / float(P);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float d = cam.color[ch * P + i] - cam.t_color[ch * P + i];
      part += fabsf(d) * inv3p;
      cam.lg_color[ch * P + i] = (d > 0.f ? inv3p : (d < 0.f ? -inv3p : 0.f));
    }
    float gd = 0.f;
    if (cam.t_depth) {
      const float td = cam.t_depth[i];
      if (td > 0.f) {
        const float d = cam.depth[i] - td;
        part += depth_w * fabsf(d) * invp;
        gd = d > 0.f ? depth_w * invp : (d < 0.f ? -depth_w * invp : 0.f);
      }
    }
    if (cam.lg_depth) cam.lg_depth[i] = gd;
  }
  for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) partial[int64_t(blockIdx.y) * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
  if (order && blockIdx.x == gridDim.x - 1 && blockIdx.y == gridDim.y - 1)
    list_bwd_items<256>(order, total_tiles, stride, ck, ctrl, ired, icarry);
}

// the loss: the block partial sums added in a fixed order (deterministic) by one whole
// block of 256 threads (the eager sum below; in a captured step the first block of the
// backward projection), so both give the same bits
__device__ __forceinline__ void sum_loss_partials(const float* part, int count, float* loss, float* red) {
  float v = 0.f;
  for (int i = threadIdx.x; i < count; i += 256) v += part[i];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) *loss = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_loss_sum(const float* part, int count, float* loss) {
  __shared__ float red[4];
  sum_loss_partials(part, count, loss, red);
}

// ------------------------------------------------------------------------------------
// K8: backward compositing, back to front over each pixel's contributors; the
// transmittance before contributor i is T_{i+1} / (1 - alpha_i), and the colour/depth
// behind i is carried as a running blend.  The work is cut into (tile, stride) items that
// run independently: an item starts from the pixel's final state when its list ends in
// the item, else from the forward's checkpoint at the item's end.  So no wavefront walks
// more than one checkpoint stride until a tile's checkpoints run out.
//
// Each wavefront walks the staged batch only down from its own longest contributor list.
// The ten per-(pixel, splat) partials are summed across the wavefront with lane swaps
// and DPP (wave_sum10); with more than one wavefront per tile the wavefront sums meet
// in LDS and the block adds each splat's total to the 2D-gradient buffer once per item,
// with the atomics spread over all lanes.

// Block-uniform: the next backward work item, or -1; the first items (the heaviest
// tiles) take a higher wave priority, as in the forward.
__device__ __forceinline__ int next_item(uint32_t* head, int total, int* s_item) {
  __syncthreads();
  if (threadIdx.x == 0) {
    // every block takes exactly one value past the end, so the taker of the last one
    // is the last to touch the head: it resets it for the next backward
    const uint32_t v = atomicAdd(head, 1u);
    *s_item = int(v);
    if (v == uint32_t(total) + gridDim.x - 1u) *head = 0u;
  }
  __syncthreads();
  const int item = *s_item;
  if (item < total) set_wave_prio(queue_prio(item, total));
  return item < total ? item : -1;
}

// K8 with PPL vertically adjacent pixels per lane: with two (tiles of 16 and 32) a
// wavefront covers 128 pixels, so each splat's ten partials are reduced across the
// wavefront once for twice the pixels (the pair's partials are added first); tiles of 8
// use one.  Two per lane is the build's choice for the larger tiles (kBwdPixelsPerLane);
// four ran slower on the headline view.
//
// Per pixel, back to front, with g = dL/d(colour, depth) of the pixel and B the blend of
// g . (colour, depth) of the contributors behind (B = g . (bg, 0) behind the last):
//   T_i = T_(i+1) / (1 - alpha_i),  dL/dalpha_i = T_i (g . (c_i, z_i) - B) + gA T_final / (1 - alpha_i),
//   B <- alpha_i g . (c_i, z_i) + (1 - alpha_i) B,
// which is the per-channel recurrence of the colour behind, dotted with g once (g is fixed
// per pixel).  The splat's geometric partials are kept as moments of q = a dL/da over the
// pixel offsets, (sum q dx, sum q dy, sum q dx^2, sum q dx dy, sum q dy^2); the flush turns
// them into the centre and conic gradients with the splat's conic, once per splat.
struct BwdPixel {
  float T, Tfin, gC0, gC1, gC2, gD, gATf, B, fpy;
  int top;
};

// A pixel's state at the end of work item (tile, bf): its final state when the pixel's
// list ends inside the item, else the forward's checkpoint at the item's end, with the
// colour/depth behind = (total - in front + T_final bg) / T.
template <int TS>
__device__ __forceinline__ void bwd_pixel_setup(BwdPixel& s, const ViewDev& cam, const Rules& ru, const Ckpt& ck,
                                                const float* T_final, const uint32_t* n_contrib, int tile, int bf,
                                                int lo, int hi, int px, int py, int q) {
  constexpr int NP = TS * TS;  // pixels of a tile
  const bool inside = px < cam.W && py < cam.H;
  const int64_t P = int64_t(cam.W) * cam.H;
  const int64_t pix = int64_t(py) * cam.W + px;
  s.T = 1.f;
  s.Tfin = 1.f;
  s.gC0 = s.gC1 = s.gC2 = s.gD = s.gATf = s.B = 0.f;
  s.top = 0;
  s.fpy = float(py);
  if (!inside) return;
  const int nc = int(n_contrib[cam.pix_off + pix]);
  if (nc <= lo) return;
  s.Tfin = T_final[cam.pix_off + pix];
  float gA = 0.f;
  if (cam.g_color) {
    s.gC0 = cam.g_color[pix];
    s.gC1 = cam.g_color[P + pix];
    s.gC2 = cam.g_color[2 * P + pix];
  }
  if (cam.g_depth) s.gD = cam.g_depth[pix];
  if (cam.g_alpha) gA = cam.g_alpha[pix];
  if (ru.norm_depth) {  // output Dn = D / A, A = 1 - T_final: dL/dD = g / A, dL/dA -= g Dn / A
    const float A = 1.f - s.Tfin;
    if (A > 0.f) {
      const float Dn = ck.acc[cam.pix_off + pix].w / A;
      gA -= s.gD * Dn / A;
      s.gD = s.gD / A;
    } else {
      s.gD = 0.f;
    }
  }
  s.gATf = gA * s.Tfin;
  float BC0 = ru.bg[0], BC1 = ru.bg[1], BC2 = ru.bg[2], BD = 0.f;
  if (nc <= hi) {
    s.T = s.Tfin;
    s.top = nc;
  } else {  // only single-stride items end before the list: checkpoint bf + 1 <= kmax
    const float* st = ck.state + (int64_t(tile) * ck.kmax + bf) * (5 * NP) + q;
    const float4 acc = ck.acc[cam.pix_off + pix];
    s.T = st[0];
    const float inv = 1.f / s.T;
    BC0 = (acc.x - st[NP] + s.Tfin * ru.bg[0]) * inv;
    BC1 = (acc.y - st[2 * NP] + s.Tfin * ru.bg[1]) * inv;
    BC2 = (acc.z - st[3 * NP] + s.Tfin * ru.bg[2]) * inv;
    BD = (acc.w - st[4 * NP]) * inv;
    s.top = hi;
  }
  s.B = s.gC0 * BC0 + s.gC1 * BC1 + s.gC2 * BC2 + s.gD * BD;
}

// One (pixel, splat) step back to front, adding the pixel's partials to g: the five
// geometric moments, dL/dopacity's sum of dL/da G, and the colour/depth weights.  A lane
// that does not take part (past its list, or below the skip threshold) takes alpha = 0,
// which leaves B unchanged and adds zeros; its T is kept by a select (1 / (1 - 0) is not
// relied on to be exact).
// Returns q = dL/da a, whose offset moments the caller forms (the pixels of a lane share dx).
__device__ __forceinline__ float bwd_pixel_step(BwdPixel& s, bool act, float a, float G, const float4& r1,
                                                const float4& c, const Rules& ru, float (&g)[10]) {
  const bool below = a <= ru.amax;  // not clamped (shared by the clamp and its gradient)
  const float al = act ? (below ? a : ru.amax) : 0.f;
  const float om = 1.f - al;
  const float iom = __builtin_amdgcn_rcpf(om);
  s.T = s.T * iom;  // a lane that does not take the entry has om = 1, iom = 1 exactly
  const float wgt = al * s.T;
  g[6] += s.gC0 * wgt;
  g[7] += s.gC1 * wgt;
  g[8] += s.gC2 * wgt;
  g[9] += s.gD * wgt;
  const float S = s.gC0 * c.x + s.gC1 * c.y + s.gC2 * c.z + s.gD * r1.z;
  const float dal = s.T * (S - s.B) + s.gATf * iom;
  s.B = al * S + om * s.B;
  const float da = (act && below) ? dal : 0.f;
  g[5] += da * G;
  return da * a;
}

// The splat-major flush of a batch's per-splat sums (s_g: ten per splat and wavefront,
// each wavefront writing only its own; summed over the wavefronts and cleared as they are
// read) into the 2D-gradient rows: the lanes of a wavefront add consecutive sums of a
// few splats, so one atomic instruction touches a few gradient rows (cache lines), not 64.
// The moments become gradients here: with the staged conic (a', b', c') = (A, 2B, C) (-log2 e / 2),
// (A dx + B dy, B dx + C dy) = -ln 2 (2a' dx + b' dy, b' dx + 2c' dy), so
//   dmu = -ln 2 (2a' Mx + b' My, b' Mx + 2c' My),  d(A, B, C) = -(Mxx / 2, Mxy, Myy / 2).
template <int NT, int NW, int SB>
__device__ __forceinline__ void flush_splat_sums(float (&s_g)[NW][SB][10], const uint32_t* s_id, const float4* s_r0,
                                                 const float4* s_r1, const float4* s_rgb, int nstage,
                                                 float* grad2d) {
  constexpr float kNegLn2 = -0.69314718055994531f;
  // the wavefronts' sums of slot (j, k), cleared as they are read
  auto take = [&](int j, int k) {
    float v = 0.f;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      v += s_g[w][j][k];
      s_g[w][j][k] = 0.f;
    }
    return v;
  };
  for (int i = threadIdx.x; i < 10 * nstage; i += NT) {
    const int j = i / 10, k = i - 10 * j;
    if (k == 1) continue;  // the centre's y gradient goes with its x gradient (k == 0)
    float* dst = grad2d + int64_t(s_id[j]) * kGrad2D;
    if (k == 0) {
      const float mx = take(j, 0), my = take(j, 1);
      if (mx != 0.f || my != 0.f) {
        const float b = s_r0[j].w;   // b'
        const float a2 = s_r1[j].w;  // 2 a'
        const float c2 = s_rgb[j].w; // 2 c'
        unsafeAtomicAdd(dst, kNegLn2 * (a2 * mx + b * my));
        unsafeAtomicAdd(dst + 1, kNegLn2 * (b * mx + c2 * my));
      }
      continue;
    }
    const float v = take(j, k);
    if (v != 0.f) unsafeAtomicAdd(dst + k, k == 3 ? -v : ((k == 2 || k == 4) ? -0.5f * v : v));
  }
}

template <int TS, int BATCH, int PPL>
__global__ __launch_bounds__(TS* TS / PPL) void k_blend_bwd2(ViewTable vt, Rules ru, Records rec,
                                                            const uint2* ranges, const uint32_t* vals,
                                                            const float* T_final, const uint32_t* n_contrib,
                                                            float* grad2d, TileQueue q, Ckpt ck) {
  constexpr int NT = TS * TS / PPL;  // threads: pixels (PPL r + i, c), i < PPL, for t = r TS + c
  constexpr int NW = NT / 64;        // wavefronts
  constexpr int SB = kCkptStride;    // entries staged at a time: one checkpoint stride
  __shared__ float4 s_r0[SB];
  __shared__ float4 s_r1[SB];
  __shared__ float4 s_rgb[SB];
  __shared__ uint32_t s_id[SB];
  __shared__ float s_g[NW][SB][10];  // per wavefront and staged splat, its ten sums
  __shared__ uint32_t s_max;
  __shared__ int s_item;
  for (int i = threadIdx.x; i < NW * 10 * SB; i += NT) (&s_g[0][0][0])[i] = 0.f;
  const int wv = int(threadIdx.x) >> 6;
  const int total = int(q.ctrl[kItems]);
  const int lane = threadIdx.x & 63;
  const int cx = int(threadIdx.x % TS), ry = PPL * int(threadIdx.x / TS);
  for (;;) {
    const int item = next_item(q.ctrl + kHeadBwd, total, &s_item);
    if (item < 0) return;
    const uint2 it = ck.items[item];
    const int tile = int(it.x), bf = int(it.y);
    const ViewDev& cam = vt.v[view_of_tile(vt, tile)];
    const int lt = tile - cam.tile_off;
    const int ty = lt / cam.tiles_x, tx = lt - ty * cam.tiles_x;
    const int px = tx * TS + cx, py = ty * TS + ry;
    const uint2 rg = ranges[tile];
    constexpr int CK = kCkptStride;  // checkpoint stride of the forward
    const int lo = bf * CK;        // the item's list entries: [lo, hi)
    const int hi = bf < ck.kmax ? lo + CK : int(rg.y - rg.x);
    BwdPixel p[PPL];
    int ptop = 0;
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
      bwd_pixel_setup<TS>(p[i], cam, ru, ck, T_final, n_contrib, tile, bf, lo, hi, px, py + i, (ry + i) * TS + cx);
      ptop = max(ptop, p[i].top);
    }
    const int wmax = int(wave_max_u32(uint32_t(ptop)));
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    if (lane == 0 && wmax) atomicMax(&s_max, uint32_t(wmax));
    __syncthreads();
    const int bmax = int(s_max);
    const float fpx = float(px);
    for (int bend = bmax; bend > lo; bend -= SB) {
      const int bstart = max(lo, bend - SB);
      const int nstage = bend - bstart;
      __syncthreads();
      for (int j = threadIdx.x; j < nstage; j += NT) {
        const uint32_t id = vals[rg.x + bstart + j];
        s_id[j] = id;
        stage_record(rec, id, s_r0[j], s_r1[j], s_rgb[j]);
      }
      __syncthreads();
      for (int j = min(nstage, wmax - bstart) - 1; j >= 0; --j) {
        const float4 r0 = s_r0[j];
        const float4 r1 = s_r1[j];
        const float dx = fpx - r0.x;
        float dy[PPL], a[PPL], G[PPL];
        bool act[PPL];
        bool any = false;
#pragma unroll
        for (int i = 0; i < PPL; ++i) {
          dy[i] = p[i].fpy - r0.y;
          a[i] = splat_alpha(dx, dy[i], r0.z, r0.w, r1.x, r1.y, G[i]);
          act[i] = bstart + j < p[i].top && !(a[i] < ru.amin);
          any = any || act[i];
        }
        if (__ballot(any) == 0ull) continue;
        const float4 c = s_rgb[j];
        float gv[10] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        // the offset moments of the lane's pixels (one column: one dx): Σq, Σq dy, Σq dy²,
        // then Σq dx = dx Σq, Σq dx² = dx² Σq, Σq dx dy = dx Σq dy
        float Q = 0.f, QY = 0.f, QYY = 0.f;
#pragma unroll
        for (int i = 0; i < PPL; ++i) {
          const float q = bwd_pixel_step(p[i], act[i], a[i], G[i], r1, c, ru, gv);
          const float qy = q * dy[i];
          Q = i == 0 ? q : Q + q;
          QY = i == 0 ? qy : QY + qy;
          QYY = i == 0 ? qy * dy[i] : QYY + qy * dy[i];
        }
        const float Qx = Q * dx;
        gv[0] = Qx;
        gv[1] = QY;
        gv[2] = Qx * dx;
        gv[3] = QY * dx;
        gv[4] = QYY;
        float w0, w1, w2;
        wave_sum10(gv, w0, w1, w2);
        if ((lane & 15) == 0) {  // one lane per row stores its row's totals
          const int row = lane >> 4;
          const int k = row == 1 ? 2 : (row == 2 ? 1 : row);
          s_g[wv][j][k] = w0;  // this wavefront's own slots: plain stores
          s_g[wv][j][4 + k] = w1;
          if (!(row & 1)) s_g[wv][j][8 + (row >> 1)] = w2;
        }
      }
      __syncthreads();
      flush_splat_sums<NT, NW, SB>(s_g, s_id, s_r0, s_r1, s_rgb, nstage, grad2d);
    }
  }
}

// ------------------------------------------------------------------------------------
// K9: chain rule per Gaussian, summed over views in view order
// ------------------------------------------------------------------------------------
__device__ __forceinline__ void store_grad(float* p, float v, int acc) {
  if (acc)
    *p += v;
  else
    *p = v;
}

// K9a: the colour term.  Four lanes per Gaussian, one per colour channel (the fourth
// idles), so a lane holds one channel's K coefficients.  Per visible view: the basis at
// the view direction, the channel's colour before the clamp, the coefficient gradient
// Y_k * dL/dc (zero where the clamp is active) and the view-direction gradient, summed
// over the channel lanes and taken through the normalisation to the mean (dp_sh).
// Coefficients pass through LDS so the [N, K, 3] loads and stores are contiguous; a
// Gaussian invisible in every view reads none and gets zero gradients.
constexpr int kShGaussians = 64;  // Gaussians per block of k_project_bwd_sh

template <int DEG>
__global__ __launch_bounds__(256) void k_project_bwd_sh(GaussDev g, ViewTable vt, Records rec, const float* grad2d,
                                                        GradOut out, float* dp_sh, AdamDev adam) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  constexpr int KK = K * 3;
  constexpr bool kVec = KK % 4 == 0;  // degrees 1 and 3: whole float4s per Gaussian
  constexpr int STRIDE = KK | 1;
  __shared__ float s_sh[kShGaussians * STRIDE];
  __shared__ uint32_t s_vis[kShGaussians];
  const int t = threadIdx.x;
  const int64_t g0 = int64_t(blockIdx.x) * kShGaussians;
  const int nb = int(min<int64_t>(kShGaussians, g.n - g0));
  const int gl = t >> 2, ch = t & 3;
  const int64_t gi = g0 + gl;
  // this lane's mean and first view's colour gradient, loaded before the block stages the
  // coefficients (their latency overlaps the staging)
  float p0 = 0.f, p1 = 0.f, p2 = 0.f, dc0 = 0.f;
  uint32_t cnt0 = 0;
  if (gl < nb && ch < 3) {
    cnt0 = rec.counts[gi];
    if (cnt0) {
      p0 = g.means[gi * 3];
      p1 = g.means[gi * 3 + 1];
      p2 = g.means[gi * 3 + 2];
      dc0 = grad2d[gi * kGrad2D + 6 + ch];
    }
  }
  if (t < kShGaussians) {
    uint32_t vis = 0;
    if (t < nb)
      for (int v = 0; v < vt.nviews; ++v) vis |= rec.counts[int64_t(v) * g.n + g0 + t];
    s_vis[t] = vis;
  }
  __syncthreads();
  // 16-byte loads where the array allows them (with KK a multiple of 4 a float4 never
  // straddles two Gaussians)
  const bool vec_in = kVec && (reinterpret_cast<uintptr_t>(g.sh) & 15u) == 0;
  if (vec_in) {
    const float4* src = reinterpret_cast<const float4*>(g.sh + g0 * KK);
    for (int i = t; i < nb * (KK / 4); i += 256) {
      const int r = (4 * i) / KK, j = 4 * i - r * KK;
      const float4 v = s_vis[r] ? src[i] : make_float4(0.f, 0.f, 0.f, 0.f);
      float* d = s_sh + r * STRIDE + j;
      d[0] = v.x;
      d[1] = v.y;
      d[2] = v.z;
      d[3] = v.w;
    }
  } else {
    for (int i = t; i < nb * KK; i += 256) {
      const int r = i / KK;
      s_sh[r * STRIDE + (i - r * KK)] = s_vis[r] ? g.sh[g0 * KK + i] : 0.f;
    }
  }
  __syncthreads();
  const bool mine = gl < nb && s_vis[gl] != 0u;
  float dsh[K], dp[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < K; ++k) dsh[k] = 0.f;
  if (mine && ch < 3) {
    float shc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) shc[k] = s_sh[gl * STRIDE + k * 3 + ch];
    if (!cnt0) {  // visible only in later views: the mean was not loaded above
      p0 = g.means[gi * 3];
      p1 = g.means[gi * 3 + 1];
      p2 = g.means[gi * 3 + 2];
    }
    for (int v = 0; v < vt.nviews; ++v) {
      const int64_t rid = int64_t(v) * g.n + gi;
      if ((v == 0 ? cnt0 : rec.counts[rid]) == 0) continue;
      const ViewDev& cam = vt.v[v];
      const float d0 = p0 - cam.cam_pos[0], d1 = p1 - cam.cam_pos[1], d2 = p2 - cam.cam_pos[2];
      const float il = 1.f / __builtin_sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
      const float vx = d0 * il, vy = d1 * il, vz = d2 * il;
      float Y[K];
      sh_basis<DEG>(vx, vy, vz, Y);
      float raw = 0.5f;
#pragma unroll
      for (int k = 0; k < K; ++k) raw += shc[k] * Y[k];
      const float dc = raw > 0.f ? (v == 0 ? dc0 : grad2d[rid * kGrad2D + 6 + ch]) : 0.f;
#pragma unroll
      for (int k = 0; k < K; ++k) dsh[k] += Y[k] * dc;
      if (DEG > 0) {
        float wk[K], dv[3];
#pragma unroll
        for (int k = 0; k < K; ++k) wk[k] = shc[k] * dc;
        sh_grad_dot<DEG>(vx, vy, vz, wk, dv);
        const float vd = dv[0] * vx + dv[1] * vy + dv[2] * vz;
        dp[0] += (dv[0] - vx * vd) * il;
        dp[1] += (dv[1] - vy * vd) * il;
        dp[2] += (dv[2] - vz * vd) * il;
      }
    }
  }
  // the direction term is linear in the coefficients: sum the channel lanes (a quad)
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    dp[i] += dpp_move<0xB1, 0xF>(dp[i]);
    dp[i] += dpp_move<0x4E, 0xF>(dp[i]);
  }
  if (mine && ch == 0)
#pragma unroll
    for (int i = 0; i < 3; ++i) dp_sh[gi * 3 + i] = dp[i];
  if (!out.sh && !adam.on) return;
  __syncthreads();
  if (gl < nb && ch < 3)
#pragma unroll
    for (int k = 0; k < K; ++k) s_sh[gl * STRIDE + k * 3 + ch] = dsh[k];
  __syncthreads();
  if (adam.on) {  // one Adam step of every coefficient of the block's Gaussians, in place
    if (adam.skip && *adam.skip) return;  // the step overflowed: parameters stay as they are
    const float bc1 = adam.bc[0], bc2 = adam.bc[1];
    auto al = [](const float* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
    if (kVec && al(adam.p[G_SH]) && al(adam.m[G_SH]) && al(adam.v[G_SH])) {  // 16-byte accesses
      const int64_t e0 = g0 * (KK / 4);
      for (int i = t; i < nb * (KK / 4); i += 256) {
        const int r = (4 * i) / KK, j = 4 * i - r * KK;
        const float* gs = s_sh + r * STRIDE + j;
        float4 x = reinterpret_cast<const float4*>(adam.p[G_SH])[e0 + i];
        float4 m = reinterpret_cast<const float4*>(adam.m[G_SH])[e0 + i];
        float4 v = reinterpret_cast<const float4*>(adam.v[G_SH])[e0 + i];
        auto lr = [&](int k) { return j + k < 3 ? adam.lr[G_SH] : adam.lr[G_SH + 1]; };
        x.x = adam_value<G_SH>(x.x, gs[0], m.x, v.x, lr(0), adam, bc1, bc2);
        x.y = adam_value<G_SH>(x.y, gs[1], m.y, v.y, lr(1), adam, bc1, bc2);
        x.z = adam_value<G_SH>(x.z, gs[2], m.z, v.z, lr(2), adam, bc1, bc2);
        x.w = adam_value<G_SH>(x.w, gs[3], m.w, v.w, lr(3), adam, bc1, bc2);
        reinterpret_cast<float4*>(adam.p[G_SH])[e0 + i] = x;
        reinterpret_cast<float4*>(adam.m[G_SH])[e0 + i] = m;
        reinterpret_cast<float4*>(adam.v[G_SH])[e0 + i] = v;
      }
      return;
    }
    for (int i = t; i < nb * KK; i += 256) {
      const int r = i / KK, j = i - r * KK;
      const int64_t e = g0 * KK + i;
      adam_apply<G_SH>(adam, e, adam.p[G_SH][e], s_sh[r * STRIDE + j], j < 3 ? adam.lr[G_SH] : adam.lr[G_SH + 1],
                       bc1, bc2);
    }
    return;
  }
  if (kVec && (reinterpret_cast<uintptr_t>(out.sh) & 15u) == 0 && !out.accumulate) {
    float4* dst = reinterpret_cast<float4*>(out.sh + g0 * KK);
    for (int i = t; i < nb * (KK / 4); i += 256) {
      const int r = (4 * i) / KK, j = 4 * i - r * KK;
      const float* v = s_sh + r * STRIDE + j;
      dst[i] = make_float4(v[0], v[1], v[2], v[3]);
    }
    return;
  }
  for (int i = t; i < nb * KK; i += 256) {
    const int r = i / KK;
    store_grad(out.sh + g0 * KK + i, s_sh[r * STRIDE + (i - r * KK)], out.accumulate);
  }
}

// K9b: the geometric chain rule, one thread per Gaussian; adds the colour term's
// gradient with respect to the mean (dp_sh, from K9a).
__global__ __launch_bounds__(kProjThreads) void k_project_bwd_geo(GaussDev g, ViewTable vt, Rules ru, Records rec,
                                                                  const float* grad2d, const float* dp_sh,
                                                                  GradOut out, AdamDev adam, const float* loss_part,
                                                                  int loss_np, float* loss) {
  __shared__ float lred[4];
  // a captured step adds up its loss here (block-uniform; no launch of its own)
  if (loss && blockIdx.x == 0) sum_loss_partials(loss_part, loss_np, loss, lred);
  const int64_t gi = int64_t(blockIdx.x) * kProjThreads + threadIdx.x;
  if (gi >= g.n) return;
  // the geometry is read for a Gaussian some view sees (or for the Adam step, which moves
  // every element); the others only get zero gradients
  uint32_t seen = 0;
  for (int v = 0; v < vt.nviews && !seen; ++v) seen = rec.counts[int64_t(v) * g.n + gi];
  float p[3] = {0.f, 0.f, 0.f}, s[3] = {0.f, 0.f, 0.f}, q[4] = {0.f, 0.f, 0.f, 0.f};
  if (seen || adam.on) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      p[i] = g.means[gi * 3 + i];
      s[i] = g.scales[gi * 3 + i];
    }
    const float4 q4 = reinterpret_cast<const float4*>(g.quats)[gi];
    q[0] = q4.x;
    q[1] = q4.y;
    q[2] = q4.z;
    q[3] = q4.w;
  }
  float dp[3] = {0.f, 0.f, 0.f}, ds[3] = {0.f, 0.f, 0.f}, dq[4] = {0.f, 0.f, 0.f, 0.f}, dop = 0.f;
  bool any = false;
  for (int v = 0; v < vt.nviews; ++v) {
    const int64_t rid = int64_t(v) * g.n + gi;
    if (rec.counts[rid] == 0) continue;
    any = true;
    const ViewDev& cam = vt.v[v];
    const float4* G4 = reinterpret_cast<const float4*>(grad2d + rid * kGrad2D);
    const float4 ga = G4[0], gb = G4[1], gc = G4[2];
    const float dmux = ga.x, dmuy = ga.y, dA = ga.z, dB = ga.w, dC = gb.x, dO = gb.y;
    const float dz = gc.y;
    Proj pr;
    discrete_stage(p, s, q, cam, ru.k, ru.lowpass, ru.guard, ru.jclamp, pr);
    float A, B, C;
    conic_of(pr.a, pr.b, pr.c, A, B, C);
    dop += dO;
    // conic -> projected covariance: dS = -Q G_Q Q with G_Q = [[dA, dB/2], [dB/2, dC]]
    const float hB = 0.5f * dB;
    const float QG00 = A * dA + B * hB, QG01 = A * hB + B * dC;
    const float QG10 = B * dA + C * hB, QG11 = B * hB + C * dC;
    const float S00 = -(QG00 * A + QG01 * B);
    const float S01 = -(QG00 * B + QG01 * C);
    const float S11 = -(QG10 * B + QG11 * C);
    // Sigma_hat = U U^T + lowpass I with U = T M: dU = 2 dS U
    float dU[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      dU[k] = 2.f * (S00 * pr.U[k] + S01 * pr.U[3 + k]);
      dU[3 + k] = 2.f * (S01 * pr.U[k] + S11 * pr.U[3 + k]);
    }
    // dT = dU M^T, dM = T^T dU
    float dT[6], dM[9];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        dT[i * 3 + j] = dU[i * 3 + 0] * pr.m[j * 3 + 0] + dU[i * 3 + 1] * pr.m[j * 3 + 1] + dU[i * 3 + 2] * pr.m[j * 3 + 2];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k) dM[j * 3 + k] = pr.T[j] * dU[k] + pr.T[3 + j] * dU[3 + k];
    // T = J W: dJ = dT W^T (only the four non-constant entries of J matter)
    const float* W = cam.R;
    const float dJ00 = dT[0] * W[0] + dT[1] * W[1] + dT[2] * W[2];
    const float dJ02 = dT[0] * W[6] + dT[1] * W[7] + dT[2] * W[8];
    const float dJ11 = dT[3] * W[3] + dT[4] * W[4] + dT[5] * W[5];
    const float dJ12 = dT[3] * W[6] + dT[4] * W[7] + dT[5] * W[8];
    const float tx = pr.tx, ty = pr.ty, tz = pr.tz;
    const float iz = 1.f / tz, iz2 = iz * iz, iz3 = iz2 * iz;
    const float fx = cam.fx, fy = cam.fy;
    // J02 = -fx x' / z^2 with x' = tx, or +-limit tz where clamped: d/dtx of a clamped
    // entry is 0 and its d/dtz is -J02 / tz (2 fx x' / z^3 halved); likewise J12
    const float kx = pr.clx ? 1.f : 2.f, ky = pr.cly ? 1.f : 2.f;
    const float dtx = (pr.clx ? 0.f : -fx * iz2 * dJ02) + fx * iz * dmux;
    const float dty = (pr.cly ? 0.f : -fy * iz2 * dJ12) + fy * iz * dmuy;
    const float dtz = -fx * iz2 * dJ00 + kx * fx * pr.txj * iz3 * dJ02 - fy * iz2 * dJ11 + ky * fy * pr.tyj * iz3 * dJ12 -
                      fx * tx * iz2 * dmux - fy * ty * iz2 * dmuy + dz;
#pragma unroll
    for (int j = 0; j < 3; ++j) dp[j] += W[j] * dtx + W[3 + j] * dty + W[6 + j] * dtz;
    // M = R diag(s)
    float dR[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        ds[j] += dM[i * 3 + j] * pr.r[i * 3 + j];
        dR[i * 3 + j] = dM[i * 3 + j] * s[j];
      }
    // R(q^) partials contracted with dR
    const float w = pr.qw, x = pr.qx, y = pr.qy, z = pr.qz;
    const float dqw = 2.f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    const float dqx = 2.f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.f * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] -
                             2.f * x * dR[8]);
    const float dqy = 2.f * (-2.f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] -
                             2.f * y * dR[8]);
    const float dqz = 2.f * (-2.f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.f * z * dR[4] + y * dR[5] +
                             x * dR[6] + y * dR[7]);
    const float qd = dqw * w + dqx * x + dqy * y + dqz * z;
    const float inq = 1.f / pr.nq;
    dq[0] += (dqw - w * qd) * inq;
    dq[1] += (dqx - x * qd) * inq;
    dq[2] += (dqy - y * qd) * inq;
    dq[3] += (dqz - z * qd) * inq;
  }
  if (any) {
#pragma unroll
    for (int i = 0; i < 3; ++i) dp[i] += dp_sh[gi * 3 + i];
  }
  if (adam.on) {  // one Adam step of the Gaussian's geometry, in place
    if (adam.skip && *adam.skip) return;  // the step overflowed: parameters stay as they are
    const float bc1 = adam.bc[0], bc2 = adam.bc[1];
#pragma unroll
    for (int i = 0; i < 3; ++i) adam_apply<G_MEANS>(adam, gi * 3 + i, p[i], dp[i], adam.lr[G_MEANS], bc1, bc2);
#pragma unroll
    for (int i = 0; i < 3; ++i) adam_apply<G_SCALES>(adam, gi * 3 + i, s[i], ds[i], adam.lr[G_SCALES], bc1, bc2);
#pragma unroll
    for (int i = 0; i < 4; ++i) adam_apply<G_QUATS>(adam, gi * 4 + i, q[i], dq[i], adam.lr[G_QUATS], bc1, bc2);
    adam_apply<G_OPAC>(adam, gi, g.opac[gi], dop, adam.lr[G_OPAC], bc1, bc2);
    return;
  }
  const int acc = out.accumulate;
  if (out.means)
    for (int i = 0; i < 3; ++i) store_grad(out.means + gi * 3 + i, dp[i], acc);
  if (out.scales)
    for (int i = 0; i < 3; ++i) store_grad(out.scales + gi * 3 + i, ds[i], acc);
  if (out.quats) {
    if (!acc && (reinterpret_cast<uintptr_t>(out.quats) & 15u) == 0)
      reinterpret_cast<float4*>(out.quats)[gi] = make_float4(dq[0], dq[1], dq[2], dq[3]);
    else
      for (int i = 0; i < 4; ++i) store_grad(out.quats + gi * 4 + i, dq[i], acc);
  }
  if (out.opac) store_grad(out.opac + gi, dop, acc);
}

inline unsigned blocks_for(int64_t n, int per) { return unsigned((n + per - 1) / per); }

}  // namespace

// ------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------
hipError_t launch_project(int deg, const GaussDev& g, const ViewTable& vt, const Rules& ru, int tile,
                          const Records& rec, uint2* blocksums, int nblk, float* zero_rows, uint32_t* ctrl,
                          int clear_words, float exact_k, hipStream_t s) {
  if (nblk == 0) return hipSuccess;
  dim3 grid(nblk), block(kProjThreads);
  const int cw = clear_words;
  switch (deg) {
    case 0: k_project<0><<<grid, block, 0, s>>>(g, vt, ru, tile, rec, blocksums, nblk, zero_rows, ctrl, cw, exact_k); break;
    case 1: k_project<1><<<grid, block, 0, s>>>(g, vt, ru, tile, rec, blocksums, nblk, zero_rows, ctrl, cw, exact_k); break;
    case 2: k_project<2><<<grid, block, 0, s>>>(g, vt, ru, tile, rec, blocksums, nblk, zero_rows, ctrl, cw, exact_k); break;
    default: k_project<3><<<grid, block, 0, s>>>(g, vt, ru, tile, rec, blocksums, nblk, zero_rows, ctrl, cw, exact_k); break;
  }
  return hipGetLastError();
}

hipError_t launch_scan_small(uint32_t* a, int count, unsigned long long* total, hipStream_t s) {
  k_scan_u32<<<1, 1024, 0, s>>>(a, count, total);
  return hipGetLastError();
}

hipError_t launch_scan_pairs(uint2* blocksums, int count, unsigned long long* totals, hipStream_t s) {
  k_scan_pairs<<<1, 1024, 0, s>>>(blocksums, count, totals);
  return hipGetLastError();
}

hipError_t launch_compact(int64_t n, int views, const Records& rec, const uint2* blocksums, int nblk,
                          unsigned long long* totals, int64_t cap_M, uint32_t* dkeys, uint32_t* dvals,
                          int64_t cap, uint32_t* overflow, bool raw, hipStream_t s) {
  if (nblk == 0) return hipSuccess;
  if (raw && int64_t(views) * nblk > kCompactRawMax) return hipErrorInvalidValue;
  k_compact<<<dim3(nblk, views), kProjThreads, 0, s>>>(n, rec, blocksums, nblk, totals, cap_M, dkeys, dvals, cap,
                                                        overflow, raw ? 1 : 0);
  return hipGetLastError();
}

template <int BITS>
static void radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, uint32_t* hist,
                       uint32_t* digit_tot, const unsigned long long* count, int64_t cap, const uint32_t* overflow,
                       int shift, int nblk, hipStream_t s, Timer* tm) {
  if (tm) tm->begin(K_RADIX_HIST);
  k_radix_hist<BITS><<<xcd_grid(nblk), kSortThreads, 0, s>>>(kin, count, cap, overflow, shift, hist, nblk);
  if (tm) tm->end(K_RADIX_HIST);
  if (tm) tm->begin(K_RADIX_ROWSCAN);
  k_radix_rowscan<<<1 << BITS, kSortThreads, 0, s>>>(hist, nblk, digit_tot);
  if (tm) tm->end(K_RADIX_ROWSCAN);
  if (tm) tm->begin(K_RADIX_SCATTER);
  k_radix_scatter<BITS><<<xcd_grid(nblk), kSortThreads, 0, s>>>(kin, vin, kout, vout, count, cap, overflow, shift, hist,
                                                      digit_tot, nblk);
  if (tm) tm->end(K_RADIX_SCATTER);
}

int radix_hist_words(int64_t cap) { return int((cap + kSortTile - 1) / kSortTile) << kSortBits; }

hipError_t launch_radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                             uint32_t* hist, uint32_t* digit_tot, const unsigned long long* count, int64_t cap,
                             const uint32_t* overflow, int key_bits, bool* result_in_alt, int* passes, hipStream_t s,
                             Timer* tm) {
  const int np = (key_bits + kSortBits - 1) / kSortBits;
  *passes = 0;
  *result_in_alt = false;
  if (cap <= 1 || np == 0) return hipSuccess;
  *passes = np;
  const int nblk = int((cap + kSortTile - 1) / kSortTile);
  uint32_t* kin = keys;
  uint32_t* vin = vals;
  uint32_t* kout = keys_alt;
  uint32_t* vout = vals_alt;
  for (int p = 0; p < np; ++p) {
    radix_pass<kSortBits>(kin, vin, kout, vout, hist, digit_tot, count, cap, overflow, kSortBits * p, nblk, s, tm);
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
  *result_in_alt = (np % 2) == 1;
  return hipGetLastError();
}

BinPlan bin_plan(const ViewTable& vt, int64_t cap_vis, int64_t cap_M) {
  // one 64-item round per wavefront (chunks and segments of 64: the most placement waves
  // in parallel) while the count arrays stay within kMaxBinCounts entries; more rounds
  // (fewer, longer chunks) beyond that
  BinPlan p{};
  p.rows = vt.total_rows;
  const int64_t max_chunks = std::max<int64_t>(1, kMaxBinCounts / std::max(1, p.rows));
  p.rounds1 = int(std::max<int64_t>(1, (cap_vis + 64 * max_chunks - 1) / (64 * max_chunks)));
  p.nch1 = int(std::max<int64_t>(1, (cap_vis + 64 * p.rounds1 - 1) / (64 * p.rounds1)));
  const int64_t max_segs = std::max<int64_t>(1024, kMaxBinCounts / std::max(1, vt.max_tiles_x));
  p.rounds2 = int(std::max<int64_t>(1, (cap_M + 64 * max_segs - 1) / (64 * max_segs)));
  const int64_t S2 = 64 * int64_t(p.rounds2);
  const int64_t segs = (cap_M + S2 - 1) / S2;
  p.cap_M = cap_M;
  p.cap_seg = segs + p.rows;
  p.cap_flat = int64_t(vt.max_tiles_x) * segs + vt.total_tiles;
  return p;
}

// exclusive scan of a[0, min(*count, cap)) (or of a[0, cap) without count); total to *total
static void scan_u32(uint32_t* a, int64_t cap, const unsigned long long* count, uint32_t* part,
                     unsigned long long* total, hipStream_t s) {
  const int nb = int((cap + kScanTile - 1) / kScanTile);
  k_scan_reduce<<<nb, 256, 0, s>>>(a, cap, count, part);
  k_scan_down<<<nb, 256, 0, s>>>(a, cap, count, part, total);
}

hipError_t launch_bin(const ViewTable& vt, int64_t n, const Records& rec, const uint32_t* dvals,
                      const unsigned long long* nvis, int64_t cap_vis, const BinPlan& plan, uint32_t* vals,
                      uint2* ranges, uint32_t* ctrl, float exact_k, int tile, const uint32_t* hint,
                      uint32_t* order, hipStream_t s, Timer* tm) {
  if (vt.total_tiles == 0) return hipSuccess;
  if (cap_vis == 0 || plan.cap_M == 0 || plan.rows == 0) {
    k_fill_u32<<<blocks_for(int64_t(vt.total_tiles) * 2, 256), 256, 0, s>>>(reinterpret_cast<uint32_t*>(ranges), 0u,
                                                                             int64_t(vt.total_tiles) * 2);
    k_tile_order<<<1, 1024, 0, s>>>(ranges, hint, vt.total_tiles, order);
    return hipGetLastError();
  }
  auto B = [&](int k) { if (tm) tm->begin(k); };
  auto E = [&](int k) { if (tm) tm->end(k); };
  uint32_t* overflow = ctrl + kOverflow;
  const size_t lds_rows = size_t(plan.rows) * 4, lds_cols = size_t(vt.max_tiles_x) * 4;
  const int64_t n1 = int64_t(plan.rows) * plan.nch1;
  const int g_count = int(std::min<int64_t>((plan.cap_seg + 3) / 4, 4096));
  const int g_scatter = int(std::min<int64_t>(plan.cap_seg, 16384));
  const int g_scatter4 = int(std::min<int64_t>((plan.cap_seg + 3) / 4, 4096));
  B(K_BIN_COUNT);
  k_bin_rows_count<<<xcd_grid(plan.nch1), 256, lds_rows, s>>>(vt, n, rec, dvals, nvis, cap_vis, overflow, plan);
  E(K_BIN_COUNT);
  B(K_BIN_SCAN);
  scan_u32(plan.cnt1, n1, nullptr, plan.part, plan.words, s);
  E(K_BIN_SCAN);
  B(K_BIN_SCATTER);
  if (plan.rows <= 64)
    k_bin_rows_scatter_r<1><<<(plan.nch1 + 3) / 4, 256, 0, s>>>(vt, n, rec, dvals, nvis, cap_vis, overflow, plan);
  else if (plan.rows <= 128)
    k_bin_rows_scatter_r<2><<<(plan.nch1 + 3) / 4, 256, 0, s>>>(vt, n, rec, dvals, nvis, cap_vis, overflow, plan);
  else if (plan.rows <= 256)
    k_bin_rows_scatter_r<4><<<(plan.nch1 + 3) / 4, 256, 0, s>>>(vt, n, rec, dvals, nvis, cap_vis, overflow, plan);
  else
    k_bin_rows_scatter<<<plan.nch1, 64, lds_rows, s>>>(vt, n, rec, dvals, nvis, cap_vis, overflow, plan);
  E(K_BIN_SCATTER);
  B(K_BIN_COUNT);
  k_bin_tiles_count<<<g_count, 256, 4 * (lds_cols + 4), s>>>(vt, plan, rec, exact_k, tile, vt.max_tiles_x + 1);
  E(K_BIN_COUNT);
  B(K_BIN_SCAN);
  scan_u32(plan.cntF, plan.cap_flat, plan.words + 2, plan.part, plan.words + 3, s);
  E(K_BIN_SCAN);
  B(K_BIN_SCATTER);
  if (vt.max_tiles_x <= 64)
    k_bin_tiles_scatter_r<1><<<g_scatter4, 256, 0, s>>>(vt, plan, vals, overflow, ranges, hint, order);
  else if (vt.max_tiles_x <= 128)
    k_bin_tiles_scatter_r<2><<<g_scatter4, 256, 0, s>>>(vt, plan, vals, overflow, ranges, hint, order);
  else if (vt.max_tiles_x <= 256)
    k_bin_tiles_scatter_r<4><<<g_scatter4, 256, 0, s>>>(vt, plan, vals, overflow, ranges, hint, order);
  else
    k_bin_tiles_scatter<<<g_scatter, 64, lds_cols, s>>>(vt, plan, vals, overflow, ranges);
  E(K_BIN_SCATTER);
  if (!hint || vt.max_tiles_x > 256) {  // the order not taken by the placement above
    B(K_TILE_ORDER);
    k_tile_order<<<1, 1024, 0, s>>>(ranges, hint, vt.total_tiles, order);
    E(K_TILE_ORDER);
  }
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s) {
  if (count > 0) k_fill_u32<<<blocks_for(count, 256), 256, 0, s>>>(p, value, count);
  return hipGetLastError();
}

hipError_t launch_first_nonfinite(const GaussDev& g, int sh_degree, uint32_t* first, hipStream_t s) {
  k_fill_u32<<<1, 256, 0, s>>>(first, 0xFFFFFFFFu, 1);
  const int K = (sh_degree + 1) * (sh_degree + 1);
  if (g.n > 0) {
    const int64_t total = g.n * (14 + 3 * int64_t(K - 1));
    k_first_nonfinite<<<int(std::min<int64_t>(blocks_for(total, 256), 4096)), 256, 0, s>>>(g, K, first);
  }
  return hipGetLastError();
}

// Persistent grid: blocks resident at once, at most `cap_per_cu` per compute unit (the
// compositing kernels ran fastest below full occupancy: blend_fwd at 2 blocks per CU on
// one 640x480 view, where its heaviest tiles' single-wavefront chains bound it and then
// share a SIMD with fewer others, and at 4 with many tiles per CU (eight views);
// blend_bwd at 5 (one pixel per lane) and 8 (two pixels per lane, blocks of half the
// size), against more that fit).
template <auto KERN>
static int resident_blocks(int threads, int cap_per_cu) {
  static int per_cu = -1, cus = 1;  // one pair per kernel
  if (per_cu < 0) {
    int p = 0, c = 0, dev = 0;
    (void)hipGetDevice(&dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&p, KERN, threads, 0) != hipSuccess || p < 1) p = 1;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1) c = 1;
    (void)hipGetLastError();
    cus = c;
    per_cu = p;
  }
  return std::min(per_cu, cap_per_cu) * cus;
}

static int device_cus() {
  static int cus = -1;
  if (cus < 0) {
    int c = 0, dev = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1) c = 1;
    (void)hipGetLastError();
    cus = c;
  }
  return cus;
}
constexpr int kFwdBlocksPerCU = 2;        // up to kFwdManyTilesPerCU tiles per CU
constexpr int kFwdBlocksPerCUMany = 4;    // beyond
constexpr int kFwdManyTilesPerCU = 16;
constexpr int kBwdBlocksPerCU = 5;
constexpr int kBwd2BlocksPerCU = 8;
constexpr int kBwdPixelsPerLane = 2;

template <int TS, int BATCH>
static void blend_fwd_t(const ViewTable& vt, const Rules& ru, const Records& rec, const uint2* ranges,
                        const uint32_t* vals, float* T_final, uint32_t* n_contrib, const TileQueue& q,
                        const Ckpt& ck, hipStream_t s) {
  const int cap = vt.total_tiles > kFwdManyTilesPerCU * device_cus() ? kFwdBlocksPerCUMany : kFwdBlocksPerCU;
  const int grid = std::min(vt.total_tiles, resident_blocks<k_blend_fwd<TS, BATCH>>(TS * TS, cap));
  k_blend_fwd<TS, BATCH><<<grid, TS * TS, 0, s>>>(vt, ru, rec, ranges, vals, T_final, n_contrib, q, ck);
}

hipError_t launch_count_used(const ViewTable& vt, const Rules& ru, const Records& rec, const uint2* ranges,
                             const uint32_t* vals, const uint32_t* n_contrib, int tile, int64_t total_pix,
                             uint32_t* n_used, hipStream_t s) {
  if (total_pix == 0) return hipSuccess;
  k_count_used<<<unsigned((total_pix + 255) / 256), 256, 0, s>>>(vt, ru, rec, ranges, vals, n_contrib, tile, total_pix,
                                                                 n_used);
  return hipGetLastError();
}

// checkpoints every kCkptStride entries over the first 1024 list entries of each tile
int ckpt_stride(int) { return kCkptStride; }
int ckpt_per_tile(int batch) { return std::max(1, 1024 / ckpt_stride(batch)); }

int64_t bwd_items_cap(int total_tiles, int batch) { return int64_t(total_tiles) * (ckpt_per_tile(batch) + 1); }

hipError_t launch_blend_fwd(int tile, int batch, const ViewTable& vt, const Rules& ru, const Records& rec,
                            const uint2* ranges, const uint32_t* vals, float* T_final, uint32_t* n_contrib,
                            const TileQueue& q, const Ckpt& ck, hipStream_t s) {
  if (vt.total_tiles == 0) return hipSuccess;
  const bool b256 = batch == 256;
  switch (tile) {
    case 8: b256 ? blend_fwd_t<8, 256>(vt, ru, rec, ranges, vals, T_final, n_contrib, q, ck, s)
                 : blend_fwd_t<8, 128>(vt, ru, rec, ranges, vals, T_final, n_contrib, q, ck, s); break;
    case 32: b256 ? blend_fwd_t<32, 256>(vt, ru, rec, ranges, vals, T_final, n_contrib, q, ck, s)
                  : blend_fwd_t<32, 128>(vt, ru, rec, ranges, vals, T_final, n_contrib, q, ck, s); break;
    default: b256 ? blend_fwd_t<16, 256>(vt, ru, rec, ranges, vals, T_final, n_contrib, q, ck, s)
                  : blend_fwd_t<16, 128>(vt, ru, rec, ranges, vals, T_final, n_contrib, q, ck, s); break;
  }
  return hipGetLastError();
}

int loss_partials(const ViewTable& vt) {
  int64_t maxp = 0;
  for (int v = 0; v < vt.nviews; ++v) maxp = std::max<int64_t>(maxp, int64_t(vt.v[v].W) * vt.v[v].H);
  return int(blocks_for(maxp, 256)) * vt.nviews;
}

hipError_t launch_loss_l1(const ViewTable& vt, float depth_w, float* part, float* loss, hipStream_t s,
                          const uint32_t* order, int batch, const Ckpt* ck, uint32_t* ctrl) {
  const int np = loss_partials(vt);
  k_loss_l1<<<dim3(np / vt.nviews, vt.nviews), 256, 0, s>>>(vt, depth_w, part, order, vt.total_tiles,
                                                            ckpt_stride(batch), ck ? *ck : Ckpt{}, ctrl);
  if (loss) k_loss_sum<<<1, 256, 0, s>>>(part, np, loss);
  return hipGetLastError();
}

template <int TS, int BATCH>
static void blend_bwd_t(const ViewTable& vt, const Rules& ru, const Records& rec, const uint2* ranges,
                        const uint32_t* vals, const float* T_final, const uint32_t* n_contrib, float* grad2d,
                        const TileQueue& q, const Ckpt& ck, hipStream_t s) {
  constexpr int PPL = TS >= 16 ? kBwdPixelsPerLane : 1;
  constexpr int cap = TS >= 16 ? kBwd2BlocksPerCU : kBwdBlocksPerCU;
  const int grid =
      int(std::min<int64_t>(ck.cap_items, resident_blocks<k_blend_bwd2<TS, BATCH, PPL>>(TS * TS / PPL, cap)));
  k_blend_bwd2<TS, BATCH, PPL><<<grid, TS * TS / PPL, 0, s>>>(vt, ru, rec, ranges, vals, T_final, n_contrib, grad2d,
                                                              q, ck);
}

hipError_t launch_blend_bwd(int tile, int batch, const ViewTable& vt, const Rules& ru, const Records& rec,
                            const uint2* ranges, const uint32_t* vals, const float* T_final,
                            const uint32_t* n_contrib, float* grad2d, const TileQueue& q, const Ckpt& ck,
                            hipStream_t s, bool items_listed) {
  if (vt.total_tiles == 0) return hipSuccess;
  if (!items_listed) k_bwd_items<<<1, 1024, 0, s>>>(q.order, vt.total_tiles, ckpt_stride(batch), ck, q.ctrl);
  const bool b256 = batch == 256;
  switch (tile) {
    case 8: b256 ? blend_bwd_t<8, 256>(vt, ru, rec, ranges, vals, T_final, n_contrib, grad2d, q, ck, s)
                 : blend_bwd_t<8, 128>(vt, ru, rec, ranges, vals, T_final, n_contrib, grad2d, q, ck, s); break;
    case 32: b256 ? blend_bwd_t<32, 256>(vt, ru, rec, ranges, vals, T_final, n_contrib, grad2d, q, ck, s)
                  : blend_bwd_t<32, 128>(vt, ru, rec, ranges, vals, T_final, n_contrib, grad2d, q, ck, s); break;
    default: b256 ? blend_bwd_t<16, 256>(vt, ru, rec, ranges, vals, T_final, n_contrib, grad2d, q, ck, s)
                  : blend_bwd_t<16, 128>(vt, ru, rec, ranges, vals, T_final, n_contrib, grad2d, q, ck, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_project_bwd(int deg, const GaussDev& g, const ViewTable& vt, const Rules& ru,
                              const Records& rec, const float* grad2d, float* dp_sh, const GradOut& out,
                              const AdamDev& adam, hipStream_t s, const float* loss_part, int loss_np,
                              float* loss) {
  if (g.n == 0) return hipSuccess;
  const dim3 gsh(blocks_for(g.n, kShGaussians));
  switch (deg) {
    case 0: k_project_bwd_sh<0><<<gsh, 256, 0, s>>>(g, vt, rec, grad2d, out, dp_sh, adam); break;
    case 1: k_project_bwd_sh<1><<<gsh, 256, 0, s>>>(g, vt, rec, grad2d, out, dp_sh, adam); break;
    case 2: k_project_bwd_sh<2><<<gsh, 256, 0, s>>>(g, vt, rec, grad2d, out, dp_sh, adam); break;
    default: k_project_bwd_sh<3><<<gsh, 256, 0, s>>>(g, vt, rec, grad2d, out, dp_sh, adam); break;
  }
  k_project_bwd_geo<<<blocks_for(g.n, kProjThreads), kProjThreads, 0, s>>>(g, vt, ru, rec, grad2d, dp_sh, out,
                                                                           adam, loss_part, loss_np, loss);
  return hipGetLastError();
}

}  // namespace gsr
