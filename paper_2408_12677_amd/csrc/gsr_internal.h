// Internal declarations shared by the host orchestration and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "gsr.h"
#include "gsr_adam.h"
#include "gsr_tsdf.h"

namespace gsr {

// Kernel ids of the optional per-launch event timer (order matches gsr_kernel_name).
enum KernelId {
  K_PROJECT = 0,
  K_SCAN,
  K_COMPACT,
  K_RADIX_HIST,
  K_RADIX_ROWSCAN,
  K_RADIX_SCATTER,
  K_BIN_COUNT,
  K_BIN_SCAN,
  K_BIN_SCATTER,
  K_TILE_ORDER,
  K_FILL,
  K_BLEND_FWD,
  K_LOSS,
  K_BLEND_BWD,
  K_PROJECT_BWD,
  K_ADAM,
  K_TSDF_ALLOC,
  K_TSDF_FUSE,
  K_COUNT
};

// Records a HIP event pair around each launch when enabled; durations are collected
// (after a synchronisation) by Timer::collect.
struct Timer {
  bool on = false;
  hipStream_t stream = nullptr;
  struct Rec {
    int k;
    hipEvent_t a, b;
  };
  std::vector<hipEvent_t> free_events;
  std::vector<Rec> pending;
  hipEvent_t open[K_COUNT] = {};
  double ms[K_COUNT] = {};
  long long launches[K_COUNT] = {};

  hipEvent_t take() {
    hipEvent_t e = nullptr;
    if (!free_events.empty()) {
      e = free_events.back();
      free_events.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }
  void begin(int k) {
    if (!on) return;
    open[k] = take();
    if (open[k]) (void)hipEventRecord(open[k], stream);
  }
  void end(int k) {
    if (!on || !open[k]) return;
    hipEvent_t b = take();
    if (!b) return;
    (void)hipEventRecord(b, stream);
    pending.push_back(Rec{k, open[k], b});
    open[k] = nullptr;
  }
  void collect() {
    for (const Rec& r : pending) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
        ms[r.k] += t;
        launches[r.k] += 1;
      }
      free_events.push_back(r.a);
      free_events.push_back(r.b);
    }
    pending.clear();
  }
  void reset() {
    for (int i = 0; i < K_COUNT; ++i) {
      ms[i] = 0.0;
      launches[i] = 0;
    }
  }
  void destroy() {
    collect();
    for (hipEvent_t e : free_events) (void)hipEventDestroy(e);
    free_events.clear();
  }
};

constexpr int kProjThreads = 256;  // Gaussians per block in the per-Gaussian kernels
constexpr int kSortThreads = 256;
constexpr int kSortItems = 4;
constexpr int kSortTile = kSortThreads * kSortItems;  // keys per radix-sort block
constexpr int kGrad2D = 12;  // floats per (view, Gaussian) 2D-gradient record (10 used)
constexpr int kHeadFwd = 0;    // control words (see TileQueue)
constexpr int kHeadBwd = 1;
constexpr int kOverflow = 2;
constexpr int kItems = 3;      // backward work items listed
constexpr int kStepWords = 4;  // words 0..3 start at zero in every step (cleared by the projection)
// set together with kOverflow and never cleared by a step: a captured graph zeroes it once
// at creation, so it records an overflow of any launch since, and the fused optimiser
// step reads it to leave the parameters alone once one happened
constexpr int kOverflowSticky = 4;
constexpr int kCtrlWords = 8;
constexpr int kScanTile = 4096;  // elements per block of the device-wide scans
constexpr int64_t kMaxBinCounts = int64_t(1) << 22;  // entries of each binning count array (soft)

// One camera plus where its tiles and pixels live in the concatenated spaces.
struct ViewDev {
  float R[9];
  float t[3];
  float fx, fy, cx, cy, znear;
  float cam_pos[3];  // camera centre in world coordinates
  int32_t W, H, tiles_x, tiles_y;
  int32_t tile_off;  // first global tile id of this view
  int32_t row_off;   // first global tile row of this view
  int64_t pix_off;   // first pixel of this view in the per-pixel state arrays
  float* color;      // forward outputs
  float* depth;
  float* alpha;
  const float* g_color;  // backward inputs (dL/d outputs)
  const float* g_depth;
  const float* g_alpha;
  const float* t_color;  // loss targets
  const float* t_depth;
  float* lg_color;       // loss gradient outputs
  float* lg_depth;
};

struct ViewTable {
  ViewDev v[GSR_MAX_VIEWS];
  int32_t nviews;
  int32_t total_tiles;
  int32_t total_rows;  // tile rows over all views
  int32_t max_tiles_x;
};

struct Rules {
  float k, lowpass, amin, amax, Tmin, guard;
  float jclamp;  // > 0: x/z, y/z clamped inside J to +-jclamp half fields of view
  float bg[3];
  int32_t norm_depth;  // depth output D / (1 - T_final) (GSR_NORMALIZED_DEPTH)
};

struct GaussDev {
  const float* means;
  const float* scales;
  const float* quats;
  const float* opac;
  const float* sh;
  int64_t n;
};

// Per-(view, Gaussian) splat records written by the projection kernel.
struct Records {
  float4* r0;       // (mu_x, mu_y, conic A, conic B)
  float4* r1;       // (conic C, opacity, depth, unused)
  float4* rgb;      // (r, g, b, unused)
  uint2* rect;      // (tx0 | tx1 << 16, ty0 | ty1 << 16)
  uint32_t* counts; // tiles touched, 0 when culled
  uint32_t* runs;   // exact tiles only (else null): [kRowRuns] column runs of the first tile rows
};
// Column runs lo | hi << 16 (tile columns, below kRunUncut): the projection keeps the
// exact runs of a record's first kRowRuns tile rows; an empty run is kRunEmpty (lo > hi);
// kRunUncut marks a rectangle run that the binning still has to cut.
constexpr int kRowRuns = 8;
constexpr uint32_t kRunEmpty = 0x7FFFu;
constexpr uint32_t kRunUncut = 0x8000u;

// Heaviest-first tile order (k_tile_order) and the control words of the persistent
// compositing kernels: kHeadFwd / kHeadBwd queue heads, kOverflow the capacity-overflow
// flag, kItems the number of backward work items.
struct TileQueue {
  const uint32_t* order;
  uint32_t* ctrl;
  int32_t by_work;  // the order comes from measured per-tile work: queue position sets priority
};

// What the forward keeps so that the backward can run a tile's list in independent
// pieces of one checkpoint stride (64 entries) each: at the first `kmax` such boundaries
// the forward passes, per pixel, the transmittance in front of it and the colour and
// depth accumulated up to it (a "checkpoint"); per pixel the accumulated totals; per tile
// its longest contributor list.  The backward's work items are (tile, stride) pairs;
// entries past the last checkpoint of a tile form one item that walks them all.
struct Ckpt {
  float* state;         // [tiles][kmax][5][pixels of a tile]: T, colour (3), depth in front
  float4* acc;          // [pixels] colour (3) and depth accumulated, without background
  uint32_t* tile_nmax;  // [tiles] longest contributor list of the tile
  uint2* items;         // [cap_items] backward work items (tile, first batch)
  int32_t kmax;         // checkpoints per tile
  int64_t cap_items;
};

// Two-level stable binning of the depth-sorted records into per-tile lists.
//   rows:  the records are cut into chunks of 64 * rounds1; per (tile row, chunk) counts,
//          scanned row-major, place every (record, row) entry of a chunk after those of
//          earlier chunks, giving each tile row a depth-ordered list of (record, tx0..tx1)
//   tiles: each row list is cut into segments of 64 * rounds2 entries; per (tile, segment)
//          counts, flattened tile-major (row, column, segment) and scanned, place every
//          (record, tile) pair; the scan is in global tile order, so it also gives the ranges
struct BinPlan {
  int32_t rows;      // tile rows over all views
  int32_t nch1;      // chunks of the depth-sorted records
  int32_t rounds1;   // 64-record rounds per chunk
  int32_t rounds2;   // 64-entry rounds per segment
  int64_t cap_M;     // capacity of row entries and of pairs
  int64_t cap_seg;   // capacity of segments
  int64_t cap_flat;  // capacity of flat (tile, segment) counts
  uint32_t* cnt1;        // [rows][nch1] counts, then exclusive offsets
  uint2* rowlist;        // (record id, tx0 | tx1 << 16) per (record, row) entry
  uint4* rowinfo;        // per row: (list start, list length, first segment, first flat index)
  uint32_t* seg_start;   // [rows + 1] first segment of each row
  uint32_t* cntF;        // flat (tile, segment) counts, then exclusive offsets
  uint32_t* part;        // partial sums of the device-wide scans
  unsigned long long* words;  // [0] row entries, [1] segments, [2] flat size, [3] pairs placed
};

struct GradOut {
  float* means;
  float* scales;
  float* quats;
  float* opac;
  float* sh;
  int accumulate;
};

// Quadtree seeding (gsr_seed.hip): one RGB-D frame and its camera.
struct SeedImage {
  const float* rgb;    // [3,H,W]
  const float* depth;  // [H,W]
  int32_t W, H;
  double fx, fy, cx, cy;
  float R[9], t[3];    // world -> camera
};

struct SeedRules {
  int32_t measure;  // GSR_SEED_CONTRAST or GSR_SEED_DEPTH_VARIANCE
  float threshold;
  int32_t min_side;
  float opacity;
  int32_t sh_degree;
  int32_t check;    // nonzero: keep a leaf only where the map's voxel at its mean has weight 1
  TsdfDev map;
};

struct SeedOut {
  float* means;
  float* scales;
  float* quats;
  float* opac;
  float* sh;
  int32_t* leaves;
  int64_t capacity;
};

int seed_roots(int W, int H);  // 64-pixel root cells of a W x H image
// per-root Gaussian counts into root_counts[seed_roots]
hipError_t launch_seed_count(const SeedImage& im, const SeedRules& r, uint32_t* root_counts, hipStream_t s);
// writes the Gaussians at the exclusive-scanned root offsets
hipError_t launch_seed_emit(const SeedImage& im, const SeedRules& r, const uint32_t* root_offsets,
                            const SeedOut& out, hipStream_t s);

// ---- launchers (gsr_kernels.hip) --------------------------------------------------
// In-place exclusive scan of a[0, count) by one block (count up to a few 10^4); the total
// goes to *total.
hipError_t launch_scan_small(uint32_t* a, int count, unsigned long long* total, hipStream_t s);
// Device-side counts (unsigned long long) are clamped by each kernel to the capacity its
// grid and buffers were sized for.
// zero_rows (may be null): 2D-gradient rows (kGrad2D floats) zeroed for every visible record;
// the first block also zeroes the first clear_words control words `ctrl`
// rec.runs (exact tiles) gets each record's first kRowRuns exact row runs for extent exact_k
hipError_t launch_project(int deg, const GaussDev& g, const ViewTable& vt, const Rules& ru, int tile,
                          const Records& rec, uint2* blocksums, int nblk, float* zero_rows, uint32_t* ctrl,
                          int clear_words, float exact_k, hipStream_t s);
hipError_t launch_scan_pairs(uint2* blocksums, int count, unsigned long long* totals, hipStream_t s);
// raw: blocksums as the projection wrote them (not scanned; at most kCompactRawMax of
// them), and the compaction writes totals[0..1] itself; else scanned by launch_scan_pairs,
// which wrote the totals.
constexpr int64_t kCompactRawMax = 4096;
hipError_t launch_compact(int64_t n, int views, const Records& rec, const uint2* blocksums, int nblk,
                          unsigned long long* totals, int64_t cap_M, uint32_t* dkeys, uint32_t* dvals,
                          int64_t cap, uint32_t* overflow, bool raw, hipStream_t s);
// Checkpoint stride and checkpoints per tile, and the backward work items of all tiles,
// at a batch size.
int ckpt_stride(int batch);
int ckpt_per_tile(int batch);
int64_t bwd_items_cap(int total_tiles, int batch);
// Stable LSD radix sort of min(*count, cap) (key, value) pairs by their key_bits low bits
// (at most 32; 8-bit passes); the result is in the _alt arrays when *result_in_alt.  hist
// holds radix_hist_words(cap) words, digit_tot 256.
int radix_hist_words(int64_t cap);
hipError_t launch_radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                             uint32_t* hist, uint32_t* digit_tot, const unsigned long long* count, int64_t cap,
                             const uint32_t* overflow, int key_bits, bool* result_in_alt, int* passes, hipStream_t s,
                             Timer* tm);
// Sizes of a binning plan for capacities (cap_vis, cap_M); pointers are left null.
BinPlan bin_plan(const ViewTable& vt, int64_t cap_vis, int64_t cap_M);
// exact_k > 0: per tile row only the columns the ellipse d^T Q d <= exact_k^2 reaches.
// Uses the control words' overflow word.  Also writes the tile queue's order by
// decreasing expected work: hint[t] (a previous forward's longest contributor count of
// tile t) when given, else the list length.
hipError_t launch_bin(const ViewTable& vt, int64_t n, const Records& rec, const uint32_t* dvals,
                      const unsigned long long* nvis, int64_t cap_vis, const BinPlan& plan, uint32_t* vals,
                      uint2* ranges, uint32_t* ctrl, float exact_k, int tile, const uint32_t* hint,
                      uint32_t* order, hipStream_t s, Timer* tm);
hipError_t launch_blend_fwd(int tile, int batch, const ViewTable& vt, const Rules& ru, const Records& rec,
                            const uint2* ranges, const uint32_t* vals, float* T_final, uint32_t* n_contrib,
                            const TileQueue& q, const Ckpt& ck, hipStream_t s);
// Per pixel, the entries before its last contributor that passed the skip rule.
hipError_t launch_count_used(const ViewTable& vt, const Rules& ru, const Records& rec, const uint2* ranges,
                             const uint32_t* vals, const uint32_t* n_contrib, int tile, int64_t total_pix,
                             uint32_t* n_used, hipStream_t s);
int loss_partials(const ViewTable& vt);  // block partial sums launch_loss_l1 writes
// Loss partial sums, and their total into *loss unless loss is null (then the caller has
// launch_project_bwd add them up).  With order non-null (the forward's tile queue) the
// loss kernel also lists the backward's work items for a batch size (the state ck, the
// control words ctrl), so that launch_blend_bwd can skip its own listing.
hipError_t launch_loss_l1(const ViewTable& vt, float depth_w, float* part, float* loss, hipStream_t s,
                          const uint32_t* order = nullptr, int batch = 0, const Ckpt* ck = nullptr,
                          uint32_t* ctrl = nullptr);
// Lists the backward's (tile, stride) work items unless items_listed (the loss kernel
// did), then runs them.
hipError_t launch_blend_bwd(int tile, int batch, const ViewTable& vt, const Rules& ru, const Records& rec,
                            const uint2* ranges, const uint32_t* vals, const float* T_final,
                            const uint32_t* n_contrib, float* grad2d, const TileQueue& q, const Ckpt& ck,
                            hipStream_t s, bool items_listed = false);
// grad2d holds V*N rows of kGrad2D floats; dp_sh is scratch for N * 3 floats.  With
// adam.on the parameter gradients are not written to `out` but applied to the parameters
// by one Adam step (adam.bc must already hold the step's bias corrections).
// With loss non-null the first block of the geometric kernel also writes the total of the
// loss_np loss partial sums loss_part to *loss (in launch_loss_l1's order).
hipError_t launch_project_bwd(int deg, const GaussDev& g, const ViewTable& vt, const Rules& ru,
                              const Records& rec, const float* grad2d, float* dp_sh, const GradOut& out,
                              const AdamDev& adam, hipStream_t s, const float* loss_part = nullptr,
                              int loss_np = 0, float* loss = nullptr);

// ---- TSDF fusion (gsr_tsdf.hip) -----------------------------------------------------
int tsdf_band_samples(float eps, float step);
// Band allocation of one depth frame [H, W] (blocks stamped with the frame) and pool assignment.
hipError_t launch_tsdf_alloc(const float* depth, const TsdfCam& cam, const TsdfDev& m, const TsdfRules& ru,
                             uint32_t frame, hipStream_t s);
// Eq. 6-9 for every voxel of the blocks the frame met.
hipError_t launch_tsdf_fuse(const float* depth, const TsdfCam& cam, const TsdfDev& m, const TsdfRules& ru,
                            uint32_t frame, hipStream_t s);
// out[i] = weight of the voxel holding pts[i] (0 where unallocated).
hipError_t launch_tsdf_weights(const TsdfDev& m, const float* pts, int64_t n, float* out, hipStream_t s);

// ---- optimiser (gsr_optim.hip) ------------------------------------------------------
// Advances the step counter state[0] and writes the new step's bias corrections to
// state[1], state[2] (as binary32); does nothing when skip is non-null and *skip != 0.
hipError_t launch_adam_tick(uint32_t* state, float b1, float b2, const uint32_t* skip, hipStream_t s);
// One Adam step over all groups of n Gaussians of SH degree deg, gradients grads[group].
hipError_t launch_adam(const AdamDev& a, const float* const grads[G_COUNT], int64_t n, int deg, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s);
// first[0] = the smallest index of a Gaussian with a NaN or infinite parameter, else UINT32_MAX.
hipError_t launch_first_nonfinite(const GaussDev& g, int sh_degree, uint32_t* first, hipStream_t s);

}  // namespace gsr
