// Host side of the C ABI declared in gsr.h: argument validation, scratch memory from the
// device's stream-ordered pool, the launch sequence of one optimisation step (forward,
// loss, backward), its capture into a hipGraph, and the launch-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "gsr_internal.h"
#include "gsr_validate.h"

using namespace gsr;

struct gsr_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  gsr_alloc alloc{};  // the caller's allocator; alloc.alloc == nullptr: the stream-ordered pool
  std::string err;
  unsigned long long* h_total = nullptr;  // pinned read-back slots: pair count M, visible records
  Timer timer;
  void* bwd_scratch = nullptr;  // the eager backward's 2D-gradient rows, kept between calls (grow-only)
  size_t bwd_scratch_bytes = 0;
  void* noalloc_scratch = nullptr;  // this device's address of the fixed array `scratch`
  // Per tile grid (tile size and view sizes), the last eager forward's longest
  // contributor count of every tile: the next forward over the same tiles orders its tile
  // queue by it.  Scheduling only; results do not depend on it.
  struct WorkHint {
    std::vector<int> grid;
    uint32_t* tiles = nullptr;
    int64_t count = 0;
  };
  std::vector<WorkHint> hints;
  size_t next_hint = 0;  // the entry replaced next once kMaxHints are held
};
constexpr size_t kMaxHints = 8;

// All device state of one step.  Eager forwards size the sort buffers exactly and drop
// the temporaries afterwards; a graph keeps every buffer at its capacity.
struct gsr_saved {
  gsr_ctx* ctx = nullptr;
  int V = 0;
  int64_t N = 0;
  int deg = 0;
  GaussDev g{};
  gsr_settings s{};
  Rules ru{};
  ViewTable vt{};
  Records rec{};
  int nblk = 0;
  uint2* blocksums = nullptr;
  unsigned long long* d_total = nullptr;  // [0] pairs M, [1] visible records, [2] pairs written
  int64_t M = 0, n_vis = 0;               // measured sizes (eager) or sizes at creation (graph)
  int64_t cap_M = 0, cap_vis = 0;         // buffer capacities
  // depth sort and binning buffers
  uint32_t *dk = nullptr, *dv = nullptr, *dk2 = nullptr, *dv2 = nullptr;
  uint32_t *hist = nullptr, *dtot = nullptr;
  const uint32_t* order_hint = nullptr;  // per-tile work of a previous forward, or null
  BinPlan plan{};
  Ckpt ck{};                  // forward checkpoints and backward work items
  uint32_t* vals = nullptr;   // record id of every (tile, record) pair, in key order
  uint2* ranges = nullptr;
  uint32_t* order = nullptr;
  float* loss_part = nullptr;  // block partial sums of the loss
  uint32_t* ctrl = nullptr;
  float* T_final = nullptr;
  uint32_t* n_contrib = nullptr;
  float* grad2d = nullptr;  // graph only (eager backward allocates its own)
  int64_t total_pix = 0;
  int sort_passes = 0;
  bool graph = false;  // a captured step: the sticky overflow word survives its steps
  std::vector<void*> blocks;  // persistent allocations, released on free
  std::vector<void*> temps;   // eager-forward temporaries
};

struct gsr_graph {
  gsr_ctx* ctx = nullptr;
  gsr_saved* sv = nullptr;
  hipStream_t capture = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  uint32_t* h_flag = nullptr;  // pinned copy of the overflow word, written by the graph
  bool launched = false;
  bool overflowed = false;
};

struct gsr_tsdf {
  gsr_ctx* ctx = nullptr;
  gsr_tsdf_settings s{};
  TsdfDev dev{};
  TsdfRules ru{};
  uint32_t frame = 0;
  std::vector<void*> blocks;
};

// The fixed device array of gsr_backward_noalloc: the per-record 2D-gradient rows and the
// colour term's mean gradient of one backward.  Every GPU the library runs on holds its own
// copy until the process ends.  Host code never passes `scratch` itself to a kernel (on the
// host it names a stand-in, not device memory): it uses the device address that
// noalloc_scratch_address() looks up once per device.
static __device__ __align__(256) float scratch[GSR_NOALLOC_SCRATCH_BYTES / sizeof(float)];

namespace {

const char* const kKernelNames[K_COUNT] = {"project",    "scan",          "compact",       "radix_hist",
                                           "radix_rowscan", "radix_scatter", "bin_count",   "bin_scan",
                                           "bin_scatter", "tile_order",    "fill",
                                           "blend_fwd",  "loss_l1",       "blend_bwd",     "project_bwd",
                                           "adam",       "tsdf_alloc",    "tsdf_fuse"};

thread_local std::string g_noctx_err;

gsr_status fail(gsr_ctx* ctx, gsr_status st, const std::string& msg) {
  if (ctx)
    ctx->err = msg;
  else
    g_noctx_err = msg;
  return st;
}

#define GSR_HIP(ctx, expr)                                                                              \
  do {                                                                                                  \
    hipError_t e_ = (expr);                                                                             \
    if (e_ != hipSuccess) return fail(ctx, GSR_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

// Wraps one launch (or launch sequence) in the context's optional event timer.
template <class F>
hipError_t timed(gsr_ctx* ctx, hipStream_t s, int k, F&& f) {
  ctx->timer.stream = s;
  ctx->timer.begin(k);
  hipError_t e = f();
  ctx->timer.end(k);
  return e;
}

// Device memory of the library: from the caller's allocator when the context has one,
// else from the device's stream-ordered pool; released the same way, stream-ordered.
gsr_status dev_alloc(gsr_ctx* ctx, hipStream_t s, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return GSR_OK;
  if (ctx->alloc.alloc) {
    *p = ctx->alloc.alloc(ctx->alloc.user, bytes, s);
    if (!*p) return fail(ctx, GSR_ENOMEM, "the caller's allocator returned no memory for " + std::to_string(bytes) +
                                              " bytes");
    return GSR_OK;
  }
  hipError_t e = hipMallocAsync(p, bytes, s);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(ctx, GSR_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed: " +
                                     hipGetErrorString(e));
  }
  return GSR_OK;
}

void dev_free(gsr_ctx* ctx, void* p, hipStream_t s) {
  if (!p) return;
  if (ctx->alloc.free)
    ctx->alloc.free(ctx->alloc.user, p, s);
  else
    (void)hipFreeAsync(p, s);
}

template <class T>
gsr_status alloc_in(gsr_saved* sv, std::vector<void*>& list, T** p, size_t count) {
  void* q = nullptr;
  gsr_status st = dev_alloc(sv->ctx, sv->ctx->stream, &q, count * sizeof(T));
  if (st != GSR_OK) return st;
  if (q) list.push_back(q);
  *p = static_cast<T*>(q);
  return GSR_OK;
}

void free_list(gsr_saved* sv, std::vector<void*>& list) {
  for (void* p : list) dev_free(sv->ctx, p, sv->ctx->stream);
  list.clear();
}

void release(gsr_saved* sv) {
  if (!sv) return;
  free_list(sv, sv->temps);
  free_list(sv, sv->blocks);
  delete sv;
}

// Host-side argument checks (gsr_validate.cpp), reported through the context.
gsr_status checked(gsr_ctx* ctx, gsr_status st, const std::string& err) { return st == GSR_OK ? st : fail(ctx, st, err); }

gsr_status check_settings(gsr_ctx* ctx, const gsr_settings* s) {
  std::string err;
  return checked(ctx, check::settings(s, err), err);
}

gsr_status check_camera(gsr_ctx* ctx, const gsr_camera& c, int v) {
  std::string err;
  return checked(ctx, check::camera(c, v, err), err);
}

gsr_status check_forward_args(gsr_ctx* ctx, const gsr_gaussians* g, const gsr_camera* cams, int32_t V,
                              const gsr_settings* s, const gsr_view_out* outs) {
  std::string err;
  return checked(ctx, check::forward_args(g, cams, V, s, outs, err), err);
}

int bits_for(uint64_t maxval) {
  int b = 0;
  while (b < 64 && (maxval >> b) != 0) ++b;
  return b;
}

// A saved state with its view table and per-(view, Gaussian) buffers.
gsr_status make_saved(gsr_ctx* ctx, const gsr_gaussians* g, const gsr_camera* cams, int32_t V,
                      const gsr_settings* s, const gsr_view_out* outs, gsr_saved** out) {
  gsr_saved* sv = new gsr_saved;
  sv->ctx = ctx;
  sv->V = V;
  sv->N = g->n;
  sv->deg = g->sh_degree;
  sv->s = *s;
  sv->g = GaussDev{g->means, g->scales, g->quats, g->opacities, g->sh, g->n};
  sv->ru = Rules{s->extent_k, s->lowpass, s->alpha_min, s->alpha_max, s->T_min, s->guard, s->jclamp,
                 {s->bg[0], s->bg[1], s->bg[2]}, (s->flags & GSR_NORMALIZED_DEPTH) ? 1 : 0};
  ViewTable& vt = sv->vt;
  std::memset(&vt, 0, sizeof(vt));
  vt.nviews = V;
  int64_t tiles = 0, pix = 0, rows = 0;
  for (int v = 0; v < V; ++v) {
    const gsr_camera& c = cams[v];
    ViewDev& d = vt.v[v];
    std::memcpy(d.R, c.R, sizeof d.R);
    std::memcpy(d.t, c.t, sizeof d.t);
    d.fx = c.fx;
    d.fy = c.fy;
    d.cx = c.cx;
    d.cy = c.cy;
    d.znear = c.znear;
    for (int i = 0; i < 3; ++i)  // camera centre -R^T t
      d.cam_pos[i] = float(-(double(c.R[0 * 3 + i]) * c.t[0] + double(c.R[1 * 3 + i]) * c.t[1] +
                             double(c.R[2 * 3 + i]) * c.t[2]));
    d.W = c.width;
    d.H = c.height;
    d.tiles_x = (c.width + s->tile - 1) / s->tile;
    d.tiles_y = (c.height + s->tile - 1) / s->tile;
    d.tile_off = int32_t(tiles);
    d.row_off = int32_t(rows);
    d.pix_off = pix;
    d.color = outs[v].color;
    d.depth = outs[v].depth;
    d.alpha = outs[v].alpha;
    tiles += int64_t(d.tiles_x) * d.tiles_y;
    rows += d.tiles_y;
    vt.max_tiles_x = std::max(vt.max_tiles_x, d.tiles_x);
    pix += int64_t(c.width) * c.height;
  }
  vt.total_tiles = int32_t(tiles);
  vt.total_rows = int32_t(rows);
  sv->ck.kmax = ckpt_per_tile(s->batch);
  sv->ck.cap_items = bwd_items_cap(vt.total_tiles, s->batch);
  sv->total_pix = pix;
  const int64_t VN = int64_t(V) * g->n;
  sv->nblk = int((g->n + kProjThreads - 1) / kProjThreads);
  std::vector<void*>& B = sv->blocks;
  gsr_status st = GSR_OK;
  if ((st = alloc_in(sv, B, &sv->rec.r0, VN)) != GSR_OK || (st = alloc_in(sv, B, &sv->rec.r1, VN)) != GSR_OK ||
      (st = alloc_in(sv, B, &sv->rec.rgb, VN)) != GSR_OK || (st = alloc_in(sv, B, &sv->rec.rect, VN)) != GSR_OK ||
      (st = alloc_in(sv, B, &sv->rec.counts, VN)) != GSR_OK ||
      ((s->flags & GSR_EXACT_TILES) && (st = alloc_in(sv, B, &sv->rec.runs, size_t(VN) * kRowRuns)) != GSR_OK) ||
      (st = alloc_in(sv, B, &sv->blocksums, size_t(V) * sv->nblk + 1)) != GSR_OK ||
      (st = alloc_in(sv, B, &sv->d_total, 4)) != GSR_OK || (st = alloc_in(sv, B, &sv->ranges, size_t(tiles))) != GSR_OK ||
      (st = alloc_in(sv, B, &sv->order, size_t(tiles))) != GSR_OK ||
      (st = alloc_in(sv, B, &sv->loss_part, size_t(loss_partials(vt)))) != GSR_OK ||
      (st = alloc_in(sv, B, &sv->ck.tile_nmax, size_t(tiles))) != GSR_OK ||
      (st = alloc_in(sv, B, &sv->ck.acc, size_t(pix))) != GSR_OK ||
      (st = alloc_in(sv, B, &sv->ck.state, size_t(tiles) * sv->ck.kmax * 5 * s->tile * s->tile)) != GSR_OK ||
      (st = alloc_in(sv, B, &sv->ck.items, size_t(sv->ck.cap_items))) != GSR_OK ||
      (st = alloc_in(sv, B, &sv->ctrl, kCtrlWords)) != GSR_OK ||
      (st = alloc_in(sv, B, &sv->T_final, size_t(pix))) != GSR_OK ||
      (st = alloc_in(sv, B, &sv->n_contrib, size_t(pix))) != GSR_OK) {
    release(sv);
    return st;
  }
  *out = sv;
  return GSR_OK;
}

// Depth-sort and binning buffers for capacities (cap_vis, cap_M).  The pair list is kept
// with the saved state; eager forwards put everything else in `temps`.
gsr_status alloc_sort(gsr_saved* sv, int64_t cap_vis, int64_t cap_M, bool persistent) {
  sv->cap_vis = cap_vis;
  sv->cap_M = cap_M;
  std::vector<void*>& T = persistent ? sv->blocks : sv->temps;
  BinPlan& p = sv->plan;
  p = bin_plan(sv->vt, cap_vis, cap_M);
  const int64_t n1 = int64_t(p.rows) * p.nch1;
  const int64_t nparts = (std::max(n1, p.cap_flat) + kScanTile - 1) / kScanTile;
  gsr_status st = GSR_OK;
  if ((st = alloc_in(sv, T, &sv->dk, cap_vis)) != GSR_OK || (st = alloc_in(sv, T, &sv->dv, cap_vis)) != GSR_OK ||
      (st = alloc_in(sv, T, &sv->dk2, cap_vis)) != GSR_OK || (st = alloc_in(sv, T, &sv->dv2, cap_vis)) != GSR_OK ||
      (st = alloc_in(sv, T, &sv->hist, size_t(radix_hist_words(cap_vis)))) != GSR_OK ||
      (st = alloc_in(sv, T, &sv->dtot, 256)) != GSR_OK ||
      (st = alloc_in(sv, sv->blocks, &sv->vals, cap_M)) != GSR_OK ||
      (st = alloc_in(sv, T, &p.cnt1, size_t(n1))) != GSR_OK || (st = alloc_in(sv, T, &p.rowlist, cap_M)) != GSR_OK ||
      (st = alloc_in(sv, T, &p.rowinfo, size_t(p.rows))) != GSR_OK ||
      (st = alloc_in(sv, T, &p.seg_start, size_t(p.rows) + 1)) != GSR_OK ||
      (st = alloc_in(sv, T, &p.cntF, size_t(p.cap_flat))) != GSR_OK ||
      (st = alloc_in(sv, T, &p.part, size_t(nparts))) != GSR_OK || (st = alloc_in(sv, T, &p.words, 4)) != GSR_OK)
    return st;
  return GSR_OK;
}

TileQueue queue_of(const gsr_saved* sv) { return TileQueue{sv->order, sv->ctrl, sv->order_hint ? 1 : 0}; }

// The tile grid of a forward: tile size and every view's size.
std::vector<int> tile_grid(const gsr_saved* sv) {
  std::vector<int> g{sv->s.tile, sv->V};
  for (int v = 0; v < sv->V; ++v) {
    g.push_back(sv->vt.v[v].W);
    g.push_back(sv->vt.v[v].H);
  }
  return g;
}

// The context's work hint for this forward's tile grid, or null.
const uint32_t* find_hint(gsr_ctx* ctx, const gsr_saved* sv) {
  const std::vector<int> g = tile_grid(sv);
  for (auto& h : ctx->hints)
    if (h.grid == g && h.count == sv->vt.total_tiles) return h.tiles;
  return nullptr;
}

// Keeps this forward's per-tile work (enqueued after its compositing) as the hint for the
// next forward over the same tiles.  Failure to keep it only loses the hint.
void keep_hint(gsr_ctx* ctx, const gsr_saved* sv, hipStream_t s) {
  const int64_t T = sv->vt.total_tiles;
  if (T == 0) return;
  const std::vector<int> g = tile_grid(sv);
  gsr_ctx::WorkHint* slot = nullptr;
  for (auto& h : ctx->hints)
    if (h.grid == g) slot = &h;
  if (!slot) {
    if (ctx->hints.size() < kMaxHints) {
      ctx->hints.emplace_back();
      slot = &ctx->hints.back();
    } else {
      slot = &ctx->hints[ctx->next_hint];
      ctx->next_hint = (ctx->next_hint + 1) % kMaxHints;
    }
    slot->grid = g;
  }
  if (slot->count < T) {
    dev_free(ctx, slot->tiles, s);
    slot->tiles = nullptr;
    slot->count = 0;
    void* p = nullptr;
    const std::string err = ctx->err;
    if (dev_alloc(ctx, s, &p, size_t(T) * sizeof(uint32_t)) != GSR_OK) {  // a hint is optional
      ctx->err = err;
      slot->grid.clear();
      return;
    }
    slot->tiles = static_cast<uint32_t*>(p);
  }
  slot->count = T;
  if (hipMemcpyAsync(slot->tiles, sv->ck.tile_nmax, size_t(T) * sizeof(uint32_t), hipMemcpyDeviceToDevice, s) !=
      hipSuccess) {
    (void)hipGetLastError();
    slot->grid.clear();
  }
}

// Whether the compaction scans the projection's block sums itself (see launch_compact).
bool compact_scans(const gsr_saved* sv) { return sv->graph && int64_t(sv->V) * sv->nblk <= kCompactRawMax; }

// Phase A of a forward: clear the control words, project, scan the block sums.
hipError_t enqueue_project(gsr_saved* sv, hipStream_t s, bool timing) {
  gsr_ctx* ctx = sv->ctx;
  auto T = [&](int k, auto f) { return timing ? timed(ctx, s, k, f) : f(); };
  // the projection clears the control words (a captured step keeps its sticky overflow
  // word); without Gaussians a fill does
  const int clear = sv->graph ? kStepWords : kCtrlWords;
  if (sv->N == 0) return T(K_FILL, [&] { return launch_fill_u32(sv->ctrl, 0u, clear, s); });
  hipError_t e = T(K_PROJECT, [&] {
    // a captured step zeroes its 2D-gradient rows here, for the records that are visible
    return launch_project(sv->deg, sv->g, sv->vt, sv->ru, sv->s.tile, sv->rec, sv->blocksums, sv->nblk, sv->grad2d,
                          sv->ctrl, clear, (sv->s.flags & GSR_EXACT_TILES) ? sv->ru.k : 0.f, s);
  });
  // a captured step with few block sums leaves their scan to the compaction (the host
  // does not read the totals); an eager forward reads them to size its buffers
  if (e == hipSuccess && !compact_scans(sv))
    e = T(K_SCAN, [&] { return launch_scan_pairs(sv->blocksums, sv->V * sv->nblk, sv->d_total, s); });
  return e;
}

// Phase B: the depth sort of the visible records, their stable binning into tile lists
// (which also gives the tile ranges), the tile queue and the forward compositing.
hipError_t enqueue_sort_blend(gsr_saved* sv, hipStream_t s, bool timing) {
  gsr_ctx* ctx = sv->ctx;
  Timer* tm = (timing && ctx->timer.on) ? &ctx->timer : nullptr;
  ctx->timer.stream = s;
  auto T = [&](int k, auto f) { return timing ? timed(ctx, s, k, f) : f(); };
  uint32_t* ovf = sv->ctrl + kOverflow;
  hipError_t e = hipSuccess;
  sv->sort_passes = 0;
  const uint32_t* sorted = sv->dv;
  if (sv->cap_M > 0 && sv->cap_vis > 0) {
    bool alt = false;
    e = T(K_COMPACT, [&] {
      return launch_compact(sv->N, sv->V, sv->rec, sv->blocksums, sv->nblk, sv->d_total, sv->cap_M, sv->dk, sv->dv,
                            sv->cap_vis, ovf, compact_scans(sv), s);
    });
    if (e == hipSuccess)
      // depth keys are the bits of a positive binary32 depth: bit 31 is zero
      e = launch_radix_sort(sv->dk, sv->dv, sv->dk2, sv->dv2, sv->hist, sv->dtot, sv->d_total + 1, sv->cap_vis, ovf,
                            31, &alt, &sv->sort_passes, s, tm);
    if (alt) sorted = sv->dv2;
  }
  if (e == hipSuccess)
    // (the binning also writes the tile queue's order)
    e = launch_bin(sv->vt, sv->N, sv->rec, sorted, sv->d_total + 1, sv->cap_vis, sv->plan, sv->vals, sv->ranges,
                   sv->ctrl, (sv->s.flags & GSR_EXACT_TILES) ? sv->ru.k : 0.f, sv->s.tile, sv->order_hint, sv->order,
                   s, tm);
  if (e == hipSuccess)
    e = T(K_BLEND_FWD, [&] {
      return launch_blend_fwd(sv->s.tile, sv->s.batch, sv->vt, sv->ru, sv->rec, sv->ranges, sv->vals, sv->T_final,
                              sv->n_contrib, queue_of(sv), sv->ck, s);
    });
  return e;
}

// Backward launches for the view table `vt` (whose g_* pointers are set).  grad2d holds
// V*N rows of kGrad2D floats followed by N * 3 floats of scratch for the colour term.
hipError_t enqueue_backward(gsr_saved* sv, const ViewTable& vt, float* grad2d, const GradOut& go, hipStream_t s,
                            bool timing, const AdamDev& adam = AdamDev{}, uint32_t* adam_state = nullptr,
                            float* loss = nullptr) {
  gsr_ctx* ctx = sv->ctx;
  auto T = [&](int k, auto f) { return timing ? timed(ctx, s, k, f) : f(); };
  const int64_t VN = int64_t(sv->V) * sv->N;
  hipError_t e = hipSuccess;
  if (grad2d != sv->grad2d)  // the captured step's rows were zeroed by the projection
    e = T(K_FILL, [&] { return launch_fill_u32(reinterpret_cast<uint32_t*>(grad2d), 0u, VN * kGrad2D, s); });
  if (e == hipSuccess)
    e = T(K_BLEND_BWD, [&] {
      // a captured step (loss non-null) listed the work items in its loss kernel
      return launch_blend_bwd(sv->s.tile, sv->s.batch, vt, sv->ru, sv->rec, sv->ranges, sv->vals, sv->T_final,
                              sv->n_contrib, grad2d, queue_of(sv), sv->ck, s, loss != nullptr);
    });
  if (e == hipSuccess && adam.on) e = launch_adam_tick(adam_state, adam.b1, adam.b2, adam.skip, s);
  if (e == hipSuccess)
    e = T(K_PROJECT_BWD, [&] {
      return launch_project_bwd(sv->deg, sv->g, vt, sv->ru, sv->rec, grad2d, grad2d + VN * kGrad2D, go, adam, s,
                                sv->loss_part, loss ? loss_partials(vt) : 0, loss);
    });
  return e;
}

// Checks an optimiser description and fills the kernels' view of it for the parameter
// arrays p.
gsr_status adam_dev(gsr_ctx* ctx, const gsr_adam* o, float* const p[G_COUNT], AdamDev* a) {
  std::string err;
  if (check::adam(o, err) != GSR_OK) return fail(ctx, GSR_EINVAL, err);
  const float lr[G_COUNT + 1] = {o->lr_means, o->lr_scales, o->lr_quats, o->lr_opacities, o->lr_sh_dc, o->lr_sh_rest};
  *a = AdamDev{};
  for (int i = 0; i < G_COUNT; ++i) a->p[i] = p[i];
  float* const m[G_COUNT] = {o->m.means, o->m.scales, o->m.quats, o->m.opacities, o->m.sh};
  float* const v[G_COUNT] = {o->v.means, o->v.scales, o->v.quats, o->v.opacities, o->v.sh};
  for (int i = 0; i < G_COUNT; ++i) {
    a->m[i] = m[i];
    a->v[i] = v[i];
  }
  for (int i = 0; i <= G_COUNT; ++i) a->lr[i] = lr[i];
  a->bc = reinterpret_cast<const float*>(o->state + 1);
  a->b1 = o->beta1;
  a->b2 = o->beta2;
  a->eps = o->eps;
  a->on = 1;
  return GSR_OK;
}

// Device address of `scratch` on `device` (which must be current), looked up once per
// device and kept for the life of the process.
std::mutex g_noalloc_mu;
std::vector<void*> g_noalloc_ptr;

gsr_status noalloc_scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (g_noalloc_ptr.size() <= size_t(device)) g_noalloc_ptr.resize(size_t(device) + 1, nullptr);
  if (!g_noalloc_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(nullptr, GSR_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    }
    g_noalloc_ptr[device] = p;
  }
  *out = g_noalloc_ptr[device];
  return GSR_OK;
}

// The eager backward's 2D-gradient rows live in a context buffer that only grows:
// repeated steps reuse the same memory instead of a fresh allocation per call.
gsr_status bwd_scratch(gsr_ctx* ctx, size_t need) {
  if (need <= ctx->bwd_scratch_bytes) return GSR_OK;
  dev_free(ctx, ctx->bwd_scratch, ctx->stream);
  ctx->bwd_scratch = nullptr;
  ctx->bwd_scratch_bytes = 0;
  gsr_status st = dev_alloc(ctx, ctx->stream, &ctx->bwd_scratch, need + need / 8);
  if (st == GSR_OK) ctx->bwd_scratch_bytes = need + need / 8;
  return st;
}

// The saved forward's Gaussian arrays, which a fused optimiser step writes.
void saved_params(const gsr_saved* sv, float* p[G_COUNT]) {
  p[G_MEANS] = const_cast<float*>(sv->g.means);
  p[G_SCALES] = const_cast<float*>(sv->g.scales);
  p[G_QUATS] = const_cast<float*>(sv->g.quats);
  p[G_OPAC] = const_cast<float*>(sv->g.opac);
  p[G_SH] = const_cast<float*>(sv->g.sh);
}

// A full eager forward: phase A, one read-back of (M, visible), exact sort buffers, phase B.
gsr_status forward_eager(gsr_ctx* ctx, const gsr_gaussians* g, const gsr_camera* cams, int32_t V,
                         const gsr_settings* s, const gsr_view_out* outs, gsr_saved** out) {
  gsr_saved* sv = nullptr;
  gsr_status st = make_saved(ctx, g, cams, V, s, outs, &sv);
  if (st != GSR_OK) return st;
  hipStream_t strm = ctx->stream;
  if (s->flags & GSR_CHECK_FINITE) {
    // the control words are free until the projection clears them
    hipError_t e = launch_first_nonfinite(sv->g, sv->deg, sv->ctrl, strm);
    uint32_t* h = reinterpret_cast<uint32_t*>(ctx->h_total);
    if (e == hipSuccess) e = hipMemcpyAsync(h, sv->ctrl, sizeof(uint32_t), hipMemcpyDeviceToHost, strm);
    if (e == hipSuccess) e = hipStreamSynchronize(strm);
    const uint32_t first = h[0];
    if (e != hipSuccess) {
      release(sv);
      return fail(ctx, GSR_EDEVICE, std::string("finiteness check failed: ") + hipGetErrorString(e));
    }
    if (first != 0xFFFFFFFFu) {
      release(sv);
      return fail(ctx, GSR_EINVAL, "Gaussian " + std::to_string(first) + " has a NaN or infinite parameter");
    }
  }
  hipError_t e = enqueue_project(sv, strm, true);
  int64_t M = 0, NV = 0;
  if (e == hipSuccess && g->n > 0) {
    e = hipMemcpyAsync(ctx->h_total, sv->d_total, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, strm);
    if (e == hipSuccess) e = hipStreamSynchronize(strm);
    M = int64_t(ctx->h_total[0]);
    NV = int64_t(ctx->h_total[1]);
  }
  if (e != hipSuccess) {
    release(sv);
    return fail(ctx, GSR_EDEVICE, std::string("forward (projection) failed: ") + hipGetErrorString(e));
  }
  if (M >= (int64_t(1) << 32)) {
    release(sv);
    return fail(ctx, GSR_ECAPACITY, "more than 2^32 duplicated keys");
  }
  sv->M = M;
  sv->n_vis = NV;
  if ((st = alloc_sort(sv, NV, M, false)) != GSR_OK) {
    release(sv);
    return st;
  }
  sv->order_hint = find_hint(ctx, sv);
  e = enqueue_sort_blend(sv, strm, true);
  if (e != hipSuccess) {
    release(sv);
    return fail(ctx, GSR_EDEVICE, std::string("forward (sort/blend) failed: ") + hipGetErrorString(e));
  }
  keep_hint(ctx, sv, strm);
  // keep the pair list, return every temporary to the pool
  free_list(sv, sv->temps);
  *out = sv;
  return GSR_OK;
}

ViewTable with_grads(const gsr_saved* sv, const gsr_view_grad* grads) {
  ViewTable vt = sv->vt;
  for (int v = 0; v < vt.nviews; ++v) {
    vt.v[v].g_color = grads[v].color;
    vt.v[v].g_depth = grads[v].depth;
    vt.v[v].g_alpha = grads[v].alpha;
  }
  return vt;
}

gsr_status loss_table(gsr_ctx* ctx, const gsr_saved* saved, const gsr_view_out* outs, const gsr_target* targets,
                      float depth_weight, float* const* gcol, float* const* gdep, ViewTable* vt) {
  if (!(depth_weight >= 0.f)) return fail(ctx, GSR_EINVAL, "depth_weight must be >= 0");
  *vt = saved->vt;
  for (int v = 0; v < vt->nviews; ++v) {
    if (!outs[v].color || !targets[v].color || !gcol[v])
      return fail(ctx, GSR_EINVAL, "colour image, target or gradient pointer is NULL");
    if (targets[v].depth && (!outs[v].depth || !gdep || !gdep[v]))
      return fail(ctx, GSR_EINVAL, "depth target given without rendered depth / gradient buffer");
    vt->v[v].color = outs[v].color;
    vt->v[v].depth = outs[v].depth;
    vt->v[v].t_color = targets[v].color;
    vt->v[v].t_depth = targets[v].depth;
    vt->v[v].lg_color = gcol[v];
    vt->v[v].lg_depth = gdep ? gdep[v] : nullptr;
  }
  return GSR_OK;
}

}  // namespace

extern "C" {

int32_t gsr_abi_version(void) { return GSR_ABI_VERSION; }

gsr_status gsr_settings_default(gsr_settings* s) {
  if (!s) return fail(nullptr, GSR_EINVAL, "settings is NULL");
  s->tile = 16;
  s->batch = 256;
  s->extent_k = 3.33f;
  s->lowpass = 0.3f;
  s->alpha_min = 1.0f / 255.0f;
  s->alpha_max = 0.99f;
  s->T_min = 1e-4f;
  s->guard = 0.15f;
  s->bg[0] = s->bg[1] = s->bg[2] = 0.f;
  s->flags = 0;
  s->jclamp = 0.f;
  return GSR_OK;
}

const char* gsr_last_error(const gsr_ctx* ctx) { return ctx ? ctx->err.c_str() : g_noctx_err.c_str(); }

gsr_status gsr_ctx_create(int32_t device, void* hip_stream, const gsr_alloc* alloc, gsr_ctx** out) {
  if (!out) return fail(nullptr, GSR_EINVAL, "out is NULL");
  *out = nullptr;
  if (alloc && (!alloc->alloc || !alloc->free))
    return fail(nullptr, GSR_EINVAL, "an allocator needs both its alloc and free functions");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    return fail(nullptr, GSR_EDEVICE, "no HIP device available");
  }
  if (device < 0 || device >= ndev) return fail(nullptr, GSR_EINVAL, "device index out of range");
  if (hipSetDevice(device) != hipSuccess) return fail(nullptr, GSR_EDEVICE, "hipSetDevice failed");
  void* fixed = nullptr;
  gsr_status st = noalloc_scratch_address(device, &fixed);
  if (st != GSR_OK) return st;
  gsr_ctx* c = new gsr_ctx;
  c->device = device;
  c->noalloc_scratch = fixed;
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (alloc) c->alloc = *alloc;
  if (hipHostMalloc(reinterpret_cast<void**>(&c->h_total), 2 * sizeof(unsigned long long), hipHostMallocDefault) !=
      hipSuccess) {
    delete c;
    return fail(nullptr, GSR_ENOMEM, "pinned host allocation failed");
  }
  // keep freed pool memory cached: the per-step allocations are then served without the driver
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  (void)hipGetLastError();
  *out = c;
  return GSR_OK;
}

gsr_status gsr_ctx_destroy(gsr_ctx* ctx) {
  if (!ctx) return fail(nullptr, GSR_EINVAL, "ctx is NULL");
  (void)hipStreamSynchronize(ctx->stream);
  dev_free(ctx, ctx->bwd_scratch, ctx->stream);
  for (auto& h : ctx->hints) dev_free(ctx, h.tiles, ctx->stream);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->timer.destroy();
  if (ctx->h_total) (void)hipHostFree(ctx->h_total);
  delete ctx;
  return GSR_OK;
}

gsr_status gsr_ctx_set_timing(gsr_ctx* ctx, int32_t enable) {
  if (!ctx) return fail(nullptr, GSR_EINVAL, "ctx is NULL");
  ctx->timer.on = enable != 0;
  ctx->timer.stream = ctx->stream;
  return GSR_OK;
}

gsr_status gsr_ctx_get_timing(gsr_ctx* ctx, gsr_timing* out, int32_t reset) {
  if (!ctx || !out) return fail(ctx, GSR_EINVAL, "NULL argument to gsr_ctx_get_timing");
  GSR_HIP(ctx, hipStreamSynchronize(ctx->stream));
  ctx->timer.collect();
  std::memset(out, 0, sizeof(*out));
  out->count = K_COUNT;
  for (int i = 0; i < K_COUNT; ++i) {
    out->ms[i] = ctx->timer.ms[i];
    out->launches[i] = ctx->timer.launches[i];
  }
  if (reset) ctx->timer.reset();
  return GSR_OK;
}

const char* gsr_kernel_name(int32_t id) { return (id >= 0 && id < K_COUNT) ? kKernelNames[id] : ""; }

gsr_status gsr_ctx_set_stream(gsr_ctx* ctx, void* hip_stream) {
  if (!ctx) return fail(nullptr, GSR_EINVAL, "ctx is NULL");
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return GSR_OK;
}

gsr_status gsr_forward(gsr_ctx* ctx, const gsr_gaussians* g, const gsr_camera* cams, int32_t V,
                       const gsr_settings* s, const gsr_view_out* outs, gsr_saved** saved) {
  if (!ctx) return fail(nullptr, GSR_EINVAL, "ctx is NULL");
  if (saved) *saved = nullptr;
  gsr_status st = check_forward_args(ctx, g, cams, V, s, outs);
  if (st != GSR_OK) return st;
  ctx->err.clear();
  gsr_saved* sv = nullptr;
  if ((st = forward_eager(ctx, g, cams, V, s, outs, &sv)) != GSR_OK) return st;
  if (saved)
    *saved = sv;
  else
    release(sv);
  return GSR_OK;
}

gsr_status gsr_loss_l1(gsr_ctx* ctx, const gsr_saved* saved, const gsr_view_out* outs, const gsr_target* targets,
                       float depth_weight, float* const* grad_color_out, float* const* grad_depth_out,
                       float* loss_dev) {
  if (!ctx) return fail(nullptr, GSR_EINVAL, "ctx is NULL");
  if (!saved || !outs || !targets || !grad_color_out || !loss_dev)
    return fail(ctx, GSR_EINVAL, "NULL argument to gsr_loss_l1");
  ViewTable vt;
  gsr_status st = loss_table(ctx, saved, outs, targets, depth_weight, grad_color_out, grad_depth_out, &vt);
  if (st != GSR_OK) return st;
  GSR_HIP(ctx, timed(ctx, ctx->stream, K_LOSS,
                     [&] { return launch_loss_l1(vt, depth_weight, saved->loss_part, loss_dev, ctx->stream); }));
  return GSR_OK;
}

gsr_status gsr_backward(gsr_ctx* ctx, const gsr_saved* saved, const gsr_view_grad* grads,
                        const gsr_gaussian_grads* out, uint32_t flags) {
  if (!ctx) return fail(nullptr, GSR_EINVAL, "ctx is NULL");
  if (!saved || !grads || !out) return fail(ctx, GSR_EINVAL, "NULL argument to gsr_backward");
  if (flags & ~GSR_ACCUMULATE) return fail(ctx, GSR_EINVAL, "unknown flag");
  gsr_saved* sv = const_cast<gsr_saved*>(saved);
  const ViewTable vt = with_grads(sv, grads);
  const int64_t VN = int64_t(sv->V) * sv->N;
  gsr_status st = bwd_scratch(ctx, (size_t(VN) * kGrad2D + size_t(sv->N) * 3) * sizeof(float));
  if (st != GSR_OK) return st;
  GradOut go{out->means, out->scales, out->quats, out->opacities, out->sh, int(flags & GSR_ACCUMULATE)};
  hipError_t e = enqueue_backward(sv, vt, static_cast<float*>(ctx->bwd_scratch), go, ctx->stream, true);
  if (e != hipSuccess) return fail(ctx, GSR_EDEVICE, std::string("backward launch failed: ") + hipGetErrorString(e));
  return GSR_OK;
}

gsr_status gsr_backward_noalloc(gsr_ctx* ctx, const gsr_saved* saved, const gsr_view_grad* grads,
                                const gsr_gaussian_grads* out, uint32_t flags) {
  if (!ctx) return fail(nullptr, GSR_EINVAL, "ctx is NULL");
  if (!saved || !grads || !out) return fail(ctx, GSR_EINVAL, "NULL argument to gsr_backward_noalloc");
  if (flags & ~GSR_ACCUMULATE) return fail(ctx, GSR_EINVAL, "unknown flag");
  gsr_saved* sv = const_cast<gsr_saved*>(saved);
  if (sv->ctx->device != ctx->device) return fail(ctx, GSR_EINVAL, "saved state belongs to another device");
  const int64_t VN = int64_t(sv->V) * sv->N;
  const size_t need = (size_t(VN) * kGrad2D + size_t(sv->N) * 3) * sizeof(float);
  if (need > size_t(GSR_NOALLOC_SCRATCH_BYTES))
    return fail(ctx, GSR_EINVAL, "gsr_backward_noalloc needs " + std::to_string(need) +
                                     " bytes of scratch (views * Gaussians * 48 + Gaussians * 12); the fixed array "
                                     "holds " + std::to_string(size_t(GSR_NOALLOC_SCRATCH_BYTES)));
  if (!ctx->noalloc_scratch) return fail(ctx, GSR_EDEVICE, "no fixed scratch address for this device");
  const ViewTable vt = with_grads(sv, grads);
  GradOut go{out->means, out->scales, out->quats, out->opacities, out->sh, int(flags & GSR_ACCUMULATE)};
  // no event timer here: its events are created on demand
  hipError_t e = enqueue_backward(sv, vt, static_cast<float*>(ctx->noalloc_scratch), go, ctx->stream, false);
  if (e != hipSuccess) return fail(ctx, GSR_EDEVICE, std::string("backward launch failed: ") + hipGetErrorString(e));
  return GSR_OK;
}

gsr_status gsr_backward_adam(gsr_ctx* ctx, const gsr_saved* saved, const gsr_view_grad* grads,
                             const gsr_adam* opt) {
  if (!ctx) return fail(nullptr, GSR_EINVAL, "ctx is NULL");
  if (!saved || !grads || !opt) return fail(ctx, GSR_EINVAL, "NULL argument to gsr_backward_adam");
  gsr_saved* sv = const_cast<gsr_saved*>(saved);
  float* p[G_COUNT];
  saved_params(sv, p);
  AdamDev ad;
  gsr_status st = adam_dev(ctx, opt, p, &ad);
  if (st != GSR_OK) return st;
  ad.skip = sv->ctrl + kOverflowSticky;
  const ViewTable vt = with_grads(sv, grads);
  const int64_t VN = int64_t(sv->V) * sv->N;
  if ((st = bwd_scratch(ctx, (size_t(VN) * kGrad2D + size_t(sv->N) * 3) * sizeof(float))) != GSR_OK) return st;
  const GradOut go{nullptr, nullptr, nullptr, nullptr, nullptr, 0};
  hipError_t e = enqueue_backward(sv, vt, static_cast<float*>(ctx->bwd_scratch), go, ctx->stream, true, ad,
                                  opt->state);
  if (e != hipSuccess) return fail(ctx, GSR_EDEVICE, std::string("backward launch failed: ") + hipGetErrorString(e));
  return GSR_OK;
}

gsr_status gsr_adam_default(gsr_adam* a) {
  if (!a) return fail(nullptr, GSR_EINVAL, "NULL argument to gsr_adam_default");
  *a = gsr_adam{};
  a->lr_means = 1.6e-4f;
  a->lr_scales = 5e-3f;
  a->lr_quats = 1e-3f;
  a->lr_opacities = 0.05f;
  a->lr_sh_dc = 2.5e-3f;
  a->lr_sh_rest = 2.5e-3f / 20.f;
  a->beta1 = 0.9f;
  a->beta2 = 0.999f;
  a->eps = 1e-15f;
  return GSR_OK;
}

gsr_status gsr_adam_step(gsr_ctx* ctx, int64_t n, int32_t sh_degree, const gsr_gaussian_grads* params,
                         const gsr_gaussian_grads* grads, const gsr_adam* opt) {
  if (!ctx) return fail(nullptr, GSR_EINVAL, "ctx is NULL");
  if (!params || !grads || !opt) return fail(ctx, GSR_EINVAL, "NULL argument to gsr_adam_step");
  if (n < 0 || sh_degree < 0 || sh_degree > 3) return fail(ctx, GSR_EINVAL, "n must be >= 0 and sh_degree in 0..3");
  float* const p[G_COUNT] = {params->means, params->scales, params->quats, params->opacities, params->sh};
  const float* const g[G_COUNT] = {grads->means, grads->scales, grads->quats, grads->opacities, grads->sh};
  for (int i = 0; i < G_COUNT; ++i)
    if (n > 0 && (!p[i] || !g[i])) return fail(ctx, GSR_EINVAL, "every parameter and gradient array is required");
  AdamDev ad;
  gsr_status st = adam_dev(ctx, opt, p, &ad);
  if (st != GSR_OK) return st;
  hipStream_t s = ctx->stream;
  GSR_HIP(ctx, launch_adam_tick(opt->state, ad.b1, ad.b2, nullptr, s));
  GSR_HIP(ctx, timed(ctx, s, K_ADAM, [&] { return launch_adam(ad, g, n, sh_degree, s); }));
  return GSR_OK;
}

gsr_status gsr_saved_info(const gsr_saved* saved, gsr_info* info) {
  if (!saved || !info) return fail(nullptr, GSR_EINVAL, "NULL argument to gsr_saved_info");
  info->num_keys = saved->M;
  info->num_tiles = saved->vt.total_tiles;
  info->num_pixels = saved->total_pix;
  info->num_records = int64_t(saved->V) * saved->N;
  info->views = saved->V;
  info->sort_passes = saved->sort_passes;
  return GSR_OK;
}

gsr_status gsr_saved_free(gsr_saved* saved) {
  if (!saved) return fail(nullptr, GSR_EINVAL, "saved is NULL");
  release(saved);
  return GSR_OK;
}

gsr_status gsr_debug_export(gsr_ctx* ctx, const gsr_saved* sv, const gsr_debug* out) {
  if (!ctx) return fail(nullptr, GSR_EINVAL, "ctx is NULL");
  if (!sv || !out) return fail(ctx, GSR_EINVAL, "NULL argument to gsr_debug_export");
  hipStream_t s = ctx->stream;
  GSR_HIP(ctx, hipStreamSynchronize(s));
  const int64_t VN = int64_t(sv->V) * sv->N;
  auto cp = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    if (!dst || !src || bytes == 0) return hipSuccess;
    return hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost);
  };
  if (out->keys && sv->M > 0) {  // key = tile << 32 | depth bits of the pair's record
    const int64_t nt = sv->vt.total_tiles;
    std::vector<uint32_t> v(sv->M);
    std::vector<uint2> rg(nt);
    std::vector<float4> r1(VN);
    GSR_HIP(ctx, cp(v.data(), sv->vals, size_t(sv->M) * 4));
    GSR_HIP(ctx, cp(rg.data(), sv->ranges, size_t(nt) * 8));
    GSR_HIP(ctx, cp(r1.data(), sv->rec.r1, size_t(VN) * sizeof(float4)));
    // the pair list holds no tile ids: each tile's range names the tile of its pairs
    // (pairs outside every range keep tile id 0xFFFFFFFF)
    for (int64_t i = 0; i < sv->M; ++i) out->keys[i] = uint64_t(0xFFFFFFFFu) << 32;
    for (int64_t t = 0; t < nt; ++t)
      for (uint32_t i = rg[t].x; i < rg[t].y && int64_t(i) < sv->M; ++i) out->keys[i] = uint64_t(t) << 32;
    for (int64_t i = 0; i < sv->M; ++i) {
      uint32_t zb = 0;
      if (int64_t(v[i]) < VN) std::memcpy(&zb, &r1[v[i]].z, 4);
      out->keys[i] |= zb;
    }
  }
  GSR_HIP(ctx, cp(out->values, sv->vals, size_t(sv->M) * 4));
  GSR_HIP(ctx, cp(out->ranges, sv->ranges, size_t(sv->vt.total_tiles) * 8));
  GSR_HIP(ctx, cp(out->T_final, sv->T_final, size_t(sv->total_pix) * 4));
  GSR_HIP(ctx, cp(out->n_contrib, sv->n_contrib, size_t(sv->total_pix) * 4));
  if (out->n_used && sv->total_pix > 0) {  // counted on demand, off the forward's path
    void* nuv = nullptr;
    gsr_status st = dev_alloc(ctx, s, &nuv, size_t(sv->total_pix) * 4);
    if (st != GSR_OK) return st;
    uint32_t* nu = static_cast<uint32_t*>(nuv);
    hipError_t e = launch_count_used(sv->vt, sv->ru, sv->rec, sv->ranges, sv->vals, sv->n_contrib, sv->s.tile,
                                     sv->total_pix, nu, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = cp(out->n_used, nu, size_t(sv->total_pix) * 4);
    dev_free(ctx, nu, s);
    GSR_HIP(ctx, e);
  }
  GSR_HIP(ctx, cp(out->tiles_touched, sv->rec.counts, size_t(VN) * 4));
  if (out->mu || out->depth || out->conic || out->color || out->rect) {
    std::vector<float4> r0(VN), r1(VN), rgb(VN);
    std::vector<uint2> rc(VN);
    std::vector<uint32_t> cnt(VN);
    GSR_HIP(ctx, cp(r0.data(), sv->rec.r0, VN * sizeof(float4)));
    GSR_HIP(ctx, cp(r1.data(), sv->rec.r1, VN * sizeof(float4)));
    GSR_HIP(ctx, cp(rgb.data(), sv->rec.rgb, VN * sizeof(float4)));
    GSR_HIP(ctx, cp(rc.data(), sv->rec.rect, VN * sizeof(uint2)));
    GSR_HIP(ctx, cp(cnt.data(), sv->rec.counts, VN * 4));
    for (int64_t i = 0; i < VN; ++i) {
      const bool vis = cnt[i] != 0;
      if (out->mu) {
        out->mu[i * 2] = vis ? r0[i].x : 0.f;
        out->mu[i * 2 + 1] = vis ? r0[i].y : 0.f;
      }
      if (out->depth) out->depth[i] = vis ? r1[i].z : 0.f;
      if (out->conic) {
        out->conic[i * 3] = vis ? r0[i].z : 0.f;
        out->conic[i * 3 + 1] = vis ? r0[i].w : 0.f;
        out->conic[i * 3 + 2] = vis ? r1[i].x : 0.f;
      }
      if (out->color) {
        out->color[i * 3] = vis ? rgb[i].x : 0.f;
        out->color[i * 3 + 1] = vis ? rgb[i].y : 0.f;
        out->color[i * 3 + 2] = vis ? rgb[i].z : 0.f;
      }
      if (out->rect) {
        out->rect[i * 4] = vis ? int32_t(rc[i].x & 0xFFFF) : 0;
        out->rect[i * 4 + 1] = vis ? int32_t(rc[i].x >> 16) : -1;
        out->rect[i * 4 + 2] = vis ? int32_t(rc[i].y & 0xFFFF) : 0;
        out->rect[i * 4 + 3] = vis ? int32_t(rc[i].y >> 16) : -1;
      }
    }
  }
  return GSR_OK;
}

// ------------------------------------------------------------------------------------
// Captured step
// ------------------------------------------------------------------------------------
static void graph_destroy(gsr_graph* gr) {
  if (!gr) return;
  if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
  if (gr->graph) (void)hipGraphDestroy(gr->graph);
  if (gr->done) (void)hipEventDestroy(gr->done);
  if (gr->capture) (void)hipStreamDestroy(gr->capture);
  if (gr->h_flag) (void)hipHostFree(gr->h_flag);
  if (gr->sv) release(gr->sv);
  delete gr;
}

gsr_status gsr_graph_create(gsr_ctx* ctx, const gsr_gaussians* g, const gsr_camera* cams, int32_t V,
                            const gsr_settings* s, const gsr_view_out* outs, const gsr_target* targets,
                            float depth_weight, float* const* grad_color, float* const* grad_depth,
                            const gsr_gaussian_grads* grads, float* loss_dev, float headroom,
                            const gsr_adam* opt, gsr_graph** out) {
  if (!ctx) return fail(nullptr, GSR_EINVAL, "ctx is NULL");
  if (!out || !targets || (!grads && !opt) || !loss_dev || !grad_color)
    return fail(ctx, GSR_EINVAL, "NULL argument to gsr_graph_create");
  *out = nullptr;
  if (!(headroom >= 0.f) || headroom > 16.f) return fail(ctx, GSR_EINVAL, "headroom must be in [0, 16]");
  gsr_status st = check_forward_args(ctx, g, cams, V, s, outs);
  if (st != GSR_OK) return st;
  ctx->err.clear();
  // one eager forward measures the sizes the capacities are derived from
  gsr_saved* probe = nullptr;
  if ((st = forward_eager(ctx, g, cams, V, s, outs, &probe)) != GSR_OK) return st;
  const int64_t M = probe->M, NV = probe->n_vis;
  release(probe);
  const int64_t VN = int64_t(V) * g->n;
  const int64_t cap_vis = std::min<int64_t>(VN, int64_t(std::ceil(double(NV) * (1.0 + headroom))) + 256);
  int64_t cap_M = int64_t(std::ceil(double(M) * (1.0 + headroom))) + 4096;
  cap_M = std::min<int64_t>(cap_M, (int64_t(1) << 32) - 1);

  gsr_graph* gr = new gsr_graph;
  gr->ctx = ctx;
  if ((st = make_saved(ctx, g, cams, V, s, outs, &gr->sv)) != GSR_OK) {
    delete gr;
    return st;
  }
  gsr_saved* sv = gr->sv;
  sv->graph = true;
  sv->M = M;
  sv->n_vis = NV;
  if ((st = alloc_sort(sv, cap_vis, cap_M, true)) != GSR_OK ||
      (st = alloc_in(sv, sv->blocks, &sv->grad2d, size_t(VN) * kGrad2D + size_t(sv->N) * 3)) != GSR_OK) {
    graph_destroy(gr);
    return st;
  }
  // the captured forward orders its tiles by the per-tile work of the replay before it;
  // the first replay uses the measuring forward's
  if (const uint32_t* h = find_hint(ctx, sv)) {
    if (hipMemcpyAsync(sv->ck.tile_nmax, h, size_t(sv->vt.total_tiles) * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                       ctx->stream) == hipSuccess)
      sv->order_hint = sv->ck.tile_nmax;
    else
      (void)hipGetLastError();
  }
  ViewTable lvt;
  if ((st = loss_table(ctx, sv, outs, targets, depth_weight, grad_color, grad_depth, &lvt)) != GSR_OK) {
    graph_destroy(gr);
    return st;
  }
  std::vector<gsr_view_grad> vg(V);
  for (int v = 0; v < V; ++v) vg[v] = gsr_view_grad{grad_color[v], grad_depth ? grad_depth[v] : nullptr, nullptr};
  const ViewTable bvt = with_grads(sv, vg.data());
  const GradOut go = grads ? GradOut{grads->means, grads->scales, grads->quats, grads->opacities, grads->sh, 0}
                           : GradOut{nullptr, nullptr, nullptr, nullptr, nullptr, 0};
  AdamDev ad{};
  if (opt) {
    float* p[G_COUNT];
    saved_params(sv, p);
    if ((st = adam_dev(ctx, opt, p, &ad)) != GSR_OK) {
      graph_destroy(gr);
      return st;
    }
    ad.skip = sv->ctrl + kOverflowSticky;  // no update once any launch has overflowed
  }

  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&gr->h_flag), sizeof(uint32_t), hipHostMallocDefault);
  // every control word starts at zero once; the steps clear only their own words
  if (e == hipSuccess) e = launch_fill_u32(sv->ctrl, 0u, kCtrlWords, ctx->stream);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&gr->done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&gr->capture, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);  // buffers allocated on ctx->stream are ready
  if (e != hipSuccess) {
    graph_destroy(gr);
    return fail(ctx, GSR_EDEVICE, std::string("graph set-up failed: ") + hipGetErrorString(e));
  }
  *gr->h_flag = 0;
  hipStream_t cs = gr->capture;
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t k = enqueue_project(sv, cs, false);
    if (k == hipSuccess) k = enqueue_sort_blend(sv, cs, false);
    // the loss kernel also lists the backward's work items; the loss total is added up by
    // the backward projection
    if (k == hipSuccess)
      k = launch_loss_l1(lvt, depth_weight, sv->loss_part, nullptr, cs, sv->order, sv->s.batch, &sv->ck, sv->ctrl);
    if (k == hipSuccess)
      k = enqueue_backward(sv, bvt, sv->grad2d, go, cs, false, ad, opt ? opt->state : nullptr, loss_dev);
    if (k == hipSuccess)
      k = hipMemcpyAsync(gr->h_flag, sv->ctrl + kOverflowSticky, sizeof(uint32_t), hipMemcpyDeviceToHost, cs);
    e = hipStreamEndCapture(cs, &gr->graph);
    if (k != hipSuccess) e = k;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    graph_destroy(gr);
    return fail(ctx, GSR_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(e));
  }
  *out = gr;
  return GSR_OK;
}

gsr_status gsr_graph_launch(gsr_graph* gr) {
  if (!gr) return fail(nullptr, GSR_EINVAL, "graph is NULL");
  gsr_ctx* ctx = gr->ctx;
  if (gr->launched && !gr->overflowed && hipEventQuery(gr->done) == hipSuccess && *gr->h_flag) gr->overflowed = true;
  (void)hipGetLastError();
  if (gr->overflowed) return fail(ctx, GSR_ECAPACITY, "a captured step exceeded its key capacity; re-create the graph");
  GSR_HIP(ctx, hipGraphLaunch(gr->exec, ctx->stream));
  GSR_HIP(ctx, hipEventRecord(gr->done, ctx->stream));
  gr->launched = true;
  return GSR_OK;
}

gsr_status gsr_graph_sync(gsr_graph* gr) {
  if (!gr) return fail(nullptr, GSR_EINVAL, "graph is NULL");
  gsr_ctx* ctx = gr->ctx;
  if (gr->launched) GSR_HIP(ctx, hipEventSynchronize(gr->done));
  if (gr->launched && *gr->h_flag) gr->overflowed = true;
  if (gr->overflowed) return fail(ctx, GSR_ECAPACITY, "a captured step exceeded its key capacity; re-create the graph");
  return GSR_OK;
}

gsr_status gsr_graph_info(const gsr_graph* gr, gsr_info* info, int64_t* cap_keys, int64_t* cap_visible) {
  if (!gr || !info) return fail(nullptr, GSR_EINVAL, "NULL argument to gsr_graph_info");
  gsr_saved_info(gr->sv, info);
  if (cap_keys) *cap_keys = gr->sv->cap_M;
  if (cap_visible) *cap_visible = gr->sv->cap_vis;
  return GSR_OK;
}

gsr_status gsr_graph_free(gsr_graph* gr) {
  if (!gr) return fail(nullptr, GSR_EINVAL, "graph is NULL");
  if (gr->launched) (void)hipEventSynchronize(gr->done);
  graph_destroy(gr);
  return GSR_OK;
}

// ------------------------------------------------------------------------------------
// Launch-shape autotuner
// ------------------------------------------------------------------------------------
static std::string autotune_key(int dev, const gsr_gaussians* g, const gsr_camera* cams, int V) {
  hipDeviceProp_t p;
  std::string arch = "unknown";
  int cus = 0;
  if (hipGetDeviceProperties(&p, dev) == hipSuccess) {
    arch = p.gcnArchName;
    cus = p.multiProcessorCount;
  }
  int64_t pix = 0;
  for (int v = 0; v < V; ++v) pix += int64_t(cams[v].width) * cams[v].height;
  std::ostringstream k;
  k << arch.substr(0, arch.find(':')) << "|cu" << cus << "|px" << bits_for(uint64_t(pix)) << "|n"
    << bits_for(uint64_t(g->n)) << "|deg" << g->sh_degree << "|v" << V << "|x2";
  return k.str();
}

static std::string autotune_path() {
  const char* p = std::getenv("GSR_AUTOTUNE_CACHE");
  if (p && *p) return p;
  const char* home = std::getenv("HOME");
  return std::string(home ? home : "/tmp") + "/.cache/gsr_autotune.txt";
}

gsr_status gsr_autotune(gsr_ctx* ctx, const gsr_gaussians* g, const gsr_camera* cams, int32_t V, gsr_settings* s,
                        uint32_t flags, float* best_ms) {
  if (!ctx) return fail(nullptr, GSR_EINVAL, "ctx is NULL");
  if (!s) return fail(ctx, GSR_EINVAL, "settings is NULL");
  if (flags & ~GSR_AUTOTUNE_NO_CACHE) return fail(ctx, GSR_EINVAL, "unknown flag");
  std::vector<gsr_view_out> dummy(V > 0 ? V : 1, gsr_view_out{reinterpret_cast<float*>(16), nullptr, nullptr});
  gsr_status st = check_forward_args(ctx, g, cams, V, s, dummy.data());
  if (st != GSR_OK) return st;
  const std::string key = autotune_key(ctx->device, g, cams, V);
  const std::string path = autotune_path();
  const bool use_cache = !(flags & GSR_AUTOTUNE_NO_CACHE);
  if (use_cache) {
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string k;
      int t = 0, b = 0, x = 0;
      float ms = 0.f;
      if ((ls >> k >> t >> b >> x >> ms) && k == key && (t == 8 || t == 16 || t == 32) && (b == 128 || b == 256) &&
          (x == 0 || x == 1)) {
        s->tile = t;
        s->batch = b;
        s->flags = (s->flags & ~GSR_EXACT_TILES) | (x ? GSR_EXACT_TILES : 0u);
        if (best_ms) *best_ms = ms;
        return GSR_OK;
      }
    }
  }
  // scratch images, output gradients (dL/dcolour = 1/(3P)) and parameter gradients
  hipStream_t strm = ctx->stream;
  std::vector<void*> scratch;
  auto salloc = [&](size_t bytes) -> float* {
    void* p = nullptr;
    if (dev_alloc(ctx, strm, &p, bytes) != GSR_OK) return nullptr;
    if (p) scratch.push_back(p);
    return static_cast<float*>(p);
  };
  auto sfree = [&]() {
    for (void* p : scratch) dev_free(ctx, p, strm);
    (void)hipStreamSynchronize(strm);
  };
  std::vector<gsr_view_out> outs(V);
  std::vector<gsr_view_grad> vg(V);
  bool ok = true;
  for (int v = 0; v < V && ok; ++v) {
    const size_t P = size_t(cams[v].width) * cams[v].height;
    float* img = salloc(P * 5 * sizeof(float));
    float* gc = salloc(P * 3 * sizeof(float));
    ok = img && gc;
    if (!ok) break;
    outs[v] = gsr_view_out{img, img + 3 * P, img + 4 * P};
    const float val = 1.f / float(3 * P);
    uint32_t bits;
    std::memcpy(&bits, &val, 4);
    ok = launch_fill_u32(reinterpret_cast<uint32_t*>(gc), bits, int64_t(3 * P), strm) == hipSuccess;
    vg[v] = gsr_view_grad{gc, nullptr, nullptr};
  }
  const int K = (g->sh_degree + 1) * (g->sh_degree + 1);
  float* gbuf = ok ? salloc(size_t(std::max<int64_t>(g->n, 1)) * (14 + 3 * K) * sizeof(float)) : nullptr;
  if (!ok || !gbuf) {
    sfree();
    return fail(ctx, GSR_ENOMEM, "autotune scratch allocation failed");
  }
  gsr_gaussian_grads gg{gbuf, gbuf + 3 * g->n, gbuf + 6 * g->n, gbuf + 10 * g->n, gbuf + 11 * g->n};
  // each candidate is timed by the sum of its kernels' durations (the context's event
  // timer), so the host-side gap of the eager forward's count read-back does not count
  const bool timer_was = ctx->timer.on;
  ctx->timer.collect();
  double saved_ms[K_COUNT];
  long long saved_n[K_COUNT];
  std::copy(ctx->timer.ms, ctx->timer.ms + K_COUNT, saved_ms);
  std::copy(ctx->timer.launches, ctx->timer.launches + K_COUNT, saved_n);
  ctx->timer.on = true;
  // candidates: every (list kind, tile, batch); after two warm-up steps each, the
  // candidates take turns, one step per turn, so slow drift of the clocks or of the
  // memory system reaches all of them alike; each is scored by its median step
  struct Cand {
    gsr_settings c;
    int xi;
  };
  std::vector<Cand> cands;
  const int tiles[3] = {8, 16, 32}, batches[2] = {128, 256};
  for (int xi = 0; xi < 2; ++xi)
    for (int ti = 0; ti < 3; ++ti)
      for (int bi = 0; bi < 2; ++bi) {
        gsr_settings c = *s;
        c.tile = tiles[ti];
        c.batch = batches[bi];
        c.flags = (s->flags & ~GSR_EXACT_TILES) | (xi ? GSR_EXACT_TILES : 0u);
        cands.push_back({c, xi});
      }
  constexpr int kWarm = 2, kTimed = 9;
  std::vector<float> times(cands.size() * kTimed);
  auto one_step = [&](const gsr_settings& c, float* ms_out) -> gsr_status {
    ctx->timer.reset();
    gsr_saved* sv = nullptr;
    gsr_status r = forward_eager(ctx, g, cams, V, &c, outs.data(), &sv);
    if (r != GSR_OK) return r;
    r = gsr_backward(ctx, sv, vg.data(), &gg, 0);
    release(sv);
    (void)hipStreamSynchronize(strm);
    ctx->timer.collect();
    double ms = 0.0;
    for (int k = 0; k < K_COUNT; ++k) ms += ctx->timer.ms[k];
    *ms_out = float(ms);
    return r;
  };
  for (size_t i = 0; i < cands.size() && st == GSR_OK; ++i)
    for (int rep = 0; rep < kWarm && st == GSR_OK; ++rep) {
      float ms;
      st = one_step(cands[i].c, &ms);
    }
  for (int rep = 0; rep < kTimed && st == GSR_OK; ++rep)
    for (size_t i = 0; i < cands.size() && st == GSR_OK; ++i) st = one_step(cands[i].c, &times[i * kTimed + rep]);
  float best = 1e30f;
  int bt = s->tile, bb = s->batch, bx = 0;
  for (size_t i = 0; i < cands.size() && st == GSR_OK; ++i) {
    float* t = &times[i * kTimed];
    std::sort(t, t + kTimed);
    if (t[kTimed / 2] < best) {
      best = t[kTimed / 2];
      bt = cands[i].c.tile;
      bb = cands[i].c.batch;
      bx = cands[i].xi;
    }
  }
  ctx->timer.on = timer_was;
  std::copy(saved_ms, saved_ms + K_COUNT, ctx->timer.ms);
  std::copy(saved_n, saved_n + K_COUNT, ctx->timer.launches);
  sfree();
  if (st != GSR_OK) return st;
  s->tile = bt;
  s->batch = bb;
  s->flags = (s->flags & ~GSR_EXACT_TILES) | (bx ? GSR_EXACT_TILES : 0u);
  if (best_ms) *best_ms = best;
  if (use_cache) {
    std::ofstream o(path, std::ios::app);
    if (o) o << key << " " << bt << " " << bb << " " << bx << " " << best << "\n";
  }
  return GSR_OK;
}

gsr_status gsr_seed_settings_default(gsr_seed_settings* s) {
  if (!s) return fail(nullptr, GSR_EINVAL, "settings is NULL");
  s->measure = GSR_SEED_CONTRAST;
  s->threshold = 0.1f;
  s->min_side = 4;
  s->opacity = 0.5f;
  s->sh_degree = 0;
  return GSR_OK;
}

gsr_status gsr_seed(gsr_ctx* ctx, const gsr_camera* cam, const float* rgb, const float* depth,
                    const gsr_seed_settings* s, const gsr_tsdf* map, const gsr_seed_out* out, int64_t capacity,
                    int64_t* count) {
  if (!ctx) return fail(nullptr, GSR_EINVAL, "ctx is NULL");
  if (!cam || !rgb || !depth || !s || !out || !count) return fail(ctx, GSR_EINVAL, "NULL argument to gsr_seed");
  gsr_status st = check_camera(ctx, *cam, 0);
  if (st != GSR_OK) return st;
  std::string err;
  if ((st = check::seed_settings(s, capacity, out, err)) != GSR_OK) return fail(ctx, st, err);
  *count = 0;
  SeedImage im{rgb, depth, cam->width, cam->height, cam->fx, cam->fy, cam->cx, cam->cy, {}, {}};
  std::memcpy(im.R, cam->R, sizeof im.R);
  std::memcpy(im.t, cam->t, sizeof im.t);
  if (map && map->ctx != ctx) return fail(ctx, GSR_EINVAL, "the map belongs to another context");
  const SeedRules rules{s->measure, s->threshold, s->min_side, s->opacity, s->sh_degree, map ? 1 : 0,
                        map ? map->dev : TsdfDev{}};
  const SeedOut so{out->means, out->scales, out->quats, out->opacities, out->sh, out->leaves, capacity};
  const int roots = seed_roots(cam->width, cam->height);
  hipStream_t strm = ctx->stream;
  // per-root counts, then the 8-byte total at the next 8-byte boundary
  const size_t total_at = (size_t(roots) * 4 + 7) & ~size_t(7);
  void* buf = nullptr;
  if ((st = dev_alloc(ctx, strm, &buf, total_at + 8)) != GSR_OK) return st;
  uint32_t* counts = static_cast<uint32_t*>(buf);
  auto* total = reinterpret_cast<unsigned long long*>(static_cast<char*>(buf) + total_at);
  hipError_t e = launch_seed_count(im, rules, counts, strm);
  if (e == hipSuccess) e = launch_scan_small(counts, roots, total, strm);
  if (e == hipSuccess) e = hipMemcpyAsync(ctx->h_total, total, sizeof(unsigned long long), hipMemcpyDeviceToHost, strm);
  if (e == hipSuccess) e = hipStreamSynchronize(strm);
  const int64_t n = int64_t(ctx->h_total[0]);
  bool over = false;
  if (e == hipSuccess) {
    over = n > capacity;
    if (!over && n > 0) e = launch_seed_emit(im, rules, counts, so, strm);
  }
  dev_free(ctx, buf, strm);
  if (e != hipSuccess) return fail(ctx, GSR_EDEVICE, std::string("seeding failed: ") + hipGetErrorString(e));
  *count = n;
  if (over) return fail(ctx, GSR_ECAPACITY, "seeding needs " + std::to_string(n) + " Gaussians, capacity is " +
                                                std::to_string(capacity));
  return GSR_OK;
}

// ------------------------------------------------------------------------------------
// TSDF map
// ------------------------------------------------------------------------------------
gsr_status gsr_tsdf_settings_default(gsr_tsdf_settings* s) {
  if (!s) return fail(nullptr, GSR_EINVAL, "NULL argument to gsr_tsdf_settings_default");
  *s = gsr_tsdf_settings{0.01f, 0.08f, 100.f, 0.01f, GSR_TSDF_EQ9};
  return GSR_OK;
}

static void tsdf_release(gsr_tsdf* m) {
  for (void* p : m->blocks) dev_free(m->ctx, p, m->ctx->stream);
  (void)hipStreamSynchronize(m->ctx->stream);
  delete m;
}

gsr_status gsr_tsdf_create(gsr_ctx* ctx, const gsr_tsdf_settings* s, int64_t max_blocks, gsr_tsdf** out) {
  if (!ctx) return fail(nullptr, GSR_EINVAL, "ctx is NULL");
  if (!s || !out) return fail(ctx, GSR_EINVAL, "NULL argument to gsr_tsdf_create");
  *out = nullptr;
  std::string err;
  int64_t slots = 0;
  if (check::tsdf_settings(s, max_blocks, &slots, err) != GSR_OK) return fail(ctx, GSR_EINVAL, err);
  const int n_samples = tsdf_band_samples(s->trunc, s->step);
  if (n_samples > 4096) return fail(ctx, GSR_EINVAL, "more than 4096 band samples per pixel");
  gsr_tsdf* m = new gsr_tsdf;
  m->ctx = ctx;
  m->s = *s;
  m->ru = TsdfRules{s->trunc, s->step, s->w_max, n_samples, s->weighting == GSR_TSDF_UNIT_WEIGHT ? 1 : 0};
  TsdfDev& d = m->dev;
  d.slot_mask = uint32_t(slots - 1);
  d.cap_blocks = uint32_t(max_blocks);
  d.voxel = s->voxel;
  hipStream_t strm = ctx->stream;
  gsr_status st = GSR_OK;
  auto get = [&](void** p, size_t bytes) {
    if (st != GSR_OK) return;
    st = dev_alloc(ctx, strm, p, bytes);
    if (st == GSR_OK) m->blocks.push_back(*p);
  };
  const size_t vox = size_t(max_blocks) * kBlockVoxels;
  get(reinterpret_cast<void**>(&d.keys), size_t(slots) * 8);
  get(reinterpret_cast<void**>(&d.vals), size_t(slots) * 4);
  get(reinterpret_cast<void**>(&d.stamp), size_t(slots) * 4);
  get(reinterpret_cast<void**>(&d.tsdf), vox * 4);
  get(reinterpret_cast<void**>(&d.weight), vox * 4);
  get(reinterpret_cast<void**>(&d.coords), size_t(max_blocks) * sizeof(int4));
  get(reinterpret_cast<void**>(&d.ctrl), TSDF_CTRL_WORDS * 4);
  if (st != GSR_OK) {
    tsdf_release(m);
    return st;
  }
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(d.keys), 0xFFFFFFFFu, slots * 2, strm);
  if (e == hipSuccess) e = launch_fill_u32(d.vals, kUnassigned, slots, strm);
  if (e == hipSuccess) e = launch_fill_u32(d.stamp, 0xFFFFFFFFu, slots, strm);
  if (e == hipSuccess) e = launch_fill_u32(reinterpret_cast<uint32_t*>(d.tsdf), 0u, int64_t(vox), strm);
  if (e == hipSuccess) e = launch_fill_u32(reinterpret_cast<uint32_t*>(d.weight), 0u, int64_t(vox), strm);
  if (e == hipSuccess) e = launch_fill_u32(d.ctrl, 0u, TSDF_CTRL_WORDS, strm);
  if (e != hipSuccess) {
    tsdf_release(m);
    return fail(ctx, GSR_EDEVICE, std::string("map set-up failed: ") + hipGetErrorString(e));
  }
  *out = m;
  return GSR_OK;
}

gsr_status gsr_tsdf_free(gsr_tsdf* m) {
  if (!m) return fail(nullptr, GSR_EINVAL, "map is NULL");
  tsdf_release(m);
  return GSR_OK;
}

gsr_status gsr_tsdf_integrate(gsr_ctx* ctx, gsr_tsdf* m, const gsr_camera* cam, const float* depth) {
  if (!ctx) return fail(nullptr, GSR_EINVAL, "ctx is NULL");
  if (!m || !cam || !depth) return fail(ctx, GSR_EINVAL, "NULL argument to gsr_tsdf_integrate");
  if (m->ctx != ctx) return fail(ctx, GSR_EINVAL, "the map belongs to another context");
  gsr_status st = check_camera(ctx, *cam, 0);
  if (st != GSR_OK) return st;
  TsdfCam c{};
  std::memcpy(c.R, cam->R, sizeof c.R);
  std::memcpy(c.t, cam->t, sizeof c.t);
  c.fx = cam->fx;
  c.fy = cam->fy;
  c.cx = cam->cx;
  c.cy = cam->cy;
  c.W = cam->width;
  c.H = cam->height;
  hipStream_t strm = ctx->stream;
  GSR_HIP(ctx, timed(ctx, strm, K_TSDF_ALLOC, [&] { return launch_tsdf_alloc(depth, c, m->dev, m->ru, m->frame, strm); }));
  GSR_HIP(ctx, timed(ctx, strm, K_TSDF_FUSE, [&] { return launch_tsdf_fuse(depth, c, m->dev, m->ru, m->frame, strm); }));
  ++m->frame;
  if (m->frame == 0xFFFFFFFFu) m->frame = 0;  // never the value that marks an unstamped slot
  return GSR_OK;
}

gsr_status gsr_tsdf_info(gsr_ctx* ctx, const gsr_tsdf* m, int64_t* blocks, int64_t* met_last, uint32_t* flags) {
  if (!ctx) return fail(nullptr, GSR_EINVAL, "ctx is NULL");
  if (!m) return fail(ctx, GSR_EINVAL, "map is NULL");
  uint32_t w[TSDF_CTRL_WORDS];
  GSR_HIP(ctx, hipMemcpyAsync(w, m->dev.ctrl, sizeof w, hipMemcpyDeviceToHost, ctx->stream));
  GSR_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (blocks) *blocks = std::min<int64_t>(w[TSDF_ALLOCATED], m->dev.cap_blocks);
  if (met_last) *met_last = w[TSDF_MET];
  if (flags) *flags = w[TSDF_FLAGS];
  return GSR_OK;
}

gsr_status gsr_tsdf_export(gsr_ctx* ctx, const gsr_tsdf* m, int32_t* coords, float* tsdf, float* weight,
                           int64_t capacity, int64_t* count) {
  if (!ctx) return fail(nullptr, GSR_EINVAL, "ctx is NULL");
  if (!m || !count) return fail(ctx, GSR_EINVAL, "NULL argument to gsr_tsdf_export");
  int64_t n = 0;
  gsr_status st = gsr_tsdf_info(ctx, m, &n, nullptr, nullptr);
  if (st != GSR_OK) return st;
  *count = n;
  if (!coords && !tsdf && !weight) return GSR_OK;
  if (capacity < n) return fail(ctx, GSR_ECAPACITY, "export needs room for " + std::to_string(n) + " blocks");
  hipStream_t strm = ctx->stream;
  if (coords && n > 0) {
    std::vector<int4> c(static_cast<size_t>(n));
    GSR_HIP(ctx, hipMemcpyAsync(c.data(), m->dev.coords, size_t(n) * sizeof(int4), hipMemcpyDeviceToHost, strm));
    GSR_HIP(ctx, hipStreamSynchronize(strm));
    for (int64_t i = 0; i < n; ++i) {
      coords[i * 3] = c[size_t(i)].x;
      coords[i * 3 + 1] = c[size_t(i)].y;
      coords[i * 3 + 2] = c[size_t(i)].z;
    }
  }
  const size_t vb = size_t(n) * kBlockVoxels * sizeof(float);
  if (tsdf && n > 0) GSR_HIP(ctx, hipMemcpyAsync(tsdf, m->dev.tsdf, vb, hipMemcpyDeviceToHost, strm));
  if (weight && n > 0) GSR_HIP(ctx, hipMemcpyAsync(weight, m->dev.weight, vb, hipMemcpyDeviceToHost, strm));
  GSR_HIP(ctx, hipStreamSynchronize(strm));
  return GSR_OK;
}

gsr_status gsr_tsdf_weights(gsr_ctx* ctx, const gsr_tsdf* m, const float* points, int64_t n, float* out) {
  if (!ctx) return fail(nullptr, GSR_EINVAL, "ctx is NULL");
  if (!m || (n > 0 && (!points || !out)) || n < 0) return fail(ctx, GSR_EINVAL, "bad argument to gsr_tsdf_weights");
  GSR_HIP(ctx, launch_tsdf_weights(m->dev, points, n, out, ctx->stream));
  return GSR_OK;
}

}  // extern "C"
