// Host side of the C ABI declared in gsr.h: argument validation, scratch memory from the
// device's stream-ordered pool, and the launch sequences of the forward, loss and backward
// passes.  All device work goes to the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gsr_internal.h"

using namespace gsr;

struct gsr_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  unsigned long long* h_total = nullptr;  // pinned read-back slots: pair count M, visible records
  Timer timer;
};

namespace {
const char* const kKernelNames[K_COUNT] = {
    "project", "scan",   "compact", "sorted_counts", "duplicate", "radix_hist", "radix_rowscan", "radix_scatter",
    "ranges",  "fill",   "blend_fwd", "loss_l1",     "blend_bwd", "project_bwd"};

// Wraps one launch (or launch sequence) in the context's optional event timer.
template <class F>
hipError_t timed(gsr_ctx* ctx, int k, F&& f) {
  ctx->timer.stream = ctx->stream;
  ctx->timer.begin(k);
  hipError_t e = f();
  ctx->timer.end(k);
  return e;
}
}  // namespace

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
  int64_t M = 0;
  int64_t n_vis = 0;
  uint32_t* tiles = nullptr;  // sorted tile id of every pair
  uint32_t* vals = nullptr;   // sorted record id of every pair
  uint2* ranges = nullptr;
  float* T_final = nullptr;
  uint32_t* n_contrib = nullptr;
  int64_t total_pix = 0;
  int sort_passes = 0;
  std::vector<void*> blocks;  // every allocation, released on free
};

namespace {

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

gsr_status dev_alloc(gsr_ctx* ctx, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return GSR_OK;
  hipError_t e = hipMallocAsync(p, bytes, ctx->stream);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(ctx, GSR_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed: " +
                                     hipGetErrorString(e));
  }
  return GSR_OK;
}

template <class T>
gsr_status saved_alloc(gsr_saved* sv, T** p, size_t count) {
  void* q = nullptr;
  gsr_status st = dev_alloc(sv->ctx, &q, count * sizeof(T));
  if (st != GSR_OK) return st;
  if (q) sv->blocks.push_back(q);
  *p = static_cast<T*>(q);
  return GSR_OK;
}

void release(gsr_saved* sv) {
  if (!sv) return;
  for (void* p : sv->blocks) (void)hipFreeAsync(p, sv->ctx->stream);
  sv->blocks.clear();
  delete sv;
}

gsr_status check_settings(gsr_ctx* ctx, const gsr_settings* s) {
  if (!s) return fail(ctx, GSR_EINVAL, "settings is NULL");
  if (s->tile != 8 && s->tile != 16 && s->tile != 32) return fail(ctx, GSR_EINVAL, "tile must be 8, 16 or 32");
  if (s->batch != 128 && s->batch != 256) return fail(ctx, GSR_EINVAL, "batch must be 128 or 256");
  if (!(s->extent_k > 0.f) || !(s->lowpass >= 0.f) || !(s->alpha_min >= 0.f) || !(s->alpha_max > 0.f) ||
      !(s->alpha_max < 1.f) || !(s->T_min >= 0.f) || !(s->T_min < 1.f) || !(s->guard >= 0.f))
    return fail(ctx, GSR_EINVAL, "rule value out of range");
  if (s->flags != 0) return fail(ctx, GSR_EINVAL, "settings.flags must be 0");
  return GSR_OK;
}

gsr_status check_gaussians(gsr_ctx* ctx, const gsr_gaussians* g, int V) {
  if (!g) return fail(ctx, GSR_EINVAL, "gaussians is NULL");
  if (g->n < 0) return fail(ctx, GSR_EINVAL, "gaussians.n < 0");
  if (g->sh_degree < 0 || g->sh_degree > 3) return fail(ctx, GSR_EINVAL, "sh_degree must be 0..3");
  if (g->n > 0 && (!g->means || !g->scales || !g->quats || !g->opacities || !g->sh))
    return fail(ctx, GSR_EINVAL, "a Gaussian parameter pointer is NULL");
  if (g->n > 0 && (reinterpret_cast<uintptr_t>(g->quats) & 15u))
    return fail(ctx, GSR_EINVAL, "quats must be 16-byte aligned");
  if (int64_t(V) * g->n >= (int64_t(1) << 32)) return fail(ctx, GSR_EINVAL, "views * Gaussians must be < 2^32");
  return GSR_OK;
}

gsr_status check_camera(gsr_ctx* ctx, const gsr_camera& c, int v) {
  const std::string at = " (view " + std::to_string(v) + ")";
  if (c.width < 1 || c.height < 1 || c.width > 8192 || c.height > 8192)
    return fail(ctx, GSR_EINVAL, "camera size must be 1..8192" + at);
  if (!(c.fx > 0.f) || !(c.fy > 0.f) || !std::isfinite(c.cx) || !std::isfinite(c.cy))
    return fail(ctx, GSR_EINVAL, "camera intrinsics invalid" + at);
  if (!(c.znear > 0.f)) return fail(ctx, GSR_EINVAL, "camera znear must be > 0" + at);
  return GSR_OK;
}

int bits_for(uint64_t maxval) {
  int b = 0;
  while (b < 64 && (maxval >> b) != 0) ++b;
  return b;
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
  return GSR_OK;
}

const char* gsr_last_error(const gsr_ctx* ctx) { return ctx ? ctx->err.c_str() : g_noctx_err.c_str(); }

gsr_status gsr_ctx_create(int32_t device, void* hip_stream, gsr_ctx** out) {
  if (!out) return fail(nullptr, GSR_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    return fail(nullptr, GSR_EDEVICE, "no HIP device available");
  }
  if (device < 0 || device >= ndev) return fail(nullptr, GSR_EINVAL, "device index out of range");
  if (hipSetDevice(device) != hipSuccess) return fail(nullptr, GSR_EDEVICE, "hipSetDevice failed");
  gsr_ctx* c = new gsr_ctx;
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
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
  if (V < 1 || V > GSR_MAX_VIEWS) return fail(ctx, GSR_EINVAL, "V must be 1..16");
  if (!cams || !outs) return fail(ctx, GSR_EINVAL, "cams/outs is NULL");
  gsr_status st;
  if ((st = check_settings(ctx, s)) != GSR_OK) return st;
  if ((st = check_gaussians(ctx, g, V)) != GSR_OK) return st;
  for (int v = 0; v < V; ++v) {
    if ((st = check_camera(ctx, cams[v], v)) != GSR_OK) return st;
    if (!outs[v].color) return fail(ctx, GSR_EINVAL, "outs[v].color is NULL");
  }
  ctx->err.clear();

  gsr_saved* sv = new gsr_saved;
  sv->ctx = ctx;
  sv->V = V;
  sv->N = g->n;
  sv->deg = g->sh_degree;
  sv->s = *s;
  sv->g = GaussDev{g->means, g->scales, g->quats, g->opacities, g->sh, g->n};
  sv->ru = Rules{s->extent_k, s->lowpass,  s->alpha_min, s->alpha_max,
                 s->T_min,    s->guard,    {s->bg[0], s->bg[1], s->bg[2]}};
  ViewTable& vt = sv->vt;
  std::memset(&vt, 0, sizeof(vt));
  vt.nviews = V;
  int64_t tiles = 0, pix = 0;
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
    d.pix_off = pix;
    d.color = outs[v].color;
    d.depth = outs[v].depth;
    d.alpha = outs[v].alpha;
    tiles += int64_t(d.tiles_x) * d.tiles_y;
    pix += int64_t(c.width) * c.height;
  }
  vt.total_tiles = int32_t(tiles);
  sv->total_pix = pix;
  const int64_t VN = int64_t(V) * g->n;
  sv->nblk = int((g->n + kProjThreads - 1) / kProjThreads);
  hipStream_t st_ = ctx->stream;

#define TRY(x)             \
  do {                     \
    gsr_status t_ = (x);   \
    if (t_ != GSR_OK) {    \
      release(sv);         \
      return t_;           \
    }                      \
  } while (0)
#define TRYH(x)                                                                                    \
  do {                                                                                             \
    hipError_t e_ = (x);                                                                           \
    if (e_ != hipSuccess) {                                                                        \
      release(sv);                                                                                 \
      return fail(ctx, GSR_EDEVICE, std::string(#x ": ") + hipGetErrorString(e_));                 \
    }                                                                                              \
  } while (0)

  TRY(saved_alloc(sv, &sv->rec.r0, VN));
  TRY(saved_alloc(sv, &sv->rec.r1, VN));
  TRY(saved_alloc(sv, &sv->rec.rgb, VN));
  TRY(saved_alloc(sv, &sv->rec.rect, VN));
  TRY(saved_alloc(sv, &sv->rec.counts, VN));
  TRY(saved_alloc(sv, &sv->blocksums, size_t(V) * sv->nblk + 1));
  TRY(saved_alloc(sv, &sv->d_total, 4));
  TRY(saved_alloc(sv, &sv->ranges, size_t(tiles)));
  TRY(saved_alloc(sv, &sv->T_final, size_t(pix)));
  TRY(saved_alloc(sv, &sv->n_contrib, size_t(pix)));

  int64_t M = 0, NV = 0;
  if (g->n > 0) {
    TRYH(timed(ctx, K_PROJECT, [&] {
      return launch_project(sv->deg, sv->g, vt, sv->ru, s->tile, sv->rec, sv->blocksums, sv->nblk, st_);
    }));
    TRYH(timed(ctx, K_SCAN, [&] { return launch_scan_pairs(sv->blocksums, V * sv->nblk, sv->d_total, st_); }));
    TRYH(hipMemcpyAsync(ctx->h_total, sv->d_total, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st_));
    TRYH(hipStreamSynchronize(st_));
    M = int64_t(ctx->h_total[0]);
    NV = int64_t(ctx->h_total[1]);
    if (M >= (int64_t(1) << 32)) {
      release(sv);
      return fail(ctx, GSR_ECAPACITY, "more than 2^32 duplicated keys");
    }
  }
  sv->M = M;
  sv->n_vis = NV;
  if (M > 0) {
    // Stable LSD sort of the (tile << 32 | depth) keys: the depth digits on the NV records,
    // then duplication in depth order, then the tile digits on the M pairs.
    uint32_t *tk = nullptr, *tv = nullptr;
    TRY(saved_alloc(sv, &tk, size_t(M)));
    TRY(saved_alloc(sv, &tv, size_t(M)));
    const int tile_bits = bits_for(uint64_t(tiles > 0 ? tiles - 1 : 0));
    const int64_t sort_cap = std::max(NV, M);
    const int nb_sort = int((sort_cap + kSortTile - 1) / kSortTile);
    const int nb_vis = int((NV + kProjThreads - 1) / kProjThreads);
    std::vector<void*> tmp;
    auto tmp_alloc = [&](void** p, size_t bytes) -> gsr_status {
      gsr_status r = dev_alloc(ctx, p, bytes);
      if (r == GSR_OK && *p) tmp.push_back(*p);
      return r;
    };
    auto free_tmp = [&]() {
      for (void* p : tmp) (void)hipFreeAsync(p, st_);
      tmp.clear();
    };
    void *dk = nullptr, *dv = nullptr, *dk2 = nullptr, *dv2 = nullptr, *tk2 = nullptr, *tv2 = nullptr;
    void *hist = nullptr, *dtot = nullptr, *bs2 = nullptr, *ovf = nullptr;
    gsr_status a = GSR_OK;
    if ((a = tmp_alloc(&dk, size_t(NV) * 4)) != GSR_OK || (a = tmp_alloc(&dv, size_t(NV) * 4)) != GSR_OK ||
        (a = tmp_alloc(&dk2, size_t(NV) * 4)) != GSR_OK || (a = tmp_alloc(&dv2, size_t(NV) * 4)) != GSR_OK ||
        (a = tmp_alloc(&tk2, size_t(M) * 4)) != GSR_OK || (a = tmp_alloc(&tv2, size_t(M) * 4)) != GSR_OK ||
        (a = tmp_alloc(&hist, size_t(nb_sort) * 256 * 4)) != GSR_OK ||
        (a = tmp_alloc(&dtot, 256 * 4)) != GSR_OK || (a = tmp_alloc(&bs2, size_t(nb_vis + 1) * 4)) != GSR_OK ||
        (a = tmp_alloc(&ovf, 4)) != GSR_OK) {
      free_tmp();
      release(sv);
      return a;
    }
    Timer* tm = ctx->timer.on ? &ctx->timer : nullptr;
    ctx->timer.stream = st_;
    bool alt1 = false, alt2 = false;
    int p1 = 0, p2 = 0;
    hipError_t e = timed(ctx, K_FILL, [&] { return launch_fill_u32(static_cast<uint32_t*>(ovf), 0u, 1, st_); });
    if (e == hipSuccess)
      e = timed(ctx, K_COMPACT, [&] {
        return launch_compact(g->n, V, sv->rec, sv->blocksums, sv->nblk, static_cast<uint32_t*>(dk),
                              static_cast<uint32_t*>(dv), st_);
      });
    if (e == hipSuccess)
      e = launch_radix_sort(static_cast<uint32_t*>(dk), static_cast<uint32_t*>(dv), static_cast<uint32_t*>(dk2),
                            static_cast<uint32_t*>(dv2), static_cast<uint32_t*>(hist), static_cast<uint32_t*>(dtot),
                            sv->d_total + 1, NV, 32, &alt1, &p1, st_, tm);
    const uint32_t* dsorted = static_cast<const uint32_t*>(alt1 ? dv2 : dv);
    if (e == hipSuccess)
      e = launch_duplicate(vt, g->n, sv->rec, dsorted, sv->d_total + 1, NV, static_cast<uint32_t*>(bs2),
                           sv->d_total + 2, tk, tv, M, static_cast<uint32_t*>(ovf), st_, tm);
    if (e == hipSuccess)
      e = launch_radix_sort(tk, tv, static_cast<uint32_t*>(tk2), static_cast<uint32_t*>(tv2),
                            static_cast<uint32_t*>(hist), static_cast<uint32_t*>(dtot), sv->d_total, M, tile_bits,
                            &alt2, &p2, st_, tm);
    if (e != hipSuccess) {
      free_tmp();
      release(sv);
      return fail(ctx, GSR_EDEVICE, std::string("sort launch failed: ") + hipGetErrorString(e));
    }
    if (alt2) {  // the sorted pairs ended in the second buffers: keep those, recycle the first
      std::replace(sv->blocks.begin(), sv->blocks.end(), static_cast<void*>(tk), tk2);
      std::replace(sv->blocks.begin(), sv->blocks.end(), static_cast<void*>(tv), tv2);
      std::replace(tmp.begin(), tmp.end(), tk2, static_cast<void*>(tk));
      std::replace(tmp.begin(), tmp.end(), tv2, static_cast<void*>(tv));
      tk = static_cast<uint32_t*>(tk2);
      tv = static_cast<uint32_t*>(tv2);
    }
    sv->tiles = tk;
    sv->vals = tv;
    sv->sort_passes = p1 + p2;
    free_tmp();
  }
  TRYH(timed(ctx, K_RANGES,
             [&] { return launch_ranges(sv->tiles, sv->d_total, M, sv->ranges, vt.total_tiles, st_); }));
  TRYH(timed(ctx, K_BLEND_FWD, [&] {
    return launch_blend_fwd(s->tile, s->batch, vt, sv->ru, sv->rec, sv->ranges, sv->vals, sv->T_final,
                            sv->n_contrib, st_);
  }));
#undef TRY
#undef TRYH
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
  if (!(depth_weight >= 0.f)) return fail(ctx, GSR_EINVAL, "depth_weight must be >= 0");
  ViewTable vt = saved->vt;
  for (int v = 0; v < vt.nviews; ++v) {
    if (!outs[v].color || !targets[v].color || !grad_color_out[v])
      return fail(ctx, GSR_EINVAL, "colour image, target or gradient pointer is NULL");
    if (targets[v].depth && (!outs[v].depth || !grad_depth_out || !grad_depth_out[v]))
      return fail(ctx, GSR_EINVAL, "depth target given without rendered depth / gradient buffer");
    vt.v[v].color = outs[v].color;
    vt.v[v].depth = outs[v].depth;
    vt.v[v].t_color = targets[v].color;
    vt.v[v].t_depth = targets[v].depth;
    vt.v[v].lg_color = grad_color_out[v];
    vt.v[v].lg_depth = grad_depth_out ? grad_depth_out[v] : nullptr;
  }
  GSR_HIP(ctx, timed(ctx, K_LOSS, [&] { return launch_loss_l1(vt, depth_weight, loss_dev, ctx->stream); }));
  return GSR_OK;
}

gsr_status gsr_backward(gsr_ctx* ctx, const gsr_saved* saved, const gsr_view_grad* grads,
                        const gsr_gaussian_grads* out, uint32_t flags) {
  if (!ctx) return fail(nullptr, GSR_EINVAL, "ctx is NULL");
  if (!saved || !grads || !out) return fail(ctx, GSR_EINVAL, "NULL argument to gsr_backward");
  if (flags & ~GSR_ACCUMULATE) return fail(ctx, GSR_EINVAL, "unknown flag");
  ViewTable vt = saved->vt;
  for (int v = 0; v < vt.nviews; ++v) {
    vt.v[v].g_color = grads[v].color;
    vt.v[v].g_depth = grads[v].depth;
    vt.v[v].g_alpha = grads[v].alpha;
  }
  const int64_t VN = int64_t(saved->V) * saved->N;
  void* g2 = nullptr;
  gsr_status st = dev_alloc(ctx, &g2, size_t(VN) * kGrad2D * sizeof(float));
  if (st != GSR_OK) return st;
  float* grad2d = static_cast<float*>(g2);
  hipStream_t s = ctx->stream;
  hipError_t e =
      timed(ctx, K_FILL, [&] { return launch_fill_u32(reinterpret_cast<uint32_t*>(grad2d), 0u, VN * kGrad2D, s); });
  if (e == hipSuccess)
    e = timed(ctx, K_BLEND_BWD, [&] {
      return launch_blend_bwd(saved->s.tile, saved->s.batch, vt, saved->ru, saved->rec, saved->ranges,
                              saved->vals, saved->T_final, saved->n_contrib, grad2d, s);
    });
  GradOut go{out->means, out->scales, out->quats, out->opacities, out->sh, int(flags & GSR_ACCUMULATE)};
  if (e == hipSuccess)
    e = timed(ctx, K_PROJECT_BWD,
              [&] { return launch_project_bwd(saved->deg, saved->g, vt, saved->ru, saved->rec, grad2d, go, s); });
  if (g2) (void)hipFreeAsync(g2, s);
  if (e != hipSuccess) return fail(ctx, GSR_EDEVICE, std::string("backward launch failed: ") + hipGetErrorString(e));
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
    std::vector<uint32_t> t(sv->M), v(sv->M);
    std::vector<float4> r1(VN);
    GSR_HIP(ctx, cp(t.data(), sv->tiles, size_t(sv->M) * 4));
    GSR_HIP(ctx, cp(v.data(), sv->vals, size_t(sv->M) * 4));
    GSR_HIP(ctx, cp(r1.data(), sv->rec.r1, size_t(VN) * sizeof(float4)));
    for (int64_t i = 0; i < sv->M; ++i) {
      uint32_t zb;
      std::memcpy(&zb, &r1[v[i]].z, 4);
      out->keys[i] = (uint64_t(t[i]) << 32) | zb;
    }
  }
  GSR_HIP(ctx, cp(out->values, sv->vals, size_t(sv->M) * 4));
  GSR_HIP(ctx, cp(out->ranges, sv->ranges, size_t(sv->vt.total_tiles) * 8));
  GSR_HIP(ctx, cp(out->T_final, sv->T_final, size_t(sv->total_pix) * 4));
  GSR_HIP(ctx, cp(out->n_contrib, sv->n_contrib, size_t(sv->total_pix) * 4));
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

}  // extern "C"
