// Argument validation of the C ABI (declarations and contract in gsr_validate.h).
#include "gsr_validate.h"

#include <cmath>
#include <cstdint>

namespace gsr {
namespace check {
namespace {

gsr_status bad(std::string& err, const std::string& msg) {
  err = msg;
  return GSR_EINVAL;
}

bool finite_nonneg(float x) { return x >= 0.f && std::isfinite(x); }

}  // namespace

gsr_status settings(const gsr_settings* s, std::string& err) {
  if (!s) return bad(err, "settings is NULL");
  if (s->tile != 8 && s->tile != 16 && s->tile != 32) return bad(err, "tile must be 8, 16 or 32");
  if (s->batch != 128 && s->batch != 256) return bad(err, "batch must be 128 or 256");
  if (!(s->extent_k > 0.f) || !(s->lowpass >= 0.f) || !(s->alpha_min >= 0.f) || !(s->alpha_max > 0.f) ||
      !(s->alpha_max < 1.f) || !(s->T_min >= 0.f) || !(s->T_min < 1.f) || !(s->guard >= 0.f))
    return bad(err, "rule value out of range");
  if (!std::isfinite(s->extent_k) || !std::isfinite(s->lowpass) || !std::isfinite(s->guard))
    return bad(err, "rule value not finite");
  if (!(s->jclamp >= 0.f) || !std::isfinite(s->jclamp)) return bad(err, "jclamp must be finite and >= 0");
  if (s->flags & ~(GSR_EXACT_TILES | GSR_NORMALIZED_DEPTH | GSR_CHECK_FINITE)) return bad(err, "unknown settings flag");
  return GSR_OK;
}

gsr_status gaussians(const gsr_gaussians* g, int views, std::string& err) {
  if (!g) return bad(err, "gaussians is NULL");
  if (g->n < 0) return bad(err, "gaussians.n < 0");
  if (g->sh_degree < 0 || g->sh_degree > 3) return bad(err, "sh_degree must be 0..3");
  if (g->n > 0 && (!g->means || !g->scales || !g->quats || !g->opacities || !g->sh))
    return bad(err, "a Gaussian parameter pointer is NULL");
  if (g->n > 0 && (reinterpret_cast<uintptr_t>(g->quats) & 15u)) return bad(err, "quats must be 16-byte aligned");
  // record ids v * N + g are 32-bit
  if (g->n >= (int64_t(1) << 32) || int64_t(views) * g->n >= (int64_t(1) << 32))
    return bad(err, "views * Gaussians must be < 2^32");
  return GSR_OK;
}

gsr_status camera(const gsr_camera& c, int view, std::string& err) {
  const std::string at = " (view " + std::to_string(view) + ")";
  if (c.width < 1 || c.height < 1 || c.width > 8192 || c.height > 8192)
    return bad(err, "camera size must be 1..8192" + at);
  if (!(c.fx > 0.f) || !(c.fy > 0.f) || !std::isfinite(c.fx) || !std::isfinite(c.fy) || !std::isfinite(c.cx) ||
      !std::isfinite(c.cy))
    return bad(err, "camera intrinsics invalid" + at);
  if (!(c.znear > 0.f) || !std::isfinite(c.znear)) return bad(err, "camera znear must be > 0" + at);
  for (float x : c.R)
    if (!std::isfinite(x)) return bad(err, "camera rotation not finite" + at);
  for (float x : c.t)
    if (!std::isfinite(x)) return bad(err, "camera translation not finite" + at);
  return GSR_OK;
}

gsr_status forward_args(const gsr_gaussians* g, const gsr_camera* cams, int32_t V, const gsr_settings* s,
                        const gsr_view_out* outs, std::string& err) {
  if (V < 1 || V > GSR_MAX_VIEWS) return bad(err, "V must be 1..16");
  if (!cams || !outs) return bad(err, "cams/outs is NULL");
  gsr_status st;
  if ((st = settings(s, err)) != GSR_OK) return st;
  if ((st = gaussians(g, V, err)) != GSR_OK) return st;
  for (int v = 0; v < V; ++v) {
    if ((st = camera(cams[v], v, err)) != GSR_OK) return st;
    if (!outs[v].color) return bad(err, "outs[" + std::to_string(v) + "].color is NULL");
  }
  return GSR_OK;
}

gsr_status adam(const gsr_adam* o, std::string& err) {
  if (!o) return bad(err, "optimiser is NULL");
  const gsr_gaussian_grads* mv[2] = {&o->m, &o->v};
  for (const gsr_gaussian_grads* x : mv)
    if (!x->means || !x->scales || !x->quats || !x->opacities || !x->sh)
      return bad(err, "every optimiser moment array is required");
  if (!o->state) return bad(err, "optimiser state is NULL");
  const float lr[6] = {o->lr_means, o->lr_scales, o->lr_quats, o->lr_opacities, o->lr_sh_dc, o->lr_sh_rest};
  for (float r : lr)
    if (!finite_nonneg(r)) return bad(err, "learning rates must be finite and >= 0");
  if (!(o->beta1 >= 0.f && o->beta1 < 1.f) || !(o->beta2 >= 0.f && o->beta2 < 1.f))
    return bad(err, "betas must be in [0, 1)");
  if (!finite_nonneg(o->eps)) return bad(err, "eps must be finite and >= 0");
  return GSR_OK;
}

gsr_status seed_settings(const gsr_seed_settings* s, int64_t capacity, const gsr_seed_out* out, std::string& err) {
  if (!s || !out) return bad(err, "seed settings or output is NULL");
  if (s->measure != GSR_SEED_CONTRAST && s->measure != GSR_SEED_DEPTH_VARIANCE) return bad(err, "unknown seeding measure");
  const int ms = s->min_side;
  if (ms != 1 && ms != 2 && ms != 4 && ms != 8 && ms != 16 && ms != 32 && ms != 64)
    return bad(err, "min_side must be a power of two in 1..64");
  if (!(s->threshold >= 0.f) || !(s->opacity >= 0.f && s->opacity <= 1.f))
    return bad(err, "threshold or opacity out of range");
  if (s->sh_degree < 0 || s->sh_degree > 3) return bad(err, "sh_degree must be 0..3");
  if (capacity < 0) return bad(err, "capacity < 0");
  if (capacity > 0 && (!out->means || !out->scales || !out->quats || !out->opacities || !out->sh))
    return bad(err, "an output pointer is NULL");
  return GSR_OK;
}

gsr_status tsdf_settings(const gsr_tsdf_settings* s, int64_t max_blocks, int64_t* slots, std::string& err) {
  if (!s || !slots) return bad(err, "TSDF settings is NULL");
  if (!(s->voxel > 0.f) || !(s->trunc > 0.f) || !(s->step > 0.f) || !(s->w_max >= 1.f) || !std::isfinite(s->voxel) ||
      !std::isfinite(s->trunc) || !std::isfinite(s->step) || !std::isfinite(s->w_max))
    return bad(err, "voxel, trunc and step must be > 0 and w_max >= 1");
  if (s->weighting != GSR_TSDF_EQ9 && s->weighting != GSR_TSDF_UNIT_WEIGHT) return bad(err, "unknown weighting");
  if (max_blocks < 1 || max_blocks > (int64_t(1) << 28)) return bad(err, "max_blocks must be in 1..2^28");
  int64_t n = 1024;
  while (n < 2 * max_blocks) n *= 2;
  *slots = n;
  return GSR_OK;
}

}  // namespace check
}  // namespace gsr
