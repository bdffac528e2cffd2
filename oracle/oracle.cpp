// Plain, slow CPU reference of the tile-based differentiable Gaussian splatting
// rasterizer used by GSFusion's online optimisation (Sec. III-B-3, Eq. 3-5, 11-12).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
// calls this file; only the test-suite, the smoke check and the benchmark's
// CPU-baseline leg use it.  It shares no code with the HIP path.
//
// Two stages:
//  * a discrete stage (cull, splat centre, screen rectangle, tile keys) written
//    as a fixed sequence of IEEE binary32 operations, so that tile keys, sort
//    order and tile ranges are reproducible bit for bit by any other
//    implementation that performs the same sequence (no fused multiply-add,
//    correctly rounded divide and square root);
//  * a value stage in binary64: projected covariance (Eq. 5), conic, SH colour,
//    per-pixel front-to-back compositing (Eq. 11 with clamp/skip/stop rules)
//    and the exact reverse-mode gradients of all of it.
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -fno-fast-math -shared -fPIC
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <thread>
#include <unordered_map>
#include <vector>

extern "C" {

typedef struct {
  int32_t width, height;
  float fx, fy, cx, cy;
  float R[9];   // world->camera rotation, row-major
  float t[3];   // world->camera translation: x_c = R x_w + t
  float znear;
} or_camera;

typedef struct {
  int32_t tile;        // tile edge in pixels
  float extent_k;      // screen rectangle half-width in standard deviations
  float lowpass;       // added to the diagonal of the projected covariance (px^2)
  float alpha_min;     // a splat value below this is skipped
  float alpha_max;     // opacity clamp
  float T_min;         // stop once transmittance falls below this
  float guard;         // frustum guard band, as a fraction of the image size per side
  float bg[3];         // background colour
  int32_t mu_fp32;     // 1: value stage uses the binary32 splat centre and projected covariance
                       //    of the discrete stage (the conic is their binary64 inverse)
  int32_t threads;     // worker threads for the pixel loop (>=1)
  float amb_rel_a;     // relative margin around alpha_min that flags a skip decision as ambiguous
  float amb_rel_T;     // relative margin around T_min that flags a stop decision as ambiguous
  int32_t exact_tiles; // 1: a tile row keeps only the columns its ellipse can reach (row_run)
  int32_t normalized_depth;  // 1: the depth output is D / (1 - T_final) (0 where nothing is hit)
  int32_t window[4];   // pixels x0 <= x < x1, y0 <= y < y1 of every view are rendered and
                       // differentiated (outputs elsewhere untouched); x1 <= x0: every pixel
  float jclamp;        // > 0: inside the projection's Jacobian, x/z and y/z are clamped to
                       // +-jclamp times the half field of view, W / (2 fx) and H / (2 fy)
} or_settings;

}  // extern "C"

namespace {

constexpr double kPi = 3.14159265358979323846;

// ------------------------------------------------------------------------------------
// Real spherical harmonics from their definition (orthonormal, Condon-Shortley phase):
//   Y_l^0  = N_l^0 P_l^0(cos t)
//   Y_l^m  = sqrt2 N_l^m cos(m phi) P_l^m(cos t)      m > 0
//   Y_l^-m = sqrt2 N_l^m sin(m phi) P_l^m(cos t)      m > 0
//   N_l^m  = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!),  P_l^m(x) = (-1)^m (1-x^2)^(m/2) d^m/dx^m P_l(x)
// With (x,y,z) a unit vector, (1-z^2)^(m/2) e^{i m phi} = (x+iy)^m, which gives a
// polynomial extension whose gradient, projected onto the sphere's tangent plane,
// is the surface gradient.  Coefficient index k = l*l + l + m.
// ------------------------------------------------------------------------------------
struct SHBasis {
  int deg = -1;
  // pd[l][m] = coefficients (ascending powers) of the m-th derivative of P_l
  std::vector<std::vector<std::vector<double>>> pd;
  std::vector<std::vector<double>> norm;  // N_l^m

  explicit SHBasis(int degree) : deg(degree) {
    std::vector<std::vector<double>> P(degree + 2);
    P[0] = {1.0};
    if (degree + 1 >= 1) P[1] = {0.0, 1.0};
    for (int n = 1; n + 1 <= degree + 1; ++n) {  // (n+1)P_{n+1} = (2n+1) x P_n - n P_{n-1}
      std::vector<double> r(n + 2, 0.0);
      for (int i = 0; i <= n; ++i) r[i + 1] += (2.0 * n + 1.0) * P[n][i];
      for (int i = 0; i <= n - 1; ++i) r[i] -= n * P[n - 1][i];
      for (double& v : r) v /= (n + 1.0);
      P[n + 1] = r;
    }
    pd.resize(degree + 1);
    norm.resize(degree + 1);
    for (int l = 0; l <= degree; ++l) {
      pd[l].resize(l + 2);
      pd[l][0] = P[l];
      for (int m = 1; m <= l + 1; ++m) {
        const auto& prev = pd[l][m - 1];
        std::vector<double> d(prev.size() > 1 ? prev.size() - 1 : 1, 0.0);
        for (size_t i = 1; i < prev.size(); ++i) d[i - 1] = prev[i] * double(i);
        pd[l][m] = d;
      }
      norm[l].resize(l + 1);
      for (int m = 0; m <= l; ++m) {
        double ratio = 1.0;  // (l-m)!/(l+m)!
        for (int i = l - m + 1; i <= l + m; ++i) ratio /= double(i);
        norm[l][m] = std::sqrt((2.0 * l + 1.0) / (4.0 * kPi) * ratio);
      }
    }
  }

  static double poly(const std::vector<double>& c, double x) {
    double r = 0.0;
    for (size_t i = c.size(); i-- > 0;) r = r * x + c[i];
    return r;
  }

  // Y[k] and the gradient of the polynomial extension dY[k][3] at unit v.
  void eval(const double v[3], double* Y, double (*dY)[3]) const {
    const double x = v[0], y = v[1], z = v[2];
    // powers of w = x + i y: w^m = re[m] + i im[m]
    double re[8], im[8];
    re[0] = 1.0;
    im[0] = 0.0;
    for (int m = 1; m <= deg; ++m) {
      re[m] = re[m - 1] * x - im[m - 1] * y;
      im[m] = re[m - 1] * y + im[m - 1] * x;
    }
    const double s2 = std::sqrt(2.0);
    for (int l = 0; l <= deg; ++l) {
      for (int m = -l; m <= l; ++m) {
        const int am = m < 0 ? -m : m;
        const int k = l * l + l + m;
        const double f = poly(pd[l][am], z);
        const double fz = poly(pd[l][am + 1], z);
        const double sign = (am % 2) ? -1.0 : 1.0;
        double c = norm[l][am] * sign * (am ? s2 : 1.0);
        double ang, dax, day;
        if (m > 0) {
          ang = re[am];
          dax = am * re[am - 1];
          day = -am * im[am - 1];
        } else if (m < 0) {
          ang = im[am];
          dax = am * im[am - 1];
          day = am * re[am - 1];
        } else {
          ang = 1.0;
          dax = 0.0;
          day = 0.0;
        }
        Y[k] = c * f * ang;
        if (dY) {
          dY[k][0] = c * f * dax;
          dY[k][1] = c * f * day;
          dY[k][2] = c * fz * ang;
        }
      }
    }
  }
};

// ------------------------------------------------------------------------------------
// Discrete stage, binary32.  The operation order below is the contract shared (as
// text, not code) with the GPU path; every line is one correctly rounded operation.
// ------------------------------------------------------------------------------------
struct Disc {
  bool vis = false;
  float mux = 0.f, muy = 0.f, z = 0.f;
  float ca = 0.f, cb = 0.f, cc = 0.f;  // projected covariance incl. low-pass
  int x0 = 0, x1 = -1, y0 = 0, y1 = -1;  // inclusive pixel rectangle
};

// Guard-band limits of x/z and y/z inside the Jacobian (binary32): jclamp (W / 2) / fx and
// jclamp (H / 2) / fy.
void clamp_limits(const or_camera& cam, float jclamp, float& limx, float& limy) {
  limx = jclamp * ((0.5f * float(cam.width)) / cam.fx);
  limy = jclamp * ((0.5f * float(cam.height)) / cam.fy);
}

Disc discrete_stage(const float p[3], const float s[3], const float q[4], const or_camera& cam,
                    float k, float lowpass, float guard, float jclamp) {
  Disc d;
  const float* W = cam.R;
  // camera-space mean, each row summed left to right
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
  if (!(tz > cam.znear)) return d;
  // normalised quaternion
  float nq = q[0] * q[0];
  nq = nq + q[1] * q[1];
  nq = nq + q[2] * q[2];
  nq = nq + q[3] * q[3];
  nq = std::sqrt(nq);
  if (!(nq > 0.f)) return d;
  const float w = q[0] / nq, x = q[1] / nq, y = q[2] / nq, z = q[3] / nq;
  // rotation matrix of the unit quaternion
  float r[9];
  r[0] = 1.f - 2.f * (y * y + z * z);
  r[1] = 2.f * (x * y - w * z);
  r[2] = 2.f * (x * z + w * y);
  r[3] = 2.f * (x * y + w * z);
  r[4] = 1.f - 2.f * (x * x + z * z);
  r[5] = 2.f * (y * z - w * x);
  r[6] = 2.f * (x * z - w * y);
  r[7] = 2.f * (y * z + w * x);
  r[8] = 1.f - 2.f * (x * x + y * y);
  // M = R diag(s)
  float m[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) m[i * 3 + j] = r[i * 3 + j] * s[j];
  // Jacobian of the perspective projection
  const float tz2 = tz * tz;
  const float j00 = cam.fx / tz;
  const float j11 = cam.fy / tz;
  // with the guard-band clamp, an offset beyond the limit enters J as limit * z
  float txj = tx, tyj = ty;
  if (jclamp > 0.f) {
    float limx, limy;
    clamp_limits(cam, jclamp, limx, limy);
    const float ux = tx / tz, uy = ty / tz;
    if (ux < -limx) txj = -limx * tz;
    else if (ux > limx) txj = limx * tz;
    if (uy < -limy) tyj = -limy * tz;
    else if (uy > limy) tyj = limy * tz;
  }
  const float j02 = -(cam.fx * txj) / tz2;
  const float j12 = -(cam.fy * tyj) / tz2;
  // T = J W (2x3)
  float T[6];
  for (int c = 0; c < 3; ++c) {
    T[c] = j00 * W[c] + j02 * W[6 + c];
    T[3 + c] = j11 * W[3 + c] + j12 * W[6 + c];
  }
  // U = T M (2x3)
  float U[6];
  for (int i = 0; i < 2; ++i)
    for (int c = 0; c < 3; ++c) {
      float acc = T[i * 3 + 0] * m[0 * 3 + c];
      acc = acc + T[i * 3 + 1] * m[1 * 3 + c];
      acc = acc + T[i * 3 + 2] * m[2 * 3 + c];
      U[i * 3 + c] = acc;
    }
  // projected covariance U U^T + lowpass I
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
  const float det = a * c - b * b;
  if (!(det > 0.f)) return d;
  const float mux = cam.fx * (tx / tz) + cam.cx;
  const float muy = cam.fy * (ty / tz) + cam.cy;
  // view frustum: the centre must project inside the image widened by the guard band
  const float gx = guard * float(cam.width), gy = guard * float(cam.height);
  if (!(mux >= -gx && mux <= float(cam.width) + gx && muy >= -gy && muy <= float(cam.height) + gy)) return d;
  const float rx = k * std::sqrt(a);
  const float ry = k * std::sqrt(c);
  float fx0 = std::ceil(mux - rx), fx1 = std::floor(mux + rx);
  float fy0 = std::ceil(muy - ry), fy1 = std::floor(muy + ry);
  const float wmax = float(cam.width - 1), hmax = float(cam.height - 1);
  fx0 = (fx0 < 0.f) ? 0.f : fx0;
  fy0 = (fy0 < 0.f) ? 0.f : fy0;
  fx1 = (fx1 > wmax) ? wmax : fx1;
  fy1 = (fy1 > hmax) ? hmax : fy1;
  if (!(fx0 <= fx1 && fy0 <= fy1)) return d;
  d.vis = true;
  d.mux = mux;
  d.muy = muy;
  d.z = tz;
  d.ca = a;
  d.cb = b;
  d.cc = c;
  d.x0 = int(fx0);
  d.x1 = int(fx1);
  d.y0 = int(fy0);
  d.y1 = int(fy1);
  return d;
}

// The tile columns of tile row `ty` that can hold a pixel of the ellipse
// (u - mu)^T Q (u - mu) <= k^2 (Q the binary32 conic: det = a c - b b, inv = 1 / det,
// Q = (c, -b, a) * inv).  Over the row's pixel band y in [ty*ts, min(ty*ts + ts - 1, H - 1)]
// the ellipse reaches furthest right at dy = clamp(-B k / sqrt(C det_Q), u0, u1) and
// furthest left at dy = clamp(B k / sqrt(C det_Q), u0, u1), where its x offsets are
// (+-sqrt(max(0, A k^2 - det_Q dy^2)) - B dy) / A; pixels from ceil(mu_x + left) to
// floor(mu_x + right), kept inside the rectangle's columns, give the tiles.  One correctly
// rounded binary32 operation per line; false when the row keeps no tile.  A degenerate
// conic (det_Q or C det_Q not > 0) or a NaN keeps the rectangle's columns.
bool row_run(const Disc& d, float k, int ts, int ty, int W, int H, int tx0, int tx1, int* lo, int* hi) {
  *lo = tx0;
  *hi = tx1;
  float det = d.ca * d.cc;
  det = det - d.cb * d.cb;
  const float inv = 1.f / det;
  const float A = d.cc * inv;
  const float B = (-d.cb) * inv;
  const float C = d.ca * inv;
  float dq = A * C;
  dq = dq - B * B;
  if (!(dq > 0.f)) return true;
  float sq = C * dq;
  sq = std::sqrt(sq);
  if (!(sq > 0.f)) return true;
  float q = B * k;
  q = q / sq;
  const float dyr = -q, dyl = q;
  const int ylast = std::min(ty * ts + ts - 1, H - 1);
  const float u0 = float(ty * ts) - d.muy;
  const float u1 = float(ylast) - d.muy;
  const float ur = std::min(std::max(dyr, u0), u1);
  const float ul = std::min(std::max(dyl, u0), u1);
  float ak = k * k;
  ak = A * ak;
  // right edge
  float e = ur * ur;
  e = dq * e;
  e = ak - e;
  e = e > 0.f ? e : 0.f;  // also a NaN
  float sr = std::sqrt(e);
  float xr = B * ur;
  xr = sr - xr;
  xr = xr / A;
  // left edge
  e = ul * ul;
  e = dq * e;
  e = ak - e;
  e = e > 0.f ? e : 0.f;  // also a NaN
  float sl = std::sqrt(e);
  float xl = B * ul;
  xl = (-sl) - xl;
  xl = xl / A;
  float pl = d.mux + xl;
  pl = std::ceil(pl);
  float pr = d.mux + xr;
  pr = std::floor(pr);
  const float xa = float(tx0 * ts);
  const float xb = float(std::min(tx1 * ts + ts - 1, W - 1));
  if (!(pl >= xa)) pl = xa;  // also a NaN
  if (!(pr <= xb)) pr = xb;
  if (!(pl <= pr)) return false;
  *lo = int(pl) / ts;
  *hi = int(pr) / ts;
  return true;
}

uint32_t f32_bits(float v) {
  uint32_t u;
  std::memcpy(&u, &v, 4);
  return u;
}

// binary64 per-(view, Gaussian) quantities of the value stage
struct Rec {
  double mux, muy, z;
  double A, B, C;       // conic = inverse projected covariance
  double opacity;
  double color[3];
};

struct Mat3 {
  double m[9];
};

void quat_rot(const double qn[4], double R[9]) {
  const double w = qn[0], x = qn[1], y = qn[2], z = qn[3];
  R[0] = 1 - 2 * (y * y + z * z);
  R[1] = 2 * (x * y - w * z);
  R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);
  R[4] = 1 - 2 * (x * x + z * z);
  R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);
  R[7] = 2 * (y * z + w * x);
  R[8] = 1 - 2 * (x * x + y * y);
}

// Partial derivatives of R(q) (unit q) with respect to w, x, y, z.
void quat_rot_grad(const double qn[4], double dR[4][9]) {
  const double w = qn[0], x = qn[1], y = qn[2], z = qn[3];
  const double gw[9] = {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0};
  const double gx[9] = {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x};
  const double gy[9] = {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y};
  const double gz[9] = {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0};
  std::memcpy(dR[0], gw, sizeof gw);
  std::memcpy(dR[1], gx, sizeof gx);
  std::memcpy(dR[2], gy, sizeof gy);
  std::memcpy(dR[3], gz, sizeof gz);
}

// Everything of the value stage that depends only on (view, Gaussian), binary64.
struct Geo {
  double p[3], s[3], qn[4], qnorm;
  double R[9], M[9], Sig[9];      // rotation, R diag(s), Sigma = M M^T (Eq. 2)
  double W[9], t[3];              // camera rotation, camera-space mean
  double J[6], T[6];              // Jacobian (2x3) and T = J W
  bool clx, cly;                  // x/z, y/z clamped inside J (guard band)
  double S2[3];                   // projected covariance (a, b, c) incl. low-pass (Eq. 5)
  double det, A, B, C;            // conic
  double mux, muy;
  double dir[3], dnorm, v[3];     // view direction for SH
};

struct Ctx {
  // inputs
  int64_t n = 0;
  int deg = 0, K = 1;
  std::vector<double> means, scales, quats, opac, sh;
  std::vector<or_camera> cams;
  or_settings set{};
  // discrete stage
  std::vector<Disc> disc;           // [V*N]
  std::vector<int64_t> tile_off;    // [V+1]
  std::vector<int> tiles_x, tiles_y;
  std::vector<uint64_t> keys;
  std::vector<uint32_t> vals;
  std::vector<uint32_t> ranges;     // [tiles*2]
  // value stage
  std::vector<Rec> rec;             // [V*N]
  std::vector<int64_t> pix_off;     // [V+1]
};

void make_geo(const Ctx& c, int v, int64_t g, Geo& o) {
  const or_camera& cam = c.cams[v];
  for (int i = 0; i < 3; ++i) {
    o.p[i] = c.means[g * 3 + i];
    o.s[i] = c.scales[g * 3 + i];
  }
  double q[4];
  for (int i = 0; i < 4; ++i) q[i] = c.quats[g * 4 + i];
  o.qnorm = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int i = 0; i < 4; ++i) o.qn[i] = q[i] / o.qnorm;
  quat_rot(o.qn, o.R);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) o.M[i * 3 + j] = o.R[i * 3 + j] * o.s[j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += o.M[i * 3 + k] * o.M[j * 3 + k];
      o.Sig[i * 3 + j] = acc;
    }
  for (int i = 0; i < 9; ++i) o.W[i] = cam.R[i];
  for (int i = 0; i < 3; ++i)
    o.t[i] = o.W[i * 3 + 0] * o.p[0] + o.W[i * 3 + 1] * o.p[1] + o.W[i * 3 + 2] * o.p[2] + double(cam.t[i]);
  const double fx = cam.fx, fy = cam.fy, tx = o.t[0], ty = o.t[1], tz = o.t[2];
  double txj = tx, tyj = ty;
  o.clx = o.cly = false;
  if (c.set.jclamp > 0.f) {
    float limx, limy;
    clamp_limits(cam, c.set.jclamp, limx, limy);
    const double ux = tx / tz, uy = ty / tz;
    if (ux < -double(limx) || ux > double(limx)) {
      o.clx = true;
      txj = (ux < 0 ? -double(limx) : double(limx)) * tz;
    }
    if (uy < -double(limy) || uy > double(limy)) {
      o.cly = true;
      tyj = (uy < 0 ? -double(limy) : double(limy)) * tz;
    }
  }
  o.J[0] = fx / tz;
  o.J[1] = 0;
  o.J[2] = -fx * txj / (tz * tz);
  o.J[3] = 0;
  o.J[4] = fy / tz;
  o.J[5] = -fy * tyj / (tz * tz);
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += o.J[i * 3 + k] * o.W[k * 3 + j];
      o.T[i * 3 + j] = acc;
    }
  // Sigma_hat = T Sigma T^T + lowpass I
  double TS[6];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += o.T[i * 3 + k] * o.Sig[k * 3 + j];
      TS[i * 3 + j] = acc;
    }
  double S[4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += TS[i * 3 + k] * o.T[j * 3 + k];
      S[i * 2 + j] = acc;
    }
  const double lp = c.set.lowpass;
  o.S2[0] = S[0] + lp;
  o.S2[1] = S[1];
  o.S2[2] = S[3] + lp;
  o.det = o.S2[0] * o.S2[2] - o.S2[1] * o.S2[1];
  o.A = o.S2[2] / o.det;
  o.B = -o.S2[1] / o.det;
  o.C = o.S2[0] / o.det;
  o.mux = fx * tx / tz + double(cam.cx);
  o.muy = fy * ty / tz + double(cam.cy);
  // camera centre C = -W^T t_cam
  double cc[3];
  for (int i = 0; i < 3; ++i)
    cc[i] = -(o.W[0 * 3 + i] * double(cam.t[0]) + o.W[1 * 3 + i] * double(cam.t[1]) +
              o.W[2 * 3 + i] * double(cam.t[2]));
  for (int i = 0; i < 3; ++i) o.dir[i] = o.p[i] - cc[i];
  o.dnorm = std::sqrt(o.dir[0] * o.dir[0] + o.dir[1] * o.dir[1] + o.dir[2] * o.dir[2]);
  for (int i = 0; i < 3; ++i) o.v[i] = o.dir[i] / o.dnorm;
}

void build(Ctx& c) {
  const int V = int(c.cams.size());
  const int64_t N = c.n;
  c.disc.assign(size_t(V) * N, Disc{});
  c.tile_off.assign(V + 1, 0);
  c.tiles_x.resize(V);
  c.tiles_y.resize(V);
  c.pix_off.assign(V + 1, 0);
  const int ts = c.set.tile;
  for (int v = 0; v < V; ++v) {
    c.tiles_x[v] = (c.cams[v].width + ts - 1) / ts;
    c.tiles_y[v] = (c.cams[v].height + ts - 1) / ts;
    c.tile_off[v + 1] = c.tile_off[v] + int64_t(c.tiles_x[v]) * c.tiles_y[v];
    c.pix_off[v + 1] = c.pix_off[v] + int64_t(c.cams[v].width) * c.cams[v].height;
  }
  // discrete stage, keys in duplication order (view, Gaussian, tile row, tile column)
  std::vector<uint64_t> keys;
  std::vector<uint32_t> vals;
  for (int v = 0; v < V; ++v)
    for (int64_t g = 0; g < N; ++g) {
      float p[3], s[3], q[4];
      for (int i = 0; i < 3; ++i) {
        p[i] = float(c.means[g * 3 + i]);
        s[i] = float(c.scales[g * 3 + i]);
      }
      for (int i = 0; i < 4; ++i) q[i] = float(c.quats[g * 4 + i]);
      Disc d = discrete_stage(p, s, q, c.cams[v], c.set.extent_k, c.set.lowpass, c.set.guard, c.set.jclamp);
      c.disc[size_t(v) * N + g] = d;
      if (!d.vis) continue;
      const int tx0 = d.x0 / ts, tx1 = d.x1 / ts, ty0 = d.y0 / ts, ty1 = d.y1 / ts;
      for (int ty = ty0; ty <= ty1; ++ty) {
        int lo = tx0, hi = tx1;
        if (c.set.exact_tiles &&
            !row_run(d, c.set.extent_k, ts, ty, c.cams[v].width, c.cams[v].height, tx0, tx1, &lo, &hi))
          continue;
        for (int tx = lo; tx <= hi; ++tx) {
          const uint64_t tile = uint64_t(c.tile_off[v] + int64_t(ty) * c.tiles_x[v] + tx);
          keys.push_back((tile << 32) | f32_bits(d.z));
          vals.push_back(uint32_t(int64_t(v) * N + g));
        }
      }
    }
  // stable ascending sort by key
  std::vector<size_t> order(keys.size());
  std::iota(order.begin(), order.end(), size_t(0));
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return keys[a] < keys[b]; });
  c.keys.resize(keys.size());
  c.vals.resize(keys.size());
  for (size_t i = 0; i < order.size(); ++i) {
    c.keys[i] = keys[order[i]];
    c.vals[i] = vals[order[i]];
  }
  // tile ranges [start, end); empty tiles [0, 0)
  c.ranges.assign(size_t(c.tile_off[V]) * 2, 0u);
  for (size_t i = 0; i < c.keys.size(); ++i) {
    const uint64_t tile = c.keys[i] >> 32;
    if (i == 0 || (c.keys[i - 1] >> 32) != tile) c.ranges[tile * 2] = uint32_t(i);
    if (i + 1 == c.keys.size() || (c.keys[i + 1] >> 32) != tile) c.ranges[tile * 2 + 1] = uint32_t(i + 1);
  }
  // value stage per visible (view, Gaussian)
  SHBasis sh(c.deg);
  c.rec.assign(size_t(V) * N, Rec{});
  std::vector<double> Y(c.K);
  for (int v = 0; v < V; ++v)
    for (int64_t g = 0; g < N; ++g) {
      const Disc& d = c.disc[size_t(v) * N + g];
      if (!d.vis) continue;
      Geo o;
      make_geo(c, v, g, o);
      Rec& r = c.rec[size_t(v) * N + g];
      if (c.set.mu_fp32) {
        r.mux = d.mux;
        r.muy = d.muy;
      } else {
        r.mux = o.mux;
        r.muy = o.muy;
      }
      r.z = o.t[2];
      if (c.set.mu_fp32) {
        // the projected covariance as the fixed binary32 sequence leaves it (the same bits
        // on both sides), inverted in binary64
        const double a = d.ca, b = d.cb, cc = d.cc;
        const double det = a * cc - b * b;
        r.A = cc / det;
        r.B = -b / det;
        r.C = a / det;
      } else {
        r.A = o.A;
        r.B = o.B;
        r.C = o.C;
      }
      r.opacity = c.opac[g];
      sh.eval(o.v, Y.data(), nullptr);
      for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.5;
        for (int k = 0; k < c.K; ++k) acc += c.sh[(g * c.K + k) * 3 + ch] * Y[k];
        r.color[ch] = acc > 0.0 ? acc : 0.0;
      }
    }
}

struct Hit {
  uint32_t rec;
  double G, a, alpha, T, dx, dy;
};

// Depth normalised by the accumulated opacity: D / (1 - T_final), 0 where nothing is hit.
double normalized(double D, double T) {
  const double A = 1.0 - T;
  return A > 0.0 ? D / A : 0.0;
}

// One front-to-back pass of a pixel over its tile's sorted list (Eq. 11 with the
// clamp, skip and stop rules).
struct Pass {
  double out[5];       // colour (3), accumulated depth D, final transmittance
  int32_t ncontrib = 0;  // one past the list position of the last contributor
  int32_t nused = 0;     // contributors
  int events = 0;        // skip/stop decisions met within the ambiguity margins
  int32_t near_a = 0;    // splat values within kWide times the skip margin of alpha_min
  int32_t near_T = 0;    // transmittances within kWide times the stop margin of T_min
};

// A decision whose operands lie within a relative margin of the threshold (about ten
// times the binary32 rounding of a = o exp(-q/2) and of T) may fall either way in a
// binary32 renderer, and both outcomes are correct.  `flip` inverts the k-th such
// decision met along the pass (bit k), so every correct outcome of a pixel can be
// enumerated.  near_a / near_T count the values within kWide times the margins: the
// density of values near a threshold, from which the expected number of ambiguous
// decisions follows (a kWide-times narrower window holds 1/kWide of them).
constexpr double kWide = 100.0;

void composite(const Ctx& c, int64_t tile, double px, double py, uint32_t flip, Pass& p, std::vector<Hit>* hits) {
  const uint32_t s = c.ranges[tile * 2], e = c.ranges[tile * 2 + 1];
  const double amin = c.set.alpha_min, amax = c.set.alpha_max, Tmin = c.set.T_min;
  const double rel_a = c.set.amb_rel_a, rel_T = c.set.amb_rel_T;
  double T = 1.0, C[3] = {0, 0, 0}, D = 0.0;
  p.ncontrib = 0;
  p.nused = 0;
  p.events = 0;
  p.near_a = 0;
  p.near_T = 0;
  for (uint32_t i = s; i < e; ++i) {
    const uint32_t ri = c.vals[i];
    const Rec& r = c.rec[ri];
    const double dx = px - r.mux, dy = py - r.muy;
    const double power = -0.5 * (r.A * dx * dx + 2.0 * r.B * dx * dy + r.C * dy * dy);
    const double G = std::exp(power);
    const double a = r.opacity * G;
    const double da_rel = std::fabs(a - amin);
    if (da_rel <= kWide * rel_a * amin) ++p.near_a;
    bool skip = a < amin;
    if (da_rel <= rel_a * amin) {
      if (p.events < 32 && ((flip >> p.events) & 1u)) skip = !skip;
      ++p.events;
    }
    if (skip) continue;
    const double alpha = a < amax ? a : amax;
    if (hits) hits->push_back(Hit{ri, G, a, alpha, T, dx, dy});
    for (int ch = 0; ch < 3; ++ch) C[ch] += r.color[ch] * alpha * T;
    D += r.z * alpha * T;
    T = T * (1.0 - alpha);
    p.ncontrib = int32_t(i - s + 1);
    ++p.nused;
    const double dT_rel = std::fabs(T - Tmin);
    if (dT_rel <= kWide * rel_T * Tmin) ++p.near_T;
    bool stop = T < Tmin;
    if (dT_rel <= rel_T * Tmin) {
      if (p.events < 32 && ((flip >> p.events) & 1u)) stop = !stop;
      ++p.events;
    }
    if (stop) break;
  }
  for (int ch = 0; ch < 3; ++ch) p.out[ch] = C[ch] + T * double(c.set.bg[ch]);
  p.out[3] = D;
  p.out[4] = T;
}

// Every correct outcome of a pixel: calls f(pass, flip) for the reference pass (flip 0)
// and for each other combination of its ambiguous decisions (a combination counts when
// each flipped decision is met).  Returns false, after the reference pass only, when some
// combination meets more than kMaxFlips such decisions.
constexpr int kMaxFlips = 8;

template <class F>
bool outcomes(const Ctx& c, int64_t tile, double px, double py, std::vector<Hit>* hits, F&& f) {
  Pass p;
  if (hits) hits->clear();
  composite(c, tile, px, py, 0u, p, hits);
  f(p, hits, 0u);
  if (p.events > kMaxFlips) return false;
  int E = p.events;
  std::vector<Hit> hq;
  for (uint32_t m = 1; m < (1u << E); ++m) {
    Pass q;
    hq.clear();
    composite(c, tile, px, py, m, q, hits ? &hq : nullptr);
    if (q.events > kMaxFlips) return false;
    if (q.events > E) E = q.events;       // a flip exposed further decisions: enumerate them too
    if ((m >> q.events) != 0u) continue;  // flips a decision this pass never met
    f(q, hits ? &hq : nullptr, m);
  }
  return true;
}

// The reverse sweep of one pixel pass (O6): back to front over the processed
// contributors, emit(record, t, alt) with the contributor's additive 2D-gradient terms t
// (dmu 2, dconic 3, dopacity, dcolour 3, ddepth) for the output gradients (gC, gD, gA),
// and alt = the same terms under the opposite clamp decision when its splat value lies
// within the ambiguity margin of alpha_max (else NULL).
template <class Emit>
void sweep(const Ctx& c, const Pass& p, const std::vector<Hit>& hits, const double* gC_in, double gD, double gA,
           Emit&& emit) {
  const double amax = c.set.alpha_max, rel = c.set.amb_rel_a;
  const double Tfin = p.out[4];
  const double gC[3] = {gC_in[0], gC_in[1], gC_in[2]};
  if (c.set.normalized_depth) {
    // Dn = D / A with A = 1 - T_final: dL/dD = g / A, and dL/dA gains -g D / A^2
    // = -g Dn / A; through A = 1 - T_final that is +g Dn / A on the alpha
    // output's gradient route (A is the alpha output)
    const double A = 1.0 - Tfin;
    if (A > 0.0) {
      const double Dn = p.out[3] / A;
      gA += -gD * Dn / A;
      gD = gD / A;
    } else {
      gD = 0.0;
    }
  }
  double BC[3] = {c.set.bg[0], c.set.bg[1], c.set.bg[2]}, BD = 0.0;
  for (size_t i = hits.size(); i-- > 0;) {
    const Hit& hh = hits[i];
    const Rec& r = c.rec[hh.rec];
    double t[10], alt[10];
    double dal = 0.0;
    for (int ch = 0; ch < 3; ++ch) dal += gC[ch] * (r.color[ch] - BC[ch]);
    dal += gD * (r.z - BD);
    dal *= hh.T;
    dal += gA * Tfin / (1.0 - hh.alpha);
    for (int ch = 0; ch < 3; ++ch) t[6 + ch] = gC[ch] * hh.alpha * hh.T;
    t[9] = gD * hh.alpha * hh.T;
    for (int ch = 0; ch < 3; ++ch) BC[ch] = hh.alpha * r.color[ch] + (1.0 - hh.alpha) * BC[ch];
    BD = hh.alpha * r.z + (1.0 - hh.alpha) * BD;
    auto splat_terms = [&](double da, double* o) {
      o[5] = da * hh.G;
      const double dpow = da * hh.a;
      o[0] = dpow * (r.A * hh.dx + r.B * hh.dy);
      o[1] = dpow * (r.B * hh.dx + r.C * hh.dy);
      o[2] = -0.5 * dpow * hh.dx * hh.dx;
      o[3] = -dpow * hh.dx * hh.dy;
      o[4] = -0.5 * dpow * hh.dy * hh.dy;
    };
    const bool unclamped = hh.a <= amax;
    splat_terms(unclamped ? dal : 0.0, t);
    const bool edge = std::fabs(hh.a - amax) <= rel * amax;
    if (edge) {
      splat_terms(unclamped ? 0.0 : dal, alt);
      for (int k = 6; k < 10; ++k) alt[k] = t[k];
    }
    emit(hh.rec, t, edge ? alt : nullptr);
  }
}

// The pixels [xa, xb) x [ya, yb) of tile (tx, ty) inside the settings' window (the whole
// tile when the window is empty); false when none.
bool window_of_tile(const Ctx& c, int tx, int ty, int W, int H, int& xa, int& xb, int& ya, int& yb) {
  const int ts = c.set.tile;
  xa = tx * ts;
  ya = ty * ts;
  xb = std::min(W, (tx + 1) * ts);
  yb = std::min(H, (ty + 1) * ts);
  const int32_t* w = c.set.window;
  if (w[2] > w[0] && w[3] > w[1]) {
    xa = std::max(xa, int(w[0]));
    ya = std::max(ya, int(w[1]));
    xb = std::min(xb, int(w[2]));
    yb = std::min(yb, int(w[3]));
  }
  return xa < xb && ya < yb;
}

template <class F>
void parallel_tiles(const Ctx& c, F&& f) {
  const int64_t tiles = c.tile_off.back();
  int th = c.set.threads < 1 ? 1 : c.set.threads;
  if (th == 1 || tiles < 2) {
    f(0, int64_t(0), tiles);
    return;
  }
  std::vector<std::thread> pool;
  for (int w = 0; w < th; ++w) {
    const int64_t a = tiles * w / th, b = tiles * (w + 1) / th;
    pool.emplace_back([&, w, a, b] { f(w, a, b); });
  }
  for (auto& t : pool) t.join();
}

int view_of_tile(const Ctx& c, int64_t tile) {
  int v = 0;
  while (c.tile_off[v + 1] <= tile) ++v;
  return v;
}

// Per-Gaussian gradient accumulators in the parameter layouts.
struct Grad3 {
  double dp[3] = {0, 0, 0}, ds[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0}, dop = 0.0;
  std::vector<double> dk;
  explicit Grad3(int K) : dk(size_t(K) * 3, 0.0) {}
};

// Chain rule of one (view, Gaussian) record (O7): its 2D gradient G (dmu 2, dconic 3,
// dopacity, dcolour 3, ddepth) taken back to the Gaussian's parameters and added to out.
// Linear in G for a fixed Gaussian and camera.
void chain(const Ctx& c, const SHBasis& sh, std::vector<double>& Y, double (*dY)[3], int v, int64_t g, const double* G,
           Grad3& out) {
    const or_camera& cam = c.cams[v];
    Geo o;
    make_geo(c, v, g, o);
    // opacity
    out.dop += G[5];
    // colour through SH, with the clamp at zero masking the gradient
    sh.eval(o.v, Y.data(), dY);
    double dv[3] = {0, 0, 0};
    for (int ch = 0; ch < 3; ++ch) {
      double raw = 0.5;
      for (int k = 0; k < c.K; ++k) raw += c.sh[(g * c.K + k) * 3 + ch] * Y[k];
      if (!(raw > 0.0)) continue;
      const double gc = G[6 + ch];
      for (int k = 0; k < c.K; ++k) {
        out.dk[k * 3 + ch] += Y[k] * gc;
        const double kc = c.sh[(g * c.K + k) * 3 + ch] * gc;
        for (int i = 0; i < 3; ++i) dv[i] += kc * dY[k][i];
      }
    }
    const double vdot = dv[0] * o.v[0] + dv[1] * o.v[1] + dv[2] * o.v[2];
    for (int i = 0; i < 3; ++i) out.dp[i] += (dv[i] - o.v[i] * vdot) / o.dnorm;
    // conic -> projected covariance: dS = -Q G_Q Q
    const double Q[4] = {o.A, o.B, o.B, o.C};
    const double GQ[4] = {G[2], 0.5 * G[3], 0.5 * G[3], G[4]};
    double QG[4], dS[4];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) QG[i * 2 + j] = Q[i * 2 + 0] * GQ[0 * 2 + j] + Q[i * 2 + 1] * GQ[1 * 2 + j];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) dS[i * 2 + j] = -(QG[i * 2 + 0] * Q[0 * 2 + j] + QG[i * 2 + 1] * Q[1 * 2 + j]);
    // Sigma_hat = T Sigma T^T: dSigma = T^T dS T, dT = 2 dS T Sigma
    double dSig[9], dT[6];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double a = 0;
        for (int k = 0; k < 2; ++k)
          for (int l = 0; l < 2; ++l) a += o.T[k * 3 + i] * dS[k * 2 + l] * o.T[l * 3 + j];
        dSig[i * 3 + j] = a;
      }
    double TSig[6];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 3; ++j) {
        double a = 0;
        for (int k = 0; k < 3; ++k) a += o.T[i * 3 + k] * o.Sig[k * 3 + j];
        TSig[i * 3 + j] = a;
      }
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 3; ++j) dT[i * 3 + j] = 2.0 * (dS[i * 2 + 0] * TSig[0 * 3 + j] + dS[i * 2 + 1] * TSig[1 * 3 + j]);
    // T = J W: dJ = dT W^T
    double dJ[6];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 3; ++j) {
        double a = 0;
        for (int k = 0; k < 3; ++k) a += dT[i * 3 + k] * o.W[j * 3 + k];
        dJ[i * 3 + j] = a;
      }
    const double fx = cam.fx, fy = cam.fy, tx = o.t[0], ty = o.t[1], tz = o.t[2];
    double dt[3] = {0, 0, 0};
    // J02 = -fx x'/z^2 with x' = x, or +-limit z where clamped (then J02 = -+fx limit / z);
    // likewise J12: d/dx of a clamped entry is 0, and d/dz is -J02/z instead of -2 J02/z
    dt[0] += o.clx ? 0.0 : dJ[2] * (-fx / (tz * tz));
    dt[1] += o.cly ? 0.0 : dJ[5] * (-fy / (tz * tz));
    dt[2] += dJ[0] * (-fx / (tz * tz)) + dJ[2] * (o.clx ? -o.J[2] / tz : 2.0 * fx * tx / (tz * tz * tz)) +
             dJ[4] * (-fy / (tz * tz)) + dJ[5] * (o.cly ? -o.J[5] / tz : 2.0 * fy * ty / (tz * tz * tz));
    // splat centre (Eq. 4) and depth
    dt[0] += G[0] * fx / tz;
    dt[2] += -G[0] * fx * tx / (tz * tz);
    dt[1] += G[1] * fy / tz;
    dt[2] += -G[1] * fy * ty / (tz * tz);
    dt[2] += G[9];
    for (int i = 0; i < 3; ++i) out.dp[i] += o.W[0 * 3 + i] * dt[0] + o.W[1 * 3 + i] * dt[1] + o.W[2 * 3 + i] * dt[2];
    // Sigma = M M^T: dM = 2 dSigma M; M = R diag(s)
    double dM[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double a = 0;
        for (int k = 0; k < 3; ++k) a += dSig[i * 3 + k] * o.M[k * 3 + j];
        dM[i * 3 + j] = 2.0 * a;
      }
    double dR[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        out.ds[j] += dM[i * 3 + j] * o.R[i * 3 + j];
        dR[i * 3 + j] = dM[i * 3 + j] * o.s[j];
      }
    double gR[4][9];
    quat_rot_grad(o.qn, gR);
    double dqn[4];
    for (int a = 0; a < 4; ++a) {
      double s = 0;
      for (int i = 0; i < 9; ++i) s += gR[a][i] * dR[i];
      dqn[a] = s;
    }
    const double qd = dqn[0] * o.qn[0] + dqn[1] * o.qn[1] + dqn[2] * o.qn[2] + dqn[3] * o.qn[3];
    for (int a = 0; a < 4; ++a) out.dq[a] += (dqn[a] - o.qn[a] * qd) / o.qnorm;
}

}  // namespace

extern "C" {

// Build the oracle for V cameras.  Parameters are binary64 arrays (promote binary32
// inputs exactly); the discrete stage rounds them to binary32.
void* or_create(const double* means, const double* scales, const double* quats, const double* opac,
                const double* sh, int64_t n, int32_t sh_degree, const or_camera* cams, int32_t V,
                const or_settings* set) {
  Ctx* c = new Ctx;
  c->n = n;
  c->deg = sh_degree;
  c->K = (sh_degree + 1) * (sh_degree + 1);
  c->means.assign(means, means + n * 3);
  c->scales.assign(scales, scales + n * 3);
  c->quats.assign(quats, quats + n * 4);
  c->opac.assign(opac, opac + n);
  c->sh.assign(sh, sh + n * c->K * 3);
  c->cams.assign(cams, cams + V);
  c->set = *set;
  build(*c);
  return c;
}

void or_destroy(void* h) { delete static_cast<Ctx*>(h); }

int64_t or_num_keys(void* h) { return int64_t(static_cast<Ctx*>(h)->keys.size()); }
int64_t or_num_tiles(void* h) { return static_cast<Ctx*>(h)->tile_off.back(); }

void or_get_keys(void* h, uint64_t* keys, uint32_t* vals, uint32_t* ranges) {
  const Ctx& c = *static_cast<Ctx*>(h);
  if (keys) std::copy(c.keys.begin(), c.keys.end(), keys);
  if (vals) std::copy(c.vals.begin(), c.vals.end(), vals);
  if (ranges) std::copy(c.ranges.begin(), c.ranges.end(), ranges);
}

// Per (view, Gaussian): visible flag, binary32 centre/depth/projected covariance and the
// inclusive pixel rectangle of the discrete stage; binary64 conic and colour.
void or_get_records(void* h, uint8_t* vis, float* mu, float* z, float* cov, int32_t* rect, double* conic,
                    double* color) {
  const Ctx& c = *static_cast<Ctx*>(h);
  for (size_t i = 0; i < c.disc.size(); ++i) {
    const Disc& d = c.disc[i];
    if (vis) vis[i] = d.vis;
    if (mu) {
      mu[i * 2] = d.mux;
      mu[i * 2 + 1] = d.muy;
    }
    if (z) z[i] = d.z;
    if (cov) {
      cov[i * 3] = d.ca;
      cov[i * 3 + 1] = d.cb;
      cov[i * 3 + 2] = d.cc;
    }
    if (rect) {
      rect[i * 4] = d.x0;
      rect[i * 4 + 1] = d.x1;
      rect[i * 4 + 2] = d.y0;
      rect[i * 4 + 3] = d.y1;
    }
    const Rec& r = c.rec[i];
    if (conic) {
      conic[i * 3] = r.A;
      conic[i * 3 + 1] = r.B;
      conic[i * 3 + 2] = r.C;
    }
    if (color)
      for (int ch = 0; ch < 3; ++ch) color[i * 3 + ch] = r.color[ch];
  }
}

// Forward render of every view.  Image outputs are concatenated over views:
// color [3,H,W] per view, the others [H,W] per view.  n_contrib is one past the
// list position of the last contributor; n_used counts the contributors.
// Every further output may be NULL.  ambiguous (byte per pixel) is set where a skip or
// stop decision lies within its margin.  lo/hi [P,5] (views concatenated) bound each
// output value (colour 3, depth, alpha) over every correct outcome of the pixel's
// ambiguous decisions (both equal the value elsewhere); events [P] is the number of such
// decisions the reference pass met, -1 where a combination met more than kMaxFlips (its
// bounds then cover the reference pass only); near [P,2] counts the splat values and
// transmittances within kWide times the margins.
void or_forward(void* h, double* color, double* depth, double* alpha, double* T_final, int32_t* n_contrib,
                int32_t* n_used, uint8_t* ambiguous, double* lo, double* hi, int32_t* events, int32_t* near) {
  const Ctx& c = *static_cast<Ctx*>(h);
  const int ts = c.set.tile;
  parallel_tiles(c, [&](int, int64_t t0, int64_t t1) {
    for (int64_t tile = t0; tile < t1; ++tile) {
      const int v = view_of_tile(c, tile);
      const int64_t lt = tile - c.tile_off[v];
      const int W = c.cams[v].width, H = c.cams[v].height;
      const int tx = int(lt % c.tiles_x[v]), ty = int(lt / c.tiles_x[v]);
      const int64_t P = int64_t(W) * H;
      int xa, xb, ya, yb;
      if (!window_of_tile(c, tx, ty, W, H, xa, xb, ya, yb)) continue;
      for (int y = ya; y < yb; ++y)
        for (int x = xa; x < xb; ++x) {
          const int64_t pix = int64_t(y) * W + x;
          const int64_t base = c.pix_off[v];
          double l[5], u[5];
          Pass ref;
          const bool bounded = outcomes(c, tile, x, y, nullptr, [&](const Pass& p, const std::vector<Hit>*, uint32_t m) {
            const double val[5] = {p.out[0], p.out[1], p.out[2],
                                   c.set.normalized_depth ? normalized(p.out[3], p.out[4]) : p.out[3], 1.0 - p.out[4]};
            if (m == 0u) {
              ref = p;
              for (int k = 0; k < 5; ++k) l[k] = u[k] = val[k];
            } else {
              for (int k = 0; k < 5; ++k) {
                l[k] = std::min(l[k], val[k]);
                u[k] = std::max(u[k], val[k]);
              }
            }
          });
          if (color)
            for (int ch = 0; ch < 3; ++ch) color[base * 3 + ch * P + pix] = ref.out[ch];
          if (depth) depth[base + pix] = c.set.normalized_depth ? normalized(ref.out[3], ref.out[4]) : ref.out[3];
          if (alpha) alpha[base + pix] = 1.0 - ref.out[4];
          if (T_final) T_final[base + pix] = ref.out[4];
          if (n_contrib) n_contrib[base + pix] = ref.ncontrib;
          if (n_used) n_used[base + pix] = ref.nused;
          if (ambiguous) ambiguous[base + pix] = ref.events > 0;
          if (lo)
            for (int k = 0; k < 5; ++k) lo[(base + pix) * 5 + k] = l[k];
          if (hi)
            for (int k = 0; k < 5; ++k) hi[(base + pix) * 5 + k] = u[k];
          if (events) events[base + pix] = bounded ? ref.events : -1;
          if (near) {
            near[(base + pix) * 2] = ref.near_a;
            near[(base + pix) * 2 + 1] = ref.near_T;
          }
        }
    }
  });
}

// Reverse pass.  g_color/g_depth/g_alpha are dL/d(output) with the layouts of
// or_forward (NULL = zero).  Writes dL/d(parameters) in the parameter layouts.
//
// Several results are correct where a pixel's skip or stop decision, or a contributor's
// clamp decision, lies within its ambiguity margin, and where the output gradient itself
// is not unique (pix_amb: NULL = none, one byte per pixel, views concatenated, bit k set
// when output k (colour 0-2, depth 3, alpha 4) has a non-unique gradient; the L1 loss of
// Eq. 12 changes sign where the rendered value meets the target, so such an output
// gradient may change by up to twice its value).  e_* (same layouts, may be NULL)
// receive a bound on how far any correct gradient can lie from the one written: per
// pixel, the largest change of each contributor's 2D-gradient terms over every correct
// outcome (and the sum of the changes of each non-unique output gradient), summed over
// pixels, taken to the parameters through the absolute value of each term's chain rule.
// flagged (per Gaussian) marks Gaussians contributing to a pixel whose outcomes could not
// be enumerated (more than kMaxFlips ambiguous decisions); no bound covers those.
void or_backward(void* h, const double* g_color, const double* g_depth, const double* g_alpha,
                 const uint8_t* pix_amb, double* d_means, double* d_scales, double* d_quats, double* d_opac,
                 double* d_sh, uint8_t* flagged, double* e_means, double* e_scales, double* e_quats, double* e_opac,
                 double* e_sh) {
  const Ctx& c = *static_cast<Ctx*>(h);
  const int V = int(c.cams.size());
  const int64_t N = c.n;
  const int ts = c.set.tile;
  const int nth = c.set.threads < 1 ? 1 : c.set.threads;
  using Terms = std::array<double, 10>;
  using TermMap = std::unordered_map<uint32_t, Terms>;
  // per-thread accumulators of the 2D gradients: dmu(2), dconic(3), dopacity, dcolor(3), ddepth
  std::vector<std::vector<double>> acc(nth, std::vector<double>(size_t(V) * N * 10, 0.0));
  std::vector<std::vector<uint8_t>> flag(nth, std::vector<uint8_t>(size_t(V) * N, 0));
  std::vector<TermMap> env(nth);  // per record: bound of the 2D-gradient change
  parallel_tiles(c, [&](int w, int64_t t0, int64_t t1) {
    std::vector<Hit> hits;
    std::vector<double>& G2 = acc[w];
    std::vector<uint8_t>& F = flag[w];
    TermMap& E = env[w];
    TermMap ref_terms, pix_env;
    for (int64_t tile = t0; tile < t1; ++tile) {
      const int v = view_of_tile(c, tile);
      const int64_t lt = tile - c.tile_off[v];
      const int W = c.cams[v].width, H = c.cams[v].height;
      const int tx = int(lt % c.tiles_x[v]), ty = int(lt / c.tiles_x[v]);
      const int64_t P = int64_t(W) * H, base = c.pix_off[v];
      int xa, xb, ya, yb;
      if (!window_of_tile(c, tx, ty, W, H, xa, xb, ya, yb)) continue;
      for (int y = ya; y < yb; ++y)
        for (int x = xa; x < xb; ++x) {
          const int64_t pix = int64_t(y) * W + x;
          double gC[3];
          for (int ch = 0; ch < 3; ++ch) gC[ch] = g_color ? g_color[base * 3 + ch * P + pix] : 0.0;
          const double gD = g_depth ? g_depth[base + pix] : 0.0;
          const double gA = g_alpha ? g_alpha[base + pix] : 0.0;
          const uint32_t tie = pix_amb ? pix_amb[base + pix] : 0u;
          bool multi = false;  // the pixel has more than one correct outcome
          Pass ref;
          ref_terms.clear();
          pix_env.clear();
          const bool bounded =
              outcomes(c, tile, x, y, &hits, [&](const Pass& p, const std::vector<Hit>* hp, uint32_t m) {
                if (m == 0u) {
                  ref = p;
                  multi = p.events > 0;
                  sweep(c, p, *hp, gC, gD, gA, [&](uint32_t rec, const double* t, const double* alt) {
                    double* g = &G2[size_t(rec) * 10];
                    for (int k = 0; k < 10; ++k) g[k] += t[k];
                    if (alt) {  // the opposite clamp decision
                      Terms& e = E[rec];
                      for (int k = 0; k < 10; ++k) e[k] += std::fabs(alt[k] - t[k]);
                    }
                    if (multi) {
                      Terms& r = ref_terms[rec];
                      for (int k = 0; k < 10; ++k) r[k] = t[k];
                    }
                  });
                  return;
                }
                // another correct outcome: the change of every record's terms
                TermMap alt_terms;
                sweep(c, p, *hp, gC, gD, gA, [&](uint32_t rec, const double* t, const double*) {
                  Terms& r = alt_terms[rec];
                  for (int k = 0; k < 10; ++k) r[k] = t[k];
                });
                auto widen = [&](uint32_t rec, const Terms& a, const Terms* b) {
                  Terms& e = pix_env[rec];
                  for (int k = 0; k < 10; ++k) e[k] = std::max(e[k], std::fabs(a[k] - (b ? (*b)[k] : 0.0)));
                };
                for (const auto& kv : alt_terms) {
                  auto it = ref_terms.find(kv.first);
                  widen(kv.first, kv.second, it == ref_terms.end() ? nullptr : &it->second);
                }
                for (const auto& kv : ref_terms)
                  if (!alt_terms.count(kv.first)) widen(kv.first, kv.second, nullptr);
              });
          if (!bounded) {
            for (const Hit& hh : hits) F[hh.rec] = 1;
            continue;
          }
          for (const auto& kv : pix_env) {
            Terms& e = E[kv.first];
            for (int k = 0; k < 10; ++k) e[k] += kv.second[k];
          }
          if (tie) {
            // each output gradient may move by up to 2|g|: the terms are linear in it
            const double gout[5] = {gC[0], gC[1], gC[2], gD, gA};
            for (int ch = 0; ch < 5; ++ch) {
              if (!((tie >> ch) & 1u) || gout[ch] == 0.0) continue;
              double u[5] = {0, 0, 0, 0, 0};
              u[ch] = 1.0;
              const double scale = 2.0 * std::fabs(gout[ch]);
              sweep(c, ref, hits, u, u[3], u[4], [&](uint32_t rec, const double* t, const double*) {
                Terms& e = E[rec];
                for (int k = 0; k < 10; ++k) e[k] += scale * std::fabs(t[k]);
              });
            }
          }
        }
    }
  });
  for (int w = 1; w < nth; ++w) {
    for (size_t i = 0; i < acc[0].size(); ++i) acc[0][i] += acc[w][i];
    for (size_t i = 0; i < flag[0].size(); ++i) flag[0][i] |= flag[w][i];
    for (const auto& kv : env[w]) {
      Terms& e = env[0][kv.first];
      for (int k = 0; k < 10; ++k) e[k] += kv.second[k];
    }
  }
  const std::vector<double>& G2 = acc[0];
  const TermMap& E2 = env[0];
  const bool want_env = e_means || e_scales || e_quats || e_opac || e_sh;
  // chain rule per Gaussian, summed over views in view order
  SHBasis sh(c.deg);
  std::vector<double> Y(c.K);
  std::vector<double> dYbuf(size_t(c.K) * 3);
  double (*dY)[3] = reinterpret_cast<double (*)[3]>(dYbuf.data());
  for (int64_t g = 0; g < N; ++g) {
    Grad3 acc3(c.K), bound(c.K);
    uint8_t fl = 0;
    for (int v = 0; v < V; ++v) {
      const size_t ri = size_t(v) * N + g;
      if (!c.disc[ri].vis) continue;
      fl |= flag[0][ri];
      const double* G = &G2[ri * 10];
      chain(c, sh, Y, dY, v, g, G, acc3);
      if (!want_env) continue;
      auto it = E2.find(uint32_t(ri));
      if (it == E2.end()) continue;
      for (int k = 0; k < 10; ++k) {
        if (!(it->second[k] > 0.0)) continue;
        double Gk[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        Gk[k] = it->second[k];
        Grad3 one(c.K);
        chain(c, sh, Y, dY, v, g, Gk, one);
        for (int i = 0; i < 3; ++i) {
          bound.dp[i] += std::fabs(one.dp[i]);
          bound.ds[i] += std::fabs(one.ds[i]);
        }
        for (int i = 0; i < 4; ++i) bound.dq[i] += std::fabs(one.dq[i]);
        bound.dop += std::fabs(one.dop);
        for (size_t i = 0; i < one.dk.size(); ++i) bound.dk[i] += std::fabs(one.dk[i]);
      }
    }
    for (int i = 0; i < 3; ++i) {
      if (d_means) d_means[g * 3 + i] = acc3.dp[i];
      if (d_scales) d_scales[g * 3 + i] = acc3.ds[i];
      if (e_means) e_means[g * 3 + i] = bound.dp[i];
      if (e_scales) e_scales[g * 3 + i] = bound.ds[i];
    }
    for (int i = 0; i < 4; ++i) {
      if (d_quats) d_quats[g * 4 + i] = acc3.dq[i];
      if (e_quats) e_quats[g * 4 + i] = bound.dq[i];
    }
    if (d_opac) d_opac[g] = acc3.dop;
    if (e_opac) e_opac[g] = bound.dop;
    for (int i = 0; i < c.K * 3; ++i) {
      if (d_sh) d_sh[g * c.K * 3 + i] = acc3.dk[i];
      if (e_sh) e_sh[g * c.K * 3 + i] = bound.dk[i];
    }
    if (flagged) flagged[g] = fl;
  }
}

// Real SH basis values and polynomial-extension gradients at unit directions.
void or_sh_eval(int32_t degree, const double* dirs, int64_t n, double* Y, double* dY) {
  SHBasis sh(degree);
  const int K = (degree + 1) * (degree + 1);
  std::vector<double> gbuf(size_t(K) * 3);
  double (*g)[3] = reinterpret_cast<double (*)[3]>(gbuf.data());
  for (int64_t i = 0; i < n; ++i) {
    sh.eval(dirs + i * 3, Y + i * K, dY ? g : nullptr);
    if (dY)
      for (int k = 0; k < K; ++k)
        for (int j = 0; j < 3; ++j) dY[(i * K + k) * 3 + j] = g[k][j];
  }
}

int32_t or_version(void) { return 1; }

}  // extern "C"
