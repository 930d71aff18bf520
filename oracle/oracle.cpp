// Plain CPU oracle for the differentiable Gaussian-splatting hot path.
//
// TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
// benchmark's CPU-baseline leg may load this library.  The HIP product path
// shares no code with it and never calls it.
//
// What it computes (LVI-GS, Section III-B and III-E):
//   * projection of 3D Gaussians to 2D conics: the covariance factorisation
//     Sigma = R S S^T R^T (eq. Sigma) and the EWA projection
//     mu_I = [Q|T] mu_W, Sigma_I = J Q Sigma Q^T J^T (eq. muI);
//   * per-pixel front-to-back compositing of colour, depth and visibility
//     (eqs. Cp, Dp, Vp) with the per-pixel alpha of eq. alpha;
//   * the L1 colour plus lambda_d * L1 depth loss (eqs. L, Lc with the SSIM
//     weight at 0, Ld) and its analytic gradient to every Gaussian parameter;
//   * one Adam step (bias-corrected; the optimiser is not named in the paper,
//     Section III-E, so the usual Adam definition is used).
// The paper leaves thresholds, conventions and constants open; the readings
// used here are the ones listed in the design notes (camera world->camera,
// pixel centres at +0.5, exact Jacobian with a guard-band cull, 0.3 px^2
// low-pass, alpha clamp 0.99, skip below 1/255, stop before T < 1e-4,
// opacity-aware bounding box 2 ln(255 o) + 1, background 0, depth = camera z).
//
// The arithmetic is templated on the real type: float follows the FP32
// specification (the camera transform and the pixel mean use explicit
// correctly-rounded fma and IEEE division, so those values are reproducible
// bit for bit), double gives the reference for gradients.  The sort order of
// records is always the FP32 depth bits, whatever the real type.
//
// Built with -O3 -ffp-contract=off -fno-fast-math (see oracle/build.py).

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------- options
// Precision code of the FP64-values-along-FP32-decisions reference (oracle_backward).
constexpr int PREC_MIXED = 3264;

enum {
  OPT_NEAR = 0, OPT_GUARD, OPT_LOWPASS, OPT_ALPHA_MIN, OPT_ALPHA_MAX, OPT_T_MIN,
  OPT_BG0, OPT_BG1, OPT_BG2, OPT_TILE_W, OPT_TILE_H, OPT_LAMBDA_D, OPT_STOP_NEAR, OPT_LAMBDA_SSIM, OPT_COUNT
};

// stop_near: relative distance of T(1 - alpha) from t_min within which a stop decision counts as near its
// threshold (test excusal only; 1e-5 by default, wider where the compared path multiplies the transmittance
// in another association order).
// lambda_ssim: weight of the SSIM term in eq. Lc (the L1 colour term takes 1 - lambda_ssim).
struct Opts {
  double near_z, guard, lowpass, alpha_min, alpha_max, t_min, bg[3], lambda_d, stop_near, lambda_ssim;
  int tile_w, tile_h;
};

Opts read_opts(const double* o) {
  Opts r;
  r.near_z = o[OPT_NEAR];
  r.guard = o[OPT_GUARD];
  r.lowpass = o[OPT_LOWPASS];
  r.alpha_min = o[OPT_ALPHA_MIN];
  r.alpha_max = o[OPT_ALPHA_MAX];
  r.t_min = o[OPT_T_MIN];
  r.bg[0] = o[OPT_BG0];
  r.bg[1] = o[OPT_BG1];
  r.bg[2] = o[OPT_BG2];
  r.tile_w = (int)o[OPT_TILE_W];
  r.tile_h = (int)o[OPT_TILE_H];
  r.lambda_d = o[OPT_LAMBDA_D];
  r.stop_near = o[OPT_STOP_NEAR];
  r.lambda_ssim = o[OPT_LAMBDA_SSIM];
  return r;
}

// ---------------------------------------------------------------- cameras
// Per view, 22 doubles: R (row-major world->camera rotation, 9), T (3),
// fx, fy, cx, cy, width, height, camera centre in world (3), loss weight.
enum { CAM_R = 0, CAM_T = 9, CAM_FX = 12, CAM_FY, CAM_CX, CAM_CY, CAM_W, CAM_H,
       CAM_POS = 18, CAM_WEIGHT = 21, CAM_COUNT = 22 };

// weight: the view's loss weight w_v; a negative input weight marks an inactive view (reading R26: a schedule
// switches views off), which projects nothing and counts with weight 0.
template <class R>
struct Cam {
  R Rm[9], T[3], fx, fy, cx, cy, pos[3], weight;
  bool active;
  int W, H, tiles_x, tiles_y, tile_offset;
  int64_t pixel_offset;
};

template <class R>
std::vector<Cam<R>> read_cams(const double* c, int V, const Opts& op) {
  std::vector<Cam<R>> cams(V);
  int tile_off = 0;
  int64_t px_off = 0;
  for (int v = 0; v < V; ++v) {
    const double* p = c + (size_t)v * CAM_COUNT;
    Cam<R>& k = cams[v];
    for (int i = 0; i < 9; ++i) k.Rm[i] = (R)p[CAM_R + i];
    for (int i = 0; i < 3; ++i) k.T[i] = (R)p[CAM_T + i];
    k.fx = (R)p[CAM_FX];
    k.fy = (R)p[CAM_FY];
    k.cx = (R)p[CAM_CX];
    k.cy = (R)p[CAM_CY];
    k.W = (int)p[CAM_W];
    k.H = (int)p[CAM_H];
    for (int i = 0; i < 3; ++i) k.pos[i] = (R)p[CAM_POS + i];
    k.active = p[CAM_WEIGHT] >= 0;
    k.weight = k.active ? (R)p[CAM_WEIGHT] : (R)0;
    k.tiles_x = (k.W + op.tile_w - 1) / op.tile_w;
    k.tiles_y = (k.H + op.tile_h - 1) / op.tile_h;
    k.tile_offset = tile_off;
    k.pixel_offset = px_off;
    tile_off += k.tiles_x * k.tiles_y;
    px_off += (int64_t)k.W * k.H;
  }
  return cams;
}

// ---------------------------------------------------------------- small linear algebra
template <class R>
void matmul(const R* A, const R* B, R* C, int n, int k, int m) {  // C[n,m] = A[n,k] B[k,m]
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < m; ++j) {
      R s = 0;
      for (int t = 0; t < k; ++t) s += A[i * k + t] * B[t * m + j];
      C[i * m + j] = s;
    }
}
template <class R>
void transpose(const R* A, R* B, int n, int m) {  // B[m,n] = A[n,m]^T
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < m; ++j) B[j * n + i] = A[i * m + j];
}

// Rotation matrix of a unit quaternion (w, x, y, z): the matrix of v -> q v q*.
template <class R>
void quat_to_rot(const R q[4], R M[9]) {
  R w = q[0], x = q[1], y = q[2], z = q[3];
  M[0] = 1 - 2 * (y * y + z * z); M[1] = 2 * (x * y - w * z); M[2] = 2 * (x * z + w * y);
  M[3] = 2 * (x * y + w * z); M[4] = 1 - 2 * (x * x + z * z); M[5] = 2 * (y * z - w * x);
  M[6] = 2 * (x * z - w * y); M[7] = 2 * (y * z + w * x); M[8] = 1 - 2 * (x * x + y * y);
}
// d M / d q_c for c = w, x, y, z (each a 3x3 matrix), at the unit quaternion q.
template <class R>
void quat_to_rot_jac(const R q[4], R dM[4][9]) {
  R w = q[0], x = q[1], y = q[2], z = q[3];
  R dw[9] = {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0};
  R dx[9] = {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x};
  R dy[9] = {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y};
  R dz[9] = {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0};
  for (int i = 0; i < 9; ++i) { dM[0][i] = dw[i]; dM[1][i] = dx[i]; dM[2][i] = dy[i]; dM[3][i] = dz[i]; }
}

// ---------------------------------------------------------------- spherical harmonics
// Real, orthonormal spherical harmonics in polynomial form:
//   Y_lm = sqrt((2l+1)/2pi) Pi_l^m(z) A_m(x,y)        m > 0
//   Y_l0 = sqrt((2l+1)/4pi) Pi_l^0(z)
//   Y_lm = sqrt((2l+1)/2pi) Pi_l^|m|(z) B_|m|(x,y)    m < 0
// with A_m + i B_m = (x + i y)^m and
//   Pi_l^m(z) = sqrt((l-m)!/(l+m)!) sum_k (-1)^k 2^-l C(l,k) C(2l-2k,l) (l-2k)!/(l-2k-m)! r^2k z^(l-2k-m).
// Index k = l^2 + l + m.  Templated so that a dual-number type gives the
// gradient with respect to the direction.
double fact(int n) { double r = 1; for (int i = 2; i <= n; ++i) r *= i; return r; }
double binom(int n, int k) { return fact(n) / (fact(k) * fact(n - k)); }

template <class T>
T tpow(const T& x, int e) { T r = T(1.0); for (int i = 0; i < e; ++i) r = r * x; return r; }

template <class T, class R>
void sh_basis(int deg, const T& x, const T& y, const T& z, T* Y) {
  const double pi = 3.14159265358979323846;
  T A[4] = {T(1.0), T(0.0), T(0.0), T(0.0)}, B[4] = {T(0.0), T(0.0), T(0.0), T(0.0)};
  for (int m = 1; m <= 3; ++m) {
    A[m] = A[m - 1] * x - B[m - 1] * y;
    B[m] = A[m - 1] * y + B[m - 1] * x;
  }
  T r2 = x * x + y * y + z * z;
  for (int l = 0; l <= deg; ++l)
    for (int m = 0; m <= l; ++m) {
      T P = T(0.0);
      for (int k = 0; k <= (l - m) / 2; ++k) {
        double c = ((k & 1) ? -1.0 : 1.0) * std::ldexp(1.0, -l) * binom(l, k) * binom(2 * l - 2 * k, l) *
                   fact(l - 2 * k) / fact(l - 2 * k - m);
        P = P + T((R)c) * tpow(r2, k) * tpow(z, l - 2 * k - m);
      }
      P = P * T((R)std::sqrt(fact(l - m) / fact(l + m)));
      if (m == 0) {
        Y[l * l + l] = T((R)std::sqrt((2 * l + 1) / (4 * pi))) * P;
      } else {
        T nrm = T((R)std::sqrt((2 * l + 1) / (2 * pi)));
        Y[l * l + l + m] = nrm * P * A[m];
        Y[l * l + l - m] = nrm * P * B[m];
      }
    }
}

// Forward-mode dual number in three directions (value and d/dx, d/dy, d/dz).
struct Dual {
  double v, d[3];
  Dual() : v(0), d{0, 0, 0} {}
  explicit Dual(double c) : v(c), d{0, 0, 0} {}
};
Dual operator+(const Dual& a, const Dual& b) { Dual r; r.v = a.v + b.v; for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
Dual operator-(const Dual& a, const Dual& b) { Dual r; r.v = a.v - b.v; for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
Dual operator*(const Dual& a, const Dual& b) { Dual r; r.v = a.v * b.v; for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }

// ---------------------------------------------------------------- projection
template <class R>
struct Proj {
  bool vis;
  int cull_reason;        // 0 visible, 1 near, 2 guard, 3 opacity, 4 det, 5 empty rect, 6 degenerate quaternion
  double near_margin;     // relative distance of a cull decision quantity to its threshold (FP64)
  R t[3], mx, my, z;      // camera-space centre, pixel mean, depth
  float z32;              // FP32-specification depth, used for the sort key in every precision
  R S[3], qn[4], qnorm, Rq[9], M[9], Sig3[9], J[6], T2[6], A, B, C, det;
  R ca, cb, cc;           // conic (a, b, c): power = -(a dx^2 + c dy^2)/2 - b dx dy
  R o;
  R ext_x, ext_y;
  int px0, px1, py0, py1, tx0, tx1, ty0, ty1;
  double rect_margin;     // distance (px) of the unrounded rectangle bounds to the rounding boundary
  R rgb[3];
  bool pass[3];           // colour clamp: gradient passes iff the pre-clamp value >= 0
  double rgb_margin;      // min |pre-clamp value| over the 3 channels
  R dir[3], dist, Y[16];
};

// Projection of Gaussian g into view cam (Section III-B eq. Sigma and eq. muI; readings R1-R6, R12, R13).
template <class R>
Proj<R> project_one(const double* means, const double* log_scales, const double* quats, const double* opac,
                    const double* sh, int K, int64_t g, const Cam<R>& cam, const Opts& op) {
  Proj<R> p;
  std::memset((void*)&p, 0, sizeof(p));
  p.vis = false;
  p.near_margin = 1e30;
  p.rect_margin = 1e30;
  p.rgb_margin = 1e30;
  if (!cam.active) { p.cull_reason = 7; return p; }  // inactive view (reading R26)
  R mu[3] = {(R)means[g * 3], (R)means[g * 3 + 1], (R)means[g * 3 + 2]};
  // camera transform, op order fixed: t_r = fma(R_r2, mu_z, fma(R_r1, mu_y, fma(R_r0, mu_x, T_r)))
  for (int r = 0; r < 3; ++r)
    p.t[r] = std::fma(cam.Rm[3 * r + 2], mu[2], std::fma(cam.Rm[3 * r + 1], mu[1], std::fma(cam.Rm[3 * r], mu[0], cam.T[r])));
  {
    float mf[3] = {(float)means[g * 3], (float)means[g * 3 + 1], (float)means[g * 3 + 2]};
    float rz[3] = {(float)cam.Rm[6], (float)cam.Rm[7], (float)cam.Rm[8]};
    p.z32 = std::fma(rz[2], mf[2], std::fma(rz[1], mf[1], std::fma(rz[0], mf[0], (float)cam.T[2])));
  }
  const R near_z = (R)op.near_z;
  p.near_margin = std::min(p.near_margin, std::fabs((double)p.t[2] - op.near_z) / op.near_z);
  if (!(p.t[2] >= near_z)) { p.cull_reason = 1; return p; }
  R un = p.t[0] / p.t[2], vn = p.t[1] / p.t[2];
  p.mx = std::fma(cam.fx, un, cam.cx);
  p.my = std::fma(cam.fy, vn, cam.cy);
  p.z = p.t[2];
  // guard band: the pixel mean must lie in the image widened by (guard - 1)/2 of its size per side
  const R gm = ((R)op.guard - (R)1) * (R)0.5;
  const R mxw = gm * (R)cam.W, myw = gm * (R)cam.H;
  const R lox = -mxw, hix = (R)cam.W + mxw, loy = -myw, hiy = (R)cam.H + myw;
  p.near_margin = std::min({p.near_margin, std::fabs((double)p.mx - (double)lox) / cam.W,
                            std::fabs((double)p.mx - (double)hix) / cam.W, std::fabs((double)p.my - (double)loy) / cam.H,
                            std::fabs((double)p.my - (double)hiy) / cam.H});
  if (!(p.mx >= lox && p.mx <= hix && p.my >= loy && p.my <= hiy)) { p.cull_reason = 2; return p; }
  // opacity o = sigmoid(logit)
  p.o = (R)1 / ((R)1 + std::exp(-(R)opac[g]));
  p.near_margin = std::min(p.near_margin, std::fabs((double)p.o - op.alpha_min) / op.alpha_min);
  if (p.o < (R)op.alpha_min) { p.cull_reason = 3; return p; }
  // 3D covariance Sigma = M M^T with M = R(q) diag(S)  (eq. Sigma)
  for (int i = 0; i < 3; ++i) p.S[i] = std::exp((R)log_scales[g * 3 + i]);
  R q[4] = {(R)quats[g * 4], (R)quats[g * 4 + 1], (R)quats[g * 4 + 2], (R)quats[g * 4 + 3]};
  p.qnorm = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  if (!(p.qnorm > 0)) { p.cull_reason = 6; return p; }
  for (int i = 0; i < 4; ++i) p.qn[i] = q[i] / p.qnorm;
  quat_to_rot(p.qn, p.Rq);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) p.M[i * 3 + j] = p.Rq[i * 3 + j] * p.S[j];
  R Mt[9];
  transpose(p.M, Mt, 3, 3);
  matmul(p.M, Mt, p.Sig3, 3, 3, 3);
  // EWA: Sigma_I = (J W) Sigma (J W)^T + lowpass I, exact Jacobian of the pinhole at t  (eq. muI)
  const R tz = p.t[2], tz2 = tz * tz;
  p.J[0] = cam.fx / tz; p.J[1] = 0; p.J[2] = -cam.fx * p.t[0] / tz2;
  p.J[3] = 0; p.J[4] = cam.fy / tz; p.J[5] = -cam.fy * p.t[1] / tz2;
  matmul(p.J, cam.Rm, p.T2, 2, 3, 3);
  R T2t[6], tmp[6], SI[4];
  transpose(p.T2, T2t, 2, 3);
  matmul(p.T2, p.Sig3, tmp, 2, 3, 3);
  matmul(tmp, T2t, SI, 2, 3, 2);
  p.A = SI[0] + (R)op.lowpass;
  p.B = SI[1];
  p.C = SI[3] + (R)op.lowpass;
  p.det = p.A * p.C - p.B * p.B;
  if (!(p.det > 0) || !std::isfinite((double)p.det)) { p.cull_reason = 4; return p; }
  p.ca = p.C / p.det;
  p.cb = -p.B / p.det;
  p.cc = p.A / p.det;
  // opacity-aware extent: outside it alpha < exp(-1/2)/255
  R kp = (R)2 * std::log((R)255 * p.o) + (R)1;
  p.ext_x = std::sqrt(kp * p.A);
  p.ext_y = std::sqrt(kp * p.C);
  R lo_x = std::ceil(p.mx - p.ext_x - (R)0.5), hi_x = std::floor(p.mx + p.ext_x - (R)0.5);
  R lo_y = std::ceil(p.my - p.ext_y - (R)0.5), hi_y = std::floor(p.my + p.ext_y - (R)0.5);
  {
    auto frac_dist = [](double v) { return std::fabs(v - std::nearbyint(v)); };
    p.rect_margin = std::min({frac_dist((double)p.mx - (double)p.ext_x - 0.5), frac_dist((double)p.mx + (double)p.ext_x - 0.5),
                              frac_dist((double)p.my - (double)p.ext_y - 0.5), frac_dist((double)p.my + (double)p.ext_y - 0.5)});
  }
  lo_x = std::min(std::max(lo_x, (R)0), (R)cam.W);
  hi_x = std::min(std::max(hi_x, (R)-1), (R)(cam.W - 1));
  lo_y = std::min(std::max(lo_y, (R)0), (R)cam.H);
  hi_y = std::min(std::max(hi_y, (R)-1), (R)(cam.H - 1));
  p.px0 = (int)lo_x; p.px1 = (int)hi_x; p.py0 = (int)lo_y; p.py1 = (int)hi_y;
  if (p.px0 > p.px1 || p.py0 > p.py1) { p.cull_reason = 5; return p; }
  p.tx0 = p.px0 / op.tile_w; p.tx1 = p.px1 / op.tile_w;
  p.ty0 = p.py0 / op.tile_h; p.ty1 = p.py1 / op.tile_h;
  // colour from spherical harmonics at the viewing direction (Section III-E, reading R6)
  for (int i = 0; i < 3; ++i) p.dir[i] = mu[i] - cam.pos[i];
  p.dist = std::sqrt(p.dir[0] * p.dir[0] + p.dir[1] * p.dir[1] + p.dir[2] * p.dir[2]);
  R d[3] = {p.dir[0] / p.dist, p.dir[1] / p.dist, p.dir[2] / p.dist};
  int deg = (int)std::lround(std::sqrt((double)K)) - 1;
  sh_basis<R, R>(deg, d[0], d[1], d[2], p.Y);
  for (int ch = 0; ch < 3; ++ch) {
    R s = 0;
    for (int k = 0; k < K; ++k) s += (R)sh[(g * K + k) * 3 + ch] * p.Y[k];
    R pre = s + (R)0.5;
    p.rgb_margin = std::min(p.rgb_margin, std::fabs((double)pre));
    p.pass[ch] = pre >= 0;
    p.rgb[ch] = p.pass[ch] ? pre : (R)0;
  }
  p.vis = true;
  return p;
}

uint32_t float_bits(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }

// ---------------------------------------------------------------- binning and sort
struct Bins {
  std::vector<uint64_t> keys;
  std::vector<int64_t> vals;
  std::vector<int64_t> range_lo, range_hi;  // per global tile
};

// Emission in record order (view-major, then Gaussian), then tile row, then tile column;
// key = (global tile << 32) | depth bits; stable sort by key (reading R10).
Bins bin_records(const std::vector<int>& rect /*R*4: tx0,tx1,ty0,ty1*/, const std::vector<uint32_t>& zbits,
                 const std::vector<char>& vis, int64_t N, const std::vector<int>& tiles_x,
                 const std::vector<int>& tile_offset, int total_tiles) {
  Bins b;
  int64_t R = (int64_t)vis.size();
  for (int64_t r = 0; r < R; ++r) {
    if (!vis[r]) continue;
    int v = (int)(r / N);
    for (int ty = rect[r * 4 + 2]; ty <= rect[r * 4 + 3]; ++ty)
      for (int tx = rect[r * 4 + 0]; tx <= rect[r * 4 + 1]; ++tx) {
        uint64_t tile = (uint64_t)(tile_offset[v] + ty * tiles_x[v] + tx);
        b.keys.push_back((tile << 32) | (uint64_t)zbits[r]);
        b.vals.push_back(r);
      }
  }
  std::vector<int64_t> idx(b.keys.size());
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t c) { return b.keys[a] < b.keys[c]; });
  std::vector<uint64_t> k2(idx.size());
  std::vector<int64_t> v2(idx.size());
  for (size_t i = 0; i < idx.size(); ++i) { k2[i] = b.keys[idx[i]]; v2[i] = b.vals[idx[i]]; }
  b.keys.swap(k2);
  b.vals.swap(v2);
  b.range_lo.assign(total_tiles, 0);
  b.range_hi.assign(total_tiles, 0);
  for (size_t i = 0; i < b.keys.size(); ++i) {
    int t = (int)(b.keys[i] >> 32);
    if (i == 0 || (int)(b.keys[i - 1] >> 32) != t) b.range_lo[t] = (int64_t)i;
    if (i + 1 == b.keys.size() || (int)(b.keys[i + 1] >> 32) != t) b.range_hi[t] = (int64_t)i + 1;
  }
  return b;
}

// ---------------------------------------------------------------- compositing
// One record as seen by the compositor.
template <class R>
struct Splat { R mx, my, z, a, b, c, o, rgb[3]; };

struct PixelFlags { bool near; };

template <class R>
struct PixelOut {
  R C[3], D, Vis, T;
  int n_contrib;
  bool near;  // some decision within 1e-5 (relative) of its threshold
};

// Front-to-back compositing of one pixel over an ordered list (eqs. Cp, Dp, Vp, alpha; readings R9, R11).
// If `trace` is given, the contributing records are appended with their alpha, G and T before them.
template <class R>
struct Contrib { int64_t rec; R alpha, G, T; bool clamped; };

// A decision of one record at one pixel lying within its window of the threshold (kinds: bits of NEAR_*).
enum { NEAR_CLAMP = 1, NEAR_SKIP = 2, NEAR_STOP = 4 };
struct NearDec { int64_t rec; int kinds; };

template <class R>
PixelOut<R> composite_pixel(const Splat<R>* recs, const int64_t* order, int64_t n, R px, R py, const Opts& op,
                            std::vector<Contrib<R>>* trace, std::vector<NearDec>* near_recs = nullptr) {
  PixelOut<R> out;
  out.C[0] = out.C[1] = out.C[2] = 0;
  out.D = 0;
  out.Vis = 0;
  out.n_contrib = 0;
  out.near = false;
  R T = 1;
  const R amin = (R)op.alpha_min, amax = (R)op.alpha_max, tmin = (R)op.t_min;
  for (int64_t i = 0; i < n; ++i) {
    const Splat<R>& s = recs[order[i]];
    R dx = s.mx - px, dy = s.my - py;
    R power = (R)-0.5 * (s.a * dx * dx + s.c * dy * dy) - s.b * dx * dy;
    if (power > 0) continue;
    R G = std::exp(power);
    R oG = s.o * G;
    bool clamped = oG > amax;
    R alpha = clamped ? amax : oG;
    int kinds = 0;
    if (std::fabs((double)oG - op.alpha_max) <= 1e-5 * op.alpha_max) kinds |= NEAR_CLAMP;
    if (std::fabs((double)alpha - op.alpha_min) <= 1e-5 * op.alpha_min) kinds |= NEAR_SKIP;
    if (!(alpha < amin) && std::fabs((double)(T * ((R)1 - alpha)) - op.t_min) <= op.stop_near * op.t_min)
      kinds |= NEAR_STOP;
    if (kinds) {
      out.near = true;
      if (near_recs) near_recs->push_back(NearDec{order[i], kinds});
    }
    if (alpha < amin) continue;
    R Tn = T * ((R)1 - alpha);
    if (Tn < tmin) break;
    R w = alpha * T;
    for (int ch = 0; ch < 3; ++ch) out.C[ch] += w * s.rgb[ch];
    out.D += w * s.z;
    out.Vis += w;
    if (trace) trace->push_back(Contrib<R>{order[i], alpha, G, T, clamped});
    T = Tn;
    out.n_contrib++;
  }
  for (int ch = 0; ch < 3; ++ch) out.C[ch] += T * (R)op.bg[ch];
  out.T = T;
  return out;
}

// ---------------------------------------------------------------- full forward state
template <class R>
struct Scene {
  int64_t N;
  int K, V;
  Opts op;
  std::vector<Cam<R>> cams;
  std::vector<Proj<R>> proj;       // [V*N]
  std::vector<Splat<R>> splats;    // [V*N]
  Bins bins;
  int total_tiles;
  int64_t total_px;
};

template <class R>
void build_scene(Scene<R>& sc, const double* means, const double* log_scales, const double* quats, const double* opac,
                 const double* sh, int64_t N, int deg, const double* cams, int V, const double* opts) {
  sc.N = N;
  sc.K = (deg + 1) * (deg + 1);
  sc.V = V;
  sc.op = read_opts(opts);
  sc.cams = read_cams<R>(cams, V, sc.op);
  sc.total_tiles = 0;
  sc.total_px = 0;
  for (auto& c : sc.cams) { sc.total_tiles += c.tiles_x * c.tiles_y; sc.total_px += (int64_t)c.W * c.H; }
  sc.proj.resize((size_t)V * N);
  sc.splats.resize((size_t)V * N);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t r = 0; r < (int64_t)V * N; ++r) {
    int v = (int)(r / N);
    int64_t g = r % N;
    sc.proj[r] = project_one<R>(means, log_scales, quats, opac, sh, sc.K, g, sc.cams[v], sc.op);
    const Proj<R>& p = sc.proj[r];
    Splat<R>& s = sc.splats[r];
    s.mx = p.mx; s.my = p.my; s.z = p.z; s.a = p.ca; s.b = p.cb; s.c = p.cc; s.o = p.o;
    for (int ch = 0; ch < 3; ++ch) s.rgb[ch] = p.rgb[ch];
  }
  std::vector<int> rect((size_t)V * N * 4);
  std::vector<uint32_t> zb((size_t)V * N);
  std::vector<char> vis((size_t)V * N);
  for (int64_t r = 0; r < (int64_t)V * N; ++r) {
    const Proj<R>& p = sc.proj[r];
    rect[r * 4 + 0] = p.tx0; rect[r * 4 + 1] = p.tx1; rect[r * 4 + 2] = p.ty0; rect[r * 4 + 3] = p.ty1;
    zb[r] = float_bits(p.z32);
    vis[r] = p.vis;
  }
  std::vector<int> tx(V), toff(V);
  for (int v = 0; v < V; ++v) { tx[v] = sc.cams[v].tiles_x; toff[v] = sc.cams[v].tile_offset; }
  sc.bins = bin_records(rect, zb, vis, N, tx, toff, sc.total_tiles);
}

// Per-view brute-force order: every visible record of the view, by (FP32 depth bits, record index).
template <class R>
std::vector<int64_t> brute_order(const Scene<R>& sc, int v) {
  std::vector<int64_t> ord;
  for (int64_t g = 0; g < sc.N; ++g)
    if (sc.proj[(int64_t)v * sc.N + g].vis) ord.push_back((int64_t)v * sc.N + g);
  std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
    return float_bits(sc.proj[a].z32) < float_bits(sc.proj[b].z32);
  });
  return ord;
}

// Render every pixel of every view.  mode 0 = brute force (the definition), 1 = tiled lists.
template <class R>
void render_all(const Scene<R>& sc, int mode, std::vector<PixelOut<R>>& out,
                std::vector<std::vector<Contrib<R>>>* traces, std::vector<std::vector<NearDec>>* nears = nullptr) {
  out.resize(sc.total_px);
  if (traces) traces->assign(sc.total_px, {});
  if (nears) nears->assign(sc.total_px, {});
  for (int v = 0; v < sc.V; ++v) {
    const Cam<R>& cam = sc.cams[v];
    std::vector<int64_t> brute;
    if (mode == 0) brute = brute_order(sc, v);
    std::vector<int64_t> vals(sc.bins.vals.begin(), sc.bins.vals.end());
#pragma omp parallel for schedule(dynamic, 4)
    for (int y = 0; y < cam.H; ++y)
      for (int x = 0; x < cam.W; ++x) {
        int64_t pix = cam.pixel_offset + (int64_t)y * cam.W + x;
        const int64_t* ord;
        int64_t n;
        if (mode == 0) {
          ord = brute.data();
          n = (int64_t)brute.size();
        } else {
          int t = cam.tile_offset + (y / sc.op.tile_h) * cam.tiles_x + (x / sc.op.tile_w);
          ord = vals.data() + sc.bins.range_lo[t];
          n = sc.bins.range_hi[t] - sc.bins.range_lo[t];
        }
        out[pix] = composite_pixel<R>(sc.splats.data(), ord, n, (R)x + (R)0.5, (R)y + (R)0.5, sc.op,
                                      traces ? &(*traces)[pix] : nullptr, nears ? &(*nears)[pix] : nullptr);
      }
  }
}

// ---------------------------------------------------------------- loss
}  // namespace
extern "C" double oracle_ssim_plane(const double* x, const double* y, int H, int W, double* map, double* grad);
namespace {

// The SSIM term of eq. Lc for every view, lambda_ssim w_v (1 - mean SSIM_v) (oracle/ssim.cpp), computed in double
// from the colour image `img`; its gradient is added to the colour entries of g.  Returns its value.
template <class R>
double ssim_term(const Scene<R>& sc, const std::vector<PixelOut<R>>& img, const double* tgt_rgb,
                 std::vector<double>& g) {
  const double lam = sc.op.lambda_ssim;
  double L = 0;
  for (int v = 0; v < sc.V; ++v) {
    const Cam<R>& cam = sc.cams[v];
    const int64_t P = (int64_t)cam.W * cam.H, off = cam.pixel_offset;
    std::vector<double> x(P), gr(P);
    double mean = 0;
    for (int ch = 0; ch < 3; ++ch) {
      for (int64_t i = 0; i < P; ++i) x[i] = (double)img[off + i].C[ch];
      mean += oracle_ssim_plane(x.data(), tgt_rgb + 3 * off + ch * P, cam.H, cam.W, nullptr, gr.data()) / 3.0;
      for (int64_t i = 0; i < P; ++i) g[(off + i) * 5 + ch] -= (double)cam.weight * lam / 3.0 * gr[i];
    }
    L += (double)cam.weight * lam * (1.0 - mean);
  }
  return L;
}

// L = sum_v w_v [ (1 - lambda_ssim) mean_{3 P_v} |C - I| + lambda_ssim (1 - SSIM_v)
//                 + lambda_d * mean_{valid} |D - D_lidar| ]  (eqs. L, Lc, Ld; readings R14, R23)
// Returns per-pixel upstream gradients g (5 per pixel: C0..C2, D, V) and the loss value.
// near_sign[pix] has bit ch set (ch = 0..2 colour, 3 depth) where |C - I| is within the window of 0, where
// the sign of the L1 gradient could go either way; gmag (optional) receives the magnitude of each L1 upstream
// gradient entry whatever its sign (the loss weight of that term).  The SSIM term (no discrete decision) is
// computed from ssim_img when given (the FP64 image of the mixed reference), else from img.
template <class R>
double loss_and_grad(const Scene<R>& sc, const std::vector<PixelOut<R>>& img, const double* tgt_rgb,
                     const double* tgt_depth, std::vector<double>& g, std::vector<char>& near_sign,
                     std::vector<double>* gmag = nullptr, const Scene<double>* ssim_sc = nullptr,
                     const std::vector<PixelOut<double>>* ssim_img = nullptr) {
  g.assign((size_t)sc.total_px * 5, 0.0);
  near_sign.assign(sc.total_px, 0);
  if (gmag) gmag->assign((size_t)sc.total_px * 5, 0.0);
  double L = 0;
  for (int v = 0; v < sc.V; ++v) {
    const Cam<R>& cam = sc.cams[v];
    int64_t P = (int64_t)cam.W * cam.H, off = cam.pixel_offset;
    int64_t M = 0;
    for (int64_t i = 0; i < P; ++i) M += tgt_depth[off + i] > 0;
    double wrgb = (double)cam.weight * (1.0 - sc.op.lambda_ssim) / (3.0 * (double)P);
    double wd = M > 0 ? (double)cam.weight * sc.op.lambda_d / (double)M : 0.0;
    for (int64_t i = 0; i < P; ++i) {
      int64_t pix = off + i;
      for (int ch = 0; ch < 3; ++ch) {
        double c = (double)img[pix].C[ch], t = tgt_rgb[3 * off + ch * P + i];
        double e = c - t;
        L += wrgb * std::fabs(e);
        g[pix * 5 + ch] = wrgb * (e > 0 ? 1.0 : (e < 0 ? -1.0 : 0.0));
        if (gmag) (*gmag)[pix * 5 + ch] = wrgb;
        if (std::fabs(e) <= 1e-5) near_sign[pix] |= (char)(1 << ch);
      }
      double dt = tgt_depth[pix];
      if (dt > 0) {
        double e = (double)img[pix].D - dt;
        L += wd * std::fabs(e);
        g[pix * 5 + 3] = wd * (e > 0 ? 1.0 : (e < 0 ? -1.0 : 0.0));
        if (gmag) (*gmag)[pix * 5 + 3] = wd;
        if (std::fabs(e) <= 1e-5 * dt) near_sign[pix] |= (char)8;
      }
    }
  }
  if (sc.op.lambda_ssim > 0) L += ssim_sc ? ssim_term(*ssim_sc, *ssim_img, tgt_rgb, g) : ssim_term(sc, img, tgt_rgb, g);
  return L;
}

// ---------------------------------------------------------------- backward
// Gradient per record: d mu_x, d mu_y, d a, d b, d c, d o, d rgb (3), d z.
// One pixel's share: for each contributing record of its trace (front to back), the 10 partial derivatives of
// the loss through this pixel, handed to emit(record, vals).  g5 = upstream gradients of (C0, C1, C2, D, V).
template <class R, class Emit>
void pixel_backward(const Scene<R>& sc, const std::vector<Contrib<R>>& tr, R T_final, const double* g5, R px, R py,
                    Emit emit) {
  const int n = (int)tr.size();
  if (n == 0) return;
  R gC[3] = {(R)g5[0], (R)g5[1], (R)g5[2]};
  R gD = (R)g5[3], gV = (R)g5[4];
  // suffix sums: what lies behind record i, including the background seen through T_final
  std::vector<R> SC(3 * (n + 1)), SD(n + 1), SV(n + 1);
  for (int ch = 0; ch < 3; ++ch) SC[3 * n + ch] = T_final * (R)sc.op.bg[ch];
  SD[n] = 0;
  SV[n] = 0;
  for (int i = n - 1; i >= 0; --i) {
    const Splat<R>& s = sc.splats[tr[i].rec];
    R w = tr[i].alpha * tr[i].T;
    for (int ch = 0; ch < 3; ++ch) SC[3 * i + ch] = SC[3 * (i + 1) + ch] + w * s.rgb[ch];
    SD[i] = SD[i + 1] + w * s.z;
    SV[i] = SV[i + 1] + w;
  }
  for (int i = 0; i < n; ++i) {
    const Contrib<R>& c = tr[i];
    const Splat<R>& s = sc.splats[c.rec];
    R om = (R)1 - c.alpha;
    // dL/dalpha_i = sum over channels g * (value_i T_i - behind_i / (1 - alpha_i))
    R dalpha = 0;
    for (int ch = 0; ch < 3; ++ch) dalpha += gC[ch] * (s.rgb[ch] * c.T - SC[3 * (i + 1) + ch] / om);
    dalpha += gD * (s.z * c.T - SD[i + 1] / om);
    dalpha += gV * (c.T - SV[i + 1] / om);
    R w = c.alpha * c.T;
    R dx = s.mx - px, dy = s.my - py;
    R d_o = 0, dq = 0;
    if (!c.clamped) { d_o = dalpha * c.G; dq = dalpha * c.alpha; }
    R da = (R)-0.5 * dx * dx * dq, db = -dx * dy * dq, dc = (R)-0.5 * dy * dy * dq;
    R dmx = -(s.a * dx + s.b * dy) * dq, dmy = -(s.c * dy + s.b * dx) * dq;
    const R vals[10] = {dmx, dmy, da, db, dc, d_o, w * gC[0], w * gC[1], w * gC[2], w * gD};
    emit(c.rec, vals);
  }
}

template <class R>
void composite_backward(const Scene<R>& sc, const std::vector<PixelOut<R>>& img,
                        const std::vector<std::vector<Contrib<R>>>& traces, const std::vector<double>& g,
                        std::vector<R>& grec) {
  grec.assign((size_t)sc.V * sc.N * 10, (R)0);
  for (int v = 0; v < sc.V; ++v) {
    const Cam<R>& cam = sc.cams[v];
#pragma omp parallel for schedule(dynamic, 4)
    for (int y = 0; y < cam.H; ++y)
      for (int x = 0; x < cam.W; ++x) {
        int64_t pix = cam.pixel_offset + (int64_t)y * cam.W + x;
        pixel_backward<R>(sc, traces[pix], img[pix].T, &g[pix * 5], (R)x + (R)0.5, (R)y + (R)0.5,
                          [&](int64_t rec, const R* vals) {
                            R* gr = &grec[(size_t)rec * 10];
                            for (int k = 0; k < 10; ++k) {
#pragma omp atomic
                              gr[k] += vals[k];
                            }
                          });
      }
  }
}

// Projection backward of one record, accumulated into the parameter gradients of Gaussian g.
// Chain: conic -> Sigma_I -> (Sigma, J) -> (scale, rotation, t) ; mean_I -> t ; t -> mean ;
// colour -> SH coefficients and view direction -> mean ; opacity -> logit.
template <class R>
void project_backward_one(const Proj<R>& p, const Cam<R>& cam, const double* sh, int K, int64_t g, const R* gr,
                          R* gmean, R* gscale, R* gquat, R* gopac, R* gsh, bool dir_grad = true) {
  // conic (a,b,c) = inverse of [[A,B],[B,C]]; G_K is the gradient w.r.t. the symmetric matrix K
  R Kc[4] = {p.ca, p.cb, p.cb, p.cc};
  R GK[4] = {gr[2], (R)0.5 * gr[3], (R)0.5 * gr[3], gr[4]};
  R tmp[4], GS[4];
  matmul(Kc, GK, tmp, 2, 2, 2);
  matmul(tmp, Kc, GS, 2, 2, 2);
  for (int i = 0; i < 4; ++i) GS[i] = -GS[i];  // dL/dSigma_I (symmetric)
  // Sigma_I = T2 Sigma3 T2^T: G_Sigma3 = T2^T G T2 ; G_T2 = 2 G T2 Sigma3
  R T2t[6], t1[6], GSig3[9], GT2[6];
  transpose(p.T2, T2t, 2, 3);
  matmul(T2t, GS, t1, 3, 2, 2);
  matmul(t1, p.T2, GSig3, 3, 2, 3);
  R t2[6];
  matmul(GS, p.T2, t2, 2, 2, 3);
  matmul(t2, p.Sig3, GT2, 2, 3, 3);
  for (int i = 0; i < 6; ++i) GT2[i] *= 2;
  // T2 = J W: G_J = G_T2 W^T
  R Wt[9], GJ[6];
  transpose(cam.Rm, Wt, 3, 3);
  matmul(GT2, Wt, GJ, 2, 3, 3);
  // J entries as functions of t
  R tx = p.t[0], ty = p.t[1], tz = p.t[2];
  R tz2 = tz * tz, tz3 = tz2 * tz;
  R gt[3] = {0, 0, 0};
  gt[0] += GJ[2] * (-cam.fx / tz2);
  gt[1] += GJ[5] * (-cam.fy / tz2);
  gt[2] += GJ[0] * (-cam.fx / tz2) + GJ[2] * ((R)2 * cam.fx * tx / tz3) + GJ[4] * (-cam.fy / tz2) +
           GJ[5] * ((R)2 * cam.fy * ty / tz3);
  // pixel mean: mu_x = fx tx/tz + cx, mu_y = fy ty/tz + cy ; depth = tz
  gt[0] += gr[0] * cam.fx / tz;
  gt[1] += gr[1] * cam.fy / tz;
  gt[2] += -gr[0] * cam.fx * tx / tz2 - gr[1] * cam.fy * ty / tz2 + gr[9];
  // t = W mu + T
  R gm[3] = {0, 0, 0};
  for (int j = 0; j < 3; ++j)
    for (int i = 0; i < 3; ++i) gm[j] += cam.Rm[i * 3 + j] * gt[i];
  // Sigma3 = M M^T: G_M = 2 G_Sigma3 M ; M = Rq diag(S)
  R GM[9];
  matmul(GSig3, p.M, GM, 3, 3, 3);
  for (int i = 0; i < 9; ++i) GM[i] *= 2;
  for (int j = 0; j < 3; ++j) {
    R dS = 0;
    for (int i = 0; i < 3; ++i) dS += p.Rq[i * 3 + j] * GM[i * 3 + j];
    gscale[j] += dS * p.S[j];  // S = exp(log-scale)
  }
  R GR[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) GR[i * 3 + j] = GM[i * 3 + j] * p.S[j];
  R dM[4][9], gqn[4];
  quat_to_rot_jac(p.qn, dM);
  for (int c = 0; c < 4; ++c) {
    gqn[c] = 0;
    for (int i = 0; i < 9; ++i) gqn[c] += dM[c][i] * GR[i];
  }
  R dotq = gqn[0] * p.qn[0] + gqn[1] * p.qn[1] + gqn[2] * p.qn[2] + gqn[3] * p.qn[3];
  for (int c = 0; c < 4; ++c) gquat[c] += (gqn[c] - p.qn[c] * dotq) / p.qnorm;
  // opacity = sigmoid(logit)
  gopac[0] += gr[5] * p.o * ((R)1 - p.o);
  // colour: rgb_ch = max(0, sum_k f_k,ch Y_k(dir) + 0.5)
  R grgb[3];
  for (int ch = 0; ch < 3; ++ch) grgb[ch] = p.pass[ch] ? gr[6 + ch] : (R)0;
  for (int k = 0; k < K; ++k)
    for (int ch = 0; ch < 3; ++ch) gsh[k * 3 + ch] += grgb[ch] * p.Y[k];
  if (K > 1 && dir_grad) {
    int deg = (int)std::lround(std::sqrt((double)K)) - 1;
    Dual dx, dy, dz;
    dx.v = (double)p.dir[0] / (double)p.dist; dx.d[0] = 1;
    dy.v = (double)p.dir[1] / (double)p.dist; dy.d[1] = 1;
    dz.v = (double)p.dir[2] / (double)p.dist; dz.d[2] = 1;
    Dual Yd[16];
    sh_basis<Dual, double>(deg, dx, dy, dz, Yd);
    R gd[3] = {0, 0, 0};  // dL/d(unit direction)
    for (int k = 0; k < K; ++k)
      for (int ch = 0; ch < 3; ++ch) {
        R f = (R)sh[(g * K + k) * 3 + ch];
        for (int i = 0; i < 3; ++i) gd[i] += grgb[ch] * f * (R)Yd[k].d[i];
      }
    R dn[3] = {p.dir[0] / p.dist, p.dir[1] / p.dist, p.dir[2] / p.dist};
    R dot = gd[0] * dn[0] + gd[1] * dn[1] + gd[2] * dn[2];
    for (int i = 0; i < 3; ++i) gm[i] += (gd[i] - dn[i] * dot) / p.dist;
  }
  for (int i = 0; i < 3; ++i) gmean[i] += gm[i];
}

template <class R>
void project_backward_all(const Scene<R>& sc, const double* sh, const std::vector<R>& grec, double* gmean,
                          double* gscale, double* gquat, double* gopac, double* gsh) {
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t g = 0; g < sc.N; ++g) {
    R gm[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, go[1] = {0};
    std::vector<R> gf((size_t)sc.K * 3, (R)0);
    for (int v = 0; v < sc.V; ++v) {
      int64_t r = (int64_t)v * sc.N + g;
      if (!sc.proj[r].vis) continue;
      project_backward_one<R>(sc.proj[r], sc.cams[v], sh, sc.K, g, &grec[(size_t)r * 10], gm, gs, gq, go, gf.data());
    }
    for (int i = 0; i < 3; ++i) { gmean[g * 3 + i] += gm[i]; gscale[g * 3 + i] += gs[i]; }
    for (int i = 0; i < 4; ++i) gquat[g * 4 + i] += gq[i];
    gopac[g] += go[0];
    for (int i = 0; i < sc.K * 3; ++i) gsh[g * sc.K * 3 + i] += gf[i];
  }
}

// Per-pixel upstream gradients: from the loss when targets are given, else the given image gradients (the
// returned value is then sum g * image, whose gradient they are).
template <class R>
double upstream(const Scene<R>& sc, const std::vector<PixelOut<R>>& img, const double* g_rgb, const double* g_depth,
                const double* g_vis, const double* tgt_rgb, const double* tgt_depth, std::vector<double>& g,
                std::vector<char>& near_sign) {
  if (tgt_rgb) return loss_and_grad<R>(sc, img, tgt_rgb, tgt_depth, g, near_sign);
  near_sign.assign(sc.total_px, 0);
  g.assign((size_t)sc.total_px * 5, 0.0);
  double L = 0;
  for (int v = 0; v < sc.V; ++v) {
    const Cam<R>& cam = sc.cams[v];
    int64_t P = (int64_t)cam.W * cam.H, off = cam.pixel_offset;
    for (int64_t i = 0; i < P; ++i) {
      for (int ch = 0; ch < 3; ++ch) g[(off + i) * 5 + ch] = g_rgb ? g_rgb[3 * off + ch * P + i] : 0.0;
      g[(off + i) * 5 + 3] = g_depth ? g_depth[off + i] : 0.0;
      g[(off + i) * 5 + 4] = g_vis ? g_vis[off + i] : 0.0;
      for (int ch = 0; ch < 3; ++ch) L += g[(off + i) * 5 + ch] * (double)img[off + i].C[ch];
      L += g[(off + i) * 5 + 3] * (double)img[off + i].D + g[(off + i) * 5 + 4] * (double)img[off + i].Vis;
    }
  }
  return L;
}

// ---------------------------------------------------------------- rounding scale of the gradients
// Test tolerance only.  Each gradient entry is a sum over pixels and views of terms that cancel, so an FP32
// evaluation (in any summation order) can be off from the exact value by a small multiple of 2^-24 times the
// sum of the magnitudes of those terms, however small the result.  This computes that sum of magnitudes: the
// per-pixel terms of the compositing backward with every difference replaced by the sum of the magnitudes of
// its operands (the colour, depth and visibility "behind" sums bounded by the pixel's totals, which bounds
// the forward-order form T_i q_i - (S - P_i) / (1 - alpha_i) as well), carried to the parameters through the
// projection backward applied to each unit record gradient and taken entry by entry in absolute value.
constexpr double kOps = 16;
constexpr double kShTermBound = 4;

void composite_backward_abs(const Scene<double>& sc, const std::vector<PixelOut<double>>& img,
                            const std::vector<std::vector<Contrib<double>>>& traces, const std::vector<double>& g,
                            std::vector<double>& arec) {
  arec.assign((size_t)sc.V * sc.N * 10, 0.0);
  for (int v = 0; v < sc.V; ++v) {
    const Cam<double>& cam = sc.cams[v];
#pragma omp parallel for schedule(dynamic, 4)
    for (int y = 0; y < cam.H; ++y)
      for (int x = 0; x < cam.W; ++x) {
        int64_t pix = cam.pixel_offset + (int64_t)y * cam.W + x;
        const PixelOut<double>& o = img[pix];
        double gC[3] = {std::fabs(g[pix * 5 + 0]), std::fabs(g[pix * 5 + 1]), std::fabs(g[pix * 5 + 2])};
        double gD = std::fabs(g[pix * 5 + 3]), gV = std::fabs(g[pix * 5 + 4]);
        double px = x + 0.5, py = y + 0.5;
        const std::vector<Contrib<double>>& tr = traces[pix];
        const double n = (double)tr.size();
        for (size_t i = 0; i < tr.size(); ++i) {
          const Contrib<double>& c = tr[i];
          const Splat<double>& s = sc.splats[c.rec];
          double om = 1.0 - c.alpha;
          // weights: the rounding of T_i grows with the i factors it multiplies, that of a pixel total with its
          // n terms; kOps covers the fixed operation count of each term
          const double wi = (double)i + kOps, wn = n + kOps;
          double dal = 0;
          for (int ch = 0; ch < 3; ++ch) dal += gC[ch] * (wi * std::fabs(s.rgb[ch]) * c.T + wn * std::fabs(o.C[ch]) / om);
          dal += gD * (wi * std::fabs(s.z) * c.T + wn * std::fabs(o.D) / om);
          dal += gV * (wi * c.T + wn * std::fabs(o.Vis) / om);
          double w = wi * c.alpha * c.T;
          double dx = std::fabs(s.mx - px), dy = std::fabs(s.my - py);
          double d_o = 0, dq = 0;
          if (!c.clamped) { d_o = dal * c.G; dq = dal * c.alpha; }
          double vals[10] = {(std::fabs(s.a) * dx + std::fabs(s.b) * dy) * dq,
                             (std::fabs(s.c) * dy + std::fabs(s.b) * dx) * dq,
                             0.5 * dx * dx * dq, dx * dy * dq, 0.5 * dy * dy * dq, d_o,
                             w * gC[0], w * gC[1], w * gC[2], w * gD};
          double* a = &arec[(size_t)c.rec * 10];
          for (int k = 0; k < 10; ++k) {
#pragma omp atomic
            a[k] += vals[k];
          }
        }
      }
  }
}

// Magnitude arithmetic: every operation on the magnitudes of its operands (a - b and a + b both give
// |a| + |b|).  Run through the projection backward it gives, for record-gradient magnitudes, the first-order
// rounding scale of each parameter gradient (the sum of the magnitudes of all the terms the chain adds),
// including the cancellations inside the chain (e.g. the rotation gradient of an isotropic Gaussian, exactly
// zero, whose FP32 evaluation is rounding noise of that size).
struct Mag {
  double v;
  Mag() : v(0) {}
  Mag(double x) : v(std::fabs(x)) {}
  explicit operator double() const { return v; }
};
inline Mag mag_raw(double x) { Mag r; r.v = x; return r; }
inline Mag operator+(Mag a, Mag b) { return mag_raw(a.v + b.v); }
inline Mag operator-(Mag a, Mag b) { return mag_raw(a.v + b.v); }
inline Mag operator*(Mag a, Mag b) { return mag_raw(a.v * b.v); }
inline Mag operator/(Mag a, Mag b) { return mag_raw(a.v / b.v); }
inline Mag operator-(Mag a) { return a; }
inline Mag& operator+=(Mag& a, Mag b) { a.v += b.v; return a; }
inline Mag& operator-=(Mag& a, Mag b) { a.v += b.v; return a; }
inline Mag& operator*=(Mag& a, Mag b) { a.v *= b.v; return a; }

Proj<Mag> mag_of(const Proj<double>& p) {
  Proj<Mag> m;
  m.vis = p.vis; m.cull_reason = p.cull_reason; m.near_margin = p.near_margin; m.z32 = p.z32;
  m.rect_margin = p.rect_margin; m.rgb_margin = p.rgb_margin;
  m.px0 = p.px0; m.px1 = p.px1; m.py0 = p.py0; m.py1 = p.py1; m.tx0 = p.tx0; m.tx1 = p.tx1; m.ty0 = p.ty0; m.ty1 = p.ty1;
  for (int i = 0; i < 3; ++i) { m.t[i] = p.t[i]; m.S[i] = p.S[i]; m.rgb[i] = p.rgb[i]; m.dir[i] = p.dir[i]; m.pass[i] = p.pass[i]; }
  m.mx = p.mx; m.my = p.my; m.z = p.z;
  for (int i = 0; i < 4; ++i) m.qn[i] = p.qn[i];
  m.qnorm = p.qnorm;
  for (int i = 0; i < 9; ++i) { m.Rq[i] = p.Rq[i]; m.M[i] = p.M[i]; m.Sig3[i] = p.Sig3[i]; }
  for (int i = 0; i < 6; ++i) { m.J[i] = p.J[i]; m.T2[i] = p.T2[i]; }
  m.A = p.A; m.B = p.B; m.C = p.C; m.det = p.det; m.ca = p.ca; m.cb = p.cb; m.cc = p.cc; m.o = p.o;
  m.ext_x = p.ext_x; m.ext_y = p.ext_y; m.dist = p.dist;
  for (int i = 0; i < 16; ++i) m.Y[i] = p.Y[i];
  return m;
}

Cam<Mag> mag_of(const Cam<double>& c) {
  Cam<Mag> m;
  for (int i = 0; i < 9; ++i) m.Rm[i] = c.Rm[i];
  for (int i = 0; i < 3; ++i) { m.T[i] = c.T[i]; m.pos[i] = c.pos[i]; }
  m.fx = c.fx; m.fy = c.fy; m.cx = c.cx; m.cy = c.cy; m.weight = c.weight;
  m.W = c.W; m.H = c.H; m.tiles_x = c.tiles_x; m.tiles_y = c.tiles_y; m.tile_offset = c.tile_offset;
  m.pixel_offset = c.pixel_offset;
  return m;
}

void project_backward_abs(const Scene<double>& sc, const double* sh, const std::vector<double>& arec,
                          double* smean, double* sscale, double* squat, double* sopac, double* ssh) {
  const int K = sc.K;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t g = 0; g < sc.N; ++g) {
    std::vector<Mag> fm((size_t)K * 3);
    std::vector<double> f((size_t)K * 3);
    for (int v = 0; v < sc.V; ++v) {
      int64_t r = (int64_t)v * sc.N + g;
      if (!sc.proj[r].vis) continue;
      const double* a = &arec[(size_t)r * 10];
      Mag gm[10];
      bool any = false;
      for (int k = 0; k < 10; ++k) { gm[k] = a[k]; any |= a[k] != 0; }
      if (!any) continue;
      // the whole chain in magnitude arithmetic, except the colour's dependence on the view direction
      Mag m[3], s[3], q[4], o[1];
      std::fill(fm.begin(), fm.end(), Mag());
      project_backward_one<Mag>(mag_of(sc.proj[r]), mag_of(sc.cams[v]), sh, K, g, gm, m, s, q, o, fm.data(), false);
      for (int i = 0; i < 3; ++i) { smean[g * 3 + i] += m[i].v; sscale[g * 3 + i] += s[i].v; }
      for (int i = 0; i < 4; ++i) squat[g * 4 + i] += q[i].v;
      sopac[g] += o[0].v;
      for (int i = 0; i < K * 3; ++i) ssh[g * K * 3 + i] += fm[i].v;
      for (int k = 6; k <= 8; ++k) {
        if (a[k] == 0) continue;
        // the direction term (signed directions needed): each colour's unit gradient through the FP64 chain,
        // taken entry by entry in absolute value
        double e[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        e[k] = 1;
        double dm[3] = {0, 0, 0}, ds[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0}, dop[1] = {0};
        std::fill(f.begin(), f.end(), 0.0);
        project_backward_one<double>(sc.proj[r], sc.cams[v], sh, K, g, e, dm, ds, dq, dop, f.data());
        for (int i = 0; i < 3; ++i) smean[g * 3 + i] += a[k] * std::fabs(dm[i]);
        // the basis values themselves cancel (e.g. x^2 - y^2); on the unit sphere the magnitudes of the terms
        // of each real basis function of degree <= 3 sum to less than 3, so 4 bounds their rounding scale
        for (int j = 0; j < K; ++j) ssh[(g * K + j) * 3 + (k - 6)] += a[k] * kShTermBound;
      }
    }
  }
}

// Record-level bounds carried to the parameters through the projection backward's Jacobian taken entry by
// entry in absolute value: out_param += sum_k |d param gradient / d record partial k| * arec[k].  A bound on
// |J x| for any x with |x_k| <= arec[k], exact when one component dominates.
void project_backward_jac_abs(const Scene<double>& sc, const double* sh, const std::vector<double>& arec,
                              double* omean, double* oscale, double* oquat, double* oopac, double* osh) {
  const int K = sc.K;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t g = 0; g < sc.N; ++g) {
    std::vector<double> f((size_t)K * 3);
    for (int v = 0; v < sc.V; ++v) {
      const int64_t r = (int64_t)v * sc.N + g;
      if (!sc.proj[r].vis) continue;
      const double* a = &arec[(size_t)r * 10];
      for (int k = 0; k < 10; ++k) {
        if (a[k] == 0) continue;
        double e[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        e[k] = 1;
        double dm[3] = {0, 0, 0}, ds[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0}, dop[1] = {0};
        std::fill(f.begin(), f.end(), 0.0);
        project_backward_one<double>(sc.proj[r], sc.cams[v], sh, K, g, e, dm, ds, dq, dop, f.data());
        for (int i = 0; i < 3; ++i) { omean[g * 3 + i] += a[k] * std::fabs(dm[i]); oscale[g * 3 + i] += a[k] * std::fabs(ds[i]); }
        for (int i = 0; i < 4; ++i) oquat[g * 4 + i] += a[k] * std::fabs(dq[i]);
        oopac[g] += a[k] * std::fabs(dop[0]);
        for (int i = 0; i < K * 3; ++i) osh[g * K * 3 + i] += a[k] * std::fabs(f[i]);
      }
    }
  }
}

// ---------------------------------------------------------------- FP64 values along FP32 decisions
// Every discrete choice of the path (cull, tile rectangle, skip, clamp, stop, colour clamp, loss sign) is
// taken by FP32 arithmetic where the path runs in FP32; near a threshold an FP64 evaluation may choose the
// other side and then differs by a whole term, not by rounding.  This reference takes those decisions from
// the FP32 evaluation and computes every value (alpha, G, transmittance, images, gradients) in FP64 along them,
// so a comparison with it measures value error only.
struct Mixed {
  Scene<float> sf;
  Scene<double> sd;  // values; proj[r].vis = visible in both precisions, pass[] taken from FP32
  std::vector<PixelOut<float>> imf;
  std::vector<std::vector<Contrib<float>>> tf;
  std::vector<std::vector<NearDec>> nears;
  std::vector<PixelOut<double>> img;
  std::vector<std::vector<Contrib<double>>> traces;
  std::vector<char> split_vis;  // [V*N] visible in exactly one precision (near its cull threshold)
};

// FP64 values along one pixel's FP32 trace: the same contributing records in the same order with the same
// clamp decisions, alpha, G and transmittance recomputed in FP64.  A record visible in FP32 only is dropped
// (returns false; such records are excused by the callers).
bool values_along(const Scene<double>& sc, const std::vector<Contrib<float>>& tr32, double px, double py,
                  PixelOut<double>& o, std::vector<Contrib<double>>& tr) {
  o.C[0] = o.C[1] = o.C[2] = o.D = o.Vis = 0;
  o.n_contrib = 0;
  o.near = false;
  tr.clear();
  bool whole = true;
  double T = 1;
  const double amax = sc.op.alpha_max;
  for (const Contrib<float>& c : tr32) {
    if (!sc.proj[c.rec].vis) { whole = false; continue; }
    const Splat<double>& s = sc.splats[c.rec];
    double dx = s.mx - px, dy = s.my - py;
    double G = std::exp(-0.5 * (s.a * dx * dx + s.c * dy * dy) - s.b * dx * dy);
    double alpha = c.clamped ? amax : s.o * G;
    double w = alpha * T;
    for (int ch = 0; ch < 3; ++ch) o.C[ch] += w * s.rgb[ch];
    o.D += w * s.z;
    o.Vis += w;
    tr.push_back(Contrib<double>{c.rec, alpha, G, T, c.clamped});
    T *= 1.0 - alpha;
    o.n_contrib++;
  }
  for (int ch = 0; ch < 3; ++ch) o.C[ch] += T * sc.op.bg[ch];
  o.T = T;
  return whole;
}

void build_mixed(Mixed& m, const double* means, const double* log_scales, const double* quats, const double* opac,
                 const double* sh, int64_t N, int deg, const double* cams, int V, const double* opts) {
  build_scene<float>(m.sf, means, log_scales, quats, opac, sh, N, deg, cams, V, opts);
  build_scene<double>(m.sd, means, log_scales, quats, opac, sh, N, deg, cams, V, opts);
  render_all<float>(m.sf, 1, m.imf, &m.tf, &m.nears);
  const int64_t R = (int64_t)V * N;
  m.split_vis.assign(R, 0);
  for (int64_t r = 0; r < R; ++r) {
    Proj<double>& pd = m.sd.proj[r];
    const Proj<float>& pf = m.sf.proj[r];
    m.split_vis[r] = pd.vis != pf.vis;
    pd.vis = pd.vis && pf.vis;
    for (int ch = 0; ch < 3; ++ch) pd.pass[ch] = pf.pass[ch];
    if (pd.vis)
      for (int ch = 0; ch < 3; ++ch) m.sd.splats[r].rgb[ch] = pd.pass[ch] ? pd.rgb[ch] : 0.0;
  }
  const Scene<double>& sc = m.sd;
  m.img.resize(sc.total_px);
  m.traces.assign(sc.total_px, {});
  for (int v = 0; v < V; ++v) {
    const Cam<double>& cam = sc.cams[v];
#pragma omp parallel for schedule(dynamic, 4)
    for (int y = 0; y < cam.H; ++y)
      for (int x = 0; x < cam.W; ++x) {
        int64_t pix = cam.pixel_offset + (int64_t)y * cam.W + x;
        const bool whole = values_along(sc, m.tf[pix], x + 0.5, y + 0.5, m.img[pix], m.traces[pix]);
        m.img[pix].near = m.imf[pix].near || !whole;
      }
  }
}

// The FP32 trace of one pixel with one near decision of record `frec` taken the other way (kind: one NEAR_*
// bit): the clamp of alpha at alpha_max, the skip below alpha_min, or the stop before T < t_min.  Every other
// decision is evaluated as usual, so the consequences of the flip (a later stop moving) follow.
std::vector<Contrib<float>> trace_flipped(const Splat<float>* recs, const int64_t* order, int64_t n, float px,
                                          float py, const Opts& op, int64_t frec, int kind) {
  std::vector<Contrib<float>> tr;
  float T = 1;
  const float amin = (float)op.alpha_min, amax = (float)op.alpha_max, tmin = (float)op.t_min;
  for (int64_t i = 0; i < n; ++i) {
    const Splat<float>& s = recs[order[i]];
    const bool here = order[i] == frec;
    float dx = s.mx - px, dy = s.my - py;
    float power = -0.5f * (s.a * dx * dx + s.c * dy * dy) - s.b * dx * dy;
    if (power > 0) continue;
    float G = std::exp(power);
    float oG = s.o * G;
    bool clamped = oG > amax;
    if (here && (kind & NEAR_CLAMP)) clamped = !clamped;
    float alpha = clamped ? amax : oG;
    bool skip = alpha < amin;
    if (here && (kind & NEAR_SKIP)) skip = !skip;
    if (skip) continue;
    float Tn = T * (1.f - alpha);
    bool stop = Tn < tmin;
    if (here && (kind & NEAR_STOP)) stop = !stop;
    if (stop) break;
    tr.push_back(Contrib<float>{order[i], alpha, G, T, clamped});
    T = Tn;
  }
  return tr;
}

// The tile list of pixel (x, y) of view v: [*ord, *ord + *n).
template <class R>
void pixel_list(const Scene<R>& sc, const std::vector<int64_t>& vals, int v, int x, int y, const int64_t** ord,
                int64_t* n) {
  const Cam<R>& cam = sc.cams[v];
  const int t = cam.tile_offset + (y / sc.op.tile_h) * cam.tiles_x + (x / sc.op.tile_w);
  *ord = vals.data() + sc.bins.range_lo[t];
  *n = sc.bins.range_hi[t] - sc.bins.range_lo[t];
}

// Flip allowance of the gradient reference (test tolerance).  A decision within its window of a threshold (a
// skip, clamp or stop, or the sign of an L1 term) may be taken the other way by an FP32 evaluation whose
// rounding differs from the oracle's; the gradient then changes by a whole term, not by rounding.  For every
// such decision, per record, the absolute change of the pixel's 10 record partials when that decision alone is
// flipped (the pixel recomputed along the flipped FP32 decisions with FP64 values; a flipped L1 sign changes
// that term's upstream gradient by twice its weight), summed over the decisions: `allow` [V*N*10].
void flip_allowance(const Mixed& m, const std::vector<double>& g, const std::vector<char>& near_sign,
                    const std::vector<double>& gmag, std::vector<double>& allow) {
  const Scene<double>& sc = m.sd;
  const Scene<float>& sf = m.sf;
  allow.assign((size_t)sc.V * sc.N * 10, 0.0);
  std::vector<int64_t> vals(sf.bins.vals.begin(), sf.bins.vals.end());
  auto add = [&](int64_t rec, const double* d, double f) {
    double* a = &allow[(size_t)rec * 10];
    for (int k = 0; k < 10; ++k) {
      const double x = f * std::fabs(d[k]);
#pragma omp atomic
      a[k] += x;
    }
  };
  for (int v = 0; v < sc.V; ++v) {
    const Cam<double>& cam = sc.cams[v];
#pragma omp parallel for schedule(dynamic, 4)
    for (int y = 0; y < cam.H; ++y)
      for (int x = 0; x < cam.W; ++x) {
        const int64_t pix = cam.pixel_offset + (int64_t)y * cam.W + x;
        const char ns = gmag.empty() ? 0 : near_sign[pix];
        if (m.nears[pix].empty() && !ns) continue;
        const double px = x + 0.5, py = y + 0.5;
        // L1 signs: the upstream gradient of the term changes by twice its weight; the partials are linear in it
        for (int ch = 0; ch < 4; ++ch) {
          if (!((ns >> ch) & 1)) continue;
          double g5[5] = {0, 0, 0, 0, 0};
          g5[ch] = gmag[pix * 5 + ch];
          pixel_backward<double>(sc, m.traces[pix], m.img[pix].T, g5, px, py,
                                 [&](int64_t rec, const double* d) { add(rec, d, 2.0); });
        }
        if (m.nears[pix].empty()) continue;
        // the pixel's partials along the oracle's decisions
        std::vector<std::pair<int64_t, std::array<double, 10>>> base;
        pixel_backward<double>(sc, m.traces[pix], m.img[pix].T, &g[pix * 5], px, py,
                               [&](int64_t rec, const double* d) {
                                 std::array<double, 10> a;
                                 for (int k = 0; k < 10; ++k) a[k] = d[k];
                                 base.emplace_back(rec, a);
                               });
        std::sort(base.begin(), base.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
        const int64_t* ord;
        int64_t n;
        pixel_list(sf, vals, v, x, y, &ord, &n);
        for (const NearDec& nd : m.nears[pix])
          for (int kind = NEAR_CLAMP; kind <= NEAR_STOP; kind <<= 1) {
            if (!(nd.kinds & kind)) continue;
            std::vector<Contrib<float>> tf = trace_flipped(sf.splats.data(), ord, n, (float)px, (float)py, sf.op,
                                                           nd.rec, kind);
            PixelOut<double> o;
            std::vector<Contrib<double>> tr;
            values_along(sc, tf, px, py, o, tr);
            std::vector<std::pair<int64_t, std::array<double, 10>>> alt;
            pixel_backward<double>(sc, tr, o.T, &g[pix * 5], px, py, [&](int64_t rec, const double* d) {
              std::array<double, 10> a;
              for (int k = 0; k < 10; ++k) a[k] = d[k];
              alt.emplace_back(rec, a);
            });
            std::sort(alt.begin(), alt.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
            // |alt - base| over the union of the two record sets
            size_t i = 0, j = 0;
            while (i < base.size() || j < alt.size()) {
              double d[10];
              int64_t rec;
              if (j == alt.size() || (i < base.size() && base[i].first < alt[j].first)) {
                rec = base[i].first;
                for (int k = 0; k < 10; ++k) d[k] = base[i].second[k];
                ++i;
              } else if (i == base.size() || alt[j].first < base[i].first) {
                rec = alt[j].first;
                for (int k = 0; k < 10; ++k) d[k] = alt[j].second[k];
                ++j;
              } else {
                rec = base[i].first;
                for (int k = 0; k < 10; ++k) d[k] = alt[j].second[k] - base[i].second[k];
                ++i;
                ++j;
              }
              add(rec, d, 1.0);
            }
          }
      }
  }
}

// Upstream gradients for the mixed reference: loss signs from the FP32 image, loss value from the FP64 one.
double mixed_upstream(const Mixed& m, const double* g_rgb, const double* g_depth, const double* g_vis,
                      const double* tgt_rgb, const double* tgt_depth, std::vector<double>& g,
                      std::vector<char>& near_sign, std::vector<double>* gmag = nullptr) {
  if (!tgt_rgb) return upstream<double>(m.sd, m.img, g_rgb, g_depth, g_vis, tgt_rgb, tgt_depth, g, near_sign);
  std::vector<double> g64;
  std::vector<char> ns64;
  double L = loss_and_grad<double>(m.sd, m.img, tgt_rgb, tgt_depth, g64, ns64);
  loss_and_grad<float>(m.sf, m.imf, tgt_rgb, tgt_depth, g, near_sign, gmag, &m.sd, &m.img);
  return L;
}

double backward_mixed(const double* means, const double* log_scales, const double* quats, const double* opac,
                      const double* sh, int64_t N, int deg, const double* cams, int V, const double* opts,
                      const double* g_rgb, const double* g_depth, const double* g_vis, const double* tgt_rgb,
                      const double* tgt_depth, double* gmean, double* gscale, double* gquat, double* gopac,
                      double* gsh, int8_t* excused_gauss, int64_t* n_near_pixels, double* rgb, double* depth,
                      double* vis, double* const* allow_out = nullptr) {
  Mixed m;
  build_mixed(m, means, log_scales, quats, opac, sh, N, deg, cams, V, opts);
  std::vector<double> g, gmag;
  std::vector<char> near_sign;
  double L = mixed_upstream(m, g_rgb, g_depth, g_vis, tgt_rgb, tgt_depth, g, near_sign, &gmag);
  std::vector<double> grec;
  composite_backward<double>(m.sd, m.img, m.traces, g, grec);
  project_backward_all<double>(m.sd, sh, grec, gmean, gscale, gquat, gopac, gsh);
  if (allow_out) {
    // per-parameter flip allowance: the record allowances carried through the projection backward's Jacobian
    std::vector<double> arec;
    flip_allowance(m, g, near_sign, gmag, arec);
    const int K = m.sd.K;
    std::memset(allow_out[0], 0, sizeof(double) * 3 * N);
    std::memset(allow_out[1], 0, sizeof(double) * 3 * N);
    std::memset(allow_out[2], 0, sizeof(double) * 4 * N);
    std::memset(allow_out[3], 0, sizeof(double) * N);
    std::memset(allow_out[4], 0, sizeof(double) * 3 * K * N);
    project_backward_jac_abs(m.sd, sh, arec, allow_out[0], allow_out[1], allow_out[2], allow_out[3],
                             allow_out[4]);
  }
  // Excusal, judged on the FP32 evaluation (whose rounding the compared path shares up to the order of
  // operations): Gaussians visible in one precision only or with a cull or colour-clamp decision near its
  // threshold; without the flip allowance also every record with a near decision at a pixel and every
  // contributor of such a pixel.
  int64_t nn = 0;
  for (int64_t pix = 0; pix < m.sd.total_px; ++pix) nn += (m.img[pix].near || near_sign[pix]) ? 1 : 0;
  if (excused_gauss) {
    std::memset(excused_gauss, 0, (size_t)N);
    if (!allow_out)
      for (int64_t pix = 0; pix < m.sd.total_px; ++pix) {
        if (!(m.img[pix].near || near_sign[pix])) continue;
        for (const auto& c : m.tf[pix]) excused_gauss[c.rec % N] = 1;
        for (const NearDec& d : m.nears[pix]) excused_gauss[d.rec % N] = 1;
      }
    for (int64_t r = 0; r < (int64_t)V * N; ++r) {
      const Proj<float>& p = m.sf.proj[r];
      if (m.split_vis[r] || p.near_margin <= 1e-5 || (p.vis && p.rgb_margin <= 1e-5)) excused_gauss[r % N] = 1;
    }
  }
  if (n_near_pixels) *n_near_pixels = nn;
  if (rgb) {
    for (int v = 0; v < V; ++v) {
      const Cam<double>& cam = m.sd.cams[v];
      int64_t P = (int64_t)cam.W * cam.H, off = cam.pixel_offset;
      for (int64_t i = 0; i < P; ++i) {
        for (int ch = 0; ch < 3; ++ch) rgb[3 * off + ch * P + i] = m.img[off + i].C[ch];
        depth[off + i] = m.img[off + i].D;
        vis[off + i] = m.img[off + i].Vis;
      }
    }
  }
  return L;
}

template <class R>
int forward_impl(const double* means, const double* log_scales, const double* quats, const double* opac,
                 const double* sh, int64_t N, int deg, const double* cams, int V, const double* opts, int mode,
                 double* rgb, double* depth, double* vis, double* final_T, int32_t* n_contrib, int8_t* near) {
  Scene<R> sc;
  build_scene<R>(sc, means, log_scales, quats, opac, sh, N, deg, cams, V, opts);
  std::vector<PixelOut<R>> img;
  render_all<R>(sc, mode, img, nullptr);
  for (int v = 0; v < V; ++v) {
    const Cam<R>& cam = sc.cams[v];
    int64_t P = (int64_t)cam.W * cam.H, off = cam.pixel_offset;
    for (int64_t i = 0; i < P; ++i) {
      const PixelOut<R>& o = img[off + i];
      for (int ch = 0; ch < 3; ++ch) rgb[3 * off + ch * P + i] = (double)o.C[ch];
      depth[off + i] = (double)o.D;
      vis[off + i] = (double)o.Vis;
      if (final_T) final_T[off + i] = (double)o.T;
      if (n_contrib) n_contrib[off + i] = o.n_contrib;
      if (near) near[off + i] = o.near;
    }
  }
  return 0;
}

template <class R>
double backward_impl(const double* means, const double* log_scales, const double* quats, const double* opac,
                     const double* sh, int64_t N, int deg, const double* cams, int V, const double* opts,
                     const double* g_rgb, const double* g_depth, const double* g_vis, const double* tgt_rgb,
                     const double* tgt_depth, double* gmean, double* gscale, double* gquat, double* gopac, double* gsh,
                     int8_t* excused_gauss, int64_t* n_near_pixels, double* rgb, double* depth, double* vis) {
  Scene<R> sc;
  build_scene<R>(sc, means, log_scales, quats, opac, sh, N, deg, cams, V, opts);
  std::vector<PixelOut<R>> img;
  std::vector<std::vector<Contrib<R>>> traces;
  std::vector<std::vector<NearDec>> nears;
  render_all<R>(sc, 1, img, &traces, &nears);
  std::vector<double> g;
  std::vector<char> near_sign;
  double L = upstream<R>(sc, img, g_rgb, g_depth, g_vis, tgt_rgb, tgt_depth, g, near_sign);
  std::vector<R> grec;
  composite_backward<R>(sc, img, traces, g, grec);
  project_backward_all<R>(sc, sh, grec, gmean, gscale, gquat, gopac, gsh);
  // Excusal: at a pixel with a decision within 1e-5 of its threshold (a skip, clamp or stop, or the sign of
  // its loss), the records with that decision and every contributor of the pixel; plus Gaussians with a
  // cull or colour-clamp decision near its threshold.
  int64_t nn = 0;
  if (excused_gauss) {
    std::memset(excused_gauss, 0, (size_t)N);
    for (int64_t pix = 0; pix < sc.total_px; ++pix) {
      bool nr = img[pix].near || near_sign[pix];
      if (!nr) continue;
      ++nn;
      for (const auto& c : traces[pix]) excused_gauss[c.rec % N] = 1;
      for (const NearDec& d : nears[pix]) excused_gauss[d.rec % N] = 1;
    }
    for (int64_t r = 0; r < (int64_t)V * N; ++r) {
      const Proj<R>& p = sc.proj[r];
      if (p.near_margin <= 1e-5 || (p.vis && p.rgb_margin <= 1e-5)) excused_gauss[r % N] = 1;
    }
  }
  if (n_near_pixels) *n_near_pixels = nn;
  if (rgb) {
    for (int v = 0; v < V; ++v) {
      const Cam<R>& cam = sc.cams[v];
      int64_t P = (int64_t)cam.W * cam.H, off = cam.pixel_offset;
      for (int64_t i = 0; i < P; ++i) {
        for (int ch = 0; ch < 3; ++ch) rgb[3 * off + ch * P + i] = (double)img[off + i].C[ch];
        depth[off + i] = (double)img[off + i].D;
        vis[off + i] = (double)img[off + i].Vis;
      }
    }
  }
  return L;
}

}  // namespace

// ======================================================================== C ABI (for ctypes)
extern "C" {

int oracle_version(void) { return 1; }

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_quat_to_rot(const double* q, double* M) { quat_to_rot<double>(q, M); }

// Real SH basis values (K = (deg+1)^2) at the unit direction d; optionally d Y / d direction [K,3].
void oracle_sh_basis(int deg, const double* d, double* Y, double* dY) {
  Dual x, y, z;
  x.v = d[0]; x.d[0] = 1;
  y.v = d[1]; y.d[1] = 1;
  z.v = d[2]; z.d[2] = 1;
  Dual Yd[16];
  sh_basis<Dual, double>(deg, x, y, z, Yd);
  int K = (deg + 1) * (deg + 1);
  for (int k = 0; k < K; ++k) {
    Y[k] = Yd[k].v;
    if (dY)
      for (int i = 0; i < 3; ++i) dY[k * 3 + i] = Yd[k].d[i];
  }
}

// Projection of every (view, Gaussian) record.  prec 32 = FP32 specification, 64 = FP64.
// Outputs are dense over r = v*N + g.
int oracle_project(int prec, const double* means, const double* log_scales, const double* quats, const double* opac,
                   const double* sh, int64_t N, int deg, const double* cams, int V, const double* opts,
                   int32_t* visible, int32_t* cull_reason, double* mean2d, double* z, uint32_t* zbits32,
                   double* conic, double* opacity, double* rgb, int32_t* pxrect, int32_t* tilerect,
                   double* rect_margin, double* near_margin, int32_t* pass_mask) {
  auto run = [&](auto tag) {
    using R = decltype(tag);
    Opts op = read_opts(opts);
    std::vector<Cam<R>> cs = read_cams<R>(cams, V, op);
    int K = (deg + 1) * (deg + 1);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t r = 0; r < (int64_t)V * N; ++r) {
      int v = (int)(r / N);
      int64_t g = r % N;
      Proj<R> p = project_one<R>(means, log_scales, quats, opac, sh, K, g, cs[v], op);
      visible[r] = p.vis;
      cull_reason[r] = p.cull_reason;
      mean2d[r * 2] = (double)p.mx; mean2d[r * 2 + 1] = (double)p.my;
      z[r] = (double)p.z;
      zbits32[r] = float_bits(p.z32);
      conic[r * 3] = (double)p.ca; conic[r * 3 + 1] = (double)p.cb; conic[r * 3 + 2] = (double)p.cc;
      opacity[r] = (double)p.o;
      for (int ch = 0; ch < 3; ++ch) rgb[r * 3 + ch] = (double)p.rgb[ch];
      pxrect[r * 4] = p.px0; pxrect[r * 4 + 1] = p.px1; pxrect[r * 4 + 2] = p.py0; pxrect[r * 4 + 3] = p.py1;
      tilerect[r * 4] = p.tx0; tilerect[r * 4 + 1] = p.tx1; tilerect[r * 4 + 2] = p.ty0; tilerect[r * 4 + 3] = p.ty1;
      rect_margin[r] = p.rect_margin;
      near_margin[r] = p.near_margin;
      pass_mask[r] = (p.pass[0] ? 1 : 0) | (p.pass[1] ? 2 : 0) | (p.pass[2] ? 4 : 0);
    }
  };
  if (prec == 32) run(float{}); else run(double{});
  return 0;
}

// Binning of given records: tile rectangles [R,4] (tx0, tx1, ty0, ty1), FP32 depth bits, visibility.
// Records are r = v*N + g.  Returns the instance count; writes at most `capacity` pairs.
int64_t oracle_bin(const int32_t* tilerect, const uint32_t* zbits, const int32_t* visible, int64_t N, int V,
                   const int32_t* tiles_x, const int32_t* tile_offset, int total_tiles, uint64_t* keys,
                   int64_t* vals, int64_t capacity, int64_t* range_lo, int64_t* range_hi) {
  int64_t R = (int64_t)V * N;
  std::vector<int> rect(tilerect, tilerect + R * 4);
  std::vector<uint32_t> zb(zbits, zbits + R);
  std::vector<char> vis(R);
  for (int64_t r = 0; r < R; ++r) vis[r] = visible[r] != 0;
  std::vector<int> tx(tiles_x, tiles_x + V), to(tile_offset, tile_offset + V);
  Bins b = bin_records(rect, zb, vis, N, tx, to, total_tiles);
  int64_t I = (int64_t)b.keys.size();
  for (int64_t i = 0; i < I && i < capacity; ++i) { keys[i] = b.keys[i]; vals[i] = b.vals[i]; }
  for (int t = 0; t < total_tiles; ++t) { range_lo[t] = b.range_lo[t]; range_hi[t] = b.range_hi[t]; }
  return I;
}

// Compositing of given records (per record: mean2d[2], z, conic[3], opacity, rgb[3], tile rect[4], visible).
// mode 0 = brute force over every visible record of the view, 1 = tiled lists.  FP32 or FP64.
int oracle_composite(int prec, int mode, const double* mean2d, const double* z, const uint32_t* zbits,
                     const double* conic, const double* opacity, const double* rgbrec, const int32_t* tilerect,
                     const int32_t* visible, int64_t N, const double* cams, int V, const double* opts, double* rgb,
                     double* depth, double* vis, double* final_T, int32_t* n_contrib, int8_t* near) {
  auto run = [&](auto tag) {
    using R = decltype(tag);
    Scene<R> sc;
    sc.N = N;
    sc.K = 1;
    sc.V = V;
    sc.op = read_opts(opts);
    sc.cams = read_cams<R>(cams, V, sc.op);
    sc.total_tiles = 0;
    sc.total_px = 0;
    for (auto& c : sc.cams) { sc.total_tiles += c.tiles_x * c.tiles_y; sc.total_px += (int64_t)c.W * c.H; }
    int64_t Rn = (int64_t)V * N;
    sc.proj.resize(Rn);
    sc.splats.resize(Rn);
    std::vector<int> rect(Rn * 4);
    std::vector<uint32_t> zb(zbits, zbits + Rn);
    std::vector<char> vv(Rn);
    for (int64_t r = 0; r < Rn; ++r) {
      Splat<R>& s = sc.splats[r];
      s.mx = (R)mean2d[r * 2]; s.my = (R)mean2d[r * 2 + 1]; s.z = (R)z[r];
      s.a = (R)conic[r * 3]; s.b = (R)conic[r * 3 + 1]; s.c = (R)conic[r * 3 + 2];
      s.o = (R)opacity[r];
      for (int ch = 0; ch < 3; ++ch) s.rgb[ch] = (R)rgbrec[r * 3 + ch];
      sc.proj[r].vis = visible[r] != 0;
      float zf;
      std::memcpy(&zf, &zbits[r], 4);
      sc.proj[r].z32 = zf;
      for (int k = 0; k < 4; ++k) rect[r * 4 + k] = tilerect[r * 4 + k];
      vv[r] = visible[r] != 0;
    }
    std::vector<int> tx(V), to(V);
    for (int v = 0; v < V; ++v) { tx[v] = sc.cams[v].tiles_x; to[v] = sc.cams[v].tile_offset; }
    sc.bins = bin_records(rect, zb, vv, N, tx, to, sc.total_tiles);
    std::vector<PixelOut<R>> img;
    render_all<R>(sc, mode, img, nullptr);
    for (int v = 0; v < V; ++v) {
      const Cam<R>& cam = sc.cams[v];
      int64_t P = (int64_t)cam.W * cam.H, off = cam.pixel_offset;
      for (int64_t i = 0; i < P; ++i) {
        const PixelOut<R>& o = img[off + i];
        for (int ch = 0; ch < 3; ++ch) rgb[3 * off + ch * P + i] = (double)o.C[ch];
        depth[off + i] = (double)o.D;
        vis[off + i] = (double)o.Vis;
        if (final_T) final_T[off + i] = (double)o.T;
        if (n_contrib) n_contrib[off + i] = o.n_contrib;
        if (near) near[off + i] = o.near;
      }
    }
  };
  if (prec == 32) run(float{}); else run(double{});
  return 0;
}

// End-to-end forward from parameters.  Images are concatenated over views: rgb planar [3,H,W] per view.
int oracle_forward(int prec, int mode, const double* means, const double* log_scales, const double* quats,
                   const double* opac, const double* sh, int64_t N, int deg, const double* cams, int V,
                   const double* opts, double* rgb, double* depth, double* vis, double* final_T, int32_t* n_contrib,
                   int8_t* near) {
  if (prec == 32)
    return forward_impl<float>(means, log_scales, quats, opac, sh, N, deg, cams, V, opts, mode, rgb, depth, vis,
                               final_T, n_contrib, near);
  return forward_impl<double>(means, log_scales, quats, opac, sh, N, deg, cams, V, opts, mode, rgb, depth, vis,
                              final_T, n_contrib, near);
}

// Loss and analytic gradient.  Either targets (tgt_rgb, tgt_depth; 0 = no LiDAR depth) or upstream
// image gradients (g_rgb, g_depth, g_vis; any may be NULL) are given.  Gradients are accumulated (+=).
double oracle_backward(int prec, const double* means, const double* log_scales, const double* quats,
                       const double* opac, const double* sh, int64_t N, int deg, const double* cams, int V,
                       const double* opts, const double* g_rgb, const double* g_depth, const double* g_vis,
                       const double* tgt_rgb, const double* tgt_depth, double* gmean, double* gscale, double* gquat,
                       double* gopac, double* gsh, int8_t* excused, int64_t* n_near_pixels, double* rgb,
                       double* depth, double* vis) {
  if (prec == PREC_MIXED)
    return backward_mixed(means, log_scales, quats, opac, sh, N, deg, cams, V, opts, g_rgb, g_depth, g_vis, tgt_rgb,
                          tgt_depth, gmean, gscale, gquat, gopac, gsh, excused, n_near_pixels, rgb, depth, vis);
  if (prec == 32)
    return backward_impl<float>(means, log_scales, quats, opac, sh, N, deg, cams, V, opts, g_rgb, g_depth, g_vis,
                                tgt_rgb, tgt_depth, gmean, gscale, gquat, gopac, gsh, excused, n_near_pixels, rgb,
                                depth, vis);
  return backward_impl<double>(means, log_scales, quats, opac, sh, N, deg, cams, V, opts, g_rgb, g_depth, g_vis,
                               tgt_rgb, tgt_depth, gmean, gscale, gquat, gopac, gsh, excused, n_near_pixels, rgb,
                               depth, vis);
}

// The gradient reference of the tests: FP64 values along FP32 decisions (as oracle_backward with the mixed
// precision code) plus, per gradient entry, the flip allowance (allow_*, shapes of the gradients): the change
// the entry would see if one decision within its window of a threshold were taken the other way, summed over
// such decisions.  `excused` then marks only Gaussians with a cull or colour-clamp decision near its threshold
// or visible in one precision only.
double oracle_reference(const double* means, const double* log_scales, const double* quats, const double* opac,
                        const double* sh, int64_t N, int deg, const double* cams, int V, const double* opts,
                        const double* g_rgb, const double* g_depth, const double* g_vis, const double* tgt_rgb,
                        const double* tgt_depth, double* gmean, double* gscale, double* gquat, double* gopac,
                        double* gsh, double* amean, double* ascale, double* aquat, double* aopac, double* ash,
                        int8_t* excused, int64_t* n_near_pixels, double* rgb, double* depth, double* vis) {
  double* const allow[5] = {amean, ascale, aquat, aopac, ash};
  return backward_mixed(means, log_scales, quats, opac, sh, N, deg, cams, V, opts, g_rgb, g_depth, g_vis, tgt_rgb,
                        tgt_depth, gmean, gscale, gquat, gopac, gsh, excused, n_near_pixels, rgb, depth, vis, allow);
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

// Loss value only (FP64), for finite differences.
// Sum of the magnitudes of the terms of every gradient entry (FP64 along FP32 decisions; zeroed here).
// Same inputs as oracle_backward; outputs have the shapes of the gradients.
void oracle_gradient_scale(const double* means, const double* log_scales, const double* quats, const double* opac,
                           const double* sh, int64_t N, int deg, const double* cams, int V, const double* opts,
                           const double* g_rgb, const double* g_depth, const double* g_vis, const double* tgt_rgb,
                           const double* tgt_depth, double* smean, double* sscale, double* squat, double* sopac,
                           double* ssh) {
  Mixed m;
  build_mixed(m, means, log_scales, quats, opac, sh, N, deg, cams, V, opts);
  std::vector<double> g;
  std::vector<char> near_sign;
  mixed_upstream(m, g_rgb, g_depth, g_vis, tgt_rgb, tgt_depth, g, near_sign);
  std::vector<double> arec;
  composite_backward_abs(m.sd, m.img, m.traces, g, arec);
  const int K = m.sd.K;
  std::memset(smean, 0, sizeof(double) * 3 * N);
  std::memset(sscale, 0, sizeof(double) * 3 * N);
  std::memset(squat, 0, sizeof(double) * 4 * N);
  std::memset(sopac, 0, sizeof(double) * N);
  std::memset(ssh, 0, sizeof(double) * 3 * K * N);
  project_backward_abs(m.sd, sh, arec, smean, sscale, squat, sopac, ssh);
}

double oracle_loss(const double* means, const double* log_scales, const double* quats, const double* opac,
                   const double* sh, int64_t N, int deg, const double* cams, int V, const double* opts,
                   const double* tgt_rgb, const double* tgt_depth) {
  Scene<double> sc;
  build_scene<double>(sc, means, log_scales, quats, opac, sh, N, deg, cams, V, opts);
  std::vector<PixelOut<double>> img;
  render_all<double>(sc, 1, img, nullptr);
  std::vector<double> g;
  std::vector<char> ns;
  return loss_and_grad<double>(sc, img, tgt_rgb, tgt_depth, g, ns);
}

// One Adam step (bias-corrected; eps added to the corrected root), in FP64, on a flat array.
// `step` is the step number after increment (1 for the first step).
// Opacity pruning (Section III-C, the prunable opacity threshold): the indices, in order, of the Gaussians whose
// opacity sigmoid(logit) is at least min_opacity.  The decision is taken as the FP32 path takes it: the FP32
// logit against the FP32-rounded logit of the threshold.  Returns the count; keep_idx has room for n.
int64_t oracle_prune(const double* opac_logit, int64_t n, double min_opacity, int64_t* keep_idx) {
  const float thr = (float)std::log(min_opacity / (1.0 - min_opacity));
  int64_t k = 0;
  for (int64_t i = 0; i < n; ++i)
    if ((float)opac_logit[i] >= thr) keep_idx[k++] = i;
  return k;
}

void oracle_adam(double* p, const double* g, double* m, double* v, int64_t n, double lr, double beta1, double beta2,
                 double eps, int64_t step) {
  double bc1 = 1.0 - std::pow(beta1, (double)step);
  double bc2 = 1.0 - std::pow(beta2, (double)step);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
    v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
    double denom = std::sqrt(v[i]) / std::sqrt(bc2) + eps;
    p[i] -= (lr / bc1) * m[i] / denom;
  }
}

}  // extern "C"
