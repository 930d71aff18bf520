// Plain CPU oracle of the SSIM term of the photometric loss.
//
// TEST INFRASTRUCTURE ONLY (see oracle.cpp): the HIP product path shares no code with it.
//
// Section III-E, eq. Lc: the image loss is (1 - lambda) L1 + lambda L_ssim, the SSIM error between the rendered
// colour image and the keyframe image.  The paper gives neither the SSIM window nor its constants; the
// readings are those of the 3DGS work it builds on:
//   * SSIM per colour channel over an 11 x 11 Gaussian window with standard deviation 1.5 px, normalised to
//     sum 1; pixels outside the image count as 0 (zero padding, the window is not renormalised at borders);
//   * C1 = (0.01)^2, C2 = (0.03)^2 (dynamic range 1);
//   * mean over the three channels and all pixels of a view; L_ssim = 1 - that mean.
// Per pixel p and channel, with sums over the window w centred at p:
//   mu_x = sum w x,  mu_y = sum w y,  E_xx = sum w x^2,  E_yy = sum w y^2,  E_xy = sum w x y,
//   s_x = E_xx - mu_x^2,  s_y = E_yy - mu_y^2,  s_xy = E_xy - mu_x mu_y,
//   SSIM = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x + s_y + C2)).
// The gradient with respect to the rendered image x follows the chain rule through mu_x, E_xx and E_xy
// (the three window sums that contain x), written out per (output pixel, window pixel) pair.
//
// Everything is in double, with plain loops over the 2D window (no separable filtering).

#include <cmath>
#include <cstdint>
#include <vector>

namespace {

constexpr int kRadius = 5;  // 11 x 11 window
constexpr double kSigma = 1.5;
constexpr double kC1 = 0.01 * 0.01;
constexpr double kC2 = 0.03 * 0.03;

// The 2D window: the product of two normalised 1D Gaussians (so it sums to 1).
std::vector<double> window() {
  double g[2 * kRadius + 1], s = 0.0;
  for (int i = -kRadius; i <= kRadius; ++i) {
    g[i + kRadius] = std::exp(-(double)(i * i) / (2.0 * kSigma * kSigma));
    s += g[i + kRadius];
  }
  std::vector<double> w((2 * kRadius + 1) * (2 * kRadius + 1));
  for (int a = 0; a <= 2 * kRadius; ++a)
    for (int b = 0; b <= 2 * kRadius; ++b) w[a * (2 * kRadius + 1) + b] = (g[a] / s) * (g[b] / s);
  return w;
}

struct Stats { double mx, my, exx, eyy, exy; };

Stats stats_at(const double* x, const double* y, int H, int W, int py, int px, const std::vector<double>& w) {
  Stats s{0, 0, 0, 0, 0};
  for (int dy = -kRadius; dy <= kRadius; ++dy)
    for (int dx = -kRadius; dx <= kRadius; ++dx) {
      const int u = px + dx, v = py + dy;
      if (u < 0 || u >= W || v < 0 || v >= H) continue;  // zero padding
      const double g = w[(dy + kRadius) * (2 * kRadius + 1) + dx + kRadius];
      const double a = x[(int64_t)v * W + u], b = y[(int64_t)v * W + u];
      s.mx += g * a;
      s.my += g * b;
      s.exx += g * a * a;
      s.eyy += g * b * b;
      s.exy += g * a * b;
    }
  return s;
}

}  // namespace

extern "C" {

// The window (121 values, row-major), for tests.
void oracle_ssim_window(double* out) {
  const std::vector<double> w = window();
  for (size_t i = 0; i < w.size(); ++i) out[i] = w[i];
}

// SSIM of one channel plane: per-pixel map (H*W, nullable) and its mean; with grad non-NULL, also
// d(mean SSIM)/dx per pixel of x.
double oracle_ssim_plane(const double* x, const double* y, int H, int W, double* map, double* grad) {
  const std::vector<double> w = window();
  const int64_t P = (int64_t)H * W;
  std::vector<double> A(P), Bc(P), Cc(P);  // dS/dmu_x, dS/dE_xx, dS/dE_xy per output pixel
  std::vector<double> row_total(H, 0.0);    // per-row sums, added in row order below (a fixed summation order)
#pragma omp parallel for schedule(static)
  for (int py = 0; py < H; ++py)
    for (int px = 0; px < W; ++px) {
      const Stats s = stats_at(x, y, H, W, py, px, w);
      const double sx = s.exx - s.mx * s.mx, sy = s.eyy - s.my * s.my, sxy = s.exy - s.mx * s.my;
      const double a1 = 2.0 * s.mx * s.my + kC1, b1 = 2.0 * sxy + kC2;
      const double a2 = s.mx * s.mx + s.my * s.my + kC1, b2 = sx + sy + kC2;
      const double d = a2 * b2;
      const double S = a1 * b1 / d;
      const int64_t p = (int64_t)py * W + px;
      if (map) map[p] = S;
      row_total[py] += S;
      // S = a1 b1 / (a2 b2) as a function of (mu_x, E_xx, E_xy) with the y sums fixed:
      //   d a1/d mu_x = 2 mu_y, d b1/d mu_x = -2 mu_y, d a2/d mu_x = 2 mu_x, d b2/d mu_x = -2 mu_x,
      //   d b2/d E_xx = 1, d b1/d E_xy = 2
      A[p] = (2.0 * s.my * (b1 - a1)) / d - S * (2.0 * s.mx * (b2 - a2)) / d;
      Bc[p] = -S / b2;
      Cc[p] = 2.0 * a1 / d;
    }
  double total = 0.0;
  for (int py = 0; py < H; ++py) total += row_total[py];
  if (grad) {
    // d mean / d x(q) = (1/P) sum_p w(q - p) [A(p) + 2 x(q) B(p) + y(q) C(p)] over the p whose window holds q
#pragma omp parallel for schedule(static)
    for (int qy = 0; qy < H; ++qy)
      for (int qx = 0; qx < W; ++qx) {
        const int64_t q = (int64_t)qy * W + qx;
        double acc = 0.0;
        for (int dy = -kRadius; dy <= kRadius; ++dy)
          for (int dx = -kRadius; dx <= kRadius; ++dx) {
            const int px = qx - dx, py = qy - dy;  // q = p + (dx, dy)
            if (px < 0 || px >= W || py < 0 || py >= H) continue;
            const int64_t p = (int64_t)py * W + px;
            const double g = w[(dy + kRadius) * (2 * kRadius + 1) + dx + kRadius];
            acc += g * (A[p] + 2.0 * x[q] * Bc[p] + y[q] * Cc[p]);
          }
        grad[q] = acc / (double)P;
      }
  }
  return total / (double)P;
}

// The SSIM term over views: L = sum_v w_v lambda (1 - mean over 3 channels and P_v pixels of SSIM), images planar
// [3][H_v][W_v] concatenated over views (sizes[2v] = H_v, sizes[2v+1] = W_v).  grad (nullable, same layout as x)
// receives dL/dx.  Returns L.
double oracle_ssim_loss(const double* x, const double* y, int V, const int32_t* sizes, const double* weights,
                        double lambda, double* grad) {
  double L = 0.0;
  int64_t off = 0;
  for (int v = 0; v < V; ++v) {
    const int H = sizes[2 * v], W = sizes[2 * v + 1];
    const int64_t P = (int64_t)H * W;
    double mean = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double* xc = x + off + c * P;
      const double* yc = y + off + c * P;
      double* gc = grad ? grad + off + c * P : nullptr;
      mean += oracle_ssim_plane(xc, yc, H, W, nullptr, gc) / 3.0;
      if (gc)
        for (int64_t i = 0; i < P; ++i) gc[i] *= -weights[v] * lambda / 3.0;
    }
    L += weights[v] * lambda * (1.0 - mean);
    off += 3 * P;
  }
  return L;
}

}  // extern "C"
