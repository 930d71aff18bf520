// SSIM term of the photometric loss (LVI-GS Section III-E, eq. Lc: (1 - lambda) L1 + lambda L_ssim) and its
// gradient with respect to the rendered colour image.
//
// Per view v, channel c and pixel p, over an 11 x 11 Gaussian window w (standard deviation 1.5, summing to 1,
// zero padding outside the image): mu_x, mu_y, E_xx, E_yy, E_xy are window sums, s_x = E_xx - mu_x^2,
// s_y = E_yy - mu_y^2, s_xy = E_xy - mu_x mu_y and
//   SSIM(p) = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x + s_y + C2)),  C1 = 1e-4, C2 = 9e-4.
// The term is lambda w_v (1 - mean over channels and pixels of SSIM).  With SSIM seen as a function of the
// three window sums that contain the rendered image x (mu_x, E_xx, E_xy), and A, B, C its partial derivatives,
//   d SSIM(p) / d x(q) = w(q - p) [A(p) + 2 x(q) B(p) + y(q) C(p)],
// so the image gradient is three more window sums: (w * A)(q) + 2 x(q) (w * B)(q) + y(q) (w * C)(q).
//
// One workgroup of 256 threads per 16 x 16 output tile of one channel of one view.  Everything stays in LDS:
// the tile plus a halo of 10 pixels of x and y (36 x 36), the separable window sums of the five moments over
// the tile plus a halo of 5 (26 x 26), A, B, C there, and their window sums over the tile.  HBM traffic is the
// two images read (with the halo) and the gradient written once; the ALU work is a few hundred operations per
// pixel and channel.
#include "common.h"

namespace {

constexpr int kT = 16;             // output tile
constexpr int kR = 5;              // window radius (11 taps)
constexpr int kS = kT + 2 * kR;    // 26: where the moments, SSIM, A, B, C are needed
constexpr int kL = kT + 4 * kR;    // 36: where x and y are needed
constexpr int kThreads = kT * kT;  // 256
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct SsimArgs {
  const float* rgb;
  const float* tgt;
  const gs_camera* cams;
  float* g_rgb;
  float* loss;  // [1 + kLossSlots]: partial sums in loss[1..]
  float lambda;
  int n_views;
  int tile_off[GS_MAX_VIEWS + 1];  // first output tile of each view (16 x 16 tiles)
  float w[2 * kR + 1];             // the normalised 1D window
};

__global__ __launch_bounds__(kThreads) void k_ssim(const SsimArgs a) {
  __shared__ float sx[kL][kL + 1], sy[kL][kL + 1];
  __shared__ float h[5][kL][kS];       // row sums of mu_x, mu_y, E_xx, E_yy, E_xy (reused for A, B, C)
  __shared__ float abc[3][kS][kS + 1];
  __shared__ float part[kThreads / 64];
  const int b = blockIdx.x;
  const int ch = blockIdx.y;
  int v = 0;
  for (int i = 1; i < a.n_views; ++i)
    if (a.tile_off[i] <= b) v = i;
  const gs_camera& cam = a.cams[v];
  const int W = cam.width, H = cam.height;
  const int tiles_x = (W + kT - 1) / kT;
  const int tl = b - a.tile_off[v];
  const int x0 = (tl % tiles_x) * kT, y0 = (tl / tiles_x) * kT;
  const int64_t P = (int64_t)W * H;
  const float* x = a.rgb + 3 * (int64_t)cam.pixel_offset + ch * P;
  const float* y = a.tgt + 3 * (int64_t)cam.pixel_offset + ch * P;
  const int tid = threadIdx.x;

  // 1. x and y over the tile plus a halo of 2 window radii, zero outside the image
  for (int i = tid; i < kL * kL; i += kThreads) {
    const int r = i / kL, c = i - r * kL;
    const int gy = y0 - 2 * kR + r, gx = x0 - 2 * kR + c;
    const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
    const int64_t q = (int64_t)gy * W + gx;
    sx[r][c] = in ? x[q] : 0.f;
    sy[r][c] = in ? y[q] : 0.f;
  }
  __syncthreads();
  // 2. row sums of the five moments: loaded rows x the 26 columns of the moment region
  for (int i = tid; i < kL * kS; i += kThreads) {
    const int r = i / kS, c = i - r * kS;
    float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f, m4 = 0.f;
#pragma unroll
    for (int k = 0; k <= 2 * kR; ++k) {
      const float wk = a.w[k], p = sx[r][c + k], q = sy[r][c + k];
      m0 += wk * p;
      m1 += wk * q;
      m2 += wk * p * p;
      m3 += wk * q * q;
      m4 += wk * p * q;
    }
    h[0][r][c] = m0;
    h[1][r][c] = m1;
    h[2][r][c] = m2;
    h[3][r][c] = m3;
    h[4][r][c] = m4;
  }
  __syncthreads();
  // 3. column sums -> moments at the 26 x 26 positions; SSIM and its partials A, B, C there (0 outside the
  // image: only in-image pixels are terms of the mean)
  float ssim_acc = 0.f;
  for (int i = tid; i < kS * kS; i += kThreads) {
    const int r = i / kS, c = i - r * kS;
    float mx = 0.f, my = 0.f, exx = 0.f, eyy = 0.f, exy = 0.f;
#pragma unroll
    for (int k = 0; k <= 2 * kR; ++k) {
      const float wk = a.w[k];
      mx += wk * h[0][r + k][c];
      my += wk * h[1][r + k][c];
      exx += wk * h[2][r + k][c];
      eyy += wk * h[3][r + k][c];
      exy += wk * h[4][r + k][c];
    }
    const int gy = y0 - kR + r, gx = x0 - kR + c;
    float A = 0.f, Bc = 0.f, Cc = 0.f;
    if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
      const float vx = exx - mx * mx, vy = eyy - my * my, cxy = exy - mx * my;
      const float a1 = 2.f * mx * my + kC1, b1 = 2.f * cxy + kC2;
      const float a2 = mx * mx + my * my + kC1, b2 = vx + vy + kC2;
      const float id = 1.f / (a2 * b2);
      const float S = a1 * b1 * id;
      A = 2.f * my * (b1 - a1) * id - 2.f * S * mx * (b2 - a2) * id;
      Bc = -S / b2;
      Cc = 2.f * a1 * id;
      if (r >= kR && r < kR + kT && c >= kR && c < kR + kT) ssim_acc += S;
    }
    abc[0][r][c] = A;
    abc[1][r][c] = Bc;
    abc[2][r][c] = Cc;
  }
  __syncthreads();
  // 4. row sums of A, B, C: the 26 rows x the 16 output columns
  for (int i = tid; i < kS * kT; i += kThreads) {
    const int r = i / kT, c = i - r * kT;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int k = 0; k <= 2 * kR; ++k) {
      const float wk = a.w[k];
      s0 += wk * abc[0][r][c + k];
      s1 += wk * abc[1][r][c + k];
      s2 += wk * abc[2][r][c + k];
    }
    h[0][r][c] = s0;
    h[1][r][c] = s1;
    h[2][r][c] = s2;
  }
  __syncthreads();
  // 5. column sums at the output pixel of this thread, and its gradient
  {
    const int r = tid / kT, c = tid - r * kT;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int k = 0; k <= 2 * kR; ++k) {
      const float wk = a.w[k];
      s0 += wk * h[0][r + k][c];
      s1 += wk * h[1][r + k][c];
      s2 += wk * h[2][r + k][c];
    }
    const int gy = y0 + r, gx = x0 + c;
    if (gx < W && gy < H) {
      const float xq = sx[r + 2 * kR][c + 2 * kR], yq = sy[r + 2 * kR][c + 2 * kR];
      const float scale = -fmaxf(cam.loss_weight, 0.f) * a.lambda / (3.f * (float)P);
      a.g_rgb[3 * (int64_t)cam.pixel_offset + ch * P + (int64_t)gy * W + gx] = scale * (s0 + 2.f * xq * s1 + yq * s2);
    }
  }
  // 6. the loss: lambda w_v (1 - mean SSIM) = lambda w_v - lambda w_v / (3 P) sum SSIM; the constant is added once
  // per view, by its first tile's channel 0
  float ls = gsk::wave_sum_last(ssim_acc);
  if ((tid & 63) == 63) part[tid >> 6] = ls;
  __syncthreads();
  if (tid == 0) {
    float sum = 0.f;
    for (int i = 0; i < kThreads / 64; ++i) sum += part[i];
    const float wv = fmaxf(cam.loss_weight, 0.f);  // an inactive view (weight < 0) adds nothing
    float add = -wv * a.lambda / (3.f * (float)P) * sum;
    if (tl == 0 && ch == 0) add += wv * a.lambda;
    gsk::atomic_add_f32(a.loss + 1 + ((b * 3 + ch) % gsk::kLossSlots), add);
  }
}

}  // namespace

namespace gs_launch {

hipError_t ssim(const gs_camera* cams_host, const gs_camera* cams_dev, int n_views, const float* rgb,
                const float* tgt, float lambda, float* g_rgb, float* loss, hipStream_t st) {
  SsimArgs a;
  a.rgb = rgb;
  a.tgt = tgt;
  a.cams = cams_dev;
  a.g_rgb = g_rgb;
  a.loss = loss;
  a.lambda = lambda;
  a.n_views = n_views;
  int tiles = 0;
  for (int v = 0; v <= GS_MAX_VIEWS; ++v) a.tile_off[v] = 0;
  for (int v = 0; v < n_views; ++v) {
    a.tile_off[v] = tiles;
    tiles += ((cams_host[v].width + kT - 1) / kT) * ((cams_host[v].height + kT - 1) / kT);
  }
  a.tile_off[n_views] = tiles;
  double g[2 * kR + 1], s = 0.0;
  for (int i = -kR; i <= kR; ++i) {
    g[i + kR] = exp(-(double)(i * i) / (2.0 * 1.5 * 1.5));
    s += g[i + kR];
  }
  for (int i = 0; i <= 2 * kR; ++i) a.w[i] = (float)(g[i] / s);
  hipError_t e = fill_f32(loss, 0.f, 1 + gsk::kLossSlots, st);
  if (e != hipSuccess) return e;
  k_ssim<<<dim3((unsigned)tiles, 3), kThreads, 0, st>>>(a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return loss_total(loss, st);
}

}  // namespace gs_launch
