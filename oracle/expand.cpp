// Plain CPU oracle of the map expansion (TEST INFRASTRUCTURE ONLY, see oracle.cpp; the HIP path shares no code
// with it).
//
// LVI-GS grows its Gaussian map from the colourised LiDAR points of each keyframe:
//   * visibility filter (Section III-C): the keyframe's visibility image V (eq. Vp, rendered from the current
//     map) decides whether a point is needed.  The sentence is garbled ("if V_p <= tau_alpha, then filter out the
//     point"); its purpose is to avoid adding Gaussians where the map already explains the view, so the reading
//     is: a point is KEPT where the map is still transparent at its pixel, V_p <= tau_alpha, and dropped where
//     V_p > tau_alpha.  A point that does not project into the image (behind the near plane or outside the
//     pixel grid) is not judged and kept;
//   * voxel deduplication and density cap (Section III-A): points live in fixed-size voxels (0.1 m in the
//     paper's example); a point whose voxel already holds `cap` points - the map's Gaussians plus the points of
//     this batch accepted before it, in input order - is discarded (cap = 1 is "if a point already exists in
//     that position, it is discarded");
//   * initialisation (Section III-E): each accepted point becomes a Gaussian centred on it; its three
//     log-scales are log sqrt of the mean squared distance to its 3 nearest accepted neighbours, at least 1e-7
//     (the garbled "squared distance ... minimum value" read as the usual nearest-neighbour spacing); rotation
//     identity; opacity logit = inverse sigmoid of the initial opacity; SH degree-0 coefficients from the point's
//     colour ((rgb - 0.5) / Y_0), higher bands 0.
// The discrete decisions (pixel, visibility comparison, voxel index) are taken in FP32 exactly as specified
// below, so that any FP32 implementation of the same operations takes the same decisions; the spacing is
// computed in double (brute force over all accepted points).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <tuple>
#include <vector>

namespace {

constexpr double kY0 = 0.28209479177387814;  // 1 / (2 sqrt(pi)), the degree-0 real SH basis function

// Voxel of a point: floor(x / s) per axis with the FP32 coordinate and voxel size (IEEE division).
std::tuple<int, int, int> voxel_of(const double* p, float s) {
  return std::make_tuple((int)std::floor((float)p[0] / s), (int)std::floor((float)p[1] / s),
                         (int)std::floor((float)p[2] / s));
}

}  // namespace

extern "C" {

// cam: R (9, row-major world -> camera), T (3), fx, fy, cx, cy, W, H (16 doubles); vis: [H * W] visibility image.
// Returns the number of Gaussians added; kept[i] = 1 for accepted points (in input order), and the new Gaussians'
// parameters (in input order of their points) in the out arrays (room for M; sh [M, (deg+1)^2, 3]).
int64_t oracle_expand(const double* pts, const double* rgb, int64_t M, const double* cam, const double* vis,
                      double tau_alpha, double near_z, const double* map_means, int64_t N, double voxel, int cap,
                      double init_opacity, int sh_degree, int32_t* kept, double* out_means, double* out_log_scales,
                      double* out_quats, double* out_opacity, double* out_sh) {
  const float R[9] = {(float)cam[0], (float)cam[1], (float)cam[2], (float)cam[3], (float)cam[4],
                      (float)cam[5], (float)cam[6], (float)cam[7], (float)cam[8]};
  const float T[3] = {(float)cam[9], (float)cam[10], (float)cam[11]};
  const float fx = (float)cam[12], fy = (float)cam[13], cx = (float)cam[14], cy = (float)cam[15];
  const int W = (int)cam[16], H = (int)cam[17];
  const float tau = (float)tau_alpha, nz = (float)near_z, vs = (float)voxel;
  // 1. visibility filter
  std::vector<char> pass(M, 1);
  for (int64_t i = 0; i < M; ++i) {
    const float x = (float)pts[3 * i], y = (float)pts[3 * i + 1], z = (float)pts[3 * i + 2];
    float t[3];
    for (int r = 0; r < 3; ++r) t[r] = std::fma(R[3 * r + 2], z, std::fma(R[3 * r + 1], y, std::fma(R[3 * r], x, T[r])));
    if (!(t[2] >= nz)) continue;
    const float u = std::fma(fx, t[0] / t[2], cx), v = std::fma(fy, t[1] / t[2], cy);
    if (!(u >= 0.f && u < (float)W && v >= 0.f && v < (float)H)) continue;
    const int px = (int)u, py = (int)v;
    pass[i] = (float)vis[(int64_t)py * W + px] <= tau;
  }
  // 2. voxel occupancy: the map's Gaussians, then this batch's passing points in input order
  std::map<std::tuple<int, int, int>, int> occ;
  for (int64_t j = 0; j < N; ++j) occ[voxel_of(map_means + 3 * j, vs)] += 1;
  std::vector<int64_t> acc;
  for (int64_t i = 0; i < M; ++i) {
    kept[i] = 0;
    if (!pass[i]) continue;
    int& c = occ[voxel_of(pts + 3 * i, vs)];
    if (c < cap) {
      c += 1;
      kept[i] = 1;
      acc.push_back(i);
    }
  }
  // 3. initialisation; spacing by brute force over the accepted points
  const int64_t A = (int64_t)acc.size();
  const int K = (sh_degree + 1) * (sh_degree + 1);
  const double logit = std::log(init_opacity / (1.0 - init_opacity));
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t a = 0; a < A; ++a) {
    const double* p = pts + 3 * acc[a];
    double best[3] = {INFINITY, INFINITY, INFINITY};
    for (int64_t b = 0; b < A; ++b) {
      if (b == a) continue;
      const double* q = pts + 3 * acc[b];
      const double d = (p[0] - q[0]) * (p[0] - q[0]) + (p[1] - q[1]) * (p[1] - q[1]) + (p[2] - q[2]) * (p[2] - q[2]);
      if (d < best[2]) {
        best[2] = d;
        if (best[2] < best[1]) std::swap(best[1], best[2]);
        if (best[1] < best[0]) std::swap(best[0], best[1]);
      }
    }
    int found = 0;
    double sum = 0.0;
    for (int k = 0; k < 3; ++k)
      if (std::isfinite(best[k])) {
        sum += best[k];
        ++found;
      }
    const double d2 = std::max(found ? sum / found : 0.0, 1e-7);
    const double ls = 0.5 * std::log(d2);
    for (int k = 0; k < 3; ++k) {
      out_means[3 * a + k] = (double)(float)p[k];
      out_log_scales[3 * a + k] = ls;
    }
    out_quats[4 * a] = 1.0;
    out_quats[4 * a + 1] = out_quats[4 * a + 2] = out_quats[4 * a + 3] = 0.0;
    out_opacity[a] = logit;
    double* f = out_sh + (int64_t)a * K * 3;
    for (int k = 0; k < K * 3; ++k) f[k] = 0.0;
    for (int ch = 0; ch < 3; ++ch) f[ch] = (rgb[3 * acc[a] + ch] - 0.5) / kY0;
  }
  return A;
}

}  // extern "C"

extern "C" {

// Spatial order of Gaussians (a memory layout, not a step of the method): the stable order of their Morton codes,
// each coordinate quantised to 21 bits over the means' bounding box in FP32 as the library does it:
// q = min(2^21 - 1, floor((x - lo) * s)), s = (2^21 - 1) / max(hi - lo, 1e-30), interleaved x, y, z from bit 0.
void oracle_spatial_order(const double* means, int64_t n, int32_t* perm) {
  float lo[3], hi[3];
  for (int k = 0; k < 3; ++k) {
    lo[k] = INFINITY;
    hi[k] = -INFINITY;
    for (int64_t g = 0; g < n; ++g) {
      const float x = (float)means[3 * g + k];
      lo[k] = std::min(lo[k], x);
      hi[k] = std::max(hi[k], x);
    }
  }
  std::vector<uint64_t> code(n, 0);
  for (int64_t g = 0; g < n; ++g)
    for (int k = 0; k < 3; ++k) {
      const float s = 2097151.0f / std::max(hi[k] - lo[k], 1e-30f);
      const float t = ((float)means[3 * g + k] - lo[k]) * s;
      const uint32_t q = (uint32_t)std::min(std::floor(t), 2097151.0f);
      for (int b = 0; b < 21; ++b) code[g] |= (uint64_t)((q >> b) & 1u) << (3 * b + k);
    }
  std::vector<int64_t> idx(n);
  for (int64_t g = 0; g < n; ++g) idx[g] = g;
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return code[a] < code[b]; });
  for (int64_t g = 0; g < n; ++g) perm[g] = (int32_t)idx[g];
}

}  // extern "C"
