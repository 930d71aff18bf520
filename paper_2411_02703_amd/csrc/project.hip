// Projection of 3D Gaussians to per-view 2D conics and its backward (LVI-GS Section III-B:
// covariance factorisation eq. Sigma, EWA projection eq. muI; colour from real spherical harmonics,
// Section III-E).  One thread per Gaussian; it reads the Gaussian once and loops over all views.
#include "common.h"

namespace {

using gsk::DevOpts;

// Real orthonormal spherical harmonics up to degree 3 (Cartesian form on the unit sphere),
// ordered by l then m = -l..l.
constexpr float kC0 = 0.28209479177387814f;
constexpr float kC1 = 0.4886025119029199f;
constexpr float kC2a = 1.0925484305920792f;   // xy, yz, xz
constexpr float kC2b = 0.31539156525252005f;  // 3z^2 - 1
constexpr float kC2c = 0.5462742152960396f;   // x^2 - y^2
constexpr float kC3a = 0.5900435899266435f;   // y(3x^2 - y^2), x(x^2 - 3y^2)
constexpr float kC3b = 2.890611442640554f;    // xyz
constexpr float kC3c = 0.4570457994644658f;   // y(5z^2 - 1), x(5z^2 - 1)
constexpr float kC3d = 0.3731763325901154f;   // z(5z^2 - 3)
constexpr float kC3e = 1.445305721320277f;    // z(x^2 - y^2)

template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
  Y[0] = kC0;
  if (DEG >= 1) {
    Y[1] = kC1 * y;
    Y[2] = kC1 * z;
    Y[3] = kC1 * x;
  }
  if (DEG >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kC2a * (x * y);
    Y[5] = kC2a * (y * z);
    Y[6] = kC2b * (3.f * zz - 1.f);
    Y[7] = kC2a * (x * z);
    Y[8] = kC2c * (xx - yy);
    if (DEG >= 3) {
      Y[9] = kC3a * y * (3.f * xx - yy);
      Y[10] = kC3b * (x * y) * z;
      Y[11] = kC3c * y * (5.f * zz - 1.f);
      Y[12] = kC3d * z * (5.f * zz - 3.f);
      Y[13] = kC3c * x * (5.f * zz - 1.f);
      Y[14] = kC3e * z * (xx - yy);
      Y[15] = kC3a * x * (xx - 3.f * yy);
    }
  }
}

// sum_k w_k grad Y_k at (x, y, z) for the forms above (the radial part is removed by the caller).
template <int DEG>
__device__ __forceinline__ void sh_dir_grad(float x, float y, float z, const float* w, float& gx, float& gy,
                                            float& gz) {
  gx = gy = gz = 0.f;
  if (DEG >= 1) {
    gy += kC1 * w[1];
    gz += kC1 * w[2];
    gx += kC1 * w[3];
  }
  if (DEG >= 2) {
    gx += kC2a * y * w[4];
    gy += kC2a * x * w[4];
    gy += kC2a * z * w[5];
    gz += kC2a * y * w[5];
    gz += 6.f * kC2b * z * w[6];
    gx += kC2a * z * w[7];
    gz += kC2a * x * w[7];
    gx += 2.f * kC2c * x * w[8];
    gy -= 2.f * kC2c * y * w[8];
    if (DEG >= 3) {
      const float xx = x * x, yy = y * y, zz = z * z;
      gx += 6.f * kC3a * x * y * w[9];
      gy += 3.f * kC3a * (xx - yy) * w[9];
      gx += kC3b * y * z * w[10];
      gy += kC3b * x * z * w[10];
      gz += kC3b * x * y * w[10];
      gy += kC3c * (5.f * zz - 1.f) * w[11];
      gz += 10.f * kC3c * y * z * w[11];
      gz += kC3d * (15.f * zz - 3.f) * w[12];
      gx += kC3c * (5.f * zz - 1.f) * w[13];
      gz += 10.f * kC3c * x * z * w[13];
      gx += 2.f * kC3e * x * z * w[14];
      gy -= 2.f * kC3e * y * z * w[14];
      gz += kC3e * (xx - yy) * w[14];
      gx += 3.f * kC3a * (xx - yy) * w[15];
      gy -= 6.f * kC3a * x * y * w[15];
    }
  }
}

// Camera transform with a fixed operation order (reproducible bit for bit):
// t_r = fma(R_r2, mu_z, fma(R_r1, mu_y, fma(R_r0, mu_x, T_r))).
__device__ __forceinline__ void camera_point(const gs_camera& c, float m0, float m1, float m2, float& tx, float& ty,
                                             float& tz) {
  tx = __builtin_fmaf(c.R[2], m2, __builtin_fmaf(c.R[1], m1, __builtin_fmaf(c.R[0], m0, c.T[0])));
  ty = __builtin_fmaf(c.R[5], m2, __builtin_fmaf(c.R[4], m1, __builtin_fmaf(c.R[3], m0, c.T[1])));
  tz = __builtin_fmaf(c.R[8], m2, __builtin_fmaf(c.R[7], m1, __builtin_fmaf(c.R[6], m0, c.T[2])));
}

// View-independent part of one Gaussian.
struct Shape {
  float S[3];
  float q[4], qnorm;
  float Rq[9];
  float M[9];
  float Sig[6];  // s00 s01 s02 s11 s12 s22
  float o;
};

__device__ __forceinline__ void shape_of(const float* ls, const float* qq, float ol, Shape& s) {
  for (int i = 0; i < 3; ++i) s.S[i] = expf(ls[i]);
  s.qnorm = sqrtf(qq[0] * qq[0] + qq[1] * qq[1] + qq[2] * qq[2] + qq[3] * qq[3]);
  const float iq = 1.f / s.qnorm;
  for (int i = 0; i < 4; ++i) s.q[i] = qq[i] * iq;
  const float w = s.q[0], x = s.q[1], y = s.q[2], z = s.q[3];
  s.Rq[0] = 1.f - 2.f * (y * y + z * z);
  s.Rq[1] = 2.f * (x * y - w * z);
  s.Rq[2] = 2.f * (x * z + w * y);
  s.Rq[3] = 2.f * (x * y + w * z);
  s.Rq[4] = 1.f - 2.f * (x * x + z * z);
  s.Rq[5] = 2.f * (y * z - w * x);
  s.Rq[6] = 2.f * (x * z - w * y);
  s.Rq[7] = 2.f * (y * z + w * x);
  s.Rq[8] = 1.f - 2.f * (x * x + y * y);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) s.M[i * 3 + j] = s.Rq[i * 3 + j] * s.S[j];
  // Sigma = M M^T
  auto row_dot = [&](int i, int j) {
    return s.M[i * 3] * s.M[j * 3] + s.M[i * 3 + 1] * s.M[j * 3 + 1] + s.M[i * 3 + 2] * s.M[j * 3 + 2];
  };
  s.Sig[0] = row_dot(0, 0);
  s.Sig[1] = row_dot(0, 1);
  s.Sig[2] = row_dot(0, 2);
  s.Sig[3] = row_dot(1, 1);
  s.Sig[4] = row_dot(1, 2);
  s.Sig[5] = row_dot(2, 2);
  s.o = 1.f / (1.f + expf(-ol));
}

// EWA: rows u, w of T2 = J W and the 2x2 covariance A, B, C (with the low-pass on the diagonal).
struct Ewa {
  float u[3], w[3], su[3], sw[3];
  float A, B, C, det;
  float inv_tz;
};

__device__ __forceinline__ void ewa(const gs_camera& c, const float* Sig, float tx, float ty, float tz, float lowpass,
                                    Ewa& e) {
  e.inv_tz = 1.f / tz;
  const float j00 = c.fx * e.inv_tz, j11 = c.fy * e.inv_tz;
  const float j02 = -c.fx * tx * e.inv_tz * e.inv_tz;
  const float j12 = -c.fy * ty * e.inv_tz * e.inv_tz;
  for (int k = 0; k < 3; ++k) {
    e.u[k] = j00 * c.R[k] + j02 * c.R[6 + k];
    e.w[k] = j11 * c.R[3 + k] + j12 * c.R[6 + k];
  }
  const float s00 = Sig[0], s01 = Sig[1], s02 = Sig[2], s11 = Sig[3], s12 = Sig[4], s22 = Sig[5];
  e.su[0] = s00 * e.u[0] + s01 * e.u[1] + s02 * e.u[2];
  e.su[1] = s01 * e.u[0] + s11 * e.u[1] + s12 * e.u[2];
  e.su[2] = s02 * e.u[0] + s12 * e.u[1] + s22 * e.u[2];
  e.sw[0] = s00 * e.w[0] + s01 * e.w[1] + s02 * e.w[2];
  e.sw[1] = s01 * e.w[0] + s11 * e.w[1] + s12 * e.w[2];
  e.sw[2] = s02 * e.w[0] + s12 * e.w[1] + s22 * e.w[2];
  e.A = e.u[0] * e.su[0] + e.u[1] * e.su[1] + e.u[2] * e.su[2] + lowpass;
  e.B = e.u[0] * e.sw[0] + e.u[1] * e.sw[1] + e.u[2] * e.sw[2];
  e.C = e.w[0] * e.sw[0] + e.w[1] * e.sw[1] + e.w[2] * e.sw[2] + lowpass;
  e.det = e.A * e.C - e.B * e.B;
}

template <int DEG>
__device__ __forceinline__ void colour(const float* f, float dx, float dy, float dz, float* Y, float* pre) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  sh_basis<DEG>(dx, dy, dz, Y);
  for (int ch = 0; ch < 3; ++ch) {
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) s += f[k * 3 + ch] * Y[k];
    pre[ch] = s + 0.5f;
  }
}

template <int DEG>
__global__ __launch_bounds__(256) void k_project(const float* __restrict__ means, const float* __restrict__ log_scales,
                                                 const float* __restrict__ quats, const float* __restrict__ opac,
                                                 const float* __restrict__ sh, int64_t n,
                                                 const gs_camera* __restrict__ cams, int V, DevOpts op,
                                                 float4* __restrict__ rec, short4* __restrict__ rect,
                                                 uint64_t* __restrict__ vis_mask,
                                                 uint32_t* __restrict__ zbits, int32_t* __restrict__ n_rec,
                                                 int32_t* __restrict__ n_inst, int32_t* __restrict__ flags) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  float mu[3], ls[3], qq[4], f[K * 3];
  bool finite = true;
  for (int i = 0; i < 3; ++i) {
    mu[i] = means[g * 3 + i];
    ls[i] = log_scales[g * 3 + i];
    finite &= isfinite(mu[i]) && isfinite(ls[i]);
  }
  for (int i = 0; i < 4; ++i) {
    qq[i] = quats[g * 4 + i];
    finite &= isfinite(qq[i]);
  }
  const float ol = opac[g];
  finite &= isfinite(ol);
#pragma unroll
  for (int i = 0; i < K * 3; ++i) {
    f[i] = sh[g * (K * 3) + i];
    finite &= isfinite(f[i]);
  }
  uint64_t mask = 0;
  int cnt = 0, inst = 0;
  if (!finite) {
    atomicOr(flags, GS_FLAG_NONFINITE);
  } else {
    Shape s;
    shape_of(ls, qq, ol, s);
    if (s.qnorm > 0.f && s.o >= op.alpha_min) {
      // opacity-aware radius factor: outside sqrt(kp * Sigma_I,diag) alpha < exp(-1/2) / 255
      const float kp = 2.f * logf(255.f * s.o) + 1.f;
      const bool pow2 = (op.tile_w & (op.tile_w - 1)) == 0 && (op.tile_h & (op.tile_h - 1)) == 0;
      const int lw = __builtin_ctz((unsigned)op.tile_w), lh = __builtin_ctz((unsigned)op.tile_h);
      for (int v = 0; v < V; ++v) {
        const gs_camera& c = cams[v];
        if (c.loss_weight < 0.f) continue;  // an inactive view: nothing is projected into it
        float tx, ty, tz;
        camera_point(c, mu[0], mu[1], mu[2], tx, ty, tz);
        if (!(tz >= op.near_z)) continue;
        const float un = tx / tz, vn = ty / tz;
        const float mx = __builtin_fmaf(c.fx, un, c.cx);
        const float my = __builtin_fmaf(c.fy, vn, c.cy);
        if (!(mx >= c.guard_lo_x && mx <= c.guard_hi_x && my >= c.guard_lo_y && my <= c.guard_hi_y)) continue;
        Ewa e;
        ewa(c, s.Sig, tx, ty, tz, op.lowpass, e);
        if (!(e.det > 0.f) || !isfinite(e.det)) continue;
        const float ext_x = sqrtf(kp * e.A), ext_y = sqrtf(kp * e.C);
        float lo_x = ceilf(mx - ext_x - 0.5f), hi_x = floorf(mx + ext_x - 0.5f);
        float lo_y = ceilf(my - ext_y - 0.5f), hi_y = floorf(my + ext_y - 0.5f);
        lo_x = fminf(fmaxf(lo_x, 0.f), (float)c.width);
        hi_x = fminf(fmaxf(hi_x, -1.f), (float)(c.width - 1));
        lo_y = fminf(fmaxf(lo_y, 0.f), (float)c.height);
        hi_y = fminf(fmaxf(hi_y, -1.f), (float)(c.height - 1));
        const int px0 = (int)lo_x, px1 = (int)hi_x, py0 = (int)lo_y, py1 = (int)hi_y;
        if (px0 > px1 || py0 > py1) continue;
        // (pixel indices are non-negative here: a power-of-two tile size divides by a shift)
        const int tx0 = pow2 ? px0 >> lw : px0 / op.tile_w, tx1 = pow2 ? px1 >> lw : px1 / op.tile_w;
        const int ty0 = pow2 ? py0 >> lh : py0 / op.tile_h, ty1 = pow2 ? py1 >> lh : py1 / op.tile_h;
        const float det_inv = 1.f / e.det;
        // colour at the direction from the camera centre
        const float d0 = mu[0] - c.campos[0], d1 = mu[1] - c.campos[1], d2 = mu[2] - c.campos[2];
        const float idist = 1.f / sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
        float Y[K], pre[3];
        colour<DEG>(f, d0 * idist, d1 * idist, d2 * idist, Y, pre);
        const int64_t r = (int64_t)v * n + g;
        rec[3 * r + 0] = make_float4(mx, my, tz, s.o);
        rec[3 * r + 1] = make_float4(e.C * det_inv, -e.B * det_inv, e.A * det_inv, fmaxf(pre[0], 0.f));
        // the pixel rectangle rides in the record's last two words (int16 pairs) for sub-tile culling
        rec[3 * r + 2] = make_float4(fmaxf(pre[1], 0.f), fmaxf(pre[2], 0.f),
                                     __int_as_float((px0 & 0xffff) | (px1 << 16)),
                                     __int_as_float((py0 & 0xffff) | (py1 << 16)));
        rect[r] = make_short4((short)tx0, (short)tx1, (short)ty0, (short)ty1);
        zbits[r] = __float_as_uint(tz);
        mask |= 1ull << v;
        ++cnt;
        inst += (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
      }
    }
  }
  vis_mask[g] = mask;
  n_rec[g] = cnt;
  n_inst[g] = inst;
}

// The partials of each wide record (more than kWideRecord tile instances), summed by a wave per record into the
// record's first slot; the padding word of that slot is set to 1 to mark the sum, so that a second projection
// backward of the same compositing output does not sum it again (the compositing writes 0 there).  Waves take
// the listed records in a grid-stride loop.
__global__ __launch_bounds__(256) void k_sum_wide(float4* __restrict__ ipart, const int32_t* __restrict__ big_rec,
                                                  const short4* __restrict__ rect,
                                                  const int32_t* __restrict__ rec_slot,
                                                  const int32_t* __restrict__ counters, int64_t rcap,
                                                  int64_t capacity) {
  const int lane = threadIdx.x & 63;
  const int64_t nbig = min((int64_t)counters[198], rcap);
  const int64_t n_stored = min((int64_t)counters[0], capacity);
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t b = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); b < nbig; b += waves) {
    const int32_t r = big_rec[b];
    const short4 rc = rect[r];
    const int cnt = (rc.y - rc.x + 1) * (rc.w - rc.z + 1);
    const int64_t i = rec_slot[r];
    if (i < 0 || i >= n_stored || ipart[3 * i + 2].w != 0.f) continue;  // not stored, or already summed
    float sm[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) sm[k] = 0.f;
    for (int k = lane; k < cnt && i + k < n_stored; k += 64) {
      const float4* pp = ipart + 3 * (i + k);
      const float4 a0 = pp[0], a1 = pp[1], a2 = pp[2];
      sm[0] += a0.x; sm[1] += a0.y; sm[2] += a0.z; sm[3] += a0.w;
      sm[4] += a1.x; sm[5] += a1.y; sm[6] += a1.z; sm[7] += a1.w;
      sm[8] += a2.x; sm[9] += a2.y;
    }
#pragma unroll
    for (int k = 0; k < 10; ++k) sm[k] = gsk::wave_sum_last(sm[k]);
    // every lane has read its instances of the record before the sum is written over the first one
    __builtin_amdgcn_wave_barrier();
    if (lane == 63) {
      ipart[3 * i + 0] = make_float4(sm[0], sm[1], sm[2], sm[3]);
      ipart[3 * i + 1] = make_float4(sm[4], sm[5], sm[6], sm[7]);
      ipart[3 * i + 2] = make_float4(sm[8], sm[9], 0.f, 1.f);
    }
  }
}

// Adam's part of the fused backward: moments and parameters of one Gaussian, updated in place (the same
// update as the separate Adam step: bias-corrected moments, eps added to the corrected root).
struct AdamArgs {
  float* m_means; float* m_scales; float* m_quats; float* m_opac; float* m_sh;
  float* v_means; float* v_scales; float* v_quats; float* v_opac; float* v_sh;
  float lr[6];
  float b1, b2, eps;
  const float* bias;  // {1 - b1^t, sqrt(1 - b2^t), skip}
  int sparse;         // only Gaussians visible in some view of the frame take the step
};

__device__ __forceinline__ void adam_one(float& p, float& m, float& v, float g, float s, float b1, float b2,
                                         float eps, float bc2s) {
  m = b1 * m + (1.f - b1) * g;
  v = b2 * v + (1.f - b2) * g * g;
  p -= s * m / (sqrtf(v) / bc2s + eps);
}

// Projection backward, one thread per Gaussian.  ADAM = false: the parameter gradient is added to g_* (+=).
// ADAM = true: every Gaussian (also those with no visible record, whose gradient is zero) takes its Adam step
// here: params, m and v are updated in place and the gradient is written (=) to g_* only when g_means is
// non-NULL.
template <int DEG, bool ADAM>
__global__ __launch_bounds__(256) void k_project_bwd(float* __restrict__ means, float* __restrict__ log_scales,
                                                     float* __restrict__ quats, float* __restrict__ opac,
                                                     float* __restrict__ sh, int64_t n,
                                                     const gs_camera* __restrict__ cams, int V, DevOpts op,
                                                     const float4* __restrict__ ipart,
                                                     const int32_t* __restrict__ rec_slot, const short4* __restrict__ rect,
                                                     const int32_t* __restrict__ count_dev, int64_t capacity,
                                                     const uint64_t* __restrict__ vis_mask, float* __restrict__ g_means,
                                                     float* __restrict__ g_scales, float* __restrict__ g_quats,
                                                     float* __restrict__ g_opac, float* __restrict__ g_sh,
                                                     AdamArgs ad) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  constexpr int F = K * 3;   // SH floats per Gaussian
  constexpr int FP = F + 1;  // LDS row stride (odd, so a lane per row hits distinct banks)
  // The SH gradient of a lane's Gaussian is summed in its LDS row (FP floats; with ADAM the last one flags a
  // Gaussian that takes no step) rather than in registers, which halves the kernel's register footprint; with
  // ADAM the wave then steps its 64 rows in coalesced runs of parameters and moments instead of one 4F-byte
  // row per lane.
  __shared__ float sbuf[4 * 64 * FP];
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const int64_t g0 = g - lane;  // first Gaussian of this wave
  const int nw = (int)max<int64_t>(0, min<int64_t>(64, n - g0));  // Gaussians of this wave
  float* wb = sbuf + (threadIdx.x >> 6) * 64 * FP;
  float* gf = wb + lane * FP;  // this lane's row: dL/d SH coefficients
  // every lane stays to the end of the view loop (the wave sums large records together)
  const uint64_t mask = g < n ? vis_mask[g] : 0ull;
  // lanes without a visible record read Gaussian 0 and discard it, unless they take an Adam step of their own
  const int64_t gg = (ADAM ? g < n : mask != 0) ? g : 0;
  float mu[3], ls[3], qq[4], f[F];
  for (int i = 0; i < 3; ++i) mu[i] = means[gg * 3 + i];
#pragma unroll
  for (int i = 0; i < F; ++i) f[i] = sh[gg * F + i];
  // only the covariance is needed in the view loop; scales, rotation and the rest of the shape are read and
  // formed again after it
  auto load_shape = [&]() {
    for (int i = 0; i < 3; ++i) ls[i] = log_scales[gg * 3 + i];
    for (int i = 0; i < 4; ++i) qq[i] = quats[gg * 4 + i];
  };
  float Sig[6];
  {
    load_shape();
    Shape s;
    shape_of(ls, qq, opac[gg], s);
    for (int i = 0; i < 6; ++i) Sig[i] = s.Sig[i];
  }

  float gmu[3] = {0.f, 0.f, 0.f};
  float gs[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // symmetric dL/dSigma: 00 01 02 11 12 22
  float go = 0.f;
#pragma unroll
  for (int i = 0; i < F; ++i) gf[i] = 0.f;

  // each visible record's instances: a contiguous run of partial slots from rec_slot (each record's tiles in
  // turn; binning lays the wave's records out view by view, so the lanes, which take the views together, read
  // one contiguous run per view).  A wide record (more than kWideRecord tiles) has its partials pre-summed into
  // its first slot (k_sum_wide), so one slot is read for it.  Slots outside the stored instances (an
  // overflowed frame, whose gradient is undefined) are not read.
  const int64_t n_stored = min((int64_t)count_dev[0], capacity);
  // the tile rectangle and first slot of this lane's next visible view are fetched one visible view ahead, so
  // that the partial loads of a view do not wait for them
  uint64_t rest = mask;
  short4 rc_next = make_short4(0, -1, 0, -1);
  int32_t slot_next = 0;
  if (rest) {
    const int64_t rn = (int64_t)__builtin_ctzll(rest) * n + g;
    rc_next = rect[rn];
    slot_next = rec_slot[rn];
  }
  for (int v = 0; v < V; ++v) {
    const bool vis = (mask >> v) & 1ull;
    if (__ballot(vis) == 0) continue;
    const gs_camera& c = cams[v];
    const int64_t r = (int64_t)v * n + g;
    int cnt = 0;
    int64_t i = 0;
    if (vis) {
      const short4 rc = rc_next;  // bit v is the lowest bit of rest
      i = slot_next;
      rest &= rest - 1;
      if (rest) {
        const int64_t rn = (int64_t)__builtin_ctzll(rest) * n + g;
        rc_next = rect[rn];
        slot_next = rec_slot[rn];
      }
      cnt = (rc.y - rc.x + 1) * (rc.w - rc.z + 1);
      if (cnt > gsk::kWideRecord) cnt = 1;
      if (i < 0 || i >= n_stored) cnt = 0;
    }
    // the record's gradient: the sum of its instances' partials over the tiles it covers (a contiguous run,
    // read four instances at a time so that their loads are in flight together)
    float4 q0 = make_float4(0.f, 0.f, 0.f, 0.f), q1 = q0, q2 = q0;
    auto add = [&](const float4* pp) {
      const float4 a0 = pp[0], a1 = pp[1], a2 = pp[2];
      q0.x += a0.x; q0.y += a0.y; q0.z += a0.z; q0.w += a0.w;
      q1.x += a1.x; q1.y += a1.y; q1.z += a1.z; q1.w += a1.w;
      q2.x += a2.x; q2.y += a2.y;
    };
    if (vis) {
      int64_t j = i;
      const int64_t j_stop = min(i + cnt, n_stored);
      for (; j + 4 <= j_stop; j += 4) {
        const float4* pp = ipart + 3 * j;
        float4 b[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) b[k] = pp[k];
#pragma unroll
        for (int k = 0; k < 4; ++k) add(b + 3 * k);
      }
      for (; j < j_stop; ++j) add(ipart + 3 * j);
    }
    if (!vis) continue;
    const float dmx = q0.x, dmy = q0.y, da = q0.z, db = q0.w;
    const float dc = q1.x, d_o = q1.y, dr = q1.z, dg = q1.w;
    const float dbl = q2.x, dz = q2.y;
    float tx, ty, tz;
    camera_point(c, mu[0], mu[1], mu[2], tx, ty, tz);
    Ewa e;
    ewa(c, Sig, tx, ty, tz, op.lowpass, e);
    const float idet = 1.f / e.det;
    const float a = e.C * idet, b = -e.B * idet, cc = e.A * idet;
    // conic (a, b, c) = inverse of [[A, B], [B, C]]
    const float GA = -(a * a * da + a * b * db + b * b * dc);
    const float GC = -(b * b * da + b * cc * db + cc * cc * dc);
    const float GB = -(2.f * a * b * da + (a * cc + b * b) * db + 2.f * b * cc * dc);
    // A = u.Sigma.u, B = u.Sigma.w, C = w.Sigma.w
    const float* u = e.u;
    const float* w = e.w;
    gs[0] += GA * u[0] * u[0] + GB * u[0] * w[0] + GC * w[0] * w[0];
    gs[1] += GA * u[0] * u[1] + 0.5f * GB * (u[0] * w[1] + w[0] * u[1]) + GC * w[0] * w[1];
    gs[2] += GA * u[0] * u[2] + 0.5f * GB * (u[0] * w[2] + w[0] * u[2]) + GC * w[0] * w[2];
    gs[3] += GA * u[1] * u[1] + GB * u[1] * w[1] + GC * w[1] * w[1];
    gs[4] += GA * u[1] * u[2] + 0.5f * GB * (u[1] * w[2] + w[1] * u[2]) + GC * w[1] * w[2];
    gs[5] += GA * u[2] * u[2] + GB * u[2] * w[2] + GC * w[2] * w[2];
    float Gu[3], Gw[3];
    for (int k = 0; k < 3; ++k) {
      Gu[k] = 2.f * GA * e.su[k] + GB * e.sw[k];
      Gw[k] = 2.f * GC * e.sw[k] + GB * e.su[k];
    }
    // u = J00 W_0 + J02 W_2, w = J11 W_1 + J12 W_2 (W_i rows of the camera rotation)
    const float GJ00 = Gu[0] * c.R[0] + Gu[1] * c.R[1] + Gu[2] * c.R[2];
    const float GJ02 = Gu[0] * c.R[6] + Gu[1] * c.R[7] + Gu[2] * c.R[8];
    const float GJ11 = Gw[0] * c.R[3] + Gw[1] * c.R[4] + Gw[2] * c.R[5];
    const float GJ12 = Gw[0] * c.R[6] + Gw[1] * c.R[7] + Gw[2] * c.R[8];
    const float it = e.inv_tz, it2 = it * it, it3 = it2 * it;
    const float gtx = -c.fx * it2 * GJ02 + dmx * c.fx * it;
    const float gty = -c.fy * it2 * GJ12 + dmy * c.fy * it;
    const float gtz = -c.fx * it2 * GJ00 + 2.f * c.fx * tx * it3 * GJ02 - c.fy * it2 * GJ11 +
                      2.f * c.fy * ty * it3 * GJ12 - dmx * c.fx * tx * it2 - dmy * c.fy * ty * it2 + dz;
    for (int j = 0; j < 3; ++j) gmu[j] += c.R[j] * gtx + c.R[3 + j] * gty + c.R[6 + j] * gtz;
    go += d_o;
    // colour
    const float d0 = mu[0] - c.campos[0], d1 = mu[1] - c.campos[1], d2 = mu[2] - c.campos[2];
    const float idist = 1.f / sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
    const float x = d0 * idist, y = d1 * idist, z = d2 * idist;
    float Y[K], pre[3];
    colour<DEG>(f, x, y, z, Y, pre);
    const float grgb[3] = {pre[0] >= 0.f ? dr : 0.f, pre[1] >= 0.f ? dg : 0.f, pre[2] >= 0.f ? dbl : 0.f};
#pragma unroll
    for (int k = 0; k < K; ++k)
      for (int ch = 0; ch < 3; ++ch) gf[k * 3 + ch] += grgb[ch] * Y[k];
    if (DEG > 0) {
      float wk[K];
#pragma unroll
      for (int k = 0; k < K; ++k) wk[k] = grgb[0] * f[k * 3] + grgb[1] * f[k * 3 + 1] + grgb[2] * f[k * 3 + 2];
      float gx, gy, gz;
      sh_dir_grad<DEG>(x, y, z, wk, gx, gy, gz);
      const float dot = gx * x + gy * y + gz * z;
      gmu[0] += (gx - x * dot) * idist;
      gmu[1] += (gy - y * dot) * idist;
      gmu[2] += (gz - z * dot) * idist;
    }
  }
  if (!ADAM && mask == 0) return;
  load_shape();
  float out_mu[3] = {0.f, 0.f, 0.f}, out_ls[3] = {0.f, 0.f, 0.f}, out_q[4] = {0.f, 0.f, 0.f, 0.f}, out_o = 0.f;
  if (mask != 0) {
    Shape s;
    shape_of(ls, qq, opac[gg], s);
    // Sigma = M M^T: dL/dM = 2 Gs M ; M = Rq diag(S)
    const float Gs[9] = {gs[0], gs[1], gs[2], gs[1], gs[3], gs[4], gs[2], gs[4], gs[5]};
    float GM[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        GM[i * 3 + j] = 2.f * (Gs[i * 3] * s.M[j] + Gs[i * 3 + 1] * s.M[3 + j] + Gs[i * 3 + 2] * s.M[6 + j]);
    float GR[9];
    for (int j = 0; j < 3; ++j) {
      const float dS = s.Rq[j] * GM[j] + s.Rq[3 + j] * GM[3 + j] + s.Rq[6 + j] * GM[6 + j];
      out_ls[j] = dS * s.S[j];
      for (int i = 0; i < 3; ++i) GR[i * 3 + j] = GM[i * 3 + j] * s.S[j];
    }
    const float qw = s.q[0], qx = s.q[1], qy = s.q[2], qz = s.q[3];
    float gq[4];
    gq[0] = 2.f * (-qz * GR[1] + qy * GR[2] + qz * GR[3] - qx * GR[5] - qy * GR[6] + qx * GR[7]);
    gq[1] = 2.f * (qy * GR[1] + qz * GR[2] + qy * GR[3] - 2.f * qx * GR[4] - qw * GR[5] + qz * GR[6] + qw * GR[7] -
                   2.f * qx * GR[8]);
    gq[2] = 2.f * (-2.f * qy * GR[0] + qx * GR[1] + qw * GR[2] + qx * GR[3] + qz * GR[5] - qw * GR[6] + qz * GR[7] -
                   2.f * qy * GR[8]);
    gq[3] = 2.f * (-2.f * qz * GR[0] - qw * GR[1] + qx * GR[2] + qw * GR[3] - 2.f * qz * GR[4] + qy * GR[5] +
                   qx * GR[6] + qy * GR[7]);
    const float dq = gq[0] * qw + gq[1] * qx + gq[2] * qy + gq[3] * qz;
    const float iq = 1.f / s.qnorm;
    for (int i = 0; i < 3; ++i) out_mu[i] = gmu[i];
    for (int i = 0; i < 4; ++i) out_q[i] = (gq[i] - s.q[i] * dq) * iq;
    out_o = go * s.o * (1.f - s.o);
  }
  if (!ADAM) {
    for (int i = 0; i < 3; ++i) {
      g_means[g * 3 + i] += out_mu[i];
      g_scales[g * 3 + i] += out_ls[i];
    }
    for (int i = 0; i < 4; ++i) g_quats[g * 4 + i] += out_q[i];
    g_opac[g] += out_o;
#pragma unroll
    for (int i = 0; i < F; ++i) g_sh[g * F + i] += gf[i];
    return;
  }
  const bool live = g < n;
  if (g_means && live) {
    for (int i = 0; i < 3; ++i) {
      g_means[g * 3 + i] = out_mu[i];
      g_scales[g * 3 + i] = out_ls[i];
    }
    for (int i = 0; i < 4; ++i) g_quats[g * 4 + i] = out_q[i];
    g_opac[g] = out_o;
#pragma unroll
    for (int i = 0; i < F; ++i) g_sh[g * F + i] = gf[i];
  }
  if (ad.bias[2] != 0.f) return;  // skipped step (instance capacity overflowed); the same in every thread
  const bool step = live && !(ad.sparse && mask == 0);  // visible-only step: invisible Gaussians stay
  const float bc1 = ad.bias[0], bc2s = ad.bias[1];
  const float b1 = ad.b1, b2 = ad.b2, eps = ad.eps;
  {
    // SH: the wave steps its gradient rows in coalesced runs; the three degree-0 coefficients take lr[4], the
    // others lr[5]
    wb[lane * FP + F] = step ? 0.f : 1.f;
    __syncthreads();
    // U elements per lane at a time: all their loads are issued before the first is used, so a lane waits
    // for memory once per U elements rather than once per element
    constexpr int U = 8;
    const float s4 = ad.lr[4] / bc1, s5 = ad.lr[5] / bc1;
    const int total = nw * F;
    for (int e0 = lane; e0 < total; e0 += 64 * U) {
      float pv[U], mm[U], vv[U];
      bool on[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + 64 * u;
        on[u] = e < total && wb[(e / F) * FP + F] == 0.f;
        const int64_t idx = g0 * F + (on[u] ? e : 0);
        pv[u] = sh[idx];
        mm[u] = ad.m_sh[idx];
        vv[u] = ad.v_sh[idx];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (!on[u]) continue;
        const int e = e0 + 64 * u;
        const int r = e / F, c = e - r * F;
        const int64_t idx = g0 * F + e;
        adam_one(pv[u], mm[u], vv[u], wb[r * FP + c], c < 3 ? s4 : s5, b1, b2, eps, bc2s);
        sh[idx] = pv[u];
        ad.m_sh[idx] = mm[u];
        ad.v_sh[idx] = vv[u];
      }
    }
  }
  if (!step) return;
  // every moment is loaded before the first store (the stores could alias the later loads as far as the
  // compiler knows), so the lane waits for memory once
  float o = opac[g], mo = ad.m_opac[g], vo = ad.v_opac[g];
  float mmu[3], vmu[3], mls[3], vls[3];
  for (int i = 0; i < 3; ++i) {
    mmu[i] = ad.m_means[g * 3 + i];
    vmu[i] = ad.v_means[g * 3 + i];
    mls[i] = ad.m_scales[g * 3 + i];
    vls[i] = ad.v_scales[g * 3 + i];
  }
  float4 mq = reinterpret_cast<const float4*>(ad.m_quats)[g], vq = reinterpret_cast<const float4*>(ad.v_quats)[g];
  const float s0 = ad.lr[0] / bc1, s1 = ad.lr[1] / bc1, s2 = ad.lr[2] / bc1, s3 = ad.lr[3] / bc1;
  adam_one(o, mo, vo, out_o, s3, b1, b2, eps, bc2s);
  for (int i = 0; i < 3; ++i) {
    adam_one(mu[i], mmu[i], vmu[i], out_mu[i], s0, b1, b2, eps, bc2s);
    adam_one(ls[i], mls[i], vls[i], out_ls[i], s1, b1, b2, eps, bc2s);
  }
  adam_one(qq[0], mq.x, vq.x, out_q[0], s2, b1, b2, eps, bc2s);
  adam_one(qq[1], mq.y, vq.y, out_q[1], s2, b1, b2, eps, bc2s);
  adam_one(qq[2], mq.z, vq.z, out_q[2], s2, b1, b2, eps, bc2s);
  adam_one(qq[3], mq.w, vq.w, out_q[3], s2, b1, b2, eps, bc2s);
  opac[g] = o;
  ad.m_opac[g] = mo;
  ad.v_opac[g] = vo;
  for (int i = 0; i < 3; ++i) {
    means[g * 3 + i] = mu[i];
    ad.m_means[g * 3 + i] = mmu[i];
    ad.v_means[g * 3 + i] = vmu[i];
    log_scales[g * 3 + i] = ls[i];
    ad.m_scales[g * 3 + i] = mls[i];
    ad.v_scales[g * 3 + i] = vls[i];
  }
  reinterpret_cast<float4*>(quats)[g] = make_float4(qq[0], qq[1], qq[2], qq[3]);
  reinterpret_cast<float4*>(ad.m_quats)[g] = mq;
  reinterpret_cast<float4*>(ad.v_quats)[g] = vq;
}

}  // namespace

namespace gs_launch {

hipError_t project(const gs_params& p, const gs_frame& f, const gs_opts& o, hipStream_t st) {
  const int threads = 256;
  const int blocks = (int)((p.n + threads - 1) / threads);
  const DevOpts op = gsk::dev_opts(o);
  auto* rec = reinterpret_cast<float4*>(f.rec);
  auto* rect = reinterpret_cast<short4*>(f.rect);
  int32_t* flags = f.counters + 1;
  switch (p.sh_degree) {
    case 0:
      k_project<0><<<blocks, threads, 0, st>>>(p.means, p.log_scales, p.quats, p.opacity, p.sh, p.n, f.cams,
                                               f.n_views, op, rec, rect, f.vis_mask, f.zbits, f.n_rec, f.n_inst, flags);
      break;
    case 1:
      k_project<1><<<blocks, threads, 0, st>>>(p.means, p.log_scales, p.quats, p.opacity, p.sh, p.n, f.cams,
                                               f.n_views, op, rec, rect, f.vis_mask, f.zbits, f.n_rec, f.n_inst, flags);
      break;
    case 2:
      k_project<2><<<blocks, threads, 0, st>>>(p.means, p.log_scales, p.quats, p.opacity, p.sh, p.n, f.cams,
                                               f.n_views, op, rec, rect, f.vis_mask, f.zbits, f.n_rec, f.n_inst, flags);
      break;
    default:
      k_project<3><<<blocks, threads, 0, st>>>(p.means, p.log_scales, p.quats, p.opacity, p.sh, p.n, f.cams,
                                               f.n_views, op, rec, rect, f.vis_mask, f.zbits, f.n_rec, f.n_inst, flags);
      break;
  }
  return hipGetLastError();
}

template <bool ADAM>
static hipError_t project_bwd_launch(const gs_params& p, const gs_frame& f, const gs_opts& o, const gs_params* gr,
                                     const AdamArgs& ad, hipStream_t st) {
  const int threads = 256;
  const int blocks = (int)((p.n + threads - 1) / threads);
  const DevOpts op = gsk::dev_opts(o);
  const auto* ip = reinterpret_cast<const float4*>(f.ipart);
  const auto* rect = reinterpret_cast<const short4*>(f.rect);
  float* gm = gr ? gr->means : nullptr;
  float* gl = gr ? gr->log_scales : nullptr;
  float* gq = gr ? gr->quats : nullptr;
  float* go = gr ? gr->opacity : nullptr;
  float* gsh = gr ? gr->sh : nullptr;
  k_sum_wide<<<1024, 256, 0, st>>>(reinterpret_cast<float4*>(f.ipart), f.big_rec, rect, f.rec_slot, f.counters,
                                   f.rec_cap, f.capacity);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
#define GS_PB(D)                                                                                              \
  k_project_bwd<D, ADAM><<<blocks, threads, 0, st>>>(p.means, p.log_scales, p.quats, p.opacity, p.sh, p.n,     \
                                                     f.cams, f.n_views, op, ip, f.rec_slot, rect, f.counters,    \
                                                     f.capacity, f.vis_mask, gm, gl, gq, go, gsh, ad)
  switch (p.sh_degree) {
    case 0: GS_PB(0); break;
    case 1: GS_PB(1); break;
    case 2: GS_PB(2); break;
    default: GS_PB(3); break;
  }
#undef GS_PB
  return hipGetLastError();
}

hipError_t project_bwd(const gs_params& p, const gs_frame& f, const gs_opts& o, const gs_params& gr, hipStream_t st) {
  AdamArgs none{};
  return project_bwd_launch<false>(p, f, o, &gr, none, st);
}

hipError_t project_bwd_adam(const gs_params& p, const gs_frame& f, const gs_opts& o, const gs_params& m,
                            const gs_params& v, const gs_adam& a, const gs_params* grads_out, hipStream_t st) {
  AdamArgs ad;
  ad.m_means = m.means; ad.m_scales = m.log_scales; ad.m_quats = m.quats; ad.m_opac = m.opacity; ad.m_sh = m.sh;
  ad.v_means = v.means; ad.v_scales = v.log_scales; ad.v_quats = v.quats; ad.v_opac = v.opacity; ad.v_sh = v.sh;
  for (int i = 0; i < 6; ++i) ad.lr[i] = a.lr[i];
  ad.b1 = a.beta1;
  ad.b2 = a.beta2;
  ad.eps = a.eps;
  ad.bias = a.bias;
  ad.sparse = (a.flags & GS_ADAM_SPARSE) ? 1 : 0;
  return project_bwd_launch<true>(p, f, o, grads_out, ad, st);
}

}  // namespace gs_launch
