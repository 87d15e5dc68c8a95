// Device helpers shared by the libjpet kernels: the ellipse rows of an event and the kernel
// P(e|i) along a pixel row.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "jpet_internal.h"

namespace jpet {

constexpr int WAVE = 64;
constexpr double kPi = 3.14159265358979323846;
// exp(x) = exp2(x log2 e); the kernel's exponent is -(q - gamma^2 / kappa) / 2
constexpr double kHalfLog2e = 0.72134752044448170368;
// fixed-point unit of the back-projection accumulators: 2^-32
constexpr float kFix = 4294967296.0f;

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// Cross-lane data movement within a wavefront through DPP (VALU, no LDS round trip).
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, true));
}

// Sum over the 64 lanes of a wavefront (all lanes active), returned to every lane: quad
// permutations, half-row and row mirrors give each 16-lane row its sum; two row broadcasts
// accumulate the rows into lane 63, which is read back as a wavefront-uniform value.
__device__ __forceinline__ float wave_sum_dpp(float v) {
  v += dpp_f<0xB1>(v);       // quad_perm [1,0,3,2]
  v += dpp_f<0x4E>(v);       // quad_perm [2,3,0,1]
  v += dpp_f<0x141>(v);      // row_half_mirror
  v += dpp_f<0x140>(v);      // row_mirror
  v += dpp_f<0x142, 0xa>(v); // row_bcast:15 into rows 1 and 3
  v += dpp_f<0x143, 0xc>(v); // row_bcast:31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Lane k's value of v, as a wavefront-uniform value.
__device__ __forceinline__ float lane_value(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

// Sums over each half of a wavefront (all lanes active): the row sums as above, then one row
// broadcast adds row 0 into row 1 and row 2 into row 3, so that lane 31 holds the sum of lanes
// 0-31 and lane 63 the sum of lanes 32-63.
__device__ __forceinline__ float half_sums_dpp(float v) {
  v += dpp_f<0xB1>(v);
  v += dpp_f<0x4E>(v);
  v += dpp_f<0x141>(v);
  v += dpp_f<0x140>(v);
  v += dpp_f<0x142, 0xa>(v);
  return v;
}

__device__ inline int wave_max_i(int v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, WAVE));
  return v;
}

// Column shift of row r in the frame sheared along slope tc (see Plan).
__device__ inline int shear_offset(const Geo& g, double tc, int r) {
  return (int)rint(tc * (g.y0 + (double)r * g.pixel) * g.ipix);
}

// Central slope of t bin b (0 when the binning has no shear).
__device__ inline double bin_slope(const Plan& p, int b) {
  return p.ntb > 1 ? p.tmin + ((double)b + 0.5) * p.dt : 0.0;
}

// Pixel columns [klo, khi] of row i inside the 3-sigma ellipse of event e, for the mask
// resolution (um, wm), um scaled by the event's su (its own sigma_z).  In a row of fixed y the quadratic form b C^-1 b equals
// 2 um b1^2 + 4 wm c^2 dy^2 with b1 = z - z~ - dy tan (Eq. 10-12), so the ellipse (Sec. 3) is the
// interval |z - (z~ + dy tan)| <= sqrt((9 - 4 wm c^2 dy^2) / (2 um)).  Double precision, so the
// pixel set is the one a per-pixel double-precision test b C^-1 b <= 9 selects.
__device__ inline bool row_interval(const Geo& g, const EventRec& e, int i, int* klo, int* khi) {
  const double Y = g.y0 + (double)i * g.pixel;
  const double dy = Y - e.y;
  const double c = e.c;
  const double rem = 9.0 - 4.0 * g.wm * c * c * dy * dy;
  if (!(rem >= 0.0)) return false;
  const double H = sqrt(rem * (0.5 / (g.um * e.su)));
  const double zc = e.z + e.t * dy;
  double a = ceil((zc - H - g.z0) * g.ipix);
  double b = floor((zc + H - g.z0) * g.ipix);
  if (a < 0.0) a = 0.0;
  if (b > (double)(g.n_z - 1)) b = (double)(g.n_z - 1);
  if (a > b) return false;
  *klo = (int)a;
  *khi = (int)b;
  return true;
}

// Single-precision constants of the kernel along one pixel row (Eq. 7-12).
// With Y the row's y, dy = Y - y~ and b1 = z - z~ - dy tan the running coordinate:
//   kappa = aC^-1a + 2 oC^-1b = 2u c^4 (R^2 + Y^2) + w fa^2 Y^2 c^2 t^2 + 4 w c^2 (1 + 2t^2) Y dy
//                              - 4 u t c^2 Y b1
//   gamma = bC^-1a           = 2 fa w c^2 t Y dy - 2 u c^2 Y b1
//   q     = bC^-1b           = 2 u b1^2 + 4 w c^2 dy^2
// and P / cnorm = kappa^-1/2 exp2(S (gamma^2 / kappa - q)) with S = log2(e) / 2.
struct RowK {
  float b10, pix;    // b1 at the row's first pixel and its step
  float kap0, dkap;  // kappa at the first pixel and its step
  float gs0, dgs;    // sqrt(S) gamma at the first pixel and its step
  float a2, aq;      // S q = a2 b1^2 + aq
};

__device__ inline RowK row_constants(const Geo& g, const EventRec& e, int i, int klo, double* kap_first,
                                     double* kap_step) {
  const double Y = g.y0 + (double)i * g.pixel;
  const double dy = Y - e.y;
  const double t = e.t, c = e.c, c2 = c * c;
  const double u = g.u * e.su, w = g.w, f = g.fa;  // u: this event's sigma_z^-2
  const double zc = e.z + t * dy;
  const double b10 = g.z0 + (double)klo * g.pixel - zc;
  const double kap_r = 2.0 * u * c2 * c2 * (g.R * g.R + Y * Y) + w * f * f * Y * Y * c2 * t * t +
                       4.0 * w * c2 * (1.0 + 2.0 * t * t) * Y * dy +
                       -4.0 * g.gamma * g.R * c2 * c * t * (f * Y + 2.0 * dy);
  const double kap_b = -4.0 * u * t * c2 * Y;
  // gamma (Eq. 12): kappa += -4 gamma R c^3 t (f Y + 2 dy), gamma^ += -4 gamma R c^3 dy
  const double c3g = -4.0 * g.gamma * g.R * c2 * c;
  const double gam_r = 2.0 * f * w * c2 * t * Y * dy + c3g * dy;
  const double gam_b = -2.0 * u * c2 * Y;
  const double rs = 0.84932180028801904272;  // sqrt(log2(e) / 2)
  RowK r;
  r.b10 = (float)b10;
  r.pix = (float)g.pixel;
  *kap_first = kap_r + kap_b * b10;
  *kap_step = kap_b * g.pixel;
  r.kap0 = (float)*kap_first;
  r.dkap = (float)*kap_step;
  r.gs0 = (float)(rs * (gam_r + gam_b * b10));
  r.dgs = (float)(rs * gam_b * g.pixel);
  r.a2 = (float)(kHalfLog2e * 2.0 * u);
  r.aq = (float)(kHalfLog2e * 4.0 * w * c2 * dy * dy);
  return r;
}

// P / cnorm at the j-th pixel of the row; kappa must be positive.
__device__ inline float kernel_fast(const RowK& r, float jf) {
  const float b1 = fmaf(jf, r.pix, r.b10);
  const float kap = fmaf(jf, r.dkap, r.kap0);
  const float gs = fmaf(jf, r.dgs, r.gs0);
  const float rk = __builtin_amdgcn_rsqf(kap);
  const float sq = fmaf(r.a2 * b1, b1, r.aq);
  const float arg = fmaf(gs * gs, rk * rk, -sq);
  return rk * __builtin_amdgcn_exp2f(arg);
}

// The same with the kappa <= 0 case (P := 0) handled per pixel; such pixels are counted in nbad.
__device__ inline float kernel_guarded(const RowK& r, float jf, int* nbad) {
  const float kap = fmaf(jf, r.dkap, r.kap0);
  if (!(kap > 0.0f)) {
    ++*nbad;
    return 0.0f;
  }
  return kernel_fast(r, jf);
}

}  // namespace jpet
