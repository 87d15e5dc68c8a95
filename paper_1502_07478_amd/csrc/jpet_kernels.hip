// gfx950 kernels of libjpet: sensitivity (Eq. 4), per-event preparation (Eq. 2, App. B),
// the MLEM event pass (Eq. 7-12 inside the 3-sigma ellipse, Sec. 4 listing), the pixel
// update (Eq. 3/5) and the log-likelihood / gradient pass.
#include <hip/hip_runtime.h>
#include <math.h>

#include "jpet_internal.h"

namespace jpet {

namespace {

constexpr int WAVE = 64;
constexpr double kPi = 3.14159265358979323846;
// exp(x) = exp2(x * log2(e)); the kernel's exponent is -1/2 (q - gamma^2 / kappa)
constexpr double kHalfLog2e = 0.72134752044448170368;

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

// Pixel columns of row i that lie inside the 3-sigma ellipse of event e (mask resolution).
// In a row of fixed y, b C^-1 b = 2 u_m b1^2 + 4 w_m c^2 dy^2 with b1 = z - z~ - dy tan, so the
// ellipse is the interval |z - (z~ + dy tan)| <= sqrt((9 - 4 w_m c^2 dy^2) / (2 u_m)).
// Double precision, so that the pixel set matches a per-pixel test b C^-1 b <= 9.
__device__ inline bool row_interval(const Geo& g, const EventRec& e, int i, int* klo, int* khi) {
  const double Y = g.y0 + (double)i * g.pixel;
  const double dy = Y - e.y;
  const double c = e.c;
  const double rem = 9.0 - 4.0 * g.wm * c * c * dy * dy;
  if (!(rem >= 0.0)) return false;
  const double H = sqrt(rem / (2.0 * g.um));
  const double zc = e.z + e.t * dy;
  double a = ceil((zc - H - g.z0) / g.pixel);
  double b = floor((zc + H - g.z0) / g.pixel);
  if (a < 0.0) a = 0.0;
  if (b > (double)(g.n_z - 1)) b = (double)(g.n_z - 1);
  if (a > b) return false;
  *klo = (int)a;
  *khi = (int)b;
  return true;
}

// Row constants of the kernel (Eq. 7-11, gamma = 0) in single precision, for a row of fixed y.
// With b1 = z - z~ - dy tan along the row and Y the pixel's y:
//   kappa = aC^-1a + 2 oC^-1b = 2u c^4 (R^2 + Y^2) + w fa^2 Y^2 c^2 t^2 + 4 w c^2 (1 + 2t^2) Y dy
//                              - 4 u t c^2 Y b1
//   gamma = bC^-1a           = 2 fa w c^2 t Y dy - 2 u c^2 Y b1
//   q     = bC^-1b           = 2 u b1^2 + 4 w c^2 dy^2
// and P / (u sqrt(w) / 2 pi) = kappa^-1/2 exp2(S (gamma^2 / kappa - q)), S = log2(e) / 2.
struct RowK {
  float b10, pix;      // b1 at the first pixel, step of b1
  float kap0, dkap;    // kappa at the first pixel, step
  float gs0, dgs;      // sqrt(S) gamma at the first pixel, step
  float a2, aq;        // S q = a2 b1^2 + aq
};

__device__ inline RowK row_constants(const Geo& g, const EventRec& e, int i, int klo) {
  const double Y = g.y0 + (double)i * g.pixel;
  const double dy = Y - e.y;
  const double t = e.t, c = e.c, c2 = c * c;
  const double u = g.u, w = g.w, f = g.fa;
  const double zc = e.z + t * dy;
  const double b10 = g.z0 + (double)klo * g.pixel - zc;
  const double kap_r = 2.0 * u * c2 * c2 * (g.R * g.R + Y * Y) + w * f * f * Y * Y * c2 * t * t +
                       4.0 * w * c2 * (1.0 + 2.0 * t * t) * Y * dy;
  const double kap_b = -4.0 * u * t * c2 * Y;
  const double gam_r = 2.0 * f * w * c2 * t * Y * dy;
  const double gam_b = -2.0 * u * c2 * Y;
  const double rs = sqrt(kHalfLog2e);
  RowK r;
  r.b10 = (float)b10;
  r.pix = (float)g.pixel;
  r.kap0 = (float)(kap_r + kap_b * b10);
  r.dkap = (float)(kap_b * g.pixel);
  r.gs0 = (float)(rs * (gam_r + gam_b * b10));
  r.dgs = (float)(rs * gam_b * g.pixel);
  r.a2 = (float)(kHalfLog2e * 2.0 * u);
  r.aq = (float)(kHalfLog2e * 4.0 * w * c2 * dy * dy);
  return r;
}

// Kernel value (without the constant u sqrt(w) / 2 pi) at the j-th pixel of the row.
__device__ inline float kernel_at(const RowK& r, float jf, bool* bad) {
  const float b1 = fmaf(jf, r.pix, r.b10);
  const float kap = fmaf(jf, r.dkap, r.kap0);
  const float gs = fmaf(jf, r.dgs, r.gs0);
  if (!(kap > 0.0f)) {
    *bad = true;
    return 0.0f;
  }
  const float rk = __builtin_amdgcn_rsqf(kap);
  const float sq = fmaf(r.a2 * b1, b1, r.aq);
  const float arg = fmaf(gs * gs, rk * rk, -sq);
  return rk * __builtin_amdgcn_exp2f(arg);
}

// ------------------------------------------------------------------------------------------

__global__ void k_sensitivity(Geo g, float* s) {
  const int64_t npix = (int64_t)g.n_y * g.n_z;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(p / g.n_z), k = (int)(p - (int64_t)i * g.n_z);
    const double y = g.y0 + i * g.pixel, z = g.z0 + k * g.pixel;
    const double hl = 0.5 * g.L, R = g.R;
    const double hi = fmin((hl - z) / (R - y), (hl + z) / (R + y));
    const double lo = fmax(-(hl + z) / (R - y), (z - hl) / (R + y));
    const double v = (atan(hi) - atan(lo)) / kPi;
    s[p] = v > 0.0 ? (float)v : 0.0f;
  }
}

// One thread per event: direct reconstruction (Eq. 2), ellipse rows (App. B), pixel count.
__global__ void k_prepare(Geo g, const float* __restrict__ events, int64_t n, EventRec* __restrict__ ev,
                          unsigned long long* __restrict__ cnt) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long valid = 0, pairs = 0;
  if (j < n) {
    const float zu = events[3 * j], zd = events[3 * j + 1], dl = events[3 * j + 2];
    EventRec e;
    e.r0 = 0;
    e.r1 = -1;
    e.npix = 0;
    e.pad = 0;
    e.t = e.c = e.y = e.z = 0.0;
    const double hl = 0.5 * g.L;
    if (isfinite(zu) && isfinite(zd) && isfinite(dl) && fabs((double)zu) <= hl && fabs((double)zd) <= hl) {
      const double t = ((double)zu - (double)zd) / (2.0 * g.R);
      const double c = sqrt(1.0 + t * t);
      const double y = -0.5 * (double)dl / c;
      const double z = 0.5 * ((double)zu + (double)zd + 2.0 * y * t);
      e.t = t;
      e.c = c;
      e.y = y;
      e.z = z;
      // rows whose centre lies within the half height 1.5 sigma_dl / c of the ellipse
      const double hy = 1.5 / (sqrt(g.wm) * c);
      double a = ceil((y - hy - g.y0) / g.pixel);
      double b = floor((y + hy - g.y0) / g.pixel);
      if (a < 0.0) a = 0.0;
      if (b > (double)(g.n_y - 1)) b = (double)(g.n_y - 1);
      int first = 1 << 30, last = -1;
      long long cntp = 0;
      for (int i = (int)a; i <= (int)b && a <= b; ++i) {
        int klo, khi;
        if (row_interval(g, e, i, &klo, &khi)) {
          if (first > i) first = i;
          last = i;
          cntp += khi - klo + 1;
        }
      }
      if (cntp > 0) {
        e.r0 = first;
        e.r1 = last;
        e.npix = (int)cntp;
        valid = 1;
        pairs = (unsigned long long)cntp;
      }
    }
    ev[j] = e;
  }
  const unsigned long long v = wave_sum_u64(valid), p = wave_sum_u64(pairs),
                           in = wave_sum_u64(j < n ? 1ull : 0ull);
  if ((threadIdx.x & (WAVE - 1)) == 0 && in) {
    atomicAdd(&cnt[C_VALID], v);
    atomicAdd(&cnt[C_DROPPED], in - v);
    atomicAdd(&cnt[C_PAIRS], p);
  }
}

__global__ void k_fill_u64(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

__global__ void k_fill_f32(float* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

// One wavefront per event, one lane per ellipse row.  Pass 1 forms D = sum P rho, pass 2 adds
// rho P / D into the accumulator image.
__global__ void __launch_bounds__(256) k_event_pass(Geo g, int64_t n, const EventRec* __restrict__ ev,
                                                    const float* __restrict__ rho, float* __restrict__ acc,
                                                    unsigned long long* __restrict__ cnt) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t j = (int64_t)blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x / WAVE);
  if (j >= n) return;
  const EventRec e = ev[j];
  if (e.r1 < e.r0) return;
  bool bad = false;
  float D = 0.0f;
  for (int base = e.r0; base <= e.r1; base += WAVE) {
    const int i = base + lane;
    int klo, khi;
    if (i <= e.r1 && row_interval(g, e, i, &klo, &khi)) {
      const RowK r = row_constants(g, e, i, klo);
      const float* rr = rho + (int64_t)i * g.n_z;
      for (int k = klo; k <= khi; ++k) D += kernel_at(r, (float)(k - klo), &bad) * rr[k];
    }
  }
  D = wave_sum(D);
  const unsigned long long nbad = wave_sum_u64(bad ? 1ull : 0ull);
  if (lane == 0 && nbad) atomicAdd(&cnt[C_KAPPA_BAD], nbad);
  if (!(D > 0.0f)) {
    if (lane == 0) atomicAdd(&cnt[C_ZERO_DEN], 1ull);
    return;
  }
  const float invD = 1.0f / D;
  for (int base = e.r0; base <= e.r1; base += WAVE) {
    const int i = base + lane;
    int klo, khi;
    if (i <= e.r1 && row_interval(g, e, i, &klo, &khi)) {
      const RowK r = row_constants(g, e, i, klo);
      const float* rr = rho + (int64_t)i * g.n_z;
      float* aa = acc + (int64_t)i * g.n_z;
      for (int k = klo; k <= khi; ++k) {
        const float m = kernel_at(r, (float)(k - klo), &bad) * rr[k];
        if (m != 0.0f) unsafeAtomicAdd(&aa[k], m * invD);
      }
    }
  }
}

// rho_l = acc_l / s_l (0 where s_l = 0), or acc_l without a sensitivity image; acc is cleared.
__global__ void k_update(int64_t npix, const float* __restrict__ s, float* __restrict__ rho, float* __restrict__ acc) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (int64_t)gridDim.x * blockDim.x) {
    const float a = acc[p];
    float v;
    if (s) {
      const float sv = s[p];
      v = sv > 0.0f ? a / sv : 0.0f;
    } else {
      v = a;
    }
    rho[p] = v;
    acc[p] = 0.0f;
  }
}

// ------------------------------------------------------------------------------------------
// log-likelihood and gradient

// d log P / du and d log P / dw at a pixel (gamma = 0), from the quadratic forms' parts:
//   kappa = u Kz + w Kl, gamma = u Gz + w Gl, q = u Bz + w Bl,
//   dlogP/du = 1/u - Kz/(2 kappa) - (Bz - 2 (gamma/kappa) Gz + (gamma/kappa)^2 Kz) / 2
//   dlogP/dw = 1/(2w) - Kl/(2 kappa) - (Bl - 2 (gamma/kappa) Gl + (gamma/kappa)^2 Kl) / 2
struct RowG {
  float b10, pix;
  float kz0, kzb;   // Kz = kz0 + kzb b1
  float gzb;        // Gz = gzb b1
  float kl, gl, bl; // row constants
  float u, w;
};

__device__ inline RowG row_gradient_constants(const Geo& g, const EventRec& e, int i, int klo) {
  const double Y = g.y0 + (double)i * g.pixel;
  const double dy = Y - e.y;
  const double t = e.t, c = e.c, c2 = c * c, f = g.fa;
  const double zc = e.z + t * dy;
  RowG r;
  r.b10 = (float)(g.z0 + (double)klo * g.pixel - zc);
  r.pix = (float)g.pixel;
  r.kz0 = (float)(2.0 * c2 * c2 * (g.R * g.R + Y * Y));
  r.kzb = (float)(-4.0 * t * c2 * Y);
  r.gzb = (float)(-2.0 * c2 * Y);
  r.kl = (float)(f * f * Y * Y * c2 * t * t + 4.0 * c2 * (1.0 + 2.0 * t * t) * Y * dy);
  r.gl = (float)(2.0 * f * c2 * t * Y * dy);
  r.bl = (float)(4.0 * c2 * dy * dy);
  r.u = (float)g.u;
  r.w = (float)g.w;
  return r;
}

__device__ inline void dlogp(const RowG& r, float jf, float* du, float* dw) {
  const float b1 = fmaf(jf, r.pix, r.b10);
  const float kz = fmaf(r.kzb, b1, r.kz0);
  const float gz = r.gzb * b1;
  const float bz = 2.0f * b1 * b1;
  const float kap = r.u * kz + r.w * r.kl;
  const float gam = r.u * gz + r.w * r.gl;
  const float ik = 1.0f / kap;
  const float gk = gam * ik;
  *du = 1.0f / r.u - 0.5f * kz * ik - 0.5f * (bz - 2.0f * gk * gz + gk * gk * kz);
  *dw = 0.5f / r.w - 0.5f * r.kl * ik - 0.5f * (r.bl - 2.0f * gk * r.gl + gk * gk * r.kl);
}

// Grid-stride over events, one wavefront per event.  Per block: double partial sums of
// log D', (sum rho P dlogP/du)/D', (sum rho P dlogP/dw)/D' into red[3 * block + c].
__global__ void __launch_bounds__(256) k_loglik_pass(Geo g, int64_t n, const EventRec* __restrict__ ev,
                                                     const float* __restrict__ rho, float* __restrict__ B,
                                                     float* __restrict__ D_out, double* __restrict__ red,
                                                     unsigned long long* __restrict__ cnt) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wave = threadIdx.x / WAVE;
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
  double s_log = 0.0, s_du = 0.0, s_dw = 0.0;
  unsigned long long nzero = 0, nbad_tot = 0;
  for (int64_t j = (int64_t)blockIdx.x * (blockDim.x / WAVE) + wave; j < n; j += nwaves) {
    const EventRec e = ev[j];
    if (e.r1 < e.r0) {
      if (D_out && lane == 0) D_out[j] = 0.0f;
      continue;
    }
    bool bad = false;
    float D = 0.0f, Du = 0.0f, Dw = 0.0f;
    for (int base = e.r0; base <= e.r1; base += WAVE) {
      const int i = base + lane;
      int klo, khi;
      if (i <= e.r1 && row_interval(g, e, i, &klo, &khi)) {
        const RowK r = row_constants(g, e, i, klo);
        const RowG rg = row_gradient_constants(g, e, i, klo);
        const float* rr = rho + (int64_t)i * g.n_z;
        for (int k = klo; k <= khi; ++k) {
          const float jf = (float)(k - klo);
          const float m = kernel_at(r, jf, &bad) * rr[k];
          float du, dw;
          dlogp(rg, jf, &du, &dw);
          D += m;
          Du = fmaf(m, du, Du);
          Dw = fmaf(m, dw, Dw);
        }
      }
    }
    D = wave_sum(D);
    Du = wave_sum(Du);
    Dw = wave_sum(Dw);
    nbad_tot += wave_sum_u64(bad ? 1ull : 0ull);
    if (D_out && lane == 0) D_out[j] = D * (float)(g.u * sqrt(g.w) / (2.0 * kPi));
    if (!(D > 0.0f)) {
      nzero += 1;
      continue;
    }
    s_log += log((double)D);
    s_du += (double)Du / (double)D;
    s_dw += (double)Dw / (double)D;
    if (B) {
      const float invD = 1.0f / D;
      for (int base = e.r0; base <= e.r1; base += WAVE) {
        const int i = base + lane;
        int klo, khi;
        if (i <= e.r1 && row_interval(g, e, i, &klo, &khi)) {
          const RowK r = row_constants(g, e, i, klo);
          float* bb = B + (int64_t)i * g.n_z;
          for (int k = klo; k <= khi; ++k) {
            const float p = kernel_at(r, (float)(k - klo), &bad);
            if (p != 0.0f) unsafeAtomicAdd(&bb[k], p * invD);
          }
        }
      }
    }
  }
  __shared__ double part[3][256 / WAVE];
  if (lane == 0) {
    part[0][wave] = s_log;
    part[1][wave] = s_du;
    part[2][wave] = s_dw;
    if (nzero) atomicAdd(&cnt[C_ZERO_DEN], nzero);
    if (nbad_tot) atomicAdd(&cnt[C_KAPPA_BAD], nbad_tot);
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double v = 0.0;
    for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) v += part[threadIdx.x][w];
    red[3 * blockIdx.x + threadIdx.x] = v;
  }
}

// Single block: fixed-order sum of the block partials, sum_l s_l rho_l, and the final scalars.
__global__ void __launch_bounds__(256) k_loglik_finish(Geo g, int nblocks, const double* __restrict__ red,
                                                       const float* __restrict__ rho, const float* __restrict__ s,
                                                       const unsigned long long* __restrict__ cnt,
                                                       double* __restrict__ out3) {
  __shared__ double sh[4][256];
  double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
  for (int q = threadIdx.x; q < nblocks; q += blockDim.x) {
    a += red[3 * q];
    b += red[3 * q + 1];
    c += red[3 * q + 2];
  }
  const int64_t npix = (int64_t)g.n_y * g.n_z;
  for (int64_t p = threadIdx.x; p < npix; p += blockDim.x) d += (double)(s ? s[p] : 1.0f) * (double)rho[p];
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  sh[2][threadIdx.x] = c;
  sh[3][threadIdx.x] = d;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
      for (int m = 0; m < 4; ++m) sh[m][threadIdx.x] += sh[m][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double nvalid = (double)cnt[C_VALID];
    // log(D / pi) with D = (u sqrt(w) / 2 pi) D'
    const double lognorm = log(g.u * sqrt(g.w) / (2.0 * kPi) / kPi);
    const double nz = (double)cnt[C_ZERO_DEN];
    const double ll = sh[0][0] + (nvalid - nz) * lognorm - sh[3][0];
    out3[0] = nz > 0.0 ? -INFINITY : ll;
    out3[1] = sh[1][0] * (-2.0 * g.u / g.sigma_z);
    out3[2] = sh[2][0] * (-2.0 * g.w / g.sigma_dl);
  }
}

// grad_rho = B - s (s = 1 when absent)
__global__ void k_grad_rho(int64_t npix, const float* __restrict__ B, const float* __restrict__ s, float* __restrict__ out) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (int64_t)gridDim.x * blockDim.x)
    out[p] = B[p] - (s ? s[p] : 1.0f);
}

int grid_for(int64_t n, int block, int cap = 65536) {
  int64_t b = (n + block - 1) / block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

}  // namespace

hipError_t launch_sensitivity(const Geo& g, float* s, hipStream_t st) {
  const int64_t npix = (int64_t)g.n_y * g.n_z;
  hipLaunchKernelGGL(k_sensitivity, dim3(grid_for(npix, 256)), dim3(256), 0, st, g, s);
  return hipGetLastError();
}

hipError_t launch_prepare(const Geo& g, const float* events, int64_t n, const Workspace& ws, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_prepare, dim3((unsigned)blocks), dim3(256), 0, st, g, events, n, ws.ev, ws.cnt);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u64, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_event_pass(const Geo& g, int64_t n, const Workspace& ws, const float* rho, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 3) / 4;
  hipLaunchKernelGGL(k_event_pass, dim3((unsigned)blocks), dim3(256), 0, st, g, n, ws.ev, rho, ws.acc, ws.cnt);
  return hipGetLastError();
}

hipError_t launch_update(const Geo& g, const float* s, float* rho, const Workspace& ws, hipStream_t st) {
  const int64_t npix = (int64_t)g.n_y * g.n_z;
  hipLaunchKernelGGL(k_update, dim3(grid_for(npix, 256)), dim3(256), 0, st, npix, s, rho, ws.acc);
  return hipGetLastError();
}

hipError_t launch_loglik(const Geo& g, int64_t n, const Workspace& ws, const float* rho, const float* s,
                         float* D_out, float* grad_rho, double* out3, hipStream_t st) {
  const int64_t npix = (int64_t)g.n_y * g.n_z;
  const int blocks = grid_for(n, 256 / WAVE, RED_SLOTS / 3);
  if (grad_rho) {
    hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(npix, 256)), dim3(256), 0, st, ws.acc, npix);
  }
  hipLaunchKernelGGL(k_loglik_pass, dim3(blocks), dim3(256), 0, st, g, n, ws.ev, rho, grad_rho ? ws.acc : nullptr,
                     D_out, ws.red, ws.cnt);
  hipLaunchKernelGGL(k_loglik_finish, dim3(1), dim3(256), 0, st, g, blocks, ws.red, rho, s, ws.cnt, out3);
  if (grad_rho) {
    hipLaunchKernelGGL(k_grad_rho, dim3(grid_for(npix, 256)), dim3(256), 0, st, npix, ws.acc, s, grad_rho);
  }
  return hipGetLastError();
}

}  // namespace jpet
