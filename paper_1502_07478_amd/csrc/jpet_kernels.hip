// gfx950 kernels of libjpet: sensitivity (Eq. 4), buffer fills and the log-likelihood /
// gradient pass.
#include "jpet_device.h"

namespace jpet {

namespace {

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

__global__ void k_fill_u64(unsigned long long* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

__global__ void k_fill_f32(float* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

__global__ void k_fill_f64(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// Direct-reconstruction image: each valid event counted at the pixel containing (y~, z~) of
// Eq. 2 (first forms, double precision); the image is zeroed by the caller.
__global__ void __launch_bounds__(256) k_direct_image(Geo g, double L, const float* __restrict__ events, int64_t n,
                                                      float* __restrict__ img) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const float zu = events[3 * j], zd = events[3 * j + 1], dl = events[3 * j + 2];
    if (!isfinite(zu) || !isfinite(zd) || !isfinite(dl)) continue;
    if (fabs((double)zu) > 0.5 * L || fabs((double)zd) > 0.5 * L) continue;
    const double t = ((double)zu - (double)zd) / (2.0 * g.R);
    const double c = sqrt(1.0 + t * t);
    const double y = -0.5 * (double)dl / c;
    const double z = 0.5 * ((double)zu + (double)zd + 2.0 * y * t);
    const double fi = floor(y / g.pixel + 0.5 * (double)g.n_y);
    const double fk = floor(z / g.pixel + 0.5 * (double)g.n_z);
    if (fi < 0.0 || fi >= (double)g.n_y || fk < 0.0 || fk >= (double)g.n_z) continue;
    atomicAdd(&img[(int64_t)fi * g.n_z + (int64_t)fk], 1.0f);
  }
}

// ------------------------------------------------------------------------------------------
// log-likelihood and gradient

// d log P / du and d log P / dw at a pixel, from the quadratic forms' parts:
//   kappa = u Kz + w Kl + gamma Kg, gamma^ = u Gz + w Gl + gamma Gg, q = u Bz + w Bl,
//   dlogP/du = cu - Kz/(2 kappa) - (Bz - 2 (gamma^/kappa) Gz + (gamma^/kappa)^2 Kz) / 2
//   dlogP/dw = cw - Kl/(2 kappa) - (Bl - 2 (gamma^/kappa) Gl + (gamma^/kappa)^2 Kl) / 2
// with cu, cw the prefactor's share (1/u and 1/(2w) for gamma = 0).
struct RowG {
  float b10, pix;
  float kz0, kzb;   // Kz = kz0 + kzb b1
  float gzb;        // Gz = gzb b1
  float kl, gl, bl; // row constants
  float kg, gg;     // gamma Kg and gamma Gg (row constants)
  float u, w, cu, cw;
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
  r.kg = (float)(-4.0 * g.gamma * g.R * c2 * c * t * (f * Y + 2.0 * dy));
  r.gg = (float)(-4.0 * g.gamma * g.R * c2 * c * dy);
  r.u = (float)g.u;
  r.w = (float)g.w;
  r.cu = (float)g.cu;
  r.cw = (float)g.cw;
  return r;
}

__device__ inline void dlogp(const RowG& r, float jf, float* du, float* dw) {
  const float b1 = fmaf(jf, r.pix, r.b10);
  const float kz = fmaf(r.kzb, b1, r.kz0);
  const float gz = r.gzb * b1;
  const float bz = 2.0f * b1 * b1;
  const float kap = r.u * kz + r.w * r.kl + r.kg;
  const float gam = r.u * gz + r.w * r.gl + r.gg;
  const float ik = 1.0f / kap;
  const float gk = gam * ik;
  *du = r.cu - 0.5f * kz * ik - 0.5f * (bz - 2.0f * gk * gz + gk * gk * kz);
  *dw = r.cw - 0.5f * r.kl * ik - 0.5f * (r.bl - 2.0f * gk * r.gl + gk * gk * r.kl);
}

// Grid-stride over events, one wavefront per event, one lane per ellipse row.  Per block: double
// partial sums of log D', (sum_i rho_i P'_i dlogP_i/du) / D' and the same for w, where
// D' = sum_i rho_i P'_i and P' = P / cnorm; written to red[3 * block + c].
// With B given, sum_j P'_jl / D'_j (= sum_j P_jl / D_j) is added into B with double atomics.
__global__ void __launch_bounds__(256) k_loglik_pass(Geo g, int64_t n, const EventRec* __restrict__ ev,
                                                     const float* __restrict__ rho, double* __restrict__ B,
                                                     float* __restrict__ D_out, double* __restrict__ red,
                                                     unsigned long long* __restrict__ cnt) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wave = threadIdx.x / WAVE;
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
  const float norm = (float)g.cnorm;
  double s_log = 0.0, s_du = 0.0, s_dw = 0.0;
  unsigned long long nzero = 0, nbad_tot = 0;
  for (int64_t j = (int64_t)blockIdx.x * (blockDim.x / WAVE) + wave; j < n; j += nwaves) {
    const EventRec e = ev[j];
    if (e.r1 < e.r0) {
      if (D_out && lane == 0) D_out[j] = 0.0f;
      continue;
    }
    int nbad = 0;  // pixels of this lane's row with kappa <= 0 (P := 0)
    float D = 0.0f, Du = 0.0f, Dw = 0.0f;
    for (int b0 = e.r0; b0 <= e.r1; b0 += WAVE) {
      const int i = b0 + lane;
      int klo, khi;
      if (i <= e.r1 && row_interval(g, e, i, &klo, &khi)) {
        double kf, ks;
        const RowK r = row_constants(g, e, i, klo, &kf, &ks);
        const RowG rg = row_gradient_constants(g, e, i, klo);
        const float* rr = rho + (int64_t)i * g.n_z;
        for (int k = klo; k <= khi; ++k) {
          const float jf = (float)(k - klo);
          const float m = kernel_guarded(r, jf, &nbad) * rr[k];
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
    nbad_tot += wave_sum_u64((unsigned long long)nbad);
    if (D_out && lane == 0) D_out[j] = D * norm;
    if (!(D > 0.0f)) {
      nzero += 1;
      continue;
    }
    s_log += log((double)D);
    s_du += (double)Du / (double)D;
    s_dw += (double)Dw / (double)D;
    if (B) {
      const double invD = 1.0 / (double)D;
      for (int b0 = e.r0; b0 <= e.r1; b0 += WAVE) {
        const int i = b0 + lane;
        int klo, khi;
        if (i <= e.r1 && row_interval(g, e, i, &klo, &khi)) {
          double kf, ks;
          const RowK r = row_constants(g, e, i, klo, &kf, &ks);
          double* bb = B + (int64_t)i * g.n_z;
          int again = 0;  // recomputed values: not counted twice
          for (int k = klo; k <= khi; ++k) {
            const float pv = kernel_guarded(r, (float)(k - klo), &again);
            if (pv != 0.0f) unsafeAtomicAdd(&bb[k], (double)pv * invD);
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
                                                       double* __restrict__ out3, int value_only) {
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
    const double nz = (double)cnt[C_ZERO_DEN];
    // log(D / pi) = log D' + log(cnorm / pi)
    const double lognorm = log(g.cnorm / kPi);
    const double ll = sh[0][0] + (nvalid - nz) * lognorm - sh[3][0];
    out3[0] = nz > 0.0 ? -INFINITY : ll;
    out3[1] = value_only ? NAN : sh[1][0] * (-2.0 * g.u / g.sigma_z);
    out3[2] = value_only ? NAN : sh[2][0] * (-2.0 * g.w / g.sigma_dl);
  }
}

// grad_rho = B - s (s = 1 when absent)
__global__ void k_grad_rho(int64_t npix, const double* __restrict__ B, const float* __restrict__ s,
                           float* __restrict__ out) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (int64_t)gridDim.x * blockDim.x)
    out[p] = (float)(B[p] - (s ? (double)s[p] : 1.0));
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

hipError_t launch_direct_image(const Geo& g, double L, const float* events, int64_t n, float* img, hipStream_t st) {
  const int64_t npix = (int64_t)g.n_y * g.n_z;
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(npix, 256)), dim3(256), 0, st, img, npix);
  if (n > 0) hipLaunchKernelGGL(k_direct_image, dim3(grid_for(n, 256)), dim3(256), 0, st, g, L, events, n, img);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_loglik(const Geo& g, const Plan& p, int64_t n, const Workspace& ws, const float* rho,
                         const float* s, float* D_out, float* grad_rho, double* out3, bool value_only,
                         hipStream_t st) {
  const int64_t npix = (int64_t)g.n_y * g.n_z;
  int nparts;
  if (p.tiled) {
    // binned pass: B accumulated (unless the value alone is asked for), three partial sums
    if (!value_only) hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(npix, 256)), dim3(256), 0, st, ws.B, npix);
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, st, ws.red, (int64_t)3);
    if (D_out) hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n, 256)), dim3(256), 0, st, D_out, n);
    const hipError_t e = launch_loglik_tiled(g, p, n, ws, rho, D_out, value_only, st);
    if (e != hipSuccess) return e;
    nparts = 1;
  } else {
    nparts = grid_for(n, 256 / WAVE, RED_SLOTS / 3);
    if (grad_rho) hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(npix, 256)), dim3(256), 0, st, ws.B, npix);
    hipLaunchKernelGGL(k_loglik_pass, dim3(nparts), dim3(256), 0, st, g, n, ws.ev, rho, grad_rho ? ws.B : nullptr,
                       D_out, ws.red, ws.cnt);
  }
  hipLaunchKernelGGL(k_loglik_finish, dim3(1), dim3(256), 0, st, g, nparts, ws.red, rho, s, ws.cnt, out3,
                     value_only ? 1 : 0);
  if (grad_rho) hipLaunchKernelGGL(k_grad_rho, dim3(grid_for(npix, 256)), dim3(256), 0, st, npix, ws.B, s, grad_rho);
  return hipGetLastError();
}

}  // namespace jpet
