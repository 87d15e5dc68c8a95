// The MLEM event pass (Sec. 4 listing with the kernel of Eq. 7-12) and the pixel update (Eq. 3/5).
//
// Tiled pass: one workgroup per (bin, chunk of events).  The workgroup stages its bin's region of
// the current image in LDS, then processes the chunk in batches.  Within a batch every thread
// owns one pixel row of one event's 3-sigma ellipse:
//   pass 1  walks its row, evaluates the kernel at each pixel, multiplies by rho from LDS and
//           keeps m = P rho in registers; the per-event denominators D = sum m are formed by a
//           segmented wavefront reduction and a double-precision LDS add;
//   pass 2  adds m / D in 2^-32 fixed point into the region's 64-bit LDS accumulators.
// After the last batch the region's accumulators are added to the global 64-bit accumulator
// image with one atomic per touched pixel.  Integer accumulation makes the new image exact
// and independent of the order in which events are processed.
//
// The constant factor u sqrt(w) / (2 pi) of Eq. 7 cancels in m / D and is not applied.
#include "jpet_device.h"

namespace jpet {

namespace {

constexpr int kMaxBatch = 64;

struct BatchShared {
  EventRec ev[2][kMaxBatch];  // double buffer: the next batch is fetched while this one runs
  int cum[kMaxBatch + 1];
  double D[kMaxBatch];
  unsigned zero, bad, outside;
};

// The region is stored column-major with a row pitch that is a multiple of the LDS bank count:
// the lanes of a wavefront hold consecutive rows of one event, so the pixel at column offset j
// of every lane's row falls into a different bank whatever the slant of the ellipse.
constexpr int kChunk = 4;  // pixels evaluated per branch-free step

template <int MAXLEN, bool GUARD>
__device__ __forceinline__ float pass1(const RowK& rk, const float* __restrict__ rho_s, int base, int pitch, int len,
                                       int wl, float (&m)[MAXLEN], bool* bad) {
  float D = 0.0f;
#pragma unroll
  for (int j0 = 0; j0 < MAXLEN; j0 += kChunk) {
    if (j0 < wl) {  // wavefront-uniform
      float r[kChunk];
#pragma unroll
      for (int jj = 0; jj < kChunk; ++jj) r[jj] = rho_s[base + (j0 + jj) * pitch];
#pragma unroll
      for (int jj = 0; jj < kChunk; ++jj) {
        const int j = j0 + jj;
        const float pv = GUARD ? kernel_guarded(rk, (float)j, bad) : kernel_fast(rk, (float)j);
        const float v = j < len ? pv * r[jj] : 0.0f;
        m[j] = v;
        D += v;
      }
    } else {
#pragma unroll
      for (int jj = 0; jj < kChunk; ++jj) m[j0 + jj] = 0.0f;
    }
  }
  return D;
}

template <int MAXLEN, bool PRESCALE>
__device__ __forceinline__ void pass2(const float (&m)[MAXLEN], float sc, int base, int pitch, int len, int wl,
                                      unsigned long long* __restrict__ acc_s) {
#pragma unroll
  for (int j = 0; j < MAXLEN; ++j) {
    if (j < wl && j < len) {
      const float x = PRESCALE ? m[j] * 18446744073709551616.0f : m[j];
      atomicAdd(&acc_s[base + j * pitch], (unsigned long long)(unsigned)fmaf(x, sc, 0.5f));
    }
  }
}

template <int MAXLEN, int WAVES>
__global__ void __launch_bounds__(WAVES * 64, 4) k_event_pass_tiled(Geo g, Plan p, const EventRec* __restrict__ evs,
                                                           const BinItem* __restrict__ items,
                                                           const float* __restrict__ rho,
                                                           unsigned long long* __restrict__ acc,
                                                           unsigned long long* __restrict__ cnt) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ BatchShared bs;
  const int pitch = p.pitch;  // rows of a column in LDS (a multiple of the bank count)
  const int npx = pitch * p.W;
  // the image first, then the accumulators: reads past the end of a row (masked lanes) land in
  // the accumulator array, which is larger than MAXLEN columns of the image
  float* rho_s = reinterpret_cast<float*>(smem);
  unsigned long long* acc_s = reinterpret_cast<unsigned long long*>(smem + (size_t)npx * sizeof(float));

  if ((unsigned long long)blockIdx.x >= cnt[C_ITEMS]) return;  // uniform over the workgroup
  const BinItem it = items[blockIdx.x];
  const int tz = it.bin % p.ntz;
  const int rest = it.bin / p.ntz;
  const int ty = rest % p.nty;
  const int tb = rest / p.nty;
  const double tc = bin_slope(p, tb);
  const int kmin = -max(shear_offset(g, tc, 0), shear_offset(g, tc, g.n_y - 1));
  const int rbase = ty * p.TY - p.HY;
  const int kbase = kmin + tz * p.TZ - p.HZ;
  const int tid = threadIdx.x;
  const int lane = tid & (WAVE - 1);

  // stage the region of the current image (column-major), clear the accumulators
  for (int q = tid; q < npx; q += blockDim.x) {
    const int cl = q / pitch;
    const int rl = q - cl * pitch;
    const int r = rbase + rl;
    float v = 0.0f;
    if (rl < p.RY && r >= 0 && r < g.n_y) {
      const int k = kbase + cl + shear_offset(g, tc, r);
      if (k >= 0 && k < g.n_z) v = rho[(int64_t)r * g.n_z + k];
    }
    rho_s[q] = v;
    acc_s[q] = 0ull;
  }
  if (tid == 0) {
    bs.zero = 0u;
    bs.bad = 0u;
    bs.outside = 0u;
  }
  if (tid < min(p.ev_per_batch, it.count)) bs.ev[0][tid] = evs[it.start + tid];

  int buf = 0;
  for (int e0 = 0; e0 < it.count; e0 += p.ev_per_batch, buf ^= 1) {
    const int nb = min(p.ev_per_batch, it.count - e0);
    if (tid < nb) bs.D[tid] = 0.0;
    __syncthreads();
    // fetch the next batch into the other buffer; it is read only after this batch's barriers
    {
      const int n1 = min(p.ev_per_batch, it.count - e0 - nb);
      if (tid < n1) bs.ev[buf ^ 1][tid] = evs[it.start + e0 + nb + tid];
    }
    const EventRec* bev = bs.ev[buf];
    if (tid < WAVE) {  // rows per event, exclusive scan by the first wavefront
      int nr = tid < nb ? bev[tid].r1 - bev[tid].r0 + 1 : 0;
      int incl = nr;
#pragma unroll
      for (int off = 1; off < WAVE; off <<= 1) {
        const int o = __shfl_up(incl, off, WAVE);
        if (lane >= off) incl += o;
      }
      if (tid < nb) bs.cum[tid] = incl - nr;
      if (tid == nb - 1) bs.cum[nb] = incl;
    }
    __syncthreads();

    // this thread's row: event e (largest with cum[e] <= tid), row i
    const int total = bs.cum[nb];
    int e = 0, len = 0, base = 0;
    bool safe = true;
    RowK rk;
    if (tid < total) {
      int lo = 0, hi = nb - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bs.cum[mid] <= tid) lo = mid; else hi = mid - 1;
      }
      e = lo;
      const EventRec ev = bev[e];
      const int i = ev.r0 + (tid - bs.cum[e]);
      int klo, khi;
      if (row_interval(g, ev, i, &klo, &khi)) {
        const int rl = i - rbase;
        const int kl = klo - shear_offset(g, tc, i) - kbase;
        const int n = khi - klo + 1;
        if (rl < 0 || rl >= p.RY || kl < 0 || kl + n > p.W || n > MAXLEN) {
          atomicAdd(&bs.outside, 1u);
        } else {
          double kf, ks;
          rk = row_constants(g, ev, i, klo, &kf, &ks);
          const double kl_end = kf + ks * (double)(n - 1);
          safe = kf > 1e-3 * fabs(kf) + 1e-30 && kl_end > 1e-3 * fabs(kf) + 1e-30;
          len = n;
          base = kl * pitch + rl;
        }
      }
    }

    // pass 1: m = P rho along the row, D partial sums
    float m[MAXLEN];
    const int wl = wave_max_i(len);
    bool bad = false;
    float D;
    if (__any(!safe)) {
      D = pass1<MAXLEN, true>(rk, rho_s, base, pitch, len, wl, m, &bad);
    } else {
      D = pass1<MAXLEN, false>(rk, rho_s, base, pitch, len, wl, m, &bad);
    }
    if (bad) atomicAdd(&bs.bad, 1u);

    // per-event denominators: segmented reduction over the wavefront's rows
    unsigned long long act = __ballot(len > 0);
    while (act) {
      const int leader = __ffsll((long long)act) - 1;
      const int el = __shfl(e, leader, WAVE);
      const bool mine = len > 0 && e == el;
      const float v = wave_sum(mine ? D : 0.0f);
      if (lane == leader) atomicAdd(&bs.D[el], (double)v);
      act &= ~__ballot(mine);
    }
    __syncthreads();

    // pass 2: m / D into the region accumulators (2^-32 fixed point)
    {
      const double Dd = len > 0 ? bs.D[e] : 1.0;
      if (len > 0 && !(Dd > 0.0) && tid == bs.cum[e]) atomicAdd(&bs.zero, 1u);
      const int n2 = Dd > 0.0 ? len : 0;
      // 2^32 / D overflows a float only for D < 1.3e-29; such wavefronts pre-scale m by 2^64
      if (__any(n2 > 0 && Dd < 1e-28)) {
        const float sc = (float)(4294967296.0 / (Dd * 18446744073709551616.0));
        pass2<MAXLEN, true>(m, sc, base, pitch, n2, wl, acc_s);
      } else {
        const float sc = (float)(4294967296.0 / Dd);
        pass2<MAXLEN, false>(m, sc, base, pitch, n2, wl, acc_s);
      }
    }
    __syncthreads();
  }

  // add the region's accumulators to the global image
  for (int q = tid; q < npx; q += blockDim.x) {
    const unsigned long long a = acc_s[q];
    if (a == 0ull) continue;
    const int cl = q / pitch;
    const int rl = q - cl * pitch;
    const int r = rbase + rl;
    const int k = kbase + cl + shear_offset(g, tc, r);
    if (rl < p.RY && r >= 0 && r < g.n_y && k >= 0 && k < g.n_z) atomicAdd(&acc[(int64_t)r * g.n_z + k], a);
  }
  if (tid == 0) {
    if (bs.zero) atomicAdd(&cnt[C_ZERO_DEN], (unsigned long long)bs.zero);
    if (bs.bad) atomicAdd(&cnt[C_KAPPA_BAD], (unsigned long long)bs.bad);
    if (bs.outside) atomicAdd(&cnt[C_OUTSIDE], (unsigned long long)bs.outside);
  }
}

// Generic pass for geometries whose rows or regions do not fit the tiled pass: one wavefront per
// event, one lane per row, kernel values recomputed in pass 2, fixed-point global atomics.
__global__ void __launch_bounds__(256) k_event_pass_generic(Geo g, int64_t n, const EventRec* __restrict__ ev,
                                                            const float* __restrict__ rho,
                                                            unsigned long long* __restrict__ acc,
                                                            unsigned long long* __restrict__ cnt) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t j = (int64_t)blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x / WAVE);
  if (j >= n) return;
  const EventRec e = ev[j];
  if (e.r1 < e.r0) return;
  bool bad = false;
  float D = 0.0f;
  for (int b0 = e.r0; b0 <= e.r1; b0 += WAVE) {
    const int i = b0 + lane;
    int klo, khi;
    if (i <= e.r1 && row_interval(g, e, i, &klo, &khi)) {
      double kf, ks;
      const RowK r = row_constants(g, e, i, klo, &kf, &ks);
      const float* rr = rho + (int64_t)i * g.n_z;
      for (int k = klo; k <= khi; ++k) D += kernel_guarded(r, (float)(k - klo), &bad) * rr[k];
    }
  }
  D = wave_sum(D);
  const unsigned long long nbad = wave_sum_u64(bad ? 1ull : 0ull);
  if (lane == 0 && nbad) atomicAdd(&cnt[C_KAPPA_BAD], nbad);
  if (!(D > 0.0f)) {
    if (lane == 0) atomicAdd(&cnt[C_ZERO_DEN], 1ull);
    return;
  }
  const float sc = (float)(4294967296.0 / (double)D);
  for (int b0 = e.r0; b0 <= e.r1; b0 += WAVE) {
    const int i = b0 + lane;
    int klo, khi;
    if (i <= e.r1 && row_interval(g, e, i, &klo, &khi)) {
      double kf, ks;
      const RowK r = row_constants(g, e, i, klo, &kf, &ks);
      const float* rr = rho + (int64_t)i * g.n_z;
      unsigned long long* aa = acc + (int64_t)i * g.n_z;
      for (int k = klo; k <= khi; ++k) {
        const float m = kernel_guarded(r, (float)(k - klo), &bad) * rr[k];
        if (m > 0.0f) atomicAdd(&aa[k], (unsigned long long)(unsigned)fmaf(m, sc, 0.5f));
      }
    }
  }
}

// rho_l = acc_l 2^-32 / s_l (0 where s_l = 0), or acc_l 2^-32 without sensitivity; acc cleared.
__global__ void k_update(int64_t npix, const float* __restrict__ s, float* __restrict__ rho,
                         unsigned long long* __restrict__ acc) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < npix; q += (int64_t)gridDim.x * blockDim.x) {
    const double a = (double)acc[q] * 2.3283064365386962890625e-10;
    double v;
    if (s) {
      const float sv = s[q];
      v = sv > 0.0f ? a / (double)sv : 0.0;
    } else {
      v = a;
    }
    rho[q] = (float)v;
    acc[q] = 0ull;
  }
}

template <int MAXLEN, int WAVES>
hipError_t launch_tiled(const Geo& g, const Plan& p, const Workspace& ws, const float* rho, hipStream_t st) {
  auto kern = k_event_pass_tiled<MAXLEN, WAVES>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)p.max_items), dim3(64 * p.waves), p.lds_bytes, st, g, p, ws.evs, ws.items,
                     rho, ws.acc, ws.cnt);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_event_pass(const Geo& g, const Plan& p, int64_t n, const Workspace& ws, const float* rho,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (p.tiled) {
    const int key = p.maxlen * 100 + p.waves;
    switch (key) {
      case 1608: return launch_tiled<16, 8>(g, p, ws, rho, st);
      case 3208: return launch_tiled<32, 8>(g, p, ws, rho, st);
      case 4808: return launch_tiled<48, 8>(g, p, ws, rho, st);
      case 6408: return launch_tiled<64, 8>(g, p, ws, rho, st);
      case 1616: return launch_tiled<16, 16>(g, p, ws, rho, st);
      case 3216: return launch_tiled<32, 16>(g, p, ws, rho, st);
      case 4816: return launch_tiled<48, 16>(g, p, ws, rho, st);
      case 6416: return launch_tiled<64, 16>(g, p, ws, rho, st);
      default: return hipErrorInvalidValue;
    }
  }
  const int64_t blocks = (n + 3) / 4;
  hipLaunchKernelGGL(k_event_pass_generic, dim3((unsigned)blocks), dim3(256), 0, st, g, n, ws.ev, rho, ws.acc, ws.cnt);
  return hipGetLastError();
}

hipError_t launch_update(const Geo& g, const float* s, float* rho, const Workspace& ws, hipStream_t st) {
  const int64_t npix = (int64_t)g.n_y * g.n_z;
  int64_t blocks = (npix + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_update, dim3((unsigned)blocks), dim3(256), 0, st, npix, s, rho, ws.acc);
  return hipGetLastError();
}

}  // namespace jpet
