// Per-event preparation and spatial binning (iteration-invariant, run once per event list).
//
//   k_prepare   direct reconstruction (Eq. 2), ellipse rows (App. B, Sec. 3), pixel count,
//               validity and the bin of each event
//   k_histogram events per bin
//   k_scan      exclusive prefix sums of bin sizes and of workgroup items per bin
//   k_scatter   records in bin order
//   k_items     workgroup items: (bin, first event, count) with at most ev_per_wg events
#include "jpet_device.h"

namespace jpet {

namespace {

__device__ inline int clamp_index(double v, int lo, int hi) {
  if (!(v >= (double)lo)) return lo;   // also catches NaN
  if (v > (double)hi) return hi;
  return (int)v;
}

__device__ uint32_t bin_of(const Geo& g, const Plan& p, const EventRec& e) {
  int b = 0;
  if (p.ntb > 1) b = clamp_index(floor((e.t - p.tmin) / p.dt), 0, p.ntb - 1);
  const double tc = bin_slope(p, b);
  const int ic = clamp_index(rint((e.y - g.y0) * g.ipix), 0, g.n_y - 1);
  const int ty = ic / p.TY;
  const int kmin = -max(shear_offset(g, tc, 0), shear_offset(g, tc, g.n_y - 1));
  const double kz = (e.z - tc * e.y - g.z0) * g.ipix;
  const int tz = clamp_index(floor((kz - (double)kmin) / (double)p.TZ), 0, p.ntz - 1);
  return (uint32_t)(((int64_t)b * p.nty + ty) * p.ntz + tz);
}

__global__ void __launch_bounds__(256) k_prepare(Geo g, Plan p, const float* __restrict__ events, int64_t n,
                                                 EventRec* __restrict__ ev, uint32_t* __restrict__ key,
                                                 unsigned long long* __restrict__ cnt) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long valid = 0, pairs = 0;
  if (j < n) {
    const float zu = events[3 * j], zd = events[3 * j + 1], dl = events[3 * j + 2];
    EventRec e;
    e.r0 = 0;
    e.r1 = -1;
    e.npix = 0;
    e.index = (int32_t)j;
    e.t = e.c = e.y = e.z = 0.0;
    e.su = 1.0;
    uint32_t k = kNoBin;
    const double hl = 0.5 * g.L;
    if (isfinite(zu) && isfinite(zd) && isfinite(dl) && fabs((double)zu) <= hl && fabs((double)zd) <= hl) {
      // Eq. 2, first forms
      const double t = ((double)zu - (double)zd) / (2.0 * g.R);
      const double c = sqrt(1.0 + t * t);
      const double y = -0.5 * (double)dl / c;
      const double z = 0.5 * ((double)zu + (double)zd + 2.0 * y * t);
      e.t = t;
      e.c = c;
      e.y = y;
      e.z = z;
      // this event's sigma_z: sigma_z (1 + zedge zeta), zeta the mean of (z / (L/2))^2 over the
      // two hits (Sec. 3 after Eq. 12); u scales by the inverse square
      {
        const double xu = (double)zu / hl, xd = (double)zd / hl;
        const double f = 1.0 + g.zedge * (0.5 * (xu * xu + xd * xd));
        e.su = 1.0 / (f * f);
      }
      // rows within the ellipse's half height 1.5 sigma_dl / c (App. B)
      const double hy = 1.5 / (sqrt(g.wm) * c);
      double a = ceil((y - hy - g.y0) * g.ipix);
      double b = floor((y + hy - g.y0) * g.ipix);
      if (a < 0.0) a = 0.0;
      if (b > (double)(g.n_y - 1)) b = (double)(g.n_y - 1);
      int first = 1 << 30, last = -1;
      long long cntp = 0;
      if (a <= b) {
        for (int i = (int)a; i <= (int)b; ++i) {
          int klo, khi;
          if (row_interval(g, e, i, &klo, &khi)) {
            if (first > i) first = i;
            last = i;
            cntp += khi - klo + 1;
          }
        }
      }
      if (cntp > 0) {
        e.r0 = first;
        e.r1 = last;
        e.npix = (int)cntp;
        valid = 1;
        pairs = (unsigned long long)cntp;
        if (p.tiled) k = bin_of(g, p, e);
      }
    }
    ev[j] = e;
    key[j] = k;
  }
  const unsigned long long v = wave_sum_u64(valid), pr = wave_sum_u64(pairs),
                           in = wave_sum_u64(j < n ? 1ull : 0ull);
  if ((threadIdx.x & (WAVE - 1)) == 0 && in) {
    atomicAdd(&cnt[C_VALID], v);
    atomicAdd(&cnt[C_DROPPED], in - v);
    atomicAdd(&cnt[C_PAIRS], pr);
  }
}

__global__ void k_fill_u32(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ void __launch_bounds__(256) k_histogram(const uint32_t* __restrict__ key, int64_t n,
                                                   uint32_t* __restrict__ bin_count) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n && key[j] != kNoBin) atomicAdd(&bin_count[key[j]], 1u);
}

// Single workgroup: exclusive scans of the bin sizes, of the workgroup items per bin and of the
// batch blocks per bin.
__global__ void __launch_bounds__(1024) k_scan(int nbins, int ev_per_wg, int ev_per_batch,
                                               const uint32_t* __restrict__ bin_count, uint32_t* __restrict__ bin_start,
                                               uint32_t* __restrict__ item_start, uint32_t* __restrict__ batch_start,
                                               unsigned long long* __restrict__ cnt) {
  __shared__ uint32_t s_ev[1024], s_it[1024], s_ba[1024];
  const int T = blockDim.x;
  const int chunk = (nbins + T - 1) / T;
  const int lo = min(nbins, (int)threadIdx.x * chunk), hi = min(nbins, lo + chunk);
  uint32_t se = 0, si = 0, sb = 0;
  for (int b = lo; b < hi; ++b) {
    const uint32_t c = bin_count[b];
    se += c;
    si += (c + ev_per_wg - 1) / ev_per_wg;
    sb += (c + ev_per_batch - 1) / ev_per_batch;
  }
  s_ev[threadIdx.x] = se;
  s_it[threadIdx.x] = si;
  s_ba[threadIdx.x] = sb;
  __syncthreads();
  for (int off = 1; off < T; off <<= 1) {
    uint32_t ae = 0, ai = 0, ab = 0;
    if ((int)threadIdx.x >= off) {
      ae = s_ev[threadIdx.x - off];
      ai = s_it[threadIdx.x - off];
      ab = s_ba[threadIdx.x - off];
    }
    __syncthreads();
    s_ev[threadIdx.x] += ae;
    s_it[threadIdx.x] += ai;
    s_ba[threadIdx.x] += ab;
    __syncthreads();
  }
  uint32_t re = threadIdx.x ? s_ev[threadIdx.x - 1] : 0u, ri = threadIdx.x ? s_it[threadIdx.x - 1] : 0u,
           rb = threadIdx.x ? s_ba[threadIdx.x - 1] : 0u;
  for (int b = lo; b < hi; ++b) {
    const uint32_t c = bin_count[b];
    bin_start[b] = re;
    item_start[b] = ri;
    batch_start[b] = rb;
    re += c;
    ri += (c + ev_per_wg - 1) / ev_per_wg;
    rb += (c + ev_per_batch - 1) / ev_per_batch;
  }
  if (threadIdx.x == T - 1) {
    bin_start[nbins] = s_ev[T - 1];
    item_start[nbins] = s_it[T - 1];
    batch_start[nbins] = s_ba[T - 1];
    cnt[C_ITEMS] = s_it[T - 1];
  }
}

__global__ void __launch_bounds__(256) k_scatter(const EventRec* __restrict__ ev, const uint32_t* __restrict__ key,
                                                 int64_t n, const uint32_t* __restrict__ bin_start,
                                                 uint32_t* __restrict__ bin_fill, EventRec* __restrict__ evs) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const uint32_t k = key[j];
  if (k == kNoBin) return;
  const uint32_t pos = bin_start[k] + atomicAdd(&bin_fill[k], 1u);
  evs[pos] = ev[j];
}

__global__ void __launch_bounds__(256) k_items(int nbins, int ev_per_wg, int ev_per_batch,
                                               const uint32_t* __restrict__ bin_count,
                                               const uint32_t* __restrict__ bin_start,
                                               const uint32_t* __restrict__ item_start,
                                               const uint32_t* __restrict__ batch_start, BinItem* __restrict__ items) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  const uint32_t c = bin_count[b];
  uint32_t q = item_start[b];
  for (uint32_t s = 0; s < c; s += ev_per_wg, ++q) {
    BinItem it;
    it.bin = b;
    it.start = (int32_t)(bin_start[b] + s);
    it.count = (int32_t)min((uint32_t)ev_per_wg, c - s);
    it.batch = (int32_t)(batch_start[b] + s / ev_per_batch);
    items[q] = it;
  }
}

// The per-event constants of the binned MLEM pass (EvRow) for a bin whose region starts at pixel
// row rbase and (sheared) column kbase, in double precision.  With r the region row, the row's
// y is Y = Yb + pix r and dy = Y - y~ = pix r - yr, both linear in r; each row constant of the
// kernel (Eq. 7-12; see EvRow) is then a polynomial of degree <= 2 in r, expanded here.
__device__ EvRow event_row_constants(const Geo& g, const EventRec& e, int rbase, int kbase) {
  const double pix = g.pixel, t = e.t, c = e.c, c2 = c * c, f = g.fa;
  const double u = g.u * e.su, w = g.w;  // u: this event's sigma_z^-2
  const double Yb = g.y0 + (double)rbase * pix;
  const double yr = e.y - Yb;                          // dy = pix r - yr
  const double zr = e.z - (g.z0 + (double)kbase * pix);
  const double rs = 0.84932180028801904272;            // sqrt(log2(e) / 2)
  const double S = kHalfLog2e;
  // kappa without its b1 term: A1 (R^2 + Y^2) + A2 Y^2 + A3 Y dy + GK (fa Y + 2 dy)
  const double A1 = 2.0 * u * c2 * c2, A2 = w * f * f * c2 * t * t, A3 = 4.0 * w * c2 * (1.0 + 2.0 * t * t);
  const double GK = -4.0 * g.gamma * g.R * c2 * c * t;
  const double KB = -4.0 * u * t * c2;                 // kappa's slope in b1 per unit Y
  // sqrt(S) gamma^ without its b1 term: rs (G1 Y dy + GG dy); its slope in b1 per unit Y: rs GB
  const double G1 = 2.0 * f * w * c2 * t, GG = -4.0 * g.gamma * g.R * c2 * c, GB = -2.0 * u * c2;
  const double Q3 = S * 4.0 * w * c2;                  // S q = S 2u b1^2 + Q3 dy^2
  EvRow k;
  k.B0 = (float)(t * yr - zr);
  k.BT = (float)(-t * pix);
  // Y^2 = Yb^2 + 2 Yb pix r + pix^2 r^2,  Y dy = -Yb yr + (Yb - yr) pix r + pix^2 r^2
  k.K0 = (float)(A1 * g.R * g.R + (A1 + A2) * Yb * Yb - A3 * Yb * yr + GK * (f * Yb - 2.0 * yr));
  k.K1 = (float)(((A1 + A2) * 2.0 * Yb + A3 * (Yb - yr) + GK * (f + 2.0)) * pix);
  k.K2 = (float)((A1 + A2 + A3) * pix * pix);
  k.KB0 = (float)(KB * Yb);
  k.KB1 = (float)(KB * pix);
  k.S0 = (float)(rs * (-G1 * Yb * yr - GG * yr));
  k.S1 = (float)(rs * (G1 * (Yb - yr) + GG) * pix);
  k.S2 = (float)(rs * G1 * pix * pix);
  k.GB0 = (float)(rs * GB * Yb);
  k.GB1 = (float)(rs * GB * pix);
  k.Q0 = (float)(Q3 * yr * yr);
  k.Q1 = (float)(-2.0 * Q3 * yr * pix);
  k.Q2 = (float)(Q3 * pix * pix);
  const double s2u = S * 2.0 * u;
  k.qa = (float)(s2u * pix * pix);
  k.QB = (float)(2.0 * s2u * pix);
  k.s2u = (float)s2u;
  k.index = e.index;
  k.pad = 0;
  return k;
}

// Batch blocks of the binned pass: one workgroup per item builds, for each batch of ev_per_batch
// events, the per-event constants and the thread words.  A thread owns one row segment of at most
// the register cache's length: every ellipse row has a first segment, and when the plan splits
// rows (p.segs = 2) each row longer than the cache also has a second one, its remaining pixels.
// The segments of one level of one event form a "group" of consecutive rows.  Rows are given to
// threads so that a wavefront holds rows of nearly equal length: each group's rows are cut into
// rings of 32 rows around its central row (ring 0: the 32 central rows; ring k: 16 rows above and
// 16 below ring k-1) and a remainder at its two tips.  Half-wavefront slots take the rings ordered
// by ring index, then by group, so a wavefront pairs two rings at the same distance from their
// ellipses' centres; the tips of all groups fill the remaining threads.  Within a half-wavefront
// the rows are consecutive, so its LDS accesses fall into distinct banks (the two halves of a
// wavefront can still meet in a bank).
constexpr int kBuildBatch = 32;
constexpr int kBuildGroups = 2 * kBuildBatch;
constexpr int kBuildSlots = 64;

__global__ void __launch_bounds__(1024) k_build_batches(Geo g, Plan p, const EventRec* __restrict__ evs,
                                                        const BinItem* __restrict__ items,
                                                        unsigned char* __restrict__ blocks,
                                                        unsigned long long* __restrict__ cnt) {
  __shared__ EventRec ev_s[kBuildBatch];
  // groups: g < nb is event g's first segments over all its rows; nb + g its second segments,
  // over the rows from its first to its last row longer than the register cache (none: 0 rows)
  __shared__ int grp_r0[kBuildGroups], grp_n[kBuildGroups];
  __shared__ int K_s[kBuildGroups], top_s[kBuildGroups];
  __shared__ unsigned char slot_g[kBuildSlots], slot_k[kBuildSlots];
  __shared__ int tip_cum[kBuildGroups + 1];
  __shared__ int nslots_s;
  __shared__ unsigned outside_s;
  if ((unsigned long long)blockIdx.x >= cnt[C_ITEMS]) return;
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
  if (tid == 0) outside_s = 0u;
  for (int e0 = 0, bi = 0; e0 < it.count; e0 += p.ev_per_batch, ++bi) {
    const int nb = min(p.ev_per_batch, it.count - e0);
    const int ng = p.segs > 1 ? 2 * nb : nb;
    unsigned char* blk = blocks + (size_t)(it.batch + bi) * (size_t)p.batch_bytes;
    uint32_t* words = reinterpret_cast<uint32_t*>(blk + p.cbytes);
    __syncthreads();
    if (tid < nb) {
      const EventRec e = evs[it.start + e0 + tid];
      ev_s[tid] = e;
      grp_r0[tid] = 0;
      grp_n[tid] = e.r1 - e.r0 + 1;
      if (p.segs > 1) {  // the rows longer than the register cache
        int first = -1, last = -2;
        for (int i = e.r0; i <= e.r1; ++i) {
          int klo, khi;
          if (row_interval(g, e, i, &klo, &khi) && khi - klo + 1 > p.maxlen) {
            if (first < 0) first = i - e.r0;
            last = i - e.r0;
          }
        }
        grp_r0[nb + tid] = first < 0 ? 0 : first;
        grp_n[nb + tid] = last - first + 1 > 0 ? last - first + 1 : 0;
      }
      if (p.loglik) {
        const float t = (float)e.t, c2 = (float)(e.c * e.c), u = (float)(g.u * e.su), w = (float)g.w,
                    fa = (float)g.fa;
        EvConst k;
        k.yr = (float)(e.y - (g.y0 + (double)rbase * g.pixel));
        k.zr = (float)(e.z - (g.z0 + (double)kbase * g.pixel));
        k.index = e.index;
        k.S2u = (float)(kHalfLog2e * 2.0 * (g.u * e.su));
        k.t = t;
        k.A1 = 2.0f * u * c2 * c2;
        k.A2 = w * fa * fa * c2 * t * t;
        k.A3 = 4.0f * w * c2 * (1.0f + 2.0f * t * t);
        k.KB = -4.0f * u * t * c2;
        k.G1 = 2.0f * fa * w * c2 * t;
        k.GB = -2.0f * u * c2;
        k.Q3s = (float)kHalfLog2e * 4.0f * w * c2;
        {
          const double c3 = e.c * e.c * e.c;
          k.GK = (float)(-4.0 * g.gamma * g.R * c3 * e.t);
          k.GG = (float)(-4.0 * g.gamma * g.R * c3);
        }
        k.pad[0] = k.pad[1] = 0;
        reinterpret_cast<EvConst*>(blk)[tid] = k;
      } else {
        reinterpret_cast<EvRow*>(blk)[tid] = event_row_constants(g, e, rbase, kbase);
      }
    }
    __syncthreads();
    if (tid < WAVE) {  // ring slots (ring-major, then group) and the tip prefix
      const int nrows = tid < ng ? grp_n[tid] : 0;
      const int mrow = nrows >> 1;
      const int K = min(mrow, nrows - mrow) >> 4;
      const int T = nrows - 32 * K;
      if (tid < ng) {
        K_s[tid] = K;
        top_s[tid] = mrow - 16 * K;
      }
      const int Kmax = wave_max_i(K);
      int base_slot = 0;
      for (int k = 0; k < Kmax; ++k) {
        const unsigned long long msk = __ballot(K > k);
        const int before = __popcll(msk & ((1ull << lane) - 1ull));
        if (K > k) {
          slot_g[base_slot + before] = (unsigned char)tid;
          slot_k[base_slot + before] = (unsigned char)k;
        }
        base_slot += __popcll(msk);
      }
      int incl = T;
#pragma unroll
      for (int off = 1; off < WAVE; off <<= 1) {
        const int o = __shfl_up(incl, off, WAVE);
        if (lane >= off) incl += o;
      }
      if (tid < ng) tip_cum[tid] = incl - T;
      if (tid == ng - 1) tip_cum[ng] = incl;
      if (tid == 0) nslots_s = base_slot;
    }
    __syncthreads();
    const int nslots = nslots_s;
    int gi = -1, ri = 0;  // group and row within the group
    if (tid < 32 * nslots) {
      const int sl = tid >> 5, l = tid & 31;
      gi = slot_g[sl];
      const int k = slot_k[sl];
      const int mrow = grp_n[gi] >> 1;
      ri = k == 0 ? mrow - 16 + l : (l < 16 ? mrow - 16 * (k + 1) + l : mrow + 16 * k + (l - 16));
    } else if (tid - 32 * nslots < tip_cum[ng]) {
      const int q = tid - 32 * nslots;
      int lo = 0, hi = ng - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tip_cum[mid] <= q) lo = mid; else hi = mid - 1;
      }
      gi = lo;
      const int qq = q - tip_cum[gi];
      const int top = top_s[gi];
      ri = qq < top ? qq : (grp_n[gi] >> 1) + 16 * K_s[gi] + (qq - top);
    }
    uint32_t word = 0u;
    bool guard = false;  // this segment may reach kappa <= 0: the pass tests every pixel
    if (gi >= 0) {
      const int e = gi < nb ? gi : gi - nb;
      const EventRec ev = ev_s[e];
      const int i = ev.r0 + grp_r0[gi] + ri;
      int klo, khi;
      if (row_interval(g, ev, i, &klo, &khi)) {
        int n = khi - klo + 1;
        if (gi < nb) {  // first segment
          if (n > p.maxlen && p.segs > 1) n = p.maxlen;
        } else {        // second segment: the pixels past the first
          klo += p.maxlen;
          n -= p.maxlen;
        }
        if (n > 0) {
          const int rl = i - rbase;
          const int kl = klo - shear_offset(g, tc, i) - kbase;
          if (rl < 0 || rl >= p.RY || kl < 0 || kl + n > p.W || n > p.maxlen) {
            atomicAdd(&outside_s, 1u);
          } else {
            word = ((uint32_t)kl << kWordCol) | ((uint32_t)rl << kWordRow) | ((uint32_t)n << kWordLen) |
                   ((uint32_t)e << kWordEv);
            // kappa is affine along the row: its smallest value is at one of the segment's two
            // ends; segments whose ends both keep a margin of 1e-3 of the first value can skip
            // the test
            double kf, ks;
            (void)row_constants(g, ev, i, klo, &kf, &ks);
            const double kend = kf + (double)(n - 1) * ks;
            guard = !(kf > 1e-3 * fabs(kf) && kend > 1e-3 * fabs(kf));
          }
        }
      }
    }
    if (tid < 64 * p.waves) {
      words[tid] = word;
      const int len = (int)((word >> kWordLen) & 127u);
      const int wl = wave_max_i(len);
      const int wmin = -wave_max_i(len > 0 ? -len : -wl);  // shortest non-empty row (0: none)
      const bool wguard = __any(guard);
      // does each half-wavefront hold rows of one event only (the pass then reduces the
      // denominators per half, without the per-event loop)?
      const int ev = (int)((word >> kWordEv) & 31u);
      const unsigned long long act = __ballot(len > 0);
      const unsigned long long half = lane < 32 ? 0xffffffffull : 0xffffffff00000000ull;
      const unsigned long long mine = act & half;
      const int lead = mine ? __ffsll((long long)mine) - 1 : (lane & 32);
      const int ev_lead = __shfl(ev, lead, WAVE);
      const bool split = __any(len > 0 && ev != ev_lead);
      // (a half with no rows takes the other half's event)
      int ev_lo = __shfl(ev_lead, 0, WAVE), ev_hi = __shfl(ev_lead, 32, WAVE);
      if (!(act & 0xffffffffull)) ev_lo = ev_hi;
      if (!(act >> 32)) ev_hi = ev_lo;
      if (lane == 0) {
        words[64 * p.waves + (tid >> 6)] = (uint32_t)wl | (wguard ? 1u << kGuardBit : 0u);
        words[65 * p.waves + (tid >> 6)] =
            (uint32_t)wmin |
            (split ? 0u : (1u << kHalfBit) | ((uint32_t)ev_lo << kHalfLo) | ((uint32_t)ev_hi << kHalfHi));
      }
    }
  }
  __syncthreads();
  if (tid == 0 && outside_s) atomicAdd(&cnt[C_OUTSIDE], (unsigned long long)outside_s);
}

int blocks_for(int64_t n, int block) { return (int)((n + block - 1) / block); }

}  // namespace

hipError_t launch_prepare(const Geo& g, const Plan& p, const float* events, int64_t n, const Workspace& ws,
                          hipStream_t st) {
  if (n > 0) {
    hipLaunchKernelGGL(k_prepare, dim3(blocks_for(n, 256)), dim3(256), 0, st, g, p, events, n, ws.ev, ws.key, ws.cnt);
  }
  if (!p.tiled) return hipGetLastError();
  const int64_t nb = p.nbins;
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(nb, 256)), dim3(256), 0, st, ws.bin_count, nb);
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(nb, 256)), dim3(256), 0, st, ws.bin_fill, nb);
  if (n > 0) hipLaunchKernelGGL(k_histogram, dim3(blocks_for(n, 256)), dim3(256), 0, st, ws.key, n, ws.bin_count);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, p.nbins, p.ev_per_wg, p.ev_per_batch, ws.bin_count,
                     ws.bin_start, ws.item_start, ws.batch_start, ws.cnt);
  if (n > 0) {
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(n, 256)), dim3(256), 0, st, ws.ev, ws.key, n, ws.bin_start,
                       ws.bin_fill, ws.evs);
  }
  hipLaunchKernelGGL(k_items, dim3(blocks_for(nb, 256)), dim3(256), 0, st, p.nbins, p.ev_per_wg, p.ev_per_batch,
                     ws.bin_count, ws.bin_start, ws.item_start, ws.batch_start, ws.items);
  if (n > 0) {
    hipLaunchKernelGGL(k_build_batches, dim3((unsigned)p.max_items), dim3(64 * p.waves), 0, st, g, p, ws.evs, ws.items,
                       ws.batches, ws.cnt);
  }
  return hipGetLastError();
}

}  // namespace jpet
