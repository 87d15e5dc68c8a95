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
// The constant factor sqrt(det C^-1) / (2 pi) of Eq. 7 cancels in m / D and is not applied.
#include <type_traits>

#include "jpet_device.h"

namespace jpet {

namespace {

constexpr int kMaxBatch = 32;  // events per batch (the plan keeps ev_per_batch <= 32)
constexpr int kChunk = 4;      // pixels evaluated per branch-free step

// Static LDS of the pass; the per-event constants (double buffer: the next batch is copied in
// while this one runs) and the per-row column shifts sit in the dynamic LDS after the region.
struct PassShared {
  double D[3][kMaxBatch];    // batch b's denominators in D[b % 3]: filled, read, cleared in turn
  unsigned zero, bad;
};

// Single-precision kernel constants along one pixel row (Eq. 7-12); j is the pixel's
// offset in the row:
//   kappa_j = kap0 + j dkap,  sqrt(S) gamma_j = gs0 + j dgs,  S q_j = (qa j + qb) j + qc
// (qa = S 2u pixel^2 depends on the event through its sigma_z)
// and P / (sqrt(det C^-1) / 2 pi) = kappa^-1/2 exp2(S gamma^2 / kappa - S q), S = log2(e) / 2.
// The off-diagonal gamma of C^-1 enters only kappa and gamma^ through per-row constants: with
// b1 = b2, the gamma terms of b C^-1 b cancel (so the ellipse does not depend on gamma) while
// kappa gains -4 gamma R c^3 t (fa y + 2 dy) and gamma^ gains -4 gamma R c^3 dy.
struct RowF {
  float kap0, dkap, gs0, dgs, qa, qb, qc;
};

// A register-cache entry that pass 2 does not read: any value, set by no instruction (keeping the
// previous batch's value would keep the whole cache live through pass 1).
__device__ __forceinline__ float unread() { return __builtin_nondeterministic_value(0.0f); }

// Pass 1 along one row.  Chunks below the wavefront's shortest row (wmin, uniform) need no row-end
// mask; idle lanes carry row constants that make every kernel value 0.  Chunks from the
// wavefront's longest row (wl) on are skipped, and their register-cache entries left unset.
template <int MAXLEN, bool GUARD>
__device__ __forceinline__ float pass1(const RowF& rk, float qa, const float* __restrict__ rho_s, int base, int pitch,
                                       int len, int wmin, int wl, float (&m)[MAXLEN], int* nbad) {
  float D = 0.0f;
  const float* const rr = rho_s + base;  // the row's first pixel
#pragma unroll
  for (int j0 = 0; j0 < MAXLEN; j0 += kChunk) {
    if (j0 < wl) {  // wavefront-uniform
      float r[kChunk];
#pragma unroll
      for (int jj = 0; jj < kChunk; ++jj) r[jj] = rr[(j0 + jj) * pitch];
      if (!GUARD && j0 + kChunk <= wmin) {  // wavefront-uniform: every active lane's row is longer
#pragma unroll
        for (int jj = 0; jj < kChunk; ++jj) {
          const int j = j0 + jj;
          const float jf = (float)j;
          const float kap = fmaf(jf, rk.dkap, rk.kap0);
          const float gs = fmaf(jf, rk.dgs, rk.gs0);
          const float rq = __builtin_amdgcn_rsqf(kap);
          const float sq = fmaf(fmaf(qa, jf, rk.qb), jf, rk.qc);
          const float tg = gs * rq;
          const float pv = rq * __builtin_amdgcn_exp2f(fmaf(tg, tg, -sq));
          const float v = pv * r[jj];
          m[j] = v;
          D += v;
        }
      } else {
#pragma unroll
        for (int jj = 0; jj < kChunk; ++jj) {
          const int j = j0 + jj;
          const float jf = (float)j;
          float kap = fmaf(jf, rk.dkap, rk.kap0);
          bool keep = j < len;
          if (GUARD && !(kap > 0.0f)) {
            if (keep) ++*nbad;
            keep = false;
            kap = 1.0f;
          }
          const float gs = fmaf(jf, rk.dgs, rk.gs0);
          const float rq = __builtin_amdgcn_rsqf(kap);
          const float sq = fmaf(fmaf(qa, jf, rk.qb), jf, rk.qc);
          const float tg = gs * rq;
          const float pv = rq * __builtin_amdgcn_exp2f(fmaf(tg, tg, -sq));
          const float v = keep ? pv * r[jj] : 0.0f;
          m[j] = v;
          D += v;
        }
      }
    } else {
#pragma unroll
      for (int jj = 0; jj < kChunk; ++jj) m[j0 + jj] = unread();
    }
  }
  return D;
}

// Pass 2 along one row: m sc rounded into the fixed-point accumulators.  In chunks below wmin
// every lane adds with no per-pixel test; past it the row end masks.  Idle lanes and lanes whose
// event has D = 0 do not enter (one exec mask for the whole row: an LDS atomic that adds 0 still
// takes its share of the LDS atomic rate, measured 1% of the pass at 400x400).
template <int MAXLEN, bool PRESCALE, typename AccT>
__device__ __forceinline__ void pass2(const float (&m)[MAXLEN], float sc, int base, int pitch, int len, int wmin,
                                      int wl, AccT* __restrict__ acc_s) {
  // the row's first accumulator, formed once (the per-pixel offsets are then immediates when the
  // pitch is a compile-time constant)
  AccT* const a = acc_s + base;
  // chunks below wmin need no row-end test; past it each row's end masks
#pragma unroll
  for (int j0 = 0; j0 < MAXLEN; j0 += kChunk) {
    if (j0 + kChunk <= wmin) {  // wavefront-uniform
#pragma unroll
      for (int jj = 0; jj < kChunk; ++jj) {
        const int j = j0 + jj;
        const float x = PRESCALE ? m[j] * 18446744073709551616.0f : m[j];
        atomicAdd(&a[j * pitch], (AccT)(unsigned)fmaf(x, sc, 0.5f));
      }
    } else if (j0 < wl) {  // wavefront-uniform
#pragma unroll
      for (int jj = 0; jj < kChunk; ++jj) {
        const int j = j0 + jj;
        const float x = PRESCALE ? m[j] * 18446744073709551616.0f : m[j];
        if (j < len) atomicAdd(&a[j * pitch], (AccT)(unsigned)fmaf(x, sc, 0.5f));
      }
    }
  }
}

// Log-likelihood mode.  Per pixel, besides P' (the kernel without its constant factor), the
// derivatives of log P with respect to u = sigma_z^-2 and w = sigma_dl^-2, written with
// kappa = u Kz + w Kl + gamma Kg, gamma^ = u Gz + w Gl + gamma Gg, q = u Bz + w Bl, Bz = 2 b1^2,
// g = gamma^ / kappa and h = 1/kappa + g^2:
//   dlogP/du = cu - b1^2 + g Gz - Kz h / 2,    dlogP/dw = cw - Bl/2 + g Gl - Kl h / 2,
// cu, cw being the prefactor's share (1/u and 1/(2w) for gamma = 0).
// Along a row Kl, Gl, Bl are constant, and so are c = w Kl + gamma Kg and e = w Gl + gamma Gg.
// The pass needs only each row's sums of v dlogP/du and v dlogP/dw (v = rho P'), and these follow
// from four sums over the row's pixels.  With t = sqrt(S) gamma^ kappa^-1/2, the exponent of P' is
// x = t^2 - S q; let
//   S0 = sum v (the row's share of D),  X = sum v x,  G = sum v t kappa^-1/2 = sqrt(S) sum v g,
//   H = sum v h.
// Substituting b1^2 = (S q - S w Bl) / (2 S u), g Gz = (gamma^2/kappa - e g) / u with
// gamma^2/kappa = t^2 / S, Kz = (kappa - c) / u and kappa h = 1 + t^2 / S gives
//   sum v dlogP/du = (cu + w Bl / (2u) - 1/(2u)) S0 + X / (2 S u) - e G / (sqrt(S) u) + c H / (2u),
//   sum v dlogP/dw = (cw - Bl/2) S0 + Gl G / sqrt(S) - Kl H / 2.
// Per pixel that is 7 VALU operations besides P', against 15 for du and dw themselves.
struct RowD {
  float a0, aG, aH;  // the row's coefficients of S0, G and H in sum v dlogP/du
  float b0, bG, bH;  // and in sum v dlogP/dw
};

struct GradShared {
  float Du[3][kMaxBatch];  // per-event sums of rho P' dlogP/du, buffered like D
  float Dw[3][kMaxBatch];
  double sum[3][kMaxBatch];  // per batch slot: sums of log D', Du / D', Dw / D' over the item's events
};

// Pass 1 of the log-likelihood mode: P' into the register cache, and the row's sums S0 (= D), X, G
// and H (mom[0..2] = X, G, H).
template <int MAXLEN, bool GUARD>
__device__ __forceinline__ void pass1g(const RowF& rk, float qa, float iS, const float* __restrict__ rho_s, int base,
                                       int pitch, int len, int wmin, int wl, float (&m)[MAXLEN], int* nbad, float& D,
                                       float (&mom)[3]) {
  D = 0.0f;
  float X = 0.0f, G = 0.0f, H = 0.0f;
#pragma unroll
  for (int j0 = 0; j0 < MAXLEN; j0 += kChunk) {
    if (j0 < wl) {  // wavefront-uniform
      float r[kChunk];
#pragma unroll
      for (int jj = 0; jj < kChunk; ++jj) r[jj] = rho_s[base + (j0 + jj) * pitch];
      const bool full = !GUARD && j0 + kChunk <= wmin;  // wavefront-uniform
#pragma unroll
      for (int jj = 0; jj < kChunk; ++jj) {
        const int j = j0 + jj;
        const float jf = (float)j;
        float kap = fmaf(jf, rk.dkap, rk.kap0);
        bool keep = full || j < len;
        if (GUARD && !(kap > 0.0f)) {
          if (keep) ++*nbad;
          keep = false;
          kap = 1.0f;
        }
        const float gs = fmaf(jf, rk.dgs, rk.gs0);
        const float rq = __builtin_amdgcn_rsqf(kap);
        const float sq = fmaf(fmaf(qa, jf, rk.qb), jf, rk.qc);
        const float tg = gs * rq;
        const float x = fmaf(tg, tg, -sq);
        const float pv = rq * __builtin_amdgcn_exp2f(x);
        // masked reads past the row's end may land in the region's double accumulators, whose
        // low words can be any bit pattern (NaN included): select, do not multiply by 0
        const float pk = keep ? pv : 0.0f;
        const float v = keep ? pv * r[jj] : 0.0f;
        m[j] = pk;
        D += v;
        X = fmaf(v, x, X);
        const float gq = tg * rq;  // sqrt(S) g
        G = fmaf(v, gq, G);
        H = fmaf(v, fmaf(gq * gq, iS, rq * rq), H);  // h = 1/kappa + g^2
      }
    } else {
#pragma unroll
      for (int jj = 0; jj < kChunk; ++jj) m[j0 + jj] = unread();
    }
  }
  mom[0] = X;
  mom[1] = G;
  mom[2] = H;
}

// B += P' / D' (= P / D) into the region's double accumulators.
template <int MAXLEN>
__device__ __forceinline__ void pass2g(const float (&m)[MAXLEN], float invD, int base, int pitch, int len, int wmin,
                                       int wl, double* __restrict__ B_s) {
  double* const b = B_s + base;
#pragma unroll
  for (int j0 = 0; j0 < MAXLEN; j0 += kChunk) {
    if (j0 + kChunk <= wmin) {  // wavefront-uniform
#pragma unroll
      for (int jj = 0; jj < kChunk; ++jj) unsafeAtomicAdd(&b[(j0 + jj) * pitch], (double)(m[j0 + jj] * invD));
    } else if (j0 < wl) {  // wavefront-uniform
#pragma unroll
      for (int jj = 0; jj < kChunk; ++jj) {
        if (j0 + jj < len) unsafeAtomicAdd(&b[(j0 + jj) * pitch], (double)(m[j0 + jj] * invD));
      }
    }
  }
}

// Copies a batch's per-event constants into LDS with direct global-to-LDS loads issued by the
// first wavefront (16 bytes per lane, 1 KB per instruction); completion is awaited before the
// next workgroup barrier.
__device__ __forceinline__ void copy_consts(const unsigned char* __restrict__ src, unsigned char* dst, int bytes,
                                            int tid) {
  if (tid < WAVE) {
    for (int off = 0; off < bytes; off += WAVE * 16) {
      if (off + tid * 16 < bytes)
        __builtin_amdgcn_global_load_lds(reinterpret_cast<const uint4*>(src + off + tid * 16), dst + off, 16, 0, 0);
    }
  }
}

// The region is stored column-major with a row pitch that is a multiple of the LDS bank count.
// Each thread owns the pixel row its thread word names (built at prepare time so that a
// wavefront holds rows of nearly equal length, consecutive within each half-wavefront), so the
// pixel at column offset j of the rows of one half-wavefront falls into 32 different banks
// whatever the slant of the ellipse.  The two halves of a ring wavefront hold rings of two events
// of the same bin, whose rows overlap, and may meet in a bank; tip wavefronts mix rows of several
// events.  Measured at 400x400: conflict cycles are 20% of the LDS-active cycles, and moving every
// lane's word to its own bank (a timing-only copy) saved 1% of the pass.
// One workgroup item.  GRAD = false: the MLEM event pass (acc: 2^-32 fixed-point image; the LDS
// accumulators are 64-bit in 2^-32 units, or with ACC32 32-bit in 2^-acc_shift units, acc_shift = 23
// for items of up to 511 events).
// With D_out (MLEM mode) each event's denominator times the kernel's constant factor is also
// written at the event's input position (evs: the bin-sorted records).
// GRAD = true: the log-likelihood pass (acc: double image B = sum P / D; per-event log D' and the
// sigma-derivative sums into red[0..2]; D' times the kernel's constant factor into D_out).
// VALUE (with GRAD): the log-likelihood value only: per-event log D' sums, no B, no
// sigma-derivative terms (pass 1 as in the MLEM pass, no pass 2).
template <int MAXLEN, int WAVES, bool GRAD, bool ACC32, int PITCH, bool VALUE = false>
__device__ __forceinline__ void event_pass_item(const Geo& g, const Plan& p, const unsigned char* __restrict__ blocks,
                                                const BinItem it, const float* __restrict__ rho,
                                                unsigned long long* __restrict__ acc,
                                                unsigned long long* __restrict__ cnt, unsigned char* smem,
                                                PassShared& ps, GradShared* gsh, float* __restrict__ D_out,
                                                double* __restrict__ red, const EventRec* __restrict__ evs) {
  // rows of a column in LDS; a compile-time pitch turns the per-pixel LDS addresses into
  // immediate offsets
  const int pitch = PITCH ? PITCH : p.pitch;
  const int npx = pitch * p.W;
  // the image first, then the accumulators: reads past the end of a row (masked lanes) land in
  // the accumulator array, which is larger than MAXLEN columns of the image
  float* rho_s = reinterpret_cast<float*>(smem);
  static_assert(!(GRAD && ACC32), "the log-likelihood pass accumulates doubles");
  using AccT = typename std::conditional<ACC32, unsigned, unsigned long long>::type;
  AccT* acc_s = reinterpret_cast<AccT*>(smem + (size_t)npx * sizeof(float));
  // accumulator units per count: 2^32, or 2^acc_shift for 32-bit slots (the plan keeps an item's
  // events below 2^(32 - acc_shift), so no slot can overflow before the flush)
  const float kUnit = ACC32 ? __builtin_ldexpf(1.0f, p.acc_shift) : 4294967296.0f;
  const int flush_shift = ACC32 ? 32 - p.acc_shift : 0;

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
  const float pixf = (float)g.pixel;
  const float S2u = (float)(kHalfLog2e * 2.0 * g.u);
  const float qa = S2u * pixf * pixf;
  const float R2 = (float)(g.R * g.R);
  const float rs = 0.84932180028801904272f;  // sqrt(log2(e) / 2)
  const float faf = (float)g.fa;
  const int nbatch = (it.count + p.ev_per_batch - 1) / p.ev_per_batch;
  const int cbytes = p.cbytes;
  const unsigned char* blk0 = blocks + (size_t)it.batch * (size_t)p.batch_bytes;
  unsigned char* const ev_lds = smem + p.lds_ev;  // two buffers of cbytes
  int* const off_s = reinterpret_cast<int*>(smem + p.lds_off);

  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wl_off = cbytes + 4 * 64 * WAVES + 4 * wave;  // this wavefront's longest row
  const int wn_off = wl_off + 4 * WAVES;                   // and its shortest non-empty row
  // first batch: constants to LDS, this thread's word and its wavefront's row lengths (and whether
  // a row of the wavefront needs the per-pixel kappa test)
  copy_consts(blk0, ev_lds, cbytes, tid);
  uint32_t word = reinterpret_cast<const uint32_t*>(blk0 + cbytes)[tid];
  uint32_t wlw = *reinterpret_cast<const uint32_t*>(blk0 + wl_off);
  uint32_t wnw = *reinterpret_cast<const uint32_t*>(blk0 + wn_off);
  if (tid < kMaxBatch) {
    ps.D[0][tid] = 0.0;
    ps.D[1][tid] = 0.0;
    ps.D[2][tid] = 0.0;
    if constexpr (GRAD) {
      for (int b = 0; b < 3; ++b) {
        gsh->Du[b][tid] = 0.0f;
        gsh->Dw[b][tid] = 0.0f;
        gsh->sum[b][tid] = 0.0;
      }
    }
  }
  const float iu = (float)(1.0 / g.u), iw = (float)(1.0 / g.w);
  const float cuf = (float)g.cu, cwf = (float)g.cw;  // prefactor terms of d log P / du, dw
  const float irs = 1.1774100225154747f;     // 1 / sqrt(log2(e) / 2)
  const float iS = 1.3862943611198906f;      // 1 / (log2(e) / 2)
  const float iS2u = (float)(1.0 / (kHalfLog2e * 2.0 * g.u));  // 1 / (2 S u)
  const float Dnorm = (float)g.cnorm;
  if (tid == 0) {
    ps.zero = 0u;
    ps.bad = 0u;
  }
  // stage the region of the current image (column-major), clear the accumulators: wavefronts take
  // columns, lanes take rows
  for (int r = tid; r < p.RY; r += blockDim.x) off_s[r] = shear_offset(g, tc, rbase + r);
  __syncthreads();
  for (int cl = wave; cl < p.W; cl += WAVES) {
    const int kc = kbase + cl;
    for (int rl = lane; rl < pitch; rl += WAVE) {
      const int q = cl * pitch + rl;
      const int r = rbase + rl;
      float v = 0.0f;
      if (rl < p.RY && r >= 0 && r < g.n_y) {
        const int k = kc + off_s[rl];
        if (k >= 0 && k < g.n_z) v = rho[(int64_t)r * g.n_z + k];
      }
      rho_s[q] = v;
      acc_s[q] = 0;
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  // Software pipeline, one workgroup barrier per batch: step bi runs pass 2 of batch bi - 1 (its
  // denominators were completed before the previous barrier) and then pass 1 of batch bi, so
  // one wavefront's LDS atomics overlap other wavefronts' kernel evaluation.
  float m[MAXLEN];
  int plen = 0, pbase = 0, pe = 0, pwl = 0, pwn = 0;  // the row held in m (previous batch)
  const float Yb = (float)(g.y0 + (double)rbase * g.pixel);  // y of the region's first row
  for (int bi = 0; bi <= nbatch; ++bi) {
    // pass 2 of batch bi - 1: m / D into the region accumulators (2^-32 fixed point), or in the
    // log-likelihood mode P / D into B and the per-event terms
    if (bi > 0) {
      const double* Dp = ps.D[(bi - 1) % 3];
      const double Dd = plen > 0 ? Dp[pe] : 1.0;
      const int n2 = Dd > 0.0 ? plen : 0;
      if constexpr (GRAD) {
        if constexpr (!VALUE) {
          const float invD = n2 > 0 ? (float)(1.0 / Dd) : 0.0f;
          if (n2 > 0) pass2g<MAXLEN>(m, invD, pbase, pitch, n2, pwn, pwl, reinterpret_cast<double*>(acc_s));
        }
        const int nbp = min(p.ev_per_batch, it.count - (bi - 1) * p.ev_per_batch);
        if (wave == 0 && tid < nbp) {  // the batch slot's own sums (one thread each, in LDS, not registers)
          const double De = Dp[tid];
          if (De > 0.0) {
            gsh->sum[0][tid] += log(De);
            if constexpr (!VALUE) {
              gsh->sum[1][tid] += (double)gsh->Du[(bi - 1) % 3][tid] / De;
              gsh->sum[2][tid] += (double)gsh->Dw[(bi - 1) % 3][tid] / De;
            }
          } else {
            atomicAdd(&ps.zero, 1u);
          }
          if (D_out)
            D_out[evs[it.start + (bi - 1) * p.ev_per_batch + tid].index] =
                (float)(De > 0.0 ? De * (double)Dnorm : 0.0);
        }
      } else {
        // 2^32 / D overflows a float only for D < 1.3e-29; such wavefronts pre-scale m by 2^64
        if (__any(n2 > 0 && Dd < 1e-28)) {
          const float sc = n2 > 0 ? (float)((double)kUnit / (Dd * 18446744073709551616.0)) : 0.0f;
          if (n2 > 0) pass2<MAXLEN, true>(m, sc, pbase, pitch, n2, pwn, pwl, acc_s);
        } else {
          const float sc = n2 > 0 ? kUnit * __builtin_amdgcn_rcpf((float)Dd) : 0.0f;
          if (n2 > 0) pass2<MAXLEN, false>(m, sc, pbase, pitch, n2, pwn, pwl, acc_s);
        }
        const int nbp = min(p.ev_per_batch, it.count - (bi - 1) * p.ev_per_batch);
        if (wave == 0 && tid < nbp && !(Dp[tid] > 0.0)) atomicAdd(&ps.zero, 1u);
        // the denominators themselves (with P's constant factor), by input position
        if (D_out && wave == 0 && tid < nbp)
          D_out[evs[it.start + (bi - 1) * p.ev_per_batch + tid].index] = (float)(Dp[tid] * g.cnorm);
      }
    }
    if (bi < nbatch) {
      const int buf = bi & 1;
      const unsigned char* evb = ev_lds + buf * cbytes;  // this batch's constants
      const int wl = (int)(wlw & 0x7fffffffu);
      const bool guard = (wlw >> kGuardBit) != 0u;  // wavefront-uniform
      const int wn = (int)(wnw & 0xffu);
      // prefetch the next batch: constants into the other LDS buffer, this thread's next word
      uint32_t next = 0u, wlw_next = 0u, wnw_next = 0u;
      if (bi + 1 < nbatch) {
        const unsigned char* blk = blk0 + (size_t)(bi + 1) * (size_t)p.batch_bytes;
        copy_consts(blk, ev_lds + (buf ^ 1) * cbytes, cbytes, tid);
        next = reinterpret_cast<const uint32_t*>(blk + cbytes)[tid];
        wlw_next = *reinterpret_cast<const uint32_t*>(blk + wl_off);
        wnw_next = *reinterpret_cast<const uint32_t*>(blk + wn_off);
      }

      // this thread's row
      const int len = (int)((word >> kWordLen) & 127u);
      const int e = (int)((word >> kWordEv) & 31u);
      int base = 0;
      RowF rk = {1.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 1e30f};  // idle lane: every kernel value is 0
      if constexpr (GRAD) {
        if (len > 0) {
          const int kl = (int)((word >> kWordCol) & 255u);
          const int rl = (int)((word >> kWordRow) & 511u);
          const float rlf = (float)rl;
          const EvConst& c = reinterpret_cast<const EvConst*>(evb)[e];
          // region-relative coordinates: the row's y, y - y~, and z of its first pixel - z~ - t (y - y~)
          const float Y = fmaf(rlf, pixf, Yb);
          const float dy = fmaf(rlf, pixf, -c.yr);
          const float b10 = fmaf((float)(kl + off_s[rl]), pixf, -fmaf(c.t, dy, c.zr));
          const float kr =
              fmaf(c.GK, fmaf(faf, Y, 2.0f * dy), fmaf(c.A1, R2 + Y * Y, Y * fmaf(c.A2, Y, c.A3 * dy)));
          const float kb = c.KB * Y;
          const float gb = c.GB * Y;
          rk.kap0 = fmaf(kb, b10, kr);
          rk.dkap = kb * pixf;
          rk.gs0 = rs * fmaf(gb, b10, fmaf(c.GG, dy, c.G1 * Y * dy));
          rk.dgs = rs * gb * pixf;
          // the log-likelihood mode has one sigma_z for all events
          rk.qa = S2u * pixf * pixf;
          rk.qb = 2.0f * S2u * b10 * pixf;
          rk.qc = fmaf(S2u * b10, b10, c.Q3s * dy * dy);
          base = kl * pitch + rl;
        }
      } else {
        // the row constants from the event's polynomials in the region row (see EvRow), in every
        // lane (an idle lane's word is 0: event 0, the region's first row and column, finite
        // values); idle lanes then take kappa = 1 and S q = 1e30, so that every kernel value is 0
        const int kl = (int)((word >> kWordCol) & 255u);
        const int rl = (int)((word >> kWordRow) & 511u);
        const float rlf = (float)rl;
        const EvRow& c = reinterpret_cast<const EvRow*>(evb)[e];
        const float b10 = fmaf(pixf, (float)(kl + off_s[rl]), fmaf(c.BT, rlf, c.B0));
        const float kb = fmaf(c.KB1, rlf, c.KB0);
        const float gb = fmaf(c.GB1, rlf, c.GB0);
        const bool act = len > 0;
        rk.kap0 = act ? fmaf(kb, b10, fmaf(fmaf(c.K2, rlf, c.K1), rlf, c.K0)) : 1.0f;
        rk.dkap = act ? kb * pixf : 0.0f;
        rk.gs0 = fmaf(gb, b10, fmaf(fmaf(c.S2, rlf, c.S1), rlf, c.S0));
        rk.dgs = gb * pixf;
        rk.qa = c.qa;
        rk.qb = c.QB * b10;
        rk.qc = act ? fmaf(c.s2u * b10, b10, fmaf(fmaf(c.Q2, rlf, c.Q1), rlf, c.Q0)) : 1e30f;
        base = kl * pitch + rl;
      }

      // pass 1: m = P rho along the row (log-likelihood mode: m = P), D partial sums; the per-pixel
      // kappa test only in wavefronts whose rows may need it (decided at prepare time)
      int nbad = 0;  // pixels of this thread's row with kappa <= 0 (P := 0)
      float D, Du = 0.0f, Dw = 0.0f;
      if constexpr (GRAD && !VALUE) {
        float mom[3];
        if (guard) {
          pass1g<MAXLEN, true>(rk, qa, iS, rho_s, base, pitch, len, wn, wl, m, &nbad, D, mom);
        } else {
          pass1g<MAXLEN, false>(rk, qa, iS, rho_s, base, pitch, len, wn, wl, m, &nbad, D, mom);
        }
        if (len > 0) {
          // the row's sums of v dlogP/du and v dlogP/dw from S0 = D, X, G, H (see RowD), with the
          // row constants c = w Kl + gamma Kg, e = w Gl + gamma Gg and S w Bl
          const int rl = (int)((word >> kWordRow) & 511u);
          const float rlf = (float)rl;
          const EvConst& c = reinterpret_cast<const EvConst*>(evb)[e];
          const float Y = fmaf(rlf, pixf, Yb);
          const float dy = fmaf(rlf, pixf, -c.yr);
          const float wKl = Y * fmaf(c.A2, Y, c.A3 * dy);
          const float cr = fmaf(c.GK, fmaf(faf, Y, 2.0f * dy), wKl);
          const float wGl = c.G1 * Y * dy;
          const float er = fmaf(c.GG, dy, wGl);
          const float SwBl = c.Q3s * dy * dy;
          RowD rd;
          rd.a0 = fmaf(SwBl, iS2u, cuf - 0.5f * iu);
          rd.aG = -iu * irs * er;
          rd.aH = 0.5f * iu * cr;
          rd.b0 = fmaf(-0.5f * iS * iw, SwBl, cwf);
          rd.bG = irs * iw * wGl;
          rd.bH = -0.5f * iw * wKl;
          Du = fmaf(rd.a0, D, fmaf(iS2u, mom[0], fmaf(rd.aG, mom[1], rd.aH * mom[2])));
          Dw = fmaf(rd.b0, D, fmaf(rd.bG, mom[1], rd.bH * mom[2]));
        }
      } else {
        if (guard) {
          D = pass1<MAXLEN, true>(rk, rk.qa, rho_s, base, pitch, len, wn, wl, m, &nbad);
        } else {
          D = pass1<MAXLEN, false>(rk, rk.qa, rho_s, base, pitch, len, wn, wl, m, &nbad);
        }
      }
      if (nbad) atomicAdd(&ps.bad, (unsigned)nbad);

      // per-event denominators: a reduction over the wavefront's rows, then one double-precision
      // LDS add per event and wavefront.  In most wavefronts (the rings) each half holds rows of
      // one event (decided at prepare time): one reduction gives both halves' sums, which lanes
      // 31 and 63 hold.  Otherwise a segmented reduction takes one event at a time.  (Adding
      // every row's partial sum with its own LDS atomic instead puts all lanes of a wavefront on
      // two or three addresses; measured 5% slower at 400x400.)
      double* Dc = ps.D[bi % 3];
      if (wnw >> kHalfBit) {
        const int elo = (int)((wnw >> kHalfLo) & 31u), ehi = (int)((wnw >> kHalfHi) & 31u);
        const float h = half_sums_dpp(len > 0 ? D : 0.0f);
        const float lo = lane_value(h, 31), hi = lane_value(h, 63);
        if (lane == 0) {
          if (elo == ehi) {
            unsafeAtomicAdd(&Dc[elo], (double)lo + (double)hi);
          } else {
            unsafeAtomicAdd(&Dc[elo], (double)lo);
            unsafeAtomicAdd(&Dc[ehi], (double)hi);
          }
        }
        if constexpr (GRAD && !VALUE) {
          const float hu = half_sums_dpp(len > 0 ? Du : 0.0f), hw = half_sums_dpp(len > 0 ? Dw : 0.0f);
          const float ulo = lane_value(hu, 31), uhi = lane_value(hu, 63);
          const float vlo = lane_value(hw, 31), vhi = lane_value(hw, 63);
          if (lane == 0) {
            atomicAdd(&gsh->Du[bi % 3][elo], ulo);
            atomicAdd(&gsh->Du[bi % 3][ehi], uhi);
            atomicAdd(&gsh->Dw[bi % 3][elo], vlo);
            atomicAdd(&gsh->Dw[bi % 3][ehi], vhi);
          }
        }
      } else {
        unsigned long long act = __ballot(len > 0);
        while (act) {
          const int leader = __ffsll((long long)act) - 1;
          const int el = __builtin_amdgcn_readlane(e, leader);
          const bool mine = len > 0 && e == el;
          const float v = wave_sum_dpp(mine ? D : 0.0f);
          if (lane == 0) unsafeAtomicAdd(&Dc[el], (double)v);
          if constexpr (GRAD && !VALUE) {
            const float vu = wave_sum_dpp(mine ? Du : 0.0f);
            const float vw = wave_sum_dpp(mine ? Dw : 0.0f);
            if (lane == 0) {
              atomicAdd(&gsh->Du[bi % 3][el], vu);
              atomicAdd(&gsh->Dw[bi % 3][el], vw);
            }
          }
          act &= ~__ballot(mine);
        }
      }
      // batch bi + 1 accumulates into D[(bi + 1) % 3], last read (as batch bi - 2's) before the
      // previous barrier
      if (wave == 0 && tid < kMaxBatch) {
        ps.D[(bi + 1) % 3][tid] = 0.0;
        if constexpr (GRAD) {
          gsh->Du[(bi + 1) % 3][tid] = 0.0f;
          gsh->Dw[(bi + 1) % 3][tid] = 0.0f;
        }
      }
      plen = len;
      pbase = base;
      pe = e;
      pwl = wl;
      pwn = wn;
      word = next;
      wlw = wlw_next;
      wnw = wnw_next;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }

  // add the region's accumulators to the global image (wavefronts take columns, lanes rows)
  for (int cl = wave; cl < (VALUE ? 0 : p.W); cl += WAVES) {
    const int kc = kbase + cl;
    for (int rl = lane; rl < p.RY; rl += WAVE) {
      const unsigned long long a = (unsigned long long)acc_s[cl * pitch + rl] << flush_shift;
      if (a == 0ull) continue;
      const int r = rbase + rl;
      const int k = kc + off_s[rl];
      if (r >= 0 && r < g.n_y && k >= 0 && k < g.n_z) {
        if constexpr (GRAD) {
          unsafeAtomicAdd(reinterpret_cast<double*>(acc) + (int64_t)r * g.n_z + k, __longlong_as_double((long long)a));
        } else {
          atomicAdd(&acc[(int64_t)r * g.n_z + k], a);
        }
      }
    }
  }
  if constexpr (GRAD) {  // the batch slots' sums, held by the first wavefront's lanes
    if (tid < WAVE) {
      const bool slot = tid < kMaxBatch;
      const double a = wave_sum_d(slot ? gsh->sum[0][tid] : 0.0), b = wave_sum_d(slot ? gsh->sum[1][tid] : 0.0),
                   c = wave_sum_d(slot ? gsh->sum[2][tid] : 0.0);
      if (tid == 0) {
        unsafeAtomicAdd(&red[0], a);
        unsafeAtomicAdd(&red[1], b);
        unsafeAtomicAdd(&red[2], c);
      }
    }
  }
  if (tid == 0) {
    if (ps.zero) atomicAdd(&cnt[C_ZERO_DEN], (unsigned long long)ps.zero);
    if (ps.bad) atomicAdd(&cnt[C_KAPPA_BAD], (unsigned long long)ps.bad);
  }
}

// Resident wavefronts per SIMD the tiled pass is compiled for (the plan's cost model assumes
// them): the register cache of MAXLEN pixels leaves room for 8, 6, 5 or 4.
template <int MAXLEN>
constexpr int pass_waves_per_simd() {
  return MAXLEN <= 16 ? 8 : MAXLEN <= 32 ? 6 : MAXLEN <= 48 ? 5 : 4;
}

template <int MAXLEN, int WAVES, bool ACC32, int PITCH>
__global__ void __launch_bounds__(WAVES * 64, pass_waves_per_simd<MAXLEN>()) k_event_pass_tiled(Geo g, Plan p,
                                                                    const unsigned char* __restrict__ blocks,
                                                                    const BinItem* __restrict__ items,
                                                                    const float* __restrict__ rho,
                                                                    unsigned long long* __restrict__ acc,
                                                                    unsigned long long* __restrict__ cnt,
                                                                    const EventRec* __restrict__ evs,
                                                                    float* __restrict__ D_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ PassShared ps;
  if ((unsigned long long)blockIdx.x >= cnt[C_ITEMS]) return;  // uniform over the workgroup
  event_pass_item<MAXLEN, WAVES, false, ACC32, PITCH>(g, p, blocks, items[blockIdx.x], rho, acc, cnt, smem, ps,
                                                     nullptr, D_out, nullptr, evs);
}

// The log-likelihood pass on the binned layout (B: double image of sum P / D, zeroed by the
// caller; red[0..2]: log D', Du / D', Dw / D' sums, zeroed by the caller).
template <int MAXLEN>
constexpr int loglik_waves_per_simd() {
  return MAXLEN <= 16 ? 6 : 4;
}

template <int MAXLEN, int WAVES, bool VALUE, int PITCH>
__global__ void __launch_bounds__(WAVES * 64, loglik_waves_per_simd<MAXLEN>())
    k_loglik_tiled(Geo g, Plan p, const unsigned char* __restrict__ blocks, const BinItem* __restrict__ items,
                   const float* __restrict__ rho, double* __restrict__ B, float* __restrict__ D_out,
                   double* __restrict__ red, unsigned long long* __restrict__ cnt, const EventRec* __restrict__ evs) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ PassShared ps;
  __shared__ GradShared gsh;
  if ((unsigned long long)blockIdx.x >= cnt[C_ITEMS]) return;  // uniform over the workgroup
  event_pass_item<MAXLEN, WAVES, true, false, PITCH, VALUE>(g, p, blocks, items[blockIdx.x], rho,
                                                reinterpret_cast<unsigned long long*>(B), cnt, smem, ps, &gsh, D_out,
                                                red, evs);
}

// The same pass over many independent reconstructions: one workgroup per workgroup item of a
// class of instances (the grid is the class's item count, total).  Work index w = blockIdx.x is
// item w - item_begin of the last instance (in table order, heaviest items first) whose
// item_begin <= w.  Every instance of a class has the same region row pitch, PITCH (0: a runtime
// value), so that the per-pixel LDS addresses are immediates as in the single-image pass.
template <int MAXLEN, int WAVES, int PITCH>
__global__ void __launch_bounds__(WAVES * 64, pass_waves_per_simd<MAXLEN>())
    k_event_pass_batched(const BatchInst* __restrict__ inst, int count, unsigned total) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ PassShared ps;
  const unsigned w = blockIdx.x;
  if (w >= total) return;  // uniform over the workgroup
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (inst[mid].item_begin <= (int64_t)w) lo = mid;
    else hi = mid - 1;
  }
  const BatchInst& I = inst[lo];
  const BinItem it = I.items[(int64_t)w - I.item_begin];
  event_pass_item<MAXLEN, WAVES, false, true, PITCH>(I.g, I.p, I.blocks, it, I.rho, I.acc, I.cnt, smem, ps, nullptr,
                                                    nullptr, nullptr, nullptr);
}

// Generic pass for geometries whose rows or regions do not fit the tiled pass: one wavefront per
// event, one lane per row, kernel values recomputed in pass 2, fixed-point global atomics.
__global__ void __launch_bounds__(256) k_event_pass_generic(Geo g, int64_t n, const EventRec* __restrict__ ev,
                                                            const float* __restrict__ rho,
                                                            unsigned long long* __restrict__ acc,
                                                            unsigned long long* __restrict__ cnt,
                                                            float* __restrict__ D_out) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t j = (int64_t)blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x / WAVE);
  if (j >= n) return;
  const EventRec e = ev[j];
  if (e.r1 < e.r0) return;
  int nbad = 0;  // pixels of this lane's row with kappa <= 0 (P := 0)
  float D = 0.0f;
  for (int b0 = e.r0; b0 <= e.r1; b0 += WAVE) {
    const int i = b0 + lane;
    int klo, khi;
    if (i <= e.r1 && row_interval(g, e, i, &klo, &khi)) {
      double kf, ks;
      const RowK r = row_constants(g, e, i, klo, &kf, &ks);
      const float* rr = rho + (int64_t)i * g.n_z;
      for (int k = klo; k <= khi; ++k) D += kernel_guarded(r, (float)(k - klo), &nbad) * rr[k];
    }
  }
  D = wave_sum(D);
  const unsigned long long nbad_w = wave_sum_u64((unsigned long long)nbad);
  if (lane == 0 && nbad_w) atomicAdd(&cnt[C_KAPPA_BAD], nbad_w);
  int again = 0;  // pass 2 recomputes the same values: not counted twice
  if (lane == 0 && D_out) D_out[j] = (float)((double)D * g.cnorm);
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
        const float m = kernel_guarded(r, (float)(k - klo), &again) * rr[k];
        if (m > 0.0f) atomicAdd(&aa[k], (unsigned long long)(unsigned)fmaf(m, sc, 0.5f));
      }
    }
  }
}

// Thread-granularity pass (comparison only): one thread per event walks every pixel of its
// ellipse twice, first for D, then adding the back-projection with global fixed-point atomics.
// This is the GPU work split the paper measures as its "thread" variant (Sec. 4, Table 1); lanes
// of a wavefront hold events of different sizes and read unrelated image rows.
__global__ void __launch_bounds__(256) k_event_pass_thread(Geo g, int64_t n, const EventRec* __restrict__ ev,
                                                           const float* __restrict__ rho,
                                                           unsigned long long* __restrict__ acc,
                                                           unsigned long long* __restrict__ cnt,
                                                           float* __restrict__ D_out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const EventRec e = ev[j];
  if (e.r1 < e.r0) return;
  int nbad = 0;  // pixels of this event with kappa <= 0 (P := 0)
  float D = 0.0f;
  for (int i = e.r0; i <= e.r1; ++i) {
    int klo, khi;
    if (!row_interval(g, e, i, &klo, &khi)) continue;
    double kf, ks;
    const RowK r = row_constants(g, e, i, klo, &kf, &ks);
    const float* rr = rho + (int64_t)i * g.n_z;
    for (int k = klo; k <= khi; ++k) D += kernel_guarded(r, (float)(k - klo), &nbad) * rr[k];
  }
  if (nbad) atomicAdd(&cnt[C_KAPPA_BAD], (unsigned long long)nbad);
  int again = 0;  // pass 2 recomputes the same values: not counted twice
  if (D_out) D_out[j] = (float)((double)D * g.cnorm);
  if (!(D > 0.0f)) {
    atomicAdd(&cnt[C_ZERO_DEN], 1ull);
    return;
  }
  const float sc = (float)(4294967296.0 / (double)D);
  for (int i = e.r0; i <= e.r1; ++i) {
    int klo, khi;
    if (!row_interval(g, e, i, &klo, &khi)) continue;
    double kf, ks;
    const RowK r = row_constants(g, e, i, klo, &kf, &ks);
    const float* rr = rho + (int64_t)i * g.n_z;
    unsigned long long* aa = acc + (int64_t)i * g.n_z;
    for (int k = klo; k <= khi; ++k) {
      const float m = kernel_guarded(r, (float)(k - klo), &again) * rr[k];
      if (m > 0.0f) atomicAdd(&aa[k], (unsigned long long)(unsigned)fmaf(m, sc, 0.5f));
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

template <int MAXLEN, int WAVES, bool ACC32>
hipError_t launch_tiled(const Geo& g, const Plan& p, const Workspace& ws, const float* rho, float* D_out,
                        hipStream_t st) {
  auto kern = p.pitch == 64    ? k_event_pass_tiled<MAXLEN, WAVES, ACC32, 64>
              : p.pitch == 128 ? k_event_pass_tiled<MAXLEN, WAVES, ACC32, 128>
              : p.pitch == 192 ? k_event_pass_tiled<MAXLEN, WAVES, ACC32, 192>
              : p.pitch == 256 ? k_event_pass_tiled<MAXLEN, WAVES, ACC32, 256>
                               : k_event_pass_tiled<MAXLEN, WAVES, ACC32, 0>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)p.max_items), dim3(64 * p.waves), p.lds_bytes, st, g, p, ws.batches,
                     ws.items, rho, ws.acc, ws.cnt, ws.evs, D_out);
  return hipGetLastError();
}

__global__ void k_write_insts(InstWrite w, BatchInst* __restrict__ table) {
  const int t = threadIdx.x;
  if (t < w.count) table[w.first + t] = w.v[t];
}

// per-iteration counters of every instance: zero-denominator events, non-positive kappa pairs
__global__ void k_batched_reset(const BatchInst* __restrict__ table, int count) {
  for (int k = threadIdx.x; k < count; k += blockDim.x) {
    table[k].cnt[C_ZERO_DEN] = 0ull;
    table[k].cnt[C_KAPPA_BAD] = 0ull;
  }
}

// rho = acc 2^-32 / s of every instance (blockIdx.y: table entry)
__global__ void k_update_batched(const BatchInst* __restrict__ table) {
  const BatchInst& I = table[blockIdx.y];
  const int64_t npix = (int64_t)I.g.n_y * I.g.n_z;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < npix; q += (int64_t)gridDim.x * blockDim.x) {
    const double a = (double)I.acc[q] * 2.3283064365386962890625e-10;
    double v;
    if (I.s) {
      const float sv = I.s[q];
      v = sv > 0.0f ? a / (double)sv : 0.0;
    } else {
      v = a;
    }
    I.rho[q] = (float)v;
    I.acc[q] = 0ull;
  }
}

template <int MAXLEN, int WAVES, int PITCH>
hipError_t launch_loglik_p(const Geo& g, const Plan& p, const Workspace& ws, const float* rho, float* D_out,
                           bool value_only, hipStream_t st) {
  auto kern = value_only ? k_loglik_tiled<MAXLEN, WAVES, true, PITCH> : k_loglik_tiled<MAXLEN, WAVES, false, PITCH>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)p.max_items), dim3(64 * p.waves), p.lds_bytes, st, g, p, ws.batches,
                     ws.items, rho, ws.B, D_out, ws.red, ws.cnt, ws.evs);
  return hipGetLastError();
}

// regions whose row pitch is 64, 128, 192 or 256 take kernels compiled for it (immediate LDS offsets)
template <int MAXLEN, int WAVES>
hipError_t launch_loglik_t(const Geo& g, const Plan& p, const Workspace& ws, const float* rho, float* D_out,
                           bool value_only, hipStream_t st) {
  return p.pitch == 64    ? launch_loglik_p<MAXLEN, WAVES, 64>(g, p, ws, rho, D_out, value_only, st)
         : p.pitch == 128 ? launch_loglik_p<MAXLEN, WAVES, 128>(g, p, ws, rho, D_out, value_only, st)
         : p.pitch == 192 ? launch_loglik_p<MAXLEN, WAVES, 192>(g, p, ws, rho, D_out, value_only, st)
         : p.pitch == 256 ? launch_loglik_p<MAXLEN, WAVES, 256>(g, p, ws, rho, D_out, value_only, st)
                          : launch_loglik_p<MAXLEN, WAVES, 0>(g, p, ws, rho, D_out, value_only, st);
}

}  // namespace

hipError_t launch_loglik_tiled(const Geo& g, const Plan& p, int64_t n, const Workspace& ws, const float* rho,
                               float* D_out, bool value_only, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const bool v = value_only;
  switch (p.maxlen * 100 + p.waves) {
    case 1608: return launch_loglik_t<16, 8>(g, p, ws, rho, D_out, v, st);
    case 3208: return launch_loglik_t<32, 8>(g, p, ws, rho, D_out, v, st);
    case 4808: return launch_loglik_t<48, 8>(g, p, ws, rho, D_out, v, st);
    case 6408: return launch_loglik_t<64, 8>(g, p, ws, rho, D_out, v, st);
    case 1616: return launch_loglik_t<16, 16>(g, p, ws, rho, D_out, v, st);
    case 3216: return launch_loglik_t<32, 16>(g, p, ws, rho, D_out, v, st);
    case 4816: return launch_loglik_t<48, 16>(g, p, ws, rho, D_out, v, st);
    case 6416: return launch_loglik_t<64, 16>(g, p, ws, rho, D_out, v, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_write_insts(const InstWrite& w, BatchInst* table, hipStream_t st) {
  hipLaunchKernelGGL(k_write_insts, dim3(1), dim3(64), 0, st, w, table);
  return hipGetLastError();
}

hipError_t launch_batched_reset(const BatchInst* table, int count, hipStream_t st) {
  hipLaunchKernelGGL(k_batched_reset, dim3(1), dim3(256), 0, st, table, count);
  return hipGetLastError();
}

namespace {
template <int MAXLEN, int WAVES, int PITCH>
hipError_t launch_batched_t(const BatchInst* table, int count, unsigned items, size_t lds_bytes, hipStream_t st) {
  // the dynamic LDS limit is raised beforehand (set_batched_lds), outside any stream capture
  auto kern = k_event_pass_batched<MAXLEN, WAVES, PITCH>;
  hipLaunchKernelGGL(kern, dim3(items), dim3(64 * WAVES), lds_bytes, st, table, count, items);
  return hipGetLastError();
}

template <int MAXLEN, int WAVES>
const void* batched_kernel_p(int pitch) {
  switch (pitch) {
    case 64: return (const void*)k_event_pass_batched<MAXLEN, WAVES, 64>;
    case 128: return (const void*)k_event_pass_batched<MAXLEN, WAVES, 128>;
    case 192: return (const void*)k_event_pass_batched<MAXLEN, WAVES, 192>;
    case 256: return (const void*)k_event_pass_batched<MAXLEN, WAVES, 256>;
    default: return (const void*)k_event_pass_batched<MAXLEN, WAVES, 0>;
  }
}

const void* batched_kernel(int maxlen, int waves, int pitch) {
  switch (maxlen * 100 + waves) {
    case 1608: return batched_kernel_p<16, 8>(pitch);
    case 3208: return batched_kernel_p<32, 8>(pitch);
    case 4808: return batched_kernel_p<48, 8>(pitch);
    case 6408: return batched_kernel_p<64, 8>(pitch);
    case 1616: return batched_kernel_p<16, 16>(pitch);
    case 3216: return batched_kernel_p<32, 16>(pitch);
    case 4816: return batched_kernel_p<48, 16>(pitch);
    case 6416: return batched_kernel_p<64, 16>(pitch);
    default: return nullptr;
  }
}

template <int MAXLEN, int WAVES>
hipError_t launch_batched_p(const BatchInst* table, int count, int pitch, unsigned items, size_t lds_bytes,
                            hipStream_t st) {
  switch (pitch) {
    case 64: return launch_batched_t<MAXLEN, WAVES, 64>(table, count, items, lds_bytes, st);
    case 128: return launch_batched_t<MAXLEN, WAVES, 128>(table, count, items, lds_bytes, st);
    case 192: return launch_batched_t<MAXLEN, WAVES, 192>(table, count, items, lds_bytes, st);
    case 256: return launch_batched_t<MAXLEN, WAVES, 256>(table, count, items, lds_bytes, st);
    default: return launch_batched_t<MAXLEN, WAVES, 0>(table, count, items, lds_bytes, st);
  }
}
}  // namespace

hipError_t launch_event_pass_batched(const BatchInst* table, int count, int maxlen, int waves, int pitch,
                                     size_t lds_bytes, int64_t items, hipStream_t st) {
  if (count <= 0 || items <= 0) return hipSuccess;
  if (items > 0x7fffffffll) return hipErrorInvalidValue;
  const unsigned n = (unsigned)items;
  switch (maxlen * 100 + waves) {
    case 1608: return launch_batched_p<16, 8>(table, count, pitch, n, lds_bytes, st);
    case 3208: return launch_batched_p<32, 8>(table, count, pitch, n, lds_bytes, st);
    case 4808: return launch_batched_p<48, 8>(table, count, pitch, n, lds_bytes, st);
    case 6408: return launch_batched_p<64, 8>(table, count, pitch, n, lds_bytes, st);
    case 1616: return launch_batched_p<16, 16>(table, count, pitch, n, lds_bytes, st);
    case 3216: return launch_batched_p<32, 16>(table, count, pitch, n, lds_bytes, st);
    case 4816: return launch_batched_p<48, 16>(table, count, pitch, n, lds_bytes, st);
    case 6416: return launch_batched_p<64, 16>(table, count, pitch, n, lds_bytes, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t set_batched_lds(int maxlen, int waves, int pitch, size_t lds_bytes) {
  const void* k = batched_kernel(maxlen, waves, pitch);
  if (!k) return hipErrorInvalidValue;
  return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

hipError_t launch_update_batched(const BatchInst* table, int count, int64_t max_npix, hipStream_t st) {
  if (count <= 0 || max_npix <= 0) return hipSuccess;
  int64_t bx = (max_npix + 255) / 256;
  if (bx > 1024) bx = 1024;
  hipLaunchKernelGGL(k_update_batched, dim3((unsigned)bx, (unsigned)count), dim3(256), 0, st, table);
  return hipGetLastError();
}

hipError_t launch_event_pass(const Geo& g, const Plan& p, int64_t n, const Workspace& ws, const float* rho,
                             hipStream_t st, int granularity, float* D_out) {
  if (n <= 0) return hipSuccess;
  if (granularity == kPassThreadPerEvent) {
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_event_pass_thread, dim3((unsigned)blocks), dim3(256), 0, st, g, n, ws.ev, rho, ws.acc, ws.cnt,
                       D_out);
    return hipGetLastError();
  }
  if (p.tiled && granularity == kPassPlanned) {
    const int key = p.maxlen * 100 + p.waves + (p.acc32 ? 10000 : 0);
    switch (key) {
      case 1608: return launch_tiled<16, 8, false>(g, p, ws, rho, D_out, st);
      case 3208: return launch_tiled<32, 8, false>(g, p, ws, rho, D_out, st);
      case 4808: return launch_tiled<48, 8, false>(g, p, ws, rho, D_out, st);
      case 6408: return launch_tiled<64, 8, false>(g, p, ws, rho, D_out, st);
      case 1616: return launch_tiled<16, 16, false>(g, p, ws, rho, D_out, st);
      case 3216: return launch_tiled<32, 16, false>(g, p, ws, rho, D_out, st);
      case 4816: return launch_tiled<48, 16, false>(g, p, ws, rho, D_out, st);
      case 6416: return launch_tiled<64, 16, false>(g, p, ws, rho, D_out, st);
      case 11608: return launch_tiled<16, 8, true>(g, p, ws, rho, D_out, st);
      case 13208: return launch_tiled<32, 8, true>(g, p, ws, rho, D_out, st);
      case 14808: return launch_tiled<48, 8, true>(g, p, ws, rho, D_out, st);
      case 16408: return launch_tiled<64, 8, true>(g, p, ws, rho, D_out, st);
      case 11616: return launch_tiled<16, 16, true>(g, p, ws, rho, D_out, st);
      case 13216: return launch_tiled<32, 16, true>(g, p, ws, rho, D_out, st);
      case 14816: return launch_tiled<48, 16, true>(g, p, ws, rho, D_out, st);
      case 16416: return launch_tiled<64, 16, true>(g, p, ws, rho, D_out, st);
      default: return hipErrorInvalidValue;
    }
  }
  const int64_t blocks = (n + 3) / 4;
  hipLaunchKernelGGL(k_event_pass_generic, dim3((unsigned)blocks), dim3(256), 0, st, g, n, ws.ev, rho, ws.acc, ws.cnt,
                     D_out);
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
